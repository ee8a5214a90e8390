"""GPU parity: ragged batches (work queue ordered largest first, one launch
per segment of tile configuration and occupancy with smaller instances filling
each segment's end, hipGraph replay), against the oracle."""
import numpy as np
import pytest

from gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bi():
    import paper_2607_28897_amd as m
    m.lib()
    return m


def _ragged(g, lens):
    off = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    flat = g.integers(0, 2**32, size=int(off[-1]), dtype=np.uint64).astype(np.uint32)
    return flat, off


def _run(bi, la, lb, a, a_off, b, b_off, flags):
    import torch
    plan = bi.MulPlan(la, lb, flags)
    out, out_off = plan(dev(a), torch.from_numpy(a_off).cuda(), dev(b), torch.from_numpy(b_off).cuda())
    res = host(out)
    oo = out_off.cpu().numpy()
    plan.close()
    return res, oo


@pytest.mark.parametrize("flags", [0, 2, 1])   # graph, direct launch, plain kernel
def test_small_ragged_mixed_sizes(bi, orc, flags):
    g = np.random.default_rng(17 + flags)
    B = 40
    la = g.integers(1, 3000, B)
    lb = g.integers(1, 3000, B)
    la[:3] = [1, 16384, 64]
    lb[:3] = [1, 16384, 7]
    a, a_off = _ragged(g, la)
    b, b_off = _ragged(g, lb)
    res, oo = _run(bi, la, lb, a, a_off, b, b_off, flags)
    for i in range(B):
        want = orc.mul1(a[a_off[i]:a_off[i + 1]], b[b_off[i]:b_off[i + 1]])
        assert np.array_equal(res[oo[i]:oo[i + 1]], want), i


def test_ragged_4096_sampled_and_replay(bi, orc):
    import torch
    from paper_2607_28897_amd import inputs
    c = inputs.ragged_mul_2e15_2e19()
    lens = c["lens"]
    plan = bi.MulPlan(lens, lens)
    ta, tao = dev(c["a"]), torch.from_numpy(c["a_off"]).cuda()
    tb, tbo = dev(c["b"]), torch.from_numpy(c["b_off"]).cuda()
    out_off, total = None, int(2 * lens.sum())
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    off = np.zeros(lens.size + 1, np.int64)
    np.cumsum(2 * lens, out=off[1:])
    out_off = torch.from_numpy(off).cuda()
    plan(ta, tao, tb, tbo, out=out, out_off=out_off)       # captures the graph
    r1 = host(out).copy()
    out.zero_()
    plan(ta, tao, tb, tbo, out=out, out_off=out_off)       # replays it
    r2 = host(out)
    assert np.array_equal(r1, r2)
    order = np.argsort(-lens)
    sample = list(order[:4]) + list(order[-4:]) + list(range(0, 4096, 257))
    for i in sample:
        a = c["a"][c["a_off"][i]:c["a_off"][i + 1]]
        b = c["b"][c["b_off"][i]:c["b_off"][i + 1]]
        assert np.array_equal(r1[off[i]:off[i + 1]], orc.mul1(a, b)), i
    plan.close()


def test_plan_errors(bi):
    import ctypes
    L = bi.lib()
    h = ctypes.c_void_p()
    la = np.array([5, 0], np.int64)
    assert L.bigint_plan_create(ctypes.byref(h), bi.OP_MUL, la.ctypes.data_as(ctypes.c_void_p),
                                la.ctypes.data_as(ctypes.c_void_p), 2, 0) == bi.EINVAL
    assert L.bigint_plan_create(ctypes.byref(h), 99, None, None, 0, 0) == bi.EINVAL
    assert L.bigint_plan_destroy(None) == bi.EINVAL


@pytest.mark.parametrize("dw", [7, 8])
def test_ragged_with_loaded_table(bi, orc, tmp_path, dw):
    # plans read the tuned table: a loaded table with one digit width drives
    # every configuration of the persistent kernel (P = 4, 8, 16)
    import json
    path = str(tmp_path / f"tune{dw}.json")
    bins = [{"max_limbs": 1500, "strips_per_band": 4, "waves": 8, "digit_bits": dw},
            {"max_limbs": 6000, "strips_per_band": 8, "waves": 8, "digit_bits": dw},
            {"max_limbs": 18432, "strips_per_band": 16, "waves": 8, "digit_bits": dw}]
    json.dump({"arch": "gfx950", "op": "mul_mfma", "bins": bins}, open(path, "w"))
    bi.autotune_load(path)
    try:
        g = np.random.default_rng(40 + dw)
        la = np.array([1, 1000, 1499, 1501, 5000, 6100, 12000, 16384, 7, 3333], np.int64)
        lb = np.array([9, 1000, 1400, 1501, 100, 6100, 12000, 16384, 7000, 3], np.int64)
        a, a_off = _ragged(g, la)
        b, b_off = _ragged(g, lb)
        res, oo = _run(bi, la, lb, a, a_off, b, b_off, 0)
        for i in range(la.size):
            want = orc.mul1(a[a_off[i]:a_off[i + 1]], b[b_off[i]:b_off[i + 1]])
            assert np.array_equal(res[oo[i]:oo[i + 1]], want), i
    finally:
        bi.autotune_load(None)


@pytest.mark.parametrize("flags", [0, 2])
def test_ragged_segments_and_fillers(bi, orc, flags):
    """Sizes spread over every tile configuration (1 to 18432 limbs, unequal
    operand lengths), so the plan cuts several segments and fills their ends
    with smaller instances; every product checked."""
    g = np.random.default_rng(91 + flags)
    B = 160
    la = np.exp(g.uniform(0, np.log(12000), B)).astype(np.int64) + 1
    lb = np.maximum(1, (la * g.uniform(0.3, 1.0, B)).astype(np.int64))
    la[:4] = [18432, 1, 5000, 11585]
    lb[:4] = [18432, 18432, 1, 11586]
    a, a_off = _ragged(g, la)
    b, b_off = _ragged(g, lb)
    res, oo = _run(bi, la, lb, a, a_off, b, b_off, flags)
    for i in range(B):
        want = orc.mul1(a[a_off[i]:a_off[i + 1]], b[b_off[i]:b_off[i + 1]])
        assert np.array_equal(res[oo[i]:oo[i + 1]], want), (i, la[i], lb[i])


@pytest.mark.parametrize("n", [1, 700, 16384])
def test_ragged_single_instance(bi, orc, n):
    g = np.random.default_rng(n)
    la = np.array([n], np.int64)
    lb = np.array([max(1, n // 3)], np.int64)
    a, a_off = _ragged(g, la)
    b, b_off = _ragged(g, lb)
    for flags in (0, 2, 1):
        res, oo = _run(bi, la, lb, a, a_off, b, b_off, flags)
        assert np.array_equal(res, orc.mul1(a, b)), flags


@pytest.mark.parametrize("case", ["equal", "unequal"])
def test_plain_ragged_sizes(bi, orc, case):
    """The plain ragged multiply (one 1024-thread work-group per instance in
    queue order) on equal operands spread over 1..16384 limbs, and on unequal
    operands whose sizes go up and down along the queue."""
    g = np.random.default_rng(91 if case == "equal" else 92)
    if case == "equal":
        la = np.maximum(np.exp(g.uniform(0.0, np.log(16384), 60)).astype(np.int64), 1)
        lb = la.copy()
    else:
        la = np.array([100, 1100, 9000, 3, 2048, 700, 16000, 50] * 3, np.int64)
        lb = np.array([10000, 1100, 200, 4000, 2048, 700, 16384, 5000] * 3, np.int64)
    a, a_off = _ragged(g, la)
    b, b_off = _ragged(g, lb)
    a[a_off[1]:a_off[2]] = 0xFFFFFFFF
    b[b_off[1]:b_off[2]] = 0xFFFFFFFF
    res, oo = _run(bi, la, lb, a, a_off, b, b_off, 1)
    for i in range(len(la)):
        want = orc.mul1(a[a_off[i]:a_off[i + 1]], b[b_off[i]:b_off[i + 1]])
        assert np.array_equal(res[oo[i]:oo[i + 1]], want), i
