"""GPU parity: ragged batches (work queue ordered largest first, one launch
per segment of tile configuration and occupancy with smaller instances filling
each segment's end, hipGraph replay), against the oracle."""
import numpy as np
import pytest

from gpu_util import dev, host, oracle_map

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


@pytest.fixture(scope="module")
def ragged_4096(orc):
    """The 4096-product ragged configuration (bit lengths log-uniform in
    [2^15, 2^19]) and the oracle's product of every pair, flattened like the
    library's output."""
    from paper_2607_28897_amd import inputs
    c = inputs.ragged_mul_2e15_2e19()
    lens = c["lens"]
    rows = oracle_map(lambda i: orc.mul1(c["a"][c["a_off"][i]:c["a_off"][i + 1]],
                                         c["b"][c["b_off"][i]:c["b_off"][i + 1]]), range(lens.size))
    c["want"] = np.concatenate(rows)
    off = np.zeros(lens.size + 1, np.int64)
    np.cumsum(2 * lens, out=off[1:])
    c["out_off"] = off
    return c


def _first_bad_instance(got, c):
    off = c["out_off"]
    bad = np.nonzero(got != c["want"])[0]
    return None if bad.size == 0 else int(np.searchsorted(off, bad[0], side="right") - 1)


@pytest.mark.parametrize("stream", ["default", "side"])
def test_ragged_4096_every_instance_graph_replays(bi, ragged_4096, stream):
    """Every product of the 4096-instance configuration against the oracle,
    from the captured graph's first launch and from three replays (with
    other work on the stream in between, each replay into a cleared buffer),
    on torch's default stream (the null stream) and on a side stream; the
    plan's counters show one graph instantiated and replayed."""
    import torch
    c = ragged_4096
    lens = c["lens"]
    st = torch.cuda.Stream() if stream == "side" else torch.cuda.default_stream()
    with torch.cuda.stream(st):
        plan = bi.MulPlan(lens, lens)
        ta, tao = dev(c["a"]), torch.from_numpy(c["a_off"]).cuda()
        tb, tbo = dev(c["b"]), torch.from_numpy(c["b_off"]).cuda()
        out = torch.empty(int(2 * lens.sum()), dtype=torch.int32, device="cuda")
        out_off = torch.from_numpy(c["out_off"]).cuda()
        scratch = torch.zeros(1 << 20, dtype=torch.int32, device="cuda")
        for rep in range(4):
            out.fill_(-1)
            plan(ta, tao, tb, tbo, out=out, out_off=out_off)
            scratch.add_(1)                               # eager work between replays
            st.synchronize()
            assert _first_bad_instance(host(out), c) is None, rep
        info = plan.info()
        assert info["graphs_instantiated"] == 1 and info["graph_replays"] == 3, info
        assert info["launches_per_call"] >= 1
        plan.close()


def test_ragged_4096_direct_launch(bi, ragged_4096):
    """The same batch without a graph (BIGINT_PLAN_NO_GRAPH), every product."""
    import torch
    c = ragged_4096
    lens = c["lens"]
    plan = bi.MulPlan(lens, lens, bi.PLAN_NO_GRAPH)
    out, _ = plan(dev(c["a"]), torch.from_numpy(c["a_off"]).cuda(), dev(c["b"]),
                  torch.from_numpy(c["b_off"]).cuda())
    assert _first_bad_instance(host(out), c) is None
    assert plan.info()["graphs_instantiated"] == 0
    plan.close()


def test_ragged_4096_segments_one_by_one(bi, ragged_4096):
    """The plan's segment table covers the queue once, in order; launching
    every segment alone, last first, into a cleared buffer gives every
    product; a segment index out of range is refused."""
    import torch
    c = ragged_4096
    lens = c["lens"]
    plan = bi.MulPlan(lens, lens)
    segs = plan.segments()
    assert all(s["parts"] == 1 for s in segs)               # many instances: none split
    assert len(segs) == plan.info()["launches_per_call"] >= 1
    assert plan.workspace_size() == 0
    assert segs[0]["first"] == 0
    for s0, s1 in zip(segs, segs[1:]):
        assert s1["first"] == s0["first"] + s0["instances"]
    assert sum(s["instances"] for s in segs) == lens.size
    for s in segs:
        assert s["digit_bits"] in (7, 8) and s["strips_per_band"] in (4, 8, 16)
        assert s["slots"] >= 256 and 0.0 < s["modelled_busy"] <= 1.0
    # at least (4n)^2 digit products per instance (8-bit digits; 7-bit ones have more)
    assert sum(s["digit_products"] for s in segs) >= int(((4 * lens.astype(np.int64)) ** 2).sum())
    ta, tao = dev(c["a"]), torch.from_numpy(c["a_off"]).cuda()
    tb, tbo = dev(c["b"]), torch.from_numpy(c["b_off"]).cuda()
    out = torch.full((int(2 * lens.sum()),), -1, dtype=torch.int32, device="cuda")
    oo = torch.from_numpy(c["out_off"]).cuda()
    for k in reversed(range(len(segs))):
        plan.run_segment(k, ta, tao, tb, tbo, out, oo)
    torch.cuda.synchronize()
    assert _first_bad_instance(host(out), c) is None
    with pytest.raises(bi.BigIntError):
        plan.run_segment(len(segs), ta, tao, tb, tbo, out, oo)
    plan.close()


def _few_large(g):
    # a few large products (some far from square) among small ones
    la = np.array([16384, 16000, 12000, 9000, 18432, 3000, 500, 7, 1, 2048, 14000, 6000], np.int64)
    lb = np.array([16384, 15000, 11000, 9500, 1, 3333, 40, 7000, 1, 2048, 200, 6000], np.int64)
    a, a_off = _ragged(g, la)
    b, b_off = _ragged(g, lb)
    a[a_off[0]:a_off[1]] = 0xFFFFFFFF      # carries through whole strips
    b[b_off[0]:b_off[1]] = 0xFFFFFFFF
    return la, lb, a, a_off, b, b_off


@pytest.mark.parametrize("flags", [0, 2])   # graph, direct launch
def test_ragged_few_large_instances_split(bi, orc, flags):
    """A plan whose largest segment holds a few instances splits their bands
    over work-groups (parts > 1, two launches, the plan's workspace): every
    product against the oracle, on the first call and on replays into a
    cleared buffer, and each segment launched alone."""
    import torch
    g = np.random.default_rng(123 + flags)
    la, lb, a, a_off, b, b_off = _few_large(g)
    plan = bi.MulPlan(la, lb, flags)
    segs = plan.segments()
    assert any(s["parts"] >= 4 for s in segs), segs
    assert plan.info()["launches_per_call"] == sum(2 if s["parts"] > 1 else 1 for s in segs)
    assert plan.workspace_size() > 0
    want = oracle_map(lambda i: orc.mul1(a[a_off[i]:a_off[i + 1]], b[b_off[i]:b_off[i + 1]]),
                      range(la.size))
    ta, tao = dev(a), torch.from_numpy(a_off).cuda()
    tb, tbo = dev(b), torch.from_numpy(b_off).cuda()
    out_off = np.zeros(la.size + 1, np.int64)
    np.cumsum(la + lb, out=out_off[1:])
    oo = torch.from_numpy(out_off).cuda()
    out = torch.empty(int(out_off[-1]), dtype=torch.int32, device="cuda")
    for rep in range(3):
        out.fill_(-1)
        plan(ta, tao, tb, tbo, out=out, out_off=oo)
        res = host(out)
        for i in range(la.size):
            assert np.array_equal(res[out_off[i]:out_off[i + 1]], want[i]), (rep, i)
    out.fill_(-1)
    for k in reversed(range(len(segs))):
        plan.run_segment(k, ta, tao, tb, tbo, out, oo)
    res = host(out)
    for i in range(la.size):
        assert np.array_equal(res[out_off[i]:out_off[i + 1]], want[i]), ("segments", i)
    plan.close()


def test_ragged_split_with_caller_workspace(bi, orc):
    """The same plan with a workspace the caller provides (too small: refused)."""
    import torch
    g = np.random.default_rng(321)
    la, lb, a, a_off, b, b_off = _few_large(g)
    plan = bi.MulPlan(la, lb)
    need = plan.workspace_size()
    with pytest.raises(bi.BigIntError):
        plan.set_workspace(torch.empty(need // 4 - 1, dtype=torch.int32, device="cuda"))
    plan.set_workspace(torch.zeros(need // 4 + 16, dtype=torch.int32, device="cuda"))
    out, oo = plan(dev(a), torch.from_numpy(a_off).cuda(), dev(b), torch.from_numpy(b_off).cuda())
    res = host(out)
    off = oo.cpu().numpy()
    for i in range(la.size):
        assert np.array_equal(res[off[i]:off[i + 1]], orc.mul1(a[a_off[i]:a_off[i + 1]], b[b_off[i]:b_off[i + 1]])), i
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
