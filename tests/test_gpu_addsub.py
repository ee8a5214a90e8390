"""GPU parity: batched add / sub (carry and borrow scans) against the oracle,
bit for bit, through the C-ABI."""
import numpy as np
import pytest

from gpu_util import dev, host, rand_limbs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bi():
    import paper_2607_28897_amd as m
    m.lib()
    return m


def _check(bi, orc, a, b):
    out, c = bi.add(dev(a), dev(b))
    want, wc = orc.add(a, b)
    assert np.array_equal(host(out), want)
    assert np.array_equal(host(c), wc)
    out, c = bi.sub(dev(a), dev(b))
    want, wc = orc.sub(a, b)
    assert np.array_equal(host(out), want)
    assert np.array_equal(host(c), wc)


def test_pairs_2e15(bi, orc):
    from paper_2607_28897_amd import inputs
    c = inputs.pairs_2e15()
    _check(bi, orc, c["a"], c["b"])
    out, br = bi.sub(dev(c["sub_a"]), dev(c["sub_b"]))
    want, wb = orc.sub(c["sub_a"], c["sub_b"])
    assert np.array_equal(host(out), want) and not host(br).any()


def test_pairs_2e17_uniform_and_carry_adversarial(bi, orc):
    from paper_2607_28897_amd import inputs
    c = inputs.pairs_2e17_mixed()
    _check(bi, orc, c["a"], c["b"])
    out, br = bi.sub(dev(c["sub_a"]), dev(c["sub_b"]))
    want, _ = orc.sub(c["sub_a"], c["sub_b"])
    assert np.array_equal(host(out), want) and not host(br).any()


@pytest.mark.parametrize("n", [1, 2, 3, 5, 63, 64, 65, 255, 1023, 1025, 4097, 16384, 16385, 40000, 65536])
def test_sizes_ragged_tails(bi, orc, n):
    g = np.random.default_rng(n)
    batch = 3 if n > 10000 else 7
    a = rand_limbs(g, batch, n)
    b = rand_limbs(g, batch, n)
    # make long propagate runs straddle thread and wave boundaries
    a[0, :] = 0xFFFFFFFF
    b[0, :] = 0
    b[0, 0] = 1
    a[1, : n // 2] = 0xFFFFFFFF
    b[1, : n // 2] = 0xFFFFFFFF
    _check(bi, orc, a, b)


def test_full_ripple_closed_forms(bi, orc):
    n = 4096
    ones = np.full((2, n), 0xFFFFFFFF, np.uint32)
    one = np.zeros((2, n), np.uint32)
    one[:, 0] = 1
    out, c = bi.add(dev(ones), dev(one))          # (B^n - 1) + 1 = B^n
    assert not host(out).any() and (host(c) == 1).all()
    out, br = bi.sub(dev(np.zeros((2, n), np.uint32)), dev(one))   # 0 - 1
    assert (host(out) == 0xFFFFFFFF).all() and (host(br) == 1).all()
    top = np.zeros((2, n), np.uint32)
    top[:, -1] = 1
    out, br = bi.sub(dev(top), dev(one))           # B^(n-1) - 1
    h = host(out)
    assert (h[:, :-1] == 0xFFFFFFFF).all() and not h[:, -1].any() and not host(br).any()


def test_in_place(bi, orc):
    g = np.random.default_rng(5)
    a = rand_limbs(g, 4, 999)
    b = rand_limbs(g, 4, 999)
    ta, tb = dev(a), dev(b)
    bi.add(ta, tb, out=ta)
    assert np.array_equal(host(ta), orc.add(a, b)[0])
    bi.sub(ta, tb, out=tb)
    s = orc.add(a, b)[0]
    assert np.array_equal(host(tb), orc.sub(s, b)[0])


def test_empty_batch_and_errors(bi):
    import ctypes
    import torch
    L = bi.lib()
    x = torch.zeros(8, dtype=torch.int32, device="cuda")
    p = ctypes.c_void_p(x.data_ptr())
    assert L.bigint_add(p, None, p, p, 8, 0, None) == 0
    assert L.bigint_add(None, None, p, p, 8, 1, None) == bi.EINVAL
    assert L.bigint_add(p, None, p, p, 0, 1, None) == bi.EINVAL
    # partial overlap between out and a is rejected
    q = ctypes.c_void_p(x.data_ptr() + 4)
    assert L.bigint_add(q, None, p, p, 4, 1, None) == bi.EINVAL


@pytest.mark.parametrize("n", [1, 3, 4, 7, 16, 33, 128, 200, 256])
@pytest.mark.parametrize("batch", [1, 9, 301])
def test_several_instances_per_wave(bi, orc, n, batch):
    """Up to 256 limbs several instances share a wave (segmented carry scan):
    carries must stop at every instance boundary, including all-ones
    instances next to each other and a last work-group that is not full."""
    g = np.random.default_rng(n * 1000 + batch)
    a = rand_limbs(g, batch, n)
    b = rand_limbs(g, batch, n)
    a[::3] = 0xFFFFFFFF                  # every third instance: full ripple on add
    b[::3] = 0
    b[::3, 0] = 1
    a[1::3] = 0                          # and borrow ripple on sub
    b[1::3] = 0
    b[1::3, 0] = 1
    _check(bi, orc, a, b)
    out, ovf = bi.add6(dev(a), dev(b))
    out, ovf = host(out), ovf.cpu().numpy()
    for i in range(batch):
        want, wo = orc.add6_1(a[i], b[i])
        assert np.array_equal(out[i], want), i
        assert int(ovf[i]) == int(wo), i


@pytest.mark.parametrize("n", [2049, 3001, 4096])
def test_batches_of_two_to_four_groups_per_cu(bi, orc, n):
    """Between 2048 and 4096 limbs a batch of 2..4 instances per CU runs on
    512-thread work-groups instead of 1024-thread ones."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    batch = 3 * cus
    g = np.random.default_rng(n + 17)
    a = rand_limbs(g, batch, n)
    b = rand_limbs(g, batch, n)
    a[::5] = 0xFFFFFFFF                  # full ripples across every thread
    b[::5] = 0
    b[::5, 0] = 1
    a[1::5] = 0
    b[1::5] = 0
    b[1::5, 0] = 1
    _check(bi, orc, a, b)
