"""GPU parity for the fixed-precision product and the evaluation's fused
workloads (Section 6): bigint_mullo (a*b mod B^n), bigint_add6 (six
dependent additions in one pass) and bigint_poly ((a a + b)(b b + b) + a b
mod B^n), against the oracle, bit for bit."""
import numpy as np
import pytest

from gpu_util import dev, host, rand_limbs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bi():
    import paper_2607_28897_amd as m
    m.lib()
    yield m
    m.set_mfma_config(0, 0, 0)


@pytest.mark.parametrize("dw", [7, 8])
@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 1000, 4096, 16384])
def test_mullo(bi, orc, n, dw):
    g = np.random.default_rng(n + dw)
    a = rand_limbs(g, 3, n)
    b = rand_limbs(g, 3, n)
    a[1] = 0xFFFFFFFF
    b[1] = 0xFFFFFFFF                 # (B^n - 1)^2 mod B^n = 1
    b[2] = 0
    bi.set_mfma_config(0, 0, dw)
    try:
        p = host(bi.mullo(dev(a), dev(b)))
    finally:
        bi.set_mfma_config(0, 0, 0)
    for i in range(3):
        assert np.array_equal(p[i], orc.mullo1(a[i], b[i])), i


@pytest.mark.parametrize("n", [1, 3, 64, 1023, 1024, 1025, 4096, 8192, 16384])
def test_add6(bi, orc, n):
    from paper_2607_28897_amd import inputs
    g = np.random.default_rng(n)
    a = rand_limbs(g, 4, n)
    b = rand_limbs(g, 4, n)
    a[1] = 0xFFFFFFFF
    b[1] = 0xFFFFFFFF                 # every addition overflows
    a[2] = inputs.carry_adversarial_row(g, n)
    b[2] = inputs.carry_adversarial_row(g, n)
    b[3] = 0
    r, ovf = bi.add6(dev(a), dev(b))
    r, ovf = host(r), host(ovf)
    for i in range(4):
        want, wo = orc.add6_1(a[i], b[i])
        assert np.array_equal(r[i], want), i
        assert int(ovf[i]) == wo, i


def test_add6_in_place(bi, orc):
    g = np.random.default_rng(11)
    a = rand_limbs(g, 3, 2000)
    b = rand_limbs(g, 3, 2000)
    ta = dev(a)
    bi.add6(ta, dev(b), out=ta)
    for i in range(3):
        assert np.array_equal(host(ta)[i], orc.add6_1(a[i], b[i])[0])


# up to 1448 limbs Poly runs one wave per instance, beyond on one work-group each
@pytest.mark.parametrize("n,batch", [(1, 5), (2, 3), (33, 4), (128, 9), (700, 5), (1024, 8),
                                     (1448, 3), (1449, 3), (4096, 4), (16384, 2)])
def test_poly(bi, orc, n, batch):
    g = np.random.default_rng(n * 3 + batch)
    a = rand_limbs(g, batch, n)
    b = rand_limbs(g, batch, n)
    a[0] = 0xFFFFFFFF
    p = host(bi.poly(dev(a), dev(b)))
    for i in range(batch):
        assert np.array_equal(p[i], orc.poly1(a[i], b[i])), i


@pytest.mark.parametrize("n,batch", [(64, 3000), (256, 20000)])
def test_poly_more_instances_than_work_groups(bi, orc, n, batch):
    # four instances per work-group, a batch that is not a multiple of four
    g = np.random.default_rng(5)
    batch += 1
    a = rand_limbs(g, batch, n)
    b = rand_limbs(g, batch, n)
    p = host(bi.poly(dev(a), dev(b)))
    for i in list(range(0, batch, 97)) + [batch - 1]:
        assert np.array_equal(p[i], orc.poly1(a[i], b[i])), i


def test_fused_argument_checks(bi):
    import ctypes
    import torch
    L = bi.lib()
    x = torch.zeros(64, dtype=torch.int32, device="cuda")
    p = ctypes.c_void_p(x.data_ptr())
    q = ctypes.c_void_p(x.data_ptr() + 4)
    assert L.bigint_add6(p, None, p, p, 16385, 1, None) == bi.EUNSUPPORTED
    assert L.bigint_add6(q, None, p, p, 8, 1, None) == bi.EINVAL       # partial overlap
    assert L.bigint_poly(p, p, p, 8, 1, None) == bi.EINVAL            # out overlaps a
    assert L.bigint_mullo(p, p, p, 8, 1, None) == bi.EINVAL
    assert L.bigint_mullo(p, p, p, 0, 1, None) == bi.EINVAL
    assert L.bigint_add6(p, None, p, p, 8, 0, None) == 0              # empty batch
