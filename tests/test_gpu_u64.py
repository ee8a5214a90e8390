"""GPU parity with 64-bit limb tensors: an int64 row of n digits is the same
bytes as 2n u32 limbs (little-endian), and the binding hands results back as
int64 views of the same bytes."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bi():
    import paper_2607_28897_amd as m
    m.lib()
    return m


def _u64(g, rows, n):
    return g.integers(0, 2**64, (rows, n), dtype=np.uint64)


def _dev(x):
    return torch.from_numpy(x.view(np.int64)).cuda()


def _host32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("n", [1, 3, 512, 2049])
def test_u64_add_sub_mul(bi, orc, n):
    g = np.random.default_rng(n)
    a, b = _u64(g, 3, n), _u64(g, 3, n)
    a32, b32 = a.view(np.uint32), b.view(np.uint32)
    r, c = bi.add(_dev(a), _dev(b))
    assert r.dtype == torch.int64 and r.shape == (3, n)
    want, wc = orc.add(a32, b32)
    assert np.array_equal(_host32(r), want) and np.array_equal(c.cpu().numpy().view(np.uint32), wc)
    r, c = bi.sub(_dev(a), _dev(b))
    assert np.array_equal(_host32(r), orc.sub(a32, b32)[0])
    p = bi.mul(_dev(a), _dev(b))
    assert p.dtype == torch.int64 and p.shape == (3, 2 * n)
    assert np.array_equal(_host32(p), orc.mul(a32, b32))


def test_u64_divmod_mullo(bi, orc):
    g = np.random.default_rng(9)
    u, v = _u64(g, 4, 1000), _u64(g, 4, 300)
    q, r, st = bi.divmod(_dev(u), _dev(v))
    assert q.dtype == torch.int64 and q.shape == (4, 1000) and r.shape == (4, 300)
    for i in range(4):
        wq, wr, ws = orc.divmod1(u[i].view(np.uint32), v[i].view(np.uint32))
        assert np.array_equal(_host32(q)[i], wq) and np.array_equal(_host32(r)[i], wr)
    a, b = _u64(g, 2, 700), _u64(g, 2, 700)
    lo = bi.mullo(_dev(a), _dev(b))
    assert lo.dtype == torch.int64 and lo.shape == (2, 700)
    for i in range(2):
        assert np.array_equal(_host32(lo)[i], orc.mullo1(a[i].view(np.uint32), b[i].view(np.uint32)))
