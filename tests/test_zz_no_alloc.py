"""The allocation-free division (bigint_divmod_noalloc) against bigint_divmod:
same bytes, called through the C-ABI, twice in a row on the device's shared
scratch array, the second call with a smaller input."""
import ctypes

import numpy as np
import pytest

from gpu_util import dev, host, rand_limbs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bi():
    import paper_2607_28897_amd as m
    m.lib()
    return m


def _call(bi, fn, u, v):
    import torch
    batch, nu = u.shape
    nv = v.shape[1]
    tu, tv = dev(u), dev(v)
    q = torch.full((batch, nu), -1, dtype=torch.int32, device="cuda")
    r = torch.full((batch, nv), -1, dtype=torch.int32, device="cuda")
    st = torch.full((batch,), -1, dtype=torch.int32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = fn(p(q), p(r), p(st), p(tu), nu, p(tv), nv, batch, s)
    assert rc == bi.OK, rc
    torch.cuda.synchronize()
    return host(q), host(r), st.cpu().numpy()


def test_noalloc_matches_divmod_twice(bi):
    L = bi.lib()
    g = np.random.default_rng(2607)
    # first call: 8192 / 4096-limb divisions, more than the 128 MiB array
    # holds at once (164 KB of workspace each), so two launches reuse it
    u1 = rand_limbs(g, 1000, 8192)
    v1 = rand_limbs(g, 1000, 4096)
    v1[:, -1] |= 1
    v1[3] = 0                                  # a zero divisor
    u1[4, 4096:] = 0                           # u < v
    # second call, smaller: 300 / 7-limb divisions, leading zero limbs in v
    u2 = rand_limbs(g, 50, 300)
    v2 = rand_limbs(g, 50, 7)
    v2[1, 4:] = 0
    for u, v in ((u1, v1), (u2, v2)):
        want = _call(bi, L.bigint_divmod, u, v)
        got = _call(bi, L.bigint_divmod_noalloc, u, v)
        for w, x in zip(want, got):
            assert np.array_equal(w, x)


def test_noalloc_argument_checks(bi):
    L = bi.lib()
    assert L.bigint_divmod_noalloc(None, None, None, None, 1, None, 1, 1, None) == bi.EINVAL
    x = ctypes.c_void_p(16)
    assert L.bigint_divmod_noalloc(x, ctypes.c_void_p(1 << 20), None, ctypes.c_void_p(2 << 20), 16385,
                                   ctypes.c_void_p(3 << 20), 5, 1, None) == bi.EUNSUPPORTED
    assert L.bigint_divmod_noalloc(x, x, None, x, 5, x, 5, -1, None) == bi.EINVAL
