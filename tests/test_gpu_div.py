"""GPU parity: division through the whole shifted inverse (Newton steps on the
MFMA-split multiply) against the oracle's Knuth division, and the shifted
inverse itself against floor(B^h / v)."""
import numpy as np
import pytest

from gpu_util import dev, host, oracle_map, rand_limbs

pytestmark = pytest.mark.gpu

EDGE = np.array([0, 1, 2, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFE, 0xFFFFFFFF], np.uint32)


@pytest.fixture(scope="module")
def bi():
    import paper_2607_28897_amd as m
    m.lib()
    return m


def _check_batch(bi, orc, u, v):
    q, r, st = bi.divmod(dev(u), dev(v))
    q, r, st = host(q), host(r), st.cpu().numpy()
    for i in range(u.shape[0]):
        wq, wr, ws = orc.divmod1(u[i], v[i])
        assert st[i] == ws, i
        assert np.array_equal(q[i], wq), i
        assert np.array_equal(r[i], wr), i


@pytest.mark.parametrize("nu,nv", [(1, 1), (2, 1), (5, 1), (2, 2), (3, 2), (4, 3), (7, 3), (8, 4),
                                   (20, 10), (64, 3), (100, 99), (257, 128), (1000, 500), (2048, 1024),
                                   (3000, 7), (9, 20)])
def test_shapes_random(bi, orc, nu, nv):
    g = np.random.default_rng(nu * 131 + nv)
    B = 6
    u = rand_limbs(g, B, nu)
    v = rand_limbs(g, B, nv)
    v[1, -1] = 1                           # small top limb
    v[2] = 0xFFFFFFFF                       # all ones
    v[3, nv // 2:] = 0                      # leading zero limbs: precision below nv
    if nv > 1:
        v[3, 0] = max(v[3, 0], 1)
    u[4] = 0xFFFFFFFF
    u[5, :] = 0
    _check_batch(bi, orc, u, v)


def test_special_values(bi, orc):
    n = 40
    rows_u, rows_v = [], []
    g = np.random.default_rng(3)
    base = rand_limbs(g, 1, n)[0]
    one = np.zeros(n, np.uint32); one[0] = 1
    rows_u.append(base); rows_v.append(one)                        # v = 1
    rows_u.append(base); rows_v.append(base.copy())                # u = v
    small = base.copy(); small[-1] = 0
    rows_u.append(small); rows_v.append(base.copy())               # u < v
    rows_u.append(base); rows_v.append(np.zeros(n, np.uint32))     # v = 0
    half = np.zeros(n, np.uint32); half[: n // 2] = 0xFFFFFFFF     # (B^2m - 1) / (B^m - 1)
    rows_u.append(np.full(n, 0xFFFFFFFF, np.uint32)); rows_v.append(half)
    pw = np.zeros(n, np.uint32); pw[n // 2] = 1                     # v = B^m
    rows_u.append(base); rows_v.append(pw)
    u = np.stack(rows_u); v = np.stack(rows_v)
    _check_batch(bi, orc, u, v)


def test_edge_alphabet(bi, orc):
    g = np.random.default_rng(11)
    for nu, nv in ((3, 2), (4, 3), (6, 4), (9, 5)):
        u = g.choice(EDGE, size=(64, nu))
        v = g.choice(EDGE, size=(64, nv))
        _check_batch(bi, orc, u, v)


def _to_int(x):
    return int.from_bytes(np.ascontiguousarray(x, dtype="<u4").tobytes(), "little")


@pytest.fixture(scope="module")
def divs_512(orc):
    """The 512-division configuration (dividends log-uniform in [2^16, 2^18]
    bits, divisors half the limbs) and the oracle's quotient and remainder of
    every division."""
    from paper_2607_28897_amd import inputs
    c = inputs.ragged_div_2e16_2e18()
    u_off, v_off = c["u_off"], c["v_off"]
    res = oracle_map(lambda i: orc.divmod1(c["u"][u_off[i]:u_off[i + 1]],
                                           c["v"][v_off[i]:v_off[i + 1]]), range(512))
    c["want_q"] = np.concatenate([x[0] for x in res])
    c["want_r"] = np.concatenate([x[1] for x in res])
    return c


def _check_512(c, q, r, st):
    """Every division: the unique characterisation u = q v + r, 0 <= r < v
    (Python integers), then limb-by-limb equality with the oracle."""
    assert not st.any()
    u_off, v_off = c["u_off"], c["v_off"]
    for i in range(512):
        U = _to_int(c["u"][u_off[i]:u_off[i + 1]])
        V = _to_int(c["v"][v_off[i]:v_off[i + 1]])
        Q = _to_int(q[u_off[i]:u_off[i + 1]])
        R = _to_int(r[v_off[i]:v_off[i + 1]])
        assert U == Q * V + R and 0 <= R < V, i
    assert np.array_equal(q, c["want_q"])
    assert np.array_equal(r, c["want_r"])


def test_ragged_512_divisions_every_instance(bi, divs_512):
    """All 512 divisions, from the captured graph and from two replays."""
    import torch
    c = divs_512
    plan = bi.DivPlan(c["nu"], c["nv"])
    tu, tuo = dev(c["u"]), torch.from_numpy(c["u_off"]).cuda()
    tv, tvo = dev(c["v"]), torch.from_numpy(c["v_off"]).cuda()
    for rep in range(3):
        q, r, st = plan(tu, tuo, tv, tvo)
        _check_512(c, host(q), host(r), st.cpu().numpy())
    info = plan.info()
    assert info["graphs_instantiated"] >= 1, info
    plan.close()


def test_ragged_512_divisions_direct_and_counters(bi, divs_512):
    """All 512 divisions launched without a graph, and through the counting
    diagnostic (same bytes; every division issues MFMA work)."""
    import torch
    c = divs_512
    plan = bi.DivPlan(c["nu"], c["nv"], bi.PLAN_NO_GRAPH)
    tu, tuo = dev(c["u"]), torch.from_numpy(c["u_off"]).cuda()
    tv, tvo = dev(c["v"]), torch.from_numpy(c["v_off"]).cuda()
    q, r, st = plan(tu, tuo, tv, tvo)
    _check_512(c, host(q), host(r), st.cpu().numpy())
    q2, r2, st2, cnt = plan.counters(tu, tuo, tv, tvo)
    assert torch.equal(q, q2) and torch.equal(r, r2) and torch.equal(st, st2)
    assert (cnt.cpu().numpy()[:, 3] > 0).all()
    plan.close()


@pytest.mark.parametrize("nv,h", [(1, 1), (1, 9), (2, 2), (2, 7), (3, 3), (5, 40), (64, 130), (500, 2000)])
def test_shifted_inverse(bi, orc, nv, h):
    g = np.random.default_rng(nv * 7 + h)
    v = rand_limbs(g, 4, nv)
    v[:, -1] |= 1
    v[1, -1] = 1
    v[2] = 0xFFFFFFFF
    w = host(bi.shinv(dev(v), h))
    for i in range(4):
        want, _ = orc.shinv1(v[i], h)
        assert np.array_equal(w[i], want), i


def test_knuth_add_back_inputs(bi, orc):
    # inputs on which schoolbook division needs its rarest correction step
    from conftest import from_int
    from test_oracle_pins import ADD_BACK_CASES
    for u, v in ADD_BACK_CASES:
        nu, nv = -(-u.bit_length() // 32), -(-v.bit_length() // 32)
        _check_batch(bi, orc, from_int(u, nu)[None], from_int(v, nv)[None])


@pytest.mark.parametrize("nu,nv", [(40, 17), (2000, 600), (2000, 1000), (4100, 2049)])
def test_divisor_structures(bi, orc, nu, nv):
    # the Newton steps read only the top limbs of v: divisors whose low limbs
    # are zero, whose top limbs are a power of B or all ones, or whose low
    # limbs alone differ, must still give the exact quotient
    g = np.random.default_rng(nu + 7 * nv)
    u = rand_limbs(g, 6, nu)
    v = rand_limbs(g, 6, nv)
    v[0, :] = 0
    v[0, -1] = 1                                   # B^(nv-1)
    v[1, : nv - 3] = 0                             # three random top limbs, zeros below
    v[2, nv // 2:] = 0xFFFFFFFF                    # all-ones top half
    v[3] = v[2]
    v[3, 0] ^= 1                                   # differs from row 2 in the lowest bit only
    u[4] = 0xFFFFFFFF
    v[4, :] = 0xFFFFFFFF
    v[4, 0] = 0xFFFFFFFE                           # B^nv - 2
    u[5, :] = 0
    u[5, -1] = 1                                   # u = B^(nu-1)
    _check_batch(bi, orc, u, v)


def _newton_steps(k1, h):
    """Steps of the shifted-inverse schedule (start at scale k1 + 2, grow by
    m = min(h - cur, cur - k1 - 1) limbs per step -- one guard limb -- until
    the scale reaches h)."""
    cur = min(k1 + 2, h)
    steps = 0
    while cur < h:
        cur += min(h - cur, cur - k1 - 1)
        steps += 1
    return steps


def _prec(x):
    nz = np.nonzero(x)[0]
    return int(nz[-1]) + 1 if len(nz) else 0


def test_ragged_counters(bi, orc):
    """The diagnostic entry point gives the same bytes as the plain ragged
    call, Newton step counts that follow the schedule, bounded fix-up and
    quotient corrections, and zeros where no Newton iteration runs."""
    import torch
    g = np.random.default_rng(77)
    shapes = [(3, 2), (5, 2), (40, 20), (100, 3), (257, 128), (1000, 500), (2000, 1000),
              (64, 64), (9, 1), (30, 4), (300, 299)]
    us, vs = [], []
    for nu, nv in shapes:
        us.append(rand_limbs(g, 1, nu)[0])
        v = rand_limbs(g, 1, nv)[0]
        v[-1] = max(v[-1], 1)
        vs.append(v)
    us[7][-1] = 0                      # u < v (same limb count, smaller top limb)
    vs[7][-1] = 0xFFFFFFFF
    vs[9][:] = 0                       # v = 0
    nu = np.array([len(x) for x in us], np.int64)
    nv = np.array([len(x) for x in vs], np.int64)
    u_off = np.concatenate([[0], np.cumsum(nu)]).astype(np.int64)
    v_off = np.concatenate([[0], np.cumsum(nv)]).astype(np.int64)
    U, V = np.concatenate(us), np.concatenate(vs)
    tuo, tvo = torch.from_numpy(u_off).cuda(), torch.from_numpy(v_off).cuda()
    plan = bi.DivPlan(nu, nv)
    q0, r0, s0 = plan(dev(U), tuo, dev(V), tvo)
    q1, r1, s1, cnt = plan.counters(dev(U), tuo, dev(V), tvo)
    assert torch.equal(q0, q1) and torch.equal(r0, r1) and torch.equal(s0, s1)
    q, r, st, cnt = host(q1), host(r1), s1.cpu().numpy(), cnt.cpu().numpy()
    for i in range(len(shapes)):
        wq, wr, ws = orc.divmod1(us[i], vs[i])
        assert st[i] == ws, i
        assert np.array_equal(q[u_off[i]:u_off[i + 1]], wq), i
        assert np.array_equal(r[v_off[i]:v_off[i + 1]], wr), i
        k1, h = _prec(vs[i]), _prec(us[i])
        if k1 <= 1 or h < k1:
            assert cnt[i].tolist() == [0, 0, 0, 0], i
            continue
        assert cnt[i, 0] == _newton_steps(k1, h), (i, cnt[i])
        assert 0 <= cnt[i, 1] <= cnt[i, 0], (i, cnt[i])      # negative-branch steps
        assert 0 <= cnt[i, 2] <= 3, (i, cnt[i])               # quotient corrections
        # MFMA work: none when every product has operands of at most 64 limbs;
        # otherwise below the digit pairs of ten full h x h products
        if h <= 64:
            assert cnt[i, 3] == 0, (i, cnt[i])
        else:
            assert 0 < cnt[i, 3] <= 10 * (4 * h) ** 2, (i, cnt[i])
    plan.close()


def test_negative_branch_steps(bi, orc):
    """Divisors whose shifted inverse overshoots, so the Newton steps take
    the paper's negative branch (w B^m minus a ceiling, with nonzero dropped
    limbs): B^(n-1) + small and B^(n-1) + B^(n/2) + 1; and powers of the base
    (e = 0 exactly at every step).  Exact results, and the counters show the
    branch was taken."""
    import torch
    g = np.random.default_rng(123)
    us, vs, kinds = [], [], []
    for nv in (5, 17, 100, 600, 1000):
        for kind in ("pow_plus", "pow_mid", "pow"):
            v = np.zeros(nv, np.uint32)
            v[-1] = 1
            if kind == "pow_plus":
                v[0] = int(g.integers(1, 1000))
            elif kind == "pow_mid":
                v[nv // 2] = 1
                v[0] = 1
            for urow in (rand_limbs(g, 1, 2 * nv)[0], np.full(2 * nv, 0xFFFFFFFF, np.uint32)):
                us.append(urow)
                vs.append(v)
                kinds.append((kind, nv))
    nu = np.array([len(x) for x in us], np.int64)
    nv_ = np.array([len(x) for x in vs], np.int64)
    u_off = np.concatenate([[0], np.cumsum(nu)]).astype(np.int64)
    v_off = np.concatenate([[0], np.cumsum(nv_)]).astype(np.int64)
    plan = bi.DivPlan(nu, nv_)
    q, r, st, cnt = plan.counters(dev(np.concatenate(us)), torch.from_numpy(u_off).cuda(),
                                  dev(np.concatenate(vs)), torch.from_numpy(v_off).cuda())
    q, r, st, cnt = host(q), host(r), st.cpu().numpy(), cnt.cpu().numpy()
    for i in range(len(us)):
        wq, wr, ws = orc.divmod1(us[i], vs[i])
        assert st[i] == ws == 0, i
        assert np.array_equal(q[u_off[i]:u_off[i + 1]], wq), (i, kinds[i])
        assert np.array_equal(r[v_off[i]:v_off[i + 1]], wr), (i, kinds[i])
        # (the 5-limb B^4 + B^2 + 1 starts below its inverse and stays there)
        if kinds[i] != ("pow_mid", 5):
            assert cnt[i, 0] >= 2 and cnt[i, 1] >= 1, (i, kinds[i], cnt[i])
    plan.close()



@pytest.mark.parametrize("nu,nv", [(16384, 8192), (16384, 2), (16384, 16000), (16384, 5000),
                                   (16383, 9)])
def test_dividends_2e19(bi, orc, nu, nv):
    """2^19-bit dividends (the top of the 2^15..2^19-bit range): random,
    all-ones and divisor-multiple dividends, checked by u = q v + r,
    0 <= r < v and against the oracle."""
    g = np.random.default_rng(nu + nv)
    u = rand_limbs(g, 3, nu)
    v = rand_limbs(g, 3, nv)
    v[:, -1] |= 1
    u[1] = 0xFFFFFFFF
    q, r, st = bi.divmod(dev(u), dev(v))
    q, r, st = host(q), host(r), st.cpu().numpy()
    for i in range(3):
        U, V, Q, R = _to_int(u[i]), _to_int(v[i]), _to_int(q[i]), _to_int(r[i])
        assert st[i] == 0 and U == Q * V + R and 0 <= R < V, i
        wq, wr, _ = orc.divmod1(u[i], v[i])
        assert np.array_equal(q[i], wq) and np.array_equal(r[i], wr), i


def test_ragged_with_2e19_dividends(bi, orc):
    """A ragged plan whose largest dividends have 16384 limbs (one
    work-group per CU for the whole launch), mixed with small divisions."""
    import torch
    g = np.random.default_rng(5)
    nu = np.array([16384, 3, 16384, 700, 9000, 40], np.int64)
    nv = np.array([8192, 2, 3, 350, 8999, 39], np.int64)
    us = [rand_limbs(g, 1, n)[0] for n in nu]
    vs = [rand_limbs(g, 1, n)[0] for n in nv]
    for v in vs:
        v[-1] |= 1
    u_off = np.concatenate([[0], np.cumsum(nu)]).astype(np.int64)
    v_off = np.concatenate([[0], np.cumsum(nv)]).astype(np.int64)
    plan = bi.DivPlan(nu, nv)
    q, r, st = plan(dev(np.concatenate(us)), torch.from_numpy(u_off).cuda(),
                    dev(np.concatenate(vs)), torch.from_numpy(v_off).cuda())
    q, r, st = host(q), host(r), st.cpu().numpy()
    for i in range(nu.size):
        wq, wr, _ = orc.divmod1(us[i], vs[i])
        assert st[i] == 0, i
        assert np.array_equal(q[u_off[i]:u_off[i + 1]], wq), i
        assert np.array_equal(r[v_off[i]:v_off[i + 1]], wr), i
    plan.close()


def test_shifted_inverse_2e19(bi, orc):
    g = np.random.default_rng(19)
    for nv, h in ((8192, 16384), (3, 16384)):
        v = rand_limbs(g, 2, nv)
        v[:, -1] |= 1
        w = host(bi.shinv(dev(v), h))
        for i in range(2):
            want, _ = orc.shinv1(v[i], h)
            assert np.array_equal(w[i], want), (nv, h, i)
