"""GPU parity on seeded random shapes: operand lengths log-uniform over the
whole supported range, batches from one instance to a few hundred (so the
one-wave, one-work-group and split multiply paths all occur, and divisions
run on every work-group size), rows mixing uniform limbs with all-ones and
zero runs; every instance against the oracle, bit for bit."""
import numpy as np
import pytest

from gpu_util import dev, host, oracle_map

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bi():
    import paper_2607_28897_amd as m
    m.lib()
    return m


def _rows(g, batch, n):
    x = g.integers(0, 2**32, (batch, n), dtype=np.uint64).astype(np.uint32)
    for i in range(batch):
        mode = int(g.integers(0, 5))
        if mode == 1:
            x[i] = 0xFFFFFFFF
        elif mode in (2, 3):                # a run of all-ones or zero limbs
            k = int(g.integers(0, n))
            x[i, k:k + int(g.integers(1, n + 1))] = 0xFFFFFFFF if mode == 2 else 0
    return x


def _len(g, lo, hi, big=False):
    # log-uniform on [lo, hi], or on [hi / 8, hi] for the cases meant to be large
    lo = max(lo, hi // 8) if big else lo
    return int(min(hi, max(lo, round(np.exp(g.uniform(np.log(lo), np.log(hi + 1)))))))


# limb products the oracle may spend per case (a few hundred ms on the host pool)
BUDGET = 4e9


ALGOS = ["auto", "mfma", "plain", "karatsuba"]


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("algo", ALGOS)
def test_mul_random_shapes(bi, orc, seed, algo):
    g = np.random.default_rng(5000 + 97 * seed + ALGOS.index(algo))
    big = seed % 2 == 1
    na = _len(g, 1, 18432, big)
    nb = na if algo == "karatsuba" else _len(g, 1, 18432, big and seed % 4 == 1)
    if algo == "karatsuba":
        na = nb = max(na, 2)
    if algo == "plain" and na + nb > 32768:
        nb = 32768 - na
    batch = int(max(1, min(int(g.integers(1, 301)), BUDGET // (na * nb))))
    a = _rows(g, batch, na)
    b = _rows(g, batch, nb)
    code = {"auto": bi.MUL_AUTO, "mfma": bi.MUL_MFMA, "plain": bi.MUL_PLAIN,
            "karatsuba": bi.MUL_KARATSUBA}[algo]
    p = host(bi.mul(dev(a), dev(b), code))
    want = oracle_map(lambda i: orc.mul1(a[i], b[i]), range(batch))
    bad = [i for i in range(batch) if not np.array_equal(p[i], want[i])]
    assert not bad, (na, nb, batch, bad[:8])


@pytest.mark.parametrize("seed", range(16))
def test_divmod_random_shapes(bi, orc, seed):
    g = np.random.default_rng(7000 + seed)
    nu = _len(g, 1, 16384, seed % 2 == 1)
    x = g.uniform()
    if x < 0.45:
        nv = _len(g, 1, nu)                  # small divisors
    elif x < 0.85:
        nv = _len(g, max(1, nu // 8), nu)    # divisors of a few to all of the dividend's limbs
    else:
        nv = _len(g, 1, 16384)               # sometimes u < v
    work = max(1, nu - nv + 1) * (nu + nv)
    batch = int(max(1, min(int(g.integers(1, 257)), BUDGET // (8 * work))))
    u = _rows(g, batch, nu)
    v = _rows(g, batch, nv)
    for i in range(batch):                  # leading zero limbs in some divisors
        if g.uniform() < 0.2 and nv > 1:
            v[i, int(g.integers(1, nv)):] = 0
    v[:, 0] |= np.uint32(1)                 # never zero (division by zero has its own tests)
    q, r, st = bi.divmod(dev(u), dev(v))
    q, r, st = host(q), host(r), st.cpu().numpy()
    want = oracle_map(lambda i: orc.divmod1(u[i], v[i]), range(batch))
    bad = [i for i in range(batch)
           if not (np.array_equal(q[i], want[i][0]) and np.array_equal(r[i], want[i][1])
                   and st[i] == want[i][2])]
    assert not bad, (nu, nv, batch, bad[:8])
