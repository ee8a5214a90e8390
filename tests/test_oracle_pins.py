"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself: Python's own
arbitrary-precision integers (an independent bignum library), brute force on
an edge alphabet of limbs, closed forms, algebraic invariants and residues
modulo small primes.  Each check is chosen so that a plausible slip in the
oracle (a dropped carry, a wrong index, a swapped operand, a missing
correction step) fails at least one of them.
"""
import itertools

import numpy as np
import pytest

from conftest import from_int, to_int

B = 1 << 32
EDGE = [0, 1, 2, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFE, 0xFFFFFFFF]

ADD_BACK_CASES = [
    # (u, v) pairs on which Knuth's Algorithm D (64-bit digits) needs the
    # add-back step (D6): q-hat survives the two-digit test of D3 and is still
    # one too large.  Found by a plain-Python search of Algorithm D over
    # structured digits; the expected results come from Python's divmod.
    (0x7fffffffffffffff000000000000000100000000000000028000000000000001,
     0x7fffffffffffffff00000000000000017fffffffffffffff),
    (0x8000000000000000ffffffffffffffff00000000ffffffff7fffffffffffffff8000000000000000,
     0x10000000000000001ffffffffffffffff),
    (0x80000000000000007fffffffffffffff00000000000000010000000100000000,
     0xffffffffffffffff00000000000000008000000000000000),
    (0xffffffffffffffffffffffffffffffff00000001000000007fffffffffffffff,
     0x800000000000000080000000000000000000000100000000),
]


def edge_values(n):
    for limbs in itertools.product(EDGE, repeat=n):
        yield np.array(limbs, np.uint32)


# ---- addition / subtraction --------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2])
def test_add_sub_edge_alphabet_bruteforce(orc, n):
    vals = list(edge_values(n))
    M = 1 << (32 * n)
    for a in vals:
        ia = to_int(a)
        for b in vals:
            ib = to_int(b)
            r, c = orc.add1(a, b)
            assert to_int(r) == (ia + ib) % M and c == (ia + ib) // M
            r, br = orc.sub1(a, b)
            assert to_int(r) == (ia - ib) % M and br == int(ia < ib)


def test_add_sub_edge_alphabet_three_limbs_sampled(orc):
    vals = list(edge_values(3))
    g = np.random.default_rng(5)
    M = 1 << 96
    for _ in range(4000):
        a = vals[g.integers(len(vals))]
        b = vals[g.integers(len(vals))]
        ia, ib = to_int(a), to_int(b)
        r, c = orc.add1(a, b)
        assert to_int(r) == (ia + ib) % M and c == (ia + ib) // M
        r, br = orc.sub1(a, b)
        assert to_int(r) == (ia - ib) % M and br == int(ia < ib)


@pytest.mark.parametrize("n", [1, 3, 7, 64, 1024, 4096])
def test_add_sub_random_vs_python(orc, n):
    g = np.random.default_rng(n)
    M = 1 << (32 * n)
    for _ in range(6):
        a = g.integers(0, B, n, dtype=np.uint64).astype(np.uint32)
        b = g.integers(0, B, n, dtype=np.uint64).astype(np.uint32)
        ia, ib = to_int(a), to_int(b)
        r, c = orc.add1(a, b)
        assert to_int(r) == (ia + ib) % M and c == (ia + ib) // M
        r, br = orc.sub1(a, b)
        assert to_int(r) == (ia - ib) % M and br == int(ia < ib)
        # invariants a + b - b = a and a - b + b = a, a + b = b + a
        s, _ = orc.add1(a, b)
        back, _ = orc.sub1(s, b)
        assert np.array_equal(back, a)
        d, _ = orc.sub1(a, b)
        back, _ = orc.add1(d, b)
        assert np.array_equal(back, a)
        s2, _ = orc.add1(b, a)
        assert np.array_equal(s, s2)


@pytest.mark.parametrize("n", [1, 2, 5, 1024])
def test_add_sub_closed_forms(orc, n):
    ones = np.full(n, 0xFFFFFFFF, np.uint32)
    one = from_int(1, n)
    zero = np.zeros(n, np.uint32)
    r, c = orc.add1(ones, one)           # (B^n - 1) + 1 = B^n: full ripple
    assert not r.any() and c == 1
    r, br = orc.sub1(zero, one)          # 0 - 1 = B^n - 1 with borrow
    assert np.array_equal(r, ones) and br == 1
    top = from_int(1 << (32 * (n - 1)), n)
    r, br = orc.sub1(top, one)           # B^(n-1) - 1: borrow ripples to the top
    assert to_int(r) == (1 << (32 * (n - 1))) - 1 and br == 0


def test_add_sub_carry_adversarial_rows(orc):
    from paper_2607_28897_amd import inputs
    g = inputs.rng(77)
    n = 2048
    M = 1 << (32 * n)
    for _ in range(4):
        a = inputs.carry_adversarial_row(g, n, max_run=512)
        b = inputs.carry_adversarial_row(g, n, max_run=512)
        ia, ib = to_int(a), to_int(b)
        r, c = orc.add1(a, b)
        assert to_int(r) == (ia + ib) % M and c == (ia + ib) // M
        r, br = orc.sub1(a, b)
        assert to_int(r) == (ia - ib) % M and br == int(ia < ib)


# ---- multiplication -----------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2])
def test_mul_edge_alphabet_bruteforce(orc, n):
    vals = list(edge_values(n))
    for a in vals:
        ia = to_int(a)
        for b in vals:
            assert to_int(orc.mul1(a, b)) == ia * to_int(b)


@pytest.mark.parametrize("na,nb", [(1, 1), (3, 1), (1, 4), (7, 9), (64, 64), (1024, 1024), (333, 1000), (4096, 4096)])
def test_mul_random_vs_python(orc, na, nb):
    g = np.random.default_rng(na * 7919 + nb)
    for _ in range(3):
        a = g.integers(0, B, na, dtype=np.uint64).astype(np.uint32)
        b = g.integers(0, B, nb, dtype=np.uint64).astype(np.uint32)
        p = orc.mul1(a, b)
        assert p.size == na + nb
        assert to_int(p) == to_int(a) * to_int(b)


def test_mul_2e19_bits_vs_python(orc):
    g = np.random.default_rng(19)
    a = g.integers(0, B, 16384, dtype=np.uint64).astype(np.uint32)
    b = g.integers(0, B, 16384, dtype=np.uint64).astype(np.uint32)
    assert to_int(orc.mul1(a, b)) == to_int(a) * to_int(b)


@pytest.mark.parametrize("n", [1, 2, 3, 100, 1024])
def test_mul_closed_form_all_ones(orc, n):
    # (B^n - 1)^2 = B^2n - 2 B^n + 1: limbs [1, 0 x (n-1), 0xFFFFFFFE, 0xFFFFFFFF x (n-1)]
    ones = np.full(n, 0xFFFFFFFF, np.uint32)
    p = orc.mul1(ones, ones)
    want = np.concatenate([[1], np.zeros(n - 1), [0xFFFFFFFE], np.full(n - 1, 0xFFFFFFFF)]).astype(np.uint32)
    assert np.array_equal(p, want)


def test_mul_identities(orc):
    g = np.random.default_rng(3)
    n = 257
    a = g.integers(0, B, n, dtype=np.uint64).astype(np.uint32)
    b = g.integers(0, B, n, dtype=np.uint64).astype(np.uint32)
    c = g.integers(0, B, n, dtype=np.uint64).astype(np.uint32)
    zero = np.zeros(n, np.uint32)
    one = from_int(1, n)
    assert not orc.mul1(a, zero).any()
    assert np.array_equal(orc.mul1(a, one)[:n], a) and not orc.mul1(a, one)[n:].any()
    # a * B^j is a limb shift, a * 2^s a bit shift
    j = 37
    bj = from_int(1 << (32 * j), n)
    assert np.array_equal(orc.mul1(a, bj)[j:j + n], a)
    s = 13
    assert to_int(orc.mul1(a, from_int(1 << s, n))) == to_int(a) << s
    # commutativity and distributivity a(b + c) = ab + ac
    assert np.array_equal(orc.mul1(a, b), orc.mul1(b, a))
    bc, carry = orc.add1(b, c)
    bc = np.append(bc, np.uint32(carry))
    lhs = to_int(orc.mul1(a, bc))
    rhs = to_int(orc.add1(np.append(orc.mul1(a, b), 0).astype(np.uint32),
                          np.append(orc.mul1(a, c), 0).astype(np.uint32))[0])
    assert lhs == rhs


@pytest.mark.parametrize("p", [2**32 - 1, 2**32 + 1, 2**31 - 1, 998244353])
def test_mul_residues(orc, p):
    g = np.random.default_rng(p % 1000)
    for n in (5, 640):
        a = g.integers(0, B, n, dtype=np.uint64).astype(np.uint32)
        b = g.integers(0, B, n + 3, dtype=np.uint64).astype(np.uint32)
        prod = orc.mul1(a, b)
        # residue by Horner over limbs, independent of Python's big multiply
        def res(x):
            r = 0
            for limb in x[::-1]:
                r = (r * (B % p) + int(limb)) % p
            return r
        assert res(prod) == (res(a) * res(b)) % p


def test_mullo(orc):
    g = np.random.default_rng(11)
    for m in (1, 2, 9, 300):
        a = g.integers(0, B, m, dtype=np.uint64).astype(np.uint32)
        b = g.integers(0, B, m, dtype=np.uint64).astype(np.uint32)
        assert to_int(orc.mullo1(a, b)) == (to_int(a) * to_int(b)) % (1 << (32 * m))


# ---- division -----------------------------------------------------------------------

def _check_divmod(orc, u, v):
    q, r, st = orc.divmod1(u, v)
    iu, iv = to_int(u), to_int(v)
    assert st == 0
    iq, ir = to_int(q), to_int(r)
    # u = q v + r with 0 <= r < v determines (q, r) uniquely
    assert iu == iq * iv + ir and 0 <= ir < iv
    assert (iq, ir) == divmod(iu, iv)


@pytest.mark.parametrize("n", [1, 2])
def test_divmod_edge_alphabet_bruteforce(orc, n):
    vals = list(edge_values(n))
    for u in vals:
        for v in vals:
            if to_int(v) == 0:
                continue
            _check_divmod(orc, u, v)
            _check_divmod(orc, np.concatenate([u, u]), v)


@pytest.mark.parametrize("nu,nv", [(1, 1), (2, 1), (3, 2), (4, 2), (9, 4), (64, 32), (200, 7), (1000, 500), (4096, 2048)])
def test_divmod_random_vs_python(orc, nu, nv):
    g = np.random.default_rng(nu * 31 + nv)
    for _ in range(4):
        u = g.integers(0, B, nu, dtype=np.uint64).astype(np.uint32)
        v = g.integers(0, B, nv, dtype=np.uint64).astype(np.uint32)
        if not v.any():
            v[0] = 1
        _check_divmod(orc, u, v)
        # divisor with a small top limb exercises normalisation shifts
        v2 = v.copy()
        v2[-1] = 1 + (v2[-1] % 3)
        _check_divmod(orc, u, v2)


def test_divmod_knuth_add_back_cases(orc):
    # Divisors whose top digits make q-hat overshoot: (B^2n - 1) / (B^n - 1) = B^n + 1
    for n in (2, 3, 8):
        u = np.full(2 * n, 0xFFFFFFFF, np.uint32)
        v = np.full(n, 0xFFFFFFFF, np.uint32)
        q, r, _ = orc.divmod1(u, v)
        assert to_int(q) == (1 << (32 * n)) + 1 and not r.any()
    # u = 2^(64k) * (something) with divisor 0x80000000_00000000 ... patterns
    g = np.random.default_rng(99)
    for _ in range(200):
        nv = int(g.integers(2, 6))
        nu = nv + int(g.integers(0, 5))
        v = g.choice(np.array(EDGE, np.uint32), nv)
        u = g.choice(np.array(EDGE, np.uint32), nu)
        if to_int(v) == 0:
            continue
        _check_divmod(orc, u, v)


def test_divmod_add_back_step(orc):
    for u, v in ADD_BACK_CASES:
        nu, nv = -(-u.bit_length() // 32), -(-v.bit_length() // 32)
        q, r, st = orc.divmod1(from_int(u, nu), from_int(v, nv))
        assert st == 0 and (to_int(q), to_int(r)) == divmod(u, v)


def test_divmod_special_cases(orc):
    g = np.random.default_rng(4)
    u = g.integers(0, B, 50, dtype=np.uint64).astype(np.uint32)
    v = g.integers(0, B, 20, dtype=np.uint64).astype(np.uint32)
    # v = 1
    q, r, _ = orc.divmod1(u, from_int(1, 20))
    assert np.array_equal(q, u) and not r.any()
    # u < v
    small = from_int(to_int(v) - 1, 50)
    q, r, _ = orc.divmod1(small, v)
    assert not q.any() and to_int(r) == to_int(v) - 1
    # u = v
    q, r, _ = orc.divmod1(from_int(to_int(v), 50), v)
    assert to_int(q) == 1 and not r.any()
    # zero divisor: status 1, q = 0, r = low limbs of u
    q, r, st = orc.divmod1(u, np.zeros(20, np.uint32))
    assert st == 1 and not q.any() and np.array_equal(r, u[:20])


def test_shinv(orc):
    g = np.random.default_rng(8)
    for nv, h in ((1, 1), (1, 5), (3, 3), (3, 4), (5, 40), (64, 130)):
        v = g.integers(0, B, nv, dtype=np.uint64).astype(np.uint32)
        v[-1] |= 1
        w, st = orc.shinv1(v, h)
        iw, iv = to_int(w), to_int(v)
        Bh = 1 << (32 * h)
        assert st == 0 and iv * iw <= Bh < iv * (iw + 1)


# ---- digit form ------------------------------------------------------------------------

@pytest.mark.parametrize("w", [7, 6])
@pytest.mark.parametrize("n", [1, 7, 8, 100, 1024])
def test_digits_reconstruct(orc, n, w):
    g = np.random.default_rng(n + w)
    a = g.integers(0, B, n, dtype=np.uint64).astype(np.uint32)
    d = orc.digits1(a, w)
    assert d.size == -(-32 * n // w)
    assert int(d.max()) < (1 << w)
    ia = to_int(a)
    # digit k = floor(a / 2^(w k)) mod 2^w, from Python's shifts
    want = [(ia >> (w * k)) & ((1 << w) - 1) for k in range(d.size)]
    assert d.tolist() == want
    assert sum(int(x) << (w * k) for k, x in enumerate(d)) == ia


def test_conv_vs_numpy_convolve(orc):
    g = np.random.default_rng(12)
    for Na, Nb in ((1, 1), (5, 3), (64, 64), (300, 17), (1000, 999)):
        al = g.integers(0, 128, Na).astype(np.uint8)
        be = g.integers(0, 128, Nb).astype(np.uint8)
        c = orc.conv1(al, be)
        assert np.array_equal(c, np.convolve(al.astype(np.int64), be.astype(np.int64)))


def test_recombine_gives_the_product(orc):
    g = np.random.default_rng(13)
    for na, nb in ((1, 1), (7, 7), (33, 90), (512, 512)):
        a = g.integers(0, B, na, dtype=np.uint64).astype(np.uint32)
        b = g.integers(0, B, nb, dtype=np.uint64).astype(np.uint32)
        for w in (7, 6):
            c = orc.conv1(orc.digits1(a, w), orc.digits1(b, w))
            p = orc.recombine1(c, na + nb, w)
            assert to_int(p) == to_int(a) * to_int(b)


def test_conv_all_ones_bound(orc):
    # all-ones operands: every 7-bit digit is 127 except the top partial digit;
    # coefficients stay below min(Na, Nb) * 127^2 < 2^31
    n = 2048
    ones = np.full(n, 0xFFFFFFFF, np.uint32)
    d = orc.digits1(ones, 7)
    assert (d[:-1] == 127).all()
    c = orc.conv1(d, d)
    assert int(c.max()) <= d.size * 127 * 127 < 2**31
    assert to_int(orc.recombine1(c, 2 * n)) == ((1 << (32 * n)) - 1) ** 2


# ---- fused workloads of the evaluation: 6-Add and Poly (Section 6) ----------------

@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 1000])
def test_add6_vs_python(orc, n):
    # six additions alternating the inputs: 4a + 3b, reduced mod B^n, with the
    # number of additions that carried out of the top limb
    g = np.random.default_rng(700 + n)
    M = 1 << (32 * n)
    for _ in range(6):
        a = g.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        b = g.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        r, ovf = orc.add6_1(a, b)
        ia, ib = to_int(a), to_int(b)
        assert to_int(r) == (4 * ia + 3 * ib) % M
        # each partial sum is taken mod M, so the count is the floor of the
        # exact result: 4a + 3b = r + ovf * M
        assert ovf == (4 * ia + 3 * ib) // M


def test_add6_closed_forms(orc):
    n = 5
    ones = np.full(n, 0xFFFFFFFF, np.uint32)
    r, ovf = orc.add6_1(ones, ones)           # 7 (B^n - 1) = 6 B^n + (B^n - 7)
    assert to_int(r) == (1 << (32 * n)) - 7 and ovf == 6
    z = np.zeros(n, np.uint32)
    r, ovf = orc.add6_1(z, z)
    assert not r.any() and ovf == 0
    one = from_int(1, n)
    r, ovf = orc.add6_1(one, z)               # 4
    assert to_int(r) == 4 and ovf == 0


@pytest.mark.parametrize("n", [1, 2, 5, 33, 300])
def test_poly_vs_python(orc, n):
    g = np.random.default_rng(900 + n)
    M = 1 << (32 * n)
    for _ in range(4):
        a = g.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        b = g.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        ia, ib = to_int(a), to_int(b)
        want = ((ia * ia + ib) * (ib * ib + ib) + ia * ib) % M
        assert to_int(orc.poly1(a, b)) == want


def test_poly_special_values(orc):
    n = 4
    M = 1 << (32 * n)
    one, z = from_int(1, n), np.zeros(n, np.uint32)
    assert to_int(orc.poly1(one, one)) == 5                  # (1+1)(1+1) + 1
    b = from_int(123456789123456789, n)
    ib = to_int(b)
    assert to_int(orc.poly1(z, b)) == (ib * (ib * ib + ib)) % M   # b^3 + b^2
    assert to_int(orc.poly1(b, z)) == 0                      # (a^2)(0) + 0
    m1 = from_int(M - 1, n)                                  # a = -1 mod M: a*a = 1, a*b = -b
    assert to_int(orc.poly1(m1, b)) == ((1 + ib) * (ib * ib + ib) - ib) % M
