"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a private copy of oracle/oracle.c (a dropped
carry, a wrong index, a missing correction step, ...), builds it on the CPU
and runs a compact set of the pins against it: Python integers, the edge
alphabet and closed forms.  Every mutant must fail at least one pin, and the
unmodified copy must pass them all.
"""
import ctypes
import itertools
import os
import subprocess

import numpy as np
import pytest

from conftest import from_int, to_int

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, text to find, replacement): each a slip someone could make
MUTANTS = [
    ("add drops the carry", "u128 t = (u128)x[i] + y[i] + c;", "u128 t = (u128)x[i] + y[i];"),
    ("add carry from the wrong half", "c = (uint64_t)(t >> 64);\n    }\n    /* an odd",
     "c = (uint64_t)(t >> 63) & 1;\n    }\n    /* an odd"),
    ("sub ignores the incoming borrow", "uint64_t d2 = d - br;", "uint64_t d2 = d;"),
    ("sub borrow test reversed", "uint64_t b1 = x[i] < y[i];", "uint64_t b1 = x[i] > y[i];"),
    ("mul drops the row carry", "r[i + mb] = c;", "r[i + mb] = 0;"),
    ("mul writes one column off", "r[i + j] = (uint64_t)t;", "r[i + j + (j == 1)] = (uint64_t)t;"),
    ("mul keeps only the low word", "u128 t = (u128)x[i] * y[j] + r[i + j] + c;",
     "u128 t = (u128)(x[i] * y[j]) + r[i + j] + c;"),
    ("divmod skips the q-hat correction", "qhat -= 1;\n            rhat += vn[n - 1];",
     "rhat += vn[n - 1];"),
    ("divmod skips the add-back", "if (b1 | b2) {\n            q[j] -= 1;", "if (0) {\n            q[j] -= 1;"),
    ("divmod unnormalises with the wrong shift", "r[n - 1] = un[n - 1] >> s;", "r[n - 1] = un[n - 1] >> (s ? s - 1 : 0);"),
    ("short division loses the remainder", "rem = (uint64_t)(t % d);", "rem = 0;"),
    ("digits read one bit too high", "d |= bit_of(a, n, (int64_t)w * k + t) << t;",
     "d |= bit_of(a, n, (int64_t)w * k + t + 1) << t;"),
    ("convolution uses i-j", "c[i + j] += (int64_t)alpha[i] * (int64_t)beta[j];",
     "c[i + j] += (int64_t)alpha[i] * (int64_t)beta[(j + 1) % Nb];"),
    ("recombination shifts by w-1", "int64_t bit = (int64_t)w * k;", "int64_t bit = (int64_t)(w - 1) * k;"),
]


def _build(tmp_path, text, tag):
    src = tmp_path / f"o_{tag}.c"
    lib = tmp_path / f"o_{tag}.so"
    src.write_text(text)
    subprocess.check_call(["gcc", "-std=c99", "-O1", "-fPIC", "-shared", "-o", str(lib), str(src)])
    return str(lib)


def _pins(path):
    """A compact pin set; returns the list of failed pins."""
    L = ctypes.CDLL(path)
    u32p, u8p, i64p = (ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint8),
                       ctypes.POINTER(ctypes.c_int64))
    P = lambda a, t: a.ctypes.data_as(t)  # noqa: E731
    fails = []

    def add(a, b):
        out = np.zeros_like(a); c = np.zeros(1, np.uint32)
        L.orc_add(P(out, u32p), P(c, u32p), P(a, u32p), P(b, u32p), ctypes.c_int64(a.size))
        return out, int(c[0])

    def sub(a, b):
        out = np.zeros_like(a); c = np.zeros(1, np.uint32)
        L.orc_sub(P(out, u32p), P(c, u32p), P(a, u32p), P(b, u32p), ctypes.c_int64(a.size))
        return out, int(c[0])

    def mul(a, b):
        out = np.zeros(a.size + b.size, np.uint32)
        L.orc_mul(P(out, u32p), P(a, u32p), ctypes.c_int64(a.size), P(b, u32p), ctypes.c_int64(b.size))
        return out

    def divmod_(u, v):
        q = np.zeros(u.size, np.uint32); r = np.zeros(v.size, np.uint32)
        L.orc_divmod(P(q, u32p), P(r, u32p), P(u, u32p), ctypes.c_int64(u.size), P(v, u32p),
                     ctypes.c_int64(v.size))
        return q, r

    g = np.random.default_rng(1)
    edge = np.array([0, 1, 2, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFE, 0xFFFFFFFF], np.uint32)
    vals = [np.array(t, np.uint32) for t in itertools.product(edge, repeat=2)]
    rnd = [g.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32) for n in (1, 3, 8, 33, 200)]
    M = lambda n: 1 << (32 * n)  # noqa: E731
    # add / sub vs Python
    for a, b in list(zip(vals, vals[::-1])) + [(x, x[::-1].copy()) for x in rnd]:
        r, c = add(a, b)
        if to_int(r) + c * M(a.size) != to_int(a) + to_int(b):
            fails.append("add"); break
    for a, b in list(zip(vals, vals[::-1])) + [(x, x[::-1].copy()) for x in rnd]:
        r, c = sub(a, b)
        if to_int(r) != (to_int(a) - to_int(b)) % M(a.size) or c != int(to_int(a) < to_int(b)):
            fails.append("sub"); break
    # mul vs Python, closed form
    for a, b in [(x, y) for x in rnd for y in rnd] + [(vals[-1], vals[-1])]:
        if to_int(mul(a, b)) != to_int(a) * to_int(b):
            fails.append("mul"); break
    # divmod: u = q v + r, 0 <= r < v
    for nu, nv in ((2, 1), (3, 2), (9, 4), (40, 17)):
        for _ in range(20):
            u = g.integers(0, 2**32, nu, dtype=np.uint64).astype(np.uint32)
            v = g.integers(0, 2**32, nv, dtype=np.uint64).astype(np.uint32)
            v[-1] = max(v[-1] >> g.integers(0, 32), 1)
            q, r = divmod_(u, v)
            if (to_int(q), to_int(r)) != divmod(to_int(u), to_int(v)):
                fails.append("divmod"); break
        if fails and fails[-1] == "divmod":
            break
    from test_oracle_pins import ADD_BACK_CASES
    for uu, vv in ADD_BACK_CASES:
        nu, nv = -(-uu.bit_length() // 32), -(-vv.bit_length() // 32)
        q, r = divmod_(from_int(uu, nu), from_int(vv, nv))
        if (to_int(q), to_int(r)) != divmod(uu, vv):
            fails.append("divmod add-back")
            break
    # digits / convolution / recombination against Python and numpy
    a = rnd[3]
    D = -(-32 * a.size // 7)
    d = np.zeros(D, np.uint8)
    L.orc_digits(P(d, u8p), P(a, u32p), ctypes.c_int64(a.size), ctypes.c_int(7), ctypes.c_int64(D))
    if [int(x) for x in d] != [(to_int(a) >> (7 * k)) & 127 for k in range(D)]:
        fails.append("digits")
    al, be = g.integers(0, 128, 50).astype(np.uint8), g.integers(0, 128, 31).astype(np.uint8)
    c = np.zeros(80, np.int64)
    L.orc_conv(P(c, i64p), P(al, u8p), ctypes.c_int64(50), P(be, u8p), ctypes.c_int64(31))
    if not np.array_equal(c, np.convolve(al.astype(np.int64), be.astype(np.int64))):
        fails.append("conv")
    out = np.zeros(20, np.uint32)
    L.orc_recombine(P(out, u32p), ctypes.c_int64(20), P(c, i64p), ctypes.c_int64(80), ctypes.c_int(7))
    if to_int(out) != sum(int(x) << (7 * k) for k, x in enumerate(c)) % M(20):
        fails.append("recombine")
    return fails


def test_unmodified_oracle_passes(tmp_path):
    text = open(SRC).read()
    assert _pins(_build(tmp_path, text, "orig")) == []


@pytest.mark.parametrize("name,find,repl", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, name, find, repl):
    text = open(SRC).read()
    assert text.count(find) == 1, f"mutation site not found: {name}"
    fails = _pins(_build(tmp_path, text.replace(find, repl), "m"))
    assert fails, f"no pin caught the mutant: {name}"
