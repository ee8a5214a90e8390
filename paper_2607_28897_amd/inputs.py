"""Seeded synthetic inputs for the batched big-integer path.

This module only draws random limbs and lays them out; it holds none of the
arithmetic of the method.  Both the GPU tests/benchmark and the CPU oracle
tests take their inputs from here, so the two sides always see identical
bytes.

Layout: uniform batches are ``[batch, n]`` ``uint32`` arrays, little-endian
limbs, one row per instance.  Ragged batches are a flat ``uint32`` array plus
an ``int64`` prefix-offset array of length ``batch + 1`` (instance ``i`` is
``flat[off[i]:off[i+1]]``).

The paper's evaluation uses random digits for addition and multiplication
because their cost depends only on the size (Section 6, datasets paragraph);
the five workloads below (sizes 2^15..2^19 bits) each draw from a fixed seed
(1000 .. 1004).
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 1000
LIMB_BITS = 32


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform(g: np.random.Generator, batch: int, n: int) -> np.ndarray:
    """Uniform random u32 limbs, shape [batch, n]."""
    return g.integers(0, 2**32, size=(batch, n), dtype=np.uint32)


def carry_adversarial_row(g: np.random.Generator, n: int, max_run: int = 4096) -> np.ndarray:
    """Runs of 0xFFFFFFFF of length U[1, max_run] alternating with single
    uniform random limbs, truncated to n limbs."""
    out = np.empty(n, np.uint32)
    i = 0
    while i < n:
        run = int(g.integers(1, max_run + 1))
        j = min(n, i + run)
        out[i:j] = 0xFFFFFFFF
        i = j
        if i < n:
            out[i] = np.uint32(g.integers(0, 2**32, dtype=np.uint64))
            i += 1
    return out


def compare_rows(a: np.ndarray, b: np.ndarray) -> int:
    """-1, 0, 1 as the integers a <, =, > b (same limb count); top limb first."""
    diff = np.nonzero(a != b)[0]
    if diff.size == 0:
        return 0
    k = diff[-1]
    return 1 if a[k] > b[k] else -1


def order_pairs(a: np.ndarray, b: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Swap rows so that a[i] >= b[i] as integers (for a - b without borrow)."""
    a = a.copy()
    b = b.copy()
    for i in range(a.shape[0]):
        if compare_rows(a[i], b[i]) < 0:
            a[i], b[i] = b[i].copy(), a[i].copy()
    return a, b


def log_uniform_bits(g: np.random.Generator, count: int, lo_bits: int, hi_bits: int) -> np.ndarray:
    """Bit lengths L = exp(U[ln lo, ln hi])."""
    return np.exp(g.uniform(np.log(lo_bits), np.log(hi_bits), size=count))


def limbs_for_bits(bits: np.ndarray) -> np.ndarray:
    return np.ceil(np.asarray(bits) / LIMB_BITS).astype(np.int64)


def ragged_uniform(g: np.random.Generator, lens: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    lens = np.asarray(lens, np.int64)
    off = np.zeros(lens.size + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    flat = g.integers(0, 2**32, size=int(off[-1]), dtype=np.uint32)
    return flat, off


def ragged_rows(flat: np.ndarray, off: np.ndarray):
    return [flat[off[i]:off[i + 1]] for i in range(off.size - 1)]


# ---- the five workloads ---------------------------------------------------------

def pairs_2e15():
    """64 pairs of 2^15-bit integers (1024 u32 limbs), uniform; for a - b the
    pair is ordered so that a >= b."""
    g = rng(SEED_BASE + 0)
    a = uniform(g, 64, 1024)
    b = uniform(g, 64, 1024)
    sa, sb = order_pairs(a, b)
    return {"a": a, "b": b, "sub_a": sa, "sub_b": sb, "n": 1024}


def pairs_2e17_mixed():
    """1024 pairs of 2^17-bit integers (4096 limbs): pairs 0..511 uniform,
    512..1023 carry-adversarial (runs of 0xFFFFFFFF)."""
    g = rng(SEED_BASE + 1)
    n = 4096
    a = uniform(g, 1024, n)
    b = uniform(g, 1024, n)
    for i in range(512, 1024):
        a[i] = carry_adversarial_row(g, n)
        b[i] = carry_adversarial_row(g, n)
    sa, sb = order_pairs(a, b)
    return {"a": a, "b": b, "sub_a": sa, "sub_b": sb, "n": n}


def pairs_2e19(batch: int = 256):
    """256 pairs of 2^19-bit integers (16384 limbs), uniform."""
    g = rng(SEED_BASE + 2)
    n = 16384
    a = uniform(g, batch, n)
    b = uniform(g, batch, n)
    return {"a": a, "b": b, "n": n}


def ragged_mul_2e15_2e19(batch: int = 4096):
    """4096 multiplications, bit lengths log-uniform in [2^15, 2^19] rounded
    up to 32-bit limbs, one length per pair (both operands), uniform limbs."""
    g = rng(SEED_BASE + 3)
    bits = log_uniform_bits(g, batch, 2**15, 2**19)
    lens = limbs_for_bits(bits)
    a, a_off = ragged_uniform(g, lens)
    b, b_off = ragged_uniform(g, lens)
    return {"a": a, "a_off": a_off, "b": b, "b_off": b_off, "lens": lens}


def ragged_div_2e16_2e18(batch: int = 512):
    """512 divisions: dividend bit length log-uniform in [2^16, 2^18] (limbs
    rounded up), divisor half as many limbs with a nonzero top limb."""
    g = rng(SEED_BASE + 4)
    bits = log_uniform_bits(g, batch, 2**16, 2**18)
    nu = limbs_for_bits(bits)
    nv = nu // 2
    u, u_off = ragged_uniform(g, nu)
    v, v_off = ragged_uniform(g, nv)
    for i in range(batch):
        top = v_off[i + 1] - 1
        while v[top] == 0:
            v[top] = np.uint32(g.integers(0, 2**32, dtype=np.uint64))
    return {"u": u, "u_off": u_off, "v": v, "v_off": v_off, "nu": nu, "nv": nv}
