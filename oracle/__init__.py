"""CPU oracle for batched big-integer arithmetic -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does.

This module is a thin ctypes wrapper around ``oracle.c`` (plain C99 on 64-bit
digits, see the header of that file for what each function computes and which
passage of the paper it follows).  Arrays are numpy ``uint32`` limb arrays,
little-endian, one row per instance.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_u32p = ctypes.POINTER(ctypes.c_uint32)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i64 = ctypes.c_int64


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, no vectorisation tricks)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.orc_add.argtypes = [_u32p, _u32p, _u32p, _u32p, _i64]
        L.orc_sub.argtypes = [_u32p, _u32p, _u32p, _u32p, _i64]
        L.orc_mul.argtypes = [_u32p, _u32p, _i64, _u32p, _i64]
        L.orc_mullo.argtypes = [_u32p, _u32p, _u32p, _i64]
        L.orc_add6.argtypes = [_u32p, _u32p, _u32p, _u32p, _i64]
        L.orc_poly.argtypes = [_u32p, _u32p, _u32p, _i64]
        L.orc_divmod.argtypes = [_u32p, _u32p, _u32p, _i64, _u32p, _i64]
        L.orc_shinv.argtypes = [_u32p, _u32p, _i64, _i64]
        L.orc_digits.argtypes = [_u8p, _u32p, _i64, ctypes.c_int, _i64]
        L.orc_conv.argtypes = [_i64p, _u8p, _i64, _u8p, _i64]
        L.orc_recombine.argtypes = [_u32p, _i64, _i64p, _i64, ctypes.c_int]
        for f in ("orc_add", "orc_sub", "orc_mul", "orc_mullo", "orc_add6", "orc_poly", "orc_divmod",
                  "orc_shinv", "orc_digits", "orc_conv", "orc_recombine"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _row(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a


# ---- single-instance functions ------------------------------------------------

def add1(a, b):
    a, b = _row(a), _row(b)
    out = np.zeros_like(a)
    c = np.zeros(1, np.uint32)
    lib().orc_add(_p(out, _u32p), _p(c, _u32p), _p(a, _u32p), _p(b, _u32p), a.size)
    return out, int(c[0])


def sub1(a, b):
    a, b = _row(a), _row(b)
    out = np.zeros_like(a)
    c = np.zeros(1, np.uint32)
    lib().orc_sub(_p(out, _u32p), _p(c, _u32p), _p(a, _u32p), _p(b, _u32p), a.size)
    return out, int(c[0])


def mul1(a, b):
    a, b = _row(a), _row(b)
    out = np.zeros(a.size + b.size, np.uint32)
    lib().orc_mul(_p(out, _u32p), _p(a, _u32p), a.size, _p(b, _u32p), b.size)
    return out


def mullo1(a, b):
    a, b = _row(a), _row(b)
    assert a.size == b.size
    out = np.zeros(a.size, np.uint32)
    lib().orc_mullo(_p(out, _u32p), _p(a, _u32p), _p(b, _u32p), a.size)
    return out


def add6_1(a, b):
    a, b = _row(a), _row(b)
    out = np.zeros_like(a)
    c = np.zeros(1, np.uint32)
    lib().orc_add6(_p(out, _u32p), _p(c, _u32p), _p(a, _u32p), _p(b, _u32p), a.size)
    return out, int(c[0])


def poly1(a, b):
    a, b = _row(a), _row(b)
    assert a.size == b.size
    out = np.zeros_like(a)
    lib().orc_poly(_p(out, _u32p), _p(a, _u32p), _p(b, _u32p), a.size)
    return out


def divmod1(u, v):
    u, v = _row(u), _row(v)
    q = np.zeros(u.size, np.uint32)
    r = np.zeros(v.size, np.uint32)
    st = lib().orc_divmod(_p(q, _u32p), _p(r, _u32p), _p(u, _u32p), u.size, _p(v, _u32p), v.size)
    return q, r, int(st)


def shinv1(v, h):
    v = _row(v)
    w = np.zeros(h + 1, np.uint32)
    st = lib().orc_shinv(_p(w, _u32p), _p(v, _u32p), v.size, h)
    return w, int(st)


def digits1(a, w=7, D=None):
    a = _row(a)
    if D is None:
        D = -(-32 * a.size // w)
    out = np.zeros(D, np.uint8)
    lib().orc_digits(_p(out, _u8p), _p(a, _u32p), a.size, w, D)
    return out


def conv1(alpha, beta):
    alpha = np.ascontiguousarray(alpha, dtype=np.uint8)
    beta = np.ascontiguousarray(beta, dtype=np.uint8)
    c = np.zeros(max(alpha.size + beta.size - 1, 0), np.int64)
    lib().orc_conv(_p(c, _i64p), _p(alpha, _u8p), alpha.size, _p(beta, _u8p), beta.size)
    return c


def recombine1(c, nout, w=7):
    c = np.ascontiguousarray(c, dtype=np.int64)
    out = np.zeros(nout, np.uint32)
    st = lib().orc_recombine(_p(out, _u32p), nout, _p(c, _i64p), c.size, w)
    assert st == 0
    return out


# ---- batched helpers (one row per instance) ------------------------------------

def add(a, b):
    outs, cs = zip(*(add1(x, y) for x, y in zip(a, b)))
    return np.stack(outs), np.array(cs, np.uint32)


def sub(a, b):
    outs, cs = zip(*(sub1(x, y) for x, y in zip(a, b)))
    return np.stack(outs), np.array(cs, np.uint32)


def mul(a, b):
    return np.stack([mul1(x, y) for x, y in zip(a, b)])


def divmod_(u, v):
    qs, rs, st = zip(*(divmod1(x, y) for x, y in zip(u, v)))
    return np.stack(qs), np.stack(rs), np.array(st, np.int32)
