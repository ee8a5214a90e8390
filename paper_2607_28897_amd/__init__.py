"""Batched big-integer arithmetic on AMD MI355X (gfx950).

Python binding of the C-ABI in ``include/bigint_rocm.h``; it only marshals
arguments (device pointers, sizes, the current torch stream) and allocates
output tensors.  Every step of the arithmetic runs in the HIP library
``_lib/libbigint_rocm.so``; if that library is missing the binding raises.

Method: Oancea and Watt, "High-Level Big Integer Arithmetic in Futhark for
GPUs" -- addition and subtraction as a carry scan (Section 5.1),
multiplication as a digit convolution plus carry resolution (Section 5.2),
division through the whole shifted inverse by Newton steps (Section 5.3).

Tensors: limbs are little-endian u32 stored in ``torch.int32`` (or
``torch.uint32``) CUDA tensors, one row per instance.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "lib", "add", "sub", "mul", "divmod", "digits7", "conv7", "shinv",
    "MulPlan", "DivPlan", "autotune", "autotune_load", "set_mfma_config", "mfma_config",
    "set_mfma_tile", "mfma_tile", "BigIntError",
    "mullo", "add6", "poly",
    "MUL_AUTO", "MUL_PLAIN", "MUL_MFMA", "MUL_KARATSUBA",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libbigint_rocm.so")

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4
DIV_OK, DIVZERO = 0, 1
MUL_AUTO, MUL_PLAIN, MUL_MFMA, MUL_KARATSUBA = 0, 1, 2, 3
OP_MUL, OP_DIVMOD = 1, 2
PLAN_DEFAULT, PLAN_PLAIN, PLAN_NO_GRAPH = 0, 1, 2
MFMA_MAX_LIMBS = 18432
DIV_MAX_LIMBS = 16384


class BigIntError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = lib().bigint_strerror(code).decode()
        if code == EHIP:
            msg += f" (hipError {lib().bigint_last_hip_error()})"
        super().__init__(f"{what}: {msg} [{code}]")
        self.code = code


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_pint = ctypes.POINTER(ctypes.c_int)
_int = ctypes.c_int


def lib() -> ctypes.CDLL:
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime (same SONAME as the system one);
        # loading torch first makes this library bind to that copy, so both
        # share one runtime, one device context and one set of streams
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2607_28897_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "bigint_version": ([], _int),
            "bigint_strerror": ([_int], ctypes.c_char_p),
            "bigint_last_hip_error": ([], _int),
            "bigint_add": ([_vp, _vp, _vp, _vp, _i64, _i64, _vp], _int),
            "bigint_sub": ([_vp, _vp, _vp, _vp, _i64, _i64, _vp], _int),
            "bigint_mul": ([_vp, _vp, _i64, _vp, _i64, _i64, _int, _vp], _int),
            "bigint_divmod": ([_vp, _vp, _vp, _vp, _i64, _vp, _i64, _i64, _vp], _int),
            "bigint_divmod_noalloc": ([_vp, _vp, _vp, _vp, _i64, _vp, _i64, _i64, _vp], _int),
            "bigint_plan_create": ([ctypes.POINTER(_vp), _int, _vp, _vp, _i64, _int], _int),
            "bigint_plan_workspace_size": ([_vp, ctypes.POINTER(ctypes.c_size_t)], _int),
            "bigint_plan_set_workspace": ([_vp, _vp, ctypes.c_size_t], _int),
            "bigint_plan_destroy": ([_vp], _int),
            "bigint_plan_info": ([_vp, _vp, _int], _int),
            "bigint_mul_ragged": ([_vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp], _int),
            "bigint_plan_segments": ([_vp, _vp, _int, _vp], _int),
            "bigint_mul_ragged_segment": ([_vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _int, _vp], _int),
            "bigint_divmod_ragged": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp], _int),
            "bigint_autotune": ([ctypes.c_char_p, _int], _int),
            "bigint_autotune_load": ([ctypes.c_char_p], _int),
            "bigint_digits7": ([_vp, _vp, _i64, _i64, _i64, _vp], _int),
            "bigint_conv7": ([_vp, _vp, _i64, _vp, _i64, _i64, _vp], _int),
            "bigint_shinv": ([_vp, _vp, _i64, _i64, _i64, _vp], _int),
            "bigint_set_mfma_config": ([_int, _int, _int], _int),
            "bigint_mfma_config": ([_i64, _i64, _pint, _pint, _pint], _int),
            "bigint_mfma_split_parts": ([_i64, _i64, _i64, _pint], _int),
            "bigint_set_mfma_tile": ([_int], _int),
            "bigint_mfma_tile": ([_i64, _i64], _int),
            "bigint_mullo": ([_vp, _vp, _vp, _i64, _i64, _vp], _int),
            "bigint_add6": ([_vp, _vp, _vp, _vp, _i64, _i64, _vp], _int),
            "bigint_poly": ([_vp, _vp, _vp, _i64, _i64, _vp], _int),
            "bigint_diag_mfma_rate": ([_vp, _i64, _i64, _int, _vp], _int),
            "bigint_diag_mad_rate": ([_vp, _i64, _i64, _vp], _int),
            "bigint_diag_divmod_ragged": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64,
                                           _vp, _vp], _int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(code: int, what: str):
    if code != OK:
        raise BigIntError(code, what)


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _limbs(t, name):
    """The tensor as u32 limbs.  64-bit limb tensors (int64/uint64) are viewed
    as twice as many u32 limbs: on little-endian hosts and gfx950 the bytes of
    n u64 digits are those of 2n u32 limbs."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    wide = (torch.int64, getattr(torch, "uint64", torch.int64))
    narrow = (torch.int32, getattr(torch, "uint32", torch.int32))
    if t.dtype not in wide + narrow:
        raise TypeError(f"{name} must hold 32- or 64-bit limbs, got {t.dtype}")
    if not t.is_contiguous():
        t = t.contiguous()
    if t.dtype in wide:
        t = t.view(torch.int32)
    return t


def _wide(t):
    """The dtype to hand results back in: 64-bit limb inputs get 64-bit limb
    outputs (a view of the same bytes), 32-bit inputs 32-bit outputs."""
    torch = _torch()
    return t.dtype if t.dtype in (torch.int64, getattr(torch, "uint64", torch.int64)) else None


def _back(t, dtype):
    return t if dtype is None else t.view(dtype)


def _rows(t):
    return (1, t.numel()) if t.dim() == 1 else (t.shape[0], t.shape[1])


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def add(a, b, out=None):
    """(a + b mod 2^(32n), carry) for every row; a, b: [batch, n]."""
    return _addsub(lib().bigint_add, a, b, out, "bigint_add")


def sub(a, b, out=None):
    """(a - b mod 2^(32n), borrow) for every row."""
    return _addsub(lib().bigint_sub, a, b, out, "bigint_sub")


def _addsub(fn, a, b, out, what):
    torch = _torch()
    wd = _wide(a)
    a, b = _limbs(a, "a"), _limbs(b, "b")
    if a.shape != b.shape:
        raise ValueError("a and b must have the same shape")
    batch, n = _rows(a)
    out = torch.empty_like(a) if out is None else _limbs(out, "out")
    carry = torch.empty(batch, dtype=torch.int32, device=a.device)
    _check(fn(_p(out), _p(carry), _p(a), _p(b), n, batch, _stream()), what)
    return _back(out, wd), carry


def mul(a, b, algo: int = MUL_AUTO):
    """Full products a * b row by row: [batch, na] x [batch, nb] -> [batch, na+nb]."""
    torch = _torch()
    wd = _wide(a)
    a, b = _limbs(a, "a"), _limbs(b, "b")
    ba, na = _rows(a)
    bb, nb = _rows(b)
    if ba != bb:
        raise ValueError("batch mismatch")
    out = torch.empty((ba, na + nb), dtype=a.dtype, device=a.device)
    _check(lib().bigint_mul(_p(out), _p(a), na, _p(b), nb, ba, algo, _stream()), "bigint_mul")
    return _back(out if a.dim() == 2 else out.view(-1), wd)


def divmod(u, v):
    """(q, r, status): q = floor(u/v) ([batch, nu]), r = u - q v ([batch, nv])."""
    torch = _torch()
    wd = _wide(u)
    u, v = _limbs(u, "u"), _limbs(v, "v")
    bu, nu = _rows(u)
    bv, nv = _rows(v)
    if bu != bv:
        raise ValueError("batch mismatch")
    q = torch.empty((bu, nu), dtype=u.dtype, device=u.device)
    r = torch.empty((bu, nv), dtype=u.dtype, device=u.device)
    st = torch.empty(bu, dtype=torch.int32, device=u.device)
    _check(lib().bigint_divmod(_p(q), _p(r), _p(st), _p(u), nu, _p(v), nv, bu, _stream()),
           "bigint_divmod")
    return _back(q, wd), _back(r, wd), st


def digits7(a, D=None):
    """7-bit digits of every row (uint8 [batch, D])."""
    torch = _torch()
    a = _limbs(a, "a")
    batch, n = _rows(a)
    if D is None:
        D = (32 * n + 6) // 7
    out = torch.empty((batch, D), dtype=torch.uint8, device=a.device)
    _check(lib().bigint_digits7(_p(out), _p(a), n, D, batch, _stream()), "bigint_digits7")
    return out


def conv7(a, b):
    """Raw int32 digit-convolution coefficients of the MFMA multiply."""
    torch = _torch()
    a, b = _limbs(a, "a"), _limbs(b, "b")
    batch, na = _rows(a)
    _, nb = _rows(b)
    K = (32 * na + 6) // 7 + (32 * nb + 6) // 7 - 1
    c = torch.empty((batch, K), dtype=torch.int32, device=a.device)
    _check(lib().bigint_conv7(_p(c), _p(a), na, _p(b), nb, batch, _stream()), "bigint_conv7")
    return c


def shinv(v, h: int):
    """floor(2^(32h) / v) per row: [batch, h+1] limbs."""
    torch = _torch()
    v = _limbs(v, "v")
    batch, nv = _rows(v)
    w = torch.empty((batch, h + 1), dtype=v.dtype, device=v.device)
    _check(lib().bigint_shinv(_p(w), _p(v), nv, h, batch, _stream()), "bigint_shinv")
    return w


def set_mfma_config(strips_per_band: int = 0, waves: int = 0, digit_bits: int = 0):
    _check(lib().bigint_set_mfma_config(strips_per_band, waves, digit_bits), "bigint_set_mfma_config")


def mullo(a, b):
    """a * b mod B^n row by row ([batch, n] x [batch, n] -> [batch, n])."""
    torch = _torch()
    wd = _wide(a)
    a, b = _limbs(a, "a"), _limbs(b, "b")
    ba, n = _rows(a)
    bb, nb = _rows(b)
    if ba != bb or n != nb:
        raise ValueError("shape mismatch")
    out = torch.empty((ba, n), dtype=a.dtype, device=a.device)
    _check(lib().bigint_mullo(_p(out), _p(a), _p(b), n, ba, _stream()), "bigint_mullo")
    return _back(out if a.dim() == 2 else out.view(-1), wd)


def add6(a, b, out=None):
    """The 6-Add workload: (4a + 3b) mod B^n by six dependent additions, and
    the count of additions that overflowed (uint32 per row)."""
    torch = _torch()
    wd = _wide(a)
    a, b = _limbs(a, "a"), _limbs(b, "b")
    ba, n = _rows(a)
    if b.shape != a.shape:
        raise ValueError("shape mismatch")
    out = torch.empty_like(a) if out is None else _limbs(out, "out")
    ovf = torch.empty(ba, dtype=torch.int32, device=a.device)
    _check(lib().bigint_add6(_p(out), _p(ovf), _p(a), _p(b), n, ba, _stream()), "bigint_add6")
    return _back(out, wd), ovf


def poly(a, b):
    """The Poly workload: ((a a + b)(b b + b) + a b) mod B^n row by row."""
    torch = _torch()
    wd = _wide(a)
    a, b = _limbs(a, "a"), _limbs(b, "b")
    ba, n = _rows(a)
    if b.shape != a.shape:
        raise ValueError("shape mismatch")
    out = torch.empty_like(a)
    _check(lib().bigint_poly(_p(out), _p(a), _p(b), n, ba, _stream()), "bigint_poly")
    return _back(out, wd)


def set_mfma_tile(tile: int = 0):
    """MFMA tile of the next calls on this thread: 16, 32, or 0 (tuned)."""
    _check(lib().bigint_set_mfma_tile(tile), "bigint_set_mfma_tile")


def mfma_tile(na: int, nb: int) -> int:
    """The MFMA tile (16 or 32) bigint_mul uses for an na x nb product."""
    t = lib().bigint_mfma_tile(na, nb)
    if t < 0:
        raise BigIntError(t, "bigint_mfma_tile")
    return t


def mfma_config(na: int, nb: int):
    """(strips_per_band, waves, digit_bits) that bigint_mul uses for na x nb."""
    import ctypes
    p, w, d = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().bigint_mfma_config(na, nb, ctypes.byref(p), ctypes.byref(w), ctypes.byref(d)),
           "bigint_mfma_config")
    return p.value, w.value, d.value


def mfma_split_parts(na: int, nb: int, batch: int) -> int:
    """Work-groups per instance bigint_mul's MFMA path uses for this batch."""
    import ctypes
    k = ctypes.c_int()
    _check(lib().bigint_mfma_split_parts(na, nb, batch, ctypes.byref(k)), "bigint_mfma_split_parts")
    return k.value


def autotune(cache_path: str | None = None, flags: int = 0):
    _check(lib().bigint_autotune(cache_path.encode() if cache_path else None, flags), "bigint_autotune")


def autotune_load(cache_path: str | None):
    """Load a table written by autotune(); None restores the built-in table."""
    _check(lib().bigint_autotune_load(cache_path.encode() if cache_path else None),
           "bigint_autotune_load")


class _Plan:
    op = 0

    def __init__(self, len_a, len_b, flags: int = PLAN_DEFAULT):
        import numpy as np
        la = np.ascontiguousarray(len_a, dtype=np.int64)
        lb = np.ascontiguousarray(len_b, dtype=np.int64)
        if la.shape != lb.shape:
            raise ValueError("length arrays differ in shape")
        self.batch = la.size
        self.len_a, self.len_b = la, lb
        self._h = ctypes.c_void_p()
        _check(lib().bigint_plan_create(ctypes.byref(self._h), self.op,
                                        la.ctypes.data_as(ctypes.c_void_p),
                                        lb.ctypes.data_as(ctypes.c_void_p), self.batch, flags),
               "bigint_plan_create")

    def workspace_size(self) -> int:
        n = ctypes.c_size_t()
        _check(lib().bigint_plan_workspace_size(self._h, ctypes.byref(n)), "bigint_plan_workspace_size")
        return n.value

    def set_workspace(self, buf):
        self._ws = buf
        _check(lib().bigint_plan_set_workspace(self._h, _p(buf), buf.numel() * buf.element_size()),
               "bigint_plan_set_workspace")

    def info(self) -> dict:
        """Launches per call, graphs instantiated so far, calls replayed from a graph."""
        import numpy as np
        v = np.zeros(3, np.int64)
        _check(lib().bigint_plan_info(self._h, v.ctypes.data_as(ctypes.c_void_p), 3), "bigint_plan_info")
        return {"launches_per_call": int(v[0]), "graphs_instantiated": int(v[1]),
                "graph_replays": int(v[2])}

    def close(self):
        if self._h:
            lib().bigint_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _offsets(lens, device):
    torch = _torch()
    import numpy as np
    off = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    return torch.from_numpy(off).to(device), int(off[-1])


class MulPlan(_Plan):
    """Ragged batch of products with fixed instance sizes."""
    op = OP_MUL

    def __call__(self, a, a_off, b, b_off, out=None, out_off=None):
        torch = _torch()
        if out_off is None:
            out_off, _ = _offsets(self.len_a + self.len_b, a.device)
        if out is None:
            # the total comes from the plan's host-side lengths (no device read)
            total = int(self.len_a.sum() + self.len_b.sum())
            out = torch.empty(total, dtype=a.dtype, device=a.device)
        _check(lib().bigint_mul_ragged(_p(out), _p(out_off), _p(a), _p(a_off), _p(b), _p(b_off),
                                       self.batch, self._h, _stream()), "bigint_mul_ragged")
        return out, out_off

    def segments(self) -> list:
        """The plan's segments on the MFMA-split path, one dict per segment:
        first queue position, instances, digit bits, strips per band, waves,
        resident work-groups, digit products, modelled busy fraction, and
        work-groups per instance (parts > 1: bands split, two launches)."""
        import numpy as np
        n = ctypes.c_int()
        _check(lib().bigint_plan_segments(self._h, None, 0, ctypes.byref(n)), "bigint_plan_segments")
        v = np.zeros((max(n.value, 1), 9), np.int64)
        _check(lib().bigint_plan_segments(self._h, v.ctypes.data_as(ctypes.c_void_p), n.value,
                                          ctypes.byref(n)), "bigint_plan_segments")
        keys = ("first", "instances", "digit_bits", "strips_per_band", "waves", "slots",
                "digit_products")
        return [dict({k: int(x) for k, x in zip(keys, row[:7])}, modelled_busy=float(row[7]) / 1e6,
                     parts=int(row[8])) for row in v[:n.value]]

    def run_segment(self, k, a, a_off, b, b_off, out, out_off):
        """Launch only segment k (no graph) into out."""
        _check(lib().bigint_mul_ragged_segment(_p(out), _p(out_off), _p(a), _p(a_off), _p(b), _p(b_off),
                                               self.batch, self._h, int(k), _stream()),
               "bigint_mul_ragged_segment")
        return out


class DivPlan(_Plan):
    """Ragged batch of divisions with fixed dividend / divisor sizes."""
    op = OP_DIVMOD

    def __call__(self, u, u_off, v, v_off):
        torch = _torch()
        q = torch.empty(int(self.len_a.sum()), dtype=u.dtype, device=u.device)
        r = torch.empty(int(self.len_b.sum()), dtype=u.dtype, device=u.device)
        st = torch.empty(self.batch, dtype=torch.int32, device=u.device)
        _check(lib().bigint_divmod_ragged(_p(q), _p(u_off), _p(r), _p(v_off), _p(st), _p(u),
                                          _p(u_off), _p(v), _p(v_off), self.batch, self._h,
                                          _stream()), "bigint_divmod_ragged")
        return q, r, st

    def counters(self, u, u_off, v, v_off):
        """The same division, plus per division [Newton steps, fix-up unit
        corrections, quotient corrections, int8 MFMA multiply-accumulates] as
        an int64 [batch, 4] tensor."""
        torch = _torch()
        q = torch.empty(int(self.len_a.sum()), dtype=u.dtype, device=u.device)
        r = torch.empty(int(self.len_b.sum()), dtype=u.dtype, device=u.device)
        st = torch.empty(self.batch, dtype=torch.int32, device=u.device)
        cnt = torch.empty((self.batch, 4), dtype=torch.int64, device=u.device)
        _check(lib().bigint_diag_divmod_ragged(_p(cnt), _p(q), _p(u_off), _p(r), _p(v_off), _p(st),
                                               _p(u), _p(u_off), _p(v), _p(v_off), self.batch,
                                               self._h, _stream()), "bigint_diag_divmod_ragged")
        return q, r, st, cnt
