"""CPU-only checks of the C-ABI library: it loads, exports every function the
header declares, and rejects bad arguments on the host before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bigint_rocm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bigint_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def bi():
    import paper_2607_28897_amd as m
    if not os.path.exists(m.LIB_PATH):
        pytest.skip("library not built")
    m.lib()
    return m


def test_every_declared_symbol_is_exported(bi):
    names = declared_functions()
    assert len(names) >= 20
    L = ctypes.CDLL(bi.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_strerror(bi):
    L = bi.lib()
    assert L.bigint_version() >= 10000
    for code in (0, -1, -2, -3, -4, 12345):
        assert isinstance(L.bigint_strerror(code), bytes)
    assert L.bigint_strerror(-1) == b"invalid argument"


def test_host_side_argument_checks(bi):
    L = bi.lib()
    p = ctypes.c_void_p(0x10000)           # never dereferenced: checks fail first
    q = ctypes.c_void_p(0x20000)
    EINVAL, EUNS = bi.EINVAL, bi.EUNSUPPORTED
    assert L.bigint_add(None, None, p, p, 8, 1, None) == EINVAL
    assert L.bigint_sub(p, None, None, p, 8, 1, None) == EINVAL
    assert L.bigint_add(p, None, p, p, 0, 1, None) == EINVAL
    assert L.bigint_add(p, None, p, p, 8, -1, None) == EINVAL
    assert L.bigint_add(p, None, p, p, 70000, 1, None) == EUNS
    # partial overlap of out with an input
    assert L.bigint_add(ctypes.c_void_p(0x10004), None, p, q, 4, 1, None) == EINVAL
    assert L.bigint_mul(None, p, 4, p, 4, 1, 0, None) == EINVAL
    assert L.bigint_mul(q, p, 0, p, 4, 1, 0, None) == EINVAL
    assert L.bigint_mul(q, p, 4, p, 4, 1, 7, None) == EINVAL
    assert L.bigint_mul(p, p, 4, q, 4, 1, 1, None) == EINVAL          # out overlaps a
    assert L.bigint_mul(ctypes.c_void_p(0x100000), p, 20000, q, 20000, 1,
                        bi.MUL_MFMA, None) == EUNS
    assert L.bigint_divmod(None, q, None, p, 4, p, 4, 1, None) == EINVAL
    assert L.bigint_divmod(ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000), None, p, 16385,
                           q, 4, 1, None) == EUNS
    assert L.bigint_shinv(ctypes.c_void_p(0x100000), p, 5, 4, 1, None) == EINVAL   # h < nv
    assert L.bigint_set_mfma_config(5, 0, 0) == EINVAL
    assert L.bigint_set_mfma_config(0, 3, 0) == EINVAL
    assert L.bigint_set_mfma_config(0, 0, 6) == EINVAL
    assert L.bigint_digits7(None, p, 4, 5, 1, None) == EINVAL
    assert L.bigint_diag_mfma_rate(None, 1, 1, 0, None) == EINVAL
    k = ctypes.c_int()
    assert L.bigint_mfma_split_parts(16384, 16384, 1, None) == EINVAL
    assert L.bigint_mfma_split_parts(0, 16384, 1, ctypes.byref(k)) == EINVAL
    assert L.bigint_mfma_split_parts(16384, 16384, 0, ctypes.byref(k)) == EINVAL


def test_plan_argument_checks(bi):
    L = bi.lib()
    h = ctypes.c_void_p()
    la = np.array([5, 0], np.int64)
    assert L.bigint_plan_create(None, bi.OP_MUL, None, None, 0, 0) == bi.EINVAL
    assert L.bigint_plan_create(ctypes.byref(h), 99, None, None, 0, 0) == bi.EINVAL
    assert L.bigint_plan_create(ctypes.byref(h), bi.OP_MUL, la.ctypes.data_as(ctypes.c_void_p),
                                la.ctypes.data_as(ctypes.c_void_p), 2, 0) == bi.EINVAL
    assert L.bigint_plan_create(ctypes.byref(h), bi.OP_MUL, None, None, 1, 0) == bi.EINVAL
    assert L.bigint_plan_create(ctypes.byref(h), bi.OP_MUL, None, None, 0, 64) == bi.EINVAL
    assert L.bigint_plan_destroy(None) == bi.EINVAL
    n = ctypes.c_size_t()
    assert L.bigint_plan_workspace_size(None, ctypes.byref(n)) == bi.EINVAL
    assert L.bigint_mul_ragged(None, None, None, None, None, None, 0, None, None) == bi.EINVAL
    k = ctypes.c_int()
    assert L.bigint_plan_segments(None, None, 0, ctypes.byref(k)) == bi.EINVAL
    assert L.bigint_mul_ragged_segment(None, None, None, None, None, None, 0, None, 0, None) == bi.EINVAL


def test_binding_fails_loudly_without_library(monkeypatch):
    import paper_2607_28897_amd as m
    monkeypatch.setattr(m, "_lib", None)
    monkeypatch.setattr(m, "LIB_PATH", "/nonexistent/libbigint_rocm.so")
    with pytest.raises(RuntimeError):
        m.lib()


def test_mfma_config_query(bi):
    # host-side only: the tuned table, the LDS fit and the thread overrides
    assert bi.mfma_config(16384, 16384) == (16, 8, 8)
    assert bi.mfma_config(1024, 1024) == (8, 1, 8)   # one wave per instance
    assert bi.mfma_config(512, 512) == (4, 1, 8)
    assert bi.mfma_config(2048, 2048) == (8, 4, 8)
    bi.set_mfma_config(0, 0, 7)
    try:
        assert bi.mfma_config(16384, 16384) == (16, 8, 7)
        assert bi.mfma_config(16397, 16397)[2] == 7
        with pytest.raises(bi.BigIntError):
            bi.mfma_config(16398, 16398)          # 7-bit digits no longer fit the LDS
    finally:
        bi.set_mfma_config(0, 0, 0)
    with pytest.raises(bi.BigIntError):
        bi.mfma_config(18433, 1)                   # beyond BIGINT_MFMA_MAX_LIMBS


def test_tune_table_load_and_restore(bi, tmp_path):
    # host-side only: a loaded table changes the configuration bigint_mul
    # picks, and a null path restores the built-in one
    import json
    path = str(tmp_path / "t.json")
    json.dump({"bins": [{"max_limbs": 18432, "strips_per_band": 8, "waves": 4, "digit_bits": 7}]},
              open(path, "w"))
    bi.autotune_load(path)
    try:
        assert bi.mfma_config(4096, 4096) == (8, 4, 7)
    finally:
        bi.autotune_load(None)
    assert bi.mfma_config(4096, 4096) == (8, 8, 8)
    bad = str(tmp_path / "bad.json")
    json.dump({"bins": [{"max_limbs": 100, "strips_per_band": 5, "waves": 4, "digit_bits": 7}]},
              open(bad, "w"))
    with pytest.raises(bi.BigIntError):
        bi.autotune_load(bad)
    assert bi.mfma_config(4096, 4096) == (8, 8, 8)


def test_tune_table_tile_field(bi, tmp_path):
    # host-side only: the optional "tile" field of a table entry picks the
    # MFMA tile (absent: 16); 32x32 tiles with 7-bit digits or 4 strips per
    # band fall back to 16; a 16x16 entry with 32 strips per band is refused
    import json
    path = str(tmp_path / "t32.json")
    json.dump({"bins": [{"max_limbs": 2000, "strips_per_band": 8, "waves": 8, "digit_bits": 8},
                        {"max_limbs": 18432, "strips_per_band": 32, "waves": 8, "digit_bits": 8,
                         "tile": 32}]}, open(path, "w"))
    bi.autotune_load(path)
    try:
        assert bi.mfma_tile(1000, 1000) == 16
        assert bi.mfma_tile(16384, 16384) == 32
        assert bi.mfma_config(16384, 16384) == (32, 8, 8)
        bi.set_mfma_config(0, 0, 7)
        try:
            assert bi.mfma_tile(16384, 16384) == 16
        finally:
            bi.set_mfma_config(0, 0, 0)
    finally:
        bi.autotune_load(None)
    assert bi.mfma_tile(16384, 16384) == 16
    bad = str(tmp_path / "bad32.json")
    json.dump({"bins": [{"max_limbs": 18432, "strips_per_band": 32, "waves": 8, "digit_bits": 8,
                         "tile": 16}]}, open(bad, "w"))
    with pytest.raises(bi.BigIntError):
        bi.autotune_load(bad)


def test_tune_table_from_environment(tmp_path):
    # host-side only, in a fresh process: BIGINT_TUNE_CACHE names a table
    # loaded before the first lookup; bigint_autotune_load(NULL) still
    # restores the built-in one, and a file that does not parse leaves it
    import json
    import subprocess
    import sys
    if not os.path.exists(os.path.join(ROOT, "paper_2607_28897_amd", "_lib", "libbigint_rocm.so")):
        pytest.skip("library not built")
    good = str(tmp_path / "env.json")
    json.dump({"bins": [{"max_limbs": 18432, "strips_per_band": 8, "waves": 4, "digit_bits": 7}]},
              open(good, "w"))
    bad = str(tmp_path / "bad.json")
    open(bad, "w").write("{\"bins\": []}")
    code = ("import sys; sys.path.insert(0, %r); import paper_2607_28897_amd as m; m.lib(); "
            "a = m.mfma_config(4096, 4096); m.autotune_load(None); print(a, m.mfma_config(4096, 4096))" % ROOT)
    for path, first in ((good, "(8, 4, 7)"), (bad, "(8, 8, 8)")):
        env = dict(os.environ, BIGINT_TUNE_CACHE=path)
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        assert r.stdout.split("\n")[-2] == f"{first} (8, 8, 8)", r.stdout


def test_debug_lines_from_environment():
    # host-side only, in fresh processes: BIGINT_DEBUG prints one line per
    # configuration a plan picks (here before the device allocation that a
    # machine without a GPU then refuses); without it nothing is printed
    import subprocess
    import sys
    if not os.path.exists(os.path.join(ROOT, "paper_2607_28897_amd", "_lib", "libbigint_rocm.so")):
        pytest.skip("library not built")
    code = ("import sys; sys.path.insert(0, %r); import numpy as np; import paper_2607_28897_amd as m\n"
            "m.lib(); la = np.array([1024, 4096, 16384, 3000], np.int64)\n"
            "for mk in (lambda: m.MulPlan(la, la), lambda: m.DivPlan(la, la // 2)):\n"
            "    try:\n        mk()\n    except m.BigIntError:\n        pass\n" % ROOT)
    for flag, want in (("1", True), ("0", False), (None, False)):
        env = dict(os.environ)
        env.pop("BIGINT_DEBUG", None)
        if flag is not None:
            env["BIGINT_DEBUG"] = flag
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        lines = [ln for ln in r.stderr.splitlines() if ln.startswith("bigint: ")]
        if want:
            assert any(ln.startswith("bigint: plan segment 0:") for ln in lines), r.stderr[-2000:]
            assert any(ln.startswith("bigint: plan of 4 divisions:") for ln in lines), r.stderr[-2000:]
        else:
            assert not lines, lines
