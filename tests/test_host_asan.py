"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): every translation unit is compiled with both sanitizers on its
host pass, linked into a separate library, and driven by host_asan_driver.c
through argument checks, malformed tuning tables, the configuration logic
over the whole size range and the host-side scheduling of ragged multiply
and division plans.  A sanitizer report fails the test."""
import concurrent.futures as cf
import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2607_28897_amd", "csrc")
ROCM = "/opt/rocm"
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
CLANGXX = os.path.join(ROCM, "llvm", "bin", "clang++")

# each sanitizer flag for the host pass only (the device code is built as usual)
SAN_HOST = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-fno-sanitize-recover=undefined"]
SAN_LINK = ["-fsanitize=address,undefined", "-shared-libasan"]


def _asan_runtime_dir():
    libs = glob.glob(os.path.join(ROCM, "llvm", "lib", "clang", "*", "lib", "linux",
                                  "libclang_rt.asan-x86_64.so"))
    return os.path.dirname(libs[0]) if libs else None


def test_host_code_under_sanitizers(tmp_path):
    rt = _asan_runtime_dir()
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG) and rt):
        pytest.skip("ROCm clang with the sanitizer runtimes not found")
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               *SAN_HOST, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(tmp_path / "libbigint_rocm_hostsan.so")
    r = subprocess.run([CLANGXX, "-shared", "-fPIC", *SAN_LINK, *objs, f"-L{ROCM}/lib", "-lamdhip64",
                        f"-Wl,-rpath,{ROCM}/lib", "-o", lib], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "host_asan_driver")
    r = subprocess.run([CLANG, "-O1", "-g", *SAN_LINK, "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "host_asan_driver.c"), lib, "-lm",
                        f"-Wl,-rpath,{tmp_path}", f"-Wl,-rpath,{rt}", f"-Wl,-rpath,{ROCM}/lib", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.pop("BIGINT_TUNE_CACHE", None)
    work = tmp_path / "files"
    work.mkdir()
    r = subprocess.run([exe, str(work)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("host checks passed"), \
        (r.returncode, r.stdout[-2000:], r.stderr[-6000:])
