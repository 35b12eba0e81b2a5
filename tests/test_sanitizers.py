"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only): the
oracle's C part runs the arithmetic pins, and the library's host-only entry points run
tests/sanitize/host_abi_check.cpp, each built with both sanitizers; any report fails."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def test_oracle_c_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-o", lib,
                           os.path.join(ROOT, "oracle", "ckks_oracle.c")])
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    env = dict(ENV, ORACLE_LIB=lib, LD_PRELOAD=asan)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_oracle_arith.py")], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, \
        r.stdout[-3000:] + r.stderr[-3000:]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="needs hipcc")
def test_library_host_code_under_sanitizers(tmp_path):
    """every library source compiled with both sanitizers on its host code (kernel
    sources also carry their device code, which the checked entry points never launch)"""
    import concurrent.futures as cf
    csrc = os.path.join(ROOT, "paper_2312_04356_amd", "csrc")
    srcs = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith((".cpp", ".hip")))
    srcs.append(os.path.join(ROOT, "tests", "sanitize", "host_abi_check.cpp"))
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include")]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        host_only = [] if src.endswith(".hip") else ["--offload-host-only"]
        subprocess.check_call([HIPCC] + flags + host_only + ["-x", "hip", "-c", src, "-o", obj],
                              stderr=subprocess.DEVNULL)
        return obj

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "host_abi_check")
    subprocess.check_call([CLANG, "-fsanitize=address,undefined", "-o", exe] + objs +
                          ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    r = subprocess.run([exe], env=ENV, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "host ABI checks passed" in r.stdout, r.stdout[-3000:] + r.stderr[-3000:]
