"""Host-side AddressSanitizer / UndefinedBehaviorSanitizer runs (no GPU):
the oracle's routines on small pencils, and the C ABI's argument checks in a
copy of the library whose host code is built with both sanitizers (device
code unchanged).  A sanitizer report or an unexpected return code fails the
test."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    return r.returncode, r.stdout + r.stderr


def test_oracle_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    exe = str(tmp_path / "san_oracle")
    rc, out = _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "tests", "san_oracle.c"),
                    "-lm", "-o", exe])
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="2")
    rc, out = _run([exe], env=env, timeout=300)
    assert rc == 0 and "ok" in out and "runtime error" not in out and "ERROR: AddressSanitizer" not in out, out


def _asan_rt_dir():
    libs = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return os.path.dirname(libs[0]) if libs else None


def test_abi_argument_checks_under_asan_ubsan(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG) and _asan_rt_dir()):
        pytest.skip("hipcc / clang sanitizer runtime not available")
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_1111_6374_amd", "csrc", "*.hip")))
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "-pthread", "--offload-arch=gfx950", "-w",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    procs = []
    objs = []
    for s in srcs:
        o = str(tmp_path / (os.path.basename(s) + ".o"))
        objs.append(o)
        procs.append(subprocess.Popen([HIPCC, *flags, "-c", s, "-o", o], stdout=subprocess.PIPE,
                                      stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out = p.communicate(timeout=900)[0]
        assert p.returncode == 0, out
    lib = str(tmp_path / "libgsyeig_san.so")
    rc, out = _run([HIPCC, "-shared", "-fPIC", "-pthread", "--offload-arch=gfx950", "-Xarch_host",
                    "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libasan", *objs,
                    "-o", lib])
    assert rc == 0, out
    exe = str(tmp_path / "san_abi")
    rc, out = _run([CLANG, "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-shared-libasan",
                    "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "san_abi.c"),
                    "-L", str(tmp_path), "-lgsyeig_san", "-Wl,-rpath," + str(tmp_path), "-o", exe])
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", LD_LIBRARY_PATH=_asan_rt_dir())
    rc, out = _run([exe], env=env, timeout=300)
    assert rc == 0 and "ok" in out and "runtime error" not in out and "ERROR: AddressSanitizer" not in out, out
