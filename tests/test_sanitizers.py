"""Host sanitizer runs (CPU only, no GPU calls).

1. The oracle, built with AddressSanitizer and UndefinedBehaviorSanitizer by
   gcc, runs direct sums and butterflies in both directions for every phase
   (tests/sanitize/oracle_main.c): no sanitizer finding, every output finite.
2. libbfly's host code (argument validation, plans, workspace sizing and
   carving, batched layouts, timing) built with the same sanitizers by
   hipcc (host side only: device code is never instrumented), linked with
   the library's other objects, runs the C-ABI tests (test_abi.py) with the
   sanitizer runtime preloaded."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", "-g", "-O1", "-fopenmp", "-ffp-contract=off", "-std=c11", "-D_DEFAULT_SOURCE", *SAN, "-o", exe,
           os.path.join(ROOT, "tests", "sanitize", "oracle_main.c"), os.path.join(ROOT, "oracle", "bfly_oracle.c"),
           "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0 and "SANITIZE OK" in r.stdout


def _asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_1305_4650_amd import build as B
    objs_dir = B.BUILD
    host_srcs = ["bfly_api.cpp", "bfly_timing.cpp"]
    others = [os.path.join(objs_dir, os.path.splitext(s)[0] + ".o") for s in B.SOURCES if s not in host_srcs]
    if not os.path.exists(HIPCC) or _asan_runtime() is None:
        pytest.skip("hipcc or the clang sanitizer runtime is not available")
    if not all(os.path.exists(o) for o in others):
        pytest.skip("library objects not built (python -m paper_1305_4650_amd.build)")
    objs = []
    for s in host_srcs:
        o = str(tmp_path / (os.path.splitext(s)[0] + ".o"))
        # sanitizers on the host side only: -Xarch_host before each flag
        san = [x for f in SAN for x in ("-Xarch_host", f)]
        cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={B.ARCH}", "-ffp-contract=off",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
               *san, "-x", "hip", "-c", os.path.join(B.CSRC, s), "-o", o]
        subprocess.run(cmd, check=True, capture_output=True)
        objs.append(o)
    lib = str(tmp_path / "libbfly_san.so")
    san_link = ["-Xarch_host", "-fsanitize=address,undefined", "-shared-libasan"]
    subprocess.run([HIPCC, "-shared", f"--offload-arch={B.ARCH}", "-fPIC", *san_link, "-o", lib, *others, *objs],
                   check=True, capture_output=True)
    env = dict(os.environ, BFLY_LIBRARY=lib, LD_PRELOAD=_asan_runtime(), ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")], capture_output=True, text=True, env=env,
                       cwd=ROOT, timeout=600)
    print(r.stdout[-3000:], r.stderr[-3000:])
    assert r.returncode == 0, "C-ABI tests failed under the host sanitizers"
    assert "passed" in r.stdout
