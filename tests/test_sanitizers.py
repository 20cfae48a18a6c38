"""Sanitizer builds, run on the CPU (no GPU needed).

* The oracle compiled by gcc with AddressSanitizer and UndefinedBehavior-
  Sanitizer (first error fatal) runs its own pins, tests/test_oracle.py and
  tests/test_oracle_block.py, in a child process with gcc's libasan preloaded
  and ORACLE_LIB naming the instrumented library.
* The library's host code in api.cpp (argument validation, the workspace
  layout in sizing mode, the EWORKSPACE protocol, error paths) compiled by
  hipcc with host-side ASan/UBSan -- the device code and the kernels' host
  launchers are the release build's objects -- is driven through the C ABI by
  tests/host_abi_driver.py in a child process with clang's ASan runtime
  preloaded and GMRES_LIB naming the instrumented library.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ERR = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _run(cmd, env, timeout):
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    return r.returncode, out


def test_harness_catches_planted_overflow(tmp_path):
    """The same flags and preload report a one-past-the-end read (planted in
    a scratch C file on the CPU), so a clean run below means something."""
    src = tmp_path / "planted.c"
    src.write_text("#include <stdlib.h>\n"
                   "double f(int n) { double *a = malloc(n * sizeof(double)), s = 0;\n"
                   "  for (int i = 0; i < n; ++i) a[i] = 1.0;\n"
                   "  for (int i = 0; i <= n; ++i) s += a[i];\n"
                   "  free(a); return s; }\n")
    lib = str(tmp_path / "libplanted.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fPIC", "-shared", str(src), "-o", lib])
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    code = "import ctypes as C; l = C.CDLL(%r); l.f.restype = C.c_double; l.f(8)" % lib
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0")
    rc, out = _run([sys.executable, "-c", code], env, 120)
    assert rc != 0 and "AddressSanitizer" in out


def test_oracle_pins_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    src = [os.path.join(ROOT, "oracle", f) for f in ("oracle.c", "dgmres.c", "bgmres.c")]
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                           *src, "-o", lib, "-lm"])
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    assert os.path.isabs(asan), "gcc's libasan not found"
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    rc, out = _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                    "tests/test_oracle.py", "tests/test_oracle_block.py"], env, 900)
    print(out[-3000:])
    assert rc == 0 and not any(e in out for e in SAN_ERR)
    assert " passed" in out


def test_host_abi_under_asan_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_1906_04051_amd import build as B
    objs = [os.path.join(B.BUILD, os.path.splitext(s)[0] + ".o") for s in B.SOURCES if s != "api.cpp"]
    if not all(os.path.exists(o) for o in objs):
        B.build()
    api_o = str(tmp_path / "api_san.o")
    lib = str(tmp_path / "libgmres_hostsan.so")
    host_san = ["-Xarch_host", "-fsanitize=address",
                "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all",
                "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f for f in B.COMMON if f != "-O3"] + ["-O1", "-g", "-Wno-unused-value"]
    subprocess.check_call([B._hipcc(), *flags, *host_san, "-x", "hip", "-c",
                           os.path.join(B.CSRC, "api.cpp"), "-o", api_o],
                          stderr=subprocess.DEVNULL)
    subprocess.check_call([B._hipcc(), "-shared", "-fPIC", f"--offload-arch={B.ARCH}", *objs, api_o,
                           "-o", lib, "-Xarch_host", "-fsanitize=address",
                           "-Xarch_host", "-fsanitize=undefined", "-shared-libasan", *B.LINK])
    clang = os.path.join(B.ROCM, "llvm", "bin", "clang")
    asan = subprocess.check_output([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                                   text=True).strip()
    assert os.path.exists(asan), "clang's ASan runtime not found"
    env = dict(os.environ, GMRES_LIB=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1", PYTHONPATH=ROOT)
    rc, out = _run([sys.executable, os.path.join(ROOT, "tests", "host_abi_driver.py")], env, 300)
    print(out[-3000:])
    assert rc == 0 and not any(e in out for e in SAN_ERR)
    assert "all checks passed" in out
