"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

* The oracle (oracle/oracle.c), built with gcc and the sanitizers, runs every
  entry point on small seeded sets and cross-checks them
  (tests/native/oracle_sanitize.c).
* The library, its host code instrumented (each -fsanitize= on the hipcc
  line applies to the host pass only; the kernels are built as usual), runs
  the C ABI's argument checks and error paths, which end before any device
  call (tests/native/abi_sanitize.c).

Any sanitizer report aborts the program, so a zero exit status and "ok" mean
a clean run.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_host_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    subprocess.run(["gcc", "-std=c11", "-D_GNU_SOURCE", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    os.path.join(ROOT, "oracle", "oracle.c"),
                    os.path.join(NATIVE, "oracle_sanitize.c"), "-lm", "-o", exe],
                   check=True, capture_output=True, text=True)
    _run(exe)


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc not installed")
def test_abi_host_checks_under_host_sanitizers(tmp_path):
    from paper_1910_02639_amd import buildlib
    lib = str(tmp_path / "libbtree_san.so")
    flags = [f for f in buildlib.HIPCC_FLAGS if f != "-O3"]
    san = ["-O1", "-g",
           "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    r = subprocess.run(["/opt/rocm/bin/hipcc", *flags, *san, "-I" + buildlib.INCLUDE,
                        *[os.path.join(buildlib.CSRC, s) for s in buildlib.SOURCES], "-o", lib],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "abi_sanitize")
    clang = "/opt/rocm/llvm/bin/clang"
    r = subprocess.run([clang, "-std=c11", "-O1", "-g", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", "-I" + buildlib.INCLUDE,
                        os.path.join(NATIVE, "abi_sanitize.c"), lib,
                        "-Wl,-rpath," + str(tmp_path), "-lm", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    _run(exe)
