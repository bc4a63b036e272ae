"""AddressSanitizer and UndefinedBehaviorSanitizer runs on the host code
(CPU only): the C oracle under gcc, driven through every entry point on
small seeded problems (tests/sanitize/oracle_driver.c), and the library's
host code under clang (hipcc with the sanitizers on the host pass only),
driven through its layout, planners, argument checks and handle creation
(tests/sanitize/host_driver.c).  A reported error makes the driver exit
non-zero with the report on stderr."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, (" ".join(cmd), res.stdout[-4000:], res.stderr[-4000:])
    return res


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c99", "-Wall", "-Wextra"] + SAN_FLAGS +
         [os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "msg_oracle.c"), "-lm", "-o", exe])
    res = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"),
               timeout=600)
    assert "oracle driver ok" in res.stdout


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not available")
def test_host_library_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1907_12334_amd", "csrc")
    from paper_1907_12334_amd import build as B
    lib = str(tmp_path / "libmsg_san.so")
    host_san = []
    for f in SAN_FLAGS:                     # device code is built as usual
        host_san += ["-Xarch_host", f]
    device_flags = [f for f in B.HIPCC_FLAGS if f != "-O3"]
    _run([HIPCC] + device_flags + ["-O1", "-g"] + host_san + [os.path.join(csrc, s) for s in B.SOURCES] +
         ["-o", lib], timeout=900)
    obj = str(tmp_path / "host_driver.o")
    exe = str(tmp_path / "host_driver")
    _run([CLANG, "-c", "-O1", "-g", "-Wall", "-Wextra", "-I", os.path.join(ROOT, "include")] + SAN_FLAGS +
         [os.path.join(SAN, "host_driver.c"), "-o", obj])
    _run([CLANG + "++"] + SAN_FLAGS + [obj, "-o", exe, lib, "-Wl,-rpath," + str(tmp_path),
                                       "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    res = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"),
               timeout=600)
    assert "host driver ok" in res.stdout
