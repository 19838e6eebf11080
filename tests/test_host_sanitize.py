"""Host code of the C-ABI library under AddressSanitizer and
UndefinedBehaviorSanitizer: the library's sources are compiled again with
host-only instrumentation (the device code is unchanged), linked into a small
C driver (tests/sanitize/abi_validation.c) that walks the validation paths
and builds the host tile tables of several rigs, and run on the CPU.  A
sanitizer report or a wrong status fails the test."""
import os
import shutil
import subprocess

import pytest

from paper_1910_03517_amd import build as bld

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "sanitize", "abi_validation.c")
CLANG = "/opt/rocm/llvm/bin/clang"
# Each sanitizer flag applies to the host compilation only.
HOST_SAN = ("-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-g")


@pytest.mark.slow
@pytest.mark.skipif(not (os.path.exists(bld.HIPCC) and os.path.exists(CLANG)), reason="needs hipcc and clang")
def test_abi_validation_under_host_sanitizers(tmp_path):
    lib = str(tmp_path / "libringcorr_san.so")
    bld.build(verbose=False, out=lib, build_dir=str(tmp_path / "obj"), extra=HOST_SAN,
              link_extra=("-fsanitize=address,undefined",))
    # The host objects really are instrumented.
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_" in syms and "__ubsan_" in syms
    exe = str(tmp_path / "abi_validation")
    cmd = [CLANG, "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-g", "-O1",
           f"-I{os.path.join(ROOT, 'include')}", DRIVER, lib, f"-Wl,-rpath,{tmp_path}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ)
    # Leaks inside the HIP runtime's own start-up are not this library's.
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "all checks passed" in r.stdout
    shutil.rmtree(tmp_path / "obj", ignore_errors=True)
