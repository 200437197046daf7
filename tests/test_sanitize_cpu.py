"""The C-ABI's host code under AddressSanitizer and UBSan: api.cpp (plan creation and
its tables, argument validation, the schedulers) rebuilt with both sanitizers and
linked with the device objects of the regular build, then the CPU ABI tests run
against it in a child process with the clang ASan runtime preloaded.  Any
sanitizer report fails the test."""

import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "paper_1809_04195_amd", "_build")
CLANG = "/opt/rocm/llvm/bin/clang"

pytestmark = pytest.mark.skipif(
    not (shutil.which("/opt/rocm/bin/hipcc") and os.path.exists(os.path.join(BUILD, "kernels.hip.o"))
         and os.path.exists(os.path.join(BUILD, "unet.hip.o")) and os.path.exists(CLANG)),
    reason="needs hipcc and the objects of a regular build")


def test_abi_host_code_under_asan_and_ubsan():
    from paper_1809_04195_amd.build import build_sanitized
    lib = build_sanitized()
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True, check=True).stdout
    assert re.search(r"__asan_", syms) and re.search(r"__ubsan_", syms), "sanitizer runtime not linked in"
    asan_rt = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True,
                             check=True).stdout.strip()
    env = dict(os.environ, T2S_LIB=lib, LD_PRELOAD=asan_rt, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert re.search(r"\d+ passed", out), out[-2000:]
