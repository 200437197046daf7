"""The library's FFT building blocks (csrc/fft.hpp, the header the GPU kernels include)
built as plain C++ for the host and checked against numpy: every register codelet
(radix 2/3/4/5, the direct odd-prime codelet at 13, composites) and every two-step
plan L = R1 R2 of the column and row passes, forward and inverse, with the kernels'
thread mapping and twiddles emulated sequentially (tests/csrc/fft_host_check.cpp)."""

import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "csrc", "fft_host_check.cpp")
COL = [16, 32, 48, 64, 96, 128, 160, 192, 240, 256, 320, 384, 512]
ROW = COL + [260]


@pytest.fixture(scope="module")
def fftlib(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    out = str(tmp_path_factory.mktemp("ffthost") / "fft_host.so")
    subprocess.run([cxx, "-O2", "-std=c++17", "-shared", "-fPIC", SRC, "-o", out], check=True)
    lib = ctypes.CDLL(out)
    fp = ctypes.POINTER(ctypes.c_float)
    lib.plan_host.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, fp, fp]
    lib.codelet_host.argtypes = [ctypes.c_int, ctypes.c_int, fp, fp]
    lib.plan_factors.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.root_re.argtypes = lib.root_im.argtypes = [ctypes.c_long, ctypes.c_long]
    lib.root_re.restype = lib.root_im.restype = ctypes.c_double
    return lib


def _call(fn, n, *args):
    rng = np.random.default_rng(n)
    x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    y = np.empty_like(x)
    fp = ctypes.POINTER(ctypes.c_float)
    assert fn(*args, x.view(np.float32).ctypes.data_as(fp), y.view(np.float32).ctypes.data_as(fp)) == 0
    return x.astype(np.complex128), y.astype(np.complex128)


@pytest.mark.parametrize("R", [2, 3, 4, 5, 6, 8, 10, 12, 13, 15, 16, 20, 24, 32])
def test_codelets_match_numpy(fftlib, R):
    for inv in (0, 1):
        x, y = _call(fftlib.codelet_host, R, R, inv)
        ref = np.fft.ifft(x) * R if inv else np.fft.fft(x)
        assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 3e-7, (R, inv)


@pytest.mark.parametrize("which,L", [(0, L) for L in COL] + [(1, L) for L in ROW])
def test_two_step_plans_match_numpy(fftlib, which, L):
    r1, r2 = ctypes.c_int(), ctypes.c_int()
    assert fftlib.plan_factors(L, which, ctypes.byref(r1), ctypes.byref(r2)) == 0
    assert r1.value * r2.value == L
    if which == 0:
        assert 16 % r2.value == 0        # the column pass addresses 16-row tiles by R2 offsets
    for inv in (0, 1):
        x, y = _call(fftlib.plan_host, L, L, which, inv)
        ref = np.fft.ifft(x) * L if inv else np.fft.fft(x)
        assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-6, (L, which, inv)


def test_compile_time_roots(fftlib):
    for n in (13, 20, 260, 384):
        for m in range(0, 2 * n, 7):
            w = np.exp(-2j * np.pi * (m % n) / n)
            assert abs(fftlib.root_re(m, n) - w.real) < 2e-15 and abs(fftlib.root_im(m, n) - w.imag) < 2e-15
