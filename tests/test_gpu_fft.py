"""Kernel-level check of the LDS-resident mixed-radix FFT pass against numpy's
FFT (a library routine), through the test entry point of include/hvox_testing.h."""
import ctypes

import numpy as np
import pytest

import paper_2306_06007_amd as hv

pytestmark = pytest.mark.gpu


def fft_pass(x, n, wstart, wcount, sign, dtype):
    import torch
    lib = hv.load_library()
    f = lib.hvox_test_fft
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int32] * 7 + [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    cd = torch.complex128 if dtype == "f64" else torch.complex64
    nlines, nin = x.shape
    xin = torch.as_tensor(x).to(device="cuda", dtype=cd).contiguous()
    out = torch.zeros((nlines, wcount), dtype=cd, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    rc = f(1 if dtype == "f64" else 0, n, nin, nlines, wstart, wcount, sign,
           ctypes.c_void_p(xin.data_ptr()), ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st))
    assert rc == 0, lib.hvox_last_error()
    return out.cpu().numpy().astype(np.complex128)


def reference(x, n, wstart, wcount, sign):
    """The zero-padded DFT written out; the exponent l m / n is reduced modulo n
    in integer arithmetic first, so the float64 phases stay exact to ~1e-16
    (unreduced, 2 pi l m / n reaches ~2.6e4 rad at n = 4096 and its rounding
    alone would cost ~3e-12)."""
    nlines, nin = x.shape
    l = np.arange(nin, dtype=np.int64) - nin // 2
    m = (wstart + np.arange(wcount, dtype=np.int64)) % n
    q = np.mod(np.outer(l, m), n)
    E = np.exp(sign * 2j * np.pi * q / n)
    return x @ E


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("dtype,tol", [("f32", 2e-6), ("f64", 1e-13)])
@pytest.mark.parametrize("n", [2, 6, 12, 30, 36, 64, 100, 250, 432, 486, 810, 1000, 1152, 1250, 1296, 2048, 2160,
                               3000, 3888, 4096])
def test_fft_full_window(dtype, tol, n):
    rng = np.random.default_rng(n)
    nlines = 5 if n > 1000 else 37
    for sign in (-1, 1):
        nin = max(2, (n * 4 // 5) // 2 * 2)
        x = rng.normal(size=(nlines, nin)) + 1j * rng.normal(size=(nlines, nin))
        out = fft_pass(x, n, 0, n, sign, dtype)
        ref = reference(x, n, 0, n, sign)
        err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
        assert err < tol, (n, sign, err)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_fft_windowed_output(dtype):
    rng = np.random.default_rng(1)
    n, nin = 120, 96
    R = 50
    x = rng.normal(size=(70, nin)) + 1j * rng.normal(size=(70, nin))
    out = fft_pass(x, n, -R, 2 * R + 1, -1, dtype)
    ref = reference(x, n, -R, 2 * R + 1, -1)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < (2e-6 if dtype == "f32" else 1e-13)
