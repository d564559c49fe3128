"""Python binding of the HVOX C ABI (include/hvox.h).

Argument marshalling only: every step of the transforms runs in the HIP
library ``libhvox.so``; PyTorch provides device memory and streams.  If the
library has not been built, importing works but every call raises
``RuntimeError`` -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhvox.so")

HVOX_F32 = 0
HVOX_F64 = 1
HVOX_REAL_SKY = 0x1
HVOX_PLAN_HOST_ONLY = 0x2
HVOX_TIMING = 0x4
HVOX_PREORDERED = 0x8
HVOX_DETERMINISTIC = 0x10

KERNELS = ("zero", "spread", "fft_x", "fft_y", "fft_z", "interp", "direct", "finalize", "transpose", "prephase")

ERRORS = {0: "HVOX_OK", -1: "HVOX_ERR_ARG", -2: "HVOX_ERR_EPS", -3: "HVOX_ERR_OOM",
          -4: "HVOX_ERR_HIP", -5: "HVOX_ERR_STATE"}


class HvoxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


# device-memory hooks of hvox_opts: dev_alloc(bytes, ctx, stream) -> ptr, dev_free(ptr, bytes, ctx, stream)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class HvoxOpts(ctypes.Structure):
    _fields_ = [("max_fft_bytes", ctypes.c_double),
                ("anisotropy", ctypes.c_double),
                ("upsampfac", ctypes.c_double),
                ("inner_upsampfac", ctypes.c_double),
                ("direct_threshold", ctypes.c_double),
                ("workspace_bytes", ctypes.c_double),
                ("vis_chunk", ctypes.POINTER(ctypes.c_int32)),
                ("sky_chunk", ctypes.POINTER(ctypes.c_int32)),
                ("flags", ctypes.c_int32),
                ("ntrans_hint", ctypes.c_int32),
                ("dev_alloc", ALLOC_FN),
                ("dev_free", FREE_FN),
                ("alloc_ctx", ctypes.c_void_p)]


class HvoxPlanInfo(ctypes.Structure):
    _fields_ = [("n_vis", ctypes.c_int64), ("n_pix", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("w", ctypes.c_int32),
                ("beta", ctypes.c_double), ("sigma", ctypes.c_double),
                ("w2", ctypes.c_int32), ("pad0", ctypes.c_int32),
                ("beta2", ctypes.c_double), ("sigma2", ctypes.c_double), ("eps", ctypes.c_double),
                ("eps_sub", ctypes.c_double),
                ("h", ctypes.c_double * 3), ("eta", ctypes.c_double * 3),
                ("n_vis_chunks", ctypes.c_int32), ("n_sky_chunks", ctypes.c_int32),
                ("n_pairs_nufft", ctypes.c_int64), ("n_pairs_direct", ctypes.c_int64),
                ("n_batches", ctypes.c_int64),
                ("resident_bytes", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("max_pair_workspace_bytes", ctypes.c_int64),
                ("grid_cells", ctypes.c_double), ("direct_terms", ctypes.c_double),
                ("est_seconds", ctypes.c_double), ("plan_seconds", ctypes.c_double),
                ("device_bytes", ctypes.c_int64), ("flags", ctypes.c_int32), ("on_device", ctypes.c_int32),
                ("n_direct_layers", ctypes.c_int64), ("noalloc_scratch_bytes", ctypes.c_int64),
                ("occ_tiles", ctypes.c_int64 * 2), ("occ_xlines", ctypes.c_int64 * 2),
                ("occ_zplanes", ctypes.c_int64 * 2), ("nufft_rows", ctypes.c_int32), ("pad1", ctypes.c_int32),
                ("est_direct_seconds", ctypes.c_double)]


class HvoxStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * len(KERNELS)), ("ms", ctypes.c_double * len(KERNELS)),
                ("alg_bytes", ctypes.c_double * len(KERNELS)), ("alg_flops", ctypes.c_double * len(KERNELS))]


EXPORTS = ("hvox_plan", "hvox_plan_upload", "hvox_synthesis", "hvox_transform_noalloc", "hvox_synthesis_dde",
           "hvox_analysis_dde", "hvox_analysis", "hvox_free", "hvox_plan_info",
           "hvox_plan_permutation", "hvox_plan_chunks", "hvox_stats", "hvox_stats_reset", "hvox_set_timing",
           "hvox_kernel_params", "hvox_alg1", "hvox_partition", "hvox_error_string",
           "hvox_last_error", "hvox_version")

_lib = None


def load_library():
    """Load libhvox.so (raises RuntimeError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HVOX HIP library not built: {LIB_PATH} is missing "
                           "(run `python -c 'import __graft_entry__ as g; g.build()'`)")
    lib = ctypes.CDLL(LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    vp = ctypes.c_void_p
    lib.hvox_plan.restype = ctypes.c_int
    lib.hvox_plan.argtypes = [dp, ctypes.c_int64, dp, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                              ctypes.POINTER(HvoxOpts), vp, ctypes.POINTER(vp)]
    for name in ("hvox_synthesis", "hvox_analysis"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [vp, vp, vp, ctypes.c_int32, vp]
    for name in ("hvox_synthesis_dde", "hvox_analysis_dde"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int32, ctypes.c_int32, vp, vp]
    lib.hvox_transform_noalloc.restype = ctypes.c_int
    lib.hvox_transform_noalloc.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_int32, vp]
    lib.hvox_plan_upload.restype = ctypes.c_int
    lib.hvox_plan_upload.argtypes = [vp, vp]
    lib.hvox_free.restype = ctypes.c_int
    lib.hvox_free.argtypes = [vp]
    lib.hvox_plan_info.restype = ctypes.c_int
    lib.hvox_plan_info.argtypes = [vp, ctypes.POINTER(HvoxPlanInfo)]
    lib.hvox_plan_permutation.restype = ctypes.c_int
    lib.hvox_plan_permutation.argtypes = [vp, ip, ip]
    lib.hvox_plan_chunks.restype = ctypes.c_int
    lib.hvox_plan_chunks.argtypes = [vp, ip, ip]
    lib.hvox_stats.restype = ctypes.c_int
    lib.hvox_stats.argtypes = [vp, ctypes.POINTER(HvoxStats)]
    lib.hvox_stats_reset.restype = ctypes.c_int
    lib.hvox_stats_reset.argtypes = [vp]
    lib.hvox_set_timing.restype = ctypes.c_int
    lib.hvox_set_timing.argtypes = [vp, ctypes.c_int32]
    lib.hvox_kernel_params.restype = ctypes.c_int
    lib.hvox_kernel_params.argtypes = [ctypes.c_double, ctypes.c_double, ip, dp]
    lib.hvox_alg1.restype = ctypes.c_int
    lib.hvox_alg1.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, dp, dp]
    lib.hvox_partition.restype = ctypes.c_int64
    lib.hvox_partition.argtypes = [dp, ctypes.c_int64, dp, ip]
    lib.hvox_error_string.restype = ctypes.c_char_p
    lib.hvox_error_string.argtypes = [ctypes.c_int]
    lib.hvox_last_error.restype = ctypes.c_char_p
    lib.hvox_last_error.argtypes = []
    lib.hvox_version.restype = ctypes.c_int
    lib.hvox_version.argtypes = []
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        msg = load_library().hvox_last_error().decode(errors="replace")
        raise HvoxError(rc, msg)


def _f64_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _coords(a, name) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError(f"{name} must have shape (n, 3), got {a.shape}")
    return a


# ---- host-only helpers --------------------------------------------------------
def kernel_params(eps: float, sigma: float = 1.25):
    """(w, beta) of the exponential-of-semicircle kernel for accuracy eps."""
    lib = load_library()
    w = ctypes.c_int32(0)
    beta = ctypes.c_double(0.0)
    _check(lib.hvox_kernel_params(eps, sigma, ctypes.byref(w), ctypes.byref(beta)))
    return int(w.value), float(beta.value)


def alg1(B, P, v_max: float, alpha: float = 1.0):
    """Algorithm 1: maximum box dimensions (h, eta) for full widths B, P."""
    lib = load_library()
    B = np.ascontiguousarray(B, dtype=np.float64)
    P = np.ascontiguousarray(P, dtype=np.float64)
    h = np.zeros(3)
    eta = np.zeros(3)
    _check(lib.hvox_alg1(_f64_ptr(B), _f64_ptr(P), v_max, alpha, _f64_ptr(h), _f64_ptr(eta)))
    return h, eta


def partition(x, h) -> np.ndarray:
    """Algorithm 2: chunk labels of points x (n, 3) for box dimensions h."""
    lib = load_library()
    x = _coords(x, "x")
    h = np.ascontiguousarray(h, dtype=np.float64)
    lab = np.zeros(x.shape[0], dtype=np.int32)
    r = lib.hvox_partition(_f64_ptr(x), x.shape[0], _f64_ptr(h),
                           lab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if r < 0:
        _check(int(r))
    return lab


# ---- plans --------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _torch_alloc(nbytes, ctx, stream):
    """dev_alloc hook: a block from PyTorch's caching allocator on the current
    device, associated with ``stream`` (NULL on failure: the plan call then
    reports HVOX_ERR_OOM)."""
    torch = _torch()
    try:
        return int(torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                      int(stream or 0) or None))
    except Exception:
        return None


def _torch_free(ptr, nbytes, ctx, stream):
    try:
        _torch().cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


# kept alive for the life of the process (the library may call them from any plan)
TORCH_ALLOC = ALLOC_FN(_torch_alloc)
TORCH_FREE = FREE_FN(_torch_free)


class Plan:
    """A planned HVOX operator for fixed baselines ``uvw`` (n_vis, 3) [wavelengths]
    and sky points ``xyz`` (n_pix, 3).

    ``synthesis(sky)`` computes V = A I (sky -> vis, exp(-2 pi i <p, r>));
    ``analysis(vis)`` computes I = A^H V (vis -> sky).  Data are torch
    tensors on the plan's GPU, complex64 for dtype "f32" and complex128 for
    "f64", shaped (n,) or (ntrans, n)."""

    def __init__(self, uvw, xyz, eps: float, dtype: str = "f32", *, max_fft_bytes: float = 0.0,
                 anisotropy: float = 0.0, upsampfac: float = 0.0, inner_upsampfac: float = 0.0,
                 direct_threshold: float = -1.0,
                 workspace_bytes: float = 0.0, vis_chunk=None, sky_chunk=None, real_sky: bool = False,
                 host_only: bool = False, timing: bool = False, ntrans_hint: int = 1, stream=None,
                 preordered: bool = False, deterministic: bool = False, allocator: Optional[str] = "torch",
                 alloc_hooks=None):
        self._lib = load_library()
        self._plan = ctypes.c_void_p(None)
        uvw = _coords(uvw, "uvw")
        xyz = _coords(xyz, "xyz")
        self.n_vis, self.n_pix = uvw.shape[0], xyz.shape[0]
        if dtype not in ("f32", "f64"):
            raise ValueError("dtype must be 'f32' or 'f64'")
        self.dtype = dtype
        self.host_only = host_only
        opts = HvoxOpts()
        opts.max_fft_bytes = max_fft_bytes
        opts.anisotropy = anisotropy
        opts.upsampfac = upsampfac
        opts.inner_upsampfac = inner_upsampfac
        opts.direct_threshold = direct_threshold
        opts.workspace_bytes = workspace_bytes
        opts.ntrans_hint = int(ntrans_hint)
        keep = []
        if vis_chunk is not None:
            vc = np.ascontiguousarray(vis_chunk, dtype=np.int32)
            if vc.shape != (self.n_vis,):
                raise ValueError("vis_chunk must have one entry per visibility")
            keep.append(vc)
            opts.vis_chunk = vc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        if sky_chunk is not None:
            sc = np.ascontiguousarray(sky_chunk, dtype=np.int32)
            if sc.shape != (self.n_pix,):
                raise ValueError("sky_chunk must have one entry per sky point")
            keep.append(sc)
            opts.sky_chunk = sc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        opts.flags = ((HVOX_REAL_SKY if real_sky else 0) | (HVOX_PLAN_HOST_ONLY if host_only else 0) |
                      (HVOX_TIMING if timing else 0) | (HVOX_PREORDERED if preordered else 0) |
                      (HVOX_DETERMINISTIC if deterministic else 0))
        # device memory: PyTorch's caching allocator (default), the library's own
        # hipMalloc (allocator=None), or caller hooks (alloc_hooks=(ALLOC_FN, FREE_FN, ctx))
        if alloc_hooks is not None:
            opts.dev_alloc, opts.dev_free, opts.alloc_ctx = alloc_hooks
            self._hooks = alloc_hooks
        elif allocator == "torch":
            opts.dev_alloc, opts.dev_free = TORCH_ALLOC, TORCH_FREE
        elif allocator is not None:
            raise ValueError("allocator must be 'torch' or None")
        self.real_sky = real_sky
        self.preordered = preordered
        self.deterministic = deterministic
        st = None
        if not host_only:
            torch = _torch()
            if not torch.cuda.is_available():
                raise RuntimeError("HVOX plans need a ROCm GPU (use host_only=True to plan without one)")
            self.device = torch.device("cuda", torch.cuda.current_device())
            st = self._stream_handle(stream)
        else:
            self.device = None
        _check(self._lib.hvox_plan(_f64_ptr(uvw), self.n_vis, _f64_ptr(xyz), self.n_pix, float(eps),
                                   HVOX_F64 if dtype == "f64" else HVOX_F32, ctypes.byref(opts),
                                   ctypes.c_void_p(st), ctypes.byref(self._plan)))

    # -- helpers
    @property
    def complex_dtype(self):
        torch = _torch()
        return torch.complex128 if self.dtype == "f64" else torch.complex64

    def _stream_handle(self, stream):
        torch = _torch()
        if stream is None:
            stream = torch.cuda.current_stream()
        return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)

    def _check_runnable(self):
        if self._plan.value is None:
            raise HvoxError(-5, "plan freed")
        if self.host_only:
            raise HvoxError(-5, "host-only plan cannot run transforms")

    def _prep(self, x, n, name):
        torch = _torch()
        if not isinstance(x, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        squeeze = x.dim() == 1
        if squeeze:
            x = x.unsqueeze(0)
        if x.dim() != 2 or x.shape[1] != n:
            raise ValueError(f"{name} must have shape ({n},) or (ntrans, {n}), got {tuple(x.shape)}")
        if x.device.type != "cuda":
            raise ValueError(f"{name} must be on the GPU")
        if x.dtype != self.complex_dtype:
            x = x.to(self.complex_dtype)
        return x.contiguous(), squeeze

    def _out(self, ntrans, n, out):
        torch = _torch()
        if out is None:
            return torch.empty((ntrans, n), dtype=self.complex_dtype, device=self.device)
        if out.shape != (ntrans, n) or out.dtype != self.complex_dtype or not out.is_contiguous():
            raise ValueError("bad output tensor")
        return out

    def synthesis(self, sky, out=None, stream=None):
        """V[t, k] = sum_n sky[t, n] exp(-2 pi i <p_k, r_n>)."""
        self._check_runnable()
        x, squeeze = self._prep(sky, self.n_pix, "sky")
        y = self._out(x.shape[0], self.n_vis, out)
        _check(self._lib.hvox_synthesis(self._plan, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                        x.shape[0], ctypes.c_void_p(self._stream_handle(stream))))
        return y[0] if squeeze and out is None else y

    def analysis(self, vis, out=None, stream=None):
        """I[t, n] = sum_k vis[t, k] exp(+2 pi i <p_k, r_n>)."""
        self._check_runnable()
        x, squeeze = self._prep(vis, self.n_vis, "vis")
        y = self._out(x.shape[0], self.n_pix, out)
        _check(self._lib.hvox_analysis(self._plan, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                       x.shape[0], ctypes.c_void_p(self._stream_handle(stream))))
        return y[0] if squeeze and out is None else y

    def upload(self, stream=None):
        """Create the device part of a host-only plan (hvox_plan_upload)."""
        if self._plan.value is None:
            raise HvoxError(-5, "plan freed")
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("HVOX plans need a ROCm GPU")
        self.device = torch.device("cuda", torch.cuda.current_device())
        _check(self._lib.hvox_plan_upload(self._plan, ctypes.c_void_p(self._stream_handle(stream))))
        self.host_only = False

    def _gains(self, a, b):
        ta, _ = self._prep(a, self.n_vis, "a")
        tb, _ = self._prep(b, self.n_pix, "b")
        if ta.shape[0] != tb.shape[0]:
            raise ValueError("a and b must hold the same number of terms")
        return ta, tb

    def synthesis_dde(self, sky, a, b, out=None, stream=None):
        """Synthesis through direction-dependent gains A_k(r_n) = sum_t a[t, k] b[t, n]:
        V[r, k] = sum_n A_k(r_n) sky[r, n] exp(-2 pi i <p_k, r_n>).  a: (n_terms, n_vis),
        b: (n_terms, n_pix) complex tensors on the plan's GPU."""
        torch = _torch()
        self._check_runnable()
        x, squeeze = self._prep(sky, self.n_pix, "sky")
        ta, tb = self._gains(a, b)
        y = self._out(x.shape[0], self.n_vis, out)
        work = torch.empty((2, ta.shape[0], max(self.n_vis, self.n_pix)), dtype=self.complex_dtype, device=self.device)
        _check(self._lib.hvox_synthesis_dde(self._plan, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                            ctypes.c_void_p(ta.data_ptr()), ctypes.c_void_p(tb.data_ptr()),
                                            ta.shape[0], x.shape[0], ctypes.c_void_p(work.data_ptr()),
                                            ctypes.c_void_p(self._stream_handle(stream))))
        return y[0] if squeeze and out is None else y

    def analysis_dde(self, vis, a, b, out=None, stream=None):
        """The adjoint: I[r, n] = sum_k conj(A_k(r_n)) vis[r, k] exp(+2 pi i <p_k, r_n>)."""
        torch = _torch()
        self._check_runnable()
        x, squeeze = self._prep(vis, self.n_vis, "vis")
        ta, tb = self._gains(a, b)
        y = self._out(x.shape[0], self.n_pix, out)
        work = torch.empty((2, ta.shape[0], max(self.n_vis, self.n_pix)), dtype=self.complex_dtype, device=self.device)
        _check(self._lib.hvox_analysis_dde(self._plan, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                           ctypes.c_void_p(ta.data_ptr()), ctypes.c_void_p(tb.data_ptr()),
                                           ta.shape[0], x.shape[0], ctypes.c_void_p(work.data_ptr()),
                                           ctypes.c_void_p(self._stream_handle(stream))))
        return y[0] if squeeze and out is None else y

    def info(self) -> dict:
        inf = HvoxPlanInfo()
        _check(self._lib.hvox_plan_info(self._plan, ctypes.byref(inf)))
        d = {name: getattr(inf, name) for name, _ in HvoxPlanInfo._fields_}
        for k in ("h", "eta", "occ_tiles", "occ_xlines", "occ_zplanes"):
            d[k] = list(getattr(inf, k))
        return d

    def permutation(self):
        v = np.zeros(self.n_vis, dtype=np.int32)
        s = np.zeros(self.n_pix, dtype=np.int32)
        _check(self._lib.hvox_plan_permutation(self._plan, v.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                               s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return v, s

    def chunks(self):
        v = np.zeros(self.n_vis, dtype=np.int32)
        s = np.zeros(self.n_pix, dtype=np.int32)
        _check(self._lib.hvox_plan_chunks(self._plan, v.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                          s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return v, s

    def stats(self) -> dict:
        st = HvoxStats()
        _check(self._lib.hvox_stats(self._plan, ctypes.byref(st)))
        return {k: dict(launches=int(st.launches[i]), ms=float(st.ms[i]), alg_bytes=float(st.alg_bytes[i]),
                        alg_flops=float(st.alg_flops[i])) for i, k in enumerate(KERNELS)}

    def reset_stats(self):
        _check(self._lib.hvox_stats_reset(self._plan))

    def set_timing(self, on: bool):
        _check(self._lib.hvox_set_timing(self._plan, 1 if on else 0))

    def free(self):
        if self._plan.value is not None:
            self._lib.hvox_free(self._plan)
            self._plan = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()
        return False


def rel_l2(y, ref) -> float:
    y = np.asarray(y)
    ref = np.asarray(ref)
    n = np.linalg.norm(ref.ravel())
    d = np.linalg.norm((y - ref).ravel())
    return float(d / n) if n > 0 else float(d)


__all__ = ["Plan", "HvoxError", "load_library", "kernel_params", "alg1", "partition", "EXPORTS",
           "rel_l2", "KERNELS"]
