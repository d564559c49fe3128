"""HVOX oracle -- TEST INFRASTRUCTURE ONLY.

A plain FP64 CPU evaluation of the sums HVOX approximates (paper Sect. 2,
Eqs. 2-3, unit tesselation weights, exp(-2 pi i <p, r>) with p in
wavelengths), plus plain restatements of the partitioning steps (Sect. 3.2,
Algorithms 1 and 2) in ``oracle.partition``.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package.  It shares no code with the GPU library and the
GPU library never calls it.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhvox_oracle.so")
_lib = None

FAULT_NONE, FAULT_SIGN, FAULT_NO_TWO_PI, FAULT_SWAP_XY, FAULT_DROP_LAST, FAULT_NO_CONJ = range(6)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    lp = ctypes.POINTER(ctypes.c_int64)
    for name in ("hvox_oracle_synthesis", "hvox_oracle_analysis"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [dp, ctypes.c_int64, dp, ctypes.c_int64, dp, ctypes.c_int32,
                      lp, ctypes.c_int64, dp]
    lib.hvox_oracle_set_fault.restype = ctypes.c_int
    lib.hvox_oracle_set_fault.argtypes = [ctypes.c_int]
    lib.hvox_oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a, shape_last=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape_last is not None and (a.ndim != 2 or a.shape[1] != shape_last):
        raise ValueError(f"expected (n, {shape_last}) array, got {a.shape}")
    return a


def _c128(a, n):
    a = np.asarray(a)
    if a.ndim == 1:
        a = a[None, :]
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if a.shape[1] != n:
        raise ValueError(f"data length {a.shape[1]} != {n}")
    return a


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _run(name, uvw, xyz, data, n_in, n_out_full, rows):
    lib = _load()
    uvw = _f64(uvw, 3)
    xyz = _f64(xyz, 3)
    data = _c128(data, n_in)
    ntrans = data.shape[0]
    if rows is None:
        nout = n_out_full
        rp = None
        nr = 0
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        nout = rows.shape[0]
        rp = _ptr(rows, ctypes.c_int64)
        nr = nout
    out = np.zeros((ntrans, nout), dtype=np.complex128)
    rc = getattr(lib, name)(_ptr(uvw, ctypes.c_double), uvw.shape[0],
                            _ptr(xyz, ctypes.c_double), xyz.shape[0],
                            _ptr(data.view(np.float64), ctypes.c_double), ntrans,
                            rp, nr, _ptr(out.view(np.float64), ctypes.c_double))
    if rc != 0:
        raise ValueError(f"{name} rejected its arguments")
    return out


def synthesis(uvw, xyz, sky, rows=None):
    """V[t, k] = sum_n sky[t, n] exp(-2 pi i <uvw[k], xyz[n]>) for k in rows
    (all visibilities when rows is None).  Returns (ntrans, len(rows))."""
    uvw = _f64(uvw, 3)
    return _run("hvox_oracle_synthesis", uvw, xyz, sky, np.asarray(xyz).shape[0], uvw.shape[0], rows)


def analysis(uvw, xyz, vis, rows=None):
    """I[t, n] = sum_k vis[t, k] exp(+2 pi i <uvw[k], xyz[n]>) for n in rows
    (all pixels when rows is None).  Returns (ntrans, len(rows))."""
    xyz = _f64(xyz, 3)
    return _run("hvox_oracle_analysis", uvw, xyz, vis, np.asarray(uvw).shape[0], xyz.shape[0], rows)


def max_threads() -> int:
    return int(_load().hvox_oracle_max_threads())


class planted_fault:
    """Context manager that switches the oracle to a deliberately wrong
    variant (tests use it to show that the pins catch such mistakes)."""

    def __init__(self, kind: int):
        self.kind = kind
        self.old = 0

    def __enter__(self):
        self.old = _load().hvox_oracle_set_fault(self.kind)
        return self

    def __exit__(self, *exc):
        _load().hvox_oracle_set_fault(self.old)
        return False


# Planted mistakes of the error metrics (tests switch them on to show that the
# metric pins catch them); None = the correct metric.
_metric_fault = None
METRIC_FAULTS = ("squared", "per_row_mean", "normalised_by_y", "max_norm", "real_part_only")


class planted_metric_fault:
    """Context manager switching ``rel_l2`` / ``max_rel_err`` to a deliberately
    wrong variant (used only by the tests of the metrics' pins)."""

    def __init__(self, kind: str):
        if kind not in METRIC_FAULTS:
            raise ValueError(kind)
        self.kind = kind
        self.old = None

    def __enter__(self):
        global _metric_fault
        self.old, _metric_fault = _metric_fault, self.kind
        return self

    def __exit__(self, *exc):
        global _metric_fault
        _metric_fault = self.old
        return False


def rel_l2(y, ref) -> float:
    """Relative l2 error ||y - ref||_2 / ||ref||_2 over all entries of all rows
    (not squared, not averaged per row).  This is the reading of the paper's
    "relative accuracy" (Sect. 5.2, never defined there) that every parity
    test uses; a zero reference gives the absolute norm of y."""
    y = np.asarray(y); ref = np.asarray(ref)
    diff = y - ref
    if _metric_fault == "real_part_only":
        diff = diff.real
    if _metric_fault == "per_row_mean":
        y2 = np.atleast_2d(y); r2 = np.atleast_2d(ref)
        return float(np.mean([np.linalg.norm(a - b) / np.linalg.norm(b) for a, b in zip(y2, r2)]))
    d = np.linalg.norm(diff.ravel())
    n = np.linalg.norm((y if _metric_fault == "normalised_by_y" else ref).ravel())
    if _metric_fault == "max_norm":
        d, n = np.max(np.abs(diff)), np.max(np.abs(ref))
    r = float(d / n) if n > 0 else float(d)
    return r * r if _metric_fault == "squared" else r


def max_rel_err(y, ref) -> float:
    """Largest error of one entry relative to the largest reference entry,
    max_k |y_k - ref_k| / max_k |ref_k| over all rows: the element-wise
    companion of ``rel_l2`` (a failure confined to a few outputs, e.g. targets
    in the corners of a sub-problem's box, is not diluted by the others)."""
    y = np.asarray(y); ref = np.asarray(ref)
    diff = y - ref
    if _metric_fault == "real_part_only":
        diff = diff.real
    d = float(np.max(np.abs(diff))) if diff.size else 0.0
    n = float(np.max(np.abs(ref))) if ref.size else 0.0
    if _metric_fault == "normalised_by_y":
        n = float(np.max(np.abs(y))) if y.size else 0.0
    r = d / n if n > 0 else d
    return r * r if _metric_fault == "squared" else r
