"""Radio-astronomy front end: ``dirty2vis`` / ``vis2dirty`` on direction-cosine
images, in the shape of the HVOX package's single-use functions (Sect. 4, the
two-package split, which mimics the W-gridder API of ducc0).

Conventions (Sect. 2.1, Eq. 4): a pixel at direction cosines (l, m) of the
tangent plane at the phase centre is the sky point r = (l, m, n - 1) with
n = sqrt(1 - l^2 - m^2), so that

    V(u, v, w) = sum_pix I(l, m) exp(-2 pi i [u l + v m + w (n - 1)])

is exactly the transform ``Plan.synthesis`` computes, ``V_k = sum_n I_n
exp(-2 pi i <p_k, r_n>)``, and ``vis2dirty`` is its adjoint (Eqs. 2-3).  The
shift by -1 along n is the phase reference of DCOS gridders; the paper's own
Eq. 2 uses the full <p, r> (a factor exp(-2 pi i w) per visibility apart).
Baselines are given in metres with one or more channel frequencies: every
(row, channel) pair is one visibility point p = uvw * f / c, so all channels go
through one plan and one call.  Polarisations (or any set of images sharing
the coordinates) are the ``ntrans`` rows of a call.  Tesselation weights of the
mesh are folded into the pixel values by the caller.

Nothing here computes any part of the transform: the module converts
coordinates and reshapes arrays; the plan's HIP kernels do the rest.
"""
from __future__ import annotations

import numpy as np

from .hvox import Plan

SPEED_OF_LIGHT = 299_792_458.0   # m/s


def dcos_points(l, m) -> np.ndarray:
    """Sky points (l, m, n - 1) of direction cosines (l, m), n = sqrt(1 - l^2 - m^2)."""
    l = np.asarray(l, dtype=np.float64).ravel()
    m = np.asarray(m, dtype=np.float64).ravel()
    if l.shape != m.shape:
        raise ValueError("l and m must have the same number of pixels")
    r2 = l * l + m * m
    if np.any(r2 > 1.0):
        raise ValueError("direction cosines must satisfy l^2 + m^2 <= 1")
    # n - 1 = -r2 / (1 + n): no cancellation near the phase centre
    nm1 = -r2 / (1.0 + np.sqrt(1.0 - r2))
    return np.stack([l, m, nm1], axis=1)


def channel_uvw(uvw_m, freqs_hz) -> np.ndarray:
    """Baselines in wavelengths of every (row, channel) pair, row-major
    ([row][channel], the layout of a measurement set's data column)."""
    uvw_m = np.asarray(uvw_m, dtype=np.float64)
    if uvw_m.ndim != 2 or uvw_m.shape[1] != 3:
        raise ValueError("uvw must have shape (n_rows, 3), in metres")
    f = np.atleast_1d(np.asarray(freqs_hz, dtype=np.float64))
    if f.ndim != 1 or f.size == 0 or np.any(~(f > 0.0)):
        raise ValueError("freqs must be positive frequencies in Hz")
    return (uvw_m[:, None, :] * (f / SPEED_OF_LIGHT)[None, :, None]).reshape(-1, 3)


class RadioPlan:
    """A plan for fixed baselines (metres), channel frequencies and image
    pixels (direction cosines).  ``dirty2vis(dirty)`` maps images of shape
    ``(n_pix,)`` or ``(n_pol, n_pix)`` to visibilities ``(n_rows, n_chan)`` or
    ``(n_pol, n_rows, n_chan)``; ``vis2dirty`` is the adjoint.  Inputs and
    outputs are torch tensors on the GPU (NumPy inputs are copied there)."""

    def __init__(self, uvw_m, freqs_hz, l, m, eps: float = 1e-4, dtype: str = "f32", **plan_kw):
        self.n_rows = int(np.asarray(uvw_m).shape[0])
        self.n_chan = int(np.atleast_1d(freqs_hz).size)
        self.xyz = dcos_points(l, m)
        self.n_pix = self.xyz.shape[0]
        self.plan = Plan(channel_uvw(uvw_m, freqs_hz), self.xyz, eps, dtype, **plan_kw)

    def _rows(self, x, trailing, name):
        """x as a GPU tensor of rows: its trailing dimensions (which must be
        ``trailing``) merged into one."""
        import torch
        t = x if isinstance(x, torch.Tensor) else torch.as_tensor(np.asarray(x))
        k = len(trailing)
        if tuple(t.shape[-k:]) != tuple(trailing):
            raise ValueError(f"{name} must end with dimensions {tuple(trailing)}")
        return t.to(self.plan.device).reshape(-1, int(np.prod(trailing)))

    def export_partition(self):
        """Chunk labels of the plan's visibility points ((n_rows, n_chan)) and
        pixels ((n_pix,)), to build later plans on the same partition (pass them
        as ``vis_chunk=labels.ravel()`` and ``sky_chunk=...``), the re-use of a
        good ordering that Sect. 4 suggests."""
        v, s = self.plan.chunks()
        return v.reshape(self.n_rows, self.n_chan), s

    def dirty2vis(self, dirty):
        """Visibilities of a dirty image (the measurement operator, sky -> vis)."""
        lead = tuple(dirty.shape[:-1])
        v = self.plan.synthesis(self._rows(dirty, (self.n_pix,), "dirty"))
        return v.reshape(lead + (self.n_rows, self.n_chan))

    def vis2dirty(self, vis):
        """Dirty image of visibilities (the adjoint, vis -> sky)."""
        lead = tuple(vis.shape[:-2])
        d = self.plan.analysis(self._rows(vis, (self.n_rows, self.n_chan), "vis"))
        return d.reshape(lead + (self.n_pix,))

    def free(self):
        self.plan.free()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()
        return False


def dirty2vis(uvw_m, freqs_hz, dirty, l, m, eps: float = 1e-4, dtype: str = "f32", **plan_kw):
    """Single-use measurement operator: visibilities ``(..., n_rows, n_chan)``
    of images ``(..., n_pix)`` on the pixels (l, m)."""
    with RadioPlan(uvw_m, freqs_hz, l, m, eps, dtype, **plan_kw) as rp:
        return rp.dirty2vis(dirty)


def vis2dirty(uvw_m, freqs_hz, vis, l, m, eps: float = 1e-4, dtype: str = "f32", **plan_kw):
    """Single-use adjoint: dirty images ``(..., n_pix)`` of visibilities
    ``(..., n_rows, n_chan)``."""
    with RadioPlan(uvw_m, freqs_hz, l, m, eps, dtype, **plan_kw) as rp:
        return rp.vis2dirty(vis)
