"""Direction-dependent gains in the oracle -- TEST INFRASTRUCTURE ONLY.

The paper's measurement equation omits antenna beams and leaves
direction-dependent effects (DDEs) to future work (Sect. 2 and 6).  With a
gain A_k(r) that visibility k sees towards sky point r, the sums become

  synthesis:  V_k = sum_n A_k(r_n) I_n exp(-2 pi i <p_k, r_n>)
  analysis:   I_n = sum_k conj(A_k(r_n)) V_k exp(+2 pi i <p_k, r_n>)

(an adjoint pair).  The gains are given in separable form
A_k(r_n) = sum_t a[t, k] b[t, n].

* ``synthesis_dense`` / ``analysis_dense``: the definition written out as
  dense complex128 matrices (gain matrix A = a^T b times the exponential
  matrix, phases reduced modulo one turn before the exponential) -- small
  sizes only.
* ``synthesis_rows`` / ``analysis_rows``: the same sums for sampled output
  rows at any size, by linearity over the terms t of the gain, each term one
  call of the plain FP64 oracle of this package (Eqs. 2-3).  Tests check that
  both forms agree on small inputs.

Only tests may import this module.
"""
from __future__ import annotations

import numpy as np

from . import analysis as _analysis
from . import synthesis as _synthesis

_fault = None
FAULTS = ("no_conj", "gain_not_in_adjoint", "dropped_term")


class planted_fault:
    """Switch the dense DDE sums to a deliberately wrong variant (tests only)."""

    def __init__(self, kind):
        if kind not in FAULTS:
            raise ValueError(kind)
        self.kind, self.old = kind, None

    def __enter__(self):
        global _fault
        self.old, _fault = _fault, self.kind
        return self

    def __exit__(self, *exc):
        global _fault
        _fault = self.old
        return False


def _as2(x):
    x = np.asarray(x, dtype=np.complex128)
    return x[None, :] if x.ndim == 1 else x


def gain_matrix(a, b):
    """A[k, n] = sum_t a[t, k] b[t, n]."""
    a, b = _as2(a), _as2(b)
    if _fault == "dropped_term" and a.shape[0] > 1:
        a, b = a[:-1], b[:-1]
    return a.T @ b


def _phase_matrix(uvw, xyz):
    t = np.asarray(uvw, float) @ np.asarray(xyz, float).T      # turns
    return t - np.round(t)


def synthesis_dense(uvw, xyz, sky, a, b):
    """V[r, k] = sum_n A_k(r_n) sky[r, n] exp(-2 pi i <p_k, r_n>), dense."""
    A = gain_matrix(a, b)
    E = np.exp(-2j * np.pi * _phase_matrix(uvw, xyz))
    return _as2(sky) @ (A * E).T


def analysis_dense(uvw, xyz, vis, a, b):
    """I[r, n] = sum_k conj(A_k(r_n)) vis[r, k] exp(+2 pi i <p_k, r_n>), dense."""
    A = gain_matrix(a, b)
    if _fault != "no_conj":
        A = A.conj()
    if _fault == "gain_not_in_adjoint":
        A = np.ones_like(A)
    E = np.exp(2j * np.pi * _phase_matrix(uvw, xyz))
    return _as2(vis) @ (A * E)


def synthesis_rows(uvw, xyz, sky, a, b, rows=None):
    """The DDE synthesis on visibility rows (all if None), any size."""
    a, b, sky = _as2(a), _as2(b), _as2(sky)
    out = 0.0
    for t in range(a.shape[0]):
        Y = _synthesis(uvw, xyz, b[t][None, :] * sky, rows=rows)
        out = out + (a[t] if rows is None else a[t][rows])[None, :] * Y
    return out


def analysis_rows(uvw, xyz, vis, a, b, rows=None):
    """The DDE analysis on sky rows (all if None), any size."""
    a, b, vis = _as2(a), _as2(b), _as2(vis)
    out = 0.0
    for t in range(a.shape[0]):
        W = _analysis(uvw, xyz, a[t].conj()[None, :] * vis, rows=rows)
        out = out + (b[t] if rows is None else b[t][rows]).conj()[None, :] * W
    return out
