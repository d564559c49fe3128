"""Pins of the oracle's direction-dependent sums (oracle/dde.py).

The gain A_k(r_n) = sum_t a[t, k] b[t, n] enters the paper's sums (Sect. 2,
Eqs. 2-3) as a factor of each term.  Pinned by: the unit gain reducing them to
the plain sums (the pinned FP64 oracle), a point source (closed form with the
gain at that source), time-gated beams (each group of visibilities equals the
plain synthesis of its own beam-weighted sky), the adjoint identity, and the
agreement of the dense and the row-sampled forms.  Planted faults (a missing
conjugate, a gain left out of the adjoint, a dropped term) each break a pin."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import dde


def _frac(p, r):
    s = sum(Fraction(float(x)) * Fraction(float(y)) for x, y in zip(p, r))
    return float(s - round(s))


def _setup(rng, m=40, n=30, terms=3):
    uvw = rng.uniform(-300, 300, (m, 3))
    xyz = rng.normal(size=(n, 3)); xyz /= np.linalg.norm(xyz, axis=1, keepdims=True)
    a = rng.normal(size=(terms, m)) + 1j * rng.normal(size=(terms, m))
    b = rng.normal(size=(terms, n)) + 1j * rng.normal(size=(terms, n))
    return uvw, xyz, a, b


def dde_pins(seed=0) -> dict:
    rng = np.random.default_rng(seed)
    uvw, xyz, a, b = _setup(rng)
    m, n = uvw.shape[0], xyz.shape[0]
    x = rng.normal(size=n) + 1j * rng.normal(size=n)
    y = rng.normal(size=m) + 1j * rng.normal(size=m)
    res = {}
    # unit gain: the plain sums
    one_a, one_b = np.ones((1, m)), np.ones((1, n))
    res["unit_synthesis"] = np.allclose(dde.synthesis_dense(uvw, xyz, x, one_a, one_b), oracle.synthesis(uvw, xyz, x),
                                        rtol=0, atol=1e-11)
    res["unit_analysis"] = np.allclose(dde.analysis_dense(uvw, xyz, y, one_a, one_b), oracle.analysis(uvw, xyz, y),
                                       rtol=0, atol=1e-11)
    # a point source: V_k = A_k(r_n0) a0 exp(-2 pi i <p_k, r_n0>)
    n0, amp = 7, 0.8 - 0.3j
    sky = np.zeros(n, complex); sky[n0] = amp
    g = (a * b[:, n0][:, None]).sum(0)
    closed = np.array([g[k] * amp * complex(math.cos(2 * math.pi * _frac(uvw[k], xyz[n0])),
                                              -math.sin(2 * math.pi * _frac(uvw[k], xyz[n0]))) for k in range(m)])
    res["point_source"] = np.max(np.abs(dde.synthesis_dense(uvw, xyz, sky, a, b)[0] - closed)) < 1e-10
    # the same visibility through analysis: I_n = conj(A_k0(r_n)) v exp(+2 pi i <p_k0, r_n>)
    k0, v = 5, -1.1 + 0.6j
    vis = np.zeros(m, complex); vis[k0] = v
    gk = (a[:, k0][:, None] * b).sum(0)
    closed_i = np.array([np.conj(gk[j]) * v * complex(math.cos(2 * math.pi * _frac(uvw[k0], xyz[j])),
                                                       math.sin(2 * math.pi * _frac(uvw[k0], xyz[j]))) for j in range(n)])
    res["point_visibility"] = np.max(np.abs(dde.analysis_dense(uvw, xyz, vis, a, b)[0] - closed_i)) < 1e-10
    # time-gated beams: visibility group t sees beam b[t] only
    group = np.arange(m) % 3
    gate = np.stack([(group == t).astype(float) for t in range(3)])
    V = dde.synthesis_dense(uvw, xyz, x, gate, b)[0]
    ok = True
    for t in range(3):
        sel = np.where(group == t)[0]
        ok &= np.allclose(V[sel], oracle.synthesis(uvw[sel], xyz, b[t] * x)[0], rtol=0, atol=1e-10)
    res["time_gated"] = bool(ok)
    # adjoint identity
    Ax = dde.synthesis_dense(uvw, xyz, x, a, b)[0]
    AHy = dde.analysis_dense(uvw, xyz, y, a, b)[0]
    res["adjoint"] = abs(np.vdot(y, Ax) - np.vdot(AHy, x)) < 1e-12 * np.linalg.norm(Ax) * np.linalg.norm(y)
    return res


def test_dde_pins_hold():
    res = dde_pins()
    assert all(res.values()), res


@pytest.mark.parametrize("fault", dde.FAULTS)
def test_dde_pins_catch_planted_faults(fault):
    with dde.planted_fault(fault):
        res = dde_pins()
    assert not all(res.values()), f"planted DDE fault {fault!r} not caught: {res}"


def test_row_form_matches_dense_form():
    rng = np.random.default_rng(3)
    uvw, xyz, a, b = _setup(rng, m=60, n=50, terms=4)
    x = rng.normal(size=(2, 50)) + 1j * rng.normal(size=(2, 50))
    y = rng.normal(size=(2, 60)) + 1j * rng.normal(size=(2, 60))
    rows_v = np.array([0, 7, 59, 33])
    rows_p = np.array([49, 2, 10])
    assert np.allclose(dde.synthesis_rows(uvw, xyz, x, a, b, rows_v), dde.synthesis_dense(uvw, xyz, x, a, b)[:, rows_v],
                       rtol=0, atol=1e-10)
    assert np.allclose(dde.analysis_rows(uvw, xyz, y, a, b, rows_p), dde.analysis_dense(uvw, xyz, y, a, b)[:, rows_p],
                       rtol=0, atol=1e-10)
