"""Pins of the FP64 oracle against what the paper and mathematics fix.

The oracle evaluates the discrete sky->vis and vis->sky sums (HVOX Sect. 2,
Eqs. 2-3).  None of these checks re-types the oracle's own formula: they use
exact rational phases, closed forms (geometric series), a library routine the
sums reduce to (numpy's FFT on a DFT lattice), brute force on tiny inputs,
the adjoint identity and symmetries.  ``test_pins_catch_planted_faults``
shows that each plausible mistake (sign, 2 pi, transposed coordinates, a
dropped term, a missing conjugate) breaks at least one pin.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle

TWO_PI = 2.0 * math.pi


def exact_frac(p, r):
    """Exact fractional part of <p, r> in [-1/2, 1/2] from the binary values."""
    s = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(p, r))
    return float(s - round(s))


def pin_single_point_source(rng):
    """P1: I = a delta_{n0}  =>  V_k = a exp(-2 pi i <p_k, r_n0>), |p.r| ~ 1e5;
    one visibility  =>  I_n = V exp(+2 pi i <p, r_n>)."""
    M, N = 64, 17
    uvw = rng.uniform(-1.2e5, 1.2e5, (M, 3))
    xyz = rng.normal(size=(N, 3)); xyz /= np.linalg.norm(xyz, axis=1, keepdims=True)
    n0 = 5
    a = 0.7 - 0.2j
    sky = np.zeros(N, complex); sky[n0] = a
    V = oracle.synthesis(uvw, xyz, sky)[0]
    exp_V = np.array([a * complex(math.cos(TWO_PI * exact_frac(uvw[k], xyz[n0])),
                                  -math.sin(TWO_PI * exact_frac(uvw[k], xyz[n0]))) for k in range(M)])
    ok1 = np.max(np.abs(V - exp_V)) < 1e-13
    k0 = 9
    b = -1.3 + 0.4j
    vis = np.zeros(M, complex); vis[k0] = b
    I = oracle.analysis(uvw, xyz, vis)[0]
    exp_I = np.array([b * complex(math.cos(TWO_PI * exact_frac(uvw[k0], xyz[n])),
                                  math.sin(TWO_PI * exact_frac(uvw[k0], xyz[n]))) for n in range(N)])
    ok2 = np.max(np.abs(I - exp_I)) < 1e-13
    return bool(ok1 and ok2)


def pin_geometric_series(rng):
    """P2: collinear equispaced pixels r_n = r0 + n*D, unit weights:
    V(p) = exp(-2 pi i p.r0) (1 - q^N) / (1 - q),  q = exp(-2 pi i p.D)."""
    N = 700
    r0 = np.array([0.11, -0.07, 0.95])
    D = np.array([3.1e-4, 1.7e-4, -2.3e-4])
    xyz = r0[None, :] + np.arange(N)[:, None] * D[None, :]
    uvw = rng.uniform(-900.0, 900.0, (40, 3))
    V = oracle.synthesis(uvw, xyz, np.ones(N))[0]
    q = np.exp(-2j * np.pi * (uvw @ D))
    qN = np.exp(-2j * np.pi * N * (uvw @ D))
    closed = np.exp(-2j * np.pi * (uvw @ r0)) * (1 - qN) / (1 - q)
    return bool(np.max(np.abs(V - closed)) / np.max(np.abs(closed)) < 1e-10)


def pin_dft_lattice(rng):
    """P3: sources on a 3D lattice x = (n1/N1, n2/N2, n3/N3), targets at the
    integer frequencies k: synthesis is numpy's fftn, analysis its unnormalised
    inverse; Parseval ||A x||^2 = N ||x||^2."""
    N1, N2, N3 = 8, 6, 5
    g = np.stack(np.meshgrid(np.arange(N1) / N1, np.arange(N2) / N2, np.arange(N3) / N3,
                             indexing="ij"), -1).reshape(-1, 3)
    k = np.stack(np.meshgrid(np.arange(N1), np.arange(N2), np.arange(N3),
                             indexing="ij"), -1).reshape(-1, 3).astype(float)
    x = rng.normal(size=N1 * N2 * N3) + 1j * rng.normal(size=N1 * N2 * N3)
    V = oracle.synthesis(k, g, x)[0]
    ref = np.fft.fftn(x.reshape(N1, N2, N3)).ravel()
    ok1 = np.max(np.abs(V - ref)) / np.max(np.abs(ref)) < 1e-12
    y = rng.normal(size=k.shape[0]) + 1j * rng.normal(size=k.shape[0])
    I = oracle.analysis(k, g, y)[0]
    ref2 = np.fft.ifftn(y.reshape(N1, N2, N3)).ravel() * (N1 * N2 * N3)
    ok2 = np.max(np.abs(I - ref2)) / np.max(np.abs(ref2)) < 1e-12
    ok3 = abs(np.vdot(V, V).real - x.size * np.vdot(x, x).real) < 1e-10 * x.size * np.vdot(x, x).real
    return bool(ok1 and ok2 and ok3)


def pin_brute_force(rng):
    """P4: explicit complex128 matrix exp(-2 pi i P R^T) for tiny sizes."""
    P = rng.uniform(-300, 300, (31, 3))
    R = rng.normal(size=(23, 3)); R /= np.linalg.norm(R, axis=1, keepdims=True)
    A = np.exp(-2j * np.pi * (P @ R.T))
    x = rng.normal(size=23) + 1j * rng.normal(size=23)
    y = rng.normal(size=31) + 1j * rng.normal(size=31)
    ok1 = np.max(np.abs(oracle.synthesis(P, R, x)[0] - A @ x)) < 1e-10
    ok2 = np.max(np.abs(oracle.analysis(P, R, y)[0] - A.conj().T @ y)) < 1e-10
    return bool(ok1 and ok2)


def pin_adjoint(rng):
    """P5: <A x, y> = <x, A^H y> to 1e-13 relative."""
    P = rng.uniform(-2e4, 2e4, (300, 3))
    R = rng.normal(size=(200, 3)); R /= np.linalg.norm(R, axis=1, keepdims=True)
    x = rng.normal(size=200) + 1j * rng.normal(size=200)
    y = rng.normal(size=300) + 1j * rng.normal(size=300)
    Ax = oracle.synthesis(P, R, x)[0]
    AHy = oracle.analysis(P, R, y)[0]
    lhs = np.vdot(y, Ax)
    rhs = np.vdot(AHy, x)
    scale = np.linalg.norm(Ax) * np.linalg.norm(y)
    return bool(abs(lhs - rhs) < 1e-13 * scale)


def pin_symmetries(rng):
    """P6: real I => V(-p) = conj V(p); a shift p -> p + D multiplies column n
    by exp(-2 pi i D.r_n); p = 0 => V = sum I; linearity."""
    P = rng.uniform(-5e3, 5e3, (50, 3))
    R = rng.normal(size=(60, 3)); R /= np.linalg.norm(R, axis=1, keepdims=True)
    x = rng.random(60)
    V = oracle.synthesis(P, R, x)[0]
    Vm = oracle.synthesis(-P, R, x)[0]
    ok1 = np.max(np.abs(Vm - V.conj())) < 1e-11
    D = np.array([12.5, -3.25, 7.0])
    z = rng.normal(size=60) + 1j * rng.normal(size=60)
    lhs = oracle.synthesis(P + D, R, z)[0]
    rhs = oracle.synthesis(P, R, z * np.exp(-2j * np.pi * (R @ D)))[0]
    ok2 = np.max(np.abs(lhs - rhs)) < 1e-9
    V0 = oracle.synthesis(np.zeros((1, 3)), R, z)[0]
    ok3 = abs(V0[0] - z.sum()) < 1e-12
    z2 = rng.normal(size=60) + 1j * rng.normal(size=60)
    a, b = 0.3 - 1.1j, 2.0 + 0.5j
    lin = oracle.synthesis(P, R, a * z + b * z2)[0]
    ok4 = np.max(np.abs(lin - (a * oracle.synthesis(P, R, z)[0] + b * oracle.synthesis(P, R, z2)[0]))) < 1e-9
    return bool(ok1 and ok2 and ok3 and ok4)


PINS = {
    "single_point_source": pin_single_point_source,
    "geometric_series": pin_geometric_series,
    "dft_lattice": pin_dft_lattice,
    "brute_force": pin_brute_force,
    "adjoint": pin_adjoint,
    "symmetries": pin_symmetries,
}


def run_pins(seed=0):
    return {name: f(np.random.default_rng(seed + i)) for i, (name, f) in enumerate(PINS.items())}


@pytest.mark.parametrize("name", list(PINS))
def test_pin(name):
    assert PINS[name](np.random.default_rng(123)), name


@pytest.mark.parametrize("fault", [oracle.FAULT_SIGN, oracle.FAULT_NO_TWO_PI, oracle.FAULT_SWAP_XY,
                                   oracle.FAULT_DROP_LAST, oracle.FAULT_NO_CONJ])
def test_pins_catch_planted_faults(fault):
    with oracle.planted_fault(fault):
        res = run_pins()
    assert not all(res.values()), f"fault {fault} not caught: {res}"
    assert all(run_pins().values())


def test_rows_subset_matches_full():
    rng = np.random.default_rng(7)
    P = rng.uniform(-1e3, 1e3, (90, 3))
    R = rng.normal(size=(70, 3))
    x = rng.normal(size=(2, 70)) + 1j * rng.normal(size=(2, 70))
    y = rng.normal(size=(2, 90)) + 1j * rng.normal(size=(2, 90))
    rows = np.array([3, 0, 89, 41])
    full = oracle.synthesis(P, R, x)
    assert np.array_equal(oracle.synthesis(P, R, x, rows=rows), full[:, rows])
    fa = oracle.analysis(P, R, y)
    prow = np.array([69, 1, 2])
    assert np.array_equal(oracle.analysis(P, R, y, rows=prow), fa[:, prow])


def test_rejects_bad_rows():
    with pytest.raises(ValueError):
        oracle.synthesis(np.zeros((3, 3)), np.zeros((2, 3)), np.ones(2), rows=np.array([3]))


def test_phase_reduction_beats_naive():
    """At |p.r| ~ 1e5 cycles the compensated phase stays exact to ~1e-16, while
    a naive double dot product drifts by ~1e-11: the P1 tolerance separates them."""
    rng = np.random.default_rng(11)
    p = rng.uniform(-1e5, 1e5, 3)
    r = rng.normal(size=3); r /= np.linalg.norm(r)
    f_exact = exact_frac(p, r)
    V = oracle.synthesis(p[None, :], r[None, :], np.ones(1))[0, 0]
    expect = complex(math.cos(TWO_PI * f_exact), -math.sin(TWO_PI * f_exact))
    assert abs(V - expect) < 1e-13
