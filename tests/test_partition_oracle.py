"""Pins of the partitioning restatements in ``oracle.partition``.

Algorithm 1 (Sect. 3.2): the LP's optimal value has a closed form, because
the objective only depends on sum(u) + sum(v): the optimum is
min(0, log(V_max / prod(B P))) whatever alpha >= 1 is.  Algorithm 2: the
partition is not unique, so the checks are its invariants -- a disjoint cover
of the points, every chunk box within h, lattice cells never split, and no
two final chunks that could still be fused (a fixpoint of step 4).
"""
import math

import numpy as np
import pytest

from oracle import partition as P


@pytest.mark.parametrize("alpha", [1.0, 1.5, 4.0])
def test_alg1_optimum_closed_form(alpha):
    rng = np.random.default_rng(int(alpha * 10))
    for _ in range(5):
        B = rng.uniform(1e2, 1e5, 3)
        Pw = rng.uniform(1e-3, 1.0, 3)
        vmax = float(np.prod(B * Pw)) * rng.uniform(1e-6, 2.0)
        val, h, eta = P.lp_optimum(B, Pw, vmax, alpha)
        c = math.log(vmax / np.prod(B * Pw))
        assert abs(val - min(0.0, c)) < 1e-7
        assert P.lp_feasible(B, Pw, vmax, alpha, h, eta, rtol=1e-6)


def _clustered(rng, n):
    c = rng.normal(size=(6, 3)) * [50.0, 40.0, 5.0]
    lab = rng.integers(0, 6, n)
    return c[lab] + rng.normal(size=(n, 3)) * [4.0, 6.0, 1.0]


def _boxes(x, labels):
    out = []
    for j in range(labels.max() + 1):
        pts = x[labels == j]
        out.append((pts.min(0), pts.max(0)))
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_alg2_invariants(seed):
    rng = np.random.default_rng(seed)
    x = _clustered(rng, 400)
    h = np.array([12.0, 15.0, 3.0])
    lab = P.partition_points(x, h)
    assert lab.shape == (400,) and lab.min() == 0
    assert set(np.unique(lab)) == set(range(lab.max() + 1))          # no empty chunk
    boxes = _boxes(x, lab)
    for lo, hi in boxes:
        assert np.all(hi - lo <= h)                                    # within h
    # lattice cells are atomic: points of one cell share a chunk
    lo = x.min(0)
    K = [max(1, math.ceil((x[:, d].max() - lo[d]) / h[d])) for d in range(3)]
    cells = np.stack([np.minimum(K[d] - 1, np.floor((x[:, d] - lo[d]) / h[d]).astype(int))
                      for d in range(3)], 1)
    key = cells[:, 0] + K[0] * (cells[:, 1] + K[1] * cells[:, 2])
    for k in np.unique(key):
        assert len(np.unique(lab[key == k])) == 1
    # fixpoint: no pair of final chunks is still fusable
    for i in range(len(boxes)):
        for j in range(i + 1, len(boxes)):
            ulo = np.minimum(boxes[i][0], boxes[j][0])
            uhi = np.maximum(boxes[i][1], boxes[j][1])
            assert not np.all(uhi - ulo <= h)
    # deterministic
    assert np.array_equal(lab, P.partition_points(x, h))


def test_alg2_single_cell_and_line():
    x = np.array([[0.0, 0, 0], [0.5, 0, 0], [1.0, 0, 0]])
    assert np.array_equal(P.partition_points(x, [10.0, 1.0, 1.0]), [0, 0, 0])
    # h = 0.6 on a line of 0, 0.5, 1.0: cells {0, 0.5} and {1.0}; their union
    # spans 1.0 > 0.6, so two chunks remain
    lab = P.partition_points(x, [0.6, 1.0, 1.0])
    assert np.array_equal(lab, [0, 0, 1])
    # fusion moves volumes off the lattice: cells {0.05}, {0.65} fuse (span 0.6)
    y = np.array([[0.05, 0, 0], [0.65, 0, 0], [1.3, 0, 0]])
    lab = P.partition_points(y, [0.6, 1.0, 1.0])
    assert lab[0] == lab[1] != lab[2]


# ---- pins of the feasibility checker of Algorithm 1 -------------------------------
def feasibility_pins() -> dict:
    """Points that break exactly one constraint family of Algorithm 1 (and a
    feasible one): a checker that drops any family accepts one of them."""
    B = np.array([1.0e3, 2.0e3, 50.0])
    Pw = np.array([0.3, 0.2, 0.01])
    vol = float(np.prod(B * Pw))
    vmax = vol * 1e-6                          # closed form at alpha = 1: t = 0.1
    t = 0.1
    a = 0.5 * math.log(1.8)                    # log(1.8) > log(1.5) = log(alpha)
    res = {}
    res["feasible_closed_form"] = P.lp_feasible(B, Pw, vmax, 1.0, t * B, t * Pw)
    # FFT memory: every dimension 1.05x the optimum, prod(h eta) = 1.05^6 vmax
    res["budget"] = not P.lp_feasible(B, Pw, vmax, 1.0, 1.05 * t * B, 1.05 * t * Pw)
    # h <= B: one visibility box 1.5x the full width (alpha = 2 admits the spread, no budget)
    h = B.copy(); h[0] *= 1.5
    res["upper_bound"] = not P.lp_feasible(B, Pw, 1e300, 2.0, h, Pw.copy())
    # same-domain anisotropy: u_0 - u_1 = log 1.8 > log 1.5, cross differences a < log 1.5, same volume
    h = t * B * np.exp([a, -a, 0.0])
    res["same_domain"] = not P.lp_feasible(B, Pw, vmax, 1.5, h, t * Pw)
    # cross anisotropy: u_k - v_j = log 1.8 for every pair, same-domain differences 0, same volume
    res["cross"] = not P.lp_feasible(B, Pw, vmax, 1.5, t * B * math.exp(a), t * Pw * math.exp(-a))
    # positivity
    h = t * B; h[2] = 0.0
    res["positive"] = not P.lp_feasible(B, Pw, vmax, 1.0, h, t * Pw)
    return res


def test_feasibility_pins_hold():
    res = feasibility_pins()
    assert all(res.values()), res


@pytest.mark.parametrize("fault", P.FEASIBLE_FAULTS)
def test_feasibility_pins_catch_planted_faults(fault):
    with P.planted_feasible_fault(fault):
        res = feasibility_pins()
    assert not all(res.values()), f"planted feasibility fault {fault!r} not caught: {res}"
    assert all(feasibility_pins().values())
