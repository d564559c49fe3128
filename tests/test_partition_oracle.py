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
