"""Plain restatements of HVOX's partitioning steps -- TEST INFRASTRUCTURE ONLY.

* ``max_heisenberg_dims``: Algorithm 1 (Sect. 3.2) written as the linear
  program it is in log variables and handed to scipy's LP solver (a library
  primitive).  Variables u_k = log(h_k / B_k), v_k = log(eta_k / P_k);
  minimising the chunk count prod(B/h) * prod(P/eta) is maximising
  sum(u) + sum(v), subject to
    - FFT memory:      sum(u) + sum(v) <= log(V_max / prod(B_k P_k)),
    - non-trivial:     u_k <= 0, v_k <= 0,
    - anisotropy:      |u_k - u_j| <= log(alpha), |v_k - v_j| <= log(alpha),
                       |u_k - v_j| <= log(alpha).
  The objective is degenerate (only the sum matters), so only the optimal
  value is unique; the planner's answer is checked for feasibility and for
  reaching this value.

* ``partition_points``: Algorithm 2 (Sect. 3.2), steps 1-4, in plain Python
  loops, with the readings the planner documents for what the paper leaves
  open:
    1. lattice origin at the point-set box minimum, K_d = max(1, ceil(W_d/h_d))
       cells per dimension, cell index min(K_d - 1, floor((x_d - lo_d) / h_d));
    2. every point goes to its cell;
    3. empty cells are dropped;
    4. chunks start as the occupied cells (tight point boxes).  Chunks are
       visited in ascending cell key  key = c_x + K_x (c_y + K_y c_z).  The
       visited chunk repeatedly absorbs the admissible chunk (union box width
       <= h_d in every dimension) whose box centre is nearest in h-scaled
       distance (ties: smaller key), until none is admissible.
  Partitions are not unique in the paper; this reading is deterministic, and
  the planner implements the same reading independently.
"""
from __future__ import annotations

import math

import numpy as np


def lp_optimum(B, P, v_max, alpha=1.0):
    """Optimal value of sum(u)+sum(v) for Algorithm 1, via scipy.optimize.linprog,
    and one optimal (h, eta)."""
    from scipy.optimize import linprog

    B = np.asarray(B, dtype=float)
    P = np.asarray(P, dtype=float)
    c_rhs = math.log(v_max) - float(np.sum(np.log(B)) + np.sum(np.log(P)))
    la = math.log(alpha)
    n = 6
    A, b = [], []
    A.append([1.0] * n); b.append(c_rhs)
    for i in range(n):
        row = [0.0] * n; row[i] = 1.0
        A.append(row); b.append(0.0)
    idx_u = [0, 1, 2]
    idx_v = [3, 4, 5]
    pairs = [(i, j) for i in idx_u for j in idx_u if i != j]
    pairs += [(i, j) for i in idx_v for j in idx_v if i != j]
    pairs += [(i, j) for i in idx_u for j in idx_v]
    pairs += [(j, i) for i in idx_u for j in idx_v]
    for i, j in pairs:
        row = [0.0] * n; row[i] = 1.0; row[j] = -1.0
        A.append(row); b.append(la)
    res = linprog(c=-np.ones(n), A_ub=np.array(A), b_ub=np.array(b),
                  bounds=[(None, None)] * n, method="highs")
    if res.status != 0:
        raise RuntimeError(res.message)
    x = res.x
    h = B * np.exp(x[:3])
    eta = P * np.exp(x[3:])
    return float(np.sum(x)), h, eta


# Planted mistakes of ``lp_feasible`` (tests switch them on to show that its
# pins catch them); None = the correct checker.
_feasible_fault = None
FEASIBLE_FAULTS = ("always_true", "no_budget", "no_upper_bounds", "no_same_domain_bounds", "no_cross_bounds",
                   "no_positivity")


class planted_feasible_fault:
    """Context manager switching ``lp_feasible`` to a deliberately wrong
    variant (used only by the tests of its pins)."""

    def __init__(self, kind: str):
        if kind not in FEASIBLE_FAULTS:
            raise ValueError(kind)
        self.kind = kind
        self.old = None

    def __enter__(self):
        global _feasible_fault
        self.old, _feasible_fault = _feasible_fault, self.kind
        return self

    def __exit__(self, *exc):
        global _feasible_fault
        _feasible_fault = self.old
        return False


def lp_feasible(B, P, v_max, alpha, h, eta, rtol=1e-9):
    """Check an (h, eta) against every constraint of Algorithm 1: positive
    dimensions, the FFT memory bound prod(h eta) <= V_max, h <= B and
    eta <= P, and the anisotropy bounds |u_k - u_j|, |v_k - v_j| and
    |u_k - v_j| <= log(alpha) in the log variables u = log(h/B),
    v = log(eta/P)."""
    if _feasible_fault == "always_true":
        return True
    B = np.asarray(B, float); P = np.asarray(P, float)
    h = np.asarray(h, float); eta = np.asarray(eta, float)
    if np.any(h <= 0) or np.any(eta <= 0):
        if _feasible_fault != "no_positivity":
            return False
        return True            # the faulty checker cannot take the logarithms below
    if _feasible_fault != "no_upper_bounds" and (np.any(h > B * (1 + rtol)) or np.any(eta > P * (1 + rtol))):
        return False
    if _feasible_fault != "no_budget" and np.prod(h * eta) > v_max * (1 + rtol):
        return False
    u = np.log(h / B); v = np.log(eta / P)
    la = math.log(alpha) + 1e-9
    if _feasible_fault != "no_same_domain_bounds":
        for a in (u, v):
            for i in range(3):
                for j in range(3):
                    if abs(a[i] - a[j]) > la:
                        return False
    if _feasible_fault != "no_cross_bounds":
        for i in range(3):
            for j in range(3):
                if abs(u[i] - v[j]) > la:
                    return False
    return True


def partition_points(x, h):
    """Algorithm 2 on points ``x`` (n, 3) with maximum box dimensions ``h``.

    Returns ``labels`` (n,) int: chunk index per point, chunks numbered in
    ascending order of their key."""
    x = np.asarray(x, dtype=float)
    h = [float(v) for v in h]
    n = x.shape[0]
    lo = [float(x[:, d].min()) for d in range(3)]
    hi = [float(x[:, d].max()) for d in range(3)]
    K = []
    for d in range(3):
        width = hi[d] - lo[d]
        K.append(max(1, int(math.ceil(width / h[d]))) if width > 0 else 1)

    # steps 1-3: occupied lattice cells with their tight point boxes
    cell_of = {}
    cells = {}
    for i in range(n):
        c = []
        for d in range(3):
            q = int(math.floor((float(x[i, d]) - lo[d]) / h[d]))
            c.append(min(K[d] - 1, max(0, q)))
        key = c[0] + K[0] * (c[1] + K[1] * c[2])
        cell_of[i] = key
        if key not in cells:
            cells[key] = {"cell": tuple(c), "lo": list(x[i]), "hi": list(x[i])}
        else:
            box = cells[key]
            for d in range(3):
                box["lo"][d] = min(box["lo"][d], float(x[i, d]))
                box["hi"][d] = max(box["hi"][d], float(x[i, d]))

    # step 4: greedy fusion
    owner = {key: key for key in cells}                   # cell key -> chunk key
    chunks = {key: {"cells": [key], "lo": list(cells[key]["lo"]), "hi": list(cells[key]["hi"])}
              for key in cells}

    def coords(key):
        cx = key % K[0]
        cy = (key // K[0]) % K[1]
        cz = key // (K[0] * K[1])
        return cx, cy, cz

    for a in sorted(cells):
        if a not in chunks:
            continue
        while True:
            ca = chunks[a]
            cc = [coords(k) for k in ca["cells"]]
            rng = [(min(c[d] for c in cc) - 1, max(c[d] for c in cc) + 1) for d in range(3)]
            cand = set()
            for cz in range(max(0, rng[2][0]), min(K[2] - 1, rng[2][1]) + 1):
                for cy in range(max(0, rng[1][0]), min(K[1] - 1, rng[1][1]) + 1):
                    for cx in range(max(0, rng[0][0]), min(K[0] - 1, rng[0][1]) + 1):
                        key = cx + K[0] * (cy + K[1] * cz)
                        if key in owner and owner[key] != a:
                            cand.add(owner[key])
            best, best_d = None, None
            for b in sorted(cand):
                cb = chunks[b]
                ok = True
                dist = 0.0
                for d in range(3):
                    ulo = min(ca["lo"][d], cb["lo"][d])
                    uhi = max(ca["hi"][d], cb["hi"][d])
                    if not (uhi - ulo <= h[d]):
                        ok = False
                        break
                    ma = 0.5 * (ca["lo"][d] + ca["hi"][d])
                    mb = 0.5 * (cb["lo"][d] + cb["hi"][d])
                    t = (ma - mb) / h[d]
                    dist += t * t
                if ok and (best is None or dist < best_d):
                    best, best_d = b, dist
            if best is None:
                break
            cb = chunks.pop(best)
            for k in cb["cells"]:
                owner[k] = a
            ca["cells"].extend(cb["cells"])
            for d in range(3):
                ca["lo"][d] = min(ca["lo"][d], cb["lo"][d])
                ca["hi"][d] = max(ca["hi"][d], cb["hi"][d])

    order = {key: j for j, key in enumerate(sorted(chunks))}
    return np.array([order[owner[cell_of[i]]] for i in range(n)], dtype=np.int64)
