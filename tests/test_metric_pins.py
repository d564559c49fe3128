"""Pins of the oracle's error metrics.

Every parity test passes through ``oracle.rel_l2`` (relative l2 error over all
outputs and rows, the reading of the paper's "relative accuracy", Sect. 5.2)
and ``oracle.max_rel_err`` (largest single error over the largest reference
entry).  A squared, per-row-averaged, wrongly normalised, max-norm or
real-part-only metric would let wrong results pass, so both are fixed here by
values worked out by hand, and each planted mistake is shown to break at
least one of them.
"""
import math

import numpy as np
import pytest

import oracle


def _close(a, b, tol=1e-14):
    return abs(a - b) <= tol * max(1.0, abs(b))


def metric_pins() -> dict:
    ref2 = np.array([[3.0, 0.0], [0.0, 4.0]])
    err2 = np.array([[0.3, 0.0], [0.0, 0.0]])
    z = np.array([1.0 + 0.0j, 2.0j])
    return {
        # one entry off by 1e-3: 1e-3 (squared would give 1e-6)
        "rel_small": _close(oracle.rel_l2([1.0 + 1e-3], [1.0]), 1e-3, 1e-9),
        # doubling: ||2y - y|| / ||y|| = 1 (normalising by ||2y|| would give 1/2)
        "rel_double": _close(oracle.rel_l2(2 * np.array([1.0, -2.0, 0.5j]), np.array([1.0, -2.0, 0.5j])), 1.0),
        "rel_exact": oracle.rel_l2([1.0, 2.0], [1.0, 2.0]) == 0.0,
        # an imaginary error of half the reference: 1/2 (a real-part-only metric gives 0)
        "rel_imag": _close(oracle.rel_l2(np.array([2.0, -4.0]) * (1 + 0.5j), [2.0, -4.0]), 0.5),
        # two rows: norm over all entries, 0.3 / 5 (a per-row mean gives 0.05, a max norm 0.075)
        "rel_rows": _close(oracle.rel_l2(ref2 + err2, ref2), 0.06),
        # 3-4-5: 0.05 / 5 (a max norm gives 0.0125)
        "rel_pythagoras": _close(oracle.rel_l2(np.array([3.05, 4.0]), np.array([3.0, 4.0])), 0.01),
        # element-wise: largest error over the largest reference entry
        "max_rows": _close(oracle.max_rel_err(ref2 + err2, ref2), 0.075),
        "max_double": _close(oracle.max_rel_err(2 * z, z), 1.0),
        "max_imag": _close(oracle.max_rel_err(z + np.array([0.0, 0.1j]), z), 0.05),
        "max_exact": oracle.max_rel_err(z, z) == 0.0,
    }


def test_metric_pins_hold():
    res = metric_pins()
    assert all(res.values()), res


@pytest.mark.parametrize("fault", oracle.METRIC_FAULTS)
def test_metric_pins_catch_planted_faults(fault):
    with oracle.planted_metric_fault(fault):
        res = metric_pins()
    assert not all(res.values()), f"planted metric fault {fault!r} not caught"
    assert all(metric_pins().values())


def test_rel_l2_scale_invariance_and_zero_reference():
    rng = np.random.default_rng(3)
    y = rng.normal(size=(3, 50)) + 1j * rng.normal(size=(3, 50))
    r = y + 1e-5 * rng.normal(size=(3, 50))
    a = oracle.rel_l2(y, r)
    assert math.isclose(oracle.rel_l2(7.5 * y, 7.5 * r), a, rel_tol=1e-9)
    assert math.isclose(oracle.max_rel_err(7.5 * y, 7.5 * r), oracle.max_rel_err(y, r), rel_tol=1e-9)
    # a zero reference reports the absolute norm of the result
    assert oracle.rel_l2([3.0, 4.0], [0.0, 0.0]) == 5.0
