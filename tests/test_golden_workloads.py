"""The synthetic workloads against the sizes the paper prints for its runtime
experiments (tests/golden/, each file citing its table): the dense DCOS
ladder's visibility and pixel counts (Sect. 5.1, Table 3) and the default
benchmark configuration of its 1 km rung (Sect. 5, Table 2)."""
import inspect
import math
import os

import numpy as np
import pytest

from paper_2306_06007_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def _ladder():
    out = {}
    for r, v, p in _rows("runtime_ladder.txt"):
        out[float(r)] = (v, p)
    return out


def test_ladder_table_matches_the_paper():
    """Every rung of the generator's table rounds to the printed figures: the
    visibility target to the printed count (exact below 13k, else to the
    thousand) and the square mesh to the printed megapixels at the printed
    number of decimals."""
    gold = _ladder()
    assert sorted(gold) == sorted(W.DENSE_LADDER)
    for r, (v, p) in gold.items():
        n_vis, n_side = W.DENSE_LADDER[r]
        if v.endswith("k"):
            assert round(n_vis / 1000) == int(v[:-1]), r
        else:
            assert n_vis == int(v), r
        decimals = len(p.split(".")[1]) if "." in p else 0
        assert round(n_side * n_side / 1e6, decimals) == float(p), r


@pytest.mark.parametrize("radius_km", [0.1, 0.3, 1.0])
def test_generated_rungs_have_the_printed_sizes(radius_km):
    """The generated visibilities (three snapshots of every station pair) and
    pixels of the small rungs round to the printed figures."""
    v, p = _ladder()[radius_km]
    wl = W.dense_dcos(radius_km)
    if v.endswith("k"):
        assert round(wl.n_vis / 1000) == int(v[:-1])
    else:
        assert wl.n_vis == int(v)
    decimals = len(p.split(".")[1])
    assert round(wl.n_pix / 1e6, decimals) == float(p)


def test_one_km_rung_has_the_default_configuration():
    """Table 2's defaults: 94,878 visibilities, one channel at 150 MHz (the
    generator's 2 m wavelength is 150 MHz to 0.07%), declination -45 deg, a
    30-degree field on a 360 x 360 mesh, three time intervals over 8 hours."""
    d = {k: float(v) for k, v in _rows("benchmark_defaults.txt")}
    wl = W.dense_dcos(d["max_radius_km"])
    assert wl.n_vis == int(d["n_visibilities"])
    assert wl.n_pix == int(d["image_side_pixels"]) ** 2
    assert wl.info["fov_deg"] == d["field_of_view_deg"]
    assert inspect.signature(W.dense_dcos).parameters["dec_deg"].default == d["declination_deg"]
    assert abs(299.792458 / d["central_frequency_mhz"] - 2.0) / 2.0 < 1e-3
    # the mesh spans the field: its corner direction cosines are sin(fov / 2)
    half = math.sin(math.radians(d["field_of_view_deg"]) / 2.0)
    assert np.isclose(np.abs(wl.xyz[:, 0]).max(), half) and np.isclose(np.abs(wl.xyz[:, 1]).max(), half)
    # three snapshots: the visibility count is three times the station pairs
    n_st = wl.info["n_stations"]
    assert wl.n_vis == int(d["time_intervals"]) * n_st * (n_st - 1) // 2
