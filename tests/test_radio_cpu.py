"""Radio front end (dirty2vis / vis2dirty) on the CPU: coordinate conventions
of the direction-cosine mesh and the channel layout; plans built on the host."""
import numpy as np
import pytest

import paper_2306_06007_amd as hv
from paper_2306_06007_amd import radio


def test_dcos_points_are_unit_vectors_shifted_by_one_along_n():
    rng = np.random.default_rng(7)
    l, m = rng.uniform(-0.5, 0.5, 200), rng.uniform(-0.5, 0.5, 200)
    r = radio.dcos_points(l, m)
    n = r[:, 2] + 1.0
    assert np.allclose(r[:, 0], l) and np.allclose(r[:, 1], m)
    assert np.allclose(l * l + m * m + n * n, 1.0, atol=1e-15)
    assert np.all(n > 0)
    # the phase centre is the origin, and n - 1 keeps full relative precision near it
    assert np.array_equal(radio.dcos_points([0.0], [0.0]), np.zeros((1, 3)))
    tiny = radio.dcos_points([1e-9], [0.0])[0, 2]
    assert tiny == pytest.approx(-0.5e-18, rel=1e-12)


def test_dcos_points_reject_points_off_the_sphere():
    with pytest.raises(ValueError):
        radio.dcos_points([0.8], [0.7])
    with pytest.raises(ValueError):
        radio.dcos_points([0.1, 0.2], [0.1])


def test_channel_uvw_layout_and_scaling():
    uvw = np.array([[100.0, -50.0, 3.0], [10.0, 20.0, -1.0]])
    f = np.array([1.0e8, 1.5e8, 2.0e8])
    p = radio.channel_uvw(uvw, f)
    assert p.shape == (6, 3)
    for r in range(2):
        for c in range(3):
            assert np.allclose(p[3 * r + c], uvw[r] * f[c] / 299_792_458.0)
    with pytest.raises(ValueError):
        radio.channel_uvw(uvw, [0.0])
    with pytest.raises(ValueError):
        radio.channel_uvw(uvw[:, :2], f)


def test_radio_plan_on_the_host():
    rng = np.random.default_rng(8)
    uvw = rng.normal(0.0, 300.0, (500, 3))
    g = np.linspace(-0.05, 0.05, 16)
    l, m = np.meshgrid(g, g)
    with radio.RadioPlan(uvw, [1.2e8, 1.3e8], l, m, 1e-4, "f32", host_only=True) as rp:
        info = rp.plan.info()
        assert (rp.n_rows, rp.n_chan, rp.n_pix) == (500, 2, 256)
        assert info["n_vis"] == 1000 and info["n_pix"] == 256
