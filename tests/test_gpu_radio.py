"""GPU checks of the radio front end (dirty2vis / vis2dirty on a direction-
cosine image with the DCOS phase reference w (n - 1), Sect. 2.1 Eq. 4).

Pins independent of the oracle: a unit point source gives the closed form
exp(-2 pi i (u l0 + v m0 + w (n0 - 1))) on every visibility, and the pair is
adjoint.  Against the oracle: its direct sums on the points (l, m, n - 1)."""
import numpy as np
import pytest

import oracle
from paper_2306_06007_amd import radio

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _setup(seed=9, n_rows=3000, side=48, fov=0.2):
    rng = np.random.default_rng(seed)
    uvw = np.stack([rng.normal(0, 400.0, n_rows), rng.normal(0, 400.0, n_rows), rng.normal(0, 40.0, n_rows)], 1)
    g = np.linspace(-fov / 2, fov / 2, side)
    l, m = np.meshgrid(g, g)
    return uvw, np.array([1.0e8, 1.4e8]), l.ravel(), m.ravel(), rng


def _np(t):
    return t.detach().cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("dtype,eps", [("f32", 1e-4), ("f64", 1e-9)])
def test_point_source_closed_form(dtype, eps):
    uvw, f, l, m, _ = _setup()
    j0 = 1234
    dirty = np.zeros(l.size)
    dirty[j0] = 1.0
    V = _np(radio.dirty2vis(uvw, f, dirty, l, m, eps, dtype))
    p = radio.channel_uvw(uvw, f).reshape(uvw.shape[0], f.size, 3)
    n0 = np.sqrt(1.0 - l[j0] ** 2 - m[j0] ** 2)
    ref = np.exp(-2j * np.pi * (p[..., 0] * l[j0] + p[..., 1] * m[j0] + p[..., 2] * (n0 - 1.0)))
    assert V.shape == ref.shape
    assert oracle.rel_l2(V, ref) <= eps


@pytest.mark.parametrize("dtype,eps,thr", [("f32", 1e-4, -1.0), ("f64", 1e-9, -1.0), ("f32", 1e-4, 0.0),
                                           ("f64", 1e-9, 0.0)])
def test_against_oracle_two_polarisations(dtype, eps, thr):
    """thr = 0: every sub-problem through the NUFFT path."""
    uvw, f, l, m, rng = _setup()
    dirty = rng.uniform(0, 1, (2, l.size))
    vis = rng.normal(size=(2, uvw.shape[0], f.size)) + 1j * rng.normal(size=(2, uvw.shape[0], f.size))
    with radio.RadioPlan(uvw, f, l, m, eps, dtype, direct_threshold=thr) as rp:
        V = _np(rp.dirty2vis(dirty))
        I = _np(rp.vis2dirty(vis))
    p, r = radio.channel_uvw(uvw, f), radio.dcos_points(l, m)
    Vref = oracle.synthesis(p, r, dirty).reshape(V.shape)
    Iref = oracle.analysis(p, r, vis.reshape(2, -1))
    assert oracle.rel_l2(V, Vref) <= eps
    assert oracle.rel_l2(I, Iref) <= eps


def test_adjoint_pair():
    uvw, f, l, m, rng = _setup(seed=10)
    x = rng.normal(size=l.size) + 1j * rng.normal(size=l.size)
    y = rng.normal(size=(uvw.shape[0], f.size)) + 1j * rng.normal(size=(uvw.shape[0], f.size))
    with radio.RadioPlan(uvw, f, l, m, 1e-9, "f64") as rp:
        Ax = _np(rp.dirty2vis(x)).reshape(y.shape)
        AHy = _np(rp.vis2dirty(y)).reshape(x.shape)
    lhs, rhs = np.vdot(y, Ax), np.vdot(AHy, x)
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)


def test_channels_and_partition_reuse():
    """Two channels in one call equal two single-channel calls, and a plan built
    on an exported partition reproduces the original plan's results."""
    uvw, f, l, m, rng = _setup(seed=11)
    dirty = rng.uniform(0, 1, l.size)
    V2 = _np(radio.dirty2vis(uvw, f, dirty, l, m, 1e-9, "f64"))
    for c in range(f.size):
        Vc = _np(radio.dirty2vis(uvw, f[c:c + 1], dirty, l, m, 1e-9, "f64"))[:, 0]
        assert oracle.rel_l2(V2[:, c], Vc) <= 1e-9
    with radio.RadioPlan(uvw, f, l, m, 1e-9, "f64", max_fft_bytes=2e6) as rp:
        V = _np(rp.dirty2vis(dirty))
        vc, sc = rp.export_partition()
        n_chunks = rp.plan.info()["n_vis_chunks"]
    assert vc.shape == (uvw.shape[0], f.size) and n_chunks > 1
    with radio.RadioPlan(uvw, f, l, m, 1e-9, "f64", max_fft_bytes=2e6, vis_chunk=vc.ravel(), sky_chunk=sc) as rp2:
        V_re = _np(rp2.dirty2vis(dirty))
        assert rp2.plan.info()["n_vis_chunks"] == n_chunks
    assert oracle.rel_l2(V_re, V) <= 1e-10
