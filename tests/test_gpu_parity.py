"""GPU parity of the HIP path against the FP64 oracle.

Every case runs the library through its C ABI (Python binding) on seeded
synthetic inputs and compares element by element with the oracle's direct
sums (HVOX Sect. 2, Eqs. 2-3).  The bar is the requested accuracy: relative
l2 error <= eps over all outputs (eps 1e-4 in float32, 1e-9 / 1e-6 in
float64); direct evaluation is held to the rounding of its precision.
"""
import math

import numpy as np
import pytest

import oracle
import paper_2306_06007_amd as hv
from paper_2306_06007_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _t(a, dtype):
    import torch
    cd = torch.complex128 if dtype == "f64" else torch.complex64
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=cd)


def _np(t):
    return t.detach().cpu().numpy().astype(np.complex128)


# Element-wise bar (the max-abs error relative to max |y_ref|, besides the
# relative l2 error <= eps): every single output within C_ELEM * eps of the
# oracle, relative to the largest reference output (measured: up to 3.5 eps over every
# case here, 7.5x the l2 average at most).  Errors of chunked type-3
# evaluation are not uniform over the targets (those near the corners of a
# sub-problem box, recovered from the most strongly deconvolved modes, carry the
# largest); C_ELEM bounds how far the worst one may stand above the l2 average.
C_ELEM = 5.0
ELEM_LOG = []      # (tag, rel-l2 syn, rel-l2 ana, max syn, max ana) of every case, printed at the end


def both_directions(uvw, xyz, sky, vis, eps, dtype, rows_vis=None, rows_pix=None, elem_bound=None, **kw):
    """Run synthesis and analysis on the GPU; return (err_syn, err_ana, plan
    info) as relative l2 errors against the oracle, after asserting the
    element-wise bar (C_ELEM * eps unless elem_bound is given; eps = 0 and
    elem_bound = 0 skip it)."""
    with hv.Plan(uvw, xyz, eps, dtype, **kw) as p:
        V = _np(p.synthesis(_t(sky, dtype)))
        I = _np(p.analysis(_t(vis, dtype)))
        info = p.info()
    Vref = oracle.synthesis(uvw, xyz, sky, rows=rows_vis)
    Iref = oracle.analysis(uvw, xyz, vis, rows=rows_pix)
    if rows_vis is not None:
        V = V[..., rows_vis]
    if rows_pix is not None:
        I = I[..., rows_pix]
    V = V.reshape(Vref.shape)
    I = I.reshape(Iref.shape)
    es, ea = oracle.rel_l2(V, Vref), oracle.rel_l2(I, Iref)
    ms, ma = oracle.max_rel_err(V, Vref), oracle.max_rel_err(I, Iref)
    ELEM_LOG.append((f"{dtype} eps={eps:g}", es, ea, ms, ma))
    print(f"  element-wise: syn max {ms:.3e} ({ms / max(es, 1e-300):.2f}x l2), "
          f"ana max {ma:.3e} ({ma / max(ea, 1e-300):.2f}x l2)", flush=True)
    bound = C_ELEM * eps if elem_bound is None else elem_bound
    if bound > 0:
        assert ms <= bound and ma <= bound, (ms, ma, bound)
    return es, ea, info


def _report(tag, es, ea, info):
    print(f"[{tag}] syn={es:.3e} ana={ea:.3e} chunks={info['n_vis_chunks']}x{info['n_sky_chunks']} "
          f"nufft={info['n_pairs_nufft']} direct={info['n_pairs_direct']} w={info['w']}", flush=True)


# ---- compact disk: 2,000 vis x 3,072 pixels ------------------------------------------
@pytest.mark.parametrize("dtype,eps", [("f64", 1e-6), ("f32", 1e-4), ("f64", 1e-9)])
def test_compact_disk_monolithic_nufft(dtype, eps):
    wl = W.compact_disk()
    es, ea, info = both_directions(wl.uvw, wl.xyz, wl.sky, wl.vis, eps, dtype, direct_threshold=0.0,
                                   max_fft_bytes=math.inf)
    _report(f"monolithic {dtype} {eps:g}", es, ea, info)
    assert info["n_pairs_nufft"] == 1
    assert es <= eps and ea <= eps


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-6)])
def test_compact_disk_all_direct(dtype, tol):
    wl = W.compact_disk()
    eps = 0.0 if dtype == "f64" else 1e-4
    es, ea, info = both_directions(wl.uvw, wl.xyz, wl.sky, wl.vis, eps, dtype, direct_threshold=math.inf,
                                   elem_bound=C_ELEM * tol)
    _report(f"direct {dtype}", es, ea, info)
    assert info["n_pairs_nufft"] == 0
    assert es <= tol and ea <= tol


# ---- chunked: SKA-like subset ---------------------------------------------------------
def _ska_small():
    return W.ska_like(n_pix=20000, n_ant=40, n_times=10)


@pytest.mark.parametrize("dtype,eps", [("f32", 1e-4), ("f64", 1e-9)])
@pytest.mark.parametrize("budget", [4e6, 64e6])
def test_chunked_forced_nufft(dtype, eps, budget):
    wl = _ska_small()
    es, ea, info = both_directions(wl.uvw, wl.xyz, wl.sky, wl.vis, eps, dtype, direct_threshold=0.0,
                                   max_fft_bytes=budget)
    _report(f"chunked {dtype} {eps:g} B={budget:g}", es, ea, info)
    assert info["n_vis_chunks"] * info["n_sky_chunks"] > 1
    assert es <= eps and ea <= eps


@pytest.mark.parametrize("dtype,eps", [("f32", 1e-4), ("f64", 1e-9)])
def test_chunked_auto(dtype, eps):
    wl = _ska_small()
    es, ea, info = both_directions(wl.uvw, wl.xyz, wl.sky, wl.vis, eps, dtype, max_fft_bytes=16e6)
    _report(f"auto {dtype} {eps:g}", es, ea, info)
    assert es <= eps and ea <= eps


@pytest.mark.parametrize("dtype,eps", [("f64", 1e-2), ("f64", 1e-4), ("f64", 1e-7), ("f64", 1e-8), ("f64", 1e-10),
                                       ("f32", 1e-2), ("f32", 1e-3), ("f32", 3e-5), ("f32", 1e-5)])
def test_eps_sweep(dtype, eps):
    """Accuracy compliance over requested eps (the paper's Sect. 5.2 study):
    achieved error <= requested, in the monolithic and the chunked case."""
    wl = W.compact_disk(n_vis=1500, n_pix=2000, radius=600.0, w_half=30.0)
    for budget in (math.inf, 2e6):
        es, ea, info = both_directions(wl.uvw, wl.xyz, wl.sky, wl.vis, eps, dtype, direct_threshold=0.0,
                                       max_fft_bytes=budget)
        _report(f"sweep {dtype} {eps:g} B={budget:g}", es, ea, info)
        assert es <= eps and ea <= eps


def test_mesh_agnostic():
    """HVOX performs identically irrespective of the sky mesh (Sect. 5.2):
    Fibonacci cap, random cap and a direction-cosine grid all meet eps."""
    rng = np.random.default_rng(5)
    uvw = W.uvw_disk(1500, 800.0, 40.0, rng)
    vis = W.complex_normal(1, 1500, rng)
    for xyz in (W.fibonacci_cap(2500, 6.0), W.random_cap(2500, 6.0, rng), W.dcos_grid(50, 10.0)):
        sky = W.real_intensities(1, xyz.shape[0], rng)
        es, ea, info = both_directions(uvw, xyz, sky, vis, 1e-4, "f32", direct_threshold=0.0, max_fft_bytes=4e6)
        _report("mesh", es, ea, info)
        assert es <= 1e-4 and ea <= 1e-4


def test_point_source_sky():
    """Accuracy protocol of Sect. 5.2: a point-source sky, ground truth by
    direct evaluation."""
    wl = W.compact_disk()
    sky = np.zeros((1, wl.n_pix), complex)
    sky[0, [10, 700, 2900]] = [1.0, 0.5, 2.0]
    es, ea, info = both_directions(wl.uvw, wl.xyz, sky, wl.vis, 1e-6, "f64", direct_threshold=0.0)
    assert es <= 1e-6 and ea <= 1e-6


def test_adjoint_identity_gpu():
    import torch
    wl = _ska_small()
    rng = np.random.default_rng(9)
    x = W.complex_normal(1, wl.n_pix, rng)
    y = W.complex_normal(1, wl.n_vis, rng)
    for dtype, eps in (("f64", 1e-9), ("f32", 1e-4)):
        with hv.Plan(wl.uvw, wl.xyz, eps, dtype, max_fft_bytes=16e6) as p:
            Ax = _np(p.synthesis(_t(x, dtype)))
            AHy = _np(p.analysis(_t(y, dtype)))
        lhs = np.vdot(y, Ax)
        rhs = np.vdot(AHy, x)
        scale = np.linalg.norm(Ax) * np.linalg.norm(y)
        assert abs(lhs - rhs) <= 2 * eps * scale


def test_ntrans_batch_equals_loop():
    import torch
    wl = W.compact_disk(ntrans=3)
    with hv.Plan(wl.uvw, wl.xyz, 1e-6, "f64", max_fft_bytes=4e6) as p:
        Vb = _np(p.synthesis(_t(wl.sky, "f64")))
        Ib = _np(p.analysis(_t(wl.vis, "f64")))
        # same launches row by row; only the order of float64 atomic additions may differ
        for t in range(3):
            assert oracle.rel_l2(Vb[t], _np(p.synthesis(_t(wl.sky[t], "f64")))) < 1e-13
            assert oracle.rel_l2(Ib[t], _np(p.analysis(_t(wl.vis[t], "f64")))) < 1e-13
    Vref = oracle.synthesis(wl.uvw, wl.xyz, wl.sky)
    assert oracle.rel_l2(Vb, Vref) <= 1e-6


@pytest.mark.parametrize("dtype,eps", [("f32", 1e-4), ("f64", 1e-9)])
def test_ntrans_row_passes_forced_nufft(dtype, eps):
    """Data rows (the ntrans of Sect. 4) through NUFFT sub-problems only, in
    passes of up to four rows that share the spreading and interpolation
    weights: every row meets eps against the oracle (l2 and element-wise), and
    in deterministic plans every row equals, bit for bit, the same row through
    a plan made for one row per call, and the same row alone.  Six rows make a
    pass of four and one of two; three rows one pass of three."""
    wl = W.ska_like(n_pix=20000, n_ant=40, n_times=10, ntrans=6)
    kw = dict(direct_threshold=0.0, max_fft_bytes=16e6, deterministic=True)
    with hv.Plan(wl.uvw, wl.xyz, eps, dtype, ntrans_hint=1, **kw) as p1:
        assert p1.info()["nufft_rows"] == 1
        V1 = _np(p1.synthesis(_t(wl.sky, dtype)))
        I1 = _np(p1.analysis(_t(wl.vis, dtype)))
    with hv.Plan(wl.uvw, wl.xyz, eps, dtype, ntrans_hint=4, **kw) as p:
        info = p.info()
        assert info["n_pairs_direct"] == 0 and info["nufft_rows"] == 4
        V = _np(p.synthesis(_t(wl.sky, dtype)))
        I = _np(p.analysis(_t(wl.vis, dtype)))
        V3 = _np(p.synthesis(_t(wl.sky[:3], dtype)))
        I3 = _np(p.analysis(_t(wl.vis[:3], dtype)))
        assert np.array_equal(V, V1) and np.array_equal(I, I1)
        assert np.array_equal(V3, V1[:3]) and np.array_equal(I3, I1[:3])
        for t in (0, 5):   # a one-dimensional input gives a one-dimensional output
            assert np.array_equal(V[t], _np(p.synthesis(_t(wl.sky[t], dtype))))
            assert np.array_equal(I[t], _np(p.analysis(_t(wl.vis[t], dtype))))
    Vref = oracle.synthesis(wl.uvw, wl.xyz, wl.sky)
    Iref = oracle.analysis(wl.uvw, wl.xyz, wl.vis)
    es, ea = oracle.rel_l2(V, Vref), oracle.rel_l2(I, Iref)
    ms, ma = oracle.max_rel_err(V, Vref), oracle.max_rel_err(I, Iref)
    print(f"[forced nufft 6 rows {dtype}] syn={es:.3e}/{ms:.3e} ana={ea:.3e}/{ma:.3e}", flush=True)
    assert es <= eps and ea <= eps
    assert ms <= C_ELEM * eps and ma <= C_ELEM * eps


def test_ntrans_row_passes_atomic_accumulation():
    """The same row passes without HVOX_DETERMINISTIC (crowded spreading tiles
    split, float64 atomics): four rows through one pass stay within eps of the
    oracle and agree with the rows alone to rounding."""
    wl = W.ska_like(n_pix=20000, n_ant=40, n_times=10, ntrans=4)
    with hv.Plan(wl.uvw, wl.xyz, 1e-4, "f32", ntrans_hint=4, direct_threshold=0.0, max_fft_bytes=16e6) as p:
        V = _np(p.synthesis(_t(wl.sky, "f32")))
        I = _np(p.analysis(_t(wl.vis, "f32")))
        for t in (1, 2):
            assert oracle.rel_l2(V[t], _np(p.synthesis(_t(wl.sky[t], "f32")))) <= 1e-6
            assert oracle.rel_l2(I[t], _np(p.analysis(_t(wl.vis[t], "f32")))) <= 1e-6
    Vref = oracle.synthesis(wl.uvw, wl.xyz, wl.sky)
    Iref = oracle.analysis(wl.uvw, wl.xyz, wl.vis)
    assert oracle.rel_l2(V, Vref) <= 1e-4 and oracle.rel_l2(I, Iref) <= 1e-4
    assert oracle.max_rel_err(V, Vref) <= C_ELEM * 1e-4 and oracle.max_rel_err(I, Iref) <= C_ELEM * 1e-4


@pytest.mark.parametrize("dtype,eps", [("f32", 1e-4), ("f64", 1e-9)])
def test_ntrans_hint_plans_match_oracle(dtype, eps):
    """Plans weighed for one and for four rows per call split the sub-problems
    differently between NUFFT grids and direct blocks; four-row calls through
    either stay within eps of the oracle."""
    wl = W.dense_dcos(1.0, ntrans=4)          # 95k vis x 130k pix: the hint moves its NUFFT pairs to direct
    rv = W.sample_rows(wl.n_vis, 256, seed=61)
    rp = W.sample_rows(wl.n_pix, 256, seed=62)
    Vref = oracle.synthesis(wl.uvw, wl.xyz, wl.sky, rows=rv)
    Iref = oracle.analysis(wl.uvw, wl.xyz, wl.vis, rows=rp)
    splits = []
    for hint in (1, 4):
        with hv.Plan(wl.uvw, wl.xyz, eps, dtype, ntrans_hint=hint) as p:
            V = _np(p.synthesis(_t(wl.sky, dtype)))[:, rv]
            I = _np(p.analysis(_t(wl.vis, dtype)))[:, rp]
            splits.append(p.info()["n_pairs_nufft"])
        es, ea = oracle.rel_l2(V, Vref), oracle.rel_l2(I, Iref)
        print(f"[ntrans hint {hint} {dtype}] syn={es:.3e} ana={ea:.3e} nufft={splits[-1]}", flush=True)
        assert es <= eps and ea <= eps
    assert splits[1] < splits[0]


def test_permutation_invariance():
    wl = W.compact_disk(n_vis=800, n_pix=900)
    rng = np.random.default_rng(2)
    pv = rng.permutation(wl.n_vis)
    ps = rng.permutation(wl.n_pix)
    with hv.Plan(wl.uvw, wl.xyz, 1e-9, "f64", direct_threshold=0.0) as p:
        V = _np(p.synthesis(_t(wl.sky, "f64")))
    with hv.Plan(wl.uvw[pv], wl.xyz[ps], 1e-9, "f64", direct_threshold=0.0) as q:
        Vp = _np(q.synthesis(_t(wl.sky[:, ps], "f64")))
    assert oracle.rel_l2(Vp, V[:, pv]) <= 2e-9


def test_real_sky_option():
    wl = W.compact_disk(n_vis=500, n_pix=600)
    with hv.Plan(wl.uvw, wl.xyz, 1e-6, "f64", real_sky=True, direct_threshold=0.0) as p:
        I = _np(p.analysis(_t(wl.vis, "f64")))
    ref = oracle.analysis(wl.uvw, wl.xyz, wl.vis)
    assert np.all(I.imag == 0)
    assert oracle.rel_l2(I.real, ref.real) <= 1e-6


@pytest.mark.parametrize("case", ["one_vis", "one_pix", "w_zero", "duplicates", "zero_baseline", "planar_sky"])
def test_degenerate_inputs(case):
    rng = np.random.default_rng(11)
    uvw = W.uvw_disk(400, 500.0, 20.0, rng)
    xyz = W.fibonacci_cap(500, 5.0)
    if case == "one_vis":
        uvw = uvw[:1]
    elif case == "one_pix":
        xyz = xyz[:1]
    elif case == "w_zero":
        uvw[:, 2] = 0.0
    elif case == "duplicates":
        uvw[100:200] = uvw[0]
        xyz[50:90] = xyz[3]
    elif case == "zero_baseline":
        uvw[::7] = 0.0
    elif case == "planar_sky":
        xyz = xyz.copy(); xyz[:, 2] = 1.0
    sky = W.real_intensities(1, xyz.shape[0], rng)
    vis = W.complex_normal(1, uvw.shape[0], rng)
    for dtype, eps in (("f64", 1e-9), ("f32", 1e-4)):
        es, ea, info = both_directions(uvw, xyz, sky, vis, eps, dtype, direct_threshold=0.0)
        _report(case, es, ea, info)
        assert es <= eps and ea <= eps


@pytest.mark.parametrize("case", ["one_vis", "one_pix", "duplicates", "planar_sky"])
def test_degenerate_inputs_in_row_passes(case):
    """The degenerate inputs again, three data rows through one NUFFT pass of a
    plan made for four rows per call (every sub-problem a NUFFT)."""
    rng = np.random.default_rng(12)
    uvw = W.uvw_disk(400, 500.0, 20.0, rng)
    xyz = W.fibonacci_cap(500, 5.0)
    if case == "one_vis":
        uvw = uvw[:1]
    elif case == "one_pix":
        xyz = xyz[:1]
    elif case == "duplicates":
        uvw[100:200] = uvw[0]
        xyz[50:90] = xyz[3]
    elif case == "planar_sky":
        xyz = xyz.copy(); xyz[:, 2] = 1.0
    sky = W.complex_normal(3, xyz.shape[0], rng)
    vis = W.complex_normal(3, uvw.shape[0], rng)
    for dtype, eps in (("f64", 1e-9), ("f32", 1e-4)):
        es, ea, info = both_directions(uvw, xyz, sky, vis, eps, dtype, direct_threshold=0.0, ntrans_hint=4)
        assert info["nufft_rows"] == 4
        _report(case + " rows", es, ea, info)
        assert es <= eps and ea <= eps


def test_empty_domains():
    import torch
    xyz = W.fibonacci_cap(50, 5.0)
    with hv.Plan(np.zeros((0, 3)), xyz, 1e-4, "f32") as p:
        I = p.analysis(torch.zeros((1, 0), dtype=torch.complex64, device="cuda"))
        assert I.shape == (1, 50) and torch.all(I == 0)
        V = p.synthesis(torch.ones((1, 50), dtype=torch.complex64, device="cuda"))
        assert V.shape == (1, 0)


def test_ragged_tails():
    """Sizes that are not multiples of any tile (256-target direct tiles,
    4-wavefront spread blocks, FFT line tiles)."""
    rng = np.random.default_rng(13)
    for m, n in ((257, 1), (1, 1031), (513, 259), (2049, 4097)):
        uvw = W.uvw_disk(m, 300.0, 10.0, rng)
        xyz = W.fibonacci_cap(n, 4.0)
        sky = W.complex_normal(1, n, rng)
        vis = W.complex_normal(1, m, rng)
        for thr in (0.0, math.inf):
            es, ea, info = both_directions(uvw, xyz, sky, vis, 1e-9, "f64", direct_threshold=thr, max_fft_bytes=2e6)
            assert es <= 1e-9 and ea <= 1e-9, (m, n, thr, es, ea)


def _clustered_inputs(rng):
    """A 2,000-baseline disk plus 3,000 visibilities within 1e-3 wavelengths of
    one uvw point, and a 2,000-point cap plus 6,000 sky points within 1e-7 of
    one direction: each cluster lies inside one kernel footprint, so the grid
    tiles it touches hold thousands of points in either direction."""
    uvw = np.concatenate([W.uvw_disk(2000, 600.0, 20.0, rng),
                          np.array([123.4, -77.7, 5.0]) + 1e-3 * rng.standard_normal((3000, 3))])
    c = np.array([0.03, -0.02, 1.0])
    c /= np.linalg.norm(c)
    cl = c + 1e-7 * rng.standard_normal((6000, 3))
    cl /= np.linalg.norm(cl, axis=1, keepdims=True)
    xyz = np.concatenate([W.fibonacci_cap(2000, 6.0), cl])
    return uvw, xyz, W.complex_normal(1, xyz.shape[0], rng), W.complex_normal(1, uvw.shape[0], rng)


@pytest.mark.parametrize("dtype,eps", [("f32", 1e-4), ("f64", 1e-9)])
@pytest.mark.parametrize("budget", [math.inf, 16e6])
def test_crowded_tiles(dtype, eps, budget):
    """Tiles holding far more sources than one spreading workgroup takes (256)
    are split into parts, the further parts added atomically by a second
    launch; the result still meets eps in both directions."""
    uvw, xyz, sky, vis = _clustered_inputs(np.random.default_rng(29))
    es, ea, info = both_directions(uvw, xyz, sky, vis, eps, dtype, direct_threshold=0.0, max_fft_bytes=budget)
    _report(f"crowded {dtype} {eps:g} B={budget:g}", es, ea, info)
    assert info["n_pairs_direct"] == 0
    assert es <= eps and ea <= eps


# ---- full-size SKA-like workload (995k x 1M), sampled rows -------------------------------
@pytest.mark.slow
@pytest.mark.timeout(600)
@pytest.mark.parametrize("dtype,eps", [("f32", 1e-4), ("f64", 1e-9)])
def test_ska_like_full_size_sampled(dtype, eps):
    wl = W.ska_like()
    rv = W.sample_rows(wl.n_vis, 4096, seed=21)
    rp = W.sample_rows(wl.n_pix, 4096, seed=22)
    es, ea, info = both_directions(wl.uvw, wl.xyz, wl.sky, wl.vis, eps, dtype, rows_vis=rv, rows_pix=rp)
    _report(f"ska-like full {dtype} {eps:g}", es, ea, info)
    assert es <= eps and ea <= eps


# ---- full-size LOFAR-like workload (5.0M x 4M, wide field), sampled rows -----------------
@pytest.fixture(scope="module")
def lofar_like():
    return W.lofar_like()


@pytest.mark.slow
@pytest.mark.timeout(600)
@pytest.mark.parametrize("dtype,eps", [("f32", 1e-4), ("f64", 1e-9)])
def test_lofar_like_full_size_sampled(lofar_like, dtype, eps):
    wl = lofar_like
    rv = W.sample_rows(wl.n_vis, 4096, seed=31)
    rp = W.sample_rows(wl.n_pix, 4096, seed=32)
    es, ea, info = both_directions(wl.uvw, wl.xyz, wl.sky, wl.vis, eps, dtype, rows_vis=rv, rows_pix=rp)
    _report(f"lofar-like full {dtype} {eps:g}", es, ea, info)
    assert info["n_vis_chunks"] > 1 and info["n_sky_chunks"] > 1   # chunked evaluation
    assert es <= eps and ea <= eps


# ---- dense DCOS meshes of the paper's telescope-radius ladder, sampled rows -------------
# (the regime where most of the terms go through NUFFT sub-problems)
@pytest.mark.parametrize("dtype,eps", [("f32", 1e-4), ("f64", 1e-9)])
@pytest.mark.parametrize("radius_km", [3.0, pytest.param(10.0, marks=pytest.mark.slow)])
def test_dense_dcos_ladder_sampled(radius_km, dtype, eps):
    wl = W.dense_dcos(radius_km)
    rv = W.sample_rows(wl.n_vis, 256, seed=41)
    rp = W.sample_rows(wl.n_pix, 256, seed=42)
    es, ea, info = both_directions(wl.uvw, wl.xyz, wl.sky, wl.vis, eps, dtype, rows_vis=rv, rows_pix=rp)
    _report(f"dense {radius_km:g} km {dtype} {eps:g}", es, ea, info)
    assert info["n_pairs_nufft"] > 0          # NUFFT sub-problems take part
    assert es <= eps and ea <= eps


def test_dense_dcos_forced_nufft_sampled():
    """Every sub-problem of the 1 km rung as a NUFFT (float32, eps 1e-4)."""
    wl = W.dense_dcos(1.0)
    rv = W.sample_rows(wl.n_vis, 256, seed=43)
    rp = W.sample_rows(wl.n_pix, 256, seed=44)
    es, ea, info = both_directions(wl.uvw, wl.xyz, wl.sky, wl.vis, 1e-4, "f32", rows_vis=rv, rows_pix=rp,
                                   direct_threshold=0.0)
    _report("dense 1 km forced nufft f32", es, ea, info)
    assert info["n_pairs_direct"] == 0
    assert es <= 1e-4 and ea <= 1e-4



# ---- sparse skies of the paper's sparse-mesh experiment: 500 pixels in five patches -------
@pytest.mark.parametrize("dtype,eps", [("f32", 1e-4), ("f64", 1e-9)])
@pytest.mark.parametrize("radius_km,thr", [(3.0, -1.0), (100.0, -1.0), (100.0, 0.0)])
def test_sparse_dcos_sky(radius_km, thr, dtype, eps):
    """Analysis and synthesis on a 500-pixel sparse sky (five 10 x 10 patches of
    the rung's DCOS grid) against the oracle on every output (all 500 pixels,
    every visibility), with the automatic choice and with every sub-problem a
    NUFFT."""
    wl = W.sparse_dcos(radius_km)
    es, ea, info = both_directions(wl.uvw, wl.xyz, wl.sky, wl.vis, eps, dtype, direct_threshold=thr)
    _report(f"sparse {radius_km:g} km thr={thr:g} {dtype} {eps:g}", es, ea, info)
    if thr == 0.0:
        assert info["n_pairs_direct"] == 0
    assert es <= eps and ea <= eps


@pytest.mark.slow
@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype,eps", [("f32", 1e-4), ("f64", 1e-9)])
def test_dense_dcos_30km_sampled(dtype, eps):
    """The 30 km rung of the paper's ladder: 340,578 vis x 74,649,600 pix."""
    wl = W.dense_dcos(30.0)
    rv = W.sample_rows(wl.n_vis, 256, seed=45)
    rp = W.sample_rows(wl.n_pix, 1024, seed=46)
    es, ea, info = both_directions(wl.uvw, wl.xyz, wl.sky, wl.vis, eps, dtype, rows_vis=rv, rows_pix=rp)
    _report(f"dense 30 km {dtype} {eps:g}", es, ea, info)
    assert info["n_pairs_nufft"] > 0
    assert es <= eps and ea <= eps


def test_zz_element_wise_summary():
    """Print the element-wise errors of every case above (largest first)."""
    for tag, es, ea, ms, ma in sorted(ELEM_LOG, key=lambda r: -max(r[3] / max(r[1], 1e-300),
                                                                    r[4] / max(r[2], 1e-300)))[:20]:
        print(f"[elem] {tag}: l2 {es:.2e}/{ea:.2e} max {ms:.2e}/{ma:.2e} "
              f"ratio {ms / max(es, 1e-300):.2f}/{ma / max(ea, 1e-300):.2f}", flush=True)
