"""GPU checks of the boundary options of the C ABI (include/hvox.h):
deterministic plans (bit-identical results across calls and across plans),
data in chunk order (HVOX_PREORDERED), device-memory hooks (the caller's
allocator owns every block; a failing allocator gives HVOX_ERR_OOM and every
block obtained is handed back), and host planning followed by
hvox_plan_upload.  Every result is also held to the oracle at eps."""
import ctypes
import math

import numpy as np
import pytest

import oracle
import paper_2306_06007_amd as hv
from paper_2306_06007_amd import hvox as H
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


def _crowded():
    """A small SKA-like layout plus a cluster of sky points inside one kernel
    footprint (crowded spreading tiles) and a forced-NUFFT / direct mix."""
    rng = np.random.default_rng(17)
    wl = W.ska_like(n_pix=12000, n_ant=40, n_times=8)
    c = wl.xyz[100] + 1e-7 * rng.standard_normal((3000, 3))
    xyz = np.concatenate([wl.xyz, c / np.linalg.norm(c, axis=1, keepdims=True)])
    sky = W.complex_normal(1, xyz.shape[0], rng)
    return wl.uvw, xyz, sky, wl.vis


@pytest.mark.parametrize("dtype,eps", [("f32", 1e-4), ("f64", 1e-9)])
@pytest.mark.parametrize("thr", [0.0, -1.0])
def test_deterministic_plans_are_bit_reproducible(dtype, eps, thr):
    uvw, xyz, sky, vis = _crowded()
    outs = []
    for rep in range(2):                   # two plans built independently
        with hv.Plan(uvw, xyz, eps, dtype, deterministic=True, direct_threshold=thr, max_fft_bytes=4e6) as p:
            V1 = _np(p.synthesis(_t(sky, dtype)))
            I1 = _np(p.analysis(_t(vis, dtype)))
            V2 = _np(p.synthesis(_t(sky, dtype)))
            I2 = _np(p.analysis(_t(vis, dtype)))
            info = p.info()
        assert np.array_equal(V1, V2) and np.array_equal(I1, I2)
        outs.append((V1, I1))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    print(f"[deterministic {dtype} thr={thr}] nufft={info['n_pairs_nufft']} direct={info['n_pairs_direct']} "
          f"layers={info['n_direct_layers']} batches={info['n_batches']}", flush=True)
    Vref = oracle.synthesis(uvw, xyz, sky)
    Iref = oracle.analysis(uvw, xyz, vis)
    assert oracle.rel_l2(outs[0][0], Vref) <= eps and oracle.rel_l2(outs[0][1], Iref) <= eps


def test_preordered_data_skips_the_permutations():
    wl = W.ska_like(n_pix=15000, n_ant=40, n_times=8)
    for dtype, eps in (("f32", 1e-4), ("f64", 1e-9)):
        with hv.Plan(wl.uvw, wl.xyz, eps, dtype, max_fft_bytes=8e6, deterministic=True) as p:
            V = _np(p.synthesis(_t(wl.sky, dtype)))
            I = _np(p.analysis(_t(wl.vis, dtype)))
            vp, sp = p.permutation()
        with hv.Plan(wl.uvw, wl.xyz, eps, dtype, max_fft_bytes=8e6, deterministic=True, preordered=True) as q:
            Vq = _np(q.synthesis(_t(wl.sky[:, sp], dtype)))     # input in chunk order, output in chunk order
            Iq = _np(q.analysis(_t(wl.vis[:, vp], dtype)))
        assert np.array_equal(Vq, V[:, vp]) and np.array_equal(Iq, I[:, sp])


def test_preordered_row_passes():
    """Pre-ordered data through NUFFT passes of three rows (a plan made for four rows
    per call): bit-identical to the permuted path of the same plan options."""
    wl = W.ska_like(n_pix=15000, n_ant=40, n_times=8, ntrans=3)
    kw = dict(max_fft_bytes=8e6, deterministic=True, direct_threshold=0.0, ntrans_hint=4)
    for dtype in ("f32", "f64"):
        eps = 1e-4 if dtype == "f32" else 1e-9
        with hv.Plan(wl.uvw, wl.xyz, eps, dtype, **kw) as p:
            assert p.info()["nufft_rows"] == 4
            V = _np(p.synthesis(_t(wl.sky, dtype)))
            I = _np(p.analysis(_t(wl.vis, dtype)))
            vp, sp = p.permutation()
        with hv.Plan(wl.uvw, wl.xyz, eps, dtype, preordered=True, **kw) as q:
            Vq = _np(q.synthesis(_t(wl.sky[:, sp], dtype)))
            Iq = _np(q.analysis(_t(wl.vis[:, vp], dtype)))
        assert np.array_equal(Vq, V[:, vp]) and np.array_equal(Iq, I[:, sp])


@pytest.mark.parametrize("dtype,eps", [("f32", 1e-4), ("f64", 1e-9)])
def test_deterministic_row_passes_on_crowded_tiles(dtype, eps):
    """Crowded spreading tiles (walked whole in deterministic plans) through
    passes of two rows: each row bit-identical to the plan made for one row per
    call, and within eps of the oracle."""
    uvw, xyz, sky, vis = _crowded()
    rng = np.random.default_rng(19)
    sky2 = np.concatenate([sky, W.complex_normal(1, xyz.shape[0], rng)])
    vis2 = np.concatenate([vis, W.complex_normal(1, uvw.shape[0], rng)])
    outs = {}
    for hint in (1, 2):
        with hv.Plan(uvw, xyz, eps, dtype, deterministic=True, direct_threshold=0.0, max_fft_bytes=4e6,
                     ntrans_hint=hint) as p:
            assert p.info()["nufft_rows"] == hint
            outs[hint] = (_np(p.synthesis(_t(sky2, dtype))), _np(p.analysis(_t(vis2, dtype))))
    assert np.array_equal(outs[1][0], outs[2][0]) and np.array_equal(outs[1][1], outs[2][1])
    assert oracle.rel_l2(outs[2][0], oracle.synthesis(uvw, xyz, sky2)) <= eps
    assert oracle.rel_l2(outs[2][1], oracle.analysis(uvw, xyz, vis2)) <= eps


class CountingAllocator:
    """dev_alloc / dev_free hooks over PyTorch's caching allocator that count
    the blocks and can be told to fail after a number of bytes."""

    def __init__(self, fail_after=None):
        self.live = {}
        self.n_alloc = self.n_free = 0
        self.total = 0
        self.fail_after = fail_after
        self.hooks = (H.ALLOC_FN(self._alloc), H.FREE_FN(self._free), None)

    def _alloc(self, nbytes, ctx, stream):
        import torch
        if self.fail_after is not None and self.total + nbytes > self.fail_after:
            return None
        p = int(torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), int(stream or 0) or None))
        self.live[p] = nbytes
        self.n_alloc += 1
        self.total += nbytes
        return p

    def _free(self, ptr, nbytes, ctx, stream):
        import torch
        assert self.live.pop(int(ptr)) == nbytes
        self.n_free += 1
        torch.cuda.caching_allocator_delete(int(ptr))


def test_allocator_hooks_own_every_block():
    wl = W.ska_like(n_pix=15000, n_ant=40, n_times=8)
    al = CountingAllocator()
    p = hv.Plan(wl.uvw, wl.xyz, 1e-4, "f32", max_fft_bytes=4e6, direct_threshold=0.0, alloc_hooks=al.hooks)
    V = _np(p.synthesis(_t(wl.sky, "f32")))
    info = p.info()
    assert al.n_alloc > 10 and sum(al.live.values()) == info["device_bytes"]
    p.free()
    assert not al.live and al.n_free == al.n_alloc
    assert oracle.rel_l2(V, oracle.synthesis(wl.uvw, wl.xyz, wl.sky)) <= 1e-4
    # the library's own hipMalloc path gives the same result
    with hv.Plan(wl.uvw, wl.xyz, 1e-4, "f32", max_fft_bytes=4e6, direct_threshold=0.0, allocator=None) as q:
        assert oracle.rel_l2(_np(q.synthesis(_t(wl.sky, "f32"))), V) <= 1e-6


@pytest.mark.parametrize("frac", [0.05, 0.5, 0.95])
def test_failing_allocator_gives_oom_and_leaks_nothing(frac):
    wl = W.ska_like(n_pix=15000, n_ant=40, n_times=8)
    with hv.Plan(wl.uvw, wl.xyz, 1e-4, "f32", max_fft_bytes=4e6, direct_threshold=0.0, host_only=True) as h:
        need = h.info()["device_bytes"]
    al = CountingAllocator(fail_after=int(frac * need))
    with pytest.raises(hv.HvoxError) as ei:
        hv.Plan(wl.uvw, wl.xyz, 1e-4, "f32", max_fft_bytes=4e6, direct_threshold=0.0, alloc_hooks=al.hooks)
    assert ei.value.code == -3
    assert not al.live and al.n_free == al.n_alloc


def test_host_plan_then_upload_matches_a_direct_plan():
    wl = W.ska_like(n_pix=15000, n_ant=40, n_times=8)
    h = hv.Plan(wl.uvw, wl.xyz, 1e-4, "f32", max_fft_bytes=8e6, host_only=True, deterministic=True)
    bound = h.info()["device_bytes"]
    h.upload()
    info = h.info()
    assert info["on_device"] == 1 and 0 < info["device_bytes"] <= bound
    V = _np(h.synthesis(_t(wl.sky, "f32")))
    with pytest.raises(hv.HvoxError):
        h.upload()
    h.free()
    with hv.Plan(wl.uvw, wl.xyz, 1e-4, "f32", max_fft_bytes=8e6, deterministic=True) as p:
        assert np.array_equal(_np(p.synthesis(_t(wl.sky, "f32"))), V)
