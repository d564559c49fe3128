"""The allocation-free entry point hvox_transform_noalloc (include/hvox.h),
called through the C ABI: its output equals hvox_synthesis / hvox_analysis
on the same plan (deterministic plans: bit for bit; both within eps of the
oracle), over two calls in a row on one GPU, the second with a smaller
input, so the shared static scratch starts with the first call's contents.
A plan needing more scratch than the buffer holds is refused."""
import ctypes

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


def _noalloc(plan, direction, x):
    import torch
    lib = hv.load_library()
    n_out = plan.n_vis if direction == 0 else plan.n_pix
    out = torch.empty((x.shape[0], n_out), dtype=plan.complex_dtype, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    rc = lib.hvox_transform_noalloc(plan._plan, direction, ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(out.data_ptr()), x.shape[0], ctypes.c_void_p(st))
    return rc, out


def _t(a, cd):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", cd)


@pytest.mark.parametrize("dtype,eps", [("f32", 1e-4), ("f64", 1e-9)])
@pytest.mark.parametrize("hint", [1, 2])
def test_noalloc_matches_the_allocating_entry_point(dtype, eps, hint):
    import torch
    cd = torch.complex64 if dtype == "f32" else torch.complex128
    big = W.compact_disk(ntrans=2)                       # 2,000 vis x 3,072 pix, two rows
    small = W.compact_disk(n_vis=700, n_pix=900)          # the second call: a smaller input
    nufft = dict(max_fft_bytes=16e6, workspace_bytes=40e6, direct_threshold=0.0)   # ~38 MB of scratch
    direct = dict(max_fft_bytes=16e6, workspace_bytes=40e6, direct_threshold=1.0)
    for wl, kw in ((big, nufft), (small, nufft), (big, direct), (small, direct)):
        with hv.Plan(wl.uvw, wl.xyz, eps, dtype, deterministic=True, ntrans_hint=hint, **kw) as p:
            assert p.info()["noalloc_scratch_bytes"] <= (64 << 20)   # two-row plans: passes of two rows
            sky, vis = _t(wl.sky, cd), _t(wl.vis, cd)
            rc_s, Vs = _noalloc(p, 0, sky)
            rc_a, Is = _noalloc(p, 1, vis)
            assert rc_s == 0 and rc_a == 0, hv.load_library().hvox_last_error()
            V = p.synthesis(sky)
            I = p.analysis(vis)
            torch.cuda.synchronize()
            info = p.info()
        assert torch.equal(Vs, V) and torch.equal(Is, I), wl.name
        Vn, In = Vs.cpu().numpy(), Is.cpu().numpy()
        assert oracle.rel_l2(Vn, oracle.synthesis(wl.uvw, wl.xyz, wl.sky)) <= eps
        assert oracle.rel_l2(In, oracle.analysis(wl.uvw, wl.xyz, wl.vis)) <= eps
        print(f"[noalloc {dtype} hint={hint}] {wl.name}: nufft={info['n_pairs_nufft']} direct={info['n_pairs_direct']} "
              f"workspace={info['workspace_bytes']}", flush=True)


def test_noalloc_refuses_plans_beyond_the_buffer():
    import torch
    wl = W.compact_disk()
    with hv.Plan(wl.uvw, wl.xyz, 1e-9, "f64", direct_threshold=0.0, max_fft_bytes=float("inf")) as p:
        assert p.info()["workspace_bytes"] > (64 << 20)
        rc, _ = _noalloc(p, 0, _t(wl.sky, torch.complex128))
        assert rc == -3
        assert b"static buffer" in hv.load_library().hvox_last_error()
