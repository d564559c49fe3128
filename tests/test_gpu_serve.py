"""Continuous batching on the GPU: requests of uneven size arriving while
others run are planned on the host, admitted by their plans' device bytes onto
free streams, and overlap on the device.  With deterministic plans every
result must be bit-identical to the same request run alone, and within eps of
the oracle on sampled rows; requests sharing one geometry (and so one cached
plan and its workspace) must not disturb each other."""
import numpy as np
import pytest

import oracle
from paper_2306_06007_amd import serve
from paper_2306_06007_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _alone(req, eps=1e-4):
    ex = serve.GpuExecutor(eps=eps, dtype="f32", slots=1, planners=1, workspace_bytes=256e6, deterministic=True)
    srv = serve.Server(ex, hbm_budget_bytes=8e9)
    out = srv.run([W.Request(req.rid, 0.0, req.direction, req.layout, req.uvw, req.xyz, req.data)])[0].output
    ex.close()
    return out


def _oracle_rows(q, k=64):
    n_out = q.uvw.shape[0] if q.direction == "synthesis" else q.xyz.shape[0]
    rows = W.sample_rows(n_out, k, seed=q.rid)
    ref = (oracle.synthesis(q.uvw, q.xyz, q.data, rows=rows) if q.direction == "synthesis"
           else oracle.analysis(q.uvw, q.xyz, q.data, rows=rows))
    return rows, ref


def test_mix_equals_alone_and_oracle():
    layouts = {"ska": W.ska_like_uvw(n_ant=60, n_times=12),
               "lofar": W.lofar_like_uvw(target_vis=60000)}
    reqs = W.serving_requests(seed=4, n_req=12, mean_gap_s=0.003, log10_min=3.0, log10_max=4.3, layouts=layouts)
    ex = serve.GpuExecutor(eps=1e-4, dtype="f32", slots=4, planners=4, workspace_bytes=256e6, deterministic=True)
    srv = serve.Server(ex, hbm_budget_bytes=8e9)
    mixed = srv.run(reqs)
    ex.close()
    assert max(n for _, _, n, _ in srv.log) >= 2          # requests overlapped on the device
    assert all(used <= 8e9 for _, _, _, used in srv.log)  # admitted within the HBM budget
    for q, r in zip(reqs, mixed):
        assert np.array_equal(r.output, _alone(q)), q.rid
        rows, ref = _oracle_rows(q)
        assert oracle.rel_l2(r.output[:, rows], ref) <= 1e-4, q.rid
        assert oracle.max_rel_err(r.output[:, rows], ref) <= 4e-4, q.rid
    s = serve.summarize(mixed)
    print("serving:", s, flush=True)
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_requests_sharing_a_plan_do_not_race():
    """Synthesis and analysis requests on one geometry arrive together: they
    share one cached plan (one workspace), so their calls are ordered on the
    device; each result equals the request run alone, bit for bit."""
    wl = W.ska_like(n_pix=30000, n_ant=50, n_times=10)
    rng = np.random.default_rng(8)
    reqs = []
    for rid in range(6):
        direction = "synthesis" if rid % 2 == 0 else "analysis"
        data = (W.complex_normal(1, wl.n_pix, rng) if direction == "synthesis"
                else W.complex_normal(1, wl.n_vis, rng))
        reqs.append(W.Request(rid, 0.001 * rid, direction, "ska", wl.uvw, wl.xyz, data))
    ex = serve.GpuExecutor(eps=1e-4, dtype="f32", slots=4, planners=2, workspace_bytes=256e6, deterministic=True)
    srv = serve.Server(ex, hbm_budget_bytes=8e9)
    mixed = srv.run(reqs)
    n_plans = len(ex.plan_seconds)
    ex.close()
    assert n_plans == 1                                   # one geometry, one plan
    assert max(n for _, _, n, _ in srv.log) >= 2          # admitted together
    for q, r in zip(reqs, mixed):
        assert np.array_equal(r.output, _alone(q)), q.rid
        rows, ref = _oracle_rows(q)
        assert oracle.rel_l2(r.output[:, rows], ref) <= 1e-4, q.rid


def test_admission_waits_for_memory():
    """With a budget that holds one plan at a time, requests on distinct
    geometries run one after another (idle plans are evicted to make room)."""
    layouts = {"ska": W.ska_like_uvw(n_ant=40, n_times=8), "lofar": W.lofar_like_uvw(target_vis=30000)}
    reqs = W.serving_requests(seed=6, n_req=5, mean_gap_s=0.001, log10_min=3.0, log10_max=3.8, layouts=layouts)
    ex = serve.GpuExecutor(eps=1e-4, dtype="f32", slots=4, planners=4, workspace_bytes=32e6, cache_size=0)
    budget = 1.0     # below any plan: every admission is forced, one at a time
    srv = serve.Server(ex, hbm_budget_bytes=budget)
    res = srv.run(reqs)
    ex.close()
    assert max(n for _, _, n, _ in srv.log) == 1
    for q, r in zip(reqs, res):
        rows, ref = _oracle_rows(q, 32)
        assert oracle.rel_l2(r.output[:, rows], ref) <= 1e-4
