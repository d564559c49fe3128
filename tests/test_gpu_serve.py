"""Continuous batching on the GPU: requests of uneven size arriving while
others run are admitted onto free streams; every result must equal the same
request run alone (within 1e-6 relative: only the order of float64 atomic
additions can differ) and the oracle on sampled rows (within eps)."""
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


def test_mix_equals_alone_and_oracle():
    layouts = {"ska": W.ska_like_uvw(n_ant=60, n_times=12),
               "lofar": W.lofar_like_uvw(target_vis=60000)}
    reqs = W.serving_requests(seed=4, n_req=12, mean_gap_s=0.003, log10_min=3.0, log10_max=4.3, layouts=layouts)
    ex = serve.GpuExecutor(eps=1e-4, dtype="f32", slots=4, planners=4, workspace_bytes=256e6)
    srv = serve.Server(ex, hbm_budget_bytes=8e9)
    mixed = srv.run(reqs)
    ex.close()
    assert max(n for _, _, n, _ in srv.log) >= 2          # requests overlapped on the device
    alone_ex = serve.GpuExecutor(eps=1e-4, dtype="f32", slots=1, planners=1, workspace_bytes=256e6)
    for q, r in zip(reqs, mixed):
        h = alone_ex.submit(q, 0)
        a = alone_ex.finish(h)
        assert oracle.rel_l2(r.output, a) <= 1e-6, q.rid
        n_out = q.uvw.shape[0] if q.direction == "synthesis" else q.xyz.shape[0]
        rows = W.sample_rows(n_out, 64, seed=q.rid)
        ref = (oracle.synthesis(q.uvw, q.xyz, q.data, rows=rows) if q.direction == "synthesis"
               else oracle.analysis(q.uvw, q.xyz, q.data, rows=rows))
        assert oracle.rel_l2(r.output[:, rows], ref) <= 1e-4, q.rid
    alone_ex.close()
    s = serve.summarize(mixed)
    print("serving:", s, flush=True)
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0
