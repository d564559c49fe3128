"""Admission and accounting of the continuous-batching server, on the CPU with
the fake executor (a modelled run time per request and oracle results)."""
import numpy as np

import oracle
from paper_2306_06007_amd import serve
from paper_2306_06007_amd import workloads as W


def _requests(n=10, seed=0, gap=0.002):
    rng = np.random.default_rng(seed)
    reqs, t = [], 0.0
    for rid in range(n):
        t += rng.exponential(gap)
        nv = int(rng.integers(20, 120))
        npx = int(rng.integers(20, 120))
        uvw = W.uvw_disk(nv, 200.0, 10.0, rng)
        xyz = W.fibonacci_cap(npx, 5.0)
        direction = "synthesis" if rid % 2 == 0 else "analysis"
        data = W.real_intensities(1, npx, rng) if direction == "synthesis" else W.complex_normal(1, nv, rng)
        reqs.append(W.Request(rid, t, direction, "disk", uvw, xyz, data))
    return reqs


def _oracle(req):
    if req.direction == "synthesis":
        return oracle.synthesis(req.uvw, req.xyz, req.data)
    return oracle.analysis(req.uvw, req.xyz, req.data)


def test_server_completes_and_overlaps():
    reqs = _requests()
    ex = serve.FakeExecutor(slots=3, seconds_per_term=2e-6, compute=_oracle)
    srv = serve.Server(ex, hbm_budget_bytes=1e12)
    res = srv.run(reqs)
    ex.close()
    assert [r.rid for r in res] == [q.rid for q in reqs]
    for r, q in zip(res, reqs):
        assert r.admit_s >= q.arrival_s - 1e-3 and r.done_s >= r.admit_s and r.latency_s > 0
        assert np.array_equal(r.output, _oracle(q))
    assert ex.max_concurrent >= 2                      # requests overlapped
    assert max(n for _, _, n, _ in srv.log) <= 3       # never more than the slots
    s = serve.summarize(res)
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_server_respects_memory_budget_and_fifo():
    reqs = _requests(n=8, seed=1, gap=0.0005)
    ex = serve.FakeExecutor(slots=4, seconds_per_term=1e-6, footprint_per_point=1.0)
    budget = max(q.uvw.shape[0] + q.xyz.shape[0] for q in reqs) * 1.5
    srv = serve.Server(ex, hbm_budget_bytes=budget)
    srv.run(reqs, keep_outputs=False)
    ex.close()
    # the admitted footprint never exceeds the budget (a single request always fits)
    assert all(used <= budget or n == 1 for _, _, n, used in srv.log)
    # first-come first-served admission
    order = [rid for _, rid, _, _ in srv.log]
    arrival_order = [q.rid for q in sorted(reqs, key=lambda q: q.arrival_s)]
    assert order == arrival_order
