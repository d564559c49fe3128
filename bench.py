"""Benchmark of the HVOX hot path on one MI355X.

One step = one synthesis (sky -> vis) plus one analysis (vis -> sky) of the
SKA-like workload: 995,000 visibilities from 200 Gaussian-placed antennas
(sigma 5 km) over 50 hour angles in [-2h, +2h] at declination -30 deg, one
channel at 1 m; a 1,000,000-point Fibonacci cap of half-angle 10 deg;
synthetic data (intensities U[0,1], visibilities CN(0,1)).  The plan
(partitioning, tables) is built once and kept resident; inputs are already
in HBM when the timed region starts.

Metric: (n_vis + n_pix) per second of synthesis + analysis, headline in
float32 at eps = 1e-4, with the float64 eps = 1e-9 plan timed beside it.
The roofline entry is the kernel that takes the most time in the float32
step, timed with HIP events on the stream it runs on.  The CPU baseline is
the FP64 oracle on a bounded sample of output rows, extrapolated linearly.

``--workload dense-10km`` reports the same line for the dense 30-degree DCOS
mesh of the 10 km telescope radius (238,203 vis x 10,240,000 pix) instead.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Vector peaks from the unit counts and clock: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz = 39.3 T lane-cycles/s; float32 issues two lane-operations per
# lane-cycle (157.3 TFLOP/s counting an FMA as 2 FLOP), float64 one (78.6).
LANE_CYCLES_PER_S = 256 * 4 * 16 * 2.4e9
VECTOR_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
METRIC = "(vis+pix)/s synth+analysis at eps=1e-4 FP32 vs 1e-9 FP64; p50/p99 latency"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the device-kernel sources (kernels and their constants): counter
    summaries taken on other kernel code are not reported."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "hvox_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2306_06007_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, dtype: str, mode: str = "auto"):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's
    readings) from the committed rocprofv3 counter summary of this kernel in
    this execution mode, if it was taken on the current kernel sources; else
    None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{dtype}_{mode}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def step(plan, sky, vis, vout, sout):
    """One pass of the hot path: synthesis then analysis, into preallocated outputs."""
    plan.synthesis(sky, out=vout)
    plan.analysis(vis, out=sout)


def time_steps(plan, bufs, steps, warmup):
    import torch
    for _ in range(warmup):
        step(plan, *bufs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(plan, *bufs)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def direction_times(plan, bufs, runs):
    """Device time of each direction: ``runs`` passes of synthesis then
    analysis, with HIP events recorded on the stream the calls are enqueued on
    between them; median, p10 and p90 of synthesis, analysis and their sum."""
    import numpy as np
    import torch
    sky, vis, vout, sout = bufs
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(runs)]
    torch.cuda.synchronize()
    for e0, e1, e2 in ev:
        e0.record()
        plan.synthesis(sky, out=vout)
        e1.record()
        plan.analysis(vis, out=sout)
        e2.record()
    torch.cuda.synchronize()
    out = {"runs": runs}
    for key, pick in (("synthesis_ms", lambda e: e[0].elapsed_time(e[1])),
                      ("analysis_ms", lambda e: e[1].elapsed_time(e[2])),
                      ("step_ms", lambda e: e[0].elapsed_time(e[2]))):
        t = np.array([pick(e) for e in ev])
        out[key] = {"median": float(np.median(t)), "p10": float(np.percentile(t, 10)),
                    "p90": float(np.percentile(t, 90))}
    return out


def kernel_table(plan, bufs):
    """One step with per-launch HIP events recorded on the stream the kernels
    run on; per-kernel totals."""
    import torch
    plan.reset_stats()
    plan.set_timing(True)
    step(plan, *bufs)
    torch.cuda.synchronize()
    st = plan.stats()
    plan.set_timing(False)
    return st


HBM_KERNELS = ("zero", "spread", "fft_x", "fft_y", "fft_z", "interp", "finalize", "transpose", "prephase")


def roofline_entry(st, dtype, name=None, rows=1, mode="auto"):
    """Roofline of one kernel (default: the one taking the most time): its
    algorithmic bytes (or arithmetic) per launch over its average launch
    duration, against the MI355X peak."""
    hbm_kernels = HBM_KERNELS
    if name is None:
        name = max(st, key=lambda k: st[k]["ms"])
    v = st[name]
    n = max(1, v["launches"])
    avg_s = v["ms"] * 1e-3 / n
    if name in hbm_kernels:
        per_launch = v["alg_bytes"] / n
        achieved = per_launch / avg_s / 1e9 if avg_s > 0 else 0.0
        traffic = measured_traffic(name, dtype, mode)
        return name, {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": achieved / HBM_PEAK_GBS, "traffic": traffic}
    # direct summation: bound by the vector ALUs.  Algorithmic arithmetic per
    # term-row: ALG_OPS_PER_TERM operations (the phase dot product, its
    # reduction, sine and cosine, and the complex multiply-accumulate) against
    # the published vector peak; issue_bound compares the term rate with what
    # the loop's own instruction mix allows at the per-class issue rates.
    terms_per_s = v["alg_flops"] / n / avg_s if avg_s > 0 else 0.0
    achieved = terms_per_s * ALG_OPS_PER_TERM / 1e12
    peak = VECTOR_PEAK_TFLOPS[dtype]
    bound = LANE_CYCLES_PER_S / VALU_CYCLES_PER_TERM[(dtype, rows)]
    return name, {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                  "frac": achieved / peak, "traffic": measured_traffic(name, dtype, mode),
                  "ops_per_term": ALG_OPS_PER_TERM,
                  "issue_bound": {"term_rows_per_s": bound, "achieved_term_rows_per_s": terms_per_s,
                                  "frac": terms_per_s / bound,
                                  "valu_instr_per_term_row": VALU_OPS_PER_TERM[(dtype, rows)]}}


# Algorithmic operations of one direct-sum term (target k, source n), the count
# the roofline is graded on: the phase p_k.r_n (3 multiply-adds, 6), its
# reduction to a fraction of a turn (2), its sine and cosine (about 14) and the
# complex multiply-accumulate (8): about 30 operations per term.
ALG_OPS_PER_TERM = 30.0
# VALU instructions issued per (target, source, data row) by the direct
# kernel's inner loop, counted from its gfx950 assembly (the loop that reads
# the staged sources from LDS; LDS reads and scalar loop control excluded), by
# plan precision and rows per launch.  Per iteration of 4 sources x 2 targets:
# the float64 dot product and reduction to a fraction of a turn (shared by the
# rows), float32: conversion and hardware sine and cosine (shared), float64:
# the 1024-entry phase table's index and remainder, the remainder's Taylor
# sine and cosine and the rotation by the table entry (shared), then one
# complex multiply-accumulate per row.  Each is one lane-operation per lane.
VALU_OPS_PER_TERM = {("f32", 1): 89 / 8, ("f32", 2): 121 / 16, ("f32", 3): 153 / 24, ("f32", 4): 185 / 32,
                     ("f64", 1): 178 / 8, ("f64", 2): 210 / 16, ("f64", 3): 242 / 24, ("f64", 4): 274 / 32}
# Lane-cycles per term-row of the same loops at the per-class issue rates
# (float32 arithmetic 1/2 cycle, hardware sine / cosine 2, the rest 1): float32
# 32 / 64 / 96 / 128 float32 + 16 transcendental + 41 other per 8 / 16 / 24 / 32
# term-rows; float64 has no float32 or transcendental instructions.
VALU_CYCLES_PER_TERM = {("f32", 1): 89 / 8, ("f32", 2): 105 / 16, ("f32", 3): 121 / 24, ("f32", 4): 137 / 32,
                        ("f64", 1): 178 / 8, ("f64", 2): 210 / 16, ("f64", 3): 242 / 24, ("f64", 4): 274 / 32}


def host_cpu_model() -> str:
    """The host processor's model name (Linux /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, target_s=20.0):
    """FP64 oracle on sampled rows of both directions, extrapolated linearly
    (the direct sum's cost is exactly linear in the number of output rows).
    About target_s seconds of CPU work: a warm 64-row probe sizes the sample
    (at most 4,096 rows per direction)."""
    import oracle
    from paper_2306_06007_amd import workloads as W
    oracle.synthesis(wl.uvw, wl.xyz, wl.sky, rows=W.sample_rows(wl.n_vis, 8, seed=100))   # thread pool warm-up
    probe = 64
    rv = W.sample_rows(wl.n_vis, probe, seed=101)
    t0 = time.perf_counter()
    oracle.synthesis(wl.uvw, wl.xyz, wl.sky, rows=rv)
    per_row_v = (time.perf_counter() - t0) / probe
    k = int(max(64, min(4096, 0.5 * target_s / max(per_row_v, 1e-9))))
    rv = W.sample_rows(wl.n_vis, k, seed=102)
    rp = W.sample_rows(wl.n_pix, k, seed=103)
    t0 = time.perf_counter()
    Vs = oracle.synthesis(wl.uvw, wl.xyz, wl.sky, rows=rv)
    t_v = time.perf_counter() - t0
    t0 = time.perf_counter()
    Is = oracle.analysis(wl.uvw, wl.xyz, wl.vis, rows=rp)
    t_p = time.perf_counter() - t0
    t_full = t_v * wl.n_vis / k + t_p * wl.n_pix / k
    value = (wl.n_vis + wl.n_pix) / t_full
    info = {"value": value, "unit": "(vis+pix)/s", "cores": oracle.max_threads(), "kind": "oracle",
            "host_cpu": host_cpu_model(), "host_cpu_count": os.cpu_count(),
            "sample": f"{k} sampled visibility rows ({t_v:.1f}s) and {k} sampled pixel rows ({t_p:.1f}s) "
                      f"of the full sums, extrapolated linearly to {wl.n_vis}+{wl.n_pix} rows"}
    return info, (rv, Vs), (rp, Is)


def serving_run(slots=8, planners=8):
    """64 Poisson-arriving requests (mean gap 10 ms), each a synthesis or an
    analysis with log-uniform 1e4..1e6 visibilities and pixels on subsampled
    SKA-like / LOFAR-like baselines, float32 at eps = 1e-4, through the
    continuous-batching server; latency from arrival to observed completion.
    Afterwards every request runs again alone (one slot, nothing else on the
    device) and its result is compared with the one served in the mix."""
    import numpy as np
    from paper_2306_06007_amd import serve
    from paper_2306_06007_amd import workloads as W
    reqs = W.serving_requests(seed=4)
    log(f"serving: {len(reqs)} requests generated")
    ex = serve.GpuExecutor(eps=1e-4, dtype="f32", slots=slots, planners=planners, workspace_bytes=1 << 30)
    srv = serve.Server(ex, hbm_budget_bytes=64e9)
    res = srv.run(reqs, keep_outputs=True)
    ex.close()
    s = serve.summarize(res)
    s["max_in_flight"] = max(n for _, _, n, _ in srv.log)
    s["max_resident_bytes"] = max(u for _, _, _, u in srv.log)
    s["slots"], s["planners"] = slots, planners
    s["plan_seconds_mean"] = float(sum(ex.plan_seconds) / max(1, len(ex.plan_seconds)))
    s["plan_seconds_total"] = float(sum(ex.plan_seconds))
    s["upload_seconds_mean"] = float(sum(ex.upload_seconds) / max(1, len(ex.upload_seconds)))
    # alone vs in the mix
    alone = serve.GpuExecutor(eps=1e-4, dtype="f32", slots=1, planners=1, workspace_bytes=1 << 30, cache_size=0)
    diffs = []
    for q, r in zip(reqs, res):
        one = serve.Server(alone, hbm_budget_bytes=64e9).run(
            [W.Request(q.rid, 0.0, q.direction, q.layout, q.uvw, q.xyz, q.data)])[0].output
        d = float(np.max(np.abs(r.output - one)) / max(float(np.max(np.abs(one))), 1e-300))
        diffs.append(d)
    alone.close()
    s["alone_vs_mix_max_rel_diff"] = {"max": max(diffs), "median": float(np.median(diffs))}
    log(f"serving: p50 {s['p50_latency_s']:.3f} s, p99 {s['p99_latency_s']:.3f} s; alone vs mix max rel diff "
        f"{max(diffs):.2e}")
    return s, reqs, res


def serving_errors(reqs, res, rows=1024):
    """Error of every served result against the oracle on `rows` sampled outputs
    (part of the CPU-baseline leg: the only place bench.py runs the oracle)."""
    import numpy as np
    import oracle
    from paper_2306_06007_amd import workloads as W
    errs = []
    for q, r in zip(reqs, res):
        n_out = q.uvw.shape[0] if q.direction == "synthesis" else q.xyz.shape[0]
        rw = W.sample_rows(n_out, rows, seed=1000 + q.rid)
        ref = (oracle.synthesis(q.uvw, q.xyz, q.data, rows=rw) if q.direction == "synthesis"
               else oracle.analysis(q.uvw, q.xyz, q.data, rows=rw))
        errs.append({"rid": q.rid, "direction": q.direction, "n_vis": int(q.uvw.shape[0]),
                     "n_pix": int(q.xyz.shape[0]), "rel_l2": oracle.rel_l2(r.output[:, rw], ref),
                     "max_rel_err": oracle.max_rel_err(r.output[:, rw], ref)})
    l2 = [e["rel_l2"] for e in errs]
    mx = [e["max_rel_err"] for e in errs]
    return {"rows_per_request": rows, "rel_l2_max": max(l2), "rel_l2_median": float(np.median(l2)),
            "max_rel_err_max": max(mx), "all_within_eps": bool(max(l2) <= 1e-4), "per_request": errs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--f64-steps", type=int, default=0, help="timed float64 steps (default: max(1, steps // 5))")
    ap.add_argument("--direct-threshold", type=float, default=-1.0,
                    help="per-sub-problem NUFFT/direct choice: <0 automatic (default), 0 forced NUFFT, inf all direct")
    ap.add_argument("--serving", action="store_true",
                    help="run the 64-request serving workload (p50/p99); the default unless --no-modes")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving workload")
    ap.add_argument("--skip-f64", action="store_true", help="time the float32 plan only")
    ap.add_argument("--n-pix", type=int, default=1000000,
                    help="sky points of the SKA-like workload (default the full 1,000,000-point cap; smaller "
                         "values only for counter runs, never for the reported metric)")
    ap.add_argument("--modes", default="",
                    help="comma-separated subset of the runs reported beside the headline (forced_nufft, all_direct, "
                         "batched_ntrans4, forced_nufft_ntrans4, dense_10km, dense_10km_all_direct, dense_30km, "
                         "sparse_100km, sparse_100km_forced_nufft, compact_f64, compact_f32, lofar_f32); default all")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the runs reported beside the headline (forced NUFFT, all direct, four rows, the dense "
                         "mesh, serving)")
    ap.add_argument("--lofar", action="store_true",
                    help="time the LOFAR-like wide-field workload (5.0M vis x 4M pix, 60-degree cap) in float64 at "
                         "eps = 1e-9 too (about two minutes more; its float32 step at eps = 1e-4 is a default mode)")
    ap.add_argument("--workload", choices=("ska-like", "dense-10km"), default="ska-like",
                    help="the workload of the reported step: the SKA-like 995k vis x 1M pix cap (default, the "
                         "metric's workload) or the dense 30-degree DCOS mesh of the 10 km rung (238k vis x 10.24M "
                         "pix), e.g. for kernel traces of that mesh alone")
    ap.add_argument("--dist-runs", type=int, default=20,
                    help="passes of synthesis then analysis timed one by one with HIP events for the per-direction "
                         "median / p10 / p90 of the float32 and float64 plans (0: skip)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB mebibytes three times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library runs the whole transform on a single MI355X "
              f"(--gpus {args.gpus} is not supported)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2306_06007_amd as hv
    from paper_2306_06007_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe:
        # a plain copy of known size: what FETCH_SIZE / WRITE_SIZE read for it
        # calibrates the counters that measure the kernels' HBM traffic
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "copies": 3}), flush=True)
        return
    dense_head = args.workload == "dense-10km"
    wl = W.dense_dcos(10.0) if dense_head else W.ska_like(n_pix=args.n_pix)
    head_mode = "dense_10km" if dense_head else "auto"   # key of the counter summaries of this step
    log(f"workload {wl.name}")

    def run_mode(dtype, eps, direct_threshold, steps, warm, ntrans=1, work=None, dist=0):
        wl_m = wl if work is None else work
        return _run_mode(wl_m, dtype, eps, direct_threshold, steps, warm, ntrans, dist)

    def _run_mode(wl, dtype, eps, direct_threshold, steps, warm, ntrans, dist):
        cd = torch.complex64 if dtype == "f32" else torch.complex128
        t0 = time.perf_counter()
        plan = hv.Plan(wl.uvw, wl.xyz, eps, dtype, direct_threshold=direct_threshold, ntrans_hint=ntrans)
        plan_s = time.perf_counter() - t0
        sky, vis = wl.sky, wl.vis
        if ntrans > 1:   # further rows: the same data rotated, so every row differs
            sky = np.concatenate([np.roll(sky, 7919 * r, axis=1) for r in range(ntrans)])
            vis = np.concatenate([np.roll(vis, 7919 * r, axis=1) for r in range(ntrans)])
        bufs = (torch.as_tensor(sky).to("cuda", cd), torch.as_tensor(vis).to("cuda", cd),
                torch.empty((ntrans, wl.n_vis), dtype=cd, device="cuda"),
                torch.empty((ntrans, wl.n_pix), dtype=cd, device="cuda"))
        sec = time_steps(plan, bufs, steps, warm)
        log(f"{dtype} eps={eps:g} direct_threshold={direct_threshold:g}: {sec * 1e3:.1f} ms/step over {steps} "
            f"steps (plan {plan_s:.1f}s)")
        st = kernel_table(plan, bufs)
        dirs = direction_times(plan, bufs, dist) if dist > 0 else None
        if dirs:
            log(f"  per direction over {dist} runs (median ms): synthesis {dirs['synthesis_ms']['median']:.1f}, "
                f"analysis {dirs['analysis_ms']['median']:.1f}")
        info = plan.info()
        r = dict(sec=sec, steps=steps, warmup=warm, plan_s=plan_s, stats=st, info=info,
                 V=bufs[2][0].cpu().numpy(), I=bufs[3][0].cpu().numpy(), n_units=wl.n_vis + wl.n_pix,
                 workload=wl.name, wl=wl, dtype=dtype, directions=dirs)
        plan.free()
        del bufs
        torch.cuda.empty_cache()
        return r

    results = {"f32": run_mode("f32", 1e-4, args.direct_threshold, args.steps, args.warmup, dist=args.dist_runs)}
    if not args.skip_f64:
        results["f64"] = run_mode("f64", 1e-9, args.direct_threshold, args.f64_steps or max(1, args.steps // 5),
                                  min(1, args.warmup), dist=args.dist_runs)
    modes = {}
    wanted = set(filter(None, args.modes.split(","))) or {"forced_nufft", "all_direct", "batched_ntrans4",
                                                           "dense_10km", "dense_10km_all_direct", "dense_30km",
                                                           "sparse_100km", "sparse_100km_forced_nufft",
                                                           "forced_nufft_ntrans4", "compact_f64", "compact_f32",
                                                           "lofar_f32"}
    if not args.no_modes:
        # the two other execution modes of the float32 transform: every sub-problem as a
        # NUFFT (the path the spread / FFT / interp rooflines describe), every one direct
        if "forced_nufft" in wanted:
            modes["forced_nufft"] = run_mode("f32", 1e-4, 0.0, 1, 0)
        if "all_direct" in wanted:
            modes["all_direct"] = run_mode("f32", 0.0, -1.0, 1, 0)
        # ntrans = 4 data rows through one plan (e.g. channels or polarisations)
        if "batched_ntrans4" in wanted:
            modes["batched_ntrans4"] = run_mode("f32", 1e-4, args.direct_threshold, 1, 1, ntrans=4)
        # four rows through NUFFT sub-problems only (what a row costs on the NUFFT path)
        if "forced_nufft_ntrans4" in wanted:
            modes["forced_nufft_ntrans4"] = run_mode("f32", 1e-4, 0.0, 1, 0, ntrans=4)
    if not (args.no_modes or dense_head) and wanted & {"dense_10km", "dense_10km_all_direct"}:
        # a dense 30-degree DCOS image of the paper's telescope-radius ladder (10 km rung,
        # 238k vis x 10.24M pixels): most terms go through NUFFT sub-problems
        dense = W.dense_dcos(10.0)
        log(f"workload {dense.name}")
        if "dense_10km" in wanted:
            modes["dense_10km"] = run_mode("f32", 1e-4, args.direct_threshold, 1, 1, work=dense)
        if "dense_10km_all_direct" in wanted:
            modes["dense_10km_all_direct"] = run_mode("f32", 0.0, -1.0, 1, 0, work=dense)
        del dense
    if not (args.no_modes or dense_head) and "dense_30km" in wanted:
        # the 30 km rung (341k vis x 74.65M pixels)
        dense = W.dense_dcos(30.0)
        log(f"workload {dense.name}")
        modes["dense_30km"] = run_mode("f32", 1e-4, args.direct_threshold, 1, 0, work=dense)
        del dense
    if not (args.no_modes or dense_head) and wanted & {"sparse_100km", "sparse_100km_forced_nufft"}:
        # the sparse-mesh experiment: the 100 km rung's 394k visibilities and 500 pixels in
        # five separate 10 x 10 patches of its DCOS grid
        sparse = W.sparse_dcos(100.0)
        log(f"workload {sparse.name}")
        if "sparse_100km" in wanted:
            modes["sparse_100km"] = run_mode("f32", 1e-4, args.direct_threshold, 5, 1, work=sparse)
        if "sparse_100km_forced_nufft" in wanted:
            modes["sparse_100km_forced_nufft"] = run_mode("f32", 1e-4, 0.0, 5, 1, work=sparse)
        del sparse
    if not (args.no_modes or dense_head) and wanted & {"compact_f64", "compact_f32"}:
        # the small float64 case (2,000 vis x 3,072 pix, eps = 1e-6), timed beside the
        # oracle's full sums in the CPU leg
        compact = W.compact_disk()
        log(f"workload {compact.name}")
        if "compact_f64" in wanted:
            modes["compact_f64"] = run_mode("f64", 1e-6, args.direct_threshold, 20, 2, work=compact)
        if "compact_f32" in wanted:   # the same case in float32 at eps = 1e-4
            modes["compact_f32"] = run_mode("f32", 1e-4, args.direct_threshold, 20, 2, work=compact)
        del compact
    if not (args.no_modes or dense_head) and "lofar_f32" in wanted and not args.lofar:
        # the LOFAR-like wide field (5.0M vis x 4M pix, 60-degree cap), one float32 step
        lofar = W.lofar_like()
        log(f"workload {lofar.name}")
        modes["lofar_f32"] = run_mode("f32", 1e-4, args.direct_threshold, 1, 0, work=lofar)
        del lofar
    if args.lofar:
        lofar = W.lofar_like()
        log(f"workload {lofar.name}")
        modes["lofar_f32"] = run_mode("f32", 1e-4, args.direct_threshold, 1, 1, work=lofar)
        modes["lofar_f64"] = run_mode("f64", 1e-9, args.direct_threshold, 1, 0, work=lofar)
        del lofar

    r32, r64 = results["f32"], results.get("f64")
    n_units = wl.n_vis + wl.n_pix
    value = n_units / r32["sec"]
    if args.direct_threshold != 0 and args.direct_threshold >= 0:
        head_mode = "threshold"          # no counter summaries are taken at other thresholds
    elif args.direct_threshold == 0:
        head_mode = "dense_10km_forced_nufft" if dense_head else "forced_nufft"
    kname, roof = roofline_entry(r32["stats"], "f32", mode=head_mode)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "(vis+pix)/s",
        "n_gpus": 1,
        "steps": r32["steps"],
        "warmup": r32["warmup"],
        "ms_per_step": r32["sec"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"dense 30-deg DCOS mesh, 10 km rung, {wl.n_vis} vis x {wl.n_pix} pix, "
                                "synthesis+analysis" if dense_head else
                                f"ska-like {wl.n_vis} vis x {wl.n_pix} pix (200 antennas, 50 hour angles, "
                                "10-deg Fibonacci cap), synthesis+analysis"), "eps": 1e-4,
                   "n_vis": wl.n_vis, "n_pix": wl.n_pix, "ntrans": 1},
        "roofline": roof,
        "roofline_kernel": kname,
        "f64": ({"value": n_units / r64["sec"], "ms_per_step": r64["sec"] * 1e3, "steps": r64["steps"], "eps": 1e-9,
                 "roofline": roofline_entry(r64["stats"], "f64", mode=head_mode)[1],
                 "roofline_kernel": roofline_entry(r64["stats"], "f64", mode=head_mode)[0]}
                if r64 else None),
        "f32_over_f64": r64["sec"] / r32["sec"] if r64 else None,
        "plan_seconds": {d: results[d]["plan_s"] for d in results},
        "plan": {d: {k: results[d]["info"][k] for k in ("n_vis_chunks", "n_sky_chunks", "n_pairs_nufft",
                                                          "n_pairs_direct", "w", "w2", "sigma", "sigma2",
                                                          "grid_cells", "direct_terms")} for d in results},
        "kernels": {d: {k: {"ms": round(v["ms"], 3), "launches": v["launches"],
                            "GB_s": round(v["alg_bytes"] / (v["ms"] * 1e6), 1) if v["ms"] > 0 and v["alg_bytes"] else None}
                        for k, v in results[d]["stats"].items() if v["launches"]} for d in results},
        "mode": {"direct_threshold": args.direct_threshold},
        # device time per direction (HIP events), median / p10 / p90 over --dist-runs passes
        "directions": {d: results[d]["directions"] for d in results if results[d]["directions"]} or None,
        "source_hash": kernel_source_hash(),
    }
    if "forced_nufft" in modes:
        # the rooflines of the NUFFT kernels on the forced-NUFFT step (every sub-problem a
        # type-3 NUFFT): spreading and interpolation are the graded ones
        fr = modes["forced_nufft"]
        out["nufft_rooflines"] = {}
        for k in ("spread", "interp", "fft_x", "fft_y", "fft_z", "transpose", "prephase"):
            v = fr["stats"][k]
            if v["launches"] and v["ms"] > 0:
                _, rf = roofline_entry(fr["stats"], "f32", k, mode="forced_nufft")
                out["nufft_rooflines"][k] = {"achieved_GB_s": round(rf["achieved"], 1), "frac": round(rf["frac"], 4),
                                             "ms": round(v["ms"], 2), "launches": v["launches"],
                                             "alg_bytes": v["alg_bytes"]}
    if modes:
        out["modes"] = {}
        for m, r in modes.items():
            rows = 4 if m in ("batched_ntrans4", "forced_nufft_ntrans4") else 1
            ent = {"ms_per_step": r["sec"] * 1e3, "value": rows * r["n_units"] / r["sec"], "ntrans": rows,
                   "workload": r["workload"], "dtype": r["dtype"],
                   "n_pairs_nufft": r["info"]["n_pairs_nufft"], "n_pairs_direct": r["info"]["n_pairs_direct"],
                   "kernels": {k: {"ms": round(v["ms"], 3), "launches": v["launches"]}
                               for k, v in r["stats"].items() if v["launches"]}}
            roofs = {}
            for k, v in r["stats"].items():
                if v["launches"] and v["ms"] > 0 and (v["alg_bytes"] or k == "direct"):
                    _, rf = roofline_entry(r["stats"], r["dtype"], k, rows=rows, mode=m)
                    roofs[k] = {"bound": rf["bound"], "achieved": round(rf["achieved"], 1), "unit": rf["unit"],
                                "frac": round(rf["frac"], 4)}
                    if "issue_bound" in rf:
                        roofs[k]["issue_bound_frac"] = round(rf["issue_bound"]["frac"], 4)
                    if rf["traffic"]:
                        # measured HBM bytes per launch over the launch duration
                        avg_s = v["ms"] * 1e-3 / max(1, v["launches"])
                        roofs[k]["traffic_GB_s"] = round(rf["traffic"] / avg_s / 1e9, 1)
                        roofs[k]["traffic_frac"] = round(rf["traffic"] / avg_s / 1e9 / HBM_PEAK_GBS, 4)
            ent["rooflines"] = roofs
            out["modes"][m] = ent
    if args.serving or not (args.no_serving or args.no_modes):
        out["serving"], serving_reqs, serving_res = serving_run()
    if not args.no_cpu_baseline:
        import oracle
        log("cpu baseline (oracle on sampled rows)...")
        cb, (rv, Vs), (rp, Is) = cpu_baseline(wl)
        out["cpu_baseline"] = cb
        def errs(V, I, Vr, Ir, k):
            return {"synthesis": oracle.rel_l2(V, Vr), "analysis": oracle.rel_l2(I, Ir),
                    "synthesis_max_rel_err": oracle.max_rel_err(V, Vr),
                    "analysis_max_rel_err": oracle.max_rel_err(I, Ir), "rows": int(k)}

        out["rel_l2_vs_oracle"] = {d: errs(results[d]["V"][rv], results[d]["I"][rp], Vs[0], Is[0], len(rv))
                                   for d in results}
        for m, r in modes.items():
            if r["wl"] is wl:
                out["modes"][m]["rel_l2_vs_oracle"] = errs(r["V"][rv], r["I"][rp], Vs[0], Is[0], len(rv))
            elif m in ("compact_f64", "compact_f32"):
                # every output row, and the oracle's own time for the whole step
                ow = r["wl"]
                t0 = time.perf_counter()
                Vo = oracle.synthesis(ow.uvw, ow.xyz, ow.sky)[0]
                Io = oracle.analysis(ow.uvw, ow.xyz, ow.vis)[0]
                t_or = time.perf_counter() - t0
                out["modes"][m]["rel_l2_vs_oracle"] = errs(r["V"], r["I"], Vo, Io, ow.n_vis + ow.n_pix)
                out["modes"][m]["oracle"] = {"ms_per_step": t_or * 1e3, "value": r["n_units"] / t_or,
                                             "cores": oracle.max_threads(),
                                             "gpu_over_oracle": t_or / r["sec"]}
            else:   # another workload: its own sampled rows, the oracle's time extrapolated by rows
                ow = r["wl"]
                rv2 = W.sample_rows(ow.n_vis, 256, seed=51)
                rp2 = W.sample_rows(ow.n_pix, 256, seed=52)
                t0 = time.perf_counter()
                Vo = oracle.synthesis(ow.uvw, ow.xyz, ow.sky, rows=rv2)[0]
                t_v = time.perf_counter() - t0
                t0 = time.perf_counter()
                Io = oracle.analysis(ow.uvw, ow.xyz, ow.vis, rows=rp2)[0]
                t_p = time.perf_counter() - t0
                out["modes"][m]["rel_l2_vs_oracle"] = errs(r["V"][rv2], r["I"][rp2], Vo, Io, len(rv2))
                t_full = t_v * ow.n_vis / len(rv2) + t_p * ow.n_pix / len(rp2)
                out["modes"][m]["oracle"] = {"ms_per_step": t_full * 1e3, "value": r["n_units"] / t_full,
                                             "cores": oracle.max_threads(), "gpu_over_oracle": t_full / r["sec"],
                                             "sample": f"{len(rv2)} + {len(rp2)} sampled rows, extrapolated"}
        if "serving" in out:
            log("serving results against the oracle (1,024 sampled rows per request)...")
            out["serving"]["vs_oracle"] = serving_errors(serving_reqs, serving_res)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
