"""Host-side checks of bench.py: the one-GPU contract, the roofline
arithmetic, and the committed counter summaries it reads (no GPU needed)."""
import glob
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_unknown_workload_is_an_argument_error():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "nonexistent"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "invalid choice" in r.stderr


def test_hbm_roofline_is_algorithmic_bytes_over_average_launch_time():
    # 4 launches moving 8e9 algorithmic bytes in 2 ms: 2e9 bytes per 0.5 ms launch = 4 TB/s
    st = {"spread": {"ms": 2.0, "launches": 4, "alg_bytes": 8e9, "alg_flops": 0.0},
          "fft_x": {"ms": 1.0, "launches": 4, "alg_bytes": 1e9, "alg_flops": 0.0}}
    name, r = bench.roofline_entry(st, "f32", mode="no-such-mode")
    assert name == "spread"                       # the kernel taking the most time
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(4000.0)
    assert r["frac"] == pytest.approx(0.5)
    assert r["traffic"] is None                   # no counter summary under that key


def test_direct_roofline_counts_algorithmic_operations_and_issue_cycles():
    # 1e12 terms in 100 ms: 1e13 terms/s, 30 operations per term -> 300 TFLOP/s
    st = {"direct": {"ms": 100.0, "launches": 1, "alg_bytes": 0.0, "alg_flops": 1e12}}
    assert bench.ALG_OPS_PER_TERM == 30.0
    for dtype in ("f32", "f64"):
        name, r = bench.roofline_entry(st, dtype, mode="no-such-mode")
        assert name == "direct" and r["bound"] == "alu" and r["unit"] == "TFLOP/s"
        assert r["achieved"] == pytest.approx(300.0)
        assert r["frac"] == pytest.approx(r["achieved"] / bench.VECTOR_PEAK_TFLOPS[dtype])
        ib = r["issue_bound"]
        assert ib["term_rows_per_s"] == pytest.approx(bench.LANE_CYCLES_PER_S / bench.VALU_CYCLES_PER_TERM[(dtype, 1)])
        assert ib["frac"] == pytest.approx(1e13 / ib["term_rows_per_s"])
    # issue cycles never exceed the instruction count, and four rows share the phase work
    for key, cyc in bench.VALU_CYCLES_PER_TERM.items():
        assert cyc <= bench.VALU_OPS_PER_TERM[key]
    for dt in ("f32", "f64"):
        assert bench.VALU_OPS_PER_TERM[(dt, 4)] < bench.VALU_OPS_PER_TERM[(dt, 1)]


def test_vector_peaks_follow_from_the_unit_counts():
    lane_cycles = 256 * 4 * 16 * 2.4e9
    assert bench.LANE_CYCLES_PER_S == lane_cycles
    assert bench.VECTOR_PEAK_TFLOPS["f32"] == pytest.approx(2 * 2 * lane_cycles / 1e12, rel=1e-3)
    assert bench.VECTOR_PEAK_TFLOPS["f64"] == pytest.approx(2 * lane_cycles / 1e12, rel=1e-3)


TRAFFIC = sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")))


def test_traffic_summaries_exist():
    assert TRAFFIC, "no committed counter summaries"


@pytest.mark.parametrize("path", TRAFFIC, ids=[os.path.basename(p) for p in TRAFFIC])
def test_traffic_summary_is_consistent(path):
    """Each summary's bytes per launch are its per-dispatch counter readings
    scaled by the copy calibration; its key matches its file name; every
    command it names runs committed files only."""
    d = json.load(open(path))
    assert os.path.basename(path) == f"traffic_{d['kernel']}_{d['dtype']}_{d['mode']}.json"
    b = d["fetch_kib_per_dispatch"] * 1024 * d["fetch_scale"] + d["write_kib_per_dispatch"] * 1024 * d["write_scale"]
    assert d["bytes_per_launch"] == pytest.approx(b, rel=1e-12)
    assert d["dispatches"] > 0 and d["bytes_per_launch"] > 0
    assert 0.5 < d["fetch_scale"] < 4 and 0.5 < d["write_scale"] < 4
    assert len(d["source_hash"]) == 16
    cmds = d["commands"] + d["calibration_commands"] + ([d["timing"]["command"]] if "timing" in d else [])
    for c in cmds:
        assert c.startswith("rocprofv3 ") and " -- python3 bench.py" in c
        assert "_work" not in c
    if "timing" in d:
        t = d["timing"]
        assert t["traffic_GB_s"] == pytest.approx(b / (t["avg_us"] * 1e-6) / 1e9, rel=1e-9)


def test_stale_summaries_are_not_reported(tmp_path, monkeypatch):
    """A summary taken on other kernel sources reads as unmeasured."""
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_spread_f32_auto.json").write_text(json.dumps({"source_hash": "0" * 16, "bytes_per_launch": 1.0}))
    (prof / "traffic_interp_f32_auto.json").write_text(
        json.dumps({"source_hash": bench.kernel_source_hash(), "bytes_per_launch": 2.0}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "paper_2306_06007_amd" / "csrc").mkdir(parents=True)
    for f in ("kernels.hip", "hvox_internal.hpp"):
        src = os.path.join(ROOT, "paper_2306_06007_amd", "csrc", f)
        (tmp_path / "paper_2306_06007_amd" / "csrc" / f).write_bytes(open(src, "rb").read())
    assert bench.measured_traffic("spread", "f32", "auto") is None
    assert bench.measured_traffic("interp", "f32", "auto") == 2.0
    assert bench.measured_traffic("fft_x", "f32", "auto") is None


def test_host_cpu_model_is_a_string():
    m = bench.host_cpu_model()
    assert isinstance(m, str) and m
