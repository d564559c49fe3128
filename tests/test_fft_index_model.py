"""CPU check of the FFT pass kernel's addressing (tests/fft_index_model.cpp, a
host model of its index arithmetic built against the planner): every access
of every FFT geometry stays inside its buffer and every Stockham stage writes
each element of its lines once -- for every smooth line length, and for the
plans of small SKA-like, dense DCOS and compact inputs in both precisions with
the automatic choice and with every sub-problem a NUFFT."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2306_06007_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2306_06007_amd", "csrc")


@pytest.fixture(scope="module")
def model():
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    tmp = tempfile.mkdtemp(prefix="hvox_fft_model_")
    exe = os.path.join(tmp, "fft_index_model")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
                    os.path.join(HERE, "fft_index_model.cpp"), os.path.join(CSRC, "planner.cpp"), "-o", exe,
                    "-lpthread"], check=True)
    yield tmp, exe
    shutil.rmtree(tmp, ignore_errors=True)


def _run(exe, *args, need_checks=True):
    r = subprocess.run([exe, *map(str, args)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    g, c, e = (int(x) for x in r.stdout.split()[1::2])
    assert e == 0, r.stdout
    assert c > 0 or not need_checks, r.stdout
    return g


def test_every_line_length(model):
    assert _run(model[1], "lengths") == 110


@pytest.mark.parametrize("name,make", [
    ("ska", lambda: W.ska_like(n_pix=10000, n_ant=30, n_times=6)),
    ("dense", lambda: W.dense_dcos(1.0)),
    ("compact", lambda: W.compact_disk()),
], ids=["ska_like", "dense_1km", "compact"])
@pytest.mark.parametrize("dtype,eps", [(0, 1e-4), (1, 1e-9)], ids=["f32", "f64"])
@pytest.mark.parametrize("threshold", [-1.0, 0.0], ids=["auto", "forced_nufft"])
def test_plan_geometries(model, name, make, dtype, eps, threshold):
    tmp, exe = model
    wl = make()
    uvw, xyz = os.path.join(tmp, f"{name}_uvw.bin"), os.path.join(tmp, f"{name}_xyz.bin")
    if not os.path.exists(uvw):
        np.ascontiguousarray(wl.uvw, dtype=np.float64).tofile(uvw)
        np.ascontiguousarray(wl.xyz, dtype=np.float64).tofile(xyz)
    # a 4 MB FFT budget splits the small inputs into many sub-problems; the
    # automatic choice may take all of them direct (no FFT geometry to check)
    _run(exe, "plan", wl.n_vis, wl.n_pix, uvw, xyz, dtype, eps, 4e6, threshold, need_checks=threshold == 0.0)
