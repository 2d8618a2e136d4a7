"""Host-side checks of the benchmark's bookkeeping (no GPU): the one-GPU
refusal, the per-DOF byte model behind the roofline object, the roofline
arithmetic, the staleness rule of the measured traffic, and the lattice
enumeration the surrogate-error report uses."""
import json
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


@pytest.mark.parametrize("variant,res,fwd,bwd", [
    # residual: x 8 + b 8 + centre and 7 lower weights 64 + r (4 or 8)
    ("surr_f32", 84, 8, 20), ("surr_f64", 88, 16, 24), ("surr_f32_v1", 84, 8, 20),
    # stored factors: r, L (7 planes), w / w, 1/D, L^T (7 planes), x in and out
    ("stored_f64", 88, 72, 88), ("stored_sgs", 88, 72, 88),
    # surrogate operator: the weights are evaluated, not loaded
    ("surr_f32_sa", 20, 8, 20), ("surr_f64_sa", 24, 16, 24),
])
def test_byte_model_per_dof(variant, res, fwd, bwd):
    assert bench.kernel_bytes(variant) == {"residual": res, "forward": fwd, "backward": bwd}


def test_roofline_reports_the_slowest_kernel_with_algorithmic_bytes():
    n = 22_108_415
    res = {"kernel_ms": {"forward": 0.49, "backward": 0.535, "residual": 0.70}, "n_dof": n, "tile": [16, 32]}
    r = bench.roofline(res, "surr_f32", 6, "no_such_workload")
    assert r["kernel"] == "k_residual" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["bytes_per_dof"] == 84 and r["algorithmic_bytes_per_launch"] == 84 * n
    gbs = 84 * n / 0.70e-3 / 1e9
    assert math.isclose(r["achieved"], gbs, rel_tol=1e-3)
    assert r["peak"] == 8000.0 and math.isclose(r["frac"], gbs / 8000.0, rel_tol=1e-3)
    assert r["traffic"] is None  # no counters for this workload
    # the residual kernel that runs: LDS-staged on 8x8 and 16x16 blocks, with
    # the surrogate operator the surrogate residual
    for tile in ([8, 8], [16, 16]):
        res["tile"] = tile
        assert bench.roofline(res, "surr_f32", 6, "no_such_workload")["kernel"] == "k_residual_lds"
    assert bench.roofline(res, "surr_f32_sa", 6, "no_such_workload")["kernel"] == "k_residual_sa"
    res["kernel_ms"]["backward"] = 0.9
    assert bench.roofline(res, "surr_f32", 6, "no_such_workload")["kernel"] == "k_bwd_flow"


def test_measured_traffic_only_for_the_profiled_sources(monkeypatch):
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    key = next(iter(t["entries"]))
    workload, variant, kernel = key.split("/")
    e = t["entries"][key]
    monkeypatch.setattr(bench, "source_hash", lambda: t["source_sha256"])
    assert bench.measured_traffic(workload, variant, kernel) == e["fetch_bytes"] + e["write_bytes"]
    assert bench.measured_traffic(workload, variant, "k_no_such_kernel") is None
    monkeypatch.setattr(bench, "source_hash", lambda: "0" * 64)
    assert bench.measured_traffic(workload, variant, kernel) is None


@pytest.mark.parametrize("level", [2, 3, 4, 5])
def test_lattice_coords_enumerate_the_interior_in_lexicographic_order(level):
    import numpy as np
    n = 1 << level
    c = bench.lattice_coords(level).astype(np.int64)
    assert len(c) == math.comb(n - 1, 3)
    x, y, z = c[:, 0], c[:, 1], c[:, 2]
    assert (x >= 1).all() and (y >= 1).all() and (z >= 1).all() and (x + y + z <= n - 1).all()
    key = (z * n + y) * n + x  # z slowest, then y, then x
    assert (np.diff(key) > 0).all()


def test_step_roofline_and_latency_floor_arithmetic():
    import workloads as W
    n = 22_108_415
    wl = W.workload("jit_L9_exp")
    res = {"kernel_ms": {"forward": 0.49, "backward": 0.535, "residual": 0.70}, "n_dof": n, "ms_per_step": 1.77}
    r = bench.step_roofline(res, "surr_f32", wl)
    # residual 84 + forward 8 + backward 20; the fused step keeps r on chip (4 B out, 4 B in)
    assert r["bytes_per_dof"] == 112 and r["fused_bytes_per_dof"] == 104
    gbs = 112 * n / 1.77e-3 / 1e9
    assert math.isclose(r["achieved"], gbs, rel_tol=1e-3) and math.isclose(r["frac"], gbs / 8000.0, rel_tol=1e-3)
    assert bench.step_roofline(res, "stored_f64", wl)["bytes_per_dof"] == 88 + 72 + 88
    f = bench.latency_floor(res, "surr_f32", wl)
    assert f["hyperplanes_per_substitution"] == 3 * 512 - 11 == 1525
    assert math.isclose(f["us_per_hyperplane"], (0.49 + 0.535) * 1e3 / 3050, rel_tol=1e-3)
    hbm_us = (8 + 20) * n / 8e12 * 1e6 / 3050
    assert math.isclose(f["hbm_binds_below_us_per_hyperplane"], hbm_us, rel_tol=1e-2)


def test_overlapped_residual_reporting():
    import workloads as W
    n = 22_108_415
    wl = W.workload("jit_L9_exp")
    res = {"kernel_ms": {"forward": 1.03, "backward": 0.535, "residual": 0.925}, "n_dof": n, "ms_per_step": 1.6,
           "overlap": "overlapped", "tile": [16, 32]}
    r = bench.roofline(res, "surr_f32", 6, "no_such_workload")
    # the bandwidth-bound residual, timed on its own stream, not the waiting forward sweep
    assert r["kernel"] == "k_residual_tag" and r["kernel_ms_per_launch"] == 0.925
    res["tile"] = [16, 16]
    assert bench.roofline(res, "surr_f32", 6, "no_such_workload")["kernel"] == "k_residual_lds"
    assert math.isclose(r["achieved"], 84 * n / 0.925e-3 / 1e9, rel_tol=1e-3)
    f = bench.latency_floor(res, "surr_f32", wl)
    assert f["t_h_from"] == "backward substitution"
    assert math.isclose(f["us_per_hyperplane"], 0.535e3 / 1525, rel_tol=1e-3)
