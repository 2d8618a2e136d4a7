"""Benchmark: smoothed DOF-updates/s of the ILU(0) smoothing step on one MI355X.

One step = one smoothing sweep x <- x + C^{-1}(b - A x) over the whole
workload: FP64 residual, forward substitution, backward substitution with the
update (every part of the hot path).  The timed region is one ilu_smooth call
of K sweeps with x and b already resident in HBM (it includes the call's
layout conversion of x and b).  Prints one JSON line.

Default workload: one jittered macro-tetrahedron at refinement level 9
(22,108,415 interior DOFs), coefficient exp(0.5 sin(4 pi x) cos(4 pi y)),
surrogate degree 6: FP32 surrogate sweeps with FP64 residual and update,
beside FP64 stored-factor sweeps and FP64 surrogate sweeps.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


# Algorithmic bytes per interior DOF and kernel (each array touched once per
# kernel; stencil weights: 8 unique FP64 values per point, the other 7 are the
# neighbours' by symmetry).  w: FP64 (8 B) or FP32 (4 B).
def kernel_bytes(variant: str):
    wb = 4 if variant.startswith("surr_f32") else 8
    res = 8 + 8 + 64 + wb                    # x, b, A (8 weights), r
    if variant.endswith("_sa"):
        res = 8 + 8 + wb                      # x, b, r (the operator is evaluated, not loaded)
    if variant in ("stored_f64", "stored_sgs"):
        fwd = 8 + 56 + 8                      # r, L (7), w
        bwd = 8 + 8 + 56 + 8 + 8              # w in, 1/D, L^T (7), x in, x out
    else:
        fwd = wb + wb                         # r, w
        bwd = wb + 8 + 8                      # w in, x in, x out
    return {"residual": res, "forward": fwd, "backward": bwd}


def kernel_flops(variant: str, dg):
    res = 30                                  # 15 multiply-adds
    dg = dg if isinstance(dg, int) else dg[0]  # Horner runs over x only
    if variant in ("stored_f64", "stored_sgs"):
        return {"residual": res, "forward": 14, "backward": 16}
    # Horner: dg multiply-adds per direction (7 forward, 8 backward) plus the sweep
    return {"residual": res, "forward": 14 + 14 * dg, "backward": 16 + 16 * dg}


# variant name -> (library variant, operator of the residual, boundary variant);
# *_sa: surrogate operator in the residual; *_v1: stored exact factors at the
# boundary points (their O(h^-2) bytes are left out of the per-point traffic)
VARIANTS = {"stored_f64": (0, 0, 0), "surr_f64": (1, 0, 0), "surr_f32": (2, 0, 0), "stored_sgs": (3, 0, 0),
            "surr_f64_sa": (1, 1, 0), "surr_f32_sa": (2, 1, 0), "surr_f64_v1": (1, 0, 1), "surr_f32_v1": (2, 0, 1)}
STORED = ("stored_f64", "stored_sgs")
DTYPES = {"surr_f32": "f32 (sweeps, surrogate evaluation) + f64 (residual, update)", "surr_f64": "f64",
          "stored_f64": "f64", "stored_sgs": "f64",
          "surr_f32_sa": "f32 (sweeps, surrogate evaluation) + f64 (residual with f32-evaluated surrogate operator, update)",
          "surr_f64_sa": "f64 (surrogate operator)",
          "surr_f32_v1": "f32 (sweeps, surrogate evaluation, stored boundary factors) + f64 (residual, update)",
          "surr_f64_v1": "f64 (stored boundary factors)"}


def make_smoother(pkg, wl, variant, tile):
    v, a_mode, boundary = VARIANTS[variant]
    kw = {} if variant in STORED else dict(degree=wl.degree, stride=wl.stride, a_mode=a_mode, boundary=boundary)
    return pkg.Smoother(list(wl.tets), v, tile=tile, **kw)
OVERLAP_NAMES = {0: "sequential", 1: "overlapped", 2: "fused"}
CONTRACTION_STEPS = 20
CONTRACTION_SEED = 0x5EED
KERNEL_NAMES = {"residual": "k_residual", "forward": "k_fwd_flow", "backward": "k_bwd_flow"}


def source_hash() -> str:
    """SHA-256 over the library's kernel and host sources (sorted by name)."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2210_15280_amd", "csrc", "*"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str, variant: str, kernel: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current sources; None otherwise."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != source_hash():
        return None
    e = t.get("entries", {}).get("%s/%s/%s" % (workload, variant, kernel))
    if not e:
        return None
    return e["fetch_bytes"] + e["write_bytes"]


def start_vector(torch, n):
    """Seeded U[-1,1] start error of the contraction measurement."""
    import workloads as W
    return torch.tensor(W.SplitMix64(CONTRACTION_SEED).uniform_array(n, -1.0, 1.0), device="cuda")


def run_variant(pkg, torch, wl, variant, steps, warmup, tile=(0, 0), overlap=None, grid=None):
    """Times `steps` sweeps; also measures the smoother's contraction factor.
    overlap / grid (None: the setup's choice) pin the residual mode and the
    persistent grid.  Returns (results, handle): the caller closes the handle."""
    import numpy as np
    t0 = time.perf_counter()
    sm = make_smoother(pkg, wl, variant, tile)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    if grid is not None:
        sm.set_flow_grid(grid)
    if overlap is not None:
        sm.set_overlap(overlap)
    b = torch.tensor(np.concatenate([t.rhs() for t in wl.tets]), device="cuda")
    x = torch.zeros_like(b)
    if warmup:
        sm.smooth(x, b, warmup)
    x.zero_()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    sm.smooth(x, b, steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    loop_ms = sm.timing()[0]
    # relative residual reached, then per-kernel timing (HIP events on the
    # library's stream around every kernel) in a separate run
    rel, _ = sm.smooth(x, b, 0, want_relres=True)
    sm.set_kernel_timing(True)
    x2 = torch.zeros_like(b)
    sm.smooth(x2, b, steps)
    torch.cuda.synchronize()
    _, f_ms, b_ms, r_ms = sm.timing()
    sm.set_kernel_timing(False)
    n = sm.n_total
    # asymptotic contraction: power iteration on I - C^{-1} A from a seeded start
    x2.copy_(start_vector(torch, n))
    rho, rho_res = sm.contraction(x2, CONTRACTION_STEPS)
    grid, grid_max = sm.flow_grid
    out = dict(variant=variant, n_dof=n, setup_s=setup_s, ms_per_step=ms / steps,
               loop_ms_per_step=loop_ms / steps, value=n * steps / (ms * 1e-3), relres_after=rel,
               kernel_ms=dict(forward=f_ms, backward=b_ms, residual=r_ms), tile=list(sm.tile),
               overlap=OVERLAP_NAMES[sm.overlap()], flow_grid=[grid, grid_max],
               residual_chunk=sm.residual_chunk,
               contraction=dict(rho=rho, rho_res=rho_res, steps=CONTRACTION_STEPS))
    return out, sm


def run_to_tol(pkg, torch, wl, variant, tol, cap, tile=(0, 0)):
    """One ilu_smooth call from x = 0 until ||b - A x|| / ||b|| <= tol (FP64
    residual; for the FP32 variant this is its FP64 iterative refinement)."""
    import numpy as np
    sm = make_smoother(pkg, wl, variant, tile)
    b = torch.tensor(np.concatenate([t.rhs() for t in wl.tets]), device="cuda")
    x = torch.zeros_like(b)
    sm.smooth(x, b, 3)
    x.zero_()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    rel, ok = sm.smooth(x, b, cap, rel_tol=tol, want_relres=True)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    k = sm.last_sweeps
    out = dict(variant=variant, n_dof=sm.n_total, sweeps=k, ms=ms, value=sm.n_total * k / (ms * 1e-3),
               relres_after=rel, converged=bool(ok), tile=list(sm.tile), x=x.cpu().numpy())
    sm.close()
    return out


def lattice_coords(level: int):
    """(x, y, z) of the interior points in lexicographic order (z slowest)."""
    import numpy as np
    n = 1 << level
    parts = []
    for z in range(1, n - 2):
        m = n - 1 - z                            # x + y <= m
        cnt = np.arange(m - 1, 0, -1)            # y = 1..m-1 holds m - y points
        y = np.repeat(np.arange(1, m, dtype=np.int16), cnt)
        start = np.repeat(np.cumsum(cnt) - cnt, cnt)
        x = (np.arange(len(y)) - start + 1).astype(np.int16)
        parts.append(np.stack([x, y, np.full(len(y), z, dtype=np.int16)], axis=1))
    return np.concatenate(parts)


LOWER = ((-1, 0, 0), (0, -1, 0), (1, -1, 0), (-1, 1, -1), (0, 1, -1), (0, 0, -1), (1, 0, -1))
LOWER_NAMES = ("w", "s", "se", "bnw", "bn", "bc", "be")


def surrogate_quality(torch, stored, surr, tet_level):
    """Surrogate error per direction against the exact ILU(0) of the same tet
    (first tet of the workload): relative discrete L2 error and max-abs error
    of L_d over the points whose neighbour p + d is interior, and of 1/D over
    all points.  Both operands come from the library (exact factors of the
    stored handle, weights as the sweeps evaluate them)."""
    Lx, Dx = stored.factors(0)
    Ls, Ds = surr.surrogate_values(0)
    xyz = torch.tensor(lattice_coords(tet_level), device="cuda").to(torch.int32)
    n = 1 << tet_level
    s = xyz.sum(dim=1)
    out = {}
    for d, (dx, dy, dz) in enumerate(LOWER):
        m = ((xyz[:, 0] + dx >= 1) & (xyz[:, 1] + dy >= 1) & (xyz[:, 2] + dz >= 1) & (s + dx + dy + dz <= n - 1))
        e = (Ls[:, d] - Lx[:, d])[m]
        out[LOWER_NAMES[d]] = dict(rel_l2=float(e.norm() / Lx[:, d][m].norm()), max_abs=float(e.abs().max()))
    di = 1.0 / Dx
    e = Ds - di
    out["c (1/D)"] = dict(rel_l2=float(e.norm() / di.norm()), max_abs=float(e.abs().max()))
    del Lx, Dx, Ls, Ds, xyz
    return out


def residual_kernel(res, variant):
    """The residual kernel that runs: with the surrogate operator
    k_residual_sa; with the stencil arrays LDS-staged on 8x8 and 16x16 blocks
    (sequential or beside the forward sweep), else point-parallel
    (k_residual, or k_residual_tag beside the sweep)."""
    if variant.endswith("_sa"):
        return "k_residual_sa"
    if tuple(res["tile"]) in ((8, 8), (16, 16)):
        return "k_residual_lds"
    return "k_residual_tag" if res.get("overlap") == "overlapped" else "k_residual"


def roofline(res, variant, dg, workload):
    """The dominant kernel against the HBM roofline.  Sequential residual:
    the slowest of the three kernels.  Overlapped residual: the residual
    kernel (timed on its own stream): the forward
    substitution beside it waits for its bands, so its time is mostly the
    residual's."""
    bpd = kernel_bytes(variant)
    fpd = kernel_flops(variant, dg)
    km = res["kernel_ms"]
    ovl = res.get("overlap") == "overlapped"
    dom = "residual" if ovl else max(km, key=km.get)
    name = residual_kernel(res, variant) if dom == "residual" else KERNEL_NAMES[dom]
    n = res["n_dof"]
    t = km[dom] * 1e-3
    gbs = bpd[dom] * n / t / 1e9
    out = {"bound": "hbm", "kernel": name, "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 5),
           "traffic": measured_traffic(workload, variant, name),
           "algorithmic_bytes_per_launch": bpd[dom] * n, "bytes_per_dof": bpd[dom], "flops_per_dof": fpd[dom],
           "kernel_ms_per_launch": round(km[dom], 5)}
    if ovl:
        out["runs_beside"] = "k_fwd_flow (overlapped residual)"
    return out


def step_roofline(res, variant, wl):
    """The whole step (residual, forward and backward substitution) against
    the HBM roofline: the three kernels' algorithmic bytes per DOF (r and w
    written and read back between kernels included) over the measured time per
    step; beside it the compulsory bytes of the fused step, where r never
    leaves the chip."""
    bpd = kernel_bytes(variant)
    step_b = sum(bpd.values())
    n = res["n_dof"]
    t = res["ms_per_step"] * 1e-3
    gbs = step_b * n / t / 1e9
    wb = 4 if variant.startswith("surr_f32") else 8
    fused = step_b - 2 * wb
    return {"bound": "hbm", "bytes_per_dof": step_b, "fused_bytes_per_dof": fused, "achieved": round(gbs, 2),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 5),
            "dof_updates_per_s_at_peak": HBM_PEAK_GBS * 1e9 / step_b,
            "fused_dof_updates_per_s_at_peak": HBM_PEAK_GBS * 1e9 / fused}


def latency_floor(res, variant, wl):
    """Dependency-latency floor of the two substitutions: each runs the
    3n - 11 hyperplanes of the largest tetrahedron one after another, so a
    sweep takes at least 2 (3n - 11) t_h, t_h the time per hyperplane.  Reports
    the measured t_h (substitution kernel times over the hyperplane count) and
    the t_h at which the substitutions' algorithmic bytes would bind at the
    HBM peak instead."""
    n = 1 << max(t.level for t in wl.tets)
    hp = 3 * n - 11
    km = res["kernel_ms"]
    bpd = kernel_bytes(variant)
    hbm_ms = (bpd["forward"] + bpd["backward"]) * res["n_dof"] / (HBM_PEAK_GBS * 1e9) * 1e3
    # with the overlapped residual the forward substitution's time includes
    # waiting for the residual: t_h then comes from the backward one alone
    ovl = res.get("overlap") == "overlapped"
    t_h_ms = km["backward"] / hp if ovl else (km["forward"] + km["backward"]) / (2 * hp)
    return {"hyperplanes_per_substitution": hp, "substitutions_ms": round(km["forward"] + km["backward"], 5),
            "us_per_hyperplane": round(t_h_ms * 1e3, 4),
            "t_h_from": "backward substitution" if ovl else "both substitutions",
            "floor_ms_at_measured_t_h": round(2 * hp * t_h_ms, 5),
            "hbm_binds_below_us_per_hyperplane": round(hbm_ms * 1e3 / (2 * hp), 4),
            "substitutions_hbm_bound_ms": round(hbm_ms, 5)}


def extra_configs(pkg, torch, steps):
    """The level-8 refinement to 1e-10 (FP32 surrogate + FP64 refinement vs
    FP64 stored factors) and the batch of 256 tetrahedra (levels 5-7, FP32
    surrogate vs FP64 stored, `steps` sweeps as one graph launch)."""
    import workloads as W
    out = {}
    wl8 = W.workload("jit_L8_sin")
    c3 = {}
    for v in ("surr_f32", "stored_f64"):
        r = run_to_tol(pkg, torch, wl8, v, wl8.rel_tol, 20000)
        r.pop("x")
        c3[v] = r
        print("# %s %s: %d sweeps to relres %.3e in %.1f ms" % (wl8.name, v, r["sweeps"], r["relres_after"], r["ms"]),
              file=sys.stderr, flush=True)
    c3["time_to_tol_speedup_vs_stored_f64"] = c3["stored_f64"]["ms"] / c3["surr_f32"]["ms"]
    out[wl8.name + "_to_1e-10"] = c3
    wlb = W.workload("batch256_L567")
    c4 = {}
    for v in ("surr_f32", "stored_f64"):
        r, h = run_variant(pkg, torch, wlb, v, steps, 3)
        h.close()
        torch.cuda.empty_cache()
        c4[v] = {k: r[k] for k in ("value", "ms_per_step", "setup_s", "kernel_ms", "tile", "relres_after", "n_dof",
                                   "overlap", "flow_grid", "residual_chunk")}
        c4[v]["roofline"] = step_roofline(r, v, wlb)
        print("# %s %s: %.3e DOF-updates/s, %.4f ms/step" % (wlb.name, v, r["value"], r["ms_per_step"]),
              file=sys.stderr, flush=True)
    c4["speedup_vs_stored_f64"] = c4["surr_f32"]["value"] / c4["stored_f64"]["value"]
    c4["sweeps_per_graph_launch"] = steps
    out[wlb.name] = c4
    return out


_CPU_RUN = None  # the oracle sweep of the CPU baseline, inherited by forked workers


def _cpu_worker(k):
    tt = time.perf_counter()
    _CPU_RUN(k)
    return time.perf_counter() - tt


def host_cores():
    """Cores this process may run on, at most 8: forked workers inherit the
    parent's open GPU device handles, and processes holding a GPU are a
    limited resource on shared hosts."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(8, n))


def cpu_baseline(wl, variant, budget_s=12.0, sample_level=7):
    """The oracle (plain C, one thread per process) on a bounded sample of the
    workload: its first tetrahedron (same geometry, coefficient, surrogate
    degree and stride) at refinement level min(level, sample_level); sweeps
    timed, setup not.  One copy of the sample runs on every host core (forked
    workers, no GPU use), so the value is the host's aggregate rate; the
    single-core rate is in `sample`.  A sweep costs the same per DOF at every
    level, so the rate carries over to the workload's level."""
    global _CPU_RUN
    import numpy as np
    import oracle as O
    import workloads as W
    t0 = wl.tets[0]
    lvl = min(t0.level, sample_level)
    t = W.Tet(t0.verts, lvl, t0.coeff_kind, t0.coeff_params, t0.rhs_state)
    P = O.Problem.from_tet(t)
    L, U, D = P.ilu0()
    b = t.rhs()
    if variant == "stored_f64":
        run = lambda k: P.smooth(L, D, b, nsweeps=k)
        kind = "matrix-form ILU(0) sweep, FP64"
    else:
        s = O.effective_stride(t.level, wl.degree, wl.stride)
        c = O.fit_surrogate(t.level, L, D, wl.degree, s)
        Lw, Dinv = O.eval_surrogate(t.level, c, wl.degree)
        if variant == "surr_f32":
            Lw32, Di32 = Lw.astype(np.float32), Dinv.astype(np.float32)
            run = lambda k: P.smooth_stencil_f32(Lw32, Di32, b, nsweeps=k)
            kind = "stencil sweep with FP32 surrogate weights and substitutions, FP64 residual"
        else:
            run = lambda k: P.smooth_stencil(Lw, Dinv, b, nsweeps=k)
            kind = "stencil sweep with FP64 surrogate weights"
    tt = time.perf_counter()
    run(1)
    one = max(time.perf_counter() - tt, 1e-4)
    k = max(1, min(1000, int(budget_s / one)))
    tt = time.perf_counter()
    run(k)
    el = time.perf_counter() - tt
    single = P.N * k / el
    value, cores, wall = single, 1, el
    ncores = host_cores()
    if ncores > 1:
        import multiprocessing as mp
        _CPU_RUN = run
        try:
            with mp.get_context("fork").Pool(ncores) as pool:
                tt = time.perf_counter()
                pool.map(_cpu_worker, [k] * ncores, chunksize=1)
                wall = time.perf_counter() - tt
            value, cores = ncores * P.N * k / wall, ncores
        except (OSError, RuntimeError) as e:
            print("# cpu baseline: parallel run failed (%s); single core reported" % e, file=sys.stderr, flush=True)
        finally:
            _CPU_RUN = None
    return {"value": value, "unit": "DOF-updates/s", "cores": cores, "kind": "oracle",
            "sample": "%s tetrahedron 0 at level %d (%d DOFs; workload level %d), %d sweeps per core on %d core(s) "
                      "in %.1f s, %s; single core %.3g DOF-updates/s; the per-DOF sweep cost is the same at "
                      "every level, so the rate applies to the workload's level" % (
                          wl.name, lvl, P.N, t0.level, k, cores, wall, kind, single)}


def copy_calibration(torch, nbytes, reps=3):
    """A plain streaming copy of known size (reads and writes nbytes each launch),
    for scaling the HBM byte counters."""
    src = torch.rand(nbytes // 4, device="cuda", dtype=torch.float32)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print("# copy calibration: %d launches, %d bytes read + %d bytes written each" % (reps, nbytes, nbytes),
          file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="jit_L9_exp")
    ap.add_argument("--variants", default="surr_f32,stored_f64,surr_f64")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the level-8 refinement and the 256-tetrahedron batch of the default run")
    ap.add_argument("--tile", default="auto",
                    help="block shape BVxBW of the sweep schedule, e.g. 16x32 (one, or one per variant)")
    ap.add_argument("--overlap", default="auto",
                    help="residual beside the forward sweep: auto (the setup's choice), off or on (one, or per variant)")
    ap.add_argument("--grid", default="auto",
                    help="workgroups of the persistent sweeps: auto (the setup's choice) or a number (one, or per variant)")
    ap.add_argument("--copy-bytes", type=int, default=0, help="also run a streaming copy of this size")
    ap.add_argument("--to-tol", type=float, default=0.0,
                    help="instead of fixed sweeps: time each variant's refinement to this relative residual")
    ap.add_argument("--max-sweeps", type=int, default=20000)
    ap.add_argument("--pcg-tol", type=float, default=0.0,
                    help="instead of fixed sweeps: time CG preconditioned by each variant to this relative residual")
    ap.add_argument("--pcg-abs-tol", type=float, default=0.0, help="absolute residual target of --pcg-tol mode")
    ap.add_argument("--max-iters", type=int, default=5000)
    ap.add_argument("--degree", default="", help="surrogate degrees dx,dy,dz instead of the workload's")
    ap.add_argument("--lfa", action="store_true",
                    help="instead of sweeps: time the LFA orientation choice for every tetrahedron of the workload")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(independent tetrahedra would shard across GPUs with no exchange).", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2210_15280_amd as pkg
    import workloads as W
    pkg.lib()
    wl = W.workload(a.workload)
    if a.degree:
        import dataclasses
        dg = tuple(int(c) for c in a.degree.split(","))
        wl = dataclasses.replace(wl, degree=dg[0] if len(dg) == 1 else dg)
    variants = a.variants.split(",")
    def per_variant(arg, parse):
        items = arg.split(",")
        if len(items) == 1:
            items = items * len(variants)
        if len(items) != len(variants):
            sys.exit("bench.py: give one value or one per variant")
        return [parse(c) for c in items]
    tiles = per_variant(a.tile, lambda c: (0, 0) if c == "auto" else tuple(int(k) for k in c.split("x")))
    overlaps = per_variant(a.overlap, lambda c: {"auto": None, "off": 0, "on": 1}[c])
    grids = per_variant(a.grid, lambda c: None if c == "auto" else int(c))
    tile = tiles[0]
    if a.to_tol > 0:
        return main_to_tol(a, torch, pkg, wl, variants, tile)
    if a.pcg_tol > 0 or a.pcg_abs_tol > 0:
        return main_pcg(a, torch, pkg, wl, variants, tile)
    if a.lfa:
        return main_lfa(a, pkg, wl)
    results, handles = {}, {}
    for v in variants:
        i = variants.index(v)
        results[v], handles[v] = run_variant(pkg, torch, wl, v, a.steps, a.warmup, tiles[i], overlaps[i], grids[i])
        print("# %s: %.3e DOF-updates/s, %.4f ms/step, relres %.3e, tile %s, grid %s, %s residual, kernels %s, "
              "contraction %.6f" % (
                  v, results[v]["value"], results[v]["ms_per_step"], results[v]["relres_after"],
                  "x".join(map(str, results[v]["tile"])), "/".join(map(str, results[v]["flow_grid"])),
                  results[v]["overlap"], json.dumps(results[v]["kernel_ms"]), results[v]["contraction"]["rho"]),
              file=sys.stderr, flush=True)
        if v not in STORED and "stored_f64" not in variants:
            handles[v].close()
    quality = {v: {"contraction": r["contraction"]} for v, r in results.items()}
    if "stored_f64" in handles:
        for v in variants:
            if v not in STORED:
                quality[v]["surrogate_error_vs_exact_ilu"] = surrogate_quality(
                    torch, handles["stored_f64"], handles[v], wl.tets[0].level)
    for h in handles.values():
        h.close()
    torch.cuda.empty_cache()
    if a.copy_bytes:
        copy_calibration(torch, a.copy_bytes)
    head = variants[0]
    hr = results[head]
    line = {
        "metric": "smoothed DOF-updates/s (ILU(0) sweep) on 1 MI355X; FP32 surrogate vs FP64 stored",
        "value": hr["value"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": hr["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[head],
        "data": "synthetic (seeded jittered macro-tetrahedra, seeded RHS)",
        "config": {"workload": wl.name, "variant": head, "n_tets": len(wl.tets),
                   "levels": sorted({t.level for t in wl.tets}), "n_dof": hr["n_dof"],
                   "surrogate_degree": wl.degree, "sample_stride": wl.stride, "tile": hr["tile"],
                   "parallelism": "single GPU"},
        "variants": {v: {k: r[k] for k in ("value", "ms_per_step", "loop_ms_per_step", "relres_after", "setup_s",
                                            "kernel_ms", "tile", "overlap", "flow_grid", "residual_chunk")}
                     for v, r in results.items()},
        "roofline": roofline(hr, head, wl.degree, wl.name),
        "step_roofline": step_roofline(hr, head, wl),
        "latency_floor": latency_floor(hr, head, wl),
        "quality": quality,
    }
    if "stored_f64" in results and head != "stored_f64":
        line["speedup_vs_stored_f64"] = hr["value"] / results["stored_f64"]["value"]
    if not a.no_extra and a.workload == "jit_L9_exp":
        line["configs"] = extra_configs(pkg, torch, a.steps)
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(wl, head)
    print(json.dumps(line))


def main_to_tol(a, torch, pkg, wl, variants, tile):
    import numpy as np
    res = {}
    for v in variants:
        res[v] = run_to_tol(pkg, torch, wl, v, a.to_tol, a.max_sweeps, tile)
        r = res[v]
        print("# %s: %d sweeps to relres %.3e (%s) in %.1f ms, %.3e DOF-updates/s, tile %s" % (
            v, r["sweeps"], r["relres_after"], "converged" if r["converged"] else "NOT converged", r["ms"], r["value"],
            "x".join(map(str, r["tile"]))), file=sys.stderr, flush=True)
    head = variants[0]
    hr = res[head]
    ref = res.get("stored_f64")
    for v, r in res.items():
        r["rel_diff_vs_stored_f64"] = (float(np.linalg.norm(r["x"] - ref["x"]) / np.linalg.norm(ref["x"]))
                                       if ref is not None else None)
    line = {
        "metric": "smoothed DOF-updates/s (ILU(0) sweep) on 1 MI355X; FP32 surrogate vs FP64 stored",
        "value": hr["value"], "unit": "DOF-updates/s", "n_gpus": 1, "steps": hr["sweeps"], "warmup": 3,
        "ms_per_step": hr["ms"] / max(1, hr["sweeps"]), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[head],
        "data": "synthetic (seeded jittered macro-tetrahedra, seeded RHS)",
        "config": {"workload": wl.name, "variant": head, "n_tets": len(wl.tets), "n_dof": hr["n_dof"],
                   "levels": sorted({t.level for t in wl.tets}), "surrogate_degree": wl.degree,
                   "sample_stride": wl.stride, "rel_tol": a.to_tol, "tile": hr["tile"], "parallelism": "single GPU"},
        "to_tol": {v: {k: r[k] for k in ("sweeps", "ms", "value", "relres_after", "converged", "tile",
                                          "rel_diff_vs_stored_f64")} for v, r in res.items()},
    }
    if ref is not None and head != "stored_f64":
        line["time_to_tol_speedup_vs_stored_f64"] = ref["ms"] / hr["ms"]
    print(json.dumps(line))


def run_pcg(pkg, torch, wl, variant, rel_tol, abs_tol, cap, tile=(0, 0)):
    """CG preconditioned by one smoother variant, from x = 0, until the
    recursively updated residual meets the tolerance; device time of the call."""
    import numpy as np
    sm = make_smoother(pkg, wl, variant, tile)
    b = torch.tensor(np.concatenate([t.rhs() for t in wl.tets]), device="cuda")
    x = torch.zeros_like(b)
    sm.pcg(x, b, 2, rel_tol=rel_tol, abs_tol=abs_tol)     # warm-up (captures the iteration graph)
    x.zero_()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    k, res, ok = sm.pcg(x, b, cap, rel_tol=rel_tol, abs_tol=abs_tol)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    bn = float(b.norm())
    out = dict(variant=variant, n_dof=sm.n_total, iterations=k, ms=ms, ms_per_iteration=ms / max(k, 1),
               true_relres=res / bn, true_res=res, converged=bool(ok), tile=list(sm.tile))
    sm.close()
    return out


def main_pcg(a, torch, pkg, wl, variants, tile):
    res = {}
    for v in variants:
        res[v] = r = run_pcg(pkg, torch, wl, v, a.pcg_tol, a.pcg_abs_tol, a.max_iters, tile)
        print("# pcg %s: %d iterations in %.1f ms (%.3f ms/it), true relres %.3e, %s" % (
            v, r["iterations"], r["ms"], r["ms_per_iteration"], r["true_relres"],
            "converged" if r["converged"] else "NOT converged"), file=sys.stderr, flush=True)
    head = variants[0]
    line = {
        "metric": "PCG time to tolerance on 1 MI355X (preconditioner = smoother variant)",
        "value": res[head]["ms"], "unit": "ms", "n_gpus": 1, "higher_is_better": False,
        "dtype": DTYPES[head], "data": "synthetic (seeded jittered macro-tetrahedra, seeded RHS)",
        "config": {"workload": wl.name, "variant": head, "n_dof": res[head]["n_dof"], "rel_tol": a.pcg_tol,
                   "abs_tol": a.pcg_abs_tol, "surrogate_degree": wl.degree, "parallelism": "single GPU"},
        "pcg": res,
    }
    for ref in ("stored_f64", "stored_sgs"):
        if ref in res and head != ref:
            line["time_speedup_vs_" + ref] = res[ref]["ms"] / res[head]["ms"]
    print(json.dumps(line))


def main_lfa(a, pkg, wl, samples=16):
    """LFA orientation choice (24 permutations x samples^3 frequencies per
    tetrahedron) for the workload's tetrahedra; host clock around the
    synchronous library call."""
    tets = list(wl.tets)
    for _ in range(2):
        pkg.lfa_orientation(tets, samples)
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        mu, best = pkg.lfa_orientation(tets, samples)
    ms = (time.perf_counter() - t0) * 1e3 / reps
    nfreq = sum(1 for i in range(samples) for j in range(samples) for k in range(samples)
                if max(abs(2 * c + 1 - samples) for c in (i, j, k)) * 2 >= samples)
    nsym = len(tets) * 24 * nfreq
    line = {"metric": "LFA orientation choice: smoothing factors of 24 vertex permutations per tetrahedron",
            "value": len(tets) / (ms * 1e-3), "unit": "tetrahedra/s", "n_gpus": 1, "ms_per_call": ms,
            "symbols_per_s": nsym / (ms * 1e-3), "higher_is_better": True, "dtype": "f64",
            "data": "synthetic (seeded jittered macro-tetrahedra)",
            "config": {"workload": wl.name, "n_tets": len(tets), "samples": samples, "frequencies": nfreq},
            "best_mu": {"min": min(m[b] for m, b in zip(mu, best)), "max": max(m[b] for m, b in zip(mu, best))}}
    if not a.no_cpu:
        import oracle as O
        t0 = time.perf_counter()
        O.lfa_orientation(tets[0].verts, samples)
        el = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": 1.0 / el, "unit": "tetrahedra/s", "cores": 1, "kind": "oracle",
                                "sample": "one tetrahedron of the workload, %.2f s" % el}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
