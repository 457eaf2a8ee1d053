"""Throughput of the DVM-BGK octree step on one MI355X.

One step = one pass of the whole hot path over the state: transport across
leaf faces for every discrete velocity, the FP64 moment reduction, the
corrected-Maxwellian BGK relaxation (one fused kernel), then the global FP64
conservation sums.  Default workload: 64^3 root cubes with a seeded 40% refined
once (996,150 leaf cells), 24^3 velocities on [-6, 6]^3, FP32 f with FP64
moments, first-order upwind, periodic Sod-like jump, tau from Kn = 0.01.

Prints ONE JSON line: CVU/s (cell-velocity updates per second), the roofline
of the fused step kernel (HIP events on the launch stream), and the FP64 CPU
oracle timed on a bounded sample of the same construction.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DVM cell-velocity updates/s + % HBM roofline, FP64/FP32/hybrid, same error"
HBM_PEAK_GBS = 8000.0
# sources that define the fused step kernel: HBM counters recorded under
# profiles/ count only while these are unchanged
KERNEL_SOURCES = ["paper_1503_00707_amd/csrc/step_impl.h", "paper_1503_00707_amd/csrc/kernels.h",
                  "paper_1503_00707_amd/csrc/kernels_f32.hip", "paper_1503_00707_amd/csrc/solver.cpp"]
TRAFFIC_PROFILE = "profiles/k_step_fused_octree64_v24_p40_fp32.md"


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(n_launch_bytes):
    """HBM bytes per launch from the committed counter profile, if it was
    taken on the current kernel source (else None)"""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic_json:"):
            t = json.loads(line.split(":", 1)[1])
            if t.get("source_sha256") != kernel_source_hash():
                return None
            return dict(read_bytes=t["read_bytes"], write_bytes=t["write_bytes"],
                        total_bytes=t["read_bytes"] + t["write_bytes"],
                        vs_algorithmic=(t["read_bytes"] + t["write_bytes"]) / n_launch_bytes,
                        source=TRAFFIC_PROFILE)
    return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_case(name):
    from paper_1503_00707_amd import dvm as D
    from paper_1503_00707_amd import inputs as I
    w = I.workload(name)
    lev, ijk = D.balance(w.forest)
    import dataclasses
    forest = dataclasses.replace(w.forest, level=lev, ijk=ijk)
    solid = None
    if w.solid_ball is not None:
        cx, cy, cz, r, lv = w.solid_ball
        solid = I.solid_flags(forest, (cx, cy, cz), r, lv)
    return w, forest, solid


def gpu_bench(args):
    import torch

    from paper_1503_00707_amd import dvm as D
    from paper_1503_00707_amd import inputs as I

    t0 = time.time()
    w, forest, solid = build_case(args.workload)
    mesh = D.Mesh(forest, solid)
    t = mesh.tables()
    prim = I.fields(w.fields, I.leaf_centres(forest)[t["input"]], **w.field_args)
    prec = D.PREC_FP64 if args.precision == "fp64" else D.PREC_FP32
    p = D.make_params(w.nv[0], w.vhi[0], precision=prec, scheme=w.scheme, collision=w.collision,
                      tau_mode=w.tau_mode, tau_or_kn=w.tau_or_kn, inflow=w.inflow, t_wall=w.t_wall)
    s = D.Solver(mesh, p)
    if args.shape:
        T, W, G, NT = (int(x) for x in args.shape.split(","))
        s.set_shape(T, W, G, NT)
    s.init_maxwellian(prim)
    del prim
    dt = s.dt(w.cfl)
    torch.cuda.synchronize()
    log(f"[bench] {args.workload}: {s.n} cells x {s.nv} velocities, {args.precision}, "
        f"{2 * s.sizes.f_bytes / 1e9:.1f} GB of f, setup {time.time() - t0:.1f}s")
    s.global_sums()
    rc, g0, _, _ = s.check()

    def one_step(ev=None):
        if ev is not None:
            ev[0].record()
        s.step(1, dt=dt)
        if ev is not None:
            ev[1].record()
        s.global_sums()

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} done")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for i in range(args.steps):
        one_step(evs[i])
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = evs[0][0].elapsed_time(end)
    k_ms = [a.elapsed_time(b) for a, b in evs]
    rc, g1, bad, nsteps = s.check()
    log(f"[bench] timed {args.steps} steps: {total_ms:.2f} ms (wall {wall * 1e3:.1f} ms), "
        f"step kernel mean {np.mean(k_ms):.3f} ms, status {rc}")
    cvu = s.n * s.nv * args.steps / (total_ms / 1e3)
    fbytes = 8 if prec == D.PREC_FP64 else 4
    # algorithmic bytes of one fused step: read f once, write f once per CVU
    alg_bytes = 2 * fbytes * s.n * s.nv
    k_mean_s = float(np.mean(k_ms)) / 1e3
    achieved = alg_bytes / k_mean_s / 1e9
    drift = np.abs(g1 - g0) / np.maximum(np.abs(g0), 1e-300)
    split = s.split() == 1 and w.scheme == I.SCHEME_UPWIND1
    kernel = ("k_step fused step (transport+moments+Maxwellian+BGK) as two launches: the reduced kernel over "
              "cells without FINER/WALL faces, the full kernel over the rest; events bracket both"
              if split else "k_step (fused transport+moments+Maxwellian+BGK, one launch; cells without FINER/WALL "
              "faces take the reduced code path)")
    return dict(cvu=cvu, total_ms=total_ms, k_ms=k_ms, achieved=achieved, alg_bytes=alg_bytes, n=s.n, nv=s.nv,
                rc=rc, drift=drift, g0=g0, w=w, fbytes=fbytes, dt=dt, kernel=kernel)


def gpu_bench_batch(args):
    """64 independent periodic instances of uneven size and velocity grid,
    advanced by one recorded graph launch per step (after autotuning)."""
    import dataclasses

    import torch

    from paper_1503_00707_amd import dvm as D
    from paper_1503_00707_amd import inputs as I

    t0 = time.time()
    ws = I.batch_workloads(seed=4)
    solvers, meshes = [], []
    cvu_step, alg_bytes = 0, 0
    for w in ws:
        lev, ijk = D.balance(w.forest)
        f = dataclasses.replace(w.forest, level=lev, ijk=ijk)
        m = D.Mesh(f)
        t = m.tables()
        p = D.make_params(w.nv[0], w.vhi[0], precision=D.PREC_FP32, tau_mode=w.tau_mode, tau_or_kn=w.tau_or_kn)
        s = D.Solver(m, p)
        s.init_maxwellian(I.fields(w.fields, I.leaf_centres(f)[t["input"]], **w.field_args))
        meshes.append(m)
        solvers.append(s)
        cvu_step += s.n * s.nv
        alg_bytes += 8 * s.n * s.nv
    torch.cuda.synchronize()
    b = D.Batch(solvers, cfl=0.5)
    log(f"[bench] batch of {len(solvers)}: {sum(s.n for s in solvers)} cells, {cvu_step:.4g} CVU/step, "
        f"{alg_bytes / 2 / 1e9:.1f} GB per state buffer, setup {time.time() - t0:.1f}s")
    t1 = time.time()
    b.tune(reps=2)
    log(f"[bench] tuned in {time.time() - t1:.1f}s: {b.groups()}")
    g0 = [s.check()[1] for s in solvers]
    b.step(args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.step(args.steps)
    e1.record()
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    rcs = [s.check() for s in solvers]
    # mass and energy drift per instance relative to the instance's totals (momentum sums are ~0)
    drift = max(float(max(abs(r[1][0] - g[0]) / abs(g[0]), abs(r[1][4] - g[4]) / abs(g[4]))) for r, g in zip(rcs, g0))
    rc = min(r[0] for r in rcs)
    return dict(cvu=cvu_step * args.steps / (total_ms / 1e3), total_ms=total_ms, alg_bytes=alg_bytes, rc=rc,
                drift=drift, groups=b.groups(), n=sum(s.n for s in solvers), instances=len(solvers))


def copy_ceiling(gb=8.0, reps=5):
    """Practical bandwidth reference measured in the same run: the better of a
    plain device copy and a streaming elementwise kernel (b = 2 a) over gb GB,
    read + write bytes over the median time."""
    import torch
    torch.cuda.empty_cache()
    n = int(gb * 1e9) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    best = 0.0
    for op in (lambda: b.copy_(a), lambda: torch.mul(a, 2.0, out=b)):
        op()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            op()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        best = max(best, 8 * n / (float(np.median(ts)) / 1e3) / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return best


def copy_calibration(gb):
    """A plain device-to-device copy of known size: its HBM counters give the
    scale factor between counter units and bytes."""
    import torch
    n = int(gb * 1e9) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    log(f"[bench] copy calibration: {4 * n / 1e9:.2f} GB read + write in {ms:.3f} ms = {8 * n / ms / 1e6:.0f} GB/s")
    del a, b
    torch.cuda.empty_cache()


def cpu_baseline(args):
    """FP64 oracle on the host cores: the same construction on 16^3 roots."""
    from oracle import oracle as O
    from paper_1503_00707_amd import inputs as I
    name = "octree16_v24_p40"
    w = I.workload(name)
    lev, ijk = O.balance(w.forest)
    import dataclasses
    forest = dataclasses.replace(w.forest, level=lev, ijk=ijk)
    cores = len(os.sched_getaffinity(0))
    cores = min(cores, 16)
    O.set_threads(cores)
    m = O.Mesh(forest)
    t = m.tables()
    p = O.make_params(w.nv, w.vlo, w.vhi, scheme=w.scheme, collision=w.collision, tau_mode=w.tau_mode,
                      tau_or_kn=w.tau_or_kn)
    s = O.Solver(m, p)
    s.init_maxwellian(I.fields(w.fields, I.leaf_centres(forest)[t["input"]], **w.field_args))
    dt = s.dt_cfl(w.cfl)
    n_steps, t_used = 0, 0.0
    while t_used < args.cpu_seconds and n_steps < 50:
        t0 = time.perf_counter()
        s.step(dt, 1)
        t_used += time.perf_counter() - t0
        n_steps += 1
        log(f"[bench] oracle step {n_steps}: {t_used:.1f}s")
    cvu = m.n_cells * s.nv * n_steps / t_used
    return dict(value=cvu, unit="CVU/s", cores=int(O.get_threads()), kind="oracle",
                sample=f"{name}: {m.n_cells} cells x {s.nv} velocities, FP64, {n_steps} steps, {t_used:.1f}s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="octree64_v24_p40")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--shape", default="", help="threads,wpe,xcd_group,nt_store of the step kernel")
    ap.add_argument("--copy-calibration-gb", type=float, default=0.0,
                    help="also run a plain device copy of this many GB (read + write), for counter calibration")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration_gb > 0:
        copy_calibration(args.copy_calibration_gb)
    if args.workload == "batch64":
        r = gpu_bench_batch(args)
        ms = r["total_ms"] / args.steps
        out = {
            "metric": METRIC, "value": r["cvu"], "unit": "CVU/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "batch64", "instances": r["instances"], "cells": r["n"],
                       "velocity_grids": "12^3 / 16^3 / 24^3 on [-6, 6]^3", "graph": "one hipGraph launch per step",
                       "groups": r["groups"]},
            "roofline": {"bound": "hbm", "kernel": "batched step graph (all groups + global sums)",
                         "achieved": r["alg_bytes"] / (ms / 1e3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": r["alg_bytes"] / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                         "algorithmic_bytes_per_launch": r["alg_bytes"]},
            "conservation_drift_rel_max_mass_energy": r["drift"], "status": int(r["rc"]),
        }
        print(json.dumps(out), flush=True)
        return
    r = gpu_bench(args)
    copy_gbs = copy_ceiling()
    log(f"[bench] plain device copy: {copy_gbs:.0f} GB/s")
    cpu = None if args.no_cpu_baseline else cpu_baseline(args)
    w = r["w"]
    ms = r["total_ms"] / args.steps
    # the committed counter profile covers the default workload and launch shape only
    traffic = (measured_traffic(r["alg_bytes"])
               if args.workload == "octree64_v24_p40" and args.precision == "fp32" and not args.shape else None)
    out = {
        "metric": METRIC,
        "value": r["cvu"],
        "unit": "CVU/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "cells": r["n"], "velocities": r["nv"],
                   "velocity_grid": f"{w.nv[0]}^3 on [{w.vlo[0]}, {w.vhi[0]}]^3",
                   "scheme": "upwind1" if w.scheme == 0 else "muscl-minmod",
                   "precision": "f stored FP32, moments/Maxwellian/correction FP64" if args.precision == "fp32"
                   else "FP64", "tau": f"hard sphere, Kn={w.tau_or_kn}", "dt": r["dt"],
                   "pct_hbm_roofline_whole_step": 100.0 * (2 * r["fbytes"] * r["n"] * r["nv"]) / (ms / 1e3) / 8e12},
        "roofline": {"bound": "hbm", "kernel": r["kernel"],
                     "achieved": r["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r["achieved"] / HBM_PEAK_GBS,
                     "traffic": traffic["total_bytes"] if traffic else None, "traffic_detail": traffic,
                     "kernel_ms_mean": float(np.mean(r["k_ms"])), "algorithmic_bytes_per_launch": r["alg_bytes"],
                     "copy_gbs_same_run": copy_gbs, "frac_of_copy": r["achieved"] / copy_gbs},
        "conservation_drift_rel": {"mass": float(r["drift"][0]), "energy": float(r["drift"][4])},
        "status": int(r["rc"]),
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
