#!/usr/bin/env python3
"""Benchmark of the fused stream + quasi-equilibrium step on one MI355X.

Workload: 2-D periodic Kolmogorov flow, 1024 x 1024 lattice, four forcing
periods, Re = 60, Wi = 1.0, beta = 0.7, FENE dumbbells (b = 25) on a
16-point Q-grid (208 Q-nodes per r-node), FP64 populations, multimode seeded
perturbation of RMS amplitude 1e-4 u0.  A step is one pass of the whole hot
path (stream, moments, mixture velocity, spring term, equilibria, relaxation
of both species, lagged-field write) over the lattice.

Prints one JSON line: MLUPS (10^6 r-node updates per second, each carrying
9 + 25 * 208 populations), the roofline of the step kernel, and the FP64 CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = dict(nx=1024, ny=1024, periods=4, Re=60.0, Wi=1.0, beta=0.7, nq=16, spring=0,
                seed=0, perturbation=1e-4)
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure


def cpu_baseline(seconds_target: float = 15.0) -> dict:
    """The oracle, unchanged, on a 64 x 64 window-sized lattice that carries
    the 1024^2 workload's parameters (same Q-grid, same per-node work)."""
    import oracle

    w = WORKLOAD
    o = oracle.OracleSim(64, 64, nq=w["nq"], spring=w["spring"], Re=w["Re"], Wi=w["Wi"],
                         beta=w["beta"], periods=w["periods"], ny_param=w["ny"])
    o.rest()
    o.perturb(w["seed"], w["perturbation"] * 100, True)
    o.step(2)  # warm caches and threads
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds_target:
        o.step(5)
        n += 5
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {"value": 64 * 64 * n / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle, 64x64 lattice with the 1024^2 workload parameters "
                      f"(nq=16, 208 Q-nodes, FENE), {n} steps in {dt:.1f} s, OpenMP over rows"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--pre-steps", type=int, default=-1,
                    help="base-state column steps (-1: 5 max(l^2/nu, lambda))")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-file", default=os.path.join(
        ROOT, "profiles", "k_step_f64_kolmogorov1024_nq16_traffic.txt"))
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the lattice would shard as y-slabs; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2201_10132_amd as P

    w = WORKLOAD
    torch.cuda.init()
    stream = torch.cuda.Stream()
    t = P.Tpl(w["nx"], w["ny"], w["Re"], w["Wi"], w["beta"], periods=w["periods"],
              nq=w["nq"], spring=w["spring"], pre_steps=args.pre_steps, pert_modes=1)
    t.set_stream(stream.cuda_stream)
    t0 = time.perf_counter()
    t.init(seed=w["seed"], perturbation=w["perturbation"])
    init_s = time.perf_counter() - t0
    d0 = t.diagnostics()
    t.step(args.warmup)
    print(f"# init {init_s:.1f} s  nqd={t.nqd}  qsplit={t.query('qsplit_used'):.0f}",
          file=sys.stderr, flush=True)

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    t.step(args.steps)  # synchronises before returning
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = ev0.elapsed_time(ev1) / args.steps

    d1 = t.diagnostics()
    N = w["nx"] * w["ny"]
    nqd = t.nqd
    bytes_step = t.query("bytes_per_step")
    mlups = N * args.steps / wall / 1e6
    achieved = bytes_step / (kernel_ms * 1e-3) / 1e9
    traffic = None  # HBM bytes per launch from the committed counter runs
    try:
        rec = dict(l.split(None, 1) for l in open(args.traffic_file).read().splitlines() if l)
        if rec.get("kernel_source_sha", "").strip() == kernel_source_sha():
            traffic = float(rec["bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        pass
    out = {
        "metric": "MLUPS + % HBM roofline, FP64 vs FP32/batched/learned at stated growth-rate error",
        "value": round(mlups, 3),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded multimode perturbation of the forced laminar base state)",
        "config": {"workload": "kolmogorov_1024x1024_nq16_fene_fp64", "nx": w["nx"], "ny": w["ny"],
                   "nq": w["nq"], "nqd": nqd, "periods": w["periods"], "Re": w["Re"],
                   "Wi": w["Wi"], "beta": w["beta"], "perturbation": w["perturbation"],
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
        "mqlups": round(mlups * nqd, 1),
        "kernel_ms": round(kernel_ms, 4),
        "init_s": round(init_s, 2),
        "conservation": {"mass_S": abs(d1["mass_S"] / d0["mass_S"] - 1),
                         "mass_P": abs(d1["mass_P"] / d0["mass_P"] - 1)},
        "amplitude": d1["amplitude"],
    }
    t.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def kernel_source_sha() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in ("tpl_kernels.hip", "tpl_internal.h"):
        with open(os.path.join(ROOT, "paper_2201_10132_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
