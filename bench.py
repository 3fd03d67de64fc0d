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
# precision-form workload: 4096^2, 16 periods (same l as above), NQ = 8 (NQ = 6
# diverges at these parameters, and NQ = 8 fits only with FP32 storage)
WORKLOAD_FP32_LARGE = dict(nx=4096, ny=4096, periods=16, Re=60.0, Wi=1.0, beta=0.7, nq=8,
                           spring=0, seed=0, perturbation=1e-4)
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
    ap.add_argument("--no-forms", action="store_true", help="skip the FP32 form measurements")
    ap.add_argument("--traffic-file", default=os.path.join(
        ROOT, "profiles", "k_step_f64_kolmogorov1024_nq16_traffic.txt"))
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the lattice would shard as y-slabs; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.init()
    w = WORKLOAD
    main64 = measure(torch, w, 0, args.steps, args.warmup, args.pre_steps)
    out = {
        "metric": "MLUPS + % HBM roofline, FP64 vs FP32/batched/learned at stated growth-rate error",
        "value": round(main64["mlups"], 3),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main64["wall_ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded multimode perturbation of the forced laminar base state)",
        "config": {"workload": "kolmogorov_1024x1024_nq16_fene_fp64", "nx": w["nx"], "ny": w["ny"],
                   "nq": w["nq"], "nqd": main64["nqd"], "periods": w["periods"], "Re": w["Re"],
                   "Wi": w["Wi"], "beta": w["beta"], "perturbation": w["perturbation"],
                   "parallelism": "single GPU"},
        "roofline": roofline(main64, traffic_bytes(args.traffic_file)),
        "mqlups": round(main64["mlups"] * main64["nqd"], 1),
        "kernel_ms": round(main64["kernel_ms"], 4),
        "init_s": round(main64["init_s"], 2),
        "conservation": main64["conservation"],
        "amplitude": main64["amplitude"],
    }
    if not args.no_forms:
        forms = {}
        f32 = measure(torch, w, 1, args.steps, args.warmup, args.pre_steps)
        forms["fp32_1024x1024_nq16"] = form_entry(f32, main64)
        w3 = WORKLOAD_FP32_LARGE
        f32l = measure(torch, w3, 1, max(5, args.steps // 2), args.warmup, args.pre_steps)
        forms["fp32_4096x4096_nq8"] = form_entry(f32l, None)
        out["precision_forms"] = forms
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def measure(torch, w, precision, steps, warmup, pre_steps) -> dict:
    """Init the workload, then time `steps` steps (HIP events on the library's
    stream and wall clock, both bracketed by device synchronisation)."""
    import paper_2201_10132_amd as P

    stream = torch.cuda.Stream()
    t = P.Tpl(w["nx"], w["ny"], w["Re"], w["Wi"], w["beta"], periods=w["periods"],
              nq=w["nq"], spring=w["spring"], pre_steps=pre_steps, pert_modes=1,
              precision=precision)
    t.set_stream(stream.cuda_stream)
    t0 = time.perf_counter()
    t.init(seed=w["seed"], perturbation=w["perturbation"])
    init_s = time.perf_counter() - t0
    d0 = t.diagnostics()
    t.step(warmup)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    t.step(steps)  # synchronises before returning
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    d1 = t.diagnostics()
    N = w["nx"] * w["ny"]
    res = dict(mlups=N * steps / wall / 1e6, wall_ms=wall / steps * 1e3,
               kernel_ms=ev0.elapsed_time(ev1) / steps, init_s=init_s, nqd=t.nqd,
               bytes_step=t.query("bytes_per_step"), amplitude=d1["amplitude"],
               qsplit=t.query("qsplit_used"),
               conservation={"mass_S": abs(d1["mass_S"] / d0["mass_S"] - 1),
                             "mass_P": abs(d1["mass_P"] / d0["mass_P"] - 1)})
    print(f"# precision={precision} {w['nx']}x{w['ny']} nq={w['nq']}: init {init_s:.1f} s, "
          f"{res['kernel_ms']:.3f} ms/step, qsplit={res['qsplit']:.0f}", file=sys.stderr, flush=True)
    t.close()
    return res


def roofline(m, traffic):
    achieved = m["bytes_step"] / (m["kernel_ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic}


def form_entry(m, ref64):
    e = {"mlups": round(m["mlups"], 3), "ms_per_step": round(m["wall_ms"], 4),
         "roofline": roofline(m, None), "conservation": m["conservation"],
         "amplitude": m["amplitude"]}
    if ref64 is not None:
        e["speedup_vs_fp64"] = round(m["mlups"] / ref64["mlups"], 3)
        e["amplitude_rel_err_vs_fp64"] = abs(m["amplitude"] / ref64["amplitude"] - 1)
    return e


def traffic_bytes(path):
    """HBM bytes per launch from the committed counter runs (None when the
    kernel sources changed since they were taken)."""
    try:
        rec = dict(l.split(None, 1) for l in open(path).read().splitlines() if l)
        if rec.get("kernel_source_sha", "").strip() == kernel_source_sha():
            return float(rec["bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        pass
    return None


def kernel_source_sha() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in ("tpl_kernels.hip", "tpl_internal.h"):
        with open(os.path.join(ROOT, "paper_2201_10132_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
