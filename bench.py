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
oracle timed on a bounded sample of the same workload.  Extra entries: the
FP32 and BF16 storage forms (1024^2 at NQ 16; 4096^2 at NQ 6 beside its FP64
run), FP64 and FP32 at NQ = 6, the stress-tensor collision model, the growth
rate of the three storage forms over 2000 steps, the batched sweep of 256
seeded instances against the same instances stepped one by one, and the
learned coarse correction (training pipeline, judged errors, corrected-step
cost).  Every workload starts from a base state of
--pre-steps column steps (outside the timed region).
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
# precision-form workload: 4096^2, 16 periods (same l as above), NQ = 6 (the
# largest Q-grid at which the FP64 reference, 2 x 115 GB, fits one GPU)
WORKLOAD_FP32_LARGE = dict(nx=4096, ny=4096, periods=16, Re=60.0, Wi=1.0, beta=0.7, nq=6,
                           spring=0, seed=0, perturbation=1e-4)
# batched sweep: 256 seeded instances (sizes from {128..512}^2, Re, Wi, beta
# drawn per instance), FP32 storage, NQ = 6
BATCH = dict(instances=256, nq=6, precision=1)
# base-state column steps before the timed steps (init only, never timed);
# the library's own default is 5 max(l^2/nu, lambda), ~244k steps here
DEFAULT_PRE_STEPS = 3000
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure


def cpu_baseline(seconds_target: float = 15.0, seconds_1core: float = 8.0) -> dict:
    """The oracle, unchanged, on a 64 x 64 window-sized lattice that carries
    the 1024^2 workload's parameters (same Q-grid, same per-node work):
    first on every host thread, then on one."""
    import oracle

    w = WORKLOAD

    def rate(seconds):
        o = oracle.OracleSim(64, 64, nq=w["nq"], spring=w["spring"], Re=w["Re"], Wi=w["Wi"],
                             beta=w["beta"], periods=w["periods"], ny_param=w["ny"])
        o.rest()
        o.perturb(w["seed"], w["perturbation"] * 100, True)
        o.step(1)  # warm caches and threads
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < seconds:
            o.step(1)
            n += 1
        dt = time.perf_counter() - t0
        return 64 * 64 * n / dt / 1e6, n, dt

    cores = oracle.max_threads()
    v, n, dt = rate(seconds_target)
    oracle.set_threads(1)
    v1, n1, dt1 = rate(seconds_1core)
    oracle.set_threads(cores)
    return {"value": v, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle, 64x64 lattice with the 1024^2 workload parameters "
                      f"(nq=16, 208 Q-nodes, FENE), {n} steps in {dt:.1f} s, OpenMP over rows",
            "value_1core": v1,
            "sample_1core": f"same lattice, 1 thread, {n1} steps in {dt1:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--pre-steps", type=int, default=DEFAULT_PRE_STEPS,
                    help="base-state column steps (-1: 5 max(l^2/nu, lambda))")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the FP32 form measurements")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched sweep")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned correction")
    ap.add_argument("--no-inplace", action="store_true",
                    help="skip the in-place (one population array) measurements")
    ap.add_argument("--no-growth", action="store_true",
                    help="skip the growth-rate comparison of the storage forms")
    ap.add_argument("--growth-steps", type=int, default=2000)
    ap.add_argument("--batch-instances", type=int, default=BATCH["instances"])
    ap.add_argument("--one-by-one-steps", type=int, default=10,
                    help="steps per instance of the one-by-one comparison")
    ap.add_argument("--traffic-file", default=os.path.join(
        ROOT, "profiles", "k_step_fp64_kolmogorov1024_nq16_traffic.txt"))
    ap.add_argument("--batch-traffic-file", default=os.path.join(
        ROOT, "profiles", "k_step_batch_fp32_kolmogorov_batch256_nq6_traffic.txt"))
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the lattice would shard as y-slabs, one per GPU)", file=sys.stderr)
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
                   "base_state_pre_steps": args.pre_steps, "parallelism": "single GPU"},
        "roofline": dict(roofline(main64, traffic_bytes(args.traffic_file)),
                         **copy_ceiling(torch, main64)),
        "mqlups": round(main64["mlups"] * main64["nqd"], 1),
        "kernel_ms": round(main64["kernel_ms"], 4),
        "launch": {"qsplit": int(main64["qsplit"]), "group": main64["group"],
                   "tune_ms": main64["tune_ms"]},
        "init_s": round(main64["init_s"], 2),
        "conservation": main64["conservation"],
        "amplitude": main64["amplitude"],
    }
    if not args.no_forms:
        forms = {}
        f32 = measure(torch, w, 1, args.steps, args.warmup, args.pre_steps)
        forms["fp32_1024x1024_nq16"] = form_entry(f32, main64)
        # FP64 at the batched sweep's NQ (the matched-NQ reference)
        wq = dict(w, nq=BATCH["nq"])
        nq = BATCH["nq"]
        f64q = measure(torch, wq, 0, args.steps, args.warmup, args.pre_steps)
        forms[f"fp64_1024x1024_nq{nq}"] = form_entry(f64q, None)
        f32q = measure(torch, wq, 1, args.steps, args.warmup, args.pre_steps)
        forms[f"fp32_1024x1024_nq{nq}"] = form_entry(f32q, f64q)
        # BF16 form (precision 2)
        b16 = measure(torch, w, 2, args.steps, args.warmup, args.pre_steps)
        forms["bf16_1024x1024_nq16"] = form_entry(b16, main64)
        forms["bf16_1024x1024_nq16"]["speedup_vs_fp32"] = round(b16["mlups"] / f32["mlups"], 3)
        # the large precision-form workload, each form against the FP64 run
        w3 = WORKLOAD_FP32_LARGE
        tag = f"4096x4096_nq{w3['nq']}"
        n3 = max(5, args.steps // 2)
        f64l = measure(torch, w3, 0, n3, args.warmup, args.pre_steps)
        forms[f"fp64_{tag}"] = form_entry(f64l, None)
        f32l = measure(torch, w3, 1, n3, args.warmup, args.pre_steps)
        forms[f"fp32_{tag}"] = form_entry(f32l, f64l)
        b16l = measure(torch, w3, 2, n3, args.warmup, args.pre_steps)
        forms[f"bf16_{tag}"] = form_entry(b16l, f64l)
        forms[f"bf16_{tag}"]["speedup_vs_fp32"] = round(b16l["mlups"] / f32l["mlups"], 3)
        out["precision_forms"] = forms
    if not args.no_inplace:
        out["inplace"] = measure_inplace(torch, out.get("precision_forms"), args)
    if not args.no_forms:
        # same-step gradients: three more launches form this step's psi, M
        # and U before the step (about 1.5x the algorithmic bytes)
        e = form_entry(measure(torch, w, 0, args.steps, args.warmup, args.pre_steps, gradients=1),
                       main64)
        e["speed_vs_lagged"] = e.pop("speedup_vs_fp64")
        e["amplitude_rel_diff_vs_lagged"] = e.pop("amplitude_rel_err_vs_fp64")
        out["same_step_gradients"] = {"fp64_1024x1024_nq16": e}
        # the spring term from psi at the beads (interpolated) instead of its
        # Taylor form: one more launch sums it over Q
        e = form_entry(measure(torch, w, 0, args.steps, args.warmup, args.pre_steps,
                               spring_shift=1), main64)
        e["speed_vs_taylor"] = e.pop("speedup_vs_fp64")
        e["amplitude_rel_diff_vs_taylor"] = e.pop("amplitude_rel_err_vs_fp64")
        out["spring_shift"] = {"fp64_1024x1024_nq16": e}
    if not args.no_forms:
        # the stress-tensor quasi-equilibrium model (Sec. V model (ii)): same
        # bytes, second moments added to the arithmetic; drag time tau1_S =
        # tau2_S / 4, polymer stresses relaxing at half the flux rate
        nuS = main64["nuS"]
        m2 = dict(qe_model=2, tau_drag=0.25 * nuS * 3.0, tau_ratio_p=0.5)
        out["qe_model2"] = {
            "params": {"tau_drag": m2["tau_drag"], "tau_ratio_p": 0.5},
            "fp64_1024x1024_nq16": form_entry(
                measure(torch, w, 0, args.steps, args.warmup, args.pre_steps, **m2), main64),
            "fp32_1024x1024_nq16": form_entry(
                measure(torch, w, 1, args.steps, args.warmup, args.pre_steps, **m2), main64),
        }
        for k in ("fp64_1024x1024_nq16", "fp32_1024x1024_nq16"):
            e = out["qe_model2"][k]
            e.pop("amplitude_rel_err_vs_fp64")  # another model: not comparable
            e["speed_vs_model1_fp64"] = e.pop("speedup_vs_fp64")
    if not args.no_growth:
        # from the converged base state (the library's default column
        # pre-run): the deviations from it are then the perturbation's
        out["growth_rate"] = measure_growth(torch, dict(w, nq=BATCH["nq"]), -1, args.growth_steps)
    if not args.no_batch:
        out["batched"] = measure_batch(torch, args.batch_instances, max(5, args.steps // 2),
                                       args.warmup, args.pre_steps, args.one_by_one_steps)
        if args.batch_instances == BATCH["instances"]:
            # counters were taken with every instance active: scale to the active ones
            tb = traffic_bytes(args.batch_traffic_file)
            bt = out["batched"]
            if tb is not None:
                bt["roofline"]["traffic"] = round(tb * bt["bytes_active_fraction"])
        if args.batch_instances == BATCH["instances"] and not args.no_inplace:
            out["batched_inplace"] = {
                f"fp32_nq{nq}": measure_batch_inplace(torch, nq, max(5, args.steps // 2),
                                                      args.warmup, args.pre_steps)
                for nq in (BATCH["nq"], 10)}
            e = out["batched_inplace"][f"fp32_nq{BATCH['nq']}"]
            e["speed_vs_two_array"] = round(e["mlups"] / out["batched"]["mlups"], 3)
        if "precision_forms" in out:  # (ii) plain FP64 lattice at the sweep's NQ
            ref = out["precision_forms"][f"fp64_1024x1024_nq{BATCH['nq']}"]["mlups"]
            out["batched"]["speedup_vs_fp64_plain_matched_nq"] = round(
                out["batched"]["mlups"] / ref, 3)
    if not args.no_learned:
        out["learned"] = measure_learned(torch, args.pre_steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def measure(torch, w, precision, steps, warmup, pre_steps, **params) -> dict:
    """Init the workload, then time `steps` steps (HIP events on the library's
    stream and wall clock, both bracketed by device synchronisation).  params:
    further library parameters (the collision model)."""
    import paper_2201_10132_amd as P

    stream = torch.cuda.Stream()
    t = P.Tpl(w["nx"], w["ny"], w["Re"], w["Wi"], w["beta"], periods=w["periods"],
              nq=w["nq"], spring=w["spring"], pre_steps=pre_steps, pert_modes=1,
              precision=precision, **params)
    t.set_stream(stream.cuda_stream)
    t0 = time.perf_counter()
    t.init(seed=w["seed"], perturbation=w["perturbation"])
    init_s = time.perf_counter() - t0
    d0 = t.diagnostics()
    # in place, the autotuner times its shapes on 24 real steps of one call
    t.step(max(warmup, 24) if params.get("inplace") else warmup)
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
               qsplit=t.query("qsplit_used"), nuS=t.query("nuS"),
               group=[int(t.query(k)) for k in ("group_x_used", "group_y_used", "group_sync_used")],
               tune_ms=round(t.query("tune_ms"), 1), bytes_state=t.query("bytes_state"),
               conservation={"mass_S": abs(d1["mass_S"] / d0["mass_S"] - 1),
                             "mass_P": abs(d1["mass_P"] / d0["mass_P"] - 1)})
    print(f"# precision={precision} {w['nx']}x{w['ny']} nq={w['nq']}: init {init_s:.1f} s, "
          f"{res['kernel_ms']:.3f} ms/step, qsplit={res['qsplit']:.0f} group={res['group']}",
          file=sys.stderr, flush=True)
    t.close()
    return res


def measure_batch(torch, n, steps, warmup, pre_steps, obo_steps) -> dict:
    """The batched sweep: all instances advanced together (graph replays of
    the batched step), then the same instances stepped one by one."""
    import paper_2201_10132_amd as P
    from paper_2201_10132_amd import inputs

    insts = inputs.c4_instances(n)
    stream = torch.cuda.Stream()
    b = P.Batch(insts, precision=BATCH["precision"], nq=BATCH["nq"], pre_steps=pre_steps,
                time_kernels=1)
    b.set_stream(stream.cuda_stream)
    t0 = time.perf_counter()
    b.init()
    init_s = time.perf_counter() - t0
    b.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)  # synchronises before returning
    wall = time.perf_counter() - t0
    kernel_ms = b.query("kernel_ms")  # HIP events around the step launches only
    nodes = b.query("nodes")
    bytes_all = sum(b.instance(i).query("bytes_per_step") for i in range(n))
    res = {
        "workload": f"kolmogorov_batch_{n}_seeded_fp32_nq{BATCH['nq']}",
        "instances": n, "nodes": int(nodes), "nq": BATCH["nq"],
        "nqd": int(b.instance(0).nqd), "precision": "fp32",
        "steps": steps, "mlups": round(nodes * steps / wall / 1e6, 3),
        "ms_per_step": round(wall / steps * 1e3, 4), "kernel_ms": round(kernel_ms, 4),
        "roofline": roofline(dict(bytes_step=b.query("bytes_per_step"), kernel_ms=kernel_ms), None),
        "qsplit": int(b.query("qsplit_used")), "group": int(b.query("group_used")),
        "grid": int(b.query("grid_used")),
        "items": int(b.query("items")), "graph_steps": int(b.query("graph_steps")),
        "tune_ms": round(b.query("tune_ms"), 1), "init_s": round(init_s, 2),
        "pre_steps": pre_steps, "unstable": int(b.query("unstable")),
        "bytes_active_fraction": b.query("bytes_per_step") / bytes_all,
    }
    # the same instances one after another, each with its own launches
    status = b.status()
    res["unstable_instances"] = [i for i, u in enumerate(status) if u]
    active = [i for i, u in enumerate(status) if not u]
    for i in active:  # untimed: each lattice's first step tunes its own launch shape
        b.instance(i).step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in active:
        b.instance(i).step(obo_steps)
    wall1 = time.perf_counter() - t0
    res["one_by_one_mlups"] = round(nodes * obo_steps / wall1 / 1e6, 3)
    res["speedup_vs_one_by_one"] = round(res["mlups"] / res["one_by_one_mlups"], 3)
    print(f"# batch {n} instances: init {init_s:.1f} s, {kernel_ms:.3f} ms/step, "
          f"qsplit={res['qsplit']} group={res['group']} grid={res['grid']}, one-by-one "
          f"{res['one_by_one_mlups']} MLUPS", file=sys.stderr, flush=True)
    b.close()
    return res


def measure_batch_inplace(torch, nq, steps, warmup, pre_steps) -> dict:
    """The batched sweep with every instance streamed in place (one
    population array each): at the sweep's NQ beside the two-array batch,
    and at NQ 10, where two arrays (404 GB) would not fit one GPU."""
    import paper_2201_10132_amd as P
    from paper_2201_10132_amd import inputs

    insts = inputs.c4_instances(BATCH["instances"])
    stream = torch.cuda.Stream()
    b = P.Batch(insts, precision=BATCH["precision"], nq=nq, pre_steps=pre_steps,
                time_kernels=1, inplace=1)
    b.set_stream(stream.cuda_stream)
    t0 = time.perf_counter()
    b.init()
    init_s = time.perf_counter() - t0
    b.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    wall = time.perf_counter() - t0
    kernel_ms = b.query("kernel_ms")
    nodes = b.query("nodes")
    state = b.query("bytes_state")
    pop = sum(b.instance(i).query("bytes_XS") + b.instance(i).query("bytes_XP")
              for i in range(len(insts)))
    res = {"workload": f"kolmogorov_batch_{len(insts)}_seeded_fp32_nq{nq}_inplace",
           "nq": nq, "nqd": int(b.instance(0).nqd), "steps": steps,
           "mlups": round(nodes * steps / wall / 1e6, 3), "ms_per_step": round(wall / steps * 1e3, 4),
           "kernel_ms": round(kernel_ms, 4),
           "roofline": roofline(dict(bytes_step=b.query("bytes_per_step"), kernel_ms=kernel_ms),
                                None),
           "bytes_state_gb": round(state / 1e9, 1),
           "two_array_bytes_state_gb": round((state + pop) / 1e9, 1),
           "group": int(b.query("group_used")), "grid": int(b.query("grid_used")),
           "init_s": round(init_s, 2), "unstable": int(b.query("unstable"))}
    print(f"# batch in place nq={nq}: init {init_s:.1f} s, {kernel_ms:.3f} ms/step, "
          f"state {res['bytes_state_gb']} GB", file=sys.stderr, flush=True)
    b.close()
    return res


LEARNED = dict(train_seeds=range(1000, 1008), held_out_seeds=range(2000, 2004), fine_steps=960,
               sample_every=120, settle=10, horizon=20, epochs=40)


def measure_learned(torch, pre_steps) -> dict:
    """Learned coarse correction, scaled down from the 64-trajectory plan:
    8 fine 1024^2 FP64 trajectories (NQ = 8, Re ~ U[20, 80], Wi ~ U[0, 1.5],
    beta 0.7, 4 periods, seeds 1000-1007) of 960 fine steps, one training
    pair every 120 (coarse state 10 steps after the restriction, target the
    growth of its difference from the restricted fine run over the next 20
    coarse steps), a 256^2 coarse lattice (4x restriction), 40 epochs of
    Adam; judged on held-out seeds 2000-2003 over 400 fine steps."""
    import paper_2201_10132_amd.learned as LL
    from paper_2201_10132_amd import inputs

    c = LEARNED
    t0 = time.perf_counter()
    trs = inputs.c5_trajectories(c["train_seeds"])
    X, T, t_fine = LL.generate(torch, trs, pre_steps=pre_steps, fine_steps=c["fine_steps"],
                               sample_every=c["sample_every"], settle=c["settle"],
                               horizon=c["horizon"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mlp, l0, l1 = LL.train(torch, X, T, epochs=c["epochs"], lr=1e-3)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    rows = X.shape[0] * X.shape[1] * c["epochs"]
    # matrix-core work per training row: 92 16x16x16 MFMAs per 16 rows
    flops_row = 92 * 2 * 16 ** 3 / 16
    held = inputs.c5_trajectories(c["held_out_seeds"])
    evals = [LL.evaluate(torch, mlp, cfg, pre_steps=pre_steps) for cfg in held]
    plain_ms, corr_ms = LL.coarse_step_ms(torch, mlp, trs[0])
    # the plain fine FP64 step of the same workload (1024^2, NQ 8): what a
    # corrected coarse step stands in for
    fine = measure(torch, dict(WORKLOAD, nq=8, Re=trs[0]["Re"], Wi=trs[0]["Wi"]), 0, 10, 3,
                   pre_steps)
    nc = 256 * 256
    res = {
        "workload": "kolmogorov_learned_coarse256_from_fine1024_nq8",
        "train_trajectories": len(trs), "fine_steps": c["fine_steps"],
        "sample_every": c["sample_every"], "settle": c["settle"], "horizon": c["horizon"],
        "samples": int(X.shape[0]),
        "generate_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2),
        "loss_first_epoch": round(l0, 5), "loss_last_epoch": round(l1, 5),
        "mlp_train_tflops": round(rows * flops_row / (t2 - t1) / 1e12, 3),
        "eval": [{"seed": cfg["seed"], "Re": round(cfg["Re"], 2), "Wi": round(cfg["Wi"], 3),
                  "err_plain": e["err_plain"][-1], "err_corrected": e["err_corrected"][-1],
                  "gain": e["gain"], "accepted": e["accepted"],
                  "rejected_by_drift_gate": e["rejected_by_drift_gate"]}
                 for cfg, e in zip(held, evals)],
        "accepted": sum(e["accepted"] for e in evals),
        "gain_min": min(e["gain"] for e in evals),
        "coarse_ms_per_step_plain": round(plain_ms, 4),
        "coarse_ms_per_step_corrected": round(corr_ms, 4),
        # fine-lattice node updates the corrected coarse step stands for:
        # 16 fine nodes per coarse node, 4 fine steps per coarse step
        "mlups_equivalent": round(nc * 64 / (corr_ms * 1e-3) / 1e6, 1),
        "fine_fp64_nq8_mlups": round(fine["mlups"], 1),
        "speedup_vs_fine_fp64": round(nc * 64 / (corr_ms * 1e-3) / 1e6 / fine["mlups"], 2),
        "corrected_over_plain_coarse": round(corr_ms / plain_ms, 3),
    }
    print(f"# learned: generate {res['generate_s']} s, train {res['train_s']} s, loss "
          f"{l0:.3f} -> {l1:.3f}, accepted {res['accepted']}/{len(evals)}, gains "
          f"{[round(e['gain'], 2) for e in evals]}, coarse {plain_ms:.3f}/{corr_ms:.3f} ms",
          file=sys.stderr, flush=True)
    mlp.close()
    return res


def copy_ceiling(torch, m, gib=4, reps=10):
    """A plain device-to-device copy of `gib` GiB on the same GPU (read +
    write bytes over its time): the bandwidth a streaming kernel reaches
    here, for context beside the 8 TB/s peak."""
    n = gib << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    achieved = m["bytes_step"] / (m["kernel_ms"] * 1e-3) / 1e9
    return {"copy_ceiling_gbs": round(gbs, 1), "frac_of_copy": round(achieved / gbs, 4)}


def roofline(m, traffic):
    achieved = m["bytes_step"] / (m["kernel_ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic}


def measure_growth(torch, w, pre_steps, steps, every=100):
    """Growth rate of the perturbation amplitude, gamma = d ln A / dn (least
    squares over samples every `every` steps from steps/4 on), of the same
    seeded run stored in FP64, FP32 and BF16 form; the
    storage forms' error is stated against the FP64 run.  The same FP64 run
    with same-step gradients, and with the shifted spring term, shows what
    those readings change."""
    import numpy as np
    import paper_2201_10132_amd as P

    n_fit = steps // 4
    out = {"workload": f"kolmogorov_{w['nx']}x{w['ny']}_nq{w['nq']}", "steps": steps,
           "sample_every": every, "fit_window": [n_fit, steps], "gamma": {}, "amplitude_end": {}}
    runs = (("fp64", P.TPL_FP64, {}), ("fp32", P.TPL_FP32, {}), ("bf16", P.TPL_BF16, {}),
            ("fp64_same_step", P.TPL_FP64, {"gradients": 1}),
            ("fp64_spring_shift", P.TPL_FP64, {"spring_shift": 1}))
    for name, prec, opt in runs:
        t = P.Tpl(w["nx"], w["ny"], w["Re"], w["Wi"], w["beta"], periods=w["periods"],
                  nq=w["nq"], spring=w["spring"], pre_steps=pre_steps, pert_modes=1,
                  precision=prec, **opt)
        t.init(seed=w["seed"], perturbation=w["perturbation"])
        ns, amps = [0], [t.amplitude()]
        t0 = time.perf_counter()
        for n in range(every, steps + 1, every):
            t.step(every)
            ns.append(n)
            amps.append(t.amplitude())
        wall = time.perf_counter() - t0
        t.close()
        ns, amps = np.array(ns), np.array(amps)
        sel = ns >= n_fit
        out["gamma"][name] = float(np.polyfit(ns[sel], np.log(amps[sel]), 1)[0])
        out["amplitude_end"][name] = float(amps[-1])
        print(f"# growth {name}: gamma {out['gamma'][name]:.6e}, A(0) {amps[0]:.4e}, "
              f"A({steps}) {amps[-1]:.4e}, {wall:.1f} s", file=sys.stderr, flush=True)
    g64 = out["gamma"]["fp64"]
    out["gamma_rel_err"] = {k: abs(out["gamma"][k] / g64 - 1) for k in ("fp32", "bf16")}
    out["amplitude_end_rel_err"] = {k: abs(out["amplitude_end"][k] / out["amplitude_end"]["fp64"] - 1)
                                    for k in ("fp32", "bf16")}
    # not an error: another reading of the scheme
    out["same_step_gamma_rel_diff"] = abs(out["gamma"]["fp64_same_step"] / g64 - 1)
    out["spring_shift_gamma_rel_diff"] = abs(out["gamma"]["fp64_spring_shift"] / g64 - 1)
    return out


def measure_inplace(torch, forms, args) -> dict:
    """In-place streaming (one population array): FP64 at 4096^2 and NQ 6
    beside the two-array FP64 run of the same workload, and at NQ 8, which
    only fits one GPU in place (194 GB; two arrays would need 370 GB)."""
    w3 = WORKLOAD_FP32_LARGE
    n3 = max(5, args.steps // 2)
    res = {}
    ref = (forms or {}).get(f"fp64_4096x4096_nq{w3['nq']}")
    for nq in (w3["nq"], 8):
        m = measure(torch, dict(w3, nq=nq), 0, n3, args.warmup, args.pre_steps, inplace=1)
        e = form_entry(m, None)
        e["bytes_state_gb"] = round(m["bytes_state"] / 1e9, 1)
        e["two_array_bytes_state_gb"] = round(
            (m["bytes_state"] + m["nqd"] * 25 * 8 * w3["nx"] * w3["ny"]
             + 9 * 8 * w3["nx"] * w3["ny"]) / 1e9, 1)
        e["tune_ms"] = m["tune_ms"]
        if nq == w3["nq"] and ref is not None:
            e["speed_vs_two_array"] = round(m["mlups"] / ref["mlups"], 3)
        if nq == 8:  # counters of the two alternating kernels, one launch each on average
            tb = [traffic_bytes(os.path.join(ROOT, "profiles", f"k_step_inplace_{k}_fp64_"
                                             "kolmogorov4096_nq8_traffic.txt"))
                  for k in ("pull", "local")]
            if None not in tb:
                e["roofline"]["traffic"] = round(sum(tb) / 2)
        res[f"fp64_4096x4096_nq{nq}"] = e
    return res


def form_entry(m, ref64):
    e = {"mlups": round(m["mlups"], 3), "ms_per_step": round(m["wall_ms"], 4),
         "roofline": roofline(m, None), "conservation": m["conservation"],
         "amplitude": m["amplitude"], "launch": {"qsplit": int(m["qsplit"]), "group": m["group"]}}
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
