"""Long runs of the perturbed Kolmogorov flow that track the perturbation
amplitude A(n) (RMS of U minus its row mean, over u0) and fit its growth or
decay rate gamma = d ln A / dn, driven through the C ABI.

  stability   one forcing period on 256^2 with the parameters of the 1024^2
              workloads (Re 60, Wi 1, beta 0.7): does the scheme stay finite
              for `steps` steps at a given NQ?
  c2          1024^2, four periods, Re 60, beta 0.7, Wi in {0, 1}, FP64,
              multimode perturbation 1e-4 u0 (seed 0, or --seeds), A(n) over
              `steps` steps; gamma fitted from step 1000 to the first step
              with A > 1e-2 (or the end).
  c3          4096^2, sixteen periods, Re 60, Wi 1, beta 0.7: the same seeded
              run stored in FP64, FP32 and BF16; gamma and A(n) of the two
              reduced forms against FP64 (NQ 6: the largest Q-grid at which
              the FP64 state, two halves of 230 GB, fits one GPU).
  c4          the batched sweep: 256 seeded instances (sizes from
              {128, ..., 512}^2, Re, Wi, beta drawn per instance), FP32, NQ 6,
              one batch: A(n) of every instance every `every` steps, its
              growth rate fitted from step 1000 (to the first step with
              A > 1e-2), and the instances flagged unstable.

Usage: python -m paper_2201_10132_amd.growth_runs {stability,c2,c3,c4} [--steps N] [--nq Q]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import inputs
from .tpl import TPL_BF16, TPL_FP32, TPL_FP64, Batch, Tpl, TplError


def track(nx, ny, periods, Wi, nq, precision, steps, every, pre_steps=3000, perturbation=1e-4,
          Re=60.0, beta=0.7, seed=0, tag=""):
    t = Tpl(nx, ny, Re, Wi, beta, periods=periods, nq=nq, pre_steps=pre_steps, pert_modes=1,
            precision=precision)
    t0 = time.perf_counter()
    t.init(seed=seed, perturbation=perturbation)
    ns, amps = [0], [t.amplitude()]
    d0 = t.diagnostics()
    failed = None
    n = 0
    last = time.perf_counter()
    try:
        while n < steps:
            k = min(every, steps - n)
            t.step(k)
            n += k
            ns.append(n)
            amps.append(t.amplitude())
            if time.perf_counter() - last >= 20.0 or n >= steps:  # a line at least every ~20 s
                last = time.perf_counter()
                print(f"# {tag} step {n}: A {amps[-1]:.4e} ({last - t0:.0f} s)",
                      file=sys.stderr, flush=True)
    except TplError as e:
        failed = f"step {n}: {e}"
    d1 = t.diagnostics() if failed is None else None
    wall = time.perf_counter() - t0
    t.close()
    out = dict(n=ns, A=amps, failed=failed, wall_s=wall,
               mass_S=None if d1 is None else abs(d1["mass_S"] / d0["mass_S"] - 1),
               mass_P=None if d1 is None else abs(d1["mass_P"] / d0["mass_P"] - 1))
    return out


def fit_gamma(n, A, start, stop_amp=1e-2):
    n, A = np.asarray(n, dtype=float), np.asarray(A, dtype=float)
    end = n[-1]
    big = np.nonzero((n >= start) & (A > stop_amp))[0]
    if big.size:
        end = n[big[0]]
    sel = (n >= start) & (n <= end) & np.isfinite(A)
    if sel.sum() < 3:
        return None, [start, end]
    return float(np.polyfit(n[sel], np.log(A[sel]), 1)[0]), [float(start), float(end)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["stability", "c2", "c3", "c4"])
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--nq", type=int, default=None)
    ap.add_argument("--every", type=int, default=None)
    ap.add_argument("--pre-steps", type=int, default=3000,
                    help="base-state column steps (-1: the library's 5 max(l^2/nu, lambda))")
    ap.add_argument("--seeds", type=int, nargs="+", default=[0],
                    help="c2: perturbation seeds (one run per seed and Wi)")
    ap.add_argument("--wis", type=float, nargs="+", default=[0.0, 1.0], help="c2: Weissenberg numbers")
    args = ap.parse_args()
    res = dict(run=args.what)
    if args.what == "stability":
        steps, nq, every = args.steps or 20000, args.nq or 6, args.every or 1000
        r = track(256, 256, 1, 1.0, nq, TPL_FP64, steps, every, pre_steps=args.pre_steps,
                  tag=f"stability nq{nq}")
        res.update(nq=nq, steps=steps, failed=r["failed"], A_end=r["A"][-1],
                   mass_S=r["mass_S"], mass_P=r["mass_P"], wall_s=round(r["wall_s"], 1))
    elif args.what == "c2":
        steps, nq, every = args.steps or 20000, args.nq or 16, args.every or 250
        res.update(nq=nq, steps=steps, pre_steps=args.pre_steps, cases=[])
        for seed, Wi in [(s, w) for s in args.seeds for w in args.wis]:
            r = track(1024, 1024, 4, Wi, nq, TPL_FP64, steps, every, pre_steps=args.pre_steps,
                      seed=seed, tag=f"c2 Wi {Wi} seed {seed}")
            g, win = fit_gamma(r["n"], r["A"], 1000)
            res["cases"].append(dict(Wi=Wi, seed=seed, gamma=g, fit_window=win, A_end=r["A"][-1],
                                     A_max=float(np.nanmax(r["A"])), failed=r["failed"],
                                     mass_S=r["mass_S"], mass_P=r["mass_P"],
                                     ms_per_step=round(r["wall_s"] / max(1, steps) * 1e3, 3),
                                     n=r["n"][::8], A=r["A"][::8]))
    elif args.what == "c4":
        steps, nq, every = args.steps or 5000, args.nq or 6, args.every or 250
        insts = inputs.c4_instances(256)
        b = Batch(insts, precision=TPL_FP32, nq=nq, pre_steps=args.pre_steps)
        t0 = time.perf_counter()
        b.init()
        ns, A = [0], [list(b.amplitudes())]
        n = 0
        while n < steps:
            k = min(every, steps - n)
            b.step(k)
            n += k
            ns.append(n)
            A.append(list(b.amplitudes()))
            print(f"# c4 step {n}: {int(b.query('unstable'))} unstable ({time.perf_counter() - t0:.0f} s)",
                  file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
        status = list(b.status())
        A = np.array(A)  # [samples][instances]
        cases = []
        for i, d in enumerate(insts):
            g, win = fit_gamma(ns, A[:, i], 1000) if not status[i] else (None, None)
            cases.append(dict(i=i, nx=d["nx"], ny=d["ny"], Re=round(d["Re"], 3), Wi=round(d["Wi"], 4),
                              beta=round(d["beta"], 4), unstable=bool(status[i]), gamma=g,
                              fit_window=win, A_end=None if status[i] else float(A[-1, i])))
        gs = sorted(c["gamma"] for c in cases if c["gamma"] is not None)
        res.update(nq=nq, steps=steps, pre_steps=args.pre_steps, every=every,
                   nodes=int(b.query("nodes")), wall_s=round(wall, 1),
                   unstable=[c["i"] for c in cases if c["unstable"]],
                   growing=sum(1 for g in gs if g > 0), decaying=sum(1 for g in gs if g <= 0),
                   gamma_quartiles=[gs[len(gs) // 4], gs[len(gs) // 2], gs[3 * len(gs) // 4]] if gs else None,
                   cases=cases)
        b.close()
    else:
        steps, nq, every = args.steps or 2000, args.nq or 6, args.every or 100
        res.update(nq=nq, steps=steps, forms={})
        for name, prec in (("fp64", TPL_FP64), ("fp32", TPL_FP32), ("bf16", TPL_BF16)):
            r = track(4096, 4096, 16, 1.0, nq, prec, steps, every, pre_steps=args.pre_steps,
                      tag=f"c3 {name}")
            g, win = fit_gamma(r["n"], r["A"], steps // 4)
            res["forms"][name] = dict(gamma=g, fit_window=win, A=r["A"], failed=r["failed"],
                                      mass_S=r["mass_S"], mass_P=r["mass_P"],
                                      ms_per_step=round(r["wall_s"] / max(1, steps) * 1e3, 2))
        ref = res["forms"]["fp64"]
        for name in ("fp32", "bf16"):
            f = res["forms"][name]
            if f["gamma"] is not None and ref["gamma"] is not None:
                f["gamma_rel_err"] = abs(f["gamma"] / ref["gamma"] - 1)
            a, b = np.asarray(f["A"]), np.asarray(ref["A"])
            f["A_max_rel_err"] = float(np.nanmax(np.abs(a / b - 1)))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
