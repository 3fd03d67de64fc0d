"""Workflow of the learned coarse-lattice correction, driven through the C
ABI: generate training pairs from fine runs, fit the network, and judge a
corrected coarse run against the restricted fine run.

Every lattice and network operation runs in libtpl's kernels (restriction,
features, coarse steps, targets, training passes, corrected steps); this
module only orders the calls, keeps the device buffers (torch tensors) and
computes the bookkeeping statistics: feature and target standardisation
(means and standard deviations) and the evaluation errors.

Coarse lattice: the same Re, Wi, beta and forcing periods on an m-times
coarser grid.  Under acoustic scaling one coarse step covers m fine steps
and the coarse viscosity and relaxation time in lattice units are the fine
ones divided by m, which the library derives from the same Re and Wi.
A training pair at fine step n: the features of the restricted fine state
R(f^n), and the difference between R(f^{n+hm}) and h coarse steps from
R(f^n) in momentum and polymer stress, divided by h: the mean correction
per coarse step over a horizon of h steps (h = 1 is the one-step error; a
longer horizon averages out the acoustic transients that a restricted
state starts with and keeps the part of the error that accumulates).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from .tpl import Mlp, Tpl, TplError, TPL_NFIELDS


def _coarse_like(cfg, factor, nq):
    return Tpl(cfg["nx"] // factor, cfg["ny"] // factor, cfg["Re"], cfg["Wi"], cfg["beta"],
               periods=cfg["periods"], nq=nq, pre_steps=0)


def generate(torch, trajectories, factor=4, nq=8, fine_steps=400, sample_every=40,
             pre_steps=3000, perturbation=1e-2, horizon=None, settle=0, progress=False,
             skipped=None):
    """Training pairs from fine runs.  trajectories: list of dicts with nx, ny,
    Re, Wi, beta, periods, seed.  horizon: coarse steps per target (default
    sample_every / factor).  settle > 0: the coarse run first advances
    `settle` steps from the restricted state (past the acoustic transient a
    restricted state starts with); the features are those of the settled
    coarse state and the target is the growth of its difference from the
    restricted fine run over the next `horizon` steps, per step.  A
    trajectory whose fine or coarse lattice diverges (a relaxation time the
    coarse lattice cannot resolve) contributes no pairs; its seed is appended
    to `skipped` when a list is given.  Returns (X, T) device tensors
    [samples, N_coarse, 54] and [samples, N_coarse, 5] and the fine-step
    time."""
    h = horizon or max(1, sample_every // factor)
    assert (h + settle) * factor <= sample_every
    Xs, Ts = [], []
    t_fine = 0.0
    for cfg in trajectories:
        fine = Tpl(cfg["nx"], cfg["ny"], cfg["Re"], cfg["Wi"], cfg["beta"], periods=cfg["periods"],
                   nq=nq, pre_steps=pre_steps)
        ca, cb = _coarse_like(cfg, factor, nq), _coarse_like(cfg, factor, nq)
        n0 = len(Xs)
        try:
            fine.init(seed=cfg["seed"], perturbation=perturbation)
            ca.init(0, 0.0)
            cb.init(0, 0.0)
            t_fine += _pairs(torch, fine, ca, cb, fine_steps, sample_every, settle, h, factor,
                             Xs, Ts)
        except TplError as e:
            del Xs[n0:], Ts[n0:]
            if skipped is not None:
                skipped.append(cfg["seed"])
            if progress:
                print(f"# trajectory seed {cfg['seed']} skipped: {e}", file=sys.stderr, flush=True)
        for c in (fine, ca, cb):
            c.close()
        if progress:
            print(f"# trajectory seed {cfg['seed']} (Re {cfg['Re']:.1f}, Wi {cfg['Wi']:.2f}): "
                  f"{len(Xs)} pairs so far", file=sys.stderr, flush=True)
    return torch.stack(Xs), torch.stack(Ts), t_fine


def _pairs(torch, fine, ca, cb, fine_steps, sample_every, settle, h, factor, Xs, Ts):
    """One trajectory's training pairs (see generate); returns its fine-step
    time."""
    t_fine = 0.0
    N = ca.nx * ca.ny
    obs_ref = torch.zeros((TPL_NFIELDS, N), dtype=torch.float64, device="cuda")
    for n in range(0, fine_steps, sample_every):
        X = torch.zeros((N, 54), dtype=torch.float32, device="cuda")
        T = torch.zeros((N, 5), dtype=torch.float32, device="cuda")
        ca.restrict_from(fine)
        T0 = None
        if settle:
            ca.step(settle)
            t0 = time.perf_counter()
            fine.step(settle * factor)
            t_fine += time.perf_counter() - t0
            cb.restrict_from(fine)
            cb.moments_device(obs_ref.data_ptr(), obs_ref.numel())
            T0 = torch.zeros_like(T)
            ca.targets_device(obs_ref.data_ptr(), T0.data_ptr(), T0.numel())
        ca.features_device(X.data_ptr(), X.numel())
        ca.step(h)
        t0 = time.perf_counter()
        fine.step(h * factor)
        t_fine += time.perf_counter() - t0
        cb.restrict_from(fine)
        cb.moments_device(obs_ref.data_ptr(), obs_ref.numel())
        ca.targets_device(obs_ref.data_ptr(), T.data_ptr(), T.numel())
        if T0 is not None:
            T -= T0
        T /= h
        Xs.append(X)
        Ts.append(T)
        rest = min(sample_every, fine_steps - n) - (h + settle) * factor
        if rest > 0:
            t0 = time.perf_counter()
            fine.step(rest)
            t_fine += time.perf_counter() - t0
    return t_fine


def standardisation(torch, X, T):
    """Per-feature and per-output mean and standard deviation (FP64 sums)."""
    Xf = X.reshape(-1, X.shape[-1]).double()
    Tf = T.reshape(-1, T.shape[-1]).double()
    xm, xs = Xf.mean(0), Xf.std(0)
    tm, ts = Tf.mean(0), Tf.std(0)
    xs = torch.where(xs > 1e-12 * xm.abs() + 1e-30, xs, torch.ones_like(xs))
    ts = torch.where(ts > 0, ts, torch.ones_like(ts))
    return [v.cpu().numpy() for v in (xm, xs, tm, ts)]


def train(torch, X, T, epochs=40, lr=1e-3, seed=0, mlp=None):
    """Adam over one snapshot (all coarse nodes of one sample) per step,
    snapshots in a seeded random order every epoch.  Returns the network and
    the mean loss of the first and last epoch."""
    S = X.shape[0]
    if mlp is None:
        mlp = Mlp(54, 64, 5, seed=seed)
    mlp.set_norm(*standardisation(torch, X, T))
    rng = np.random.default_rng(seed)
    first = last = None
    for ep in range(epochs):
        order = rng.permutation(S)
        tot = 0.0
        for s in order:
            xs, ts = X[int(s)], T[int(s)]
            tot += mlp.train_step(xs.data_ptr(), ts.data_ptr(), xs.shape[0], lr)
        tot /= S
        first = tot if first is None else first
        last = tot
    return mlp, first, last


def evaluate(torch, mlp, cfg, factor=4, nq=8, fine_steps=400, every=40, pre_steps=3000,
             perturbation=1e-2, drift_bound=0.05):
    """Fine judge vs plain and corrected coarse runs from the same restricted
    initial state.  Errors: relative L2 norm of the coarse mixture velocity
    against the restricted fine one, at every `every` fine steps.  Gate: the
    correction is accepted only if it ends below the plain run's error (a
    gain above 1) and below 5 %, never exceeds twice the plain error at an
    evaluation time, and the runtime drift gate stops no step."""
    fine = Tpl(cfg["nx"], cfg["ny"], cfg["Re"], cfg["Wi"], cfg["beta"], periods=cfg["periods"],
               nq=nq, pre_steps=pre_steps)
    fine.init(seed=cfg["seed"], perturbation=perturbation)
    plain, corr, judge = (_coarse_like(cfg, factor, nq) for _ in range(3))
    for c in (plain, corr, judge):
        c.init(0, 0.0)
    plain.restrict_from(fine)
    corr.restrict_from(fine)
    corr.attach(mlp, drift_bound)

    def uerr(c):
        a, b = c.moments()[1:3], judge.moments()[1:3]
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    e_plain, e_corr, times = [], [], []
    rejected = None
    for n in range(every, fine_steps + 1, every):
        fine.step(every)
        judge.restrict_from(fine)
        try:
            plain.step(every // factor)
        except TplError as e:  # the coarse lattice itself cannot run this case
            corr.attach(None)
            for c in (fine, plain, corr, judge):
                c.close()
            return dict(times=times, err_plain=e_plain, err_corrected=e_corr, gain=0.0,
                        accepted=False, rejected_by_drift_gate=None, coarse_unstable=str(e))
        if rejected is None:
            try:
                corr.step(every // factor)
            except TplError as e:
                rejected = str(e)
        times.append(n)
        e_plain.append(uerr(plain))
        e_corr.append(uerr(corr) if rejected is None else float("nan"))
    ok = (rejected is None and all(c <= 2 * p for c, p in zip(e_corr, e_plain))
          and e_corr[-1] <= 0.05 and e_corr[-1] < e_plain[-1])
    out = dict(times=times, err_plain=e_plain, err_corrected=e_corr,
               gain=(e_plain[-1] / e_corr[-1]) if rejected is None and e_corr[-1] > 0 else 0.0,
               accepted=bool(ok), rejected_by_drift_gate=rejected, coarse_unstable=None)
    corr.attach(None)
    for c in (fine, plain, corr, judge):
        c.close()
    return out


def coarse_step_ms(torch, mlp, cfg, factor=4, nq=8, steps=20, drift_bound=1e30):
    """Mean wall time of a plain and of a corrected coarse step (the drift
    gate is opened: this times the work, not the correction's quality)."""
    c = _coarse_like(cfg, factor, nq)
    c.init(cfg["seed"], 1e-2)
    c.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.step(steps)
    plain = (time.perf_counter() - t0) / steps * 1e3
    c.attach(mlp, drift_bound)
    c.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.step(steps)
    corrected = (time.perf_counter() - t0) / steps * 1e3
    c.attach(None)
    c.close()
    return plain, corrected


def main():
    """The workflow at a chosen scale: python -m paper_2201_10132_amd.learned
    --trajectories 64 --fine-steps 2000 --held-out 16 (training seeds from
    1000, held-out seeds from 2000, parameters drawn as in the plan)."""
    import torch

    from . import inputs

    ap = argparse.ArgumentParser()
    ap.add_argument("--trajectories", type=int, default=64)
    ap.add_argument("--fine-steps", type=int, default=2000)
    ap.add_argument("--held-out", type=int, default=16)
    ap.add_argument("--sample-every", type=int, default=120)
    ap.add_argument("--settle", type=int, default=10)
    ap.add_argument("--horizon", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--pre-steps", type=int, default=3000)
    args = ap.parse_args()
    t0 = time.perf_counter()
    trs = inputs.c5_trajectories(range(1000, 1000 + args.trajectories))
    skipped = []
    X, T, _ = generate(torch, trs, fine_steps=args.fine_steps, sample_every=args.sample_every,
                       settle=args.settle, horizon=args.horizon, pre_steps=args.pre_steps,
                       progress=True, skipped=skipped)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mlp, l0, l1 = train(torch, X, T, epochs=args.epochs)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"# trained on {X.shape[0]} snapshots: loss {l0:.4f} -> {l1:.4f} ({t2 - t1:.1f} s)",
          file=sys.stderr, flush=True)
    del X, T
    rows = []
    for cfg in inputs.c5_trajectories(range(2000, 2000 + args.held_out)):
        e = evaluate(torch, mlp, cfg, pre_steps=args.pre_steps)
        rows.append(dict(seed=cfg["seed"], Re=round(cfg["Re"], 2), Wi=round(cfg["Wi"], 3),
                         err_plain=e["err_plain"][-1], err_corrected=e["err_corrected"][-1],
                         gain=e["gain"], accepted=e["accepted"],
                         rejected_by_drift_gate=e["rejected_by_drift_gate"],
                         coarse_unstable=e["coarse_unstable"]))
        print(f"# held-out seed {cfg['seed']}: gain {e['gain']:.2f} accepted {e['accepted']}"
              f"{' (plain coarse run diverges)' if e['coarse_unstable'] else ''}",
              file=sys.stderr, flush=True)
    mlp.close()
    judged = [r for r in rows if not r["coarse_unstable"]]
    gains = [r["gain"] for r in judged] or [0.0]
    print(json.dumps(dict(trajectories=args.trajectories, skipped_trajectories=skipped,
                          coarse_unstable_held_out=[r["seed"] for r in rows if r["coarse_unstable"]],
                          fine_steps=args.fine_steps,
                          sample_every=args.sample_every, settle=args.settle,
                          horizon=args.horizon, generate_s=round(t1 - t0, 1),
                          train_s=round(t2 - t1, 2), loss=[l0, l1],
                          accepted=sum(r["accepted"] for r in judged), judged=len(judged),
                          held_out=len(rows),
                          gain_min=min(gains), gain_median=float(np.median(gains)),
                          eval=rows)), flush=True)


if __name__ == "__main__":
    main()
