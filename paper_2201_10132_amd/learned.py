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

import time

import numpy as np

from .tpl import Mlp, Tpl, TplError, TPL_NFIELDS


def _coarse_like(cfg, factor, nq):
    return Tpl(cfg["nx"] // factor, cfg["ny"] // factor, cfg["Re"], cfg["Wi"], cfg["beta"],
               periods=cfg["periods"], nq=nq, pre_steps=0)


def generate(torch, trajectories, factor=4, nq=8, fine_steps=400, sample_every=40,
             pre_steps=3000, perturbation=1e-2, horizon=None, settle=0):
    """Training pairs from fine runs.  trajectories: list of dicts with nx, ny,
    Re, Wi, beta, periods, seed.  horizon: coarse steps per target (default
    sample_every / factor).  settle > 0: the coarse run first advances
    `settle` steps from the restricted state (past the acoustic transient a
    restricted state starts with); the features are those of the settled
    coarse state and the target is the growth of its difference from the
    restricted fine run over the next `horizon` steps, per step.  Returns
    (X, T) device tensors [samples, N_coarse, 54] and [samples, N_coarse, 5]
    and the fine-step time."""
    h = horizon or max(1, sample_every // factor)
    assert (h + settle) * factor <= sample_every
    Xs, Ts = [], []
    t_fine = 0.0
    for cfg in trajectories:
        fine = Tpl(cfg["nx"], cfg["ny"], cfg["Re"], cfg["Wi"], cfg["beta"], periods=cfg["periods"],
                   nq=nq, pre_steps=pre_steps)
        fine.init(seed=cfg["seed"], perturbation=perturbation)
        ca, cb = _coarse_like(cfg, factor, nq), _coarse_like(cfg, factor, nq)
        ca.init(0, 0.0)
        cb.init(0, 0.0)
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
        for c in (fine, ca, cb):
            c.close()
    return torch.stack(Xs), torch.stack(Ts), t_fine


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
    correction is rejected if its error exceeds twice the plain error at any
    evaluation time, or 5 % at the end, or if the runtime drift gate stops a
    step."""
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
        plain.step(every // factor)
        if rejected is None:
            try:
                corr.step(every // factor)
            except TplError as e:
                rejected = str(e)
        times.append(n)
        e_plain.append(uerr(plain))
        e_corr.append(uerr(corr) if rejected is None else float("nan"))
    ok = rejected is None and all(c <= 2 * p for c, p in zip(e_corr, e_plain)) and e_corr[-1] <= 0.05
    out = dict(times=times, err_plain=e_plain, err_corrected=e_corr,
               gain=(e_plain[-1] / e_corr[-1]) if rejected is None and e_corr[-1] > 0 else 0.0,
               accepted=bool(ok), rejected_by_drift_gate=rejected)
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
