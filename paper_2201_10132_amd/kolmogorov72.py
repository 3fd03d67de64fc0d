"""The paper's own viscoelastic Kolmogorov-flow experiment (Sec. VII),
driven through the C ABI: a 72 x 72 periodic cell holding four forcing
periods (l = 72 / 8 pi lattice units), Re = 3.5, beta = 0.5, FENE dumbbells
with b = 25 on a 32-point Q-grid, Wi = 0.1, 2.5 and 5, started from rest
with a seeded multimode perturbation and run to t = 2000 convective times
(t = n u0 / l).  The three Weissenberg numbers run as one batch.

What the paper reports, and what `summary` measures for each Wi: the
enstrophy first rises to the plateau of the laminar sinusoidal profile; the
inflectional instability then lowers it (early for Wi = 0.1, delayed and
slightly weaker for Wi = 2.5, not at all for Wi = 5); the RMS polymer
extension stays near the equilibrium value for Wi = 0.1 and reaches about
twice that for Wi = 5.  The paper's figures are not part of its text, so
these are qualitative checks.

Each cell is forced so that its laminar profile has amplitude u0
(calibrate_force): Re = U l / nu is defined with the amplitude U of the
laminar flow.  With F0 = nu u0 k^2 instead (--force-from-nu) the lattice
polymer's stress diffusion and the FENE shear thinning drive the elastic
cells faster than u0, which raises their effective Re with Wi.

With --spring-shift the spring term is the shift itself, psi at the two
beads r +- Q/2, instead of its first-order Taylor form: the dumbbells here
span a sizeable part of the forcing wavelength (sigma k = 1.1), where the
two differ.  Options the batched step does not take (the component-stress
quasi-equilibria, qe_model 2) run the three cells as separate contexts.

With --n N the cell has N x N nodes instead of 72 x 72, with the same four
periods and parameters: the dumbbells (sigma = 3.2 nodes on the 32-point
Q-grid) then span less of the forcing wavelength, sigma k = 1.1 x 72 / N,
as if the Q-grid spacing were 72 / N of the r-spacing.

Usage: python -m paper_2201_10132_amd.kolmogorov72 [--t-end 2000] [--spring-shift]
       [--force-from-nu] [--drag shared] [--n 72] [--out file.json]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from .tpl import TPL_FP64, Batch, Tpl, TplError

# u0 = 0.01: the lattice velocity scale is not given for this experiment; at
# 0.05 the Wi = 0.1 relaxation time would span 5.7 steps (tau2_P = 2.7) and
# the run diverges within two convective times, at 0.01 it spans 29 steps
CELL = dict(nx=72, ny=72, periods=4, Re=3.5, beta=0.5, u0=0.01)
WIS = (0.1, 2.5, 5.0)
# Cap on the Q-drift D_Q |F/kT| per step (the library's default, 0.2).  At
# Wi = 0.1 (tau2_P = 0.54) a cap of 0.1 would already bind two sigma out,
# where the FENE rest distribution is 11 % of its peak, and the rest
# extension would settle 18 % above the FENE value; at 0.2 it is within 1 %,
# and the linear Q-space equilibrium stays positive (drift below c_s^2 = 1/3
# per step, with room for the flow term).  The elastic cells (tau2_P <= 0.02)
# do not reach it.
DRIFT_CAP = 0.2


class _Cells:
    """The cells as separate contexts, with the calls of Batch that run() uses
    (for options the batched step does not take)."""

    def __init__(self, insts, precision, nq, pre_steps, **params):
        self.spec = insts
        self.cells = [Tpl(d["nx"], d["ny"], d["Re"], d["Wi"], d["beta"], periods=d["periods"],
                          u0=d["u0"], nq=nq, pre_steps=pre_steps, precision=precision, **params)
                      for d in insts]
        self.bad = [0] * len(insts)

    def init(self):
        for t, d in zip(self.cells, self.spec):
            t.init(seed=d["seed"], perturbation=d["perturbation"])

    def step(self, n):
        for i, t in enumerate(self.cells):
            if not self.bad[i]:
                try:
                    t.step(n)
                except TplError:
                    self.bad[i] = 1

    def status(self):
        return list(self.bad)

    def instance(self, i):
        return self.cells[i]

    def close(self):
        for t in self.cells:
            t.close()


def convective_steps(u0=CELL["u0"]):
    """Lattice steps per convective time l / u0."""
    l = CELL["ny"] / (2 * math.pi * CELL["periods"])
    return l / u0


def laminar_amplitude(t):
    """Amplitude of the sin(k y) component of the x-averaged U_x over u0."""
    m = t.moments()
    ny = m.shape[1]
    y = np.arange(ny)
    k = 2.0 * math.pi * CELL["periods"] / ny
    return 2.0 / ny * float(np.sum(m[1].mean(axis=1) * np.sin(k * y))) / CELL["u0"]


def calibrate_force(Wi, nq=32, iters=4, **params):
    """Force scale at which the laminar profile's amplitude is u0.

    Sec. VII defines Re = U l / nu with U the amplitude of the laminar flow
    the force induces, and F = eta U / l^2 as that force for a fluid of
    viscosity eta.  On the lattice the polymer's stress also diffuses in r
    (its r- and Q-diffusivities are tied), and FENE dumbbells thin in shear,
    so F0 = nu u0 k^2 drives a laminar flow faster than u0 (1.3 u0 at
    Wi = 5 on a 16-point Q-grid): the effective Re grows with Wi.  This
    scales F0 until the forced x-invariant state (the column pre-run,
    5 max(l^2/nu, lambda) steps, through the C ABI) has amplitude u0."""
    fs = 1.0
    for _ in range(iters):
        t = Tpl(1, CELL["ny"], CELL["Re"], Wi, CELL["beta"], periods=CELL["periods"],
                u0=CELL["u0"], nq=nq, pre_steps=-1, force_scale=fs,
                **{"drift_cap": DRIFT_CAP, **params})
        t.init(seed=0, perturbation=0.0)
        a = laminar_amplitude(t)
        t.close()
        fs /= a
    return fs


def shared_drag_time(Wi, nq=32, **params):
    """The solvent's drag time under the reading that both components share
    one drag time (Sec. V writes the momentum exchange between solvent and
    polymer with a single tau_2): the polymer's tau2_P, raised to the
    solvent's viscous time tau1_S where the ordering tau_1 <= tau_2 (needed
    for the H-theorem) requires it.  The library's own default is 1, which
    with phi = 0.01 adds phi c_s^2 to the polymer's r-diffusivity (about as
    much again as its own c_s^2 tau2_P in the elastic cells)."""
    t = Tpl(1, CELL["ny"], CELL["Re"], Wi, CELL["beta"], periods=CELL["periods"],
            u0=CELL["u0"], nq=nq, **params)
    v = max(t.query("tau1S"), t.query("tau2P"))
    t.close()
    return v


def run(t_end=2000.0, every=1.0, wis=WIS, nq=32, seed=0, perturbation=1e-3,
        precision=TPL_FP64, progress=True, laminar_u0=True, shared_drag=False, **params):
    """Advance the three cells together; sample the diagnostics every
    `every` convective times.  laminar_u0: force each cell so that its
    laminar amplitude is u0 (calibrate_force); else F0 = nu u0 k^2.  Returns
    dict(t, enstrophy[w], qrms[w], amplitude[w], unstable[w],
    force_scale[w])."""
    insts = [dict(CELL, Wi=w, seed=seed, perturbation=perturbation) for w in wis]
    cls = _Cells if params.get("qe_model", 1) != 1 else Batch
    params = {"drift_cap": DRIFT_CAP, **params}
    drag = [shared_drag_time(w, nq=nq, **params) if shared_drag else None for w in wis]
    fscale = [calibrate_force(w, nq=nq, **params, **({"tau_drag": d} if d else {}))
              if laminar_u0 else 1.0 for w, d in zip(wis, drag)]
    b = cls(insts, precision=precision, nq=nq, pre_steps=0, **params)
    for i, f in enumerate(fscale):
        b.instance(i).set_param("force_scale", f)
        if drag[i]:
            b.instance(i).set_param("tau_drag", drag[i])
    b.init()
    tc = convective_steps()
    out = dict(t=[], enstrophy=[[] for _ in wis], qrms=[[] for _ in wis],
               amplitude=[[] for _ in wis], steps_per_convective_time=tc, force_scale=fscale,
               tau_drag=[d if d else b.instance(i).query("tau2S") for i, d in enumerate(drag)])
    n_done = 0
    t0 = last = time.perf_counter()
    k = 0
    while True:
        t = k * every
        n_target = int(round(t * tc))
        if n_target > n_done:
            b.step(n_target - n_done)
            n_done = n_target
        out["t"].append(n_done / tc)
        status = b.status()
        for i in range(len(wis)):
            if status[i]:
                d = dict(enstrophy=float("nan"), qrms=float("nan"), amplitude=float("nan"))
            else:
                d = b.instance(i).diagnostics()
            out["enstrophy"][i].append(d["enstrophy"])
            out["qrms"][i].append(d["qrms"])
            out["amplitude"][i].append(d["amplitude"])
        if progress and (k % max(1, int(100 / every)) == 0 or time.perf_counter() - last > 30.0):
            last = time.perf_counter()
            print(f"# t = {n_done / tc:7.1f} ({n_done} steps, {time.perf_counter() - t0:6.1f} s): "
                  + "  ".join(f"Wi {w}: E {out['enstrophy'][i][-1]:.4e} Qrms {out['qrms'][i][-1]:.3f}"
                              for i, w in enumerate(wis)), file=sys.stderr, flush=True)
        if t >= t_end:
            break
        k += 1
    out["unstable"] = [bool(u) for u in b.status()]
    out["wall_s"] = time.perf_counter() - t0
    out["steps"] = n_done
    out["lattice_updates_per_s"] = len(wis) * CELL["nx"] * CELL["ny"] * n_done / out["wall_s"]
    b.close()
    return out


def summary(res, wis=WIS, drop=0.05):
    """Per Wi: the laminar plateau (largest enstrophy), the onset time of the
    instability (first time after the plateau at which the enstrophy has
    fallen by `drop`), the final enstrophy relative to the plateau, and the
    mean RMS extension over the last fifth of the run."""
    t = np.asarray(res["t"])
    rows = []
    for i, w in enumerate(wis):
        E = np.asarray(res["enstrophy"][i])
        Q = np.asarray(res["qrms"][i])
        j = int(np.nanargmax(E))
        below = np.nonzero(E[j:] < (1 - drop) * E[j])[0]
        tail = (t >= 0.8 * t[-1]) & np.isfinite(Q)
        rows.append(dict(Wi=w, plateau=float(E[j]), t_plateau=float(t[j]),
                         t_onset=float(t[j + below[0]]) if below.size else None,
                         final_over_plateau=float(E[-1] / E[j]),
                         qrms_tail=float(Q[tail].mean()) if tail.any() else None,
                         amplitude_end=float(res["amplitude"][i][-1]),
                         unstable=res["unstable"][i]))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--t-end", type=float, default=2000.0)
    ap.add_argument("--every", type=float, default=1.0)
    ap.add_argument("--nq", type=int, default=32)
    ap.add_argument("--out", default=None)
    ap.add_argument("--perturbation", type=float, default=1e-3)
    ap.add_argument("--spring-shift", action="store_true",
                    help="psi at the beads instead of the Taylor form of the spring term")
    ap.add_argument("--drift-cap", type=float, default=DRIFT_CAP,
                    help="cap on the Q-drift per step (0: none)")
    ap.add_argument("--n", type=int, default=CELL["nx"], help="nodes per side of the cell")
    ap.add_argument("--drag", choices=["library", "shared"], default="library",
                    help="solvent drag time: the library's (1) or the polymer's tau2_P "
                         "(at least tau1_S): one drag time for both components")
    ap.add_argument("--force-from-nu", action="store_true",
                    help="F0 = nu u0 k^2 for every cell instead of the force that makes the "
                         "laminar amplitude u0")
    args = ap.parse_args()
    CELL["nx"] = CELL["ny"] = args.n
    extra = dict(spring_shift=1) if args.spring_shift else {}
    extra["drift_cap"] = args.drift_cap
    res = run(t_end=args.t_end, every=args.every, nq=args.nq, perturbation=args.perturbation,
              laminar_u0=not args.force_from_nu, shared_drag=args.drag == "shared", **extra)
    rows = summary(res)
    line = dict(experiment="kolmogorov_%dx%d_re3.5_beta0.5_fene_nq%d%s%s%s"
                % (args.n, args.n, args.nq, "_shifted_spring" if args.spring_shift else "",
                   "_force_from_nu" if args.force_from_nu else "",
                   "_shared_drag" if args.drag == "shared" else ""), u0=CELL["u0"],
                drift_cap=args.drift_cap, force_scale=res["force_scale"],
                tau_drag=res["tau_drag"],
                steps=res["steps"], wall_s=round(res["wall_s"], 1),
                lattice_updates_per_s=res["lattice_updates_per_s"], summary=rows)
    print(json.dumps(line), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(dict(line, series=res), fh)


if __name__ == "__main__":
    main()
