"""Parity at the 1024 x 1024, NQ = 16 workload size, in the launch
configuration the benchmark uses (automatic Q-split, XCD tile mapping).

The oracle cannot step 1024^2 x 208 Q-nodes in a test, so it recomputes
sampled nodes one by one: the GPU's state in the 3 x 3 window around a node
(populations, lagged psi and U) is loaded into a 3 x 3 periodic oracle
lattice with the full lattice's parameters and forcing phase; one oracle step
then gives the exact update of the window's centre (its pull stencil, lagged
gradients and spring term only reach the window).  Conservation is checked
on the whole lattice.
"""
import numpy as np
import pytest

import oracle
import paper_2201_10132_amd as P
from tests.gpu_common import FLOOR, max_rel

pytestmark = pytest.mark.gpu

NX = NY = 1024
PARAMS = dict(Re=60.0, Wi=1.0, beta=0.7, periods=4)
SAMPLES = [(0, 0), (1023, 1023), (511, 300), (17, 1000), (800, 2), (64, 511)]


def test_fullsize_sampled_node_parity_and_conservation():
    print("fullsize: init 1024x1024 nq=16", flush=True)
    t = P.Tpl(NX, NY, PARAMS["Re"], PARAMS["Wi"], PARAMS["beta"], periods=PARAMS["periods"],
              nq=16, pre_steps=200, pert_modes=1)
    t.init(seed=0, perturbation=1e-4)
    t.step(2)  # a state whose lagged fields come from the kernel itself
    d0 = t.diagnostics()
    wins = {s: t.get_window(s[0] - 1, s[1] - 1, 3, 3) for s in SAMPLES}
    t.step(1)
    d1 = t.diagnostics()
    for (x, y), w in wins.items():
        print(f"fullsize: node ({x},{y})", flush=True)
        o = oracle.OracleSim(3, 3, nq=16, ny_param=NY, y_offset=y - 1, **PARAMS)
        o.set_state(XS=w["XS"], XP=w["XP"], psi=w["psi"], U=w["U"])
        o.step(1)
        want = o.get_state()
        got = t.get_window(x, y, 1, 1)
        for k in ("XS", "XP", "psi", "U"):
            assert max_rel(got[k][..., 0, 0], want[k][..., 1, 1], FLOOR[k]) < 1e-14, (k, x, y)
    assert abs(d1["mass_S"] / d0["mass_S"] - 1) < 1e-13
    assert abs(d1["mass_P"] / d0["mass_P"] - 1) < 1e-13
    scale = d0["mass_S"] * 0.05
    assert abs(d1["mom_x"] - d0["mom_x"]) < 1e-13 * scale
    assert abs(d1["mom_y"] - d0["mom_y"]) < 1e-13 * scale
    t.close()


def test_fullsize_nq4_whole_lattice_parity():
    """The whole 1024 x 1024 lattice at NQ = 4 (12 Q-nodes, so that the
    oracle holds it): init (base state, multimode perturbation) and 10 steps
    in the library's default launch configuration, every population, psi
    and U against the oracle (tolerances of the plain parity tests)."""
    from tests.gpu_common import compare_states

    print("fullsize nq4: library init", flush=True)
    t = P.Tpl(NX, NY, PARAMS["Re"], PARAMS["Wi"], PARAMS["beta"], periods=PARAMS["periods"],
              nq=4, pre_steps=100, pert_modes=1)
    t.init(seed=0, perturbation=1e-4)
    print("fullsize nq4: oracle init", flush=True)
    o = oracle.OracleSim(NX, NY, nq=4, **PARAMS)
    o.base_state(100)
    o.perturb(0, 1e-4, True)
    compare_states(t.get_state(), o.get_state(), 1e-13)
    t.step(10)
    print(f"fullsize nq4: 10 steps (qsplit {t.query('qsplit_used'):.0f}, group "
          f"{t.query('group_x_used'):.0f}x{t.query('group_y_used'):.0f}), oracle", flush=True)
    o.step(10)
    errs = compare_states(t.get_state(), o.get_state(), 1e-13)
    print("fullsize nq4 errors", errs, flush=True)
    assert max_rel(t.moments(), o.observables()) < 1e-13
    t.close()


@pytest.mark.parametrize("precision", [P.TPL_BF16, P.TPL_FP32], ids=["bf16", "fp32"])
def test_fullsize_reduced_precision_sampled_node_parity(precision):
    """The BF16 and FP32 forms at the same size and launch configuration.  The oracle
    steps the decoded 3 x 3 window exactly in FP64; the GPU's stored result
    differs from it by the storage rounding of the outputs: at most 2^-8 of
    a polymer population's deviation from the base state (the rest
    population 24 such roundings, the residual it takes up), 2^-24 of the
    solvent's and psi's; the mixture velocity by the rounding of the ~25 nqd
    / 9 stored polymer populations behind each of its Q-marginals (the kernel
    takes the marginals before rounding), and every population's
    equilibrium by that velocity difference.  The FP32 form rounds every
    population to 2^-24 of its deviation and has no residual to carry.
    Tested with a factor 4 margin; the deviations are measured against the
    base state of a one-column context with the same parameters."""
    bf16 = precision == P.TPL_BF16
    eps32 = 2.0 ** -24
    eps16 = 2.0 ** -8 if bf16 else eps32  # the polymer populations' unit roundoff
    rest_terms = 24 if bf16 else 1
    tag = "bf16" if bf16 else "fp32"
    print(f"fullsize {tag}: init 1024x1024 nq=16", flush=True)
    t = P.Tpl(NX, NY, PARAMS["Re"], PARAMS["Wi"], PARAMS["beta"], periods=PARAMS["periods"],
              nq=16, pre_steps=200, pert_modes=1, precision=precision)
    t.init(seed=0, perturbation=1e-4)
    t.step(2)
    base = P.Tpl(1, NY, PARAMS["Re"], PARAMS["Wi"], PARAMS["beta"], periods=PARAMS["periods"],
                 nq=16, pre_steps=200, pert_modes=1)
    base.init(seed=0, perturbation=0.0)
    nqd = t.nqd
    dP_seen = []
    d0 = t.diagnostics()
    wins = {s: t.get_window(s[0] - 1, s[1] - 1, 3, 3) for s in SAMPLES}
    t.step(1)
    d1 = t.diagnostics()
    for (x, y), w in wins.items():
        print(f"fullsize {tag}: node ({x},{y})", flush=True)
        ref = base.get_window(0, y - 1, 1, 3)  # the base state of the window's rows
        dP = max(float(np.abs(w["XP"][..., j, :] - ref["XP"][..., j, :1]).max()) for j in range(3))
        dS = max(float(np.abs(w[k][..., j, :] - ref[k][..., j, :1]).max())
                 for k in ("XS", "psi") for j in range(3))
        dP_seen.append(dP)
        o = oracle.OracleSim(3, 3, nq=16, ny_param=NY, y_offset=y - 1, **PARAMS)
        o.set_state(XS=w["XS"], XP=w["XP"], psi=w["psi"], U=w["U"])
        o.step(1)
        want = o.get_state()
        got = t.get_window(x, y, 1, 1)
        g, v = (lambda k: got[k][..., 0, 0]), (lambda k: want[k][..., 1, 1])
        fp64 = lambda k: 1e-13 * float(np.abs(v(k)).max())
        # the mixture velocity, and through the equilibria every population
        # (d f_eq / d U is at most about 3 rho w |c| < 2 rho); psi is the
        # node's pulled density, which no equilibrium changes
        dU = 4 * (25 * nqd / 9) * eps16 * dP + 1e-14
        psi_max = float(np.abs(v("psi")).max())
        bounds = {"XS": 4 * eps32 * dS + 2 * dU + fp64("XS"),
                  "psi": 4 * eps32 * dS + fp64("psi"),
                  "XP moving": 4 * eps16 * dP + 2 * psi_max * dU + fp64("XP"),
                  "XP rest": 4 * rest_terms * eps16 * dP + 2 * psi_max * dU + fp64("XP"),
                  "U": dU}
        errs = {"XS": float(np.abs(g("XS") - v("XS")).max()),
                "psi": float(np.abs(g("psi") - v("psi")).max()),
                "XP moving": float(np.abs(g("XP")[1:] - v("XP")[1:]).max()),
                "XP rest": float(np.abs(g("XP")[0] - v("XP")[0]).max()),
                "U": float(np.abs(g("U") - v("U")).max())}
        print(f"  dP {dP:.3e} dS {dS:.3e} errors {errs}", flush=True)
        for k, e in errs.items():
            assert e <= bounds[k], (k, e, bounds[k], x, y)
    # mass to FP32: in the BF16 form the rest population takes up the node's
    # rounding residual, so one step moves the polymer mass by at most one
    # FP32 rounding of every rest population (BF16 rounding of all 25
    # populations would allow 25 * 2^16 times as much); the FP32 form rounds
    # all 25
    dP_all = max(dP_seen)
    mass_bound = (1 if bf16 else 25) * NX * NY * nqd * eps32 * dP_all / d0["mass_P"]
    print(f"mass drift S {d1['mass_S'] / d0['mass_S'] - 1:.3e} P "
          f"{d1['mass_P'] / d0['mass_P'] - 1:.3e} (bound {mass_bound:.3e})", flush=True)
    assert abs(d1["mass_S"] / d0["mass_S"] - 1) < 1e-12
    assert abs(d1["mass_P"] / d0["mass_P"] - 1) <= mass_bound
    base.close()
    t.close()
