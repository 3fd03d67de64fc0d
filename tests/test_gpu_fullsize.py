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
