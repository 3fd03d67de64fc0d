"""Degenerate and extreme configurations against the FP64 oracle, through
init (base-state column run, tiling, seeded perturbation) and 20 steps:

* beta = 1: no polymer viscosity, so the spring coefficient vanishes and the
  polymer is a passive tracer advected by the solvent;
* a single-column lattice (nx = 1): every x-neighbour is the node itself;
* the largest Q-grid the library accepts (NQ 48, 1804 Q-nodes per r-node);
* Wi = 0 at the smallest NQ (4) on a lattice whose node count is not a
  multiple of the 64-node tile;
* the smallest lattice height for its periods (ny = 4 periods);
and zero-step calls, which must leave the state untouched.  Tolerances as
for the plain parity tests (1e-12 after init and 20 steps, FP64).
"""
import numpy as np
import pytest

from tests.gpu_common import compare_states, make_pair, max_rel

pytestmark = pytest.mark.gpu

EDGES = [
    dict(nx=8, ny=4, Re=20.0, Wi=0.5, beta=1.0, periods=1, nq=6),
    dict(nx=1, ny=8, Re=20.0, Wi=0.5, beta=0.7, periods=2, nq=6),
    dict(nx=8, ny=4, Re=20.0, Wi=0.5, beta=0.7, periods=1, nq=48),
    dict(nx=13, ny=5, Re=12.0, Wi=0.0, beta=0.9, periods=1, nq=4),
    dict(nx=16, ny=12, Re=35.0, Wi=1.2, beta=0.6, periods=3, nq=8),
]


@pytest.mark.parametrize("case", EDGES,
                         ids=lambda c: f"{c['nx']}x{c['ny']}q{c['nq']}b{c['beta']}w{c['Wi']}")
def test_edge_configuration_matches_oracle(case):
    c = dict(case)
    nx, ny = c.pop("nx"), c.pop("ny")
    print(f"edge case {nx}x{ny} {c}", flush=True)
    t, o = make_pair(nx, ny, c.pop("Re"), c.pop("Wi"), c.pop("beta"), c.pop("periods"),
                     pre_steps=60, pert_modes=1, **c)
    t.init(seed=5, perturbation=1e-2)
    o.base_state(60)
    o.perturb(5, 1e-2, True)
    compare_states(t.get_state(), o.get_state(), 1e-12)
    t.step(20); o.step(20)
    compare_states(t.get_state(), o.get_state(), 1e-12)
    assert max_rel(t.moments(), o.observables()) < 1e-12
    dt, do = t.diagnostics(), o.diagnostics()
    for k in ("mass_S", "mass_P"):
        assert abs(dt[k] / do[k] - 1) < 1e-12, k
    t.close()


def test_zero_steps_leave_the_state():
    t, _ = make_pair(16, 8, 20.0, 0.5, 0.8, 1, nq=6, pre_steps=20)
    t.init(seed=1, perturbation=1e-2)
    t.step(3)
    st = t.get_state()
    t.step(0)
    assert t.query("step") == 3
    after = t.get_state()
    for k in st:
        assert np.array_equal(st[k], after[k]), k
    t.close()
