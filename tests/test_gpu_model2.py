"""GPU parity of the stress-tensor quasi-equilibrium model (Sec. V model
(ii), qe_model = 2) with the FP64 oracle, in every storage form.

Tolerances as for model (i): FP64 1e-14 for one step from a random state,
1e-13 after 100 steps and through init; FP32 within n 2^-24 max|deviation|
of the oracle (factor 4 margin); BF16 within n (2^-8 max|polymer deviation|
+ 4 2^-24 max|deviation|) (factor 4).  The drag time tau1_S = tau_drag must
not exceed the viscous tau2_S = nu_S / c_s^2, so each case takes half of it.
"""
import numpy as np
import pytest

import oracle
import paper_2201_10132_amd as P
from tests.gpu_common import compare_states, make_pair, max_rel
from tests.test_gpu_fp32 import _delta_bound
from tests.test_gpu_bf16 import _bound as _bf16_bound
from tests.test_gpu_parity import _random_state

pytestmark = pytest.mark.gpu

CS2 = 1.0 / 3.0


def _pair(nx, ny, Re, Wi, beta, periods, **kw):
    nuS = oracle.OracleSim(nx, ny, Re=Re, Wi=Wi, beta=beta, periods=periods,
                           nq=kw.get("nq", 16)).derived()["nuS"]
    kw.setdefault("tau_ratio_p", 0.5)
    return make_pair(nx, ny, Re, Wi, beta, periods, qe_model=2, tau_drag=0.5 * nuS / CS2, **kw)


CASES = [
    dict(nx=8, ny=8, nq=4, spring=1, periods=1),
    dict(nx=16, ny=16, nq=6, spring=0, periods=2),
    dict(nx=13, ny=9, nq=4, spring=0, periods=1),   # ragged: N not a multiple of 64
    dict(nx=70, ny=12, nq=4, spring=1, periods=3),  # several tiles + ragged tail
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c['nx']}x{c['ny']}q{c['nq']}s{c['spring']}")
@pytest.mark.parametrize("qsplit", [1, 4])
def test_model2_step_parity_from_random_state(case, qsplit):
    c = dict(case)
    nx, ny = c.pop("nx"), c.pop("ny")
    t, o = _pair(nx, ny, 20.0, 0.5, 0.8, c.pop("periods"), qsplit=qsplit, pre_steps=0, **c)
    print(f"model 2 case {nx}x{ny} {case} qsplit={qsplit}", flush=True)
    assert t.query("qe_model") == 2 and abs(t.query("tau1S") - o.derived()["tau1S"]) < 1e-15
    t.init(seed=0, perturbation=0.0)
    st = _random_state(t.nqd, ny, nx, o, seed=31)
    t.set_state(**st)
    o.set_state(**st)
    t.step(1); o.step(1)
    compare_states(t.get_state(), o.get_state(), 1e-14)
    t.step(99); o.step(99)
    compare_states(t.get_state(), o.get_state(), 1e-13)
    assert max_rel(t.moments(), o.observables()) < 1e-13


@pytest.mark.parametrize("multimode", [False, True])
def test_model2_init_and_run_parity(multimode):
    t, o = _pair(64, 32, 20.0, 0.5, 0.8, 1, nq=6, pre_steps=300, pert_modes=int(multimode))
    print(f"model 2 init multimode={multimode}", flush=True)
    t.init(seed=2, perturbation=1e-2)
    o.base_state(300)
    o.perturb(2, 1e-2, multimode)
    compare_states(t.get_state(), o.get_state(), 1e-13)
    t.step(60); o.step(60)
    compare_states(t.get_state(), o.get_state(), 1e-13)
    assert abs(t.amplitude() / o.amplitude() - 1) < 1e-12


@pytest.mark.parametrize("precision", [P.TPL_FP32, P.TPL_BF16])
def test_model2_storage_forms(precision):
    t, o = _pair(64, 16, 20.0, 0.5, 0.8, 2, nq=6, pre_steps=300, pert_modes=1)
    t.set_param("precision", precision)
    print(f"model 2 precision {precision}", flush=True)
    t.init(seed=4, perturbation=0.02)
    o.base_state(300)
    base = o.get_state()
    o.perturb(4, 0.02, True)
    want0 = o.get_state()
    n = 100
    t.step(n); o.step(n)
    got, want = t.get_state(), o.get_state()
    if precision == P.TPL_FP32:
        bound = _delta_bound(n, want, base)
    else:
        b = _bf16_bound(n + 1, [want0, want], base)
        bound = {k: b for k in ("XS", "XP", "psi")}
    for k in ("XS", "XP", "psi"):
        err = np.abs(got[k] - want[k]).max()
        print(k, err, bound[k], flush=True)
        assert err <= bound[k], (k, err, bound[k])


def test_model2_tile_groups_bitwise():
    def run(shape):
        nuS = oracle.OracleSim(512, 64, Re=60.0, Wi=1.0, beta=0.7, periods=2).derived()["nuS"]
        t = P.Tpl(512, 64, 60.0, 1.0, 0.7, periods=2, nq=8, pre_steps=100, qe_model=2,
                  tau_drag=0.5 * nuS / CS2, qsplit=1, autotune=0)
        if shape:
            t.set_param("group_x", shape[0])
            t.set_param("group_y", shape[1])
            t.set_param("group_sync", 1)
        t.init(seed=1, perturbation=1e-3)
        t.step(5)
        st = t.get_state()
        t.close()
        return st
    a, b = run(None), run((4, 2))
    for k in a:
        assert np.array_equal(a[k], b[k]), k
