"""Same-step gradients (gradients = 1): the velocity gradient and the spring
term's psi gradient taken from this step's observables, formed from the
pulled populations by three launches before the step.  Parity with the
oracle run with the same reading, in every storage form that supports it,
through the base-state column run as well; in place equal to two arrays
bitwise."""
import numpy as np
import pytest

import paper_2201_10132_amd as P
from tests.gpu_common import compare_states, make_pair, max_rel
from tests.test_gpu_fp32 import EPS32, _delta_bound
from tests.test_gpu_parity import _random_state

pytestmark = pytest.mark.gpu

CASES = [
    dict(nx=16, ny=16, nq=6, spring=0, periods=2, qsplit=1),
    dict(nx=70, ny=12, nq=4, spring=1, periods=3, qsplit=4),   # ragged tail
    dict(nx=128, ny=8, nq=6, spring=0, periods=2, qsplit=0, qe_model=2),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c['nx']}x{c['ny']}q{c['nq']}")
def test_same_step_parity_from_random_state(case):
    c = dict(case)
    nx, ny = c.pop("nx"), c.pop("ny")
    t, o = make_pair(nx, ny, 20.0, 0.5, 0.8, c.pop("periods"), pre_steps=0, gradients=1, **c)
    print(f"same-step parity {nx}x{ny} {case}", flush=True)
    t.init(seed=0, perturbation=0.0)
    st = _random_state(t.nqd, ny, nx, o, seed=41)
    t.set_state(**st)
    o.set_state(**st)
    t.step(1); o.step(1)
    compare_states(t.get_state(), o.get_state(), 1e-14)
    t.step(49); o.step(49)
    compare_states(t.get_state(), o.get_state(), 1e-13)
    assert max_rel(t.moments(), o.observables()) < 1e-13


def test_same_step_init_and_fp32_parity():
    """Base-state column run, tiling, perturbation and 100 steps with
    same-step gradients: FP64 to the init tolerance of the plain tests, FP32
    within its deviation bound."""
    nx, ny = 64, 16
    t, o = make_pair(nx, ny, 20.0, 0.5, 0.8, 2, nq=6, pre_steps=300, pert_modes=1, gradients=1)
    t.init(seed=4, perturbation=0.02)
    o.base_state(300)
    base = o.get_state()
    o.perturb(4, 0.02, True)
    compare_states(t.get_state(), o.get_state(), 1e-12)
    f = P.Tpl(nx, ny, 20.0, 0.5, 0.8, periods=2, nq=6, pre_steps=300, pert_modes=1,
              precision=P.TPL_FP32, gradients=1)
    f.init(seed=4, perturbation=0.02)
    n = 100
    t.step(n); f.step(n); o.step(n)
    want = o.get_state()
    compare_states(t.get_state(), want, 1e-12)
    got = f.get_state()
    bound = _delta_bound(n, want, base)
    for k in ("XS", "XP", "psi"):
        err = np.abs(got[k] - want[k]).max()
        assert err <= bound[k], (k, err, bound[k])
    assert np.abs(got["U"] - want["U"]).max() <= 20 * bound["XS"]
    t.close(); f.close()


@pytest.mark.parametrize("precision", [P.TPL_FP64, P.TPL_FP32])
def test_same_step_in_place_matches_two_arrays(precision):
    def run(inplace):
        t = P.Tpl(128, 64, 60.0, 1.0, 0.7, periods=2, nq=8, pre_steps=100, pert_modes=1,
                  precision=precision, qsplit=1, autotune=0, inplace=inplace, gradients=1)
        t.init(seed=3, perturbation=1e-3)
        t.step(6)
        st = t.get_state()
        t.close()
        return st
    a, b = run(0), run(1)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_same_step_differs_from_lagged_only_slightly():
    """The two readings of the gradients' time level are different schemes
    that agree to first order: after 200 steps of the same 64 x 16 run the
    states differ, by far less than the perturbation itself."""
    def run(g):
        t = P.Tpl(64, 16, 20.0, 0.5, 0.8, periods=2, nq=6, pre_steps=300, pert_modes=1,
                  gradients=g)
        t.init(seed=4, perturbation=0.02)
        t.step(200)
        out = t.moments(), t.amplitude()
        t.close()
        return out
    (ma, aa), (mb, ab) = run(0), run(1)
    assert not np.array_equal(ma, mb)
    assert abs(ab / aa - 1) < 1e-2
