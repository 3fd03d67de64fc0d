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


def test_same_step_fullsize_sampled_node_parity():
    """The benchmark's 1024^2 NQ 16 workload with same-step gradients, in the
    launch configuration the benchmark uses: one step's update of sampled
    nodes against the oracle on the 7 x 7 window around each (this step's psi
    and U at the neighbours reach three nodes out), and conservation."""
    import oracle
    from tests.gpu_common import FLOOR

    NX = NY = 1024
    prm = dict(Re=60.0, Wi=1.0, beta=0.7, periods=4)
    print("same-step fullsize: init 1024x1024 nq=16", flush=True)
    t = P.Tpl(NX, NY, prm["Re"], prm["Wi"], prm["beta"], periods=prm["periods"], nq=16,
              pre_steps=200, pert_modes=1, gradients=1)
    t.init(seed=0, perturbation=1e-4)
    t.step(2)
    d0 = t.diagnostics()
    samples = [(0, 0), (1023, 1023), (511, 300), (64, 511)]
    wins = {s: t.get_window(s[0] - 3, s[1] - 3, 7, 7) for s in samples}
    t.step(1)
    d1 = t.diagnostics()
    for (x, y), w in wins.items():
        print(f"same-step fullsize: node ({x},{y})", flush=True)
        o = oracle.OracleSim(7, 7, nq=16, ny_param=NY, y_offset=y - 3, gradients=1, **prm)
        o.set_state(XS=w["XS"], XP=w["XP"], psi=w["psi"], U=w["U"])
        o.step(1)
        want = o.get_state()
        got = t.get_window(x, y, 1, 1)
        for k in ("XS", "XP", "psi", "U"):
            assert max_rel(got[k][..., 0, 0], want[k][..., 3, 3], FLOOR[k]) < 1e-14, (k, x, y)
    assert abs(d1["mass_S"] / d0["mass_S"] - 1) < 1e-13
    assert abs(d1["mass_P"] / d0["mass_P"] - 1) < 1e-13
    scale = d0["mass_S"] * 0.05
    assert abs(d1["mom_x"] - d0["mom_x"]) < 1e-13 * scale
    assert abs(d1["mom_y"] - d0["mom_y"]) < 1e-13 * scale
    t.close()
