"""The shifted spring term (spring_shift = 1) combined with same-step
gradients (gradients = 1: the spring-sum pass runs over this step's psi, and
the velocity pass reads its Q-sum) and with in-place streaming (inplace = 1).
Parity with the oracle run with the same options (the oracle has one
population array form only; in place and two arrays must agree bitwise),
through the base-state column run, for single lattices and batches."""
import numpy as np
import pytest

import oracle
import paper_2201_10132_amd as P
from tests.gpu_common import compare_states, make_pair, max_rel
from tests.test_gpu_fp32 import _delta_bound
from tests.test_gpu_parity import _random_state

pytestmark = pytest.mark.gpu

CASES = [
    dict(nx=16, ny=16, nq=6, spring=0, periods=2, qsplit=1),
    dict(nx=70, ny=12, nq=4, spring=1, periods=3, qsplit=4),            # ragged tail
    dict(nx=4, ny=4, nq=16, spring=0, periods=1, qsplit=0),             # offsets wrap twice
    dict(nx=128, ny=8, nq=6, spring=0, periods=2, qsplit=1, qe_model=2),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c['nx']}x{c['ny']}q{c['nq']}")
def test_shift_same_step_parity_from_random_state(case):
    c = dict(case)
    nx, ny = c.pop("nx"), c.pop("ny")
    t, o = make_pair(nx, ny, 20.0, 0.5, 0.8, c.pop("periods"), pre_steps=0, spring_shift=1,
                     gradients=1, **c)
    print(f"shift + same-step parity {nx}x{ny} {case}", flush=True)
    t.init(seed=0, perturbation=0.0)
    st = _random_state(t.nqd, ny, nx, o, seed=61)
    t.set_state(**st)
    o.set_state(**st)
    t.step(1); o.step(1)
    compare_states(t.get_state(), o.get_state(), 1e-14)
    t.step(49); o.step(49)
    compare_states(t.get_state(), o.get_state(), 1e-13)
    assert max_rel(t.moments(), o.observables()) < 1e-13
    t.close()


def test_shift_same_step_init_and_fp32_parity():
    nx, ny = 64, 16
    t, o = make_pair(nx, ny, 20.0, 0.5, 0.8, 2, nq=6, pre_steps=300, pert_modes=1,
                     spring_shift=1, gradients=1)
    t.init(seed=4, perturbation=0.02)
    o.base_state(300)
    base = o.get_state()
    o.perturb(4, 0.02, True)
    compare_states(t.get_state(), o.get_state(), 1e-12)
    f = P.Tpl(nx, ny, 20.0, 0.5, 0.8, periods=2, nq=6, pre_steps=300, pert_modes=1,
              precision=P.TPL_FP32, spring_shift=1, gradients=1)
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


def _ctx(precision, inplace, gradients, qe_model=1):
    extra = {}
    if qe_model == 2:
        nuS = oracle.OracleSim(128, 64, Re=60.0, Wi=1.0, beta=0.7, periods=2).derived()["nuS"]
        extra = dict(qe_model=2, tau_drag=0.5 * nuS * 3.0)
    t = P.Tpl(128, 64, 60.0, 1.0, 0.7, periods=2, nq=8, pre_steps=100, pert_modes=1,
              precision=precision, qsplit=1, autotune=0, inplace=inplace, spring_shift=1,
              gradients=gradients, **extra)
    t.init(seed=3, perturbation=1e-3)
    return t


@pytest.mark.parametrize("gradients", [0, 1])
@pytest.mark.parametrize("precision,qe_model",
                         [(P.TPL_FP64, 1), (P.TPL_FP32, 1), (P.TPL_FP64, 2)],
                         ids=["fp64", "fp32", "fp64-model2"])
def test_shift_in_place_matches_two_arrays_bitwise(precision, qe_model, gradients):
    print(f"shift in place: precision {precision} model {qe_model} gradients {gradients}",
          flush=True)
    a, b = _ctx(precision, 0, gradients, qe_model), _ctx(precision, 1, gradients, qe_model)
    total = 0
    for n in (1, 1, 3, 1):
        a.step(n); b.step(n)
        total += n
        assert np.array_equal(a.moments(), b.moments()), total
        assert a.diagnostics() == b.diagnostics(), total
        if total % 2 == 0:
            sa, sb = a.get_state(), b.get_state()
            for k in sa:
                assert np.array_equal(sa[k], sb[k]), (total, k)
    a.close(); b.close()


@pytest.mark.parametrize("gradients", [0, 1])
def test_shift_in_place_parity_with_oracle(gradients):
    nx, ny = 128, 8
    t, o = make_pair(nx, ny, 20.0, 0.5, 0.8, 2, nq=6, spring=0, pre_steps=0, inplace=1,
                     spring_shift=1, gradients=gradients)
    t.set_param("autotune", 0)
    t.init(seed=0, perturbation=0.0)
    st = _random_state(t.nqd, ny, nx, o, seed=71)
    t.set_state(**st)
    o.set_state(**st)
    t.step(1); o.step(1)
    assert max_rel(t.moments(), o.observables()) < 1e-14
    t.step(19); o.step(19)
    compare_states(t.get_state(), o.get_state(), 1e-13)
    t.close()


ROWS = [
    dict(nx=64, ny=16, Re=20.0, Wi=0.5, beta=0.8, periods=1, seed=5, perturbation=1e-2),
    dict(nx=128, ny=12, Re=40.0, Wi=1.5, beta=0.7, periods=2, seed=6, perturbation=1e-2),
    dict(nx=64, ny=40, Re=25.0, Wi=0.8, beta=0.6, periods=2, seed=7, perturbation=1e-2),
]


@pytest.mark.parametrize("inplace,gradients", [(1, 0), (0, 1), (1, 1)],
                         ids=["inplace", "same-step", "inplace-same-step"])
def test_batch_shift_combined_matches_single_contexts(inplace, gradients):
    """Every instance equals a context of its own with the same options and
    Q-slice count, bitwise, through graph replays; the oracle on the first."""
    b = P.Batch(ROWS, nq=6, pre_steps=30, autotune=0, qsplit=1, group=4 if inplace else 1,
                graph_steps=4, spring_shift=1, inplace=inplace, gradients=gradients)
    b.init()
    b.step(10)
    for i, d in enumerate(ROWS):
        print(f"shift batch combined: instance {i}", flush=True)
        t = P.Tpl(d["nx"], d["ny"], d["Re"], d["Wi"], d["beta"], periods=d["periods"], nq=6,
                  pre_steps=30, qsplit=1, autotune=0, spring_shift=1, inplace=inplace,
                  gradients=gradients)
        t.init(seed=d["seed"], perturbation=d["perturbation"])
        t.step(10)
        sa, sb = b.instance(i).get_state(), t.get_state()
        for k in sa:
            assert np.array_equal(sa[k], sb[k]), (i, k)
        t.close()
    d = ROWS[0]
    o = oracle.OracleSim(d["nx"], d["ny"], nq=6, Re=d["Re"], Wi=d["Wi"], beta=d["beta"],
                         periods=d["periods"], spring_shift=1, gradients=gradients)
    o.base_state(30)
    o.perturb(d["seed"], d["perturbation"], True)
    o.step(10)
    compare_states(b.instance(0).get_state(), o.get_state(), 1e-12)
    b.close()
