"""GPU parity of the HIP step (through the C ABI) with the FP64 oracle.

Tolerance (FP64): one step is O(100) round-offs on O(1)-scaled values and
the two sides sum in different orders (the GPU takes the polymer density
and spring divergence from streamed Q-marginals and M, the oracle sums over
Q directly), so single-step differences are ~1e-15 relative; the scheme is
dissipative, so over n steps they grow at most linearly: 1e-13 for <= 100
steps, 1e-11 for the 20 000-step base state plus 2 000 steps.
"""
import os

import numpy as np
import pytest

import oracle
from tests import inputs
from tests.gpu_common import compare_states, make_pair, max_rel

pytestmark = pytest.mark.gpu


def _random_state(nqd, ny, nx, o, seed):
    t = o.tables()
    d = o.derived()
    XS = inputs.positive_field(seed, (9, ny, nx), (t["wS"] * d["rhoS0"])[:, None, None], 0.05)
    psi0 = d["rhoP0"] * t["peq"]
    XP = inputs.positive_field(seed + 1, (25, nqd, ny, nx),
                               (t["wP"][:, None] * psi0[None, :])[:, :, None, None], 0.05)
    psi = inputs.positive_field(seed + 2, (nqd, ny, nx), psi0[:, None, None], 0.05)
    U = inputs.normal(seed + 3, (2, ny, nx), 1e-3)
    return dict(XS=XS, XP=XP, psi=psi, U=U)


CASES = [
    dict(nx=8, ny=8, nq=4, spring=1, periods=1),
    dict(nx=8, ny=8, nq=6, spring=0, periods=1),
    dict(nx=16, ny=16, nq=6, spring=0, periods=2),
    dict(nx=13, ny=9, nq=4, spring=0, periods=1),   # ragged: N not a multiple of 64
    dict(nx=70, ny=12, nq=4, spring=1, periods=3),  # several tiles + ragged tail
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c['nx']}x{c['ny']}q{c['nq']}s{c['spring']}")
@pytest.mark.parametrize("qsplit", [1, 4])
def test_step_parity_from_random_state(case, qsplit):
    c = dict(case)
    nx, ny = c.pop("nx"), c.pop("ny")
    t, o = make_pair(nx, ny, 20.0, 0.5, 0.8, c.pop("periods"), qsplit=qsplit, pre_steps=0, **c)
    print(f"case {nx}x{ny} {case} qsplit={qsplit}", flush=True)
    t.init(seed=0, perturbation=0.0)
    st = _random_state(t.nqd, ny, nx, o, seed=11)
    t.set_state(**st)
    o.set_state(**st)
    t.step(1); o.step(1)
    compare_states(t.get_state(), o.get_state(), 1e-14)
    t.step(99); o.step(99)
    compare_states(t.get_state(), o.get_state(), 1e-13)
    assert max_rel(t.moments(), o.observables()) < 1e-13


@pytest.mark.parametrize("multimode", [False, True])
def test_init_parity(multimode):
    """Rest state, 300-step base-state column run, tiling and the seeded
    perturbation (SplitMix64 on both sides)."""
    nx, ny = 24, 20
    t, o = make_pair(nx, ny, 20.0, 0.5, 0.8, 2, nq=6, pre_steps=300,
                     pert_modes=int(multimode))
    print(f"init parity multimode={multimode}", flush=True)
    t.init(seed=7, perturbation=1e-2)
    o.base_state(300)
    o.perturb(7, 1e-2, multimode)
    compare_states(t.get_state(), o.get_state(), 1e-12)
    assert abs(t.amplitude() / o.amplitude() - 1) < 1e-10


def test_c1_short_parity():
    """64 x 64 Kolmogorov lattice at the small-workload parameters (one period,
    Re 20, Wi 0.5, beta 0.8, NQ 16, FENE), short base-state run."""
    t, o = make_pair(64, 64, 20.0, 0.5, 0.8, 1, nq=16, pre_steps=500, pert_modes=0)
    print("c1 short", flush=True)
    t.init(seed=0, perturbation=1e-3)
    o.base_state(500)
    o.perturb(0, 1e-3, False)
    t.step(100); o.step(100)
    compare_states(t.get_state(), o.get_state(), 1e-13)
    assert max_rel(t.moments(), o.observables()) < 1e-13
    dt, do = t.diagnostics(), o.diagnostics()
    for k in ("mass_S", "mass_P", "enstrophy", "qrms", "amplitude"):
        assert abs(dt[k] / do[k] - 1) < 1e-12, k


def test_conservation_gpu():
    t, _ = make_pair(64, 64, 20.0, 0.5, 0.8, 1, nq=8, pre_steps=200)
    print("conservation", flush=True)
    t.init(seed=1, perturbation=0.05)
    d0 = t.diagnostics()
    t.step(500)
    d1 = t.diagnostics()
    assert abs(d1["mass_S"] / d0["mass_S"] - 1) < 1e-12
    assert abs(d1["mass_P"] / d0["mass_P"] - 1) < 1e-12
    st = t.get_state()
    scale = np.abs(st["U"]).sum()
    for c in ("mom_x", "mom_y"):
        assert abs(d1[c] - d0[c]) < 1e-12 * scale


def test_qsplit_invariance():
    outs = []
    for qs in (1, 2, 4, 8):
        t, _ = make_pair(32, 16, 20.0, 0.5, 0.8, 1, nq=8, pre_steps=50, qsplit=qs)
        t.init(seed=3, perturbation=0.01)
        t.step(20)
        outs.append(t.get_state())
    for s in outs[1:]:
        compare_states(s, outs[0], 1e-14)


def test_nan_is_reported_as_unstable():
    import paper_2201_10132_amd as P
    t, _ = make_pair(16, 16, 20.0, 0.5, 0.8, 1, nq=4, pre_steps=0)
    t.init(seed=0, perturbation=0.0)
    st = t.get_state()
    st["XS"][0, 3, 3] = np.nan
    t.set_state(XS=st["XS"])
    with pytest.raises(P.TplError) as e:
        t.step(2)
    assert e.value.code == P.tpl.TPL_EUNSTABLE


def test_checkpoint_resume_is_bitwise(tmp_path):
    t, _ = make_pair(32, 32, 20.0, 0.5, 0.8, 1, nq=6, pre_steps=100)
    t.init(seed=2, perturbation=0.01)
    t.step(10)
    path = tmp_path / "ck.bin"
    t.save(path)
    t.step(15)
    a = t.get_state()
    t.load(path)
    assert t.query("step") == 10
    t.step(15)
    b = t.get_state()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
