"""Failure detection of tpl_step and tpl_batch_step: a state holding NaN/Inf
or a polymer density psi below -psi_floor max psi (psi is a density of
dumbbell configurations, Sec. VI.B) returns TPL_EUNSTABLE; diag_every sets
how many steps run between checks.  Faults are planted from the host in
the populations; every kernel still runs to completion."""
import numpy as np
import pytest

import paper_2201_10132_amd as P


def _ctx(**kw):
    t = P.Tpl(16, 16, 20.0, 0.5, 0.8, periods=1, nq=6, pre_steps=20, **kw)
    t.init(seed=0, perturbation=1e-3)
    return t


def _plant_negative_psi(t, x=5, y=5, q=3):
    """Flip the populations of one (r, Q)-node to -1000 times their value:
    after one step their pull makes psi strongly negative at the nodes they
    stream to."""
    st = t.get_state()
    st["XP"][:, q, y, x] *= -1000.0
    t.set_state(XS=st["XS"], XP=st["XP"], psi=st["psi"], U=st["U"])


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [P.TPL_FP64, P.TPL_FP32])
def test_negative_psi_is_reported_as_unstable(precision):
    t = _ctx(precision=precision)
    t.step(2)
    _plant_negative_psi(t)
    with pytest.raises(P.TplError, match="polymer density negative") as e:
        t.step(1)
    assert e.value.code == P.tpl.TPL_EUNSTABLE
    assert t.diagnostics()["min_psi"] < 0
    t.close()


@pytest.mark.gpu
def test_psi_floor_sets_the_tolerance():
    t = _ctx(psi_floor=1e9)
    _plant_negative_psi(t)
    t.step(1)  # tolerated
    t.set_param("psi_floor", 0.1)  # may be changed at any time
    with pytest.raises(P.TplError) as e:
        t.step(1)
    assert e.value.code == P.tpl.TPL_EUNSTABLE
    t.close()


@pytest.mark.gpu
def test_a_healthy_fene_run_passes_the_check():
    """The 64^2 workload's FENE run: the outermost Q-nodes carry slightly
    negative psi (the linear Q-space equilibrium is not positivity
    preserving), well inside the default tolerance."""
    t = P.Tpl(64, 64, 20.0, 0.5, 0.8, periods=1, nq=16, pre_steps=500, pert_modes=0)
    t.init(seed=0, perturbation=1e-3)
    t.step(300)
    d = t.diagnostics()
    mx = t.get_state(populations=False)["psi"].max()
    assert -0.1 * mx < d["min_psi"] < 0.0
    t.close()


@pytest.mark.gpu
@pytest.mark.parametrize("every,stops_at", [(0, 20), (4, 4), (7, 7)])
def test_diag_every_stops_at_the_first_failed_check(every, stops_at):
    t = _ctx(diag_every=every)
    st = t.get_state()
    st["XS"][0, 3, 3] = np.nan
    t.set_state(XS=st["XS"])
    with pytest.raises(P.TplError, match="not finite after step %d" % stops_at) as e:
        t.step(20)
    assert e.value.code == P.tpl.TPL_EUNSTABLE
    assert t.query("step") == stops_at
    t.close()


@pytest.mark.gpu
def test_diag_every_changes_no_result():
    a, b = _ctx(), _ctx(diag_every=3)
    a.step(10)
    b.step(10)
    sa, sb = a.get_state(), b.get_state()
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
    a.close()
    b.close()


@pytest.mark.gpu
def test_batch_flags_an_instance_with_negative_psi():
    insts = [dict(nx=16, ny=16, periods=1, Re=20.0, Wi=w, beta=0.8, u0=0.05, seed=i,
                  perturbation=1e-3) for i, w in enumerate((0.5, 1.0, 1.5))]
    b = P.Batch(insts, nq=6, pre_steps=20, autotune=0, graph_steps=2)
    b.init()
    b.step(2)
    _plant_negative_psi(b.instance(1))
    b.step(2)
    assert list(b.status()) == [0, 1, 0]
    b.close()
