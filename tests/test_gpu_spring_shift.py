"""The shifted spring term (spring_shift = 1): psi at the beads,
psi(r + Q/2) - psi(r - Q/2) by periodic bilinear interpolation, in place of
the first-order Taylor form, with its Q-sum formed by a launch before the
step.  Parity with the oracle run with the same option, through the
base-state column run (a one-wide lattice, where every x-offset wraps) and
on lattices narrower than the largest offset; tile groups bitwise."""
import numpy as np
import pytest

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
def test_shift_parity_from_random_state(case):
    c = dict(case)
    nx, ny = c.pop("nx"), c.pop("ny")
    t, o = make_pair(nx, ny, 20.0, 0.5, 0.8, c.pop("periods"), pre_steps=0, spring_shift=1, **c)
    print(f"shift parity {nx}x{ny} {case}", flush=True)
    t.init(seed=0, perturbation=0.0)
    st = _random_state(t.nqd, ny, nx, o, seed=51)
    t.set_state(**st)
    o.set_state(**st)
    t.step(1); o.step(1)
    compare_states(t.get_state(), o.get_state(), 1e-14)
    t.step(49); o.step(49)
    compare_states(t.get_state(), o.get_state(), 1e-13)
    assert max_rel(t.moments(), o.observables()) < 1e-13


def test_shift_init_and_fp32_parity():
    nx, ny = 64, 16
    t, o = make_pair(nx, ny, 20.0, 0.5, 0.8, 2, nq=6, pre_steps=300, pert_modes=1,
                     spring_shift=1)
    t.init(seed=4, perturbation=0.02)
    o.base_state(300)
    base = o.get_state()
    o.perturb(4, 0.02, True)
    compare_states(t.get_state(), o.get_state(), 1e-12)
    f = P.Tpl(nx, ny, 20.0, 0.5, 0.8, periods=2, nq=6, pre_steps=300, pert_modes=1,
              precision=P.TPL_FP32, spring_shift=1)
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


def test_shift_tile_groups_bitwise():
    def run(shape):
        t = P.Tpl(512, 64, 60.0, 1.0, 0.7, periods=2, nq=8, pre_steps=100, pert_modes=1,
                  qsplit=1, autotune=0, spring_shift=1)
        if shape:
            t.set_param("group_y", 1)
            t.set_param("group_x", shape[0])
            t.set_param("group_y", shape[1])
            t.set_param("group_sync", shape[2])
        t.init(seed=2, perturbation=1e-3)
        t.step(5)
        st = t.get_state()
        t.close()
        return st
    a = run(None)
    for shape in [(4, 2, 1), (8, 1, 0)]:
        b = run(shape)
        for k in a:
            assert np.array_equal(a[k], b[k]), (shape, k)


def test_shift_differs_from_taylor_form_slightly():
    """Where the dumbbells are small against the flow scale (sigma k = 0.16
    here) the two forms agree to a few per cent of the elastic stress."""
    def run(shift):
        t = P.Tpl(64, 16, 20.0, 0.5, 0.8, periods=2, nq=6, pre_steps=300, pert_modes=1,
                  spring_shift=shift)
        t.init(seed=4, perturbation=0.02)
        t.step(200)
        out = t.moments(), t.amplitude()
        t.close()
        return out
    (ma, aa), (mb, ab) = run(0), run(1)
    assert not np.array_equal(ma, mb)
    assert abs(ab / aa - 1) < 2e-2


def test_kolmogorov72_driver_with_shift_and_as_separate_contexts():
    """The paper's cell with the shifted spring term, batched, and as
    separate contexts (the driver's path for options the batched step does
    not take): the two agree bitwise (a short run at a small Q-grid)."""
    from paper_2201_10132_amd import kolmogorov72 as K

    res = K.run(t_end=1.0, every=0.5, nq=8, progress=False, spring_shift=1)
    assert len(res["t"]) == 3 and res["unstable"] == [False, False, False]
    for i in range(3):
        assert np.all(np.isfinite(res["enstrophy"][i])) and res["enstrophy"][i][-1] > 0
    rows = K.summary(res)
    assert [r["Wi"] for r in rows] == list(K.WIS)
    cells = K._Cells([dict(K.CELL, Wi=w, seed=0, perturbation=1e-3) for w in K.WIS],
                     precision=P.TPL_FP64, nq=8, pre_steps=0, spring_shift=1)
    batch = P.Batch([dict(K.CELL, Wi=w, seed=0, perturbation=1e-3) for w in K.WIS],
                    precision=P.TPL_FP64, nq=8, pre_steps=0, spring_shift=1, autotune=0,
                    qsplit=8)
    cells.init(); batch.init()
    for t in cells.cells:
        t.set_param("qsplit", 8)
        t.set_param("autotune", 0)
    cells.step(30); batch.step(30)
    for i in range(3):
        assert cells.instance(i).diagnostics() == batch.instance(i).diagnostics(), i
    cells.close(); batch.close()


def test_shift_fullsize_sampled_node_parity():
    """The benchmark's 1024^2 NQ 16 workload with the shifted spring term, in
    the benchmark's launch configuration: one step's update of sampled nodes
    against the oracle on the 11 x 11 window around each (the beads of the
    largest Q-nodes sit up to five nodes away), and conservation."""
    import oracle
    from tests.gpu_common import FLOOR

    NX = NY = 1024
    prm = dict(Re=60.0, Wi=1.0, beta=0.7, periods=4)
    print("shift fullsize: init 1024x1024 nq=16", flush=True)
    t = P.Tpl(NX, NY, prm["Re"], prm["Wi"], prm["beta"], periods=prm["periods"], nq=16,
              pre_steps=200, pert_modes=1, spring_shift=1)
    t.init(seed=0, perturbation=1e-4)
    t.step(2)
    d0 = t.diagnostics()
    samples = [(0, 0), (1023, 1023), (511, 300), (64, 511)]
    wins = {s: t.get_window(s[0] - 5, s[1] - 5, 11, 11) for s in samples}
    t.step(1)
    d1 = t.diagnostics()
    for (x, y), w in wins.items():
        print(f"shift fullsize: node ({x},{y})", flush=True)
        o = oracle.OracleSim(11, 11, nq=16, ny_param=NY, y_offset=y - 5, spring_shift=1, **prm)
        o.set_state(XS=w["XS"], XP=w["XP"], psi=w["psi"], U=w["U"])
        o.step(1)
        want = o.get_state()
        got = t.get_window(x, y, 1, 1)
        for k in ("XS", "XP", "psi", "U"):
            assert max_rel(got[k][..., 0, 0], want[k][..., 5, 5], FLOOR[k]) < 1e-14, (k, x, y)
    assert abs(d1["mass_S"] / d0["mass_S"] - 1) < 1e-13
    assert abs(d1["mass_P"] / d0["mass_P"] - 1) < 1e-13
    scale = d0["mass_S"] * 0.05
    assert abs(d1["mom_x"] - d0["mom_x"]) < 1e-13 * scale
    assert abs(d1["mom_y"] - d0["mom_y"]) < 1e-13 * scale
    t.close()
