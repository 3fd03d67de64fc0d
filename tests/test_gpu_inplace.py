"""In-place streaming (one population array, the AA pattern with the Q-disk
bounce-back folded into its address maps).  The in-place steps read exactly
the values the two-array step pulls and run the same arithmetic, so after an
even number of steps the stored state must equal the two-array state
bitwise, and after every step the per-node fields (observables, diagnostics,
amplitude, lagged psi and U) must too.  The two-array step is the one the
oracle parity tests cover; the in-place step is also compared with the
oracle directly, and at the 4096^2 sizes on sampled nodes."""
import os
import tempfile

import numpy as np
import pytest

import oracle
import paper_2201_10132_amd as P
from tests.gpu_common import FLOOR, compare_states, make_pair, max_rel
from tests.test_gpu_parity import _random_state

pytestmark = pytest.mark.gpu

CS2 = 1.0 / 3.0


def _ctx(precision, inplace, qe_model=1, nx=128, ny=64, shape=None, autotune=0):
    extra = {}
    if qe_model == 2:
        nuS = oracle.OracleSim(nx, ny, Re=60.0, Wi=1.0, beta=0.7, periods=2).derived()["nuS"]
        extra = dict(qe_model=2, tau_drag=0.5 * nuS / CS2)
    t = P.Tpl(nx, ny, 60.0, 1.0, 0.7, periods=2, nq=8, pre_steps=100, pert_modes=1,
              precision=precision, qsplit=1, autotune=autotune, inplace=inplace, **extra)
    if shape:
        t.set_param("group_y", 1)
        t.set_param("group_x", shape[0])
        t.set_param("group_y", shape[1])
        t.set_param("group_sync", shape[2])
    t.init(seed=3, perturbation=1e-3)
    return t


def _same(a, b, what):
    for k in a:
        assert np.array_equal(a[k], b[k]), (what, k)


@pytest.mark.parametrize("qe_model", [1, 2])
@pytest.mark.parametrize("precision", [P.TPL_FP64, P.TPL_FP32])
def test_inplace_matches_two_array_bitwise(precision, qe_model):
    print(f"inplace vs two arrays: precision {precision} model {qe_model}", flush=True)
    a, b = _ctx(precision, 0, qe_model), _ctx(precision, 1, qe_model)
    total = 0
    for n in (1, 1, 1, 1, 3, 1):
        a.step(n); b.step(n)
        total += n
        assert b.query("step") == total and b.query("qsplit_used") == 1
        assert np.array_equal(a.moments(), b.moments()), total
        assert a.diagnostics() == b.diagnostics(), total
        assert a.amplitude() == b.amplitude(), total
        _same(a.get_state(populations=False), b.get_state(populations=False), total)
        odd = total % 2 == 1
        assert b.query("inplace_odd") == int(odd)
        if odd:  # populations in streamed order: population calls refused
            for call in (b.get_state, lambda: b.get_window(0, 0, 2, 2),
                         lambda: b.save(os.devnull)):
                with pytest.raises(P.TplError) as e:
                    call()
                assert e.value.code == P.tpl.TPL_ESTATE
        else:
            _same(a.get_state(), b.get_state(), total)
            _same(a.get_window(126, 62, 4, 4), b.get_window(126, 62, 4, 4), total)
    a.close(); b.close()


def test_inplace_parity_with_oracle():
    """A random state stepped in place against the oracle (tolerances of the
    plain parity tests); the observables also after the odd step."""
    nx, ny = 128, 8
    t, o = make_pair(nx, ny, 20.0, 0.5, 0.8, 2, nq=6, spring=0, pre_steps=0, inplace=1)
    t.set_param("autotune", 0)
    t.init(seed=0, perturbation=0.0)
    st = _random_state(t.nqd, ny, nx, o, seed=31)
    t.set_state(**st)
    o.set_state(**st)
    t.step(1); o.step(1)
    assert max_rel(t.moments(), o.observables()) < 1e-14
    got = t.get_state(populations=False)
    want = o.get_state()
    for k in ("psi", "U"):
        assert max_rel(got[k], want[k], FLOOR[k]) < 1e-14, k
    t.step(1); o.step(1)
    compare_states(t.get_state(), o.get_state(), 1e-14)
    t.step(18); o.step(18)
    compare_states(t.get_state(), o.get_state(), 1e-13)
    assert max_rel(t.moments(), o.observables()) < 1e-13
    t.close()


def test_inplace_group_shapes_and_autotune_bitwise():
    """Tile-group shapes and the autotuner, which times its shapes on real
    in-place steps (24 of the first call's steps), change no result."""
    ref = _ctx(P.TPL_FP64, 1, nx=512)
    ref.step(40)
    want = ref.get_state()
    ref.close()
    for shape in [(4, 1, 1), (8, 1, 0), (2, 2, 1)]:
        print(f"inplace group {shape}", flush=True)
        t = _ctx(P.TPL_FP64, 1, nx=512, shape=shape)
        t.step(40)
        assert tuple(int(t.query(k)) for k in ("group_x_used", "group_y_used",
                                               "group_sync_used")) == shape
        _same(want, t.get_state(), shape)
        t.close()
    t = _ctx(P.TPL_FP64, 1, nx=512, autotune=1)
    t.step(10)  # fewer steps than the tuner needs: not tuned yet
    assert t.query("tune_ms") == 0
    t.step(30)  # the tuner takes 24 of these
    print(f"inplace tuned group ({t.query('group_x_used')}, {t.query('group_y_used')}), "
          f"{t.query('tune_ms'):.2f} ms of tuning", flush=True)
    assert t.query("tune_ms") > 0 and t.query("step") == 40
    _same(want, t.get_state(), "autotuned")
    t.close()


def test_inplace_checkpoint_resume_and_set_state():
    t = _ctx(P.TPL_FP32, 1)
    t.step(3)
    with pytest.raises(P.TplError):
        t.set_state(**t.get_state(populations=False))
    t.step(1)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ck.bin")
        t.save(path)
        t.step(4)
        want = t.get_state()
        t.step(1)  # odd: loading restores the plain order
        t.load(path)
        assert t.query("inplace_odd") == 0 and t.query("step") == 4
        t.step(4)
        _same(want, t.get_state(), "resumed")
    st = t.get_state()
    t.set_state(**st)  # even: allowed, and a no-op on the state
    _same(st, t.get_state(), "set_state")
    t.close()


def test_inplace_fullsize_4096_nq8_fp64_sampled_node_parity():
    """The in-place benchmark workload, 4096^2 at NQ 8 in FP64 (a single
    population array of 175 GB; two would not fit): the state of the 5 x 5
    window around sampled nodes is loaded into a 5 x 5 periodic oracle
    lattice with the full lattice's parameters and forcing phase; two oracle
    steps then give the exact update of the window's centre.  Conservation
    over the whole lattice, also read after the odd step."""
    NX = NY = 4096
    prm = dict(Re=60.0, Wi=1.0, beta=0.7, periods=16)
    samples = [(0, 0), (4095, 4095), (2047, 1000), (63, 64), (64, 4000)]
    print("inplace fullsize: init 4096x4096 nq=8 fp64", flush=True)
    t = P.Tpl(NX, NY, prm["Re"], prm["Wi"], prm["beta"], periods=prm["periods"], nq=8,
              pre_steps=200, pert_modes=1, inplace=1, autotune=0)
    t.init(seed=0, perturbation=1e-4)
    t.step(2)
    d0 = t.diagnostics()
    wins = {s: t.get_window(s[0] - 2, s[1] - 2, 5, 5) for s in samples}
    t.step(1)
    dodd = t.diagnostics()
    t.step(1)
    d1 = t.diagnostics()
    for (x, y), w in wins.items():
        print(f"inplace fullsize: node ({x},{y})", flush=True)
        o = oracle.OracleSim(5, 5, nq=8, ny_param=NY, y_offset=y - 2, **prm)
        o.set_state(XS=w["XS"], XP=w["XP"], psi=w["psi"], U=w["U"])
        o.step(2)
        want = o.get_state()
        got = t.get_window(x, y, 1, 1)
        for k in ("XS", "XP", "psi", "U"):
            assert max_rel(got[k][..., 0, 0], want[k][..., 2, 2], FLOOR[k]) < 5e-14, (k, x, y)
    scale = d0["mass_S"] * 0.05
    for d in (dodd, d1):
        assert abs(d["mass_S"] / d0["mass_S"] - 1) < 1e-13
        assert abs(d["mass_P"] / d0["mass_P"] - 1) < 1e-13
        assert abs(d["mom_x"] - d0["mom_x"]) < 1e-13 * scale
        assert abs(d["mom_y"] - d0["mom_y"]) < 1e-13 * scale
    t.close()


def test_inplace_fullsize_4096_nq6_fp32_matches_two_array():
    """The 4096^2 FP32 workload at NQ 6, two arrays (113 GB) and in place
    (57 GB) side by side: observables bitwise after odd and even step
    counts, sampled windows bitwise."""
    prm = dict(periods=16, nq=6, pre_steps=200, pert_modes=1, precision=P.TPL_FP32, qsplit=1,
               autotune=0)
    print("inplace fullsize fp32: init both", flush=True)
    a = P.Tpl(4096, 4096, 60.0, 1.0, 0.7, inplace=0, **prm)
    a.init(seed=0, perturbation=1e-4)
    b = P.Tpl(4096, 4096, 60.0, 1.0, 0.7, inplace=1, **prm)
    b.init(seed=0, perturbation=1e-4)
    for n, total in ((1, 1), (1, 2), (2, 4)):
        a.step(n); b.step(n)
        print(f"inplace fullsize fp32: step {total}", flush=True)
        assert np.array_equal(a.moments(), b.moments()), total
        assert a.diagnostics() == b.diagnostics(), total
        if total % 2 == 0:
            for x0, y0 in ((4093, 4093), (1000, 2000), (0, 0)):
                _same(a.get_window(x0, y0, 6, 6), b.get_window(x0, y0, 6, 6), (total, x0, y0))
    a.close(); b.close()
