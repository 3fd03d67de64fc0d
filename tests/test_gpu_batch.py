"""GPU tests of the batched form (tpl_batch_*): every instance of a batch
must reproduce the oracle and a context of its own, whatever the launch
shape, through graph replays, interleaved single steps and the loss of an
unstable instance.

Tolerances: against the oracle as for one lattice (1e-12 after a 100-step
base state and 20 steps, FP64).  Against a context of its own with the same
Q-slice count the batch runs the same arithmetic in the same order, so the
states agree bitwise; across Q-slice counts the slice reduction changes the
summation order (1e-13).
"""
import numpy as np
import pytest

import oracle
import paper_2201_10132_amd as P
from tests import inputs
from tests.gpu_common import compare_states

pytestmark = pytest.mark.gpu

# Mixed sizes: ragged tiles (nx * ny not a multiple of 64), a column-height
# spread for the batched base-state phases, different parameters.
MIXED = [
    dict(nx=16, ny=16, Re=20.0, Wi=0.5, beta=0.8, periods=1, seed=1, perturbation=1e-2),
    dict(nx=24, ny=20, Re=35.0, Wi=1.2, beta=0.6, periods=2, seed=2, perturbation=1e-2),
    dict(nx=13, ny=9, Re=12.0, Wi=0.0, beta=0.9, periods=1, seed=3, perturbation=1e-2),
    dict(nx=70, ny=12, Re=50.0, Wi=0.3, beta=0.5, periods=3, seed=4, perturbation=1e-2),
]
# Every nx a multiple of 64: the row-tile kernel variant.
ROWS = [
    dict(nx=64, ny=16, Re=20.0, Wi=0.5, beta=0.8, periods=1, seed=5, perturbation=1e-2),
    dict(nx=128, ny=12, Re=40.0, Wi=1.5, beta=0.7, periods=2, seed=6, perturbation=1e-2),
    dict(nx=64, ny=40, Re=25.0, Wi=0.8, beta=0.6, periods=2, seed=7, perturbation=1e-2),
]


def _single(d, precision, **params):
    t = P.Tpl(d["nx"], d["ny"], d["Re"], d["Wi"], d["beta"], periods=d["periods"],
              u0=d.get("u0", 0.05), precision=precision, **params)
    t.init(seed=d["seed"], perturbation=d["perturbation"])
    return t


def _states_equal(a, b):
    return {k: float(np.abs(a[k] - b[k]).max()) for k in a}


@pytest.mark.parametrize("insts", [MIXED, ROWS], ids=["mixed", "rowtile"])
def test_batch_matches_oracle(insts):
    print(f"batch vs oracle: {len(insts)} instances", flush=True)
    b = P.Batch(insts, nq=6, pre_steps=100, graph_steps=4)
    b.init()
    assert b.query("rowtile") == (insts is ROWS)
    b.step(20)  # 5 graph replays
    for i, d in enumerate(insts):
        o = oracle.OracleSim(d["nx"], d["ny"], nq=6, Re=d["Re"], Wi=d["Wi"], beta=d["beta"],
                             periods=d["periods"])
        o.base_state(100)
        o.perturb(d["seed"], d["perturbation"], True)
        o.step(20)
        compare_states(b.instance(i).get_state(), o.get_state(), 1e-12)
    b.close()


@pytest.mark.parametrize("precision", [P.TPL_FP64, P.TPL_FP32], ids=["fp64", "fp32"])
def test_batch_bitwise_vs_single(precision):
    insts = MIXED + ROWS
    print(f"batch vs single contexts, precision={precision}", flush=True)
    b = P.Batch(insts, precision=precision, nq=8, pre_steps=60, graph_steps=4)
    b.init()
    qs = int(b.query("qsplit_used"))
    b.step(10)  # two graph replays and two plain launches
    for i, d in enumerate(insts):
        t = _single(d, precision, nq=8, pre_steps=60, qsplit=qs)
        t.step(10)
        diff = _states_equal(b.instance(i).get_state(), t.get_state())
        assert all(v == 0.0 for v in diff.values()), (i, diff)
        assert b.instance(i).query("step") == 10
        t.close()
    b.close()


def test_batch_shapes_agree():
    """Forced launch shapes: grid changes nothing, Q-slices only rounding."""
    insts = MIXED
    ref = None
    for qs, grid in [(1, 0), (1, 8), (2, 16), (4, 0), (8, 24)]:
        print(f"shape qsplit={qs} grid={grid}", flush=True)
        b = P.Batch(insts, nq=8, pre_steps=40, autotune=0, qsplit=qs, grid=grid,
                    graph_steps=0)
        b.init()
        assert b.query("qsplit_used") == qs
        assert b.query("grid_used") == (grid if grid else b.query("items"))
        b.step(6)
        st = [b.instance(i).get_state() for i in range(len(insts))]
        if ref is None:
            ref = st
        else:
            for a, r in zip(st, ref):
                compare_states(a, r, 1e-13)
        b.close()


@pytest.mark.parametrize("insts", [MIXED, ROWS], ids=["mixed", "rows"])
def test_item_groups_are_bitwise_equal(insts):
    """Consecutive tiles per workgroup (one Q-slice): which wave takes which
    tile changes nothing, in plain launches, persistent grids, graph replays
    and the autotuned shape; ragged tails leave idle waves in the last
    group."""
    def run(**kw):
        b = P.Batch(insts, precision=1, nq=6, pre_steps=40, qsplit=1, **kw)
        b.init()
        shape = (b.query("group_used"), b.query("grid_used"))
        b.step(7)
        st = [b.instance(i).get_state() for i in range(len(insts))]
        b.close()
        return st, shape
    ref, shape = run(autotune=0, group=1, graph_steps=0)
    assert shape[0] == 1
    for kw in (dict(autotune=0, group=2, graph_steps=0), dict(autotune=0, group=4, graph_steps=3),
               dict(autotune=0, group=8, grid=8, graph_steps=0), dict(autotune=1, graph_steps=4)):
        print("item groups", kw, flush=True)
        st, shape = run(**kw)
        if "group" in kw:
            assert shape[0] == kw["group"]
        for a, r in zip(st, ref):
            for k in a:
                assert np.array_equal(a[k], r[k]), (kw, k)


def test_graph_replays_match_plain_launches():
    """Replays of the captured graph, with eager work in between, against
    the same steps launched one by one."""
    insts = ROWS
    g = P.Batch(insts, nq=6, pre_steps=30, autotune=0, qsplit=2, graph_steps=4)
    e = P.Batch(insts, nq=6, pre_steps=30, autotune=0, qsplit=2, graph_steps=0)
    g.init()
    e.init()
    for rep in range(3):
        print(f"replay {rep}", flush=True)
        g.step(4)
        e.step(4)
        _ = g.amplitudes()  # eager work and synchronisation between replays
        for i in range(len(insts)):
            diff = _states_equal(g.instance(i).get_state(), e.instance(i).get_state())
            assert all(v == 0.0 for v in diff.values()), (rep, i, diff)
    g.close()
    e.close()


def test_interleaved_single_steps():
    """An instance stepped on its own: the next batch step continues from
    its current half."""
    insts = MIXED
    b = P.Batch(insts, nq=6, pre_steps=30, autotune=0, qsplit=4, graph_steps=4)
    b.init()
    b.step(5)
    b.instance(1).set_param("qsplit", 4)  # its own launches: same Q-slices
    b.instance(1).step(3)
    b.step(4)
    for i, d in enumerate(insts):
        t = _single(d, P.TPL_FP64, nq=6, pre_steps=30, qsplit=4)
        t.step(5 + (3 if i == 1 else 0) + 4)
        diff = _states_equal(b.instance(i).get_state(), t.get_state())
        assert all(v == 0.0 for v in diff.values()), (i, diff)
        t.close()
    b.close()


def test_unstable_instance_is_dropped():
    """NaN planted (from the host) in one instance: it is flagged and left
    alone, the others continue exactly as on their own."""
    insts = MIXED
    b = P.Batch(insts, nq=6, pre_steps=30, autotune=0, qsplit=4, graph_steps=4)
    b.init()
    b.step(2)
    bad = b.instance(2)
    st = bad.get_state()
    st["XS"][0, 3, 4] = np.nan
    bad.set_state(**st)
    b.step(3)
    assert list(b.status()) == [0, 0, 1, 0]
    assert b.query("active") == 3 and b.query("unstable") == 1
    amps = b.amplitudes()
    assert np.isnan(amps[2]) and np.all(np.isfinite(np.delete(amps, 2)))
    b.step(5)
    for i, d in enumerate(insts):
        if i == 2:
            continue
        t = _single(d, P.TPL_FP64, nq=6, pre_steps=30, qsplit=4)
        t.step(10)
        diff = _states_equal(b.instance(i).get_state(), t.get_state())
        assert all(v == 0.0 for v in diff.values()), (i, diff)
        t.close()
    assert b.instance(2).query("step") == 5
    b.close()


def test_c4_draw_small_sample():
    """The first instances of the batched sweep's seeded draw, at FP32 and
    NQ = 8: all stay finite over a graph of steps and the amplitudes match
    contexts of their own."""
    insts = inputs.c4_instances(4)
    b = P.Batch(insts, precision=P.TPL_FP32, nq=8, pre_steps=200)
    b.init()
    b.step(40)
    assert b.query("unstable") == 0
    amps = b.amplitudes()
    qs = int(b.query("qsplit_used"))
    for i, d in enumerate(insts):
        t = _single(d, P.TPL_FP32, nq=8, pre_steps=200, qsplit=qs)
        t.step(40)
        assert amps[i] == t.amplitude()
        t.close()
    b.close()


def test_batch_errors():
    b = P.Batch(MIXED[:1], nq=6, pre_steps=10)
    with pytest.raises(P.TplError) as e:
        b.step(1)
    assert e.value.code == -4  # TPL_ESTATE before init
    b.init()
    with pytest.raises(P.TplError) as e:
        b.set_param("nq", 8)
    assert e.value.code == -4
    with pytest.raises(P.TplError) as e:
        b.step(-1)
    assert e.value.code == -1
    b.set_param("qsplit", 2)  # launch keys may change at any time
    assert b.query("qsplit_used") == 2
    b.step(2)
    with pytest.raises(P.TplError):
        b.set_param("group", 3)
    with pytest.raises(P.TplError):  # item groups need one Q-slice
        b.set_param("group", 2)
    assert b.query("qsplit_used") == 2 and b.query("group") == 0
    b.step(2)
    b.close()


@pytest.mark.parametrize("precision", [P.TPL_FP64, P.TPL_FP32], ids=["fp64", "fp32"])
def test_batch_in_place_matches_two_arrays(precision):
    """Every instance streamed in place: the same states as the two-array
    batch in the same launch shape, bitwise, after even step counts, and the
    same per-node fields after odd ones; graph replays across step-count
    parities (a graph captured at one parity is re-captured at the other);
    population reads refused at odd parity; an instance stepped on its own
    blocks the batch until it is back at the batch's parity."""
    def make(inplace):
        b = P.Batch(ROWS, precision=precision, nq=6, pre_steps=40, qsplit=1, group=4,
                    autotune=0, graph_steps=4, inplace=inplace)
        b.init()
        return b
    a, b = make(0), make(1)
    assert b.query("qsplit_used") == 1 and b.query("group_used") == 4
    assert b.query("bytes_state") < a.query("bytes_state")
    total = 0
    for n in (5, 4, 9, 2, 1, 1):
        a.step(n); b.step(n)
        total += n
        print(f"in-place batch: step {total}", flush=True)
        for i in range(len(ROWS)):
            ta, tb = a.instance(i), b.instance(i)
            assert np.array_equal(ta.moments(), tb.moments()), (total, i)
            assert tb.query("inplace_odd") == total % 2
            if total % 2 == 0:
                sa, sb = ta.get_state(), tb.get_state()
                for k in sa:
                    assert np.array_equal(sa[k], sb[k]), (total, i, k)
            else:
                with pytest.raises(P.TplError):
                    tb.get_state()
    b.instance(0).step(1)
    with pytest.raises(P.TplError) as e:
        b.step(2)
    assert "parity" in str(e.value)
    b.instance(0).step(1)
    a.instance(0).set_param("qsplit", 1)  # its own launches: one Q-slice, as in place
    a.instance(0).step(2)
    a.step(2); b.step(2)
    for i in range(len(ROWS)):
        sa, sb = a.instance(i).get_state(), b.instance(i).get_state()
        for k in sa:
            assert np.array_equal(sa[k], sb[k]), ("after own steps", i, k)
    a.close(); b.close()


@pytest.mark.parametrize("insts", [MIXED, ROWS], ids=["mixed", "rows"])
def test_batch_shifted_spring_matches_single_contexts(insts):
    """The shifted spring term in the batched step (its Q-sums formed by a
    batched launch, also for the base-state columns): every instance equals
    a context of its own with the same option and Q-slice count, bitwise,
    through graph replays; and the oracle on the first instance."""
    b = P.Batch(insts, nq=6, pre_steps=30, autotune=0, qsplit=1, group=1, graph_steps=4,
                spring_shift=1)
    b.init()
    b.step(9)
    for i, d in enumerate(insts):
        print(f"shifted batch: instance {i}", flush=True)
        t = _single(d, P.TPL_FP64, nq=6, pre_steps=30, qsplit=1, autotune=0, spring_shift=1)
        t.step(9)
        diff = _states_equal(b.instance(i).get_state(), t.get_state())
        assert all(v == 0.0 for v in diff.values()), (i, diff)
        t.close()
    d = insts[0]
    o = oracle.OracleSim(d["nx"], d["ny"], nq=6, Re=d["Re"], Wi=d["Wi"], beta=d["beta"],
                         periods=d["periods"], spring_shift=1)
    o.base_state(30)
    o.perturb(d["seed"], d["perturbation"], True)
    o.step(9)
    compare_states(b.instance(0).get_state(), o.get_state(), 1e-12)
    b.close()


@pytest.mark.parametrize("insts,precision,inplace",
                         [(MIXED, P.TPL_FP64, 0), (ROWS, P.TPL_FP32, 0), (ROWS, P.TPL_FP64, 1)],
                         ids=["mixed-fp64", "rows-fp32", "rows-fp64-inplace"])
def test_batch_same_step_gradients_match_single_contexts(insts, precision, inplace):
    """Same-step gradients in the batched step (the three field passes
    batched too, also for the base-state columns): every instance equals a
    context of its own with the same options and Q-slice count, bitwise,
    through graph replays, also streamed in place; and the oracle on the
    first instance (FP64)."""
    group = 4 if inplace else 1
    b = P.Batch(insts, precision=precision, nq=6, pre_steps=30, autotune=0, qsplit=1,
                group=group, graph_steps=4, gradients=1, inplace=inplace)
    b.init()
    b.step(10)
    for i, d in enumerate(insts):
        print(f"same-step batch: instance {i}", flush=True)
        t = _single(d, precision, nq=6, pre_steps=30, qsplit=1, autotune=0, gradients=1,
                    inplace=inplace)
        t.step(10)
        diff = _states_equal(b.instance(i).get_state(), t.get_state())
        assert all(v == 0.0 for v in diff.values()), (i, diff)
        t.close()
    if precision == P.TPL_FP64:
        d = insts[0]
        o = oracle.OracleSim(d["nx"], d["ny"], nq=6, Re=d["Re"], Wi=d["Wi"], beta=d["beta"],
                             periods=d["periods"], gradients=1)
        o.base_state(30)
        o.perturb(d["seed"], d["perturbation"], True)
        o.step(10)
        compare_states(b.instance(0).get_state(), o.get_state(), 1e-12)
    b.close()


def _model2_params(d):
    nuS = oracle.OracleSim(d["nx"], d["ny"], Re=d["Re"], Wi=d["Wi"], beta=d["beta"],
                           periods=d["periods"]).derived()["nuS"]
    return dict(qe_model=2, tau_drag=0.5 * nuS * 3.0)


@pytest.mark.parametrize("insts,precision,inplace",
                         [(MIXED, P.TPL_FP64, 0), (ROWS, P.TPL_FP32, 0), (ROWS, P.TPL_FP64, 1)],
                         ids=["mixed-fp64", "rows-fp32", "rows-fp64-inplace"])
def test_batch_model2_matches_single_contexts(insts, precision, inplace):
    """Model (ii) (stress quasi-equilibria) in the batched step, each instance
    with its own drag time: every instance equals a context of its own with
    the same options and Q-slice count, bitwise, through graph replays and
    the base-state columns, also in place; and the oracle on the first
    instance (FP64)."""
    extra = [_model2_params(d) for d in insts]
    b = P.Batch(insts, precision=precision, nq=6, pre_steps=30, autotune=0, qsplit=1,
                group=4 if inplace else 1, graph_steps=4, inplace=inplace)
    for i, e in enumerate(extra):
        for k, v in e.items():
            b.instance(i).set_param(k, v)
    b.init()
    b.step(10)
    for i, d in enumerate(insts):
        print(f"model (ii) batch: instance {i}", flush=True)
        t = _single(d, precision, nq=6, pre_steps=30, qsplit=1, autotune=0, inplace=inplace,
                    **extra[i])
        t.step(10)
        diff = _states_equal(b.instance(i).get_state(), t.get_state())
        assert all(v == 0.0 for v in diff.values()), (i, diff)
        t.close()
    if precision == P.TPL_FP64:
        d = insts[0]
        o = oracle.OracleSim(d["nx"], d["ny"], nq=6, Re=d["Re"], Wi=d["Wi"], beta=d["beta"],
                             periods=d["periods"], **extra[0])
        o.base_state(30)
        o.perturb(d["seed"], d["perturbation"], True)
        o.step(10)
        compare_states(b.instance(0).get_state(), o.get_state(), 1e-12)
    b.close()


@pytest.mark.parametrize("option", ["spring_shift", "gradients"])
def test_autotune_leaves_the_initial_fields_unchanged(option):
    """The autotuner times repeated launches on the current half; with the
    shifted spring term or same-step gradients the passes before each step
    rewrite that half's psi and per-node fields.  After tpl_batch_init the
    instances' state, moments and diagnostics must equal those of a batch
    that timed nothing, bitwise, and so must the states after some steps."""
    kw = {option: 1}
    a = P.Batch(ROWS, nq=6, pre_steps=30, autotune=1, graph_steps=0, **kw)
    b = P.Batch(ROWS, nq=6, pre_steps=30, autotune=0, qsplit=1, group=1, graph_steps=0, **kw)
    a.init()
    b.init()
    for i in range(len(ROWS)):
        print(f"autotune {option}: instance {i}", flush=True)
        ta, tb = a.instance(i), b.instance(i)
        sa, sb = ta.get_state(), tb.get_state()
        for k in sa:
            assert np.array_equal(sa[k], sb[k]), (i, k)
        assert np.array_equal(ta.moments(), tb.moments()), i
        assert ta.diagnostics() == tb.diagnostics(), i
    a.step(6)
    b.step(6)
    for i in range(len(ROWS)):
        sa, sb = a.instance(i).get_state(), b.instance(i).get_state()
        for k in sa:
            # the tuned shape may split Q differently: the slice reduction
            # changes the summation order
            assert np.abs(sa[k] - sb[k]).max() <= 1e-13 * max(np.abs(sb[k]).max(), 1.0), (i, k)
    a.close()
    b.close()
