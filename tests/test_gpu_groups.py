"""Tile groups of the step kernel: several 64-node tiles (one wave each) per
workgroup, optionally held on the same Q-node by a barrier.  The grouping
changes which wave computes which tile and when, never what a tile computes,
so every shape must give bitwise the state of the plain launch; the plain
launch is the one the oracle parity tests cover, and one grouped shape is
also compared with the oracle directly.  The autotuner only picks among
these shapes (its timed launches must leave the state untouched)."""
import numpy as np
import pytest

import paper_2201_10132_amd as P
from tests.gpu_common import compare_states, make_pair, max_rel
from tests.test_gpu_parity import _random_state

pytestmark = pytest.mark.gpu

SHAPES = [(2, 1, 1), (4, 1, 0), (4, 1, 1), (2, 2, 1), (1, 4, 1), (8, 1, 0), (4, 2, 1), (2, 4, 1)]


def _run(precision, shape, autotune=0, steps=6):
    t = P.Tpl(512, 64, 60.0, 1.0, 0.7, periods=2, nq=8, pre_steps=100, pert_modes=1,
              precision=precision)
    t.set_param("qsplit", 1)
    t.set_param("autotune", autotune)
    if shape is not None:
        t.set_param("group_y", 1)
        t.set_param("group_x", shape[0])
        t.set_param("group_y", shape[1])
        t.set_param("group_sync", shape[2])
    t.init(seed=5, perturbation=1e-3)
    t.step(steps)
    used = tuple(int(t.query(k)) for k in ("group_x_used", "group_y_used", "group_sync_used"))
    st = t.get_state()
    tune = t.query("tune_ms")
    t.close()
    return st, used, tune


@pytest.mark.parametrize("precision", [P.TPL_FP64, P.TPL_FP32, P.TPL_BF16])
def test_group_shapes_are_bitwise_equal(precision):
    ref, used, _ = _run(precision, None)
    assert used == (0, 0, 0)
    for shape in SHAPES:
        print(f"precision {precision} group {shape}", flush=True)
        st, used, _ = _run(precision, shape)
        assert used == shape
        for k in ref:
            assert np.array_equal(st[k], ref[k]), (shape, k)


def test_grouped_step_parity_with_oracle():
    """A random state stepped in a 4 x 2 synchronised group shape against
    the oracle (tolerances of the plain parity tests)."""
    nx, ny = 256, 8
    t, o = make_pair(nx, ny, 20.0, 0.5, 0.8, 2, nq=6, spring=0, qsplit=1, pre_steps=0)
    t.set_param("autotune", 0)
    t.set_param("group_x", 4)
    t.set_param("group_y", 2)
    t.set_param("group_sync", 1)
    t.init(seed=0, perturbation=0.0)
    st = _random_state(t.nqd, ny, nx, o, seed=21)
    t.set_state(**st)
    o.set_state(**st)
    t.step(1); o.step(1)
    assert int(t.query("group_x_used")) == 4 and int(t.query("group_y_used")) == 2
    compare_states(t.get_state(), o.get_state(), 1e-14)
    t.step(19); o.step(19)
    compare_states(t.get_state(), o.get_state(), 1e-13)
    assert max_rel(t.moments(), o.observables()) < 1e-13


@pytest.mark.parametrize("precision", [P.TPL_FP64, P.TPL_BF16])
def test_autotuned_shape_is_bitwise_equal(precision):
    ref, _, _ = _run(precision, None)
    st, used, tune = _run(precision, None, autotune=1)
    print(f"precision {precision}: tuned group {used}, {tune:.2f} ms of tuning", flush=True)
    assert tune > 0
    if used != (0, 0, 0):
        assert used[0] * used[1] > 1
    for k in ref:
        assert np.array_equal(st[k], ref[k]), k

