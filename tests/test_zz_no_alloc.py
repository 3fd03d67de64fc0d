"""tpl_diagnostics_noalloc against tpl_diagnostics: the same kernels run in
the library's static per-GPU working memory instead of a context buffer.
Two calls in a row on one GPU, the second on a smaller lattice (the static
array keeps the first call's contents), FP64 and FP32 storage."""
import math

import pytest

import paper_2201_10132_amd as P


def _ctx(nx, ny, precision, seed):
    t = P.Tpl(nx, ny, 20.0, 0.5, 0.8, periods=1, nq=6, pre_steps=60, precision=precision)
    t.init(seed=seed, perturbation=1e-2)
    t.step(7)
    return t


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [P.TPL_FP64, P.TPL_FP32])
def test_noalloc_diagnostics_equal_the_allocating_call(precision):
    big = _ctx(96, 80, precision, 3)
    small = _ctx(24, 16, precision, 4)
    try:
        for t in (big, small):
            got = t.diagnostics_noalloc()
            want = t.diagnostics()
            for k, v in want.items():
                assert got[k] == v or (math.isnan(v) and math.isnan(got[k])), (k, got[k], v)
        # and again on the larger lattice after the smaller one
        assert big.diagnostics_noalloc() == big.diagnostics()
    finally:
        big.close()
        small.close()


@pytest.mark.gpu
def test_noalloc_diagnostics_reject_too_many_rows():
    t = P.Tpl(1, 65540, 20.0, 0.5, 0.8, periods=1000, nq=4, pre_steps=0)
    try:
        t.init(seed=0, perturbation=0.0)
        with pytest.raises(P.TplError, match="static working memory"):
            t.diagnostics_noalloc()
        assert t.diagnostics()["mass_S"] > 0  # the allocating call still serves it
    finally:
        t.close()
