"""The FP32 form: populations and psi stored as float deviations from the
x-invariant FP64 base state, arithmetic in FP64, per-node fields in FP64.

Error model: each step rounds the stored deviation delta = X - X_base to
FP32 (relative 2^-24); the scheme is dissipative, so after n steps the
difference from the FP64 oracle is bounded by about n 2^-24 max|delta|
(tested with a factor 4 margin).  The growth or decay rate of the
perturbation amplitude must match the oracle's within 1e-3 relative.
"""
import numpy as np
import pytest

import oracle
from tests.gpu_common import make_pair

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24


def _delta_bound(n, st, base):
    return {k: 4 * n * EPS32 * np.abs(st[k] - base[k]).max() + 1e-13 * np.abs(st[k]).max()
            for k in ("XS", "XP", "psi")}


@pytest.mark.parametrize("nx,ny,nq,spring", [(64, 16, 6, 0), (13, 9, 4, 1), (128, 8, 4, 0)])
def test_fp32_parity_with_oracle(nx, ny, nq, spring):
    t, o = make_pair(nx, ny, 20.0, 0.5, 0.8, 2 if ny >= 8 else 1, nq=nq, spring=spring,
                     pre_steps=300, pert_modes=1)
    t.set_param("precision", 1)
    print(f"fp32 parity {nx}x{ny} nq={nq} spring={spring}", flush=True)
    t.init(seed=4, perturbation=0.02)
    o.base_state(300)
    base = o.get_state()
    o.perturb(4, 0.02, True)
    st0 = t.get_state()
    want0 = o.get_state()
    for k in ("XS", "XP", "psi"):
        assert (np.abs(st0[k] - want0[k]).max()
                <= EPS32 * np.abs(want0[k] - base[k]).max() + 1e-13 * np.abs(want0[k]).max())
    n = 100
    t.step(n); o.step(n)
    got, want = t.get_state(), o.get_state()
    bound = _delta_bound(n, want, base)
    for k in ("XS", "XP", "psi"):
        err = np.abs(got[k] - want[k]).max()
        assert err <= bound[k], (k, err, bound[k])
    # U is a ratio of population sums (|c| <= 1 per component, rho ~ 1): its
    # error is at most the summed error of the 9 solvent populations plus the
    # polymer's share
    assert np.abs(got["U"] - want["U"]).max() <= 20 * bound["XS"]


def _rate(amps, steps):
    return np.polyfit(steps, np.log(amps), 1)[0]


def test_fp32_growth_rate_matches_oracle():
    """64 x 64, one forcing period (decaying perturbation), NQ = 8."""
    kw = dict(nq=8, pre_steps=1500, pert_modes=0)
    t, o = make_pair(64, 64, 20.0, 0.5, 0.8, 1, **kw)
    t.set_param("precision", 1)
    print("fp32 growth rate", flush=True)
    t.init(seed=0, perturbation=1e-3)
    o.base_state(1500)
    o.perturb(0, 1e-3, False)
    steps, at, ao = [], [], []
    for i in range(13):
        if i:
            t.step(50); o.step(50)
        steps.append(50 * i); at.append(t.amplitude()); ao.append(o.amplitude())
    gt, go = _rate(at[2:], steps[2:]), _rate(ao[2:], steps[2:])
    print(f"gamma fp32 {gt:.6e} oracle {go:.6e}", flush=True)
    assert abs(gt / go - 1) < 1e-3


def test_fp32_checkpoint_and_conservation(tmp_path):
    t, _ = make_pair(64, 32, 20.0, 0.5, 0.8, 1, nq=6, pre_steps=100)
    t.set_param("precision", 1)
    t.init(seed=9, perturbation=0.01)
    d0 = t.diagnostics()
    t.step(10)
    t.save(tmp_path / "c.bin")
    t.step(10)
    a = t.get_state()
    t.load(tmp_path / "c.bin")
    t.step(10)
    b = t.get_state()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    d1 = t.diagnostics()
    # FP32 storage: mass moves only by the rounding of the stored deviations
    assert abs(d1["mass_S"] / d0["mass_S"] - 1) < 1e-8
    assert abs(d1["mass_P"] / d0["mass_P"] - 1) < 1e-8
