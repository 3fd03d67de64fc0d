"""The BF16 form: solvent and psi as FP32 deviations from the FP32-rounded
base state (as the FP32 form), the polymer populations as the BF16 rounding
(nearest even, 8 significant bits: relative error at most 2^-8) of their
deviation from it.
Arithmetic in FP64.

The rest population (velocity 0, which never leaves its node) is stored in
FP32 and takes up the BF16 rounding residual of the node's other 24, so the
stored density of every (r, Q)-node, and the polymer mass, are exact to FP32.

Error model: every step rounds each polymer deviation to BF16 (2^-8 of its
size) and the solvent's and psi to FP32 (2^-24); the scheme is dissipative,
so after n steps the difference from the FP64 oracle is bounded by about
n (2^-8 max|delta_P| + 2^-24 max|delta|), tested with a factor 4 margin.
The deviations delta are evaluated from the oracle's own states against the
FP32 rounding of its base state (the library's reference is the FP32
rounding of its own base state, which agrees with the oracle's to ~1e-13).
So the error is set by how far the state has moved from the reference: a
perturbed, converged base state keeps it small."""
import numpy as np
import pytest

import oracle
import paper_2201_10132_amd as P
from tests.gpu_common import make_pair

pytestmark = pytest.mark.gpu

EPS32, EPS_BF16 = 2.0 ** -24, 2.0 ** -8  # unit roundoffs: 24 and 8 significant bits
# polymer mass error allowed over ~100 steps: FP32 rounding of the
# deviations gives ~1e-11, BF16 rounding without the rest population's
# residual ~2^16 times that
MASS_BAR = 1e-9


def _dev(st, base):
    return (np.abs(st["XP"] - base["XP"].astype(np.float32).astype(np.float64)).max(),
            max(np.abs(st[k] - base[k].astype(np.float32).astype(np.float64)).max()
                for k in ("XS", "psi")))


def _bound(n, states, base):
    dp = max(_dev(s, base)[0] for s in states)
    dd = max(max(_dev(s, base)) for s in states)
    return 4 * n * (EPS_BF16 * dp + 4 * EPS32 * dd)


@pytest.mark.parametrize("nx,ny,nq,spring", [(64, 16, 6, 0), (14, 9, 4, 1), (128, 8, 4, 0)])
def test_bf16_parity_with_oracle(nx, ny, nq, spring):
    t, o = make_pair(nx, ny, 20.0, 0.5, 0.8, 2 if ny >= 8 else 1, nq=nq, spring=spring,
                     pre_steps=300, pert_modes=1)
    t.set_param("precision", P.TPL_BF16)
    print(f"bf16 parity {nx}x{ny} nq={nq} spring={spring}", flush=True)
    t.init(seed=4, perturbation=0.02)
    o.base_state(300)
    base = o.get_state()
    o.perturb(4, 0.02, True)
    want0 = o.get_state()
    n = 100
    t.step(n)
    o.step(n)
    got, want = t.get_state(), o.get_state()
    bound = _bound(n + 1, [want0, want], base)
    errs = {k: float(np.abs(got[k] - want[k]).max()) for k in ("XS", "psi")}
    errs["XP moving"] = float(np.abs(got["XP"][1:] - want["XP"][1:]).max())
    # the rest population carries the rounding residual of the node's other
    # 24 populations (a sum of 24 roundings: about sqrt(24) of one), bound 6x
    errs["XP rest"] = float(np.abs(got["XP"][0] - want["XP"][0]).max()) / 6
    print("errors", errs, "bound", bound, flush=True)
    for k, e in errs.items():
        assert e <= bound, (k, e, bound)
    # the node densities, and the lattice's polymer mass, are kept to FP32:
    # about 1e-11 after these 100 steps (measured 1.3e-11 on the smallest
    # lattice), where BF16 rounding of every deviation would move it 2^16
    # times as far; the bar sits between the two
    dm = abs(got["XP"].sum() / want["XP"].sum() - 1)
    print("polymer mass against the oracle", dm, flush=True)
    assert dm < MASS_BAR


def _rate(amps, steps):
    return np.polyfit(steps, np.log(amps), 1)[0]


def test_bf16_decay_rate_close_to_oracle_from_a_converged_base_state():
    """64 x 64, one forcing period (decaying perturbation), NQ = 8, from the
    library's default (converged) base state: the decay rate of the
    amplitude against the oracle's."""
    kw = dict(nq=8, pre_steps=-1, pert_modes=0)
    t, o = make_pair(64, 64, 20.0, 0.5, 0.8, 1, **kw)
    t.set_param("precision", P.TPL_BF16)
    t.init(seed=0, perturbation=1e-3)
    o.base_state(-1)
    o.perturb(0, 1e-3, False)
    steps, at, ao = [], [], []
    for i in range(13):
        if i:
            t.step(50)
            o.step(50)
        steps.append(50 * i)
        at.append(t.amplitude())
        ao.append(o.amplitude())
    gt, go = _rate(at[2:], steps[2:]), _rate(ao[2:], steps[2:])
    print(f"gamma bf16 {gt:.6e} oracle {go:.6e} rel {abs(gt / go - 1):.2e}", flush=True)
    assert abs(gt / go - 1) < 1e-3


def test_bf16_checkpoint_conservation_and_state_exchange(tmp_path):
    t, _ = make_pair(64, 32, 20.0, 0.5, 0.8, 1, nq=6, pre_steps=100)
    t.set_param("precision", P.TPL_BF16)
    t.init(seed=9, perturbation=0.01)
    d0 = t.diagnostics()
    t.step(20)
    path = str(tmp_path / "bf16.ckpt")
    t.save(path)
    t.step(15)
    a = t.get_state()
    t.load(path)
    t.step(15)
    b = t.get_state()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    d1 = t.diagnostics()
    # mass: the solvent as in the FP32 form; the polymer's too, since the
    # rest population stored in FP32 takes up every node's BF16 rounding
    # residual (35 steps of FP32 rounding of the deviations)
    print("mass drift", d1["mass_S"] / d0["mass_S"] - 1, d1["mass_P"] / d0["mass_P"] - 1, flush=True)
    assert abs(d1["mass_S"] / d0["mass_S"] - 1) < 1e-8
    assert abs(d1["mass_P"] / d0["mass_P"] - 1) < MASS_BAR
    # state exchange: writing back what was read re-rounds nothing (the
    # stored values are exactly representable)
    st = t.get_state()
    t.set_state(**st)
    st2 = t.get_state()
    for k in ("XS", "psi", "XP"):
        assert np.abs(st2[k] - st[k]).max() <= 1e-15 * np.abs(st[k]).max(), k
