"""The BF16 non-equilibrium form: solvent and psi as FP32 deviations from
the FP32-rounded base state; per polymer (r, Q)-node FP32 moments of the
deviations delta (density m0 and fluxes J^r, J^Q) and, per population, a
BF16 remainder n_k = delta_k - w_k (m0 + 3 (v_k . J)); the stored moments
are corrected by the rounded remainders' own moments, so the reconstructed
node keeps its exact density and fluxes.  Arithmetic in FP64.

Error model: every step rounds each remainder to BF16 (round to nearest
even, relative 2^-9; the moment correction spreads that error over the
node's populations, at most doubling it) and the moments and psi to FP32
(2^-24 of their deviations); the scheme is dissipative, so after n steps
the difference from the FP64 oracle is bounded by about
n (2 2^-9 max|remainder| + 2^-24 max|delta|), tested with a factor 4 margin.
The remainders are evaluated from the oracle's own state against the FP32
rounding of its base state (the library's reference is the FP32 rounding of
its own base state, which agrees with the oracle's to ~1e-13).
"""
import numpy as np
import pytest

import oracle
import paper_2201_10132_amd as P
from tests.gpu_common import make_pair

pytestmark = pytest.mark.gpu

EPS32, EPS_BF16 = 2.0 ** -24, 2.0 ** -9
PVEL = [(0, 0, 0, 0)]
for (a, b) in [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]:
    for sa, sb in [(1, 1), (1, -1), (-1, 1), (-1, -1)]:
        v = [0, 0, 0, 0]
        v[a], v[b] = sa, sb
        PVEL.append(tuple(v))
W25 = np.array([1.0 / 3.0] + [1.0 / 36.0] * 24)


def _remainder_max(st, base):
    """max |n_k| of a state against the FP32-rounded base state."""
    d = st["XP"] - base["XP"].astype(np.float32).astype(np.float64)  # [25][nqd][ny][nx]
    m0 = d.sum(axis=0)
    V = np.array(PVEL, dtype=np.float64)               # [25][4]
    J = np.einsum("kc,kqyx->cqyx", V, d)
    lin = W25[:, None, None, None] * (m0[None] + 3.0 * np.einsum("kc,cqyx->kqyx", V, J))
    return np.abs(d - lin).max(), np.abs(d).max()


def _bound(n, states, base):
    rem = max(_remainder_max(s, base)[0] for s in states)
    dev = max(_remainder_max(s, base)[1] for s in states)
    return 4 * n * (2 * EPS_BF16 * rem + 4 * EPS32 * dev)


@pytest.mark.parametrize("nx,ny,nq,spring", [(64, 16, 6, 0), (14, 9, 4, 1), (128, 8, 4, 0)])
def test_neq_parity_with_oracle(nx, ny, nq, spring):
    t, o = make_pair(nx, ny, 20.0, 0.5, 0.8, 2 if ny >= 8 else 1, nq=nq, spring=spring,
                     pre_steps=300, pert_modes=1)
    t.set_param("precision", P.TPL_BF16NEQ)
    print(f"bf16-neq parity {nx}x{ny} nq={nq} spring={spring}", flush=True)
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
    errs = {k: float(np.abs(got[k] - want[k]).max()) for k in ("XS", "XP", "psi")}
    print("errors", errs, "bound", bound, flush=True)
    for k, e in errs.items():
        assert e <= bound, (k, e, bound)


def _rate(amps, steps):
    return np.polyfit(steps, np.log(amps), 1)[0]


def test_neq_growth_rate_close_to_oracle():
    """64 x 64, one forcing period (decaying perturbation), NQ = 8: the
    decay rate of the amplitude against the oracle's."""
    kw = dict(nq=8, pre_steps=1500, pert_modes=0)
    t, o = make_pair(64, 64, 20.0, 0.5, 0.8, 1, **kw)
    t.set_param("precision", P.TPL_BF16NEQ)
    t.init(seed=0, perturbation=1e-3)
    o.base_state(1500)
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
    print(f"gamma bf16-neq {gt:.6e} oracle {go:.6e} rel {abs(gt / go - 1):.2e}", flush=True)
    assert abs(gt / go - 1) < 1e-2


def test_neq_checkpoint_conservation_and_state_exchange(tmp_path):
    t, _ = make_pair(64, 32, 20.0, 0.5, 0.8, 1, nq=6, pre_steps=100)
    t.set_param("precision", P.TPL_BF16NEQ)
    t.init(seed=9, perturbation=0.01)
    d0 = t.diagnostics()
    t.step(20)
    path = str(tmp_path / "neq.ckpt")
    t.save(path)
    t.step(15)
    a = t.get_state()
    t.load(path)
    t.step(15)
    b = t.get_state()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    d1 = t.diagnostics()
    # mass: the solvent as in the FP32 form; the polymer's density is carried
    # by its FP32 moment m0 (the remainders' rounding is compensated)
    print("mass drift", d1["mass_S"] / d0["mass_S"] - 1, d1["mass_P"] / d0["mass_P"] - 1, flush=True)
    assert abs(d1["mass_S"] / d0["mass_S"] - 1) < 1e-8
    assert abs(d1["mass_P"] / d0["mass_P"] - 1) < 1e-10
    # state exchange: writing back what was read changes the polymer
    # populations by at most the re-encoding (a BF16 rounding of remainders,
    # spread by the moment correction: 2 2^-9 of the remainders, which stay
    # below 1e-2 of the populations for this 1e-2 perturbation); the rest
    # only by FP32 conversions
    st = t.get_state()
    t.set_state(**st)
    st2 = t.get_state()
    for k in ("XS", "psi"):
        assert np.abs(st2[k] - st[k]).max() <= 1e-15 * np.abs(st[k]).max(), k
    e = np.abs(st2["XP"] - st["XP"]).max() / np.abs(st["XP"]).max()
    print("re-encoding", e, flush=True)
    assert e <= 2 * EPS_BF16 * 1e-2
