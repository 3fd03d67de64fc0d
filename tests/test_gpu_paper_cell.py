"""The paper's own Kolmogorov cell (Sec. VII) against the oracle at its own
parameters: 72 x 72 lattice holding four forcing periods, Re = 3.5,
beta = 0.5, FENE dumbbells with b = 25 on a 32-point Q-grid (812 Q-nodes),
Wi = 0.1, 2.5 and 5, from rest with the seeded multimode perturbation of
the experiment driver (u0 = 0.01, Q-drift cap 0.2), the three cells as one
batch in the launch shape the driver uses.  Every population, psi and U of
the whole lattice is compared after 20 steps (FP64: 1e-12, the tolerance of
the other batched parity tests)."""
import pytest

import oracle
import paper_2201_10132_amd as P
from paper_2201_10132_amd import kolmogorov72 as K
from tests.gpu_common import compare_states

pytestmark = pytest.mark.gpu


def test_paper_cell_matches_oracle_at_its_own_parameters():
    insts = [dict(K.CELL, Wi=w, seed=0, perturbation=1e-3) for w in K.WIS]
    b = P.Batch(insts, precision=P.TPL_FP64, nq=32, pre_steps=0, drift_cap=K.DRIFT_CAP)
    b.init()
    assert b.instance(0).nqd == 812
    b.step(20)
    for i, w in enumerate(K.WIS):
        print(f"paper cell Wi {w}: oracle 20 steps", flush=True)
        o = oracle.OracleSim(72, 72, nq=32, periods=K.CELL["periods"], Re=K.CELL["Re"], Wi=w,
                             beta=K.CELL["beta"], u0=K.CELL["u0"], drift_cap=K.DRIFT_CAP)
        o.base_state(0)
        o.perturb(0, 1e-3, True)
        o.step(20)
        compare_states(b.instance(i).get_state(), o.get_state(), 1e-12)
        # the observables of the last step, all ten fields
        # (each field against its natural scale: the stress
        # G (M / (rho_P0 m_eq) - I) cancels against G, so G; the velocity, a
        # ratio of population sums whose round-off is set by the lattice
        # speed, u0, as in the state comparison; the conformation, whose
        # components are ratios of psi-weighted sums, its rest value 1)
        got, want = b.instance(i).moments(), o.observables()
        scale = abs(want).max(axis=(1, 2))
        G = b.instance(i).query("G")
        floors = [0.0, K.CELL["u0"], K.CELL["u0"], 0.0, 1.0, 1.0, 1.0, G, G, G]
        for f in range(10):
            floor = floors[f]
            assert abs(got[f] - want[f]).max() <= 1e-12 * max(scale[f], floor), (w, f)
        del o
    b.close()
