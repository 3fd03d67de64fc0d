"""Helpers for the GPU tests: build matching library and oracle lattices from
one configuration, and compare states.  No arithmetic of the method here."""
import numpy as np

import oracle
import paper_2201_10132_amd as P

LIB_KEYS = ("nq", "spring", "b", "phi", "tau_drag", "tau_ratio_p", "force_scale",
            "drift_cap", "drift_relax", "qe_model", "pre_steps", "qsplit", "pert_modes",
            "inplace", "gradients", "spring_shift")


def make_pair(nx, ny, Re, Wi, beta, periods, u0=0.05, **kw):
    lib_kw = {k: v for k, v in kw.items() if k in LIB_KEYS}
    orc_kw = {k: v for k, v in kw.items()
              if k in oracle.oracle.DEFAULTS and k not in ("pre_steps",)}
    t = P.Tpl(nx, ny, Re, Wi, beta, periods=periods, u0=u0, **lib_kw)
    o = oracle.OracleSim(nx, ny, Re=Re, Wi=Wi, beta=beta, periods=periods, u0=u0, **orc_kw)
    return t, o


def max_rel(a, b, floor=0.0):
    """max |a - b| / max(max |b|, floor) (b is the oracle)."""
    a = np.asarray(a, dtype=np.float64); b = np.asarray(b, dtype=np.float64)
    scale = max(float(np.abs(b).max()), floor)
    return float(np.abs(a - b).max() / (scale if scale > 0 else 1.0))


# Scale floor per array: the mixture velocity is a ratio of population sums,
# so its round-off is set by the lattice speed (1), not by |U| itself.
FLOOR = {"XS": 0.0, "XP": 0.0, "psi": 0.0, "U": 1.0}


def compare_states(t_state, o_state, tol, keys=("XS", "XP", "psi", "U")):
    out = {k: max_rel(t_state[k], o_state[k], FLOOR.get(k, 0.0)) for k in keys}
    bad = {k: v for k, v in out.items() if not v <= tol}
    assert not bad, f"parity {out} exceeds {tol}"
    return out
