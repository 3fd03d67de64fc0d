"""Pins of the oracle's equilibria and collision at one node.

P2  moments of the discrete equilibria (Sec. VI.A, VI.B; App. A equilibrium
    moments at linear order).
P3  the explicit g-update equals the trapezoidal rule of Sec. VI.C solved
    implicitly: g' = g + Omega(f) with f the root of g = f - Omega(f)/2,
    Omega(f) = (f* - f)/tau1 + (f_eq - f*)/tau2 built from f's own moments.
P5  the cross-collision exchange cancels: total momentum changes by exactly
    the body force plus the spring force.
"""
import numpy as np
import pytest
from scipy.optimize import root

import oracle
from tests import inputs

CS2 = 1.0 / 3.0


def test_solvent_equilibrium_moments():
    t = oracle.OracleSim(1, 1, nq=4).tables()
    c = t["cS"].astype(float)
    for seed in range(5):
        rho = 0.8 + 0.4 * inputs.rng(seed).random()
        u = inputs.normal(100 + seed, 2, 0.05)
        f = oracle.OracleSim.solvent_eq(rho, *u)
        assert abs(f.sum() - rho) < 1e-15
        assert np.abs(c.T @ f - rho * u).max() < 1e-16
        P = np.einsum("i,ia,ib->ab", f, c, c)
        assert np.abs(P - rho * (CS2 * np.eye(2) + np.outer(u, u))).max() < 1e-15


def test_polymer_equilibrium_moments():
    sim = oracle.OracleSim(1, 1, nq=4)
    t = sim.tables()
    c = t["cP"].astype(float)
    v, qd = c[:, :2], c[:, 2:]
    for seed in range(5):
        psi = 0.01 * (1 + inputs.rng(seed).random())
        Jr = inputs.normal(10 + seed, 2, 1e-3)
        JQ = inputs.normal(20 + seed, 2, 1e-3)
        f = sim.polymer_eq(psi, Jr, JQ)
        assert abs(f.sum() - psi) < 1e-17
        assert np.abs(v.T @ f - Jr).max() < 1e-17
        assert np.abs(qd.T @ f - JQ).max() < 1e-17
        # second moments at linear order: psi c_s^2 I, 0, psi c_s^2 I
        assert np.abs(np.einsum("k,ka,kb->ab", f, v, v) - psi * CS2 * np.eye(2)).max() < 1e-17
        assert np.abs(np.einsum("k,ka,kb->ab", f, v, qd)).max() < 1e-17
        assert np.abs(np.einsum("k,ka,kb->ab", f, qd, qd) - psi * CS2 * np.eye(2)).max() < 1e-17


def _node_inputs(sim, seed):
    t = sim.tables()
    nqd = sim.nqd
    gS = inputs.positive_field(seed, 9, t["wS"] * 0.99, 0.05)
    psi = 0.01 * t["peq"]
    gP = inputs.positive_field(seed + 1, (nqd, 25), psi[:, None] * t["wP"][None, :], 0.05)
    K = inputs.normal(seed + 2, 4, 2e-3)
    sq = inputs.normal(seed + 3, (nqd, 2), 1e-6)
    Fb = np.array([inputs.normal(seed + 4, 1, 1e-5)[0], 0.0])
    return gS, gP, K, sq, Fb


def _implicit_reference(sim, gS, gP, K, sq, Fb):
    """Solve g = f - Omega(f)/2 for f from the definitions, return g + Omega(f).

    Omega's pieces follow Sec. IV-VI: quasi-equilibria about each species' own
    velocity/fluxes, equilibria about the mixture velocity U (solvent:
    shifted by tau2 F / rho_S for the body force), imposed polymer fluxes
    J^r_eq = psi U + s, J^Q_eq = psi (K Q - D_Q Fhat).  U is the velocity for
    which the two species' momentum exchange cancels:
    U = (J_S/tau2_S + J_P/tau2_P) / (rho_S/tau2_S + rho_P/tau2_P)
    (with equal tau2 this is J/rho, the paper's mixture velocity).

    The root is found in float64 and then refined in extended precision
    (x87 long double) so that the reference is accurate well below FP64
    round-off of the explicit update."""
    t = sim.tables()
    d = {k: np.longdouble(v) for k, v in sim.derived().items()}
    nqd = sim.nqd
    L = np.longdouble
    cS = t["cS"].astype(L)
    cP = t["cP"].astype(L)
    v, qd = cP[:, :2], cP[:, 2:]
    wS, wP, Q, Fh = (t["wS"].astype(L), t["wP"].astype(L), t["Q"].astype(L),
                     t["Fhat"].astype(L))
    cs2 = L(1) / L(3)
    gS_, gP_, K_, sq_, Fb_ = (np.asarray(a, dtype=L) for a in (gS, gP, K, sq, Fb))

    def feq2(rho, u):  # Sec. VI.A quadratic equilibrium
        cu = cS @ u
        return wS * rho * (1 + cu / cs2 + cu ** 2 / (2 * cs2 ** 2) - (u @ u) / (2 * cs2))

    def flin(psi, Jr, JQ):  # Sec. VI.B linear equilibrium, psi[nqd], J[nqd,2]
        return wP[None, :] * (psi[:, None] + (Jr @ v.T + JQ @ qd.T) / cs2)

    def omega(fS, fP):
        rhoS = fS.sum(); JS = cS.T @ fS
        psi = fP.sum(1); Jr = fP @ v; JQ = fP @ qd
        rhoP = psi.sum(); JP = Jr.sum(0)
        U = (JS / d["tau2S"] + JP / d["tau2P"]) / (rhoS / d["tau2S"] + rhoP / d["tau2P"])
        fsS = feq2(rhoS, JS / rhoS)
        feS = feq2(rhoS, U + d["tau2S"] * Fb_ / rhoS)
        OmS = (fsS - fS) / d["tau1S"] + (feS - fsS) / d["tau2S"]
        Kmat = K_.reshape(2, 2)
        Jreq = psi[:, None] * U[None, :] + sq_
        JQeq = psi[:, None] * (Q @ Kmat.T - d["DQ"] * Fh)
        fsP = flin(psi, Jr, JQ)
        feP = flin(psi, Jreq, JQeq)
        OmP = (fsP - fP) / d["tau1P"] + (feP - fsP) / d["tau2P"]
        return OmS, OmP

    def resid(x):
        fS, fP = x[:9], x[9:].reshape(nqd, 25)
        OmS, OmP = omega(fS, fP)
        return np.concatenate([fS - OmS / 2 - gS_, (fP - OmP / 2 - gP_).ravel()])

    scale = np.concatenate([np.full(9, 1.0), np.full(25 * nqd, 1e-4)])
    x0 = np.concatenate([gS, gP.ravel()])
    f64 = lambda y: resid((y * scale).astype(L)).astype(np.float64) / scale  # noqa: E731
    sol = root(f64, x0 / scale, method="hybr", tol=1e-14)
    y = sol.x
    # Jacobian of the scaled residual (central differences, float64)
    n = y.size
    J = np.empty((n, n))
    h = 1e-6
    for j in range(n):
        e = np.zeros(n); e[j] = h
        J[:, j] = (f64(y + e) - f64(y - e)) / (2 * h)
    x = (y * scale).astype(L)
    for _ in range(6):  # iterative refinement with a long-double residual
        r = resid(x) / scale.astype(L)
        x = x - np.linalg.solve(J, r.astype(np.float64)).astype(L) * scale.astype(L)
    assert np.abs(resid(x) / scale.astype(L)).max() < 1e-16
    fS, fP = x[:9], x[9:].reshape(nqd, 25)
    OmS, OmP = omega(fS, fP)
    return gS_ + OmS, gP_ + OmP


@pytest.mark.parametrize("case", [
    dict(tau_drag=1.0, spring=0),          # species-specific tau2 (reading)
    dict(tau_drag=1.0, spring=1, tau_ratio_p=0.5),
])
def test_explicit_update_equals_implicit_trapezoid(case):
    # ny_param/lambda_set give tau's of order 0.1, where the implicit solve is
    # well conditioned (its error grows like 1/tau1)
    sim = oracle.OracleSim(1, 1, nq=4, Re=20.0, Wi=0.5, beta=0.8, ny_param=64,
                           lambda_set=1.2, **case)
    for seed in (1, 7):
        gS, gP, K, sq, Fb = _node_inputs(sim, seed)
        oS, oP, _ = sim.collide_node(gS, gP, K, sq, Fb)
        rS, rP = _implicit_reference(sim, gS, gP, K, sq, Fb)
        assert float(np.abs(oS - rS).max()) <= 1e-14 * float(np.abs(rS).max())
        assert float(np.abs(oP - rP).max()) <= 1e-14 * float(np.abs(rP).max())


def test_explicit_update_equals_implicit_trapezoid_equal_tau():
    """With tau2_S = tau2_P the mixture velocity is the paper's plain J/rho."""
    probe = oracle.OracleSim(1, 1, nq=4, Re=20.0, Wi=0.5, beta=0.8, ny_param=64,
                             lambda_set=1.2, spring=1)
    sim = oracle.OracleSim(1, 1, nq=4, Re=20.0, Wi=0.5, beta=0.8, ny_param=64,
                           lambda_set=1.2, spring=1, tau_drag=probe.derived()["tau2P"])
    d = sim.derived()
    assert abs(d["tau2S"] - d["tau2P"]) < 1e-15 and d["tau1S"] <= d["tau2S"]
    gS, gP, K, sq, Fb = _node_inputs(sim, 3)
    oS, oP, U = sim.collide_node(gS, gP, K, sq, Fb)
    rS, rP = _implicit_reference(sim, gS, gP, K, sq, Fb)
    assert float(np.abs(oS - rS).max()) <= 1e-14 * float(np.abs(rS).max())
    assert float(np.abs(oP - rP).max()) <= 1e-14 * float(np.abs(rP).max())


def test_momentum_exchange_cancels_and_mass_is_local():
    sim = oracle.OracleSim(1, 1, nq=6, ny_param=64)
    t = sim.tables(); d = sim.derived()
    cS = t["cS"].astype(float); v = t["cP"][:, :2].astype(float)
    for seed in (11, 12, 13):
        gS, gP, K, sq, Fb = _node_inputs(sim, seed)
        oS, oP, U = sim.collide_node(gS, gP, K, sq, Fb)
        # mass per species, and per Q-node for the polymer
        assert abs(oS.sum() - gS.sum()) <= 1e-15 * gS.sum()
        assert np.abs(oP.sum(1) - gP.sum(1)).max() <= 1e-15 * gP.sum(1).max()
        before = cS.T @ gS + (gP @ v).sum(0)
        after = cS.T @ oS + (oP @ v).sum(0)
        expected = Fb + sq.sum(0) / d["tau2P"]
        # round-off of O(10) operations on momenta of size |before|
        assert np.abs(after - before - expected).max() <= 1e-14 * np.abs(before).max()
