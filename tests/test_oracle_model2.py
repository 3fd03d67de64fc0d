"""Pins of the oracle's stress-tensor quasi-equilibrium model (Sec. V,
model (ii)): the component stresses are quasi-conserved, momenta relax with
tau1 and stresses with tau2, so the viscosity is c_s^2 tau2 and the drag and
the diffusivities follow tau1.

P2b  the second-order Hermite quasi-equilibria carry exactly the density,
     first and second moments they are built from (brute-force lattice sums).
P3b  the explicit g-update equals the trapezoidal rule solved implicitly,
     Omega(f) = (f* - f)/tau1 + (f_eq - f*)/tau2 with f* built from f's own
     stresses (the same extended-precision solve as P3).
P5b  momentum exchange cancels: total momentum changes by the body force
     plus the spring force S / tau1_P.
P6b  solvent shear-wave decay at nu = c_s^2 tau2_S, second order in L.
P7b  dilute polymer density diffusion at D = c_s^2 tau1_P.
P8b  Hookean conformation relaxation at lambda with D_Q = c_s^2 tau1_P.
P9b  Hookean laminar Kolmogorov state against the Oldroyd-B closed form.
     With tau1 = tau2 for both species both models reduce to one BGK
     relaxation: the runs agree to round-off.
"""
import numpy as np
import pytest
from scipy.optimize import root

import oracle
from tests import inputs
from tests.test_oracle_collision import _node_inputs
from tests.test_oracle_physics import _cos_amp, _sin_amp

CS2 = 1.0 / 3.0


def _hermite2(w, xi, rho, J, P, cs2):
    """w_k [rho + J.xi_k / c_s^2 + (P - rho c_s^2 I):(xi_k xi_k - c_s^2 I)/(2 c_s^4)]."""
    d = xi.shape[1]
    I = np.eye(d, dtype=xi.dtype)
    H = np.einsum("ka,kb->kab", xi, xi) - cs2 * I[None]
    D = P - rho * cs2 * I
    return w * (rho + xi @ J / cs2 + np.einsum("kab,ab->k", H, D) / (2 * cs2 * cs2))


def test_quasi_equilibria_carry_their_moments():
    sim = oracle.OracleSim(1, 1, nq=6, qe_model=2, tau_drag=0.01, ny_param=64)
    t = sim.tables()
    cS = t["cS"].astype(float); cP = t["cP"].astype(float)
    rng = np.random.default_rng(5)
    for _ in range(3):
        rho = 1 + 0.1 * rng.random()
        J = 0.05 * rng.standard_normal(2)
        A = 0.02 * rng.standard_normal((2, 2))
        P = rho * CS2 * np.eye(2) + A + A.T
        f = sim.solvent_qe2(rho, J, [P[0, 0], P[0, 1], P[1, 1]])
        assert abs(f.sum() - rho) < 1e-15
        assert np.abs(cS.T @ f - J).max() < 1e-15
        assert np.abs(np.einsum("i,ia,ib->ab", f, cS, cS) - P).max() < 1e-15
        psi = 0.01 * rng.random()
        J4 = 1e-3 * rng.standard_normal(4)
        A = 1e-3 * rng.standard_normal((4, 4))
        P4 = psi * CS2 * np.eye(4) + A + A.T
        f = sim.polymer_qe2(psi, J4, P4[np.triu_indices(4)])
        assert abs(f.sum() - psi) < 1e-16
        assert np.abs(cP.T @ f - J4).max() < 1e-17
        assert np.abs(np.einsum("k,ka,kb->ab", f, cP, cP) - P4).max() < 1e-17


def _implicit_reference2(sim, gS, gP, K, sq, Fb):
    """Model (ii): solve g = f - Omega(f)/2 for f, return g + Omega(f), in
    extended precision (as P3)."""
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

    def omega(fS, fP):
        rhoS = fS.sum(); JS = cS.T @ fS; PS = np.einsum("i,ia,ib->ab", fS, cS, cS)
        psi = fP.sum(1); Jr = fP @ v; JQ = fP @ qd
        rhoP = psi.sum(); JP = Jr.sum(0)
        # momenta relax with tau1: the exchange cancels at
        U = (JS / d["tau1S"] + JP / d["tau1P"]) / (rhoS / d["tau1S"] + rhoP / d["tau1P"])
        vS = U + d["tau1S"] * Fb_ / rhoS
        fsS = _hermite2(wS, cS, rhoS, rhoS * vS, PS, cs2)
        feS = feq2(rhoS, vS)
        OmS = (fsS - fS) / d["tau1S"] + (feS - fsS) / d["tau2S"]
        Kmat = K_.reshape(2, 2)
        Jreq = psi[:, None] * U[None, :] + sq_
        JQeq = psi[:, None] * (Q @ Kmat.T - d["DQ"] * Fh)
        OmP = np.empty_like(fP)
        for q in range(nqd):
            J4 = np.concatenate([Jreq[q], JQeq[q]])
            P4 = np.einsum("k,ka,kb->ab", fP[q], cP, cP)
            fss = _hermite2(wP, cP, psi[q], J4, P4, cs2)
            fe = wP * (psi[q] + cP @ J4 / cs2)
            OmP[q] = (fss - fP[q]) / d["tau1P"] + (fe - fss) / d["tau2P"]
        return OmS, OmP

    def resid(x):
        fS, fP = x[:9], x[9:].reshape(nqd, 25)
        OmS, OmP = omega(fS, fP)
        return np.concatenate([fS - OmS / 2 - gS_, (fP - OmP / 2 - gP_).ravel()])

    scale = np.concatenate([np.full(9, 1.0), np.full(25 * nqd, 1e-4)])
    x0 = np.concatenate([gS, gP.ravel()])
    f64 = lambda y: resid((y * scale).astype(L)).astype(np.float64) / scale  # noqa: E731
    y = root(f64, x0 / scale, method="hybr", tol=1e-14).x
    n = y.size
    Jm = np.empty((n, n))
    h = 1e-6
    for j in range(n):
        e = np.zeros(n); e[j] = h
        Jm[:, j] = (f64(y + e) - f64(y - e)) / (2 * h)
    x = (y * scale).astype(L)
    for _ in range(6):
        r = resid(x) / scale.astype(L)
        x = x - np.linalg.solve(Jm, r.astype(np.float64)).astype(L) * scale.astype(L)
    assert np.abs(resid(x) / scale.astype(L)).max() < 1e-16
    fS, fP = x[:9], x[9:].reshape(nqd, 25)
    OmS, OmP = omega(fS, fP)
    return gS_ + OmS, gP_ + OmP


@pytest.mark.parametrize("case", [dict(spring=0, tau_ratio_p=0.5), dict(spring=1, tau_ratio_p=1.0)])
def test_explicit_update_equals_implicit_trapezoid_model2(case):
    sim = oracle.OracleSim(1, 1, nq=4, Re=20.0, Wi=0.5, beta=0.8, ny_param=64, lambda_set=1.2,
                           qe_model=2, tau_drag=0.03, **case)
    d = sim.derived()
    assert d["tau1S"] == 0.03 and d["tau2S"] > d["tau1S"] and d["tau2P"] >= d["tau1P"]
    for seed in (2, 9):
        gS, gP, K, sq, Fb = _node_inputs(sim, seed)
        oS, oP, _ = sim.collide_node(gS, gP, K, sq, Fb)
        rS, rP = _implicit_reference2(sim, gS, gP, K, sq, Fb)
        assert float(np.abs(oS - rS).max()) <= 1e-14 * float(np.abs(rS).max())
        assert float(np.abs(oP - rP).max()) <= 1e-14 * float(np.abs(rP).max())


def test_momentum_exchange_cancels_model2():
    sim = oracle.OracleSim(1, 1, nq=6, ny_param=64, qe_model=2, tau_drag=0.05, tau_ratio_p=0.7)
    t = sim.tables(); d = sim.derived()
    cS = t["cS"].astype(float); v = t["cP"][:, :2].astype(float)
    for seed in (21, 22):
        gS, gP, K, sq, Fb = _node_inputs(sim, seed)
        oS, oP, U = sim.collide_node(gS, gP, K, sq, Fb)
        assert abs(oS.sum() - gS.sum()) <= 1e-15 * gS.sum()
        assert np.abs(oP.sum(1) - gP.sum(1)).max() <= 1e-15 * gP.sum(1).max()
        before = cS.T @ gS + (gP @ v).sum(0)
        after = cS.T @ oS + (oP @ v).sum(0)
        expected = Fb + sq.sum(0) / d["tau1P"]
        assert np.abs(after - before - expected).max() <= 1e-14 * np.abs(before).max()


def _shear_wave_error2(L, nu=0.05, A=1e-4, n1=100, n2=600):
    l = L / (2 * np.pi)
    sim = oracle.OracleSim(1, L, nq=4, phi=0.0, Wi=0.0, Re=0.05 * l / nu, force_scale=0.0,
                           qe_model=2, tau_drag=0.02)
    d = sim.derived()
    assert abs(d["tau2S"] * CS2 - nu) < 1e-15 and d["tau1S"] == 0.02
    y = np.arange(L)
    u = A * np.sin(2 * np.pi * y / L)
    XS = np.stack([oracle.OracleSim.solvent_eq(1.0, uj, 0.0) for uj in u], axis=1)[:, :, None]
    U = np.zeros((2, L, 1)); U[0, :, 0] = u
    sim.set_state(XS=XS, XP=np.zeros((25, sim.nqd, L, 1)), psi=np.zeros((sim.nqd, L, 1)), U=U)
    k = 2 * np.pi / L
    sim.step(n1); a1 = _sin_amp(sim.get_state()["U"][0, :, 0], k, y)
    sim.step(n2 - n1); a2 = _sin_amp(sim.get_state()["U"][0, :, 0], k, y)
    return -np.log(a2 / a1) / (n2 - n1) / (nu * k * k) - 1.0


def test_shear_wave_viscosity_follows_tau2():
    e = {L: _shear_wave_error2(L) for L in (32, 64, 128)}
    assert abs(e[64]) < 1e-3
    assert 3.5 < e[32] / e[64] < 4.5 and 3.5 < e[64] / e[128] < 4.5


def _polymer_diffusion_error2(L, tau1=0.25, eps=1e-3, n1=50, n2=1050):
    sig2 = oracle.OracleSim(1, 1, nq=4, spring=1).derived()["sigma"] ** 2
    sim = oracle.OracleSim(L, 1, nq=4, spring=1, Wi=0.0, phi=1e-6, force_scale=0.0,
                           lambda_set=3 * sig2 / (2 * tau1), ny_param=64, qe_model=2,
                           tau_drag=0.05, tau_ratio_p=0.5)
    d = sim.derived(); t = sim.tables()
    assert abs(d["tau1P"] - tau1) < 1e-14 and abs(d["tau2P"] - 2 * tau1) < 1e-14
    x = np.arange(L)
    psi = d["rhoP0"] * t["peq"][:, None, None] * (1 + eps * np.sin(2 * np.pi * x / L))[None, None, :]
    XS = np.broadcast_to(oracle.OracleSim.solvent_eq(d["rhoS0"], 0, 0)[:, None, None], (9, 1, L))
    sim.set_state(XS=XS, XP=t["wP"][:, None, None, None] * psi[None], psi=psi,
                  U=np.zeros((2, 1, L)))
    k = 2 * np.pi / L
    sim.step(n1); a1 = _sin_amp(sim.observables()[3, 0, :], k, x)
    sim.step(n2 - n1); a2 = _sin_amp(sim.observables()[3, 0, :], k, x)
    return -np.log(a2 / a1) / (n2 - n1) / (CS2 * tau1 * k * k) - 1.0


def test_polymer_density_diffusion_follows_tau1():
    e32, e64 = _polymer_diffusion_error2(32), _polymer_diffusion_error2(64)
    assert abs(e64) < 1e-3
    assert 3.5 < e32 / e64 < 4.5


def test_conformation_relaxation_time_model2():
    nq, tau1 = 16, 0.0768
    sig2 = oracle.OracleSim(1, 1, nq=nq, spring=1).derived()["sigma"] ** 2
    lam = 3 * sig2 / (2 * tau1)
    sim = oracle.OracleSim(1, 1, nq=nq, spring=1, Wi=0.0, force_scale=0.0, lambda_set=lam,
                           ny_param=64, qe_model=2, tau_drag=0.05, tau_ratio_p=0.5)
    d = sim.derived(); t = sim.tables(); Q = t["Q"]
    p = np.exp(-Q[:, 0] ** 2 / (2 * 1.5 * sig2) - Q[:, 1] ** 2 / (2 * 0.75 * sig2))
    psi = d["rhoP0"] * (p / p.sum())[:, None, None]
    XS = oracle.OracleSim.solvent_eq(d["rhoS0"], 0, 0)[:, None, None]
    sim.set_state(XS=XS, XP=t["wP"][:, None, None, None] * psi[None], psi=psi,
                  U=np.zeros((2, 1, 1)))

    def aniso():
        o = sim.observables()
        return o[4, 0, 0] - o[6, 0, 0]
    n1, n2 = int(0.4 * lam), int(4 * lam)
    sim.step(n1); a1 = aniso()
    sim.step(n2 - n1); a2 = aniso()
    assert abs(-np.log(a2 / a1) / (n2 - n1) * d["lambda"] - 1.0) < 1e-2


def test_laminar_oldroyd_b_profile_model2():
    """As P9 with the model's transport coefficients: eta_s = rho_S c_s^2
    tau2_S, kinetic polymer part rho_P c_s^2 tau2_P, r-diffusion D = c_s^2
    tau1_P."""
    ny = 64
    sim = oracle.OracleSim(1, ny, nq=16, spring=1, Re=5.0, Wi=0.5, beta=0.8, periods=1,
                           qe_model=2, tau_drag=0.1, tau_ratio_p=0.5)
    d = sim.derived()
    sim.rest()
    sim.step(int(12 * max(d["l"] ** 2 / d["nu"], d["lambda"])))
    o = sim.observables()
    y = np.arange(ny); k = d["kf"]; lam = d["lambda"]
    Dk = lam * CS2 * d["tau1P"] * k * k
    eta = d["rhoS0"] * CS2 * d["tau2S"] + d["rhoP0"] * CS2 * d["tau2P"] + d["G"] * lam / (1 + Dk)
    UL_c = d["F0"] / (k * k * eta)
    UL = _sin_amp(o[1, :, 0], k, y)
    assert abs(UL / UL_c - 1) < 2e-3
    Cxy = _cos_amp(o[5, :, 0], k, y)
    assert abs(Cxy / (lam * UL * k / (1 + Dk)) - 1) < 2e-3
    dxx = o[4, :, 0] - o[6, :, 0]
    m0 = lam ** 2 * UL ** 2 * k * k / (1 + Dk)
    assert abs(dxx.mean() / m0 - 1) < 3e-3


def test_models_agree_when_tau1_equals_tau2():
    """tau1 = tau2 for both species: both models are one BGK relaxation to
    the same equilibria, so a perturbed FENE run agrees to round-off."""
    base = dict(nq=6, Re=20.0, Wi=0.5, beta=0.8, periods=1, tau_ratio_p=1.0)
    nuS = oracle.OracleSim(12, 16, **base).derived()["nuS"]
    runs = []
    for m in (1, 2):
        o = oracle.OracleSim(12, 16, qe_model=m, tau_drag=nuS / CS2, **base)
        d = o.derived()
        assert abs(d["tau1S"] - d["tau2S"]) < 1e-15 and abs(d["tau1P"] - d["tau2P"]) < 1e-15
        o.base_state(100)
        o.perturb(4, 1e-2, True)
        o.step(50)
        runs.append(o.get_state())
    for k in runs[0]:
        a, b = runs[0][k], runs[1][k]
        assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max(), k


def test_conservation_on_lattice_model2():
    tau2S = oracle.OracleSim(16, 16, nq=6).derived()["nuS"] / CS2
    sim = oracle.OracleSim(16, 16, nq=6, qe_model=2, tau_drag=0.5 * tau2S, tau_ratio_p=0.5)
    sim.base_state(300)
    sim.perturb(seed=3, amp=0.05, multimode=True)
    d0 = sim.diagnostics()
    sim.step(200)
    d1 = sim.diagnostics()
    assert abs(d1["mass_S"] / d0["mass_S"] - 1) < 1e-13
    assert abs(d1["mass_P"] / d0["mass_P"] - 1) < 1e-13
    for c in ("mom_x", "mom_y"):
        assert abs(d1[c] - d0[c]) < 1e-12 * d0["mass_S"] * 0.05


def test_model2_parameter_errors():
    with pytest.raises(ValueError):
        oracle.OracleSim(4, 4, qe_model=3)
    with pytest.raises(ValueError):  # drag time above the viscous time
        oracle.OracleSim(4, 4, qe_model=2, tau_drag=10.0)
