"""Pins of the oracle against what the paper and closed forms fix.

P4/P5  mass of each species and total momentum conserved on a lattice run.
P6     solvent shear-wave decay at nu = c_s^2 tau1 (Sec. IV: viscosity is
       proportional to tau1), second-order convergence in L.
P7     polymer density diffusion with D = c_s^2 tau2_P in the dilute limit
       (App. A, density diffusion equation).
P8     homogeneous Hookean conformation relaxation C - I ~ exp(-t/lambda)
       (App. A, homogeneous Smoluchowski equation), converging with NQ.
P9     forced laminar Kolmogorov state with Hookean dumbbells against the
       Oldroyd-B closed form (Sec. VII forcing; Sec. III elastic stress).
P12    x-invariance: with no perturbation the amplitude stays at round-off.
P14    the parameter mapping gives the paper's Schmidt-number range (Sec. VII).
Rest distributions: the sampled FENE and Hookean equilibria on the Q-disk
       give the closed-form RMS extensions (sqrt(2 / (b + 4)) and the
       truncated Gaussian's) of the spring laws (Sec. VI.C, VII).
Same-step gradients (the reading of the gradients' time level that takes
this step's observables): the invariants and the laminar closed form as
above, and a step that ignores the recorded fields.
"""
import numpy as np
import pytest

import oracle
from tests import inputs

CS2 = 1.0 / 3.0


def _sin_amp(f, k, x):
    return 2.0 / len(x) * np.sum(f * np.sin(k * x))


def _cos_amp(f, k, x):
    return 2.0 / len(x) * np.sum(f * np.cos(k * x))


def _abs_momentum(sim):
    st = sim.get_state()
    t = sim.tables()
    cS = t["cS"].astype(float); v = t["cP"][:, :2].astype(float)
    J = np.einsum("ia,iyx->ayx", cS, st["XS"]) + np.einsum("ka,kqyx->ayx", v, st["XP"])
    return np.sqrt((J ** 2).sum(0)).sum()


@pytest.mark.parametrize("gradients", [0, 1])
@pytest.mark.parametrize("spring", [0, 1])
def test_conservation_on_lattice(spring, gradients):
    sim = oracle.OracleSim(16, 16, nq=6, spring=spring, gradients=gradients)
    sim.base_state(300)
    sim.perturb(seed=3, amp=0.05, multimode=True)
    d0 = sim.diagnostics()
    pabs = _abs_momentum(sim)
    sim.step(200)
    d1 = sim.diagnostics()
    assert abs(d1["mass_S"] / d0["mass_S"] - 1) < 1e-13
    assert abs(d1["mass_P"] / d0["mass_P"] - 1) < 1e-13
    for c in ("mom_x", "mom_y"):
        assert abs(d1[c] - d0[c]) < 1e-12 * pabs


def _shear_wave_error(L, nu=0.05, A=1e-4, n1=100, n2=600):
    l = L / (2 * np.pi)
    sim = oracle.OracleSim(1, L, nq=4, phi=0.0, Wi=0.0, Re=0.05 * l / nu, force_scale=0.0)
    d = sim.derived()
    y = np.arange(L)
    u = A * np.sin(2 * np.pi * y / L)
    XS = np.stack([oracle.OracleSim.solvent_eq(1.0, uj, 0.0) for uj in u], axis=1)[:, :, None]
    U = np.zeros((2, L, 1)); U[0, :, 0] = u
    sim.set_state(XS=XS, XP=np.zeros((25, sim.nqd, L, 1)),
                  psi=np.zeros((sim.nqd, L, 1)), U=U)
    k = 2 * np.pi / L
    sim.step(n1); a1 = _sin_amp(sim.get_state()["U"][0, :, 0], k, y)
    sim.step(n2 - n1); a2 = _sin_amp(sim.get_state()["U"][0, :, 0], k, y)
    rate = -np.log(a2 / a1) / (n2 - n1)
    return rate / (d["nuS"] * k * k) - 1.0


def test_shear_wave_viscosity():
    e = {L: _shear_wave_error(L) for L in (32, 64, 128)}
    assert abs(e[64]) < 1e-3
    # second-order lattice error
    assert 3.5 < e[32] / e[64] < 4.5 and 3.5 < e[64] / e[128] < 4.5


def _polymer_diffusion_error(L, tau2=0.25, eps=1e-3, n1=50, n2=1050):
    sig2 = oracle.OracleSim(1, 1, nq=4, spring=1).derived()["sigma"] ** 2
    sim = oracle.OracleSim(L, 1, nq=4, spring=1, Wi=0.0, phi=1e-6, force_scale=0.0,
                           lambda_set=3 * sig2 / (2 * tau2), ny_param=64)
    d = sim.derived(); t = sim.tables()
    x = np.arange(L)
    psi = d["rhoP0"] * t["peq"][:, None, None] * (1 + eps * np.sin(2 * np.pi * x / L))[None, None, :]
    XS = np.broadcast_to(oracle.OracleSim.solvent_eq(d["rhoS0"], 0, 0)[:, None, None], (9, 1, L))
    sim.set_state(XS=XS, XP=t["wP"][:, None, None, None] * psi[None], psi=psi,
                  U=np.zeros((2, 1, L)))
    k = 2 * np.pi / L
    sim.step(n1); a1 = _sin_amp(sim.observables()[3, 0, :], k, x)
    sim.step(n2 - n1); a2 = _sin_amp(sim.observables()[3, 0, :], k, x)
    rate = -np.log(a2 / a1) / (n2 - n1)
    return rate / (CS2 * d["tau2P"] * k * k) - 1.0


def test_polymer_density_diffusion():
    e32, e64 = _polymer_diffusion_error(32), _polymer_diffusion_error(64)
    assert abs(e64) < 1e-3
    assert 3.5 < e32 / e64 < 4.5


def _conformation_relaxation_error(nq, tau2=0.0768):
    sig2 = oracle.OracleSim(1, 1, nq=nq, spring=1).derived()["sigma"] ** 2
    lam = 3 * sig2 / (2 * tau2)
    sim = oracle.OracleSim(1, 1, nq=nq, spring=1, Wi=0.0, force_scale=0.0,
                           lambda_set=lam, ny_param=64)
    d = sim.derived(); t = sim.tables(); Q = t["Q"]
    # anisotropic Gaussian with C(0) = diag(1.5, 0.75)
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
    return -np.log(a2 / a1) / (n2 - n1) * d["lambda"] - 1.0


def test_conformation_relaxation_time():
    e = [abs(_conformation_relaxation_error(nq)) for nq in (8, 12, 16)]
    assert e[2] < 1e-2
    assert e[0] > e[1] > e[2]


@pytest.mark.parametrize("gradients", [0, 1])
def test_laminar_oldroyd_b_profile(gradients):
    """Hookean laminar state: U = U_L sin ky with
    U_L = F0 / (k^2 [eta_s + eta_pk + G lambda / (1 + lambda D k^2)]),
    C_xy = lambda U_L k cos(ky) / (1 + lambda D k^2),
    C_xx - C_yy = lambda^2 U_L^2 k^2 / (1 + lambda D k^2) [1 + cos 2ky / (1 + 4 lambda D k^2)].
    eta_s = rho_S c_s^2 tau1_S, eta_pk = rho_P c_s^2 tau1_P (kinetic part of the
    polymer populations), D = c_s^2 tau2_P (r-diffusion)."""
    ny = 64
    sim = oracle.OracleSim(1, ny, nq=16, spring=1, Re=5.0, Wi=0.5, beta=0.8, periods=1,
                           gradients=gradients)
    d = sim.derived()
    sim.rest()
    sim.step(int(12 * max(d["l"] ** 2 / d["nu"], d["lambda"])))
    o = sim.observables()
    y = np.arange(ny); k = d["kf"]; lam = d["lambda"]
    Dk = lam * CS2 * d["tau2P"] * k * k
    eta = d["rhoS0"] * CS2 * d["tau1S"] + d["rhoP0"] * CS2 * d["tau1P"] + d["G"] * lam / (1 + Dk)
    UL_c = d["F0"] / (k * k * eta)
    UL = _sin_amp(o[1, :, 0], k, y)
    assert abs(UL / UL_c - 1) < 2e-3
    Cxy = _cos_amp(o[5, :, 0], k, y)
    assert abs(Cxy / (lam * UL * k / (1 + Dk)) - 1) < 2e-3
    dxx = o[4, :, 0] - o[6, :, 0]
    m0 = lam ** 2 * UL ** 2 * k * k / (1 + Dk)
    assert abs(dxx.mean() / m0 - 1) < 3e-3
    assert abs(_cos_amp(dxx, 2 * k, y) / (m0 / (1 + 4 * Dk)) - 1) < 6e-3
    # cross-stream velocity: only the slow acoustic relaxation of the tiny
    # y-force of the non-uniform conformation remains
    assert np.abs(o[2]).max() < 1e-9 * d["F0"] / (k * k * eta)


def test_unperturbed_state_stays_x_invariant():
    sim = oracle.OracleSim(16, 16, nq=6, ny_param=64)
    sim.base_state(200)
    sim.step(100)
    assert sim.amplitude() < 1e-14


@pytest.mark.parametrize("Wi", [0.1, 2.5, 5.0])
def test_schmidt_number_at_paper_parameters(Wi):
    """72^2 cell, 32 Q points, 4 periods, Re = 3.5, beta = 0.5 (Sec. VII);
    the paper quotes Sc between 0.05 and 4 for its runs."""
    d = oracle.OracleSim(1, 1, nq=32, periods=4, Re=3.5, beta=0.5, Wi=Wi,
                         ny_param=72).derived()
    assert 0.01 < d["Sc"] < 10.0


def test_perturbation_amplitude():
    sim = oracle.OracleSim(32, 32, nq=4, ny_param=64)
    sim.base_state(50)
    sim.perturb(seed=5, amp=1e-3, multimode=True)
    assert abs(sim.amplitude() / 1e-3 - 1) < 1e-12
    sim2 = oracle.OracleSim(32, 32, nq=4, ny_param=64)
    sim2.base_state(50)
    sim2.perturb(seed=5, amp=1e-3, multimode=False)
    assert abs(sim2.amplitude() / (1e-3 / np.sqrt(2)) - 1) < 1e-12


def test_thread_count_does_not_change_results():
    """The oracle's OpenMP splits lattice rows only, so one thread and all
    threads give bitwise the same state (its timing at both counts is
    therefore of the same computation)."""
    def run(threads):
        oracle.set_threads(threads)
        o = oracle.OracleSim(16, 12, nq=6, Re=20.0, Wi=0.5, beta=0.8, periods=1)
        o.base_state(50)
        o.perturb(2, 1e-2, True)
        o.step(10)
        return o.get_state()

    n = oracle.max_threads()
    try:
        a, b = run(1), run(max(n, 2))
    finally:
        oracle.set_threads(n)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def _stiff_fene(relax, nq=8):
    """A 16 x 16 lattice carrying the parameters of a 256^2 one-period
    Kolmogorov flow at Re 60, Wi 1, beta 0.7 (lambda = 815 steps, so that
    tau2_P ~ 1e-3 and omega_P ~ 2): the regime of the 1024^2 workloads."""
    o = oracle.OracleSim(16, 16, nq=nq, Re=60.0, Wi=1.0, beta=0.7, periods=1, ny_param=256,
                         nx_param=256, drift_relax=relax)
    o.base_state(3000)
    o.perturb(0, 1e-2, True)
    return o


def test_fene_drift_caps_in_the_force_table():
    """Every Q-node's drift D_Q |Fhat| stays within both caps: the absolute
    drift_cap per step (0.2 by default) and 2 - omega_P (omega_P =
    2 / (2 tau1_P + 1)); the caps only bind where the continuous FENE force
    exceeds them."""
    for kw in (dict(Re=60.0, Wi=1.0, beta=0.7, ny_param=256), dict(Re=20.0, Wi=0.5, beta=0.8)):
        o = oracle.OracleSim(8, 8, nq=16, periods=1, **kw)
        d, t = o.derived(), o.tables()
        assert o.cfg["drift_cap"] == 0.2
        cap = min(0.2, 2.0 - 2.0 / (2.0 * d["tau1P"] + 1.0))
        Q, F = t["Q"], t["Fhat"]
        drift = d["DQ"] * np.hypot(F[:, 0], F[:, 1])
        assert drift.max() <= cap * (1 + 1e-12)
        s2 = d["sigma"] ** 2
        free = np.hypot(Q[:, 0], Q[:, 1]) / (s2 * (1 - (Q ** 2).sum(1) / (25.0 * s2)))
        binding = d["DQ"] * free > cap
        assert np.allclose(F[~binding], Q[~binding] * (free / np.hypot(Q[:, 0], Q[:, 1]))[~binding, None],
                           rtol=1e-13)
        assert np.allclose(drift[binding], cap, rtol=1e-12)


def test_stiff_fene_diverges_without_the_relative_cap():
    """Regression test of the drift-cap reading: in the stiff regime the
    scheme with only the absolute cap lets round-off grow into a divergence
    within a few thousand steps, while the relative cap keeps the same run
    stable (min psi stays at its initial level)."""
    def healthy(d, floor):
        # (min psi is not a number once the state holds NaN)
        return bool(np.isfinite([d["amplitude"], d["mass_P"]]).all() and floor < d["min_psi"] < 1)

    o = _stiff_fene(0.0)
    o.step(5000)
    assert not healthy(o.diagnostics(), -1e-3)
    o = _stiff_fene(1.0)
    m0 = o.diagnostics()["min_psi"]
    o.step(8000)
    assert healthy(o.diagnostics(), 2 * m0)


def test_same_step_gradients_use_this_steps_observables():
    """With same-step gradients a step ignores the recorded psi and U: two
    states that differ only there step to the same populations, and to the
    populations a lagged step reaches when the recorded fields are replaced
    by the observables this step produces.  The lagged step does depend on
    them."""
    def sim(gradients):
        o = oracle.OracleSim(8, 8, nq=6, spring=0, gradients=gradients, periods=1)
        o.base_state(100)
        o.perturb(seed=1, amp=0.05, multimode=True)
        o.step(3)
        return o

    def with_lag(o, psi, U):
        st = o.get_state()
        o.set_state(XS=st["XS"], XP=st["XP"], psi=psi, U=U)
        return o

    a = sim(1)
    st = a.get_state()
    noisy = with_lag(sim(1), st["psi"] * (1 + inputs.normal(5, st["psi"].shape, 0.1)),
                     inputs.normal(6, st["U"].shape, 1e-3))
    a.step(1); noisy.step(1)
    ra, rn = a.get_state(), noisy.get_state()
    for k in ra:
        assert np.array_equal(ra[k], rn[k]), k
    lag_sim = oracle.OracleSim(8, 8, nq=6, spring=0, gradients=0, periods=1)
    lag_sim.set_state(XS=st["XS"], XP=st["XP"], psi=ra["psi"], U=ra["U"])
    lag_sim.step(1)
    rl = lag_sim.get_state()
    for k in ("XS", "XP"):
        assert np.array_equal(ra[k], rl[k]), k
    b = sim(0)
    stb = b.get_state()
    other = with_lag(sim(0), stb["psi"], inputs.normal(6, stb["U"].shape, 1e-3))
    b.step(1); other.step(1)
    assert not np.array_equal(b.get_state()["XP"], other.get_state()["XP"])


def _interp_symbol(k, a):
    """Fourier symbol of periodic bilinear interpolation at offset a along one
    axis: value at x + a of exp(i k x) sampled on the nodes, divided by
    exp(i k x) (a = n + f: (1 - f) e^{i k n} + f e^{i k (n + 1)})."""
    n = np.floor(a)
    f = a - n
    return (1 - f) * np.exp(1j * k * n) + f * np.exp(1j * k * (n + 1))


@pytest.mark.parametrize("shift", [0, 1])
def test_spring_term_fourier_symbol(shift):
    """For psi(r, Q) = p_Q + A_Q cos(k . r + phi) the spring term is a
    closed form of k: kappa Fhat(Q) Re{A_Q e^{i(k.r + phi)} sigma(k, Q)} with
    sigma = i (Q_x sin k_x + Q_y sin k_y) for the Taylor form (central
    differences) and sigma = S(Q/2) - S(-Q/2), S the product of the axes'
    interpolation symbols, for the shifted form.  At long wavelength both
    tend to i k . Q."""
    nx, ny = 24, 20
    o = oracle.OracleSim(nx, ny, nq=8, spring=1, spring_shift=shift, periods=1)
    t, d, nqd = o.tables(), o.derived(), o.nqd
    Q, Fh = t["Q"], t["Fhat"]
    kx, ky, phi = 2 * np.pi * 3 / nx, 2 * np.pi * 2 / ny, 0.4
    A = 1e-3 * (1 + np.arange(nqd) / nqd)
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    psi = t["peq"][:, None, None] + A[:, None, None] * np.cos(kx * X + ky * Y + phi)[None]
    st = o.get_state()
    o.set_state(XS=st["XS"], XP=st["XP"], psi=psi, U=st["U"])
    for (x, y) in [(0, 0), (5, 7), (23, 19), (11, 3)]:
        got = o.spring_terms(x, y)
        if shift:
            sig = (_interp_symbol(kx, Q[:, 0] / 2) * _interp_symbol(ky, Q[:, 1] / 2)
                   - _interp_symbol(kx, -Q[:, 0] / 2) * _interp_symbol(ky, -Q[:, 1] / 2))
        else:
            sig = 1j * (Q[:, 0] * np.sin(kx) + Q[:, 1] * np.sin(ky))
        diff = np.real(A * np.exp(1j * (kx * x + ky * y + phi)) * sig)
        want = d["kappa"] * Fh * diff[:, None]
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max(), (x, y)
    # long wavelength: shifted and Taylor forms agree to second order
    k = 2 * np.pi / 4096
    s1 = (_interp_symbol(k, Q[:, 0] / 2) - _interp_symbol(k, -Q[:, 0] / 2))
    assert np.abs(s1 - 1j * k * Q[:, 0]).max() < 0.5 * (k * 8) ** 2 * k * 8


@pytest.mark.parametrize("gradients", [0, 1])
@pytest.mark.parametrize("spring", [0, 1])
def test_conservation_with_shifted_spring_term(spring, gradients):
    sim = oracle.OracleSim(16, 16, nq=6, spring=spring, spring_shift=1, gradients=gradients)
    sim.base_state(300)
    sim.perturb(seed=3, amp=0.05, multimode=True)
    d0 = sim.diagnostics()
    pabs = _abs_momentum(sim)
    sim.step(200)
    d1 = sim.diagnostics()
    assert abs(d1["mass_S"] / d0["mass_S"] - 1) < 1e-13
    assert abs(d1["mass_P"] / d0["mass_P"] - 1) < 1e-13
    for c in ("mom_x", "mom_y"):
        assert abs(d1[c] - d0[c]) < 1e-12 * pabs


def test_shift_with_same_step_gradients_on_uniform_polymer():
    """Polymer populations uniform in r (solvent sheared): this step's psi
    is uniform, so the shifted and the Taylor spring terms both vanish and
    one same-step step gives the same state in both forms; after a second
    step, once psi varies, the two differ."""
    nx, ny = 8, 8
    states = []
    for shift in (0, 1):
        sim = oracle.OracleSim(nx, ny, nq=6, Wi=0.8, spring_shift=shift, gradients=1)
        t = sim.tables(); d = sim.derived()
        y = np.arange(ny)
        u = 1e-2 * np.sin(2 * np.pi * y / ny)
        XS = np.stack([oracle.OracleSim.solvent_eq(d["rhoS0"], uj, 0.0) for uj in u], axis=1)
        XS = np.repeat(XS[:, :, None], nx, axis=2)
        psi0 = d["rhoP0"] * t["peq"]
        XP = np.broadcast_to((t["wP"][:, None] * psi0[None, :])[:, :, None, None],
                             (25, sim.nqd, ny, nx)).copy()
        U = np.zeros((2, ny, nx)); U[0] = u[:, None]
        psi = np.broadcast_to(psi0[:, None, None], (sim.nqd, ny, nx)).copy()
        sim.set_state(XS=XS, XP=XP, psi=psi, U=U)
        sim.step(1)
        one = sim.get_state()
        sim.step(1)
        states.append((one, sim.get_state()))
    for k in ("XS", "XP", "psi", "U"):
        a, b = states[0][0][k], states[1][0][k]
        assert np.abs(a - b).max() <= 1e-15 * max(np.abs(a).max(), 1e-3), k
    assert np.abs(states[0][1]["XP"] - states[1][1]["XP"]).max() > 0


def _fene_rest_qrms(drift_cap, nq=32, lam=28.6479, steps=1500):
    """RMS extension / R of a FENE polymer at rest (no flow, no forcing) after
    many relaxation times, and that of the sampled FENE rest distribution."""
    o = oracle.OracleSim(1, 8, nq=nq, Re=3.5, Wi=0.1, beta=0.5, periods=2, u0=0.01,
                         force_scale=0.0, drift_cap=drift_cap, lambda_set=lam)
    d, t = o.derived(), o.tables()
    q2 = (t["Q"] ** 2).sum(1)
    R = np.sqrt(25.0) * d["sigma"]
    o.base_state(0)
    o.step(steps)
    psi = o.get_state()["psi"][:, 0, 0]
    return (np.sqrt((psi * q2).sum() / psi.sum()) / R, np.sqrt((t["peq"] * q2).sum()) / R,
            d["tau2P"])


def test_fene_rest_distribution_is_kept_with_a_loose_drift_cap():
    """The FENE rest distribution (1 - Q^2/R^2)^(b/2) balances Q-diffusion and
    the spring drift: at rest the lattice keeps its RMS extension when the
    drift is not capped, or capped at 0.2 per step (the 72^2 experiment's
    reading); at tau2_P = 0.54 (its Wi = 0.1 cell) a cap of 0.1 binds two
    sigma out and inflates the extension by more than 10 %."""
    free, eq, tau2 = _fene_rest_qrms(0.0)
    assert abs(tau2 - 0.536) < 1e-3
    assert abs(free / eq - 1) < 3e-3
    loose, _, _ = _fene_rest_qrms(0.2)
    assert abs(loose / eq - 1) < 1e-2
    tight, _, _ = _fene_rest_qrms(0.1)
    assert tight / eq - 1 > 0.1


def test_analytic_hookean_state_is_the_laminar_steady_state():
    """The closed-form Hookean laminar state (the analytic initial state)
    against the scheme's own steady state: started from it, a column keeps
    its velocity amplitude and conformation within the closed form's
    accuracy (P9), and both agree with the long pre-run's."""
    ny = 64
    kw = dict(nq=16, spring=1, Re=5.0, Wi=0.5, beta=0.8, periods=1)
    a = oracle.OracleSim(1, ny, **kw)
    d = a.derived()
    a.analytic_state()
    o0 = a.observables()
    y = np.arange(ny); k = d["kf"]
    U0 = _sin_amp(o0[1, :, 0], k, y)
    a.step(int(2 * max(d["l"] ** 2 / d["nu"], d["lambda"])))
    o1 = a.observables()
    assert abs(_sin_amp(o1[1, :, 0], k, y) / U0 - 1) < 3e-3
    assert np.abs(o1[5] - o0[5]).max() < 5e-3 * np.abs(o0[5]).max()
    assert np.abs((o1[4] - o1[6]) - (o0[4] - o0[6])).max() < 1e-2 * np.abs(o0[4] - o0[6]).max()
    b = oracle.OracleSim(1, ny, **kw)
    b.base_state(int(12 * max(d["l"] ** 2 / d["nu"], d["lambda"])))
    assert abs(_sin_amp(b.observables()[1, :, 0], k, y) / U0 - 1) < 3e-3
    with pytest.raises(ValueError):
        oracle.OracleSim(1, ny, **dict(kw, spring=0)).analytic_state()


def _rest_extension(nq, spring):
    """RMS extension over R = sqrt(b) sigma of the oracle's sampled rest
    distribution (its Q-node table), at the 72^2 cell's parameters."""
    o = oracle.OracleSim(1, 8, nq=nq, Re=3.5, Wi=0.1, beta=0.5, periods=2, u0=0.01,
                         force_scale=0.0, lambda_set=28.6479, spring=spring)
    d, t = o.derived(), o.tables()
    q2 = (t["Q"] ** 2).sum(1)
    return np.sqrt((t["peq"] * q2).sum() / t["peq"].sum()) / (np.sqrt(25.0) * d["sigma"])


@pytest.mark.parametrize("nq,tol", [(8, 1e-4), (16, 1e-7), (32, 1e-10)])
def test_fene_rest_extension_is_the_closed_form(nq, tol):
    """FENE rest distribution (1 - Q^2/(b sigma^2))^(b/2) in two dimensions:
    with u = Q^2/(b sigma^2), <Q^2> = b sigma^2 B(2, b/2 + 1) / B(1, b/2 + 1)
    = 2 b sigma^2 / (b + 4), so Q_rms / (sqrt(b) sigma) = sqrt(2 / (b + 4))
    = 0.26261 for b = 25 (Sec. VII's equilibrium extension).  The sampled
    distribution on the half-integer nodes of the open Q-disk converges to
    it spectrally (the density vanishes at the rim with all its low
    derivatives)."""
    assert abs(_rest_extension(nq, 0) / np.sqrt(2.0 / 29.0) - 1) < tol


@pytest.mark.parametrize("nq,tol", [(16, 3e-5), (32, 1e-5)])
def test_hookean_rest_extension_is_the_truncated_gaussian(nq, tol):
    """Hookean rest distribution exp(-Q^2/(2 sigma^2)) on the disk |Q| < R =
    sqrt(b) sigma: <Q^2>/sigma^2 = 2 - a e^-a / (1 - e^-a) with
    a = R^2 / (2 sigma^2) = b/2, the Gaussian's 2 sigma^2 less the part cut
    off beyond R (about 3e-4 of it here)."""
    a = 12.5
    want = np.sqrt((2.0 - 2.0 * a * np.exp(-a) / (1.0 - np.exp(-a))) / 25.0)
    assert abs(_rest_extension(nq, 1) / want - 1) < tol
