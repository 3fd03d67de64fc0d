"""Pins of the oracle's observables and diagnostics against what the paper
and plain mathematics fix, each computed here by an independent route.

Polymer stress tau_p = G (M / (rho_P0 m_eq) - I) (Sec. III: the spring
impulse is the divergence of Theta; Sec. V: the elastic stress):
  * it vanishes in the rest state, for either spring law (isotropy of the
    Q-disk and the normalisation by the rest value m_eq);
  * in the Hookean laminar Kolmogorov state it is the Oldroyd-B stress
    G (c - I) of the closed-form conformation (shear and first normal
    stress difference);
  * in any steady laminar state it closes the momentum balance with the
    forcing: tau_xy + (eta_s + eta_pk) dU/dy = F0 cos(ky) / k, so the
    reported stress is the one whose divergence drives the flow (FENE too).
Enstrophy (1/2) sum omega^2 and Q_rms = sqrt(<psi Q^2> / <psi>) (Sec. VII
definitions) on hand-set fields: the central difference has the Fourier
symbol i sin k, and the Q-disk is enumerated here by brute force.
Perturbation: the multimode draw is recomputed in Fourier space from the
published SplitMix64 stream (its own implementation in the input module,
pinned by the published vectors): the exact mode set, amplitudes and
phases, the velocity as the curl of the stream function (divergence-free
mode by mode) and the RMS by Parseval.
"""
import math

import numpy as np
import pytest

import oracle
from tests import inputs

CS2 = 1.0 / 3.0


def _sin_amp(f, k, x):
    return 2.0 / len(x) * np.sum(f * np.sin(k * x))


def _cos_amp(f, k, x):
    return 2.0 / len(x) * np.sum(f * np.cos(k * x))


def _disk(nq):
    """Half-integer Q-grid nodes with |Q| < nq/2, row by row (b outer)."""
    R = nq / 2.0
    out = []
    for b in range(nq):
        for a in range(nq):
            qx, qy = a + 0.5 - R, b + 0.5 - R
            if qx * qx + qy * qy < R * R:
                out.append((qx, qy))
    return np.array(out)


# -- polymer stress ------------------------------------------------------------

@pytest.mark.parametrize("spring", [0, 1])
def test_polymer_stress_vanishes_at_rest(spring):
    sim = oracle.OracleSim(4, 8, nq=16, spring=spring, Re=5.0, Wi=0.5, beta=0.8,
                           periods=1, force_scale=0.0)
    sim.rest()
    o = sim.observables()
    G = sim.derived()["G"]
    assert G > 0
    assert np.abs(o[7:10]).max() < 1e-13 * G
    # the conformation of the rest state is isotropic
    assert np.abs(o[4] - o[6]).max() < 1e-13 * np.abs(o[4]).max()
    assert np.abs(o[5]).max() < 1e-13 * np.abs(o[4]).max()


def _laminar(spring, ny=64, Re=5.0, Wi=0.5, beta=0.8, nq=16):
    sim = oracle.OracleSim(1, ny, nq=nq, spring=spring, Re=Re, Wi=Wi, beta=beta, periods=1)
    d = sim.derived()
    sim.rest()
    sim.step(int(12 * max(d["l"] ** 2 / d["nu"], d["lambda"])))
    return sim, d


def test_polymer_stress_is_the_oldroyd_b_stress_in_the_hookean_laminar_state():
    """Oldroyd-B (Hookean dumbbells, stress diffusion D = c_s^2 tau2_P):
    tau_xy = G lambda U_L k cos(ky) / (1 + lambda D k^2) and
    tau_xx - tau_yy = G lambda^2 U_L^2 k^2 / (1 + lambda D k^2)
    [1 + cos(2ky) / (1 + 4 lambda D k^2)], tau_yy = 0."""
    sim, d = _laminar(spring=1)
    o = sim.observables()
    ny = o.shape[1]
    y = np.arange(ny); k = d["kf"]; lam = d["lambda"]; G = d["G"]
    Dk = lam * CS2 * d["tau2P"] * k * k
    UL = _sin_amp(o[1, :, 0], k, y)
    txy = _cos_amp(o[8, :, 0], k, y)
    assert abs(txy / (G * lam * UL * k / (1 + Dk)) - 1) < 3e-3
    n1 = o[7, :, 0] - o[9, :, 0]
    m0 = G * lam ** 2 * UL ** 2 * k * k / (1 + Dk)
    assert abs(n1.mean() / m0 - 1) < 3e-3
    assert abs(_cos_amp(n1, 2 * k, y) / (m0 / (1 + 4 * Dk)) - 1) < 6e-3
    assert np.abs(o[9, :, 0]).max() < 1e-2 * m0


@pytest.mark.parametrize("spring", [0, 1])
def test_polymer_stress_closes_the_laminar_momentum_balance(spring):
    """Steady x-invariant flow: d/dy [(eta_s + eta_pk) dUx/dy + tau_xy] +
    F0 sin(ky) = 0, so tau_xy = F0 cos(ky) / k - (eta_s + eta_pk) U_L k cos(ky)
    with eta_s = rho_S c_s^2 tau1_S, eta_pk = rho_P c_s^2 tau1_P."""
    sim, d = _laminar(spring=spring)
    o = sim.observables()
    ny = o.shape[1]
    y = np.arange(ny); k = d["kf"]
    eta = d["rhoS0"] * CS2 * d["tau1S"] + d["rhoP0"] * CS2 * d["tau1P"]
    UL = _sin_amp(o[1, :, 0], k, y)
    want = d["F0"] / k - eta * UL * k
    got = _cos_amp(o[8, :, 0], k, y)
    assert want > 0.1 * d["F0"] / k  # the polymer carries a real share
    assert abs(got / want - 1) < 1e-2
    # and the stress has no other shape than cos(ky)
    resid = o[8, :, 0] - got * np.cos(k * y)
    assert np.abs(resid).max() < 1e-2 * abs(got)


# -- enstrophy, Q_rms, masses, min psi -------------------------------------------

def test_enstrophy_and_qrms_of_set_fields():
    nx, ny, nq = 16, 12, 8
    sim = oracle.OracleSim(nx, ny, nq=nq, Re=5.0, Wi=0.5, beta=0.8, periods=1)
    sim.rest()
    st = sim.get_state()
    x = np.arange(nx)[None, :]; y = np.arange(ny)[:, None]
    kx, ky = 2 * np.pi * 2 / nx, 2 * np.pi * 1 / ny
    a, b = 3e-3, -2e-3
    U = np.zeros((2, ny, nx))
    U[0] = a * np.sin(ky * y) + 0 * x
    U[1] = b * np.sin(kx * x) + 0 * y
    disk = _disk(nq)
    nqd = len(disk)
    assert nqd == sim.nqd
    w = inputs.positive_field(7, (nqd,), 1.0, rel=0.9)
    psi = np.broadcast_to(w[:, None, None], (nqd, ny, nx)).copy()
    psi[5, 3, 4] = -1e-7
    sim.set_state(psi=psi, U=U)
    dg = sim.diagnostics()
    # omega = dUy/dx - dUx/dy; the central difference of sin(k x) is sin(k) cos(k x)
    ens = 0.5 * (b * b * math.sin(kx) ** 2 + a * a * math.sin(ky) ** 2) * nx * ny / 2
    assert abs(dg["enstrophy"] / ens - 1) < 1e-12
    q2 = (disk ** 2).sum(1)
    R = nq / 2.0
    num = math.fsum((psi * q2[:, None, None]).ravel())
    den = math.fsum(psi.ravel())
    assert abs(dg["qrms"] / (math.sqrt(num / den) / R) - 1) < 1e-13
    assert dg["min_psi"] == -1e-7
    # masses: plain sums of the populations
    assert abs(dg["mass_S"] - math.fsum(st["XS"].ravel())) < 1e-13 * abs(dg["mass_S"])
    assert abs(dg["mass_P"] - math.fsum(st["XP"].ravel())) < 1e-13 * abs(dg["mass_P"])


def test_qrms_of_a_single_q_node():
    nq = 12
    sim = oracle.OracleSim(3, 4, nq=nq)
    sim.rest()
    disk = _disk(nq)
    for q in (0, len(disk) // 3, len(disk) - 1):
        psi = np.zeros((len(disk), 4, 3))
        psi[q] = 0.25
        sim.set_state(psi=psi)
        want = math.sqrt((disk[q] ** 2).sum()) / (nq / 2.0)
        assert abs(sim.diagnostics()["qrms"] - want) < 1e-15


def test_enstrophy_of_a_uniform_flow_is_zero():
    nx = ny = 8
    sim = oracle.OracleSim(nx, ny, nq=4)
    sim.rest()
    sim.set_state(U=np.stack([np.full((ny, nx), 0.01), np.full((ny, nx), -0.02)]))
    assert sim.diagnostics()["enstrophy"] == 0.0


# -- perturbation ------------------------------------------------------------------

def _expected_multimode_spectrum(seed, nx, ny, amp, u0):
    """FFT (numpy convention) of the perturbation velocity from the recipe:
    stream function sum_m a_m cos(2 pi (kx x/nx + ky y/ny) + phi_m) over
    kx in -8..8 without 0 (outer), ky in -8..8 (inner); a_m by Box-Muller
    from two uniforms, phi_m = 2 pi u; velocity (d/dy, -d/dx), rescaled to
    RMS amp u0.  A term c sin(theta) = c (e^{i theta} - e^{-i theta}) / 2i
    puts c e^{i phi} N / 2i at bin (ky, kx) and its conjugate at (-ky, -kx)."""
    g = inputs.splitmix64(seed)
    N = nx * ny
    Fx = np.zeros((ny, nx), complex); Fy = np.zeros((ny, nx), complex)
    for kx in range(-8, 9):
        if kx == 0:
            continue
        for ky in range(-8, 9):
            u1, u2, u3 = inputs.uniform01(g), inputs.uniform01(g), inputs.uniform01(g)
            a = math.sqrt(-2.0 * math.log(1.0 - u1)) * math.cos(2 * math.pi * u2)
            ph = 2 * math.pi * u3
            cx = -a * 2 * math.pi * ky / ny  # coefficient of sin(theta) in du_x
            cy = a * 2 * math.pi * kx / nx   # ... in du_y
            e = np.exp(1j * ph) * N / 2j
            Fx[ky % ny, kx % nx] += cx * e
            Fy[ky % ny, kx % nx] += cy * e
            Fx[-ky % ny, -kx % nx] += cx * np.conj(e)  # -c e^{-i phi} N / 2i
            Fy[-ky % ny, -kx % nx] += cy * np.conj(e)
    rms = math.sqrt((np.abs(Fx) ** 2 + np.abs(Fy) ** 2).sum() / N / N)  # Parseval
    f = amp * u0 / rms
    return Fx * f, Fy * f


@pytest.mark.parametrize("seed", [0, 11])
def test_multimode_perturbation_spectrum(seed):
    nx, ny, amp = 40, 36, 1e-3
    sim = oracle.OracleSim(nx, ny, nq=4)
    sim.rest()
    u_before = sim.get_state()["U"]
    sim.perturb(seed, amp, True)
    du = sim.get_state()["U"] - u_before
    Fx, Fy = np.fft.fft2(du[0]), np.fft.fft2(du[1])
    Ex, Ey = _expected_multimode_spectrum(seed, nx, ny, amp, sim.cfg["u0"])
    scale = np.abs(Ex).max()
    assert np.abs(Fx - Ex).max() < 1e-11 * scale
    assert np.abs(Fy - Ey).max() < 1e-11 * scale
    # the mode set: nothing outside 1 <= |kx| <= 8, |ky| <= 8
    kx = np.fft.fftfreq(nx, 1.0 / nx)[None, :]; ky = np.fft.fftfreq(ny, 1.0 / ny)[:, None]
    outside = (np.abs(kx) < 1) | (np.abs(kx) > 8) | (np.abs(ky) > 8)
    assert np.abs(Fx[outside]).max() < 1e-11 * scale
    assert np.abs(Fy[outside]).max() < 1e-11 * scale
    # divergence-free mode by mode: kx du_x / nx + ky du_y / ny = 0
    div = kx / nx * Fx + ky / ny * Fy
    assert np.abs(div).max() < 1e-11 * scale / min(nx, ny)
    assert abs(np.sqrt((du ** 2).sum(0).mean()) / (amp * sim.cfg["u0"]) - 1) < 1e-12


def test_single_mode_perturbation():
    """du_y = amp u0 sin(2 pi x / nx + phi0), phi0 = 2 pi u from the first
    SplitMix64 output; du_x = 0."""
    nx, ny, amp, seed = 24, 8, 2e-3, 5
    sim = oracle.OracleSim(nx, ny, nq=4)
    sim.rest()
    u_before = sim.get_state()["U"]
    sim.perturb(seed, amp, False)
    du = sim.get_state()["U"] - u_before
    phi0 = 2 * math.pi * inputs.uniform01(inputs.splitmix64(seed))
    x = np.arange(nx)
    want = amp * sim.cfg["u0"] * np.sin(2 * math.pi * x / nx + phi0)
    assert np.abs(du[0]).max() == 0.0
    assert np.abs(du[1] - want[None, :]).max() < 1e-15
