"""Host-side logic of the run drivers (no GPU): the growth-rate fit of the
long runs and the onset/plateau summary of the 72^2 experiment, on series
with known answers."""
import math

import numpy as np

from paper_2201_10132_amd import growth_runs, kolmogorov72


def test_fit_gamma_recovers_a_known_rate_and_stops_at_the_threshold():
    n = np.arange(0, 20001, 250)
    A = 1e-4 * np.exp(3e-4 * n)
    g, win = growth_runs.fit_gamma(n, A, 1000)
    # A reaches 1e-2 at n = ln(100) / 3e-4 = 15351: the fit ends at the first
    # sample above it
    assert abs(g / 3e-4 - 1) < 1e-12
    assert win[0] == 1000 and win[1] == n[np.nonzero(A > 1e-2)[0][0]]
    g, win = growth_runs.fit_gamma(n, 1e-4 * np.exp(-2e-5 * n), 1000)
    assert abs(g / -2e-5 - 1) < 1e-12 and win[1] == 20000
    assert growth_runs.fit_gamma([0, 1], [1.0, 1.0], 1000)[0] is None


def test_kolmogorov72_summary_on_a_synthetic_history():
    t = np.arange(0, 201, 1.0)
    lam = 0.05 * (1 - np.exp(-t / 10))          # spin-up to a plateau
    drop = np.where(t > 120, 0.7 + 0.3 * np.exp(-(t - 120) / 5), 1.0)
    E = lam * drop
    res = dict(t=list(t), enstrophy=[list(E), list(lam)], qrms=[[0.3] * t.size, [0.5] * t.size],
               amplitude=[[0.1] * t.size, [1e-3] * t.size], unstable=[False, False])
    rows = kolmogorov72.summary(res, wis=(0.1, 5.0))
    a, b = rows
    # first sample after the maximum at which E is 5 % below it
    j = int(np.argmax(E))
    want = t[j + np.nonzero(E[j:] < 0.95 * E[j])[0][0]]
    assert a["t_onset"] == want and 120 < want < 125
    assert abs(a["final_over_plateau"] - E[-1] / E[j]) < 1e-15
    assert b["t_onset"] is None and abs(b["qrms_tail"] - 0.5) < 1e-15


def test_convective_time_of_the_cell():
    # l = 72 / (8 pi) lattice units at u0 = 0.01
    assert abs(kolmogorov72.convective_steps() - 72 / (8 * math.pi) / 0.01) < 1e-12


def test_shared_drag_time_is_the_polymer_one_bounded_by_the_solvent_viscous_time():
    """The shared drag-time reading (one tau_2 for both components): tau2_P,
    raised to tau1_S where the ordering tau_1 <= tau_2 requires it.  Host
    only: the derived parameters need no GPU."""
    import paper_2201_10132_amd as P

    C = kolmogorov72.CELL
    binds = {}
    for Wi in kolmogorov72.WIS:
        t = P.Tpl(1, C["ny"], C["Re"], Wi, C["beta"], periods=C["periods"], u0=C["u0"], nq=32)
        t1S, t2P = t.query("tau1S"), t.query("tau2P")
        t.close()
        v = kolmogorov72.shared_drag_time(Wi)
        assert v == max(t1S, t2P)
        binds[Wi] = t1S > t2P
    # the solvent's viscous time binds only in the most elastic cell
    assert binds == {0.1: False, 2.5: False, 5.0: True}


def test_cell_size_option_scales_the_convective_time():
    C = kolmogorov72.CELL
    old = (C["nx"], C["ny"])
    try:
        C["nx"] = C["ny"] = 144
        assert abs(kolmogorov72.convective_steps() - 144 / (8 * math.pi) / 0.01) < 1e-12
    finally:
        C["nx"], C["ny"] = old
