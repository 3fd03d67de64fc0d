"""P10: stability facts of Kolmogorov flow that the oracle must reproduce
(Sec. VII).

Newtonian limit (Wi = 0): the laminar profile is linearly unstable above
Re = sqrt(2) (the Meshalkin-Sinai threshold the paper quotes), through
perturbations much longer than the forcing wavelength.  A square cell with
four forcing periods admits streamwise wavenumbers down to a quarter of
the forcing one, as in the paper's cell: there Re = 20 must grow and Re = 1
(below the threshold for every wavelength) must decay.

Elastic stabilisation: at the paper's Re = 3.5 and beta = 0.5 the growth
rate of the inflectional instability falls as Wi rises (the stretched
dumbbells resist the short-wavelength perturbation).  The cell holds one
forcing period in a 4:1 box, which admits the same long waves (a quarter of
the forcing wavenumber) as the paper's four-period square; Hookean dumbbells
(Oldroyd-B) on an 8-point Q-grid, sigma k = 0.28, so that the polymer stress
hardly diffuses in r over one relaxation time.
"""
import math

import pytest

import oracle


def _rate(Re, transient=1000, window=600, n=128):
    o = oracle.OracleSim(n, n, nq=4, periods=4, Re=Re, Wi=0.0, beta=1.0)
    o.base_state(-1)  # converged laminar profile (5 viscous times)
    o.perturb(0, 1e-3, True)
    o.step(transient)  # the forced profile's acoustic and viscous transient
    a0 = o.amplitude()
    o.step(window)
    return math.log(o.amplitude() / a0) / window


@pytest.mark.slow
def test_newtonian_kolmogorov_flow_is_unstable_above_the_threshold():
    assert _rate(20.0) > 1e-3


@pytest.mark.slow
def test_newtonian_kolmogorov_flow_is_stable_below_the_threshold():
    assert _rate(1.0) < -1e-4


def _elastic_rate(Wi, settle=2500, window=2500):
    o = oracle.OracleSim(72, 18, nq=8, periods=1, Re=3.5, Wi=Wi, beta=0.5, spring=1)
    o.base_state(-1)
    o.perturb(0, 1e-3, True)
    o.step(settle)
    a0 = o.amplitude()
    o.step(window)
    return math.log(o.amplitude() / a0) / window


@pytest.mark.slow
def test_elasticity_slows_the_inflectional_instability():
    g = [_elastic_rate(w) for w in (0.0, 0.5, 1.0)]
    assert g[2] > 0  # still unstable at Wi = 1 in this cell
    assert g[0] > 1.25 * g[1] and g[1] > 1.25 * g[2], g
