"""P10: stability facts of Kolmogorov flow that the oracle must reproduce
(Sec. VII).

Newtonian limit (Wi = 0): the laminar profile is linearly unstable above
Re = sqrt(2) (the Meshalkin-Sinai threshold the paper quotes), through
perturbations much longer than the forcing wavelength.  A square cell with
four forcing periods admits streamwise wavenumbers down to a quarter of
the forcing one, as in the paper's cell: there Re = 20 must grow and Re = 1
(below the threshold for every wavelength) must decay.
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
