"""Seeded synthetic inputs shared by the oracle and GPU tests.

Holds none of the method's arithmetic: only seeded random arrays and the
configuration recipes (lattice sizes, parameters) of the workloads.
"""
import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def positive_field(seed: int, shape, base, rel: float = 0.1) -> np.ndarray:
    """base * (1 + rel * U(-1, 1)) elementwise; base broadcasts over shape."""
    r = rng(seed).uniform(-1.0, 1.0, size=shape)
    return np.asarray(base) * (1.0 + rel * r)


def normal(seed: int, shape, scale: float = 1.0) -> np.ndarray:
    return scale * rng(seed).standard_normal(size=shape)


# Workload recipes (synthetic stand-ins for the paper's Kolmogorov runs).
C1 = dict(nx=64, ny=64, nq=16, periods=1, Re=20.0, Wi=0.5, beta=0.8, seed=0,
          amp=1e-3, multimode=False, steps=2000)
C2 = dict(nx=1024, ny=1024, nq=16, periods=4, Re=60.0, Wi=1.0, beta=0.7, seed=0,
          amp=1e-4, multimode=True, steps=20000)
