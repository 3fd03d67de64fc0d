"""Seeded synthetic inputs of the workloads: the recipes (lattice sizes,
parameters) and seeded random arrays that the benchmark, the run drivers and
the tests (GPU path and oracle alike) start from.

Holds none of the method's arithmetic and imports nothing of the package:
only seeded draws (numpy's Generator, and SplitMix64 from its published
definition) and configuration tables.
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


# SplitMix64 (Steele, Lea & Flood 2014): the seeded draws of the batched sweep.
_M64 = (1 << 64) - 1


def splitmix64(seed: int):
    """Endless generator of SplitMix64 outputs for the given seed."""
    s = seed & _M64
    while True:
        s = (s + 0x9E3779B97F4A7C15) & _M64
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        yield z ^ (z >> 31)


def uniform01(gen) -> float:
    """Uniform double in [0, 1) from the top 53 bits of the next output."""
    return (next(gen) >> 11) * 2.0 ** -53


# Batched sweep: instance i draws, from SplitMix64(i) and in this order, nx and
# ny independently from C4_SIZES, Re ~ U[10, 100], Wi ~ U[0, 2] and
# beta ~ U[0.5, 0.9]; 4 forcing periods, multimode perturbation 1e-4, seed i.
C4_SIZES = (128, 192, 256, 384, 512)


def c4_instances(n: int = 256, periods: int = 4, perturbation: float = 1e-4):
    out = []
    for i in range(n):
        g = splitmix64(i)
        nx = C4_SIZES[min(len(C4_SIZES) - 1, int(uniform01(g) * len(C4_SIZES)))]
        ny = C4_SIZES[min(len(C4_SIZES) - 1, int(uniform01(g) * len(C4_SIZES)))]
        Re = 10.0 + 90.0 * uniform01(g)
        Wi = 2.0 * uniform01(g)
        beta = 0.5 + 0.4 * uniform01(g)
        out.append(dict(nx=nx, ny=ny, periods=periods, Re=Re, Wi=Wi, beta=beta, u0=0.05,
                        seed=i, perturbation=perturbation))
    return out


# Learned-correction trajectories: fine runs with beta = 0.7 and 4 forcing
# periods; trajectory seed s draws Re ~ U[20, 80] and Wi ~ U[0, 1.5] from
# SplitMix64(s), in that order.
def c5_trajectories(seeds, nx=1024, ny=1024, periods=4, beta=0.7, Re=(20.0, 80.0),
                    Wi=(0.0, 1.5)):
    out = []
    for s in seeds:
        g = splitmix64(s)
        re = Re[0] + (Re[1] - Re[0]) * uniform01(g)
        wi = Wi[0] + (Wi[1] - Wi[0]) * uniform01(g)
        out.append(dict(nx=nx, ny=ny, periods=periods, beta=beta, seed=s, Re=re, Wi=wi))
    return out
