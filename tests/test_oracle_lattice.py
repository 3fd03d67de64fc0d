"""Pins of the oracle's lattices (Sec. VI.A, VI.B Table I) and its RNG.

P1: velocity-set moments fixed by the paper's isotropy conditions; the
r-projection of D4Q25 is D2Q9; Q-disk geometry and the bounce-back map.
"""
import itertools
import os

import numpy as np
import pytest

import oracle

CS2 = 1.0 / 3.0


def _moments(c, w, order):
    D = c.shape[1]
    out = np.zeros((D,) * order)
    for idx in itertools.product(range(D), repeat=order):
        out[idx] = np.sum(w * np.prod([c[:, a] for a in idx], axis=0))
    return out


def _iso4(D):
    d = np.eye(D)
    return (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
            + np.einsum("ad,bc->abcd", d, d))


@pytest.fixture(scope="module")
def tabs():
    return oracle.OracleSim(1, 1, nq=16).tables()


@pytest.mark.parametrize("name", ["S", "P"])
def test_isotropy(tabs, name):
    c = (tabs["cS"] if name == "S" else tabs["cP"]).astype(float)
    w = tabs["wS"] if name == "S" else tabs["wP"]
    D = c.shape[1]
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(_moments(c, w, 1)).max() < 1e-15
    assert np.abs(_moments(c, w, 2) - CS2 * np.eye(D)).max() < 1e-15
    assert np.abs(_moments(c, w, 3)).max() < 1e-15
    # fourth order: c_s^4 (delta delta + ...) (the printed factor c_s^2 is a typo)
    assert np.abs(_moments(c, w, 4) - CS2 ** 2 * _iso4(D)).max() < 1e-15


def test_d4q25_table(tabs):
    cP = tabs["cP"]
    # Table I: rest vector + all vectors with exactly two nonzero entries +-1
    nz = (cP != 0).sum(axis=1)
    assert nz[0] == 0 and np.all(nz[1:] == 2)
    assert len({tuple(r) for r in cP}) == 25
    assert np.allclose(tabs["wP"], [1 / 3] + [1 / 36] * 24)


def test_r_projection_is_d2q9(tabs):
    """Projecting D4Q25 onto the r-plane gives D2Q9 with its weights."""
    proj = {}
    for c, w in zip(tabs["cP"], tabs["wP"]):
        proj[(c[0], c[1])] = proj.get((c[0], c[1]), 0.0) + w
    d2q9 = {tuple(c): w for c, w in zip(tabs["cS"], tabs["wS"])}
    assert set(proj) == set(d2q9)
    for k in d2q9:
        assert abs(proj[k] - d2q9[k]) < 1e-15


@pytest.mark.parametrize("nq", [4, 6, 8, 16, 32])
def test_qdisk_geometry(nq):
    sim = oracle.OracleSim(1, 1, nq=nq)
    t = sim.tables()
    Q, nbr, cP, ks = t["Q"], t["nbrQ"], t["cP"], t["kstar"]
    R = nq / 2
    # brute force over the full NQ x NQ half-integer grid
    grid = [(a + 0.5 - R, b + 0.5 - R) for b in range(nq) for a in range(nq)]
    inside = [g for g in grid if g[0] ** 2 + g[1] ** 2 < R ** 2]
    assert sim.nqd == len(inside)
    assert np.allclose(Q, np.array(inside))
    pos = {tuple(np.round(q, 6)): i for i, q in enumerate(Q)}
    for k in range(25):
        for q in range(sim.nqd):
            src = tuple(np.round(Q[q] - cP[k, 2:], 6))
            assert nbr[k, q] == pos.get(src, -1)
        assert tuple(cP[ks[k], :2]) == tuple(cP[k, :2])
        assert tuple(cP[ks[k], 2:]) == tuple(-cP[k, 2:])


@pytest.mark.parametrize("nq", [4, 6, 16])
def test_bounce_back_is_a_permutation(nq):
    """Pull streaming with half-way bounce-back maps (q, k) onto distinct
    sources (q', k') with the same r-velocity: mass and r-momentum are exact."""
    sim = oracle.OracleSim(1, 1, nq=nq)
    t = sim.tables()
    nbr, cP, ks = t["nbrQ"], t["cP"], t["kstar"]
    src = set()
    for k in range(25):
        for q in range(sim.nqd):
            s = (nbr[k, q], k) if nbr[k, q] >= 0 else (q, ks[k])
            assert tuple(cP[s[1], :2]) == tuple(cP[k, :2])
            src.add(s)
    assert len(src) == 25 * sim.nqd


def test_splitmix64_vectors():
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_vectors.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert rows
    for r in rows:
        st = int(r[0])
        for want in r[1:]:
            st, z = oracle.splitmix64_next(st)
            assert z == int(want)
