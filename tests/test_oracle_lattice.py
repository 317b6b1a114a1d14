"""Pins of the oracle's lattice tables and equilibria.

- The D3Q19 and D2Q9 tables equal the paper's printed matrices and weights
  (golden files).
- Lattice isotropy to fourth order (exact rational identities of D3Q19 in
  three dimensions and of D2Q9 in two).
- Equilibria (Eqs. alfa..ekst, zero shift) reproduce the field value as zeroth
  moment and the flux as first moment, with second moment c_s^2 u delta.
"""

import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "d3q19_paper.txt")
GOLDEN9 = os.path.join(os.path.dirname(__file__), "golden", "d2q9_paper.txt")


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        q, cx, cy, cz, w = line.split()
        rows.append((int(q), (int(cx), int(cy), int(cz)), Fraction(w)))
    return rows


def _golden9():
    rows = []
    for line in open(GOLDEN9):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        q, cx, cy, w = line.split()
        rows.append((int(q), (int(cx), int(cy), 0), Fraction(w)))
    return rows


def test_d2q9_matches_paper_table():
    c, w = oracle.lattice(9)
    rows = _golden9()
    assert len(rows) == 9
    for q, cv, wf in rows:
        assert tuple(c[q]) == cv, q
        assert w[q] == float(wf), q
    c19, w19 = oracle.lattice(19)
    c19b, w19b = oracle.lattice_d3q19()
    assert np.array_equal(c19, c19b) and np.array_equal(w19, w19b)


def test_d2q9_isotropy_exact():
    rows = _golden9()
    cs2 = Fraction(1, 3)
    d = lambda a, b: 1 if a == b else 0  # noqa: E731
    assert sum(w for _, _, w in rows) == 1
    for a in range(2):
        assert sum(w * c[a] for _, c, w in rows) == 0
        for b in range(2):
            assert sum(w * c[a] * c[b] for _, c, w in rows) == cs2 * d(a, b)
            for g in range(2):
                assert sum(w * c[a] * c[b] * c[g] for _, c, w in rows) == 0
                for e in range(2):
                    m4 = sum(w * c[a] * c[b] * c[g] * c[e] for _, c, w in rows)
                    assert m4 == cs2 * cs2 * (d(a, b) * d(g, e) + d(a, g) * d(b, e) + d(a, e) * d(b, g))


def test_d3q19_projects_onto_d2q9():
    """Summing the D3Q19 weights over the directions that share (c_x, c_y)
    gives the D2Q9 weights: on a lattice one site thick in z the two lattices
    carry the same dynamics (the basis of the D2Q9 / D3Q19 scheme pin)."""
    proj = {}
    for _, c, w in _golden():
        proj[(c[0], c[1])] = proj.get((c[0], c[1]), 0) + w
    assert proj == {(c[0], c[1]): w for _, c, w in _golden9()}


def test_d3q19_matches_paper_table():
    c, w = oracle.lattice_d3q19()
    rows = _golden()
    assert len(rows) == 19
    for q, cv, wf in rows:
        assert tuple(c[q]) == cv, q
        assert w[q] == float(wf), q  # the weights are the correctly rounded 1/3, 1/18, 1/36


def test_d3q19_isotropy_exact():
    rows = _golden()
    cs2 = Fraction(1, 3)
    d = lambda a, b: 1 if a == b else 0  # noqa: E731
    assert sum(w for _, _, w in rows) == 1
    for a in range(3):
        assert sum(w * c[a] for _, c, w in rows) == 0
        for b in range(3):
            assert sum(w * c[a] * c[b] for _, c, w in rows) == cs2 * d(a, b)
            for g in range(3):
                assert sum(w * c[a] * c[b] * c[g] for _, c, w in rows) == 0
                for e in range(3):
                    m4 = sum(w * c[a] * c[b] * c[g] * c[e] for _, c, w in rows)
                    assert m4 == cs2 * cs2 * (d(a, b) * d(g, e) + d(a, g) * d(b, e) + d(a, e) * d(b, g))


def test_d3q19_opposite_pairs():
    c, _ = oracle.lattice_d3q19()
    for q in range(1, 19, 2):
        assert tuple(c[q]) == tuple(-c[q + 1])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_equilibrium_moments(seed):
    rng = np.random.default_rng(seed)
    c, _ = oracle.lattice_d3q19()
    u = rng.uniform(-2, 2)
    F = rng.uniform(-1, 1, size=3)
    # scalar fields (alpha, gamma, V): zeroth moment u, first moment 0
    f = oracle.point_feq(0, u)
    assert abs(f.sum() - u) <= 4 * np.spacing(abs(u))
    assert np.allclose(c.T @ f, 0.0, atol=4e-16 * abs(u))
    # K components: zeroth moment K, first moment the flux F, second c_s^2 K delta
    f = oracle.point_feq(1, u, F)
    assert abs(f.sum() - u) <= 1e-15 * (abs(u) + np.abs(F).max())
    assert np.allclose(c.T @ f, F, rtol=0, atol=1e-15 * (abs(u) + np.abs(F).max()))
    m2 = np.einsum("q,qa,qb->ab", f, c, c)
    assert np.allclose(m2, u / 3.0 * np.eye(3), rtol=0, atol=1e-15 * (abs(u) + np.abs(F).max()))
