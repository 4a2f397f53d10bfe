"""Pins of the oracle's MR operators and Morton ids.

Prediction (eq:Prediction, appendix Q-terms): exact on tensor-product polynomials of
degree <= 4 per axis (checked against exact rational cell averages), not exact for
degree 5, and conservative (A(P(u)) = u).  Averaging (eq:Averaging): exact mean, uniform
fields reproduced bitwise.  Morton ids (eq:NeigboorLookup and its worked example):
brute force against coordinates.
"""
from fractions import Fraction
import itertools

import numpy as np
import pytest

P, H, N = 24, 4, 16


def _avg_monomial(a: int, lo: Fraction, hi: Fraction) -> Fraction:
    """Exact mean of x^a over [lo, hi]."""
    return (hi ** (a + 1) - lo ** (a + 1)) / ((a + 1) * (hi - lo))


def _coarse_bounds(I):
    # parent padded cell I covers [(I-12)/12, (I-11)/12] (coordinates kept in [-1, 1])
    return Fraction(I - 12, 12), Fraction(I - 11, 12)


def _fine_bounds(octant, i):
    # child padded cell i of octant o: child interior index ci = i-4 covers half a parent
    # cell: parent interior cell o*8 + floor(ci/2), lower/upper half by parity.
    ci = i - H
    I = octant * (N // 2) + (ci // 2) + H
    lo, hi = _coarse_bounds(I)
    mid = (lo + hi) / 2
    return (lo, mid) if ci % 2 == 0 else (mid, hi)


def _parent_array(a, b, c):
    ex = [_avg_monomial(a, *_coarse_bounds(I)) for I in range(P)]
    ey = [_avg_monomial(b, *_coarse_bounds(I)) for I in range(P)]
    ez = [_avg_monomial(c, *_coarse_bounds(I)) for I in range(P)]
    arr = np.empty((P, P, P))
    fx = np.array([float(v) for v in ex])
    fy = np.array([float(v) for v in ey])
    fz = np.array([float(v) for v in ez])
    arr[:] = fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
    return arr


def _fine_exact(a, b, c, octant, i, j, k):
    return float(_avg_monomial(a, *_fine_bounds(octant[0], i)) *
                 _avg_monomial(b, *_fine_bounds(octant[1], j)) *
                 _avg_monomial(c, *_fine_bounds(octant[2], k)))


@pytest.mark.parametrize("deg", [(0, 0, 0), (1, 0, 0), (0, 2, 0), (0, 0, 3), (4, 0, 0),
                                 (0, 4, 0), (0, 0, 4), (1, 1, 1), (2, 3, 1), (4, 4, 4), (3, 0, 4)])
def test_prediction_exact_for_degree_4(orc, deg):
    a, b, c = deg
    parent = _parent_array(a, b, c)
    rng = np.random.default_rng(sum(deg))
    worst = 0.0
    for octant in itertools.product((0, 1), repeat=3):
        cells = rng.integers(0, P, size=(60, 3))
        for i, j, k in cells:
            got = orc.predict_cell(parent, octant, int(i), int(j), int(k))
            exact = _fine_exact(a, b, c, octant, int(i), int(j), int(k))
            worst = max(worst, abs(got - exact))
    assert worst < 1e-14


def test_prediction_not_exact_for_degree_5(orc):
    parent = _parent_array(5, 0, 0)
    errs = []
    for i in range(H, H + N):
        got = orc.predict_cell(parent, (0, 0, 0), i, 10, 10)
        errs.append(abs(got - _fine_exact(5, 0, 0, (0, 0, 0), i, 10, 10)))
    assert max(errs) > 1e-9


def test_prediction_1d_worked_check(orc):
    # u = k^2 + 1/12 (cell averages of x^2 on unit cells centred at integers) gives the
    # lower child k^2 - k/2 + 1/12 (mean of x^2 over [k-1/2, k]).
    par = np.zeros((P, P, P))
    for I in range(P):
        kk = I - 12
        par[:, :, I] = kk * kk + 1.0 / 12.0
    for i in range(H, H + N, 2):      # lower children of octant 0 along x
        kk = (i - H) // 2 + H - 12
        got = orc.predict_cell(par, (0, 0, 0), i, 12, 12)
        # y, z constant -> the y/z Q-terms vanish
        assert abs(got - (kk * kk - kk / 2 + 1.0 / 12.0)) < 1e-12


def test_average_then_predict_is_identity(orc):
    rng = np.random.default_rng(11)
    parent = rng.normal(size=(P, P, P))
    for octant in itertools.product((0, 1), repeat=3):
        for I, J, K in rng.integers(0, N // 2, size=(20, 3)):
            vals = []
            for cz in (0, 1):
                for cy in (0, 1):
                    for cx in (0, 1):
                        vals.append(orc.predict_cell(parent, octant, H + 2 * I + cx, H + 2 * J + cy, H + 2 * K + cz))
            back = orc.average8(np.array(vals))
            pI = octant[0] * 8 + I + H
            pJ = octant[1] * 8 + J + H
            pK = octant[2] * 8 + K + H
            assert abs(back - parent[pK, pJ, pI]) < 1e-14 * max(1.0, abs(parent).max())


def test_average8(orc):
    assert orc.average8(np.arange(1, 9, dtype=float)) == 4.5
    rng = np.random.default_rng(12)
    for _ in range(100):
        v = rng.normal() * 10.0 ** int(rng.integers(-5, 5))
        assert orc.average8(np.full(8, v)) == v   # uniform field reproduced bitwise


# ------------------------------------------------------------------ Morton ids -------

def test_morton_worked_example(orc):
    # Figure of the neighbour lookup: +z neighbour of 001 111 is 101 011, and of the
    # level-0 node 000 it is 100 (headbit prepended, level-0 blocks per edge = 2).
    mid = int("1" + "001" + "111", 2)
    n, wrapped = orc.morton_neighbor(mid, 2, +1)
    assert n == int("1" + "101" + "011", 2) and not wrapped
    back, _ = orc.morton_neighbor(n, 2, -1)
    assert back == mid
    n0, _ = orc.morton_neighbor(int("1000", 2), 2, +1)
    assert n0 == int("1100", 2)
    assert orc.morton_encode(1, 0, 0, 0, 1) == int("1100", 2)


@pytest.mark.parametrize("shadow", [0, 1, 2])
def test_morton_brute_force(orc, shadow):
    for level in range(0, 3):
        n = 1 << (shadow + level)
        for bx, by, bz in itertools.product(range(n), repeat=3):
            mid = orc.morton_encode(shadow, level, bx, by, bz)
            assert orc.morton_level(mid, shadow) == level
            if level + shadow > 0:
                assert mid >> 3 == orc.morton_encode(shadow, level - 1, bx >> 1, by >> 1, bz >> 1) \
                    if level > 0 else True
            c = [bx, by, bz]
            for d in range(3):
                for s in (+1, -1):
                    got, wrapped = orc.morton_neighbor(mid, d, s)
                    cc = list(c)
                    cc[d] += s
                    out = not (0 <= cc[d] < n)
                    cc[d] %= n
                    assert got == orc.morton_encode(shadow, level, *cc)
                    assert wrapped == out
