"""Pins of the oracle's per-block pieces used by the full-size sampled GPU checks.

block_rhs (-div F of one padded block, Sec. "Numerical Scheme"): zero on a uniform
state (free-stream), telescoping to zero over a block whose halos wrap onto itself
(conservation), and equal to the simulation's right-hand side of a leaf.
block_detail (eq:DetailFunction): zero to round-off when the child holds the exact cell
averages of a tensor-product polynomial of degree <= 4 (the prediction is exact there),
equal to a planted deviation divided by its scale, and equal to the simulation's detail.
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_2012_04385_amd import workloads as W

P, H, N = 24, 4, 16


def _random_state(rng, shape, gamma=1.4):
    rho = 1.0 + 0.3 * rng.random(shape)
    u, v, w = (0.3 * rng.standard_normal(shape) for _ in range(3))
    p = 1.0 + 0.5 * rng.random(shape)
    E = p / (gamma - 1) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E])


def _wrap_self(interior):
    """Padded block whose halos are the periodic images of its own interior."""
    idx = (np.arange(P) - H) % N
    return interior[:, idx][:, :, idx][:, :, :, idx]


def test_block_rhs_free_stream(orc):
    u = np.zeros((5, P, P, P))
    u[0], u[1], u[2], u[3], u[4] = 1.3, 0.39, -0.26, 0.13, 2.6
    assert np.all(orc.block_rhs(u, 1.4, 0.0, 1 / 32) == 0.0)


def test_block_rhs_periodic_telescopes(orc):
    rng = np.random.default_rng(5)
    u = _wrap_self(_random_state(rng, (N, N, N)))
    L = orc.block_rhs(u, 1.4, 0.0, 1 / 16)
    for q in range(5):
        assert abs(L[q].sum()) <= 1e-12 * np.abs(L[q]).sum(), q
    # and it is not trivially zero
    assert np.abs(L).max() > 1.0


def test_block_rhs_matches_simulation(orc):
    pb = W.sod_single_level()
    o = orc.Sim(pb).init()
    o.step()
    o.fill_halos()
    Ls = o.rhs()
    info = o.blocks()
    leaves = [n for n in range(len(info)) if info[n, 4] == 1]
    for r, n in enumerate(leaves):
        got = orc.block_rhs(o.get_block(n), pb.gamma, pb.B, pb.dx(int(info[n, 0])))
        assert np.array_equal(got, Ls[r]), n


def _avg_monomial(a, lo, hi):
    return (hi ** (a + 1) - lo ** (a + 1)) / ((a + 1) * (hi - lo))


def _poly_blocks(deg, octant):
    """(child padded, parent padded) exact cell averages of x^a y^b z^c (one component)."""
    par = [[float(_avg_monomial(d, Fraction(I - 12, 12), Fraction(I - 11, 12))) for I in range(P)]
           for d in deg]
    ch = []
    for ax, d in enumerate(deg):
        vals = []
        for i in range(P):
            ci = i - H
            I = octant[ax] * (N // 2) + (ci // 2) + H
            lo, hi = Fraction(I - 12, 12), Fraction(I - 11, 12)
            mid = (lo + hi) / 2
            vals.append(float(_avg_monomial(d, lo, mid) if ci % 2 == 0 else _avg_monomial(d, mid, hi)))
        ch.append(vals)
    pa = np.einsum("k,j,i->kji", par[2], par[1], par[0])
    ca = np.einsum("k,j,i->kji", ch[2], ch[1], ch[0])
    return ca, pa


@pytest.mark.parametrize("deg,octant", [((4, 0, 2), (0, 1, 1)), ((1, 3, 4), (1, 0, 1)),
                                        ((2, 2, 2), (1, 1, 0))])
def test_block_detail_exact_polynomials_and_planted(orc, deg, octant):
    ca, pa = _poly_blocks(deg, octant)
    child = np.stack([1.0 + ca, 0 * ca, 0 * ca, 0 * ca, 2.0 + 3 * ca])
    parent = np.stack([1.0 + pa, 0 * pa, 0 * pa, 0 * pa, 2.0 + 3 * pa])
    d0 = orc.block_detail(child, parent, octant, 1.0, 2.5)
    assert d0 <= 1e-13
    child[4, 2, 21, 7] += 5e-4                     # a halo cell of E
    assert abs(orc.block_detail(child, parent, octant, 1.0, 2.5) - 5e-4 / 2.5) <= 1e-13
    child[0, 10, 10, 10] -= 3e-3                   # an interior cell of rho
    assert abs(orc.block_detail(child, parent, octant, 2.0, 2.5) - 3e-3 / 2.0) <= 1e-13


def test_block_detail_matches_simulation(orc):
    pb = W.blast_mr3(steps=1)
    o = orc.Sim(pb).init()
    o.project()
    o.fill_halos()
    det, _ = o.details()
    info = o.blocks()
    key = {tuple(int(v) for v in info[n, :4]): n for n in range(len(info))}
    fine = [n for n in range(len(info)) if info[n, 0] >= 1][:40]
    for n in fine:
        lv, bx, by, bz = (int(v) for v in info[n, :4])
        par = key[(lv - 1, bx // 2, by // 2, bz // 2)]
        got = orc.block_detail(o.get_block(n), o.get_block(par), (bx & 1, by & 1, bz & 1),
                               pb.scale_rho, pb.scale_E)
        assert got == det[n], n
