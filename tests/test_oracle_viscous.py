"""Pins of the oracle's viscous terms, symmetry boundaries and the growth-rate relation of
the Rayleigh-Taylor study (Sec. "Rayleigh-Taylor instability", eq:SinglePhaseGrowth).

* face flux: exact for every linear velocity field (central differences are exact there),
  against the closed form of the Newtonian stress with Stokes' hypothesis, every axis and
  a random velocity gradient; no energy flux for the barotropic (Tait) system;
* a shear wave u = A sin(k y) (and its two cyclic rotations): one SSP-RK3 step multiplies
  the momentum by the stability polynomial 1 + z + z^2/2 + z^3/6 of the discrete
  diffusion eigenvalue z = -dt nu (2 - 2 cos(k dx)) / dx^2, and runs to a fixed time
  converge at second order to the exact decay exp(-nu k^2 t);
* free stream bitwise and conservation to round-off with viscosity on a tree with
  resolution jumps (the viscous flux goes through the jump correction);
* dt: the smaller of eq:Cfl and cfl 3/16 dx^2 min(rho) / mu;
* symmetry boundaries: a block with symmetry planes on both x sides has the right-hand
  side (bitwise) and, after a step, the state of the left half of the twice as long
  periodic domain that holds the mirrored data;
* eq:SinglePhaseGrowth: its root tends to the inviscid rate sqrt(At g k) as mu -> 0 and to
  the viscous-limit rate g (rho_h - rho_l) / (4 mu k) as k -> infinity (derived from the
  relation with q ~ k + n / (2 nu k)), and lies below sqrt(At g k).
"""
import math

import numpy as np
import pytest

from paper_2012_04385_amd import workloads as W
from test_oracle_sim import cons_field, jump_tree, set_leaves

G = 1.4


def _stress(Gm, mu):
    return mu * (Gm + Gm.T) - 2.0 / 3.0 * mu * np.trace(Gm) * np.eye(3)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_face_flux_linear_field(orc, d):
    rng = np.random.default_rng(40 + d)
    Gm = rng.normal(size=(3, 3))
    v0 = rng.normal(size=3)
    mu, dx = 0.37, 0.125
    t_lo, t_hi = [a for a in range(3) if a != d]
    st = np.zeros((2, 5, 5))
    for s in range(2):
        for n, off in enumerate([(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]):
            x = np.zeros(3)
            x[d] = (s - 0.5) * dx
            x[t_lo] = off[0] * dx
            x[t_hi] = off[1] * dx
            vel = v0 + Gm @ x
            rho = 0.5 + rng.random()
            st[s, n] = [rho, *(rho * vel), 2.0 + rng.random()]
    F = orc.visc_face_flux(d, st, mu, dx)
    tau = _stress(Gm, mu)[d]
    assert F[0] == 0.0
    np.testing.assert_allclose(F[1:4], tau, rtol=1e-12, atol=1e-12)
    assert abs(F[4] - tau @ v0) < 1e-12 * (1 + abs(tau @ v0))   # the face is at x = 0
    Ft = orc.visc_face_flux(d, st, mu, dx, energy=False)
    np.testing.assert_array_equal(Ft[:4], F[:4])
    assert Ft[4] == 0.0


def _shear_problem(axis_u, axis_k, mu, n=16, A=1e-4):
    """u_{axis_u} = A sin(2 pi x_{axis_k}) on a periodic unit box of n^3 cells."""
    nb = n // 16

    def ic(x, y, z):
        c = (x, y, z)
        vel = [0 * x, 0 * x, 0 * x]
        vel[axis_u] = A * np.sin(2 * math.pi * c[axis_k])
        return (1.0 + 0 * x, *vel, 1.0 + 0 * x)

    return W.Problem(name="shear", kind="custom", custom=ic, lmax=0, n0=(nb, nb, nb), dx0=1.0 / n,
                     bc=(0, 0, 0), noise=0.0, cfl=0.5, mu=mu)


@pytest.mark.parametrize("axis_u,axis_k", [(0, 1), (1, 2), (2, 0)])
def test_shear_wave_one_step(orc, axis_u, axis_k):
    mu, A = 0.05, 1e-4
    pb = _shear_problem(axis_u, axis_k, mu, A=A)
    sim = orc.Sim(pb).init()
    m0 = sim.leaf_states()[(0, 0, 0, 0)][1 + axis_u].copy()
    dt = sim.step()
    m1 = sim.leaf_states()[(0, 0, 0, 0)][1 + axis_u]
    dx, k = 1.0 / 16, 2 * math.pi
    z = -dt * mu * (2 - 2 * math.cos(k * dx)) / dx ** 2
    R = 1 + z + z * z / 2 + z ** 3 / 6
    assert np.abs(m1 - R * m0).max() < 1e-11 * A, np.abs(m1 - R * m0).max()
    # and the viscous bound set the step (eq:Cfl alone would allow a larger one)
    assert dt == orc.visc_dt(0.5, dx, mu, 1.0)


def test_shear_wave_converges_to_exact_decay(orc):
    mu, A, T = 0.05, 1e-4, 0.1
    errs = []
    for n in (16, 32):
        sim = orc.Sim(_shear_problem(0, 1, mu, n=n, A=A)).init()
        dt = sim.dt()
        steps = int(math.ceil(T / dt))
        for _ in range(steps):
            sim.step_dt(T / steps)
        amp = math.exp(-mu * (2 * math.pi) ** 2 * T)
        e = 0.0
        for (lvl, bx, by, bz), u in sim.leaf_states().items():
            y = (by * 16 + np.arange(16) + 0.5) / n
            exact = A * amp * np.sin(2 * math.pi * y)
            e = max(e, np.abs(u[1] - exact[None, :, None]).max())
        errs.append(e / (A * amp))
    assert errs[0] < 5e-3 and 3.6 < errs[0] / errs[1] < 4.4, errs


def _viscous_tree(orc, mu=0.02):
    pb = jump_tree(orc).problem
    pb.mu = mu
    t = orc.Sim(pb, adapt=0).init()
    for args in [(1, 1, 1, 1), (1, 2, 1, 1), (2, 3, 2, 2), (1, 0, 3, 0)]:
        t.refine(*args)
    return t


def test_free_stream_and_conservation(orc):
    sim = _viscous_tree(orc)
    before = sim.leaf_states()
    sim.step()
    for k, v in sim.leaf_states().items():
        assert np.array_equal(before[k], v), k

    def bump(x, y, z):
        r2 = (x - 0.45) ** 2 + (y - 0.5) ** 2 + (z - 0.55) ** 2
        g = np.exp(-r2 / 0.01)
        return cons_field(1.0 + 0.5 * g, 0.4 + 0.3 * g * (y - 0.5), -0.2 + 0.2 * g * (z - 0.5),
                          0.3 - 0.3 * g * (x - 0.5), 1.0 + 0.2 * g)

    sim = _viscous_tree(orc, mu=0.05)
    set_leaves(sim, bump)
    sim.project()
    t0 = sim.totals()
    for _ in range(3):
        sim.step()
    t1 = sim.totals()
    assert np.all(np.abs(t1 - t0) <= 2e-14 * np.maximum(1.0, np.abs(t0))), t1 - t0
    # the viscous terms did act: the same run without them ends elsewhere
    ref = _viscous_tree(orc, mu=0.0)
    set_leaves(ref, bump)
    ref.project()
    for _ in range(3):
        ref.step()
    diff = max(np.abs(v - ref.leaf_states()[k]).max() for k, v in sim.leaf_states().items())
    assert diff > 1e-5


def test_dt_is_the_smaller_bound(orc):
    pb = _shear_problem(0, 1, mu=1e-4)
    sim = orc.Sim(pb).init()
    c = math.sqrt(G)
    conv = 0.5 * (1.0 / 16) / (c + c + (c + 1e-4))
    assert abs(sim.dt() - conv) < 1e-6 * conv             # viscous bound far larger
    pb = _shear_problem(0, 1, mu=0.5)
    sim = orc.Sim(pb).init()
    assert sim.dt() == orc.visc_dt(0.5, 1.0 / 16, 0.5, 1.0)


def _mirror_pair(orc, mu, gravity=(0.0, 0.0, 0.0)):
    """A block [0,1]^3 with symmetry planes at x = 0 and x = 1, and the periodic domain
    [0,2] x [0,1]^2 whose right half holds the left half's data mirrored (u reversed)."""
    rng = np.random.default_rng(7)
    prim = np.empty((5, 16, 16, 16))
    prim[0] = 1.0 + 0.3 * rng.random((16, 16, 16))
    prim[1:4] = 0.3 * rng.normal(size=(3, 16, 16, 16))
    prim[4] = 1.0 + 0.3 * rng.random((16, 16, 16))

    def left(level, bx, by, bz):
        return prim

    def both(level, bx, by, bz):
        if bx == 0:
            return prim
        m = prim[:, :, :, ::-1].copy()
        m[1] = -m[1]
        return m

    common = dict(kind="custom", lmax=0, dx0=1.0 / 16, noise=0.0, cfl=0.5, mu=mu, gravity=gravity)
    a = orc.Sim(W.Problem(name="sym", n0=(1, 1, 1), bc=(2, 0, 0), **common)).init(left)
    b = orc.Sim(W.Problem(name="per", n0=(2, 1, 1), bc=(0, 0, 0), **common)).init(both)
    return a, b


@pytest.mark.parametrize("mu", [0.0, 0.01])
def test_symmetry_boundary_is_a_mirror(orc, mu):
    a, b = _mirror_pair(orc, mu)
    for s in (a, b):
        s.project()
        s.fill_halos()
    np.testing.assert_array_equal(a.rhs()[0], b.rhs()[0])
    dta, dtb = a.step(), b.step()
    assert dta == dtb
    ua, ub = a.leaf_states()[(0, 0, 0, 0)], b.leaf_states()[(0, 0, 0, 0)]
    assert np.abs(ua - ub).max() < 1e-13 * np.abs(ub).max()


def test_growth_rate_limits(orc):
    rh, rl, g = 1.5, 0.5, 1.0
    at = (rh - rl) / (rh + rl)
    for k in (0.5, 2.0, 7.0):
        n = orc.rti_growth_rate(k, rh, rl, 1e-12, g)
        assert abs(n - math.sqrt(at * g * k)) < 1e-5 * n
    for k in (2e3, 1e4):
        n = orc.rti_growth_rate(k, rh, rl, 0.1, g)
        lim = g * (rh - rl) / (4 * 0.1 * k)
        assert abs(n - lim) < 2e-3 * lim, (n, lim)
    for k in (0.5, 1.0, 2.0, 5.0, 20.0):
        assert 0 < orc.rti_growth_rate(k, rh, rl, 0.1, g) < math.sqrt(at * g * k)
        assert 0 < orc.rti_growth_rate(k, 99.9, 0.1, 0.5, g) < math.sqrt(0.998 * g * k)


def test_lts_refuses_viscosity(orc):
    sim = orc.Sim(_shear_problem(0, 1, 0.05)).init()
    with pytest.raises(ValueError):
        sim.step_lts()


def _column(mu=0.0, lmax=0, bc_y=3):
    """A resting isopycnal column under gravity -1 along y: rho = 2, p = 50 - 2 y; fixed
    values (the profile continued) at top and bottom, symmetry planes on the sides."""
    def ic(x, y, z):
        return (2.0 + 0 * x, 0 * x, 0 * x, 0 * x, 50.0 - 2.0 * y)

    return W.Problem(name="column", kind="custom", custom=ic, lmax=lmax, n0=(1, 2, 1), dx0=1.0 / 16,
                     bc=(2, bc_y, 2), noise=0.0, cfl=0.5, mu=mu, gravity=(0.0, -1.0, 0.0),
                     scale_rho=2.0, scale_E=125.0)


@pytest.mark.parametrize("mu", [0.0, 0.05])
def test_fixed_values_keep_a_resting_column(orc, mu):
    # linear pressure is reconstructed exactly, so the flux divergence balances the
    # gravity source in every cell, the boundary cells too when their halo continues
    # the profile; zero-gradient or mirror halos leave the boundary cells out of balance
    sim = orc.Sim(_column(mu)).init()
    for _ in range(5):
        sim.step()
    vmax = max(np.abs(u[1:4] / u[0]).max() for u in sim.leaf_states().values())
    assert vmax < 1e-11, vmax
    for bc_y in (1, 2):
        sim = orc.Sim(_column(mu, bc_y=bc_y)).init()
        for _ in range(5):
            sim.step()
        vmax = max(np.abs(u[1:4] / u[0]).max() for u in sim.leaf_states().values())
        assert vmax > 1e-4, (bc_y, vmax)


def test_fixed_values_with_levels_and_lts(orc):
    # the same on a tree with two levels: the fixed halo states of each level, and the
    # local time stepping's own boundary fill
    pb = _column(lmax=1)
    sim = orc.Sim(pb, adapt=0).init()
    sim.coarsen(0, 0, 1, 0)   # levels 0 and 1 side by side: a resolution jump mid-column
    for _ in range(2):
        sim.step()
    sim.step_lts()
    levels = {k[0] for k in sim.leaf_states()}
    assert levels == {0, 1}
    vmax = max(np.abs(u[1:4] / u[0]).max() for u in sim.leaf_states().values())
    assert vmax < 1e-11, vmax
