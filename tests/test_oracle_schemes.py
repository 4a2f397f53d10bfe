"""Pins of the oracle's other flux kernels (Sec. "Numerical Scheme"): Roe with TENO5,
local Lax-Friedrichs (Rusanov, every characteristic field split) with WENO5-JS, and HLLC
with WENO-AO(5,3) face states.

* reconstructions: exact on quadratics (every candidate is), equal to the linear
  fifth-order upwind value (2, -13, 47, 27, -3)/60 on smooth data, ENO at a step (TENO5
  drops the stencils across it exactly); the quartic smoothness indicator of WENO-AO
  against closed forms and against its Legendre-coefficient form;
* HLLC: consistency F(u, u) = f(u); an isolated stationary contact gives the exact flux
  (0, p, 0, 0, 0); supersonic states give the upwind physical flux;
* whole runs for every kernel: free stream bitwise on a tree with resolution jumps,
  conservation to round-off with jumps and adaptation, Sod along x, y, z equal under the
  axis permutation bitwise and close to the exact solution, fifth-order convergence on a
  smooth entropy wave, a stationary contact kept to round-off.
"""
import math

import numpy as np
import pytest

from paper_2012_04385_amd import workloads as W

N, H, P = 16, 4, 24
GAMMA = 1.4
SCHEMES = ["roe_weno5", "roe_teno5", "llf_weno5", "hllc_wao53"]


def linear5(a, b, c, d, e):
    return (2 * a - 13 * b + 47 * c + 27 * d - 3 * e) / 60.0


@pytest.mark.parametrize("rec", ["teno5_minus", "wao53_minus", "weno5_minus"])
def test_reconstruction_quadratic_smooth_step(orc, rec):
    f = getattr(orc, rec)
    rng = np.random.default_rng(1)
    for _ in range(20):
        c0, c1, c2 = rng.normal(size=3)
        # cell averages of c0 + c1 x + c2 x^2 over unit cells -2..2; value at x = 1/2
        avg = [c0 + c1 * j + c2 * (j * j + 1.0 / 12.0) for j in range(-2, 3)]
        exact = c0 + c1 * 0.5 + c2 * 0.25
        assert abs(f(*avg) - exact) <= 1e-12 * (1 + abs(exact))
    # smooth small-scale data: the nonlinear weights reach the linear ones
    h = 1e-3
    for x0 in np.linspace(0, 1, 7):
        v = [math.sin(2 * math.pi * (x0 + j * h)) for j in range(-2, 3)]
        assert abs(f(*v) - linear5(*v)) <= 1e-12, (rec, x0)
    # a step between c and d: the value stays at the left state
    got = f(0.0, 0.0, 0.0, 1.0, 1.0)
    if rec == "teno5_minus":
        assert got == 0.0                       # the two stencils across the step are cut off
    else:
        assert abs(got) < 1e-3


def test_teno5_keeps_linear_weights_only_when_smooth(orc):
    # a kink in the leftmost cell: TENO5 drops the left stencil and is not the linear value
    v = (5.0, 0.0, 0.1, 0.2, 0.3)
    assert abs(orc.teno5_minus(*v) - linear5(*v)) > 1e-3
    assert abs(orc.teno5_minus(*v) - (-0.1 + 5 * 0.1 + 2 * 0.2 + 0) / 6.0 * 0 -
               (0.6 * (-0.0 + 0.5 + 0.4) / 6.0 + 0.3 * (0.2 + 1.0 - 0.3) / 6.0) / 0.9) < 1e-14


def _legendre_beta(a, b, c, d, e):
    u1 = (11 * a - 82 * b + 82 * d - 11 * e) / 120.0
    u2 = (-3 * a + 40 * b - 74 * c + 40 * d - 3 * e) / 56.0
    u3 = (-a + 2 * b - 2 * d + e) / 12.0
    u4 = (a - 4 * b + 6 * c - 4 * d + e) / 24.0
    return ((u1 + u3 / 10) ** 2 + 13.0 / 3.0 * (u2 + 123.0 / 455.0 * u4) ** 2 +
            781.0 / 20.0 * u3 ** 2 + 1421461.0 / 2275.0 * u4 ** 2)


def test_beta_quartic(orc):
    assert abs(orc.beta_quartic(3, 3, 3, 3, 3)) < 1e-24
    assert abs(orc.beta_quartic(-2, -1, 0, 1, 2) - 1.0) < 1e-13           # P = x
    avg2 = [j * j + 1.0 / 12.0 for j in range(-2, 3)]                       # P = x^2
    assert abs(orc.beta_quartic(*avg2) - 13.0 / 3.0) < 1e-12
    rng = np.random.default_rng(2)
    for _ in range(50):
        v = rng.normal(size=5)
        assert abs(orc.beta_quartic(*v) - _legendre_beta(*v)) <= 1e-12 * (1 + _legendre_beta(*v))


def _cons(rho, u, v, w, p):
    return np.array([rho, rho * u, rho * v, rho * w, p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v + w * w)])


def test_hllc_flux(orc):
    U = _cons(1.3, 0.3, -0.2, 0.1, 0.9)
    np.testing.assert_allclose(orc.hllc_flux_x(U, U), orc.flux_x(U), rtol=1e-14, atol=1e-15)
    # isolated stationary contact: density jump, no velocity, equal pressure
    F = orc.hllc_flux_x(_cons(1.0, 0, 0, 0, 0.7), _cons(0.25, 0, 0, 0, 0.7))
    np.testing.assert_allclose(F, [0, 0.7, 0, 0, 0], atol=1e-15)
    # supersonic to the right: the left physical flux; to the left: the right one
    UL, UR = _cons(1.0, 3.0, 0.1, 0, 1.0), _cons(0.8, 2.9, 0.0, 0.2, 0.9)
    np.testing.assert_array_equal(orc.hllc_flux_x(UL, UR), orc.flux_x(UL))
    UL, UR = _cons(1.0, -3.0, 0.1, 0, 1.0), _cons(0.8, -2.9, 0.0, 0.2, 0.9)
    np.testing.assert_array_equal(orc.hllc_flux_x(UL, UR), orc.flux_x(UR))


@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_scheme_flux_consistency_and_llf_count(orc, scheme):
    rng = np.random.default_rng(scheme)
    U = _cons(1.1, 0.2, -0.4, 0.3, 1.7)
    st = np.tile(U, 6)
    for d in range(3):
        F, n = orc.face_flux_scheme(scheme, d, st)
        Ux = U.copy()
        perm = [[1, 2, 3], [2, 3, 1], [3, 1, 2]][d]
        Ux[1:4] = U[perm]
        Fx = orc.flux_x(Ux)
        ref = np.zeros(5)
        ref[0], ref[4] = Fx[0], Fx[4]
        for k in range(3):
            ref[perm[k]] = Fx[1 + k]
        np.testing.assert_allclose(F, ref, rtol=1e-13, atol=1e-14)
        assert n == (5 if scheme == 2 else (0 if scheme == 3 else n))
    del rng


def _scheme_problem(pb, scheme):
    pb.scheme = scheme
    return pb


def jump_tree(orc, scheme, adapt=0):
    pb = _scheme_problem(W.uniform_flow(lmax=3, n0=(2, 2, 2)), scheme)
    sim = orc.Sim(pb, adapt=adapt).init()
    for r in [(1, 1, 1, 1), (1, 2, 1, 1), (2, 3, 2, 2), (1, 0, 3, 0)]:
        sim.refine(*r)
    return sim


@pytest.mark.parametrize("scheme", SCHEMES[1:])
def test_free_stream_and_conservation(orc, scheme):
    sim = jump_tree(orc, scheme)
    before = sim.leaf_states()
    for _ in range(3):
        sim.step()
    after = sim.leaf_states()
    for k in before:
        assert np.array_equal(before[k], after[k]), (scheme, k)
    # conservation with a smooth bump on the periodic tree with jumps and adaptation
    sim2 = jump_tree(orc, scheme, adapt=1)

    def bump(x, y, z):
        g = np.exp(-((x - 0.45) ** 2 + (y - 0.5) ** 2 + (z - 0.55) ** 2) / 0.01)
        rho, p = 1.0 + 0.5 * g, 1.0 + 2.0 * g
        return np.stack([rho, rho * 0.4, rho * -0.2, rho * 0.3,
                         p / (GAMMA - 1) + 0.5 * rho * (0.16 + 0.04 + 0.09)])

    for n, r in enumerate(sim2.blocks()):
        lvl, bx, by, bz = (int(v) for v in r[:4])
        h = sim2.problem.dx(lvl)
        ar = (np.arange(N) + 0.5) * h
        z, y, x = np.meshgrid(bz * N * h + ar, by * N * h + ar, bx * N * h + ar, indexing="ij")
        blk = sim2.get_block(n)
        blk[:, H:H + N, H:H + N, H:H + N] = bump(x, y, z)
        sim2.set_block(n, blk)
    sim2.project()
    t0 = sim2.totals()
    for _ in range(2):
        sim2.step()
    t1 = sim2.totals()
    assert np.all(np.abs(t1 - t0) <= 2e-14 * np.array([1.5, 1.0, 1.0, 1.0, 5.0])), (scheme, t1 - t0)


def _sod(axis, scheme, n=4):
    n0 = [1, 1, 1]
    n0[axis] = n
    bc = [0, 0, 0]
    bc[axis] = 1
    return W.Problem(name="sod", kind="sod", lmax=0, n0=tuple(n0), dx0=1.0 / (16 * n),
                     bc=tuple(bc), noise=0.0, cfl=0.5, scheme=scheme,
                     params={"axis": axis, "pos": 0.5, "left": (1.0, 1.0), "right": (0.125, 0.1)})


@pytest.mark.parametrize("scheme", SCHEMES[1:])
def test_sod_permutation_and_exact(orc, scheme):
    runs = []
    for axis in range(3):
        sim = orc.Sim(_sod(axis, scheme)).init()
        while sim.time < 0.1:
            sim.step()
        runs.append(sim)
    ref = runs[0].leaf_states()
    for r in (1, 2):
        got = runs[r].leaf_states()
        assert runs[r].time == runs[0].time
        for (lv, bx, by, bz), v in ref.items():
            key, vv = (lv, bx, by, bz), v
            for _ in range(r):
                key = (key[0], key[3], key[1], key[2])
                vv = np.transpose(vv, (0, 2, 3, 1))[[0, 3, 1, 2, 4]]
            assert np.array_equal(vv, got[key]), (scheme, r, key)
    # L1 against the exact Riemann solution (64 cells, t ~ 0.1)
    t = runs[0].time
    xs, rho = [], []
    for (lv, bx, by, bz), u in ref.items():
        xs.append((bx * N + np.arange(N) + 0.5) / 64.0)
        rho.append(u[0].mean(axis=(0, 1)))
    xs, rho = np.concatenate(xs), np.concatenate(rho)
    ex = orc.exact_riemann((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), GAMMA, (xs - 0.5) / t)
    e = np.abs(rho - ex[:, 0]).mean()
    print(f"{scheme}: Sod L1(rho) at 64 cells {e:.3e}")
    assert e < 1.2e-2


def _wave_error(orc, scheme, n_cells, t_end=0.1):
    cfl = 0.4 * (16.0 / n_cells) ** (2.0 / 3.0)

    def prim(x, y, z):
        return (1.0 + 0.2 * np.sin(2 * np.pi * x), 1.0 + 0 * x, 0 * x, 0 * x, 1.0 + 0 * x)

    pb = W.Problem(name="wave", kind="custom", custom=prim, lmax=0, n0=(n_cells // N, 1, 1),
                   dx0=1.0 / n_cells, bc=(0, 0, 0), noise=0.0, cfl=cfl, scheme=scheme)
    sim = orc.Sim(pb).init()
    while sim.time < t_end:
        sim.step()
    err = 0.0
    for key, u in sim.leaf_states().items():
        x = (key[1] * N + np.arange(N) + 0.5) / n_cells
        err += np.abs(u[0] - (1.0 + 0.2 * np.sin(2 * np.pi * (x - sim.time)))[None, None, :]).sum()
    return err / (n_cells * N * N)


@pytest.mark.parametrize("scheme", SCHEMES[1:])
def test_fifth_order_entropy_wave(orc, scheme):
    e = [_wave_error(orc, scheme, n) for n in (16, 32, 64)]
    o1, o2 = math.log2(e[0] / e[1]), math.log2(e[1] / e[2])
    print(f"{scheme}: entropy-wave L1 {e}, orders {o1:.2f} {o2:.2f}")
    assert o2 > 4.5, e


@pytest.mark.parametrize("scheme", SCHEMES)
def test_stationary_contact(orc, scheme):
    """An isolated stationary contact stays put to round-off with every kernel: HLLC
    resolves it exactly; the Roe/LLF split takes its speed from the two face cells, whose
    entropy-field eigenvalue u is zero there, and the acoustic characteristic variables
    are uniform across a contact, so no dissipation acts on it (a split with a global or
    acoustic speed would smear it)."""
    def prim(x, y, z):
        rho = np.where(x < 0.5, 1.0, 0.25)
        return (rho, 0 * x, 0 * x, 0 * x, 0.7 + 0 * x)

    pb = W.Problem(name="contact", kind="custom", custom=prim, lmax=0, n0=(2, 1, 1), dx0=1.0 / 32,
                   bc=(1, 0, 0), noise=0.0, cfl=0.5, scheme=scheme)
    sim = orc.Sim(pb).init()
    before = sim.leaf_states()
    for _ in range(20):
        sim.step()
    after = sim.leaf_states()
    change = max(np.abs(after[k] - before[k]).max() for k in before)
    print(f"{scheme}: stationary contact, max change after 20 steps {change:.3e}")
    assert change < 1e-12
