"""Pins of the oracle's transverse directions and of its exact Riemann solver.

* the exact Riemann solver's star state on Sod's data against the published values
  (Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", Table 4.2, test 1);
* axis permutation: the Sod tube (single level and with MR adaptation) along y and
  along z equals the x run with the axes permuted cyclically, bitwise;
* fifth-order convergence on Shu's isentropic vortex (point values, dt ~ dx^(5/3)) in
  the x-y plane, and the same vortex in the y-z plane equal to the permuted x-y run,
  bitwise.  Together these pin the y and z face fluxes (with non-uniform transverse
  data), the acoustic and shear characteristic fields, and eq:Cfl's sum over axes.
"""
import math

import numpy as np
import pytest

from paper_2012_04385_amd import workloads as W

P, H, N = 24, 4, 16
GAMMA = 1.4

# cyclic relabelling of the axes x -> y -> z -> x: a field f(x, y, z) becomes
# g(x', y', z') = f(y', z', x'); momentum components follow their axes.
Q_CYC = [0, 3, 1, 2, 4]


def cyc_state(u):
    """State [5][z][y][x] of the x-run -> the same state after the relabelling."""
    v = np.transpose(u, (0, 2, 3, 1))          # new [z'][y'][x'] = old [y=z'][x=y'][z=x']
    return v[Q_CYC]


def cyc_key(key):
    lvl, bx, by, bz = key
    return (lvl, bz, bx, by)


def test_exact_riemann_star_state(orc):
    # Toro Table 4.2, test 1: p* = 0.30313, u* = 0.92745, rho*L = 0.42632, rho*R = 0.26557
    out = orc.exact_riemann((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), GAMMA, np.array([0.5, 1.3]))
    (rl, ul, pl), (rr, ur, pr) = out
    assert abs(pl - 0.30313) < 5e-6 and abs(pr - 0.30313) < 5e-6
    assert abs(ul - 0.92745) < 5e-6 and abs(ur - 0.92745) < 5e-6
    assert abs(rl - 0.42632) < 5e-6
    assert abs(rr - 0.26557) < 5e-6
    # outside the fan: the initial states; the shock speed 1.75216 separates star and right
    far = orc.exact_riemann((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), GAMMA,
                            np.array([-2.0, 1.75, 1.755, 3.0]))
    np.testing.assert_array_equal(far[0], [1.0, 0.0, 1.0])
    assert abs(far[1, 0] - 0.26557) < 5e-6
    np.testing.assert_array_equal(far[2:], [[0.125, 0.0, 0.1]] * 2)


def _sod(axis, lmax, steps):
    n0 = [1, 1, 1]
    n0[axis] = 4 if lmax == 0 else 2
    bc = [0, 0, 0]
    bc[axis] = 1
    return W.Problem(name=f"sod{axis}", kind="sod", lmax=lmax, n0=tuple(n0),
                     dx0=1.0 / (16 * n0[axis]), bc=tuple(bc), noise=0.0, cfl=0.5, steps=steps,
                     params={"axis": axis, "pos": 0.5, "left": (1.0, 1.0),
                             "right": (0.125, 0.1)})


@pytest.mark.parametrize("lmax,steps", [(0, 12), (2, 6)])
def test_sod_axis_permutation_bitwise(orc, lmax, steps):
    runs = []
    for axis in range(3):
        sim = orc.Sim(_sod(axis, lmax, steps)).init()
        dts = [sim.step() for _ in range(steps)]
        runs.append((dts, sim.leaf_states()))
    dts_x, ref = runs[0]
    if lmax:
        assert any(k[0] == lmax for k in ref)          # the tube was refined somewhere
        assert any(k[0] < lmax for k in ref)           # and has resolution jumps
    for r in (1, 2):
        dts, got = runs[r]
        assert dts == dts_x                            # eq:Cfl, bitwise
        exp = ref
        for _ in range(r):
            exp = {cyc_key(k): cyc_state(v) for k, v in exp.items()}
        assert exp.keys() == got.keys()
        for k in exp:
            assert np.array_equal(exp[k], got[k]), (r, k)


# Shu's isentropic vortex: background (rho, u, v, w, p) = (1, 1, 1, 0, 1) on the periodic
# square [0, 10]^2 (16 cells in the third direction), strength beta = 5, centred at
# (5, 5); the exact solution is the initial field translated by (t, t).
BETA = 5.0
L_BOX = 10.0


def _vortex_prim(a, b, t=0.0):
    """Primitive state at in-plane coordinates (a, b): rho, in-plane velocities, p."""
    da = np.mod(a - t - 5.0 + 5.0, L_BOX) - 5.0
    db = np.mod(b - t - 5.0 + 5.0, L_BOX) - 5.0
    r2 = da * da + db * db
    f = np.exp(0.5 * (1.0 - r2))
    ua = 1.0 - BETA / (2 * math.pi) * f * db
    ub = 1.0 + BETA / (2 * math.pi) * f * da
    T = 1.0 - (GAMMA - 1.0) * BETA ** 2 / (8 * GAMMA * math.pi ** 2) * f * f
    rho = T ** (1.0 / (GAMMA - 1.0))
    return rho, ua, ub, rho * T


def _vortex_problem(n_cells, plane, cfl):
    nb = n_cells // N
    if plane == "xy":
        n0 = (nb, nb, 1)

        def prim(x, y, z):
            rho, ua, ub, p = _vortex_prim(x, y)
            return rho, ua, ub, 0 * x, p
    else:   # "yz": the cyclically relabelled copy
        n0 = (1, nb, nb)

        def prim(x, y, z):
            rho, ua, ub, p = _vortex_prim(y, z)
            return rho, 0 * x, ua, ub, p
    return W.Problem(name="vortex", kind="custom", custom=prim, lmax=0, n0=n0,
                     dx0=L_BOX / n_cells, bc=(0, 0, 0), noise=0.0, cfl=cfl)


def _cfl(n_cells):
    # dt ~ dx^(5/3): the third-order time error stays below the fifth-order space error
    return 0.5 * (32.0 / n_cells) ** (2.0 / 3.0)


def _vortex_run(orc, n_cells, plane, t_end):
    sim = orc.Sim(_vortex_problem(n_cells, plane, _cfl(n_cells))).init()
    while sim.time < t_end:
        sim.step()
    return sim


def _vortex_l1(sim, n_cells):
    """Mean |rho - exact| over the cells within 3 of the vortex centre (the periodic
    images' tails, e^-12 at the box edge, never reach this region by t_end)."""
    t = sim.time
    h = L_BOX / n_cells
    err, cnt = 0.0, 0
    for (lvl, bx, by, bz), u in sim.leaf_states().items():
        x = (bx * N + np.arange(N) + 0.5) * h
        y = (by * N + np.arange(N) + 0.5) * h
        X, Y = np.meshgrid(x, y, indexing="xy")        # [y][x]
        rho_ex = _vortex_prim(X, Y, t)[0]
        dxc = np.mod(X - 5.0 - t + 5.0, L_BOX) - 5.0
        dyc = np.mod(Y - 5.0 - t + 5.0, L_BOX) - 5.0
        m = (np.abs(dxc) < 3.0) & (np.abs(dyc) < 3.0)
        # the solution does not depend on z
        assert np.ptp(u[0], axis=0).max() < 1e-13
        err += np.abs(u[0][:, m] - rho_ex[m][None, :]).sum()
        cnt += m.sum() * N
    return err / cnt


def test_isentropic_vortex_fifth_order(orc):
    t_end = 0.5
    e = [_vortex_l1(_vortex_run(orc, n, "xy", t_end), n) for n in (32, 64, 128)]
    o1 = math.log2(e[0] / e[1])
    o2 = math.log2(e[1] / e[2])
    # recorded: L1 6.27e-4, 4.59e-5, 1.24e-6, orders 3.77 and 5.21.  At 32^2 the vortex
    # core (radius ~1) spans three cells and the WENO weights are still far from the
    # linear ones, so the first pair is pre-asymptotic; the second shows fifth order.
    # A third-order (or transversally inconsistent) flux fails both bounds.
    assert o1 > 3.5, e
    assert o2 > 4.5, e
    assert e[2] < 2e-6, e


def test_isentropic_vortex_rotated_bitwise(orc):
    xy = _vortex_run(orc, 32, "xy", 0.3)
    yz = _vortex_run(orc, 32, "yz", 0.3)
    assert xy.time == yz.time
    exp = {cyc_key(k): cyc_state(v) for k, v in xy.leaf_states().items()}
    got = yz.leaf_states()
    assert exp.keys() == got.keys()
    for k in exp:
        assert np.array_equal(exp[k], got[k]), k
