"""Pins of the oracle's source term (eq:Euler's S(U), here gravity: S = (0, rho g, rho v.g)).

* free fall of a uniform state on a periodic tree with resolution jumps: the flux
  divergence vanishes, rho stays, m(t) = m0 + rho g t and E(t) = E0 + m0.g t + rho |g|^2 t^2/2
  (a quadratic in t, which SSP-RK3 integrates exactly) -- to round-off after 5 steps;
* momentum balance on a non-uniform periodic problem with jumps and adaptation: the total
  momentum changes by exactly (total mass) g dt per step, to round-off;
* with zero gravity the step is bitwise the same as without a source.
"""
import numpy as np

from paper_2012_04385_amd import workloads as W

N, H = 16, 4
GAMMA = 1.4
G = (0.5, -1.0, 0.25)


def _tree(orc, pb, adapt=0):
    sim = orc.Sim(pb, adapt=adapt).init()
    for r in [(1, 1, 1, 1), (1, 2, 1, 1), (2, 3, 2, 2), (1, 0, 3, 0)]:
        sim.refine(*r)
    return sim


def test_free_fall_exact(orc):
    rho, u, v, w, p = 1.3, 0.3, -0.2, 0.1, 0.9
    pb = W.uniform_flow(lmax=3, n0=(2, 2, 2), state=(rho, u, v, w, p))
    pb.gravity = G
    sim = _tree(orc, pb)
    for _ in range(5):
        sim.step()
    t = sim.time
    m0 = np.array([rho * u, rho * v, rho * w])
    g = np.array(G)
    E0 = p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v + w * w)
    want = [rho, *(m0 + rho * g * t), E0 + m0.dot(g) * t + 0.5 * rho * g.dot(g) * t * t]
    for k, st in sim.leaf_states().items():
        for q in range(5):
            assert np.abs(st[q] - want[q]).max() <= 1e-13 * max(1.0, abs(want[q])), (k, q)


def test_momentum_balance_with_jumps(orc):
    pb = W.uniform_flow(lmax=3, n0=(2, 2, 2))
    pb.gravity = G
    sim = _tree(orc, pb, adapt=1)
    for n, r in enumerate(sim.blocks()):
        lvl, bx, by, bz = (int(v) for v in r[:4])
        h = pb.dx(lvl)
        ar = (np.arange(N) + 0.5) * h
        z, y, x = np.meshgrid(bz * N * h + ar, by * N * h + ar, bx * N * h + ar, indexing="ij")
        gb = np.exp(-((x - 0.45) ** 2 + (y - 0.5) ** 2 + (z - 0.55) ** 2) / 0.01)
        rho, pr = 1.0 + 0.5 * gb, 1.0 + 2.0 * gb
        blk = sim.get_block(n)
        blk[:, H:H + N, H:H + N, H:H + N] = np.stack(
            [rho, 0.4 * rho, -0.2 * rho, 0.3 * rho, pr / (GAMMA - 1) + 0.5 * rho * 0.29])
        sim.set_block(n, blk)
    sim.project()
    g = np.array(G)
    for _ in range(3):
        t0 = sim.totals()
        dt = sim.step()
        t1 = sim.totals()
        assert abs(t1[0] - t0[0]) <= 2e-14 * t0[0]
        np.testing.assert_allclose(t1[1:4] - t0[1:4], t0[0] * g * dt, rtol=0, atol=2e-14 * 5)


def test_zero_gravity_is_no_source(orc):
    pb = W.blast_mr3(steps=2)
    a = orc.Sim(pb).init()
    pb2 = W.blast_mr3(steps=2)
    pb2.gravity = (0.0, 0.0, 0.0)
    b = orc.Sim(pb2).init()
    for _ in range(2):
        a.step()
        b.step()
    sa, sb = a.leaf_states(), b.leaf_states()
    assert sa.keys() == sb.keys()
    assert all(np.array_equal(sa[k], sb[k]) for k in sa)
