"""The gravity source term (eq:Euler's S(U) = (0, rho g, rho v.g)) on the GPU paths.

* free fall of a uniform state on a tree with resolution jumps matches the exact
  quadratic-in-time solution (FP64 plain path to 1e-13, FP32 batched path to 1e-6);
* right-hand side with the jump correction and the source on random physical states,
  identical halos on both sides, against the oracle (FP64 <= 1e-10, FP32 <= 5e-5 relative);
* a heavy-over-light layer under gravity (the Rayleigh-Taylor configuration of the paper's
  verification, inviscid, 3 levels) for 6 steps on the FP32 batched path: identical
  leaf sets after every step and L1(rho) <= 1e-5 against the oracle.
"""
import numpy as np
import pytest

from gpu_helpers import (N, l1_diff, make_pair, oracle_padded_to_gpu, random_physical, same_tree,
                         set_interiors, slot_map)
from paper_2012_04385_amd import workloads as W

pytestmark = pytest.mark.gpu

GAMMA = 1.4
G = (0.5, -1.0, 0.25)
REFS = [(1, 1, 1, 1), (1, 2, 1, 1), (2, 3, 2, 2), (1, 0, 3, 0)]


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("dtype,batched,tol", [("f64", 0, 1e-13), ("f32", 2, 1e-6)])
def test_free_fall(orc, torch_mod, dtype, batched, tol):
    rho, u, v, w, p = 1.3, 0.3, -0.2, 0.1, 0.9
    pb = W.uniform_flow(lmax=3, n0=(2, 2, 2), state=(rho, u, v, w, p))
    pb.gravity = G
    o, g = make_pair(orc, pb, REFS, dtype, batched)
    g.advance(5)
    t = float(g.time[0])
    m0 = np.array([rho * u, rho * v, rho * w])
    gv = np.array(G)
    E0 = p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v + w * w)
    want = [rho, *(m0 + rho * gv * t), E0 + m0.dot(gv) * t + 0.5 * rho * gv.dot(gv) * t * t]
    for k, st in g.leaf_states().items():
        for q in range(5):
            assert np.abs(st[q] - want[q]).max() <= tol * max(1.0, abs(want[q])), (k, q)


@pytest.mark.parametrize("dtype,batched", [("f64", False), ("f32", False)])
def test_rhs_with_source(orc, torch_mod, dtype, batched):
    pb = W.uniform_flow(lmax=3, n0=(2, 2, 2))
    pb.bc = (0, 1, 0)
    pb.gravity = G
    o, g = make_pair(orc, pb, REFS, dtype, batched)
    rng = np.random.default_rng(8)
    set_interiors(o, g, lambda k: random_physical(rng, (N, N, N)))
    o.project()
    o.fill_halos()
    oracle_padded_to_gpu(o, g)
    Lo = o.rhs()
    g.rhs_stage()
    torch_mod.cuda.synchronize()
    Lg = g.L.double().cpu().numpy()
    gm = slot_map(g)
    leaves = [tuple(int(v) for v in r[:4]) for r in o.blocks() if r[4] == 1]
    worst = max(np.abs(Lg[gm[k]] - Lo[i]).max() / np.abs(Lo[i]).max() for i, k in enumerate(leaves))
    assert worst < (1e-10 if dtype == "f64" else 5e-5), worst


def _rt_problem():
    """Heavy (rho 2) over light (rho 1) at y = 1/2, gravity -1 along y, hydrostatic
    pressure, interface displaced by 0.01 cos(2 pi x); periodic in x and z,
    zero-gradient in y."""
    def prim(x, y, z):
        y0 = 0.5 + 0.01 * np.cos(2 * np.pi * x)
        heavy = y > y0
        rho = np.where(heavy, 2.0, 1.0)
        p = np.where(heavy, 10.0 - 2.0 * (y - 0.5), 10.0 - 1.0 * (y - 0.5))
        return rho, 0 * x, 0 * x, 0 * x, p
    return W.Problem(name="rt", kind="custom", custom=prim, lmax=2, n0=(2, 2, 2), dx0=1.0 / 32,
                     bc=(0, 1, 0), noise=0.0, cfl=0.5, steps=6, gravity=(0.0, -1.0, 0.0))


def test_rayleigh_taylor_run(orc, torch_mod):
    from paper_2012_04385_amd.mrfv import Solver
    pb = _rt_problem()
    o = orc.Sim(pb).init()
    g = Solver([pb], dtype="f32", batched=2).init()
    assert same_tree(o, g)[0]
    for s in range(pb.steps):
        o.step()
        g.step()
        ok, ol, gl = same_tree(o, g)
        assert ok, f"trees differ at step {s} ({len(ol ^ gl)} leaves)"
    g.check()
    e = l1_diff(o, g, 0)
    print(f"Rayleigh-Taylor layer: L1 rho after {pb.steps} steps {e:.3e}")
    assert e <= 1e-5
