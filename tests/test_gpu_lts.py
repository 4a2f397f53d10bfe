"""Parity of local time stepping (mrfv_step_lts; eq:LtsTimestep, algo:ComputeLoop,
algo:Integration) on the GPU with the oracle's, through the C ABI.

Tree: four levels (a level-0 leaf next to level-1 leaves, one- and two-level jumps, a
refined group touching the periodic boundary), a Gaussian pulse in density and pressure
carried by a uniform flow, so that waves cross the jumps; periodic, and once with
zero-gradient, periodic and symmetry axes.

Tolerances: FP64 -- 1e-12 relative on leaf states after the macro steps (the plain
kernels' face fluxes differ from the oracle's in summation order at the 1e-16 level,
carried through 8 micro steps), dt bitwise-close (1e-14), trees identical with
adaptation; FP32 (flux divergence from the fused kernel, batched and per-block contexts)
-- 5e-6 relative (FP32 rounding of O(1) states over 24 integrated stages), and 1e-6
against the fused global step with one level.  Conservation on the GPU is checked
against its own start, like the oracle's.
"""
import numpy as np
import pytest

from gpu_helpers import H, N, make_pair, same_tree, set_interiors
from paper_2012_04385_amd import workloads as W

pytestmark = pytest.mark.gpu

REFS = [(1, 1, 1, 1), (1, 2, 1, 1), (2, 3, 2, 2), (1, 0, 3, 0)]
GAMMA = 1.4


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


def _pulse(pb, key):
    lvl, bx, by, bz = key
    h = pb.dx(lvl)
    ar = np.arange(N) + 0.5
    z, y, x = np.meshgrid((bz * N + ar) * h, (by * N + ar) * h, (bx * N + ar) * h, indexing="ij")
    r2 = (x - 0.45) ** 2 + (y - 0.5) ** 2 + (z - 0.55) ** 2
    g = np.exp(-r2 / 0.01)
    rho, p = 1.0 + 0.5 * g, 1.0 + 2.0 * g
    u, v, w = 0.4, -0.2, 0.3
    return np.stack([rho, rho * u, rho * v, rho * w,
                     p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v + w * w)])


def _pair(orc, dtype, adapt=0, batched=False, bc=(0, 0, 0)):
    pb = W.uniform_flow(lmax=3, n0=(2, 2, 2))
    pb.bc = bc
    o, g = make_pair(orc, pb, REFS, dtype, batched, adapt=adapt)
    o.coarsen(0, 1, 0, 1)
    g.coarsen(0, 0, 1, 0, 1)
    set_interiors(o, g, lambda k: _pulse(pb, k))
    o.project()
    g.mr_project()
    return o, g


def _worst(o, g):
    ol, gl = o.leaf_states(), g.leaf_states()
    assert ol.keys() == gl.keys()
    return max(np.abs(gl[k] - v).max() / np.abs(v).max() for k, v in ol.items())


@pytest.mark.parametrize("dtype,batched,tol", [("f64", False, 1e-12), ("f32", True, 5e-6), ("f32", False, 5e-6)])
def test_lts_static_tree(orc, torch_mod, dtype, batched, tol):
    o, g = _pair(orc, dtype, batched=batched)
    print(f"[lts] static tree {dtype} batched={batched}", flush=True)
    levels = {k[0] for k in o.leaf_states()}
    assert levels == {0, 1, 2, 3}
    for m in range(2):
        dt_o = o.step_lts()
        cells = g.step_lts()
        torch_mod.cuda.synchronize()
        g.check()
        dt_g = float(g.dt.cpu()[0])
        assert abs(dt_g - dt_o) <= (1e-14 if dtype == "f64" else 1e-6) * dt_o, m
        # every leaf cell updated once per own step: 2^level steps per macro step
        expect = sum((1 << k[0]) * N ** 3 for k in o.leaf_states())
        assert cells == expect
    np.testing.assert_array_equal(o.lts_steps()[:4], [2, 4, 8, 16])
    worst = _worst(o, g)
    print(f"[lts] worst relative difference {worst:.3e}", flush=True)
    assert worst < tol, worst


@pytest.mark.parametrize("dtype,batched,tol", [("f64", False, 1e-12), ("f32", False, 5e-6), ("f32", True, 5e-6)])
def test_lts_bounded_tree(orc, torch_mod, dtype, batched, tol):
    # zero-gradient x, periodic y, symmetry z: the boundary fill before each flux
    # evaluation (FP32: before the fused kernel's flux-divergence mode) and the clamped and
    # mirrored predictions of the flux divergence
    o, g = _pair(orc, dtype, batched=batched, bc=(1, 0, 2))
    print(f"[lts] bounded tree {dtype} batched={batched}", flush=True)
    for m in range(2):
        dt_o = o.step_lts()
        g.step_lts()
        torch_mod.cuda.synchronize()
        g.check()
        dt_g = float(g.dt.cpu()[0])
        assert abs(dt_g - dt_o) <= (1e-14 if dtype == "f64" else 1e-6) * dt_o, m
    worst = _worst(o, g)
    print(f"[lts] worst relative difference {worst:.3e}", flush=True)
    assert worst < tol, worst


def test_lts_adaptive_tree(orc, torch_mod):
    o, g = _pair(orc, "f64", adapt=1)
    print("[lts] adaptive tree f64", flush=True)
    n0 = len(o.blocks())
    for m in range(2):
        o.step_lts()
        g.step_lts()
        torch_mod.cuda.synchronize()
        ok, ol, gl = same_tree(o, g)
        assert ok, (m, ol ^ gl)
    assert len(o.blocks()) != n0            # the tree changed
    worst = _worst(o, g)
    print(f"[lts] worst relative difference {worst:.3e}", flush=True)
    assert worst < 1e-12, worst


def test_lts_conservation(orc, torch_mod):
    _, g = _pair(orc, "f64")
    g.totals()
    t0 = g.tot.cpu().numpy()[0].copy()
    for _ in range(2):
        g.step_lts()
    g.totals()
    torch_mod.cuda.synchronize()
    t1 = g.tot.cpu().numpy()[0]
    scale = np.array([1.5, 1.0, 1.0, 1.0, 5.0])
    assert np.all(np.abs(t1 - t0) <= 2e-14 * scale), t1 - t0


def test_lts_single_level_is_the_global_step(orc, torch_mod):
    from paper_2012_04385_amd.mrfv import Solver
    pb = W.uniform_flow(lmax=0, n0=(2, 2, 2))
    sims = [Solver([pb], dtype="f64", batched=False, adapt=0).init() for _ in range(2)]
    keys = [tuple(int(v) for v in r[2:6]) for r in sims[0].blocks()]
    for g in sims:
        for r in g.blocks():
            k = tuple(int(v) for v in r[2:6])
            g.U[int(r[0]), :, H:H + N, H:H + N, H:H + N] = torch_mod.as_tensor(
                _pulse(pb, k), dtype=g.tdtype, device=g.device)
    a, b = sims
    for _ in range(3):
        a.step_lts()
        b.step()
    torch_mod.cuda.synchronize()
    A, B = a.leaf_states(), b.leaf_states()
    assert len(keys) == 8 and A.keys() == B.keys()
    for k in A:
        assert np.array_equal(A[k], B[k]), k


def test_lts_single_level_fp32_is_the_fused_step(torch_mod):
    # FP32 local time stepping takes L from the fused kernel's flux-divergence mode and
    # integrates it in its own update; with one level that is the fused global step up to
    # the rounding of the update's operation order
    from paper_2012_04385_amd.mrfv import Solver
    pb = W.uniform_flow(lmax=0, n0=(2, 2, 2))
    sims = [Solver([pb], dtype="f32", batched=b, adapt=0).init() for b in (False, 2)]
    for g in sims:
        for r in g.blocks():
            k = tuple(int(v) for v in r[2:6])
            g.U[int(r[0]), :, H:H + N, H:H + N, H:H + N] = torch_mod.as_tensor(
                _pulse(pb, k), dtype=g.tdtype, device=g.device)
    a, b = sims
    for _ in range(3):
        a.step_lts()
        b.step()
        torch_mod.cuda.synchronize()
        da, db = float(a.dt.cpu()[0]), float(b.dt.cpu()[0])
        assert abs(da - db) <= 1e-6 * db, (da, db)
    a.check()
    A, B = a.leaf_states(), b.leaf_states()
    assert A.keys() == B.keys()
    worst = max(np.abs(A[k] - B[k]).max() / np.abs(B[k]).max() for k in A)
    print(f"[lts] fp32 single level vs fused step {worst:.3e}", flush=True)
    assert worst < 1e-6, worst


def test_lts_rejects_mixed_lmax(torch_mod):
    from paper_2012_04385_amd.mrfv import MrfvError, Solver
    pbs = [W.uniform_flow(lmax=1, n0=(1, 1, 1)), W.uniform_flow(lmax=2, n0=(1, 1, 1))]
    g = Solver(pbs, dtype="f64", batched=False, adapt=0).init()
    with pytest.raises(MrfvError):
        g.step_lts()


def test_lts_levels_without_leaves(orc, torch_mod):
    """l_max = 3 but leaves on levels 0 and 1 only: the micro steps of the empty finer levels
    integrate nothing, level 1 steps with 4 dt and level 0 with 8 dt."""
    pb = W.uniform_flow(lmax=3, n0=(2, 2, 2))
    o, g = make_pair(orc, pb, [], "f64")
    o.coarsen(0, 1, 0, 1)
    g.coarsen(0, 0, 1, 0, 1)
    set_interiors(o, g, lambda k: _pulse(pb, k))
    o.project()
    g.mr_project()
    assert {k[0] for k in o.leaf_states()} == {0, 1}
    o.step_lts()
    g.step_lts()
    torch_mod.cuda.synchronize()
    g.check()
    worst = _worst(o, g)
    print(f"[lts] empty finer levels: worst relative difference {worst:.3e}", flush=True)
    assert worst < 1e-12, worst


def test_lts_between_graph_steps(orc, torch_mod):
    """A macro step between step-graph runs of the fused FP32 path gives the oracle's
    global, local, global sequence (the graph steps' reuse of the previous stage's
    restriction and CFL maxima must not carry across the macro step)."""
    o, g = _pair(orc, "f32", batched=2)
    for _ in range(2):
        o.step()
    g.run(2)
    o.step_lts()
    g.step_lts()
    for _ in range(2):
        o.step()
    g.run(2)
    torch_mod.cuda.synchronize()
    g.check()
    worst = _worst(o, g)
    print(f"[lts] between graph steps: worst relative difference {worst:.3e}", flush=True)
    assert worst < 5e-6, worst
