"""Tait's equation of state on the GPU (plain kernels, through the C ABI) against the oracle.

* right-hand side with the jump correction on a tree with one- and two-level jumps and
  random barotropic states (identical halos on both sides), FP64 and FP32;
* whole runs of the Sod tube with Tait's equation: single level (FP64 and FP32) and
  three levels with adaptation (FP64; identical trees after every step);
* local time stepping with Tait's flux (FP64, one macro step of the adaptive tube);
* conservation of mass and momentum with jumps, the energy component staying zero;
* the combinations the library refuses (fused FP32 path, gravity, proposer).

Tolerances: FP64 1e-10 relative on the right-hand side and 1e-11 on whole runs, dt to
1e-13 (different operation order, pow in two libraries, and the GPU's cancellation-free
form of the Roe secant c~^2); FP32 5e-5 on the right-hand side and 2e-5 on runs.
"""
import numpy as np
import pytest

from gpu_helpers import N, make_pair, oracle_padded_to_gpu, same_tree, set_interiors, slot_map
from paper_2012_04385_amd import workloads as W

pytestmark = pytest.mark.gpu

REFS = [(1, 1, 1, 1), (1, 2, 1, 1), (2, 3, 2, 2), (1, 0, 3, 0)]
TAIT = dict(B=0.937315, eos="tait", tait_A=1.0, tait_rho0=1.0)


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


def _jump_problem():
    pb = W.uniform_flow(lmax=3, n0=(2, 2, 2))
    pb.bc = (0, 1, 0)
    for k, v in TAIT.items():
        setattr(pb, k, v)
    return pb


def _sod(n0x, lmax):
    return W.Problem(name="sod_tait", kind="sod", lmax=lmax, n0=(n0x, 1, 1), dx0=1.0 / (16 * n0x),
                     bc=(1, 0, 0), noise=0.0, cfl=0.5,
                     params={"axis": 0, "pos": 0.5, "left": (1.0, 1.0), "right": (0.125, 0.1)}, **TAIT)


def _random_barotropic(rng):
    rho = 0.6 + 0.8 * rng.random((N, N, N))
    return np.stack([rho, rho * rng.normal(0, 0.4, rho.shape), rho * rng.normal(0, 0.4, rho.shape),
                     rho * rng.normal(0, 0.4, rho.shape), 0 * rho])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_rhs_with_jump_correction(orc, torch_mod, dtype):
    o, g = make_pair(orc, _jump_problem(), REFS, dtype)
    print(f"[tait] rhs {dtype}", flush=True)
    rng = np.random.default_rng(31)
    set_interiors(o, g, lambda k: _random_barotropic(rng))
    o.project()
    o.fill_halos()
    oracle_padded_to_gpu(o, g)
    Lo = o.rhs()
    g.rhs_stage()
    torch_mod.cuda.synchronize()
    Lg = g.L.double().cpu().numpy()
    gm = slot_map(g)
    leaves = [tuple(int(v) for v in r[:4]) for r in o.blocks() if r[4] == 1]
    tol = 1e-10 if dtype == "f64" else 5e-5
    worst = 0.0
    for i, k in enumerate(leaves):
        ref = Lo[i]
        assert not ref[4].any() and not Lg[gm[k]][4].any()
        worst = max(worst, np.abs(Lg[gm[k]] - ref).max() / np.abs(ref).max())
    print(f"[tait] worst {worst:.2e}", flush=True)
    assert worst < tol, worst


def _compare(o, g, tol):
    ol, gl = o.leaf_states(), g.leaf_states()
    assert ol.keys() == gl.keys()
    worst = max(np.abs(gl[k] - v).max() / np.abs(v).max() for k, v in ol.items())
    for v in gl.values():
        assert not v[4].any()
    return worst


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-11), ("f32", 2e-5)])
def test_sod_single_level(orc, torch_mod, dtype, tol):
    o, g = make_pair(orc, _sod(4, 0), (), dtype)
    print(f"[tait] sod single level {dtype}", flush=True)
    for _ in range(20):
        dto = o.step()
        g.step()
        torch_mod.cuda.synchronize()
        # the two sides' states differ at 1e-13 (pow in two libraries, another secant
        # form), and dt follows them
        assert abs(float(g.dt.cpu()[0]) - dto) <= (1e-13 if dtype == "f64" else 1e-5) * dto
    g.check()
    worst = _compare(o, g, tol)
    print(f"[tait] worst {worst:.2e}", flush=True)
    assert worst < tol, worst


def test_sod_adaptive_three_levels(orc, torch_mod):
    o, g = make_pair(orc, _sod(2, 2), (), "f64", adapt=1)
    print("[tait] sod three levels, adaptive", flush=True)
    for m in range(10):
        o.step()
        g.step()
        torch_mod.cuda.synchronize()
        ok, ol, gl = same_tree(o, g)
        assert ok, (m, ol ^ gl)
    assert {k[0] for k in o.leaf_states()} >= {1, 2}
    worst = _compare(o, g, 1e-11)
    print(f"[tait] worst {worst:.2e}", flush=True)
    assert worst < 1e-11, worst


def test_lts_with_tait(orc, torch_mod):
    o, g = make_pair(orc, _sod(2, 2), (), "f64", adapt=1)
    print("[tait] LTS", flush=True)
    for _ in range(2):
        o.step()
        g.step()
    o.step_lts()
    g.step_lts()
    torch_mod.cuda.synchronize()
    ok, ol, gl = same_tree(o, g)
    assert ok, ol ^ gl
    worst = _compare(o, g, 1e-11)
    print(f"[tait] worst {worst:.2e}", flush=True)
    assert worst < 1e-11, worst


def test_conservation_with_jumps(orc, torch_mod):
    rng = np.random.default_rng(32)
    pb = W.uniform_flow(lmax=3, n0=(2, 2, 2))   # periodic: the totals are conserved
    for k, v in TAIT.items():
        setattr(pb, k, v)
    o, g = make_pair(orc, pb, REFS, "f64")
    set_interiors(o, g, lambda k: _random_barotropic(rng))
    g.mr_project()
    g.totals()
    t0 = g.tot.cpu().numpy()[0].copy()
    for _ in range(2):
        g.step()
    g.totals()
    torch_mod.cuda.synchronize()
    t1 = g.tot.cpu().numpy()[0]
    assert np.all(np.abs(t1 - t0) <= 1e-13 * np.abs(t0).max()), t1 - t0
    assert t1[4] == 0.0


def test_refused_combinations(torch_mod):
    from paper_2012_04385_amd.mrfv import MLP, MrfvError, Solver, set_proposer
    pb = _sod(2, 1)
    with pytest.raises(MrfvError):
        Solver([pb], dtype="f32", batched=2)
    pbg = _sod(2, 1)
    pbg.gravity = (0.0, -1.0, 0.0)
    with pytest.raises(MrfvError):
        Solver([pbg], dtype="f64", batched=False)
    g = Solver([pb], dtype="f64", batched=False).init()
    m = MLP(max_rows=64)
    with pytest.raises(MrfvError):
        set_proposer(g, m, 1)
