"""The other flux kernels of Sec. "Numerical Scheme" on the GPU (Roe-TENO5, LLF-WENO5,
HLLC-WENO-AO(5,3)) against the oracle, through the C ABI.

* right-hand side with the jump correction on a tree with resolution jumps and random
  physical states, identical halos on both sides (FP64 plain path <= 1e-10 relative,
  FP32 <= 5e-5 relative; the FP64 tolerance also covers the reconstructions' different
  evaluation order: TENO5's cut-off evaluated as a ratio, WENO-AO relative to c; TENO5
  in FP32: mean <= 5e-6, max <= 5e-3, since rounding flips its cut-off switch on faces
  that sit at it);
* the Sod tube (single level, no noise) for 12 steps: FP64 plain path <= 1e-12 relative
  to the oracle, FP32 batched path (step graph) L1(rho) <= 1e-6;
* the 3-level blast (config 2's problem) for 6 steps on the FP32 batched path:
  identical leaf sets after every step and L1(rho) <= 1e-5;
* a stationary contact stays put on the GPU as on the oracle;
* the weak-scaling blast (Woodward-Colella along y, reflecting walls, l_max 3) for two
  steps on the FP32 batched path with all four kernels: identical trees, L1(rho) <= 1e-5;
* the launch variants of the fused kernel give bitwise the same run.
"""
import numpy as np
import pytest

from gpu_helpers import (H, N, l1_diff, make_pair, oracle_padded_to_gpu, random_physical,
                         same_tree, set_interiors, slot_map)
from paper_2012_04385_amd import workloads as W

pytestmark = pytest.mark.gpu

SCHEMES = ["roe_teno5", "llf_weno5", "hllc_wao53"]
REFS = [(1, 1, 1, 1), (1, 2, 1, 1), (2, 3, 2, 2), (1, 0, 3, 0)]


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


def _jump_problem(scheme):
    pb = W.uniform_flow(lmax=3, n0=(2, 2, 2))
    pb.bc = (0, 1, 0)
    pb.scheme = scheme
    return pb


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("dtype,batched", [("f64", False), ("f32", False)])
def test_rhs_with_jumps(orc, torch_mod, scheme, dtype, batched):
    o, g = make_pair(orc, _jump_problem(scheme), REFS, dtype, batched)
    rng = np.random.default_rng(4)
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
    rel = [np.abs(Lg[gm[k]] - Lo[i]) / np.abs(Lo[i]).max() for i, k in enumerate(leaves)]
    worst = max(r.max() for r in rel)
    mean = float(np.mean([r.mean() for r in rel]))
    print(f"{scheme} {dtype}: rhs worst relative difference {worst:.3e}, mean {mean:.3e}")
    if dtype == "f64" or scheme != "roe_teno5":
        assert worst < (1e-10 if dtype == "f64" else 5e-5), worst
    else:
        # TENO5's cut-off is a switch: on rough random data many faces sit near C_T and
        # FP32 rounding flips some of them, which changes that face's flux by a
        # candidate difference; the mean stays at FP32 rounding
        assert mean < 5e-6 and worst < 5e-3, (mean, worst)


def _sod(scheme):
    return W.Problem(name="sod", kind="sod", lmax=0, n0=(4, 1, 1), dx0=1.0 / 64, bc=(1, 0, 0),
                     noise=0.0, cfl=0.5, scheme=scheme,
                     params={"axis": 0, "pos": 0.5, "left": (1.0, 1.0), "right": (0.125, 0.1)})


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("dtype,batched", [("f64", 0), ("f32", 2)])
def test_sod_run(orc, torch_mod, scheme, dtype, batched):
    from paper_2012_04385_amd.mrfv import Solver
    pb = _sod(scheme)
    o = orc.Sim(pb).init()
    g = Solver([pb], dtype=dtype, batched=batched).init()
    for _ in range(12):
        o.step()
        g.step()
    g.check()
    ol, gl = o.leaf_states(), g.leaf_states()
    worst = max(np.abs(gl[k] - v).max() / np.abs(v).max() for k, v in ol.items())
    e = l1_diff(o, g, 0)
    print(f"{scheme} {dtype}: Sod max rel {worst:.3e}, L1 rho {e:.3e}")
    if dtype == "f64":
        assert worst <= 1e-12
    else:
        assert e <= 1e-6


@pytest.mark.parametrize("scheme", SCHEMES)
def test_blast_mr_fp32(orc, torch_mod, scheme):
    from paper_2012_04385_amd.mrfv import Solver
    pb = W.blast_mr3(steps=6)
    pb.scheme = scheme
    o = orc.Sim(pb).init()
    g = Solver([pb], dtype="f32", batched=2).init()
    assert same_tree(o, g)[0]
    for s in range(pb.steps):
        o.step()
        g.step()
        ok, ol, gl = same_tree(o, g)
        assert ok, f"{scheme}: trees differ at step {s} ({len(ol ^ gl)} leaves)"
    g.check()
    e = l1_diff(o, g, 0)
    print(f"{scheme}: blast L1 rho after {pb.steps} steps {e:.3e}")
    assert e <= 1e-5


@pytest.mark.parametrize("scheme", SCHEMES)
def test_stationary_contact(torch_mod, scheme):
    from paper_2012_04385_amd.mrfv import Solver

    def prim(x, y, z):
        return (np.where(x < 0.5, 1.0, 0.25), 0 * x, 0 * x, 0 * x, 0.7 + 0 * x)

    pb = W.Problem(name="contact", kind="custom", custom=prim, lmax=0, n0=(2, 1, 1), dx0=1.0 / 32,
                   bc=(1, 0, 0), noise=0.0, cfl=0.5, scheme=scheme)
    for dtype, batched, tol in (("f64", 0, 1e-12), ("f32", 2, 1e-6)):
        g = Solver([pb], dtype=dtype, batched=batched).init()
        before = g.leaf_states()
        for _ in range(20):
            g.step()
        g.check()
        after = g.leaf_states()
        change = max(np.abs(after[k] - before[k]).max() for k in before)
        print(f"{scheme} {dtype}: stationary contact max change {change:.3e}")
        assert change <= tol


@pytest.mark.parametrize("scheme", SCHEMES)
def test_variants_bitwise(torch_mod, scheme):
    from paper_2012_04385_amd.mrfv import Solver
    pb = W.blast_mr3(steps=2)
    pb.scheme = scheme
    ref = None
    g0 = Solver([pb], dtype="f32", batched=1).init()
    n = len(g0.rhs_variants())
    assert n == 3 and g0.set_rhs_variant(-1) == 0 and g0.rhs_variants()[0] == (2, 512, 1, 0)
    del g0
    for v in range(n):
        g = Solver([pb], dtype="f32", batched=1).init()
        g.set_rhs_variant(v)
        g.step()
        g.step()
        g.check()
        s = g.leaf_states()
        if ref is None:
            ref = s
        for k in s:
            assert np.array_equal(s[k], ref[k]), (scheme, v, k)


@pytest.mark.parametrize("scheme", ["roe_weno5"] + SCHEMES)
def test_weak_scaling_blast(orc, torch_mod, scheme):
    """The weak-scaling case (Woodward-Colella blast along y between reflecting walls,
    l_max 3, 128 x 512 x 128, the paper's CFL 0.9) on the FP32 batched path: identical trees
    after algo:Init and two steps, L1(rho) <= 1e-5 over the domain.  (The second stage's
    steep characteristic fluxes push WENO5's weight products past the FP32 range unless the
    reconstruction rescales its smoothness indicators: LLF-WENO5 used to stop here.)"""
    pb = W.wc_blast_mr4(scheme)
    o, g = make_pair(orc, pb, (), "f32", batched=2, adapt=1)
    print(f"[schemes] wc blast {scheme}", flush=True)
    ok, ol, gl = same_tree(o, g)
    assert ok, ol ^ gl
    for m in range(2):
        o.step()
        g.step()
        torch_mod.cuda.synchronize()
        ok, ol, gl = same_tree(o, g)
        assert ok, (m, ol ^ gl)
    g.check()
    e = l1_diff(o, g, 0)
    print(f"[schemes] L1(rho) {e:.2e}", flush=True)
    assert e <= 1e-5, e
