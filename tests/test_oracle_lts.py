"""Pins of the oracle's local time stepping (eq:LtsTimestep, algo:ComputeLoop,
algo:Integration) against facts that do not come from the oracle itself.

* the active-level set of algo:ComputeLoop (a popcount formula) equals its definition:
  level l completes a step at micro step r when r + 1 is a multiple of 2^(lmax - l);
* in one macro step every level l takes exactly 2^l steps of its own and the clock
  advances 2^lmax fine steps;
* with a single level (lmax = 0) a macro step is the global step, bitwise;
* conservation to round-off on a periodic tree with resolution jumps, with and without
  adaptation (the time-integrated jump fluxes and the coarse cell adjustment);
* free stream kept to round-off on a tree with one- and two-level jumps;
* consistency: the difference to global stepping with the same fine step shrinks
  linearly as the step is halved (first order in time at the jumps, where the halo
  cells are integrated with the coarser level's stored flux divergence), and the error
  of a smooth entropy wave against its exact translation stays within 10 % of the
  global step's;
* axis permutation: the Sod tube along y and z with adaptation equals the x run
  permuted, bitwise.
"""
import numpy as np
import pytest

from paper_2012_04385_amd import workloads as W
from test_oracle_sim import centres, cons_field, jump_tree, set_leaves, _bump
from test_oracle_symmetry import _sod, cyc_key, cyc_state

P, H, N = 24, 4, 16


def test_active_set_formula(orc):
    for lmax in range(7):
        for r in range(1 << lmax):
            expect = min(l for l in range(lmax + 1) if (r + 1) % (1 << (lmax - l)) == 0)
            assert orc.lts_lowest_ending(lmax, r) == expect, (lmax, r)


def _bump_tree(orc, lmax=3, adapt=0):
    sim = orc.Sim(W.uniform_flow(lmax=lmax, n0=(2, 2, 2)), adapt=adapt)
    sim.init()
    for args in [(1, 1, 1, 1), (1, 2, 1, 1), (2, 3, 2, 2), (1, 0, 3, 0)]:
        if args[0] < lmax:
            sim.refine(*args)
    sim.coarsen(0, 1, 0, 1)   # a level-0 leaf next to level-1 leaves
    set_leaves(sim, _bump)
    sim.project()
    return sim


def test_step_counts_and_clock(orc):
    sim = _bump_tree(orc)
    levels = {k[0] for k in sim.leaf_states()}
    assert levels == {0, 1, 2, 3}
    dt = sim.step_lts()
    np.testing.assert_array_equal(sim.lts_steps()[:5], [1, 2, 4, 8, 0])
    assert sim.time == 8 * dt


def test_single_level_is_the_global_step(orc):
    sims = []
    for _ in range(2):
        sim = orc.Sim(W.uniform_flow(lmax=0, n0=(2, 2, 2)), adapt=0).init()
        set_leaves(sim, _bump)
        sims.append(sim)
    a, g = sims
    for _ in range(3):
        assert a.step_lts() == g.step()
    A, G = a.leaf_states(), g.leaf_states()
    assert A.keys() == G.keys()
    for k in A:
        assert np.array_equal(A[k], G[k]), k
    assert a.time == g.time


@pytest.mark.parametrize("adapt", [0, 1])
def test_conservation_periodic_with_jumps(orc, adapt):
    sim = _bump_tree(orc, adapt=adapt)
    t0 = sim.totals()
    nb0 = len(sim.blocks())
    for _ in range(2):
        sim.step_lts()
    t1 = sim.totals()
    scale = np.array([1.5, 1.0, 1.0, 1.0, 5.0])
    assert np.all(np.abs(t1 - t0) <= 2e-14 * scale), (t1 - t0)
    if adapt:
        assert len(sim.blocks()) != nb0


def test_free_stream_to_round_off(orc):
    # the coarse and fine sums of equal fluxes over different step counts round
    # differently, so the adjustment leaves a few ulp where the global step is exact
    sim = jump_tree(orc)
    before = sim.leaf_states()
    sim.step_lts()
    after = sim.leaf_states()
    assert before.keys() == after.keys()
    for k in before:
        assert np.abs(after[k] - before[k]).max() <= 4e-16 * np.abs(before[k]).max(), k


def test_converges_to_global_stepping(orc):
    dt0 = _bump_tree(orc, lmax=2).dt()
    diffs = []
    for c in (1.0, 0.5):
        a, g = _bump_tree(orc, lmax=2), _bump_tree(orc, lmax=2)
        n = int(round(2 / c))
        for _ in range(n):
            a.step_lts_dt(c * dt0)
        for _ in range(4 * n):
            g.step_dt(c * dt0)
        assert abs(a.time - g.time) < 1e-15
        A, G = a.leaf_states(), g.leaf_states()
        diffs.append(max(np.abs(A[k] - G[k]).max() for k in A))
    assert diffs[0] > 1e-6                      # the two schemes do differ at jumps
    assert diffs[0] / diffs[1] > 1.8, diffs     # first order in the step


V_WAVE = (0.4, -0.2, 0.3)


def _wave(x, y, z, t=0.0):
    ph = 2 * np.pi * ((x - V_WAVE[0] * t) + (y - V_WAVE[1] * t) + (z - V_WAVE[2] * t))
    rho = 1.0 + 0.2 * np.sin(ph)
    return cons_field(rho, V_WAVE[0] + 0 * x, V_WAVE[1] + 0 * x, V_WAVE[2] + 0 * x, 1.0 + 0 * x)


def _wave_error(sim):
    e = 0.0
    for k, u in sim.leaf_states().items():
        x, y, z = centres(sim.problem, *k)
        e += np.abs(u[0] - _wave(x, y, z, sim.time)[0]).sum() * sim.problem.dx(k[0]) ** 3
    return e


def test_entropy_wave_error_close_to_global(orc):
    runs = []
    for _ in range(2):
        sim = orc.Sim(W.uniform_flow(lmax=2, n0=(2, 2, 2)), adapt=0).init()
        for args in [(1, 1, 1, 1), (1, 2, 1, 1), (1, 0, 3, 0)]:
            sim.refine(*args)
        set_leaves(sim, _wave)
        sim.project()
        runs.append(sim)
    a, g = runs
    dt = a.dt()
    for _ in range(4):
        a.step_lts_dt(dt)
    for _ in range(16):
        g.step_dt(dt)
    ea, eg = _wave_error(a), _wave_error(g)
    assert eg < 2e-6
    assert ea <= 1.1 * eg, (ea, eg)


def test_sod_axis_permutation_bitwise(orc):
    runs = []
    for axis in range(3):
        sim = orc.Sim(_sod(axis, 2, 2)).init()
        dts = [sim.step_lts() for _ in range(2)]
        runs.append((dts, sim.leaf_states()))
    dts_x, ref = runs[0]
    assert any(k[0] == 2 for k in ref) and any(k[0] < 2 for k in ref)
    for r in (1, 2):
        dts, got = runs[r]
        assert dts == dts_x
        exp = ref
        for _ in range(r):
            exp = {cyc_key(k): cyc_state(v) for k, v in exp.items()}
        assert got.keys() == exp.keys()
        for k in exp:
            assert np.array_equal(got[k], exp[k]), (r, k)
