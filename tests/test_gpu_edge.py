"""Edge and degenerate cases of the GPU path, through the C ABI.

* Free stream: a uniform state on a tree with 1- and 2-level resolution jumps, periodic
  and zero-gradient, with and without adaptation, stays bitwise uniform on the FP32
  batched (step graph) and FP64 plain paths: every face sees a constant stencil (the
  WENO5 form returns its centre exactly), restriction and prediction reproduce constants
  exactly, and the increment-form update adds an exact zero.
* A single level-0 block on a periodic box is its own neighbour across every face
  (fused kernel reading its own interior as halo); compared with the oracle.
* Error paths: a non-physical state (negative pressure) is reported as MRFV_ENONPHYS,
  an initialisation that needs more slots than the capacity as MRFV_ENOMEM; both are
  host-visible status codes, the kernels exit normally.
"""
import numpy as np
import pytest

from paper_2012_04385_amd import workloads as W

pytestmark = pytest.mark.gpu

REFS = [(1, 1, 1, 1), (1, 2, 1, 1), (2, 3, 2, 2), (1, 0, 3, 0)]


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("dtype,batched", [("f32", 2), ("f64", 0)])
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 0, 1)])
@pytest.mark.parametrize("adapt", [0, 1])
def test_free_stream_bitwise(torch_mod, dtype, batched, bc, adapt):
    from paper_2012_04385_amd.mrfv import Solver
    pb = W.uniform_flow(lmax=3, n0=(2, 2, 2))
    pb.bc = bc
    g = Solver([pb], dtype=dtype, batched=batched, adapt=adapt).init()
    if not adapt:
        for r in REFS:
            g.refine(0, *r)
    s0 = g.leaf_states()
    u0 = next(iter(s0.values()))[:, 0, 0, 0]
    levels = {k[0] for k in s0}
    for _ in range(4):
        g.step()
    g.check()
    s = g.leaf_states()
    for k, v in s.items():
        assert np.array_equal(v, np.broadcast_to(u0[:, None, None, None], v.shape)), k
    print(f"free stream {dtype} bc={bc} adapt={adapt}: levels {sorted(levels)} -> "
          f"{sorted({k[0] for k in s})}, {len(s)} leaves uniform")
    if not adapt:
        assert len(levels) >= 3


@pytest.mark.parametrize("dtype,batched,tol", [("f64", 0, 1e-11), ("f32", 2, 5e-6)])
def test_single_block_periodic(orc, torch_mod, dtype, batched, tol):
    from paper_2012_04385_amd.mrfv import Solver
    pb = W.Problem(name="wave_1block", kind="custom", lmax=0, n0=(1, 1, 1), dx0=1 / 16, noise=0.0,
                   custom=lambda x, y, z: (1.0 + 0.2 * np.sin(2 * np.pi * (x + y)) * np.cos(2 * np.pi * z),
                                           0.5, -0.3, 0.2, 1.0))
    o = orc.Sim(pb).init()
    g = Solver([pb], dtype=dtype, batched=batched).init()
    for _ in range(3):
        o.step()
        g.step()
    g.check()
    so, sg = o.leaf_states(), g.leaf_states()
    assert so.keys() == sg.keys() == {(0, 0, 0, 0)}
    err = np.abs(so[(0, 0, 0, 0)] - sg[(0, 0, 0, 0)]).max()
    print(f"single block {dtype}: max |gpu - oracle| {err:.2e}")
    assert err <= tol


@pytest.mark.parametrize("dtype,batched", [("f32", 2), ("f64", 0)])
def test_nonphysical_state_reported(torch_mod, dtype, batched):
    from paper_2012_04385_amd.mrfv import MrfvError, Solver
    pb = W.Problem(name="negative_p", kind="custom", lmax=0, n0=(2, 2, 2), dx0=1 / 32, noise=0.0,
                   custom=lambda x, y, z: (1.0, 0.0, 0.0, 0.0, np.where(x < 0.25, -0.5, 1.0)))
    g = Solver([pb], dtype=dtype, batched=batched).init()
    with pytest.raises(MrfvError) as e:
        for _ in range(2):
            g.step()
        g.check()
    assert e.value.code == -5


def test_capacity_exhausted_reported(torch_mod):
    from paper_2012_04385_amd.mrfv import MrfvError, Solver
    pb = W.blast_mr3(steps=1)          # 8 level-0 blocks refine into 64 during algo:Init
    g = Solver([pb], dtype="f32", batched=2, capacity=40)
    with pytest.raises(MrfvError) as e:
        g.init()
    assert e.value.code == -3


def test_commit_capacity_leaves_tree_unchanged(torch_mod):
    """A commit that would need more slots than are free fails with ENOMEM before it
    changes anything: the tree, and the device tables built from it, stay as they were,
    and the context keeps stepping."""
    from paper_2012_04385_amd.mrfv import MrfvError, Solver
    pb = W.uniform_flow(lmax=3, n0=(2, 1, 1))
    # algo:Init needs 2 + 16 + 128 slots at its peak; 18 blocks remain
    g = Solver([pb], dtype="f32", batched=2, capacity=146).init()
    g.refine(0, 1, 0, 0, 0)                      # 26 blocks, 120 free slots
    before = g.blocks().copy()
    flags = np.zeros(g.capacity, dtype=np.int8)
    for r in before:
        if r[6] == 1 and r[2] == 1:
            flags[r[0]] = 1                      # 15 level-1 leaves: 120 slots
    lvl2 = [r for r in before if r[6] == 1 and r[2] == 2]
    flags[lvl2[0][0]] = 1                        # and one more: 128 > 120
    with pytest.raises(MrfvError) as e:
        g.commit_flags(flags)
    assert e.value.code == -3
    after = g.blocks()
    assert np.array_equal(np.sort(before, axis=0), np.sort(after, axis=0))
    g.step()                                     # the uniform field coarsens the group again
    g.check()
