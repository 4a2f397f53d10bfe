"""The allocation-free totals entry point (mrfv_totals_noalloc) against mrfv_totals.

Two calls in a row on one device, the second on a smaller tree (the static scratch then
holds the larger call's partial sums beyond what the second call writes), on the FP32
batched and the FP64 plain path: the totals must equal those of mrfv_totals bitwise
(same kernels, same fixed summation order).
"""
import ctypes as C

import numpy as np
import pytest

from paper_2012_04385_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


def _both(g, torch):
    from paper_2012_04385_amd.mrfv import lib
    ref = g.totals().cpu().numpy().copy()
    out = torch.full_like(g.tot, float("nan"))
    rc = lib().mrfv_totals_noalloc(g.h, C.c_void_p(g.U.data_ptr()), C.c_void_p(out.data_ptr()))
    assert rc == 0, lib().mrfv_last_error(g.h)
    torch.cuda.synchronize()
    return ref, out.cpu().numpy()


@pytest.mark.parametrize("dtype,batched", [("f32", 2), ("f64", 0)])
def test_totals_noalloc_matches_totals(torch_mod, dtype, batched):
    from paper_2012_04385_amd.mrfv import Solver
    big = Solver([W.blast_mr3()], dtype=dtype, batched=batched).init()
    big.step()
    small = Solver([W.sod_single_level()], dtype=dtype, batched=batched).init()
    small.step()
    for g in (big, small):                       # the second call has fewer leaves
        ref, got = _both(g, torch_mod)
        assert np.isfinite(got).all()
        assert np.array_equal(ref, got), (ref, got)
    assert big.stats()[1] > 8 * small.stats()[1]
