"""Flags at the threshold: the GPU judge decides exactly as the oracle on identical input.

The GPU evaluates details with the separable prediction; where a slab's detail lies in a
narrow band around eps_l it evaluates them again with the appendix's Q-term sums in the
oracle's order (mrfv_set_detail_band).  Checked here on identical FP64 and FP32 input
(the oracle's padded arrays, halos included, handed to the GPU):
  * with the band forced wide open, every block's detail equals the oracle's bitwise;
  * with the default band, for thresholds placed exactly on a leaf's oracle detail and
    on the neighbouring doubles (eq:Thresholding: refine iff d >= eps_l), every flag
    equals the oracle's, and the planted leaf refines, refines, keeps respectively.
"""
import numpy as np
import pytest

from gpu_helpers import H, N, make_pair, oracle_map, oracle_padded_to_gpu, slot_map
from paper_2012_04385_amd import workloads as W

pytestmark = pytest.mark.gpu

REFS = [(1, 1, 1, 1), (1, 2, 1, 1), (2, 3, 2, 2), (1, 0, 3, 0)]


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


def _problem(eps):
    pb = W.uniform_flow(lmax=3, n0=(2, 2, 2))
    pb.eps = eps
    return pb


def _fields(orc, dtype):
    """Padded arrays of every block (oracle order keys): smooth data plus noise whose
    amplitude is spread over decades, halos filled by the oracle, rounded to the
    GPU's storage type."""
    o, _ = make_pair(orc, _problem(1e-3), REFS, dtype, adapt=1)
    rng = np.random.default_rng(11)
    om = oracle_map(o)
    for k, n in om.items():
        a = 10.0 ** rng.uniform(-7, -1)
        blk = o.get_block(n)
        base = np.ones((N, N, N))
        blk[0, H:H + N, H:H + N, H:H + N] = base + a * rng.standard_normal((N, N, N))
        blk[1:4, H:H + N, H:H + N, H:H + N] = 0.0
        blk[4, H:H + N, H:H + N, H:H + N] = 2.5 * base + a * rng.standard_normal((N, N, N))
        o.set_block(n, blk)
    o.fill_halos()
    out = {}
    for k, n in om.items():
        b = o.get_block(n)
        if dtype == "f32":
            b = b.astype(np.float32).astype(np.float64)
        out[k] = b
    return out


def _judge(orc, torch_mod, dtype, eps, fields, band=None):
    o, g = make_pair(orc, _problem(eps), REFS, dtype, adapt=1)
    om = oracle_map(o)
    assert set(om) == set(fields)
    for k, n in om.items():
        o.set_block(n, fields[k])
    oracle_padded_to_gpu(o, g)
    if band is not None:
        g.set_detail_band(band)
    det_o, fl_o = o.details()
    g.mr_flag()
    torch_mod.cuda.synchronize()
    gm = slot_map(g)
    det_g = g.det.cpu().numpy()
    fl_g = g.flags.cpu().numpy()
    d_o, d_g, f_o, f_g = {}, {}, {}, {}
    for n, r in enumerate(o.blocks()):
        k = tuple(int(v) for v in r[:4])
        d_o[k], f_o[k] = det_o[n], int(fl_o[n])
        d_g[k], f_g[k] = det_g[gm[k]], int(fl_g[gm[k]])
    return d_o, d_g, f_o, f_g


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_exact_details_bitwise(orc, torch_mod, dtype):
    fields = _fields(orc, dtype)
    d_o, d_g, f_o, f_g = _judge(orc, torch_mod, dtype, 1e-3, fields, band=1e300)
    fine = [k for k in d_o if k[0] >= 1]
    assert len(fine) > 90
    for k in fine:
        assert d_g[k] == d_o[k], (k, d_g[k], d_o[k])
    assert f_g == f_o
    # the separable form alone (band 0) agrees to round-off but not always bitwise
    d_o2, d_s, _, _ = _judge(orc, torch_mod, dtype, 1e-3, fields, band=0.0)
    assert max(abs(d_s[k] - d_o2[k]) / max(d_o2[k], 1e-300) for k in fine) <= 1e-12
    n_diff = sum(d_s[k] != d_o2[k] for k in fine)
    print(f"{dtype}: {n_diff} of {len(fine)} separable details differ from the Q-term ones in the last bits")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_flags_at_threshold(orc, torch_mod, dtype):
    fields = _fields(orc, dtype)
    d_o, _, f_o0, _ = _judge(orc, torch_mod, dtype, 1e-3, fields, band=1e300)
    lmax = 3
    # leaves that could refine (level < lmax), one per level 1 and 2, detail well above 0
    leaves = {k for k in d_o if k[0] >= 1 and f_o0[k] != 2}
    targets = []
    for lv in (1, 2):
        cand = sorted((k for k in leaves if k[0] == lv and d_o[k] > 1e-6), key=lambda k: d_o[k])
        assert cand, lv
        targets.append(cand[len(cand) // 2])
    for key in targets:
        eps_at = d_o[key] * 2.0 ** (3 * (lmax - key[0]))   # eps_l == d exactly (power-of-two scaling)
        for eps, want in ((eps_at, 1), (np.nextafter(eps_at, 0.0), 1), (np.nextafter(eps_at, np.inf), 0)):
            _, _, f_o, f_g = _judge(orc, torch_mod, dtype, float(eps), fields)
            assert f_o[key] == want, (key, eps, f_o[key])
            bad = [k for k in f_o if f_g[k] != f_o[k]]
            assert not bad, (key, eps, bad[:5])
