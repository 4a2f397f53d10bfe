"""Shared helpers of the GPU parity tests: build the same tree on both sides, move data
between the oracle's blocks and the GPU slots, compare leaf states."""
import numpy as np

H, N, P = 4, 16, 24


def make_pair(orc, problem, refs=(), dtype="f64", batched=False, adapt=0):
    from paper_2012_04385_amd.mrfv import Solver
    o = orc.Sim(problem, adapt=adapt).init()
    g = Solver([problem], dtype=dtype, batched=batched, adapt=adapt).init()
    for r in refs:
        o.refine(*r)
        g.refine(0, *r)
    return o, g


def slot_map(g, inst=0):
    info = g.blocks()
    return {tuple(int(v) for v in r[2:6]): int(r[0]) for r in info if r[1] == inst}


def oracle_map(o):
    return {tuple(int(v) for v in r[:4]): n for n, r in enumerate(o.blocks())}


def same_tree(o, g, inst=0):
    ol = {tuple(int(v) for v in r[:4]) for r in o.blocks() if r[4] == 1}
    gl = {tuple(int(v) for v in r[2:6]) for r in g.blocks() if r[6] == 1 and r[1] == inst}
    return ol == gl, ol, gl


def random_physical(rng, shape, gamma=1.4, rough=0.05):
    """Random conservative states [5, ...] with rho, p > 0 and mixed-sign velocities."""
    rho = 1.0 + 0.3 * rng.random(shape) + rough * rng.standard_normal(shape)
    rho = np.maximum(rho, 0.3)
    u = 0.4 * rng.standard_normal(shape)
    v = 0.4 * rng.standard_normal(shape)
    w = 0.4 * rng.standard_normal(shape)
    p = 1.0 + 0.5 * rng.random(shape)
    E = p / (gamma - 1) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E])


def set_interiors(o, g, fn):
    """Write fn(key) -> [5,16,16,16] into the interiors of every block on both sides."""
    import torch
    om, gm = oracle_map(o), slot_map(g)
    assert set(om) == set(gm)
    for key, n in om.items():
        data = fn(key)
        blk = o.get_block(n)
        blk[:, H:H + N, H:H + N, H:H + N] = data
        o.set_block(n, blk)
        g.U[gm[key], :, H:H + N, H:H + N, H:H + N] = torch.as_tensor(data, dtype=g.tdtype, device=g.device)
    torch.cuda.synchronize()


def oracle_padded_to_gpu(o, g):
    import torch
    om, gm = oracle_map(o), slot_map(g)
    for key, n in om.items():
        g.U[gm[key]] = torch.as_tensor(o.get_block(n), dtype=g.tdtype, device=g.device)
    torch.cuda.synchronize()


def gpu_padded(g):
    import torch
    torch.cuda.synchronize()
    gm = slot_map(g)
    U = g.U.double().cpu().numpy()
    return {k: U[s] for k, s in gm.items()}


def l1_diff(o, g, q=0, inst=0):
    """Volume-weighted L1 difference of component q over the common leaves."""
    ol = o.leaf_states()
    gl = g.leaf_states(inst)
    pb = o.problem
    tot = 0.0
    for k, v in ol.items():
        h = pb.dx(k[0])
        tot += np.abs(gl[k][q] - v[q]).sum() * h ** 3
    return tot
