"""Interface displacement and growth rate of the Rayleigh-Taylor study
(Sec. "Rayleigh-Taylor instability", eq:NumericGrowthRate).

The apparent interface position on a vertical line is where the density crosses the
mean of the two fluid densities, located to sub-cell accuracy by linear interpolation
between the cell centres on either side (the paper takes the position of the largest
density gradient; on the smoothed profile both mark its middle).  The displacement d(t)
is half the distance between the interface heights on the lines at the two ends of the
wavelength (x = dx/2, where the light fluid rises, and x = lambda/2 - dx/2, where the
heavy fluid falls), which cancels any uniform vertical motion.  The growth rate is
n = d/dt ln(d(t) / d(0)), fitted by least squares over a window of the run.
"""
from __future__ import annotations

import numpy as np

H, N = 4, 16


def column_profile(solver, pb, ix_fine: int, inst: int = 0):
    """(y, rho) at the cell centres of every leaf cell on the vertical line through the
    finest-level cell column ix_fine (x index on level lmax), mid-depth in z; sorted by y."""
    torch = solver.torch
    info = solver.blocks()
    info = info[(info[:, 6] == 1) & (info[:, 1] == inst)]
    lmax = pb.lmax
    nz_fine = pb.n0[2] * N << lmax
    iz_fine = nz_fine // 2
    ys, slots, cells = [], [], []
    for slot, _, lvl, bx, by, bz, _, _ in info:
        sh = lmax - int(lvl)
        gx, gz = ix_fine >> sh, iz_fine >> sh          # cell index on the leaf's level
        if gx // N != bx or gz // N != bz:
            continue
        h = pb.dx(int(lvl))
        ys.append((by * N + np.arange(N) + 0.5) * h)
        slots.append(int(slot))
        cells.append((gz % N, gx % N))
    if not slots:
        raise ValueError("no leaf on that line")
    sl = torch.as_tensor(slots, device=solver.device)
    kz = torch.as_tensor([c[0] for c in cells], device=solver.device) + H
    kx = torch.as_tensor([c[1] for c in cells], device=solver.device) + H
    rho = solver.U[sl, 0, kz, H:H + N, :]                       # [n, 16 (y), 24 (x)]
    rho = rho.gather(2, kx.view(-1, 1, 1).expand(-1, N, 1))[:, :, 0]
    rho = rho.double().cpu().numpy().reshape(-1)
    y = np.concatenate(ys)
    o = np.argsort(y)
    return y[o], rho[o]


def interface_height(y, rho, level: float) -> float:
    """Height where rho crosses `level`, by linear interpolation (the lowest crossing)."""
    s = np.sign(rho - level)
    idx = np.nonzero(s[:-1] != s[1:])[0]
    if len(idx) == 0:
        raise ValueError("the profile does not cross the level")
    i = idx[0]
    t = (level - rho[i]) / (rho[i + 1] - rho[i])
    return float(y[i] + t * (y[i + 1] - y[i]))


def displacement(solver, pb, inst: int = 0) -> float:
    """Half the height difference of the interface between x = dx/2 and x = lambda/2 - dx/2."""
    prm = pb.params
    level = 0.5 * (prm["rho_h"] + prm["rho_l"])
    nx = pb.n0[0] * N << pb.lmax
    y0, r0 = column_profile(solver, pb, 0, inst)
    y1, r1 = column_profile(solver, pb, nx // 2 - 1, inst)
    return 0.5 * (interface_height(y0, r0, level) - interface_height(y1, r1, level))


def growth_rate(t, d, t_lo: float, t_hi: float) -> float:
    """Least-squares slope of ln d(t) over t_lo <= t <= t_hi."""
    t, d = np.asarray(t), np.asarray(d)
    m = (t >= t_lo) & (t <= t_hi)
    if m.sum() < 3:
        raise ValueError("too few samples in the window")
    return float(np.polyfit(t[m], np.log(d[m]), 1)[0])
