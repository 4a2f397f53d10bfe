"""Seeded synthetic workloads: problem definitions and initial conditions.

This module only generates inputs.  It holds none of the method's arithmetic: initial
conditions are returned as primitive fields (rho, u, v, w, p) sampled at cell centres,
and every consumer (the GPU library and the CPU oracle) converts them to conservative
variables with its own equation of state.  Both sides of a parity check receive the
same arrays from here.

Cell-centre sampling and a per-cell, per-level additive density noise follow the
paper's level-by-level initialisation (algo:Init): every level of the tree samples the
initial condition on its own grid.  The noise is a counter-based generator (SplitMix64
finaliser over a hash of seed, instance, level and global cell index), so any block
can be generated independently and in any order.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional, Tuple

import numpy as np

IC = 16  # interior cells per block edge
BASE_SEED = 201204385

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea & Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, instance: int, level: int, gx, gy, gz) -> np.ndarray:
    """Counter-based uniform [0,1) numbers for global cell indices (gx, gy, gz)."""
    gx = np.asarray(gx, dtype=np.uint64)
    gy = np.asarray(gy, dtype=np.uint64)
    gz = np.asarray(gz, dtype=np.uint64)
    with np.errstate(over="ignore"):
        key = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        key = _splitmix64(key ^ np.uint64(instance))
        key = _splitmix64(key ^ np.uint64(level))
        h = _splitmix64(key ^ gz)
        h = _splitmix64(h ^ gy)
        h = _splitmix64(h ^ gx)
    return (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


@dataclasses.dataclass
class Problem:
    """One MR problem instance (one octree forest)."""

    name: str
    kind: str                      # "sod", "blast", "kh", "shock_blobs", "uniform", "custom"
    gamma: float = 1.4
    B: float = 0.0
    cfl: float = 0.5
    eps: float = 1e-3              # threshold on the finest level
    scale_rho: float = 1.0         # normalisation of rho details
    scale_E: float = 1.0           # normalisation of E details
    lmax: int = 0
    n0: Tuple[int, int, int] = (1, 1, 1)
    dx0: float = 1.0 / 16.0
    # per axis: 0 periodic, 1 zero-gradient, 2 symmetry, 3 fixed values (the initial
    # condition continued into the halo, see bc_fixed_states)
    bc: Tuple[int, int, int] = (0, 0, 0)
    steps: int = 10
    seed: int = BASE_SEED
    instance: int = 0
    noise: float = 1e-3
    params: dict = dataclasses.field(default_factory=dict)
    custom: Optional[Callable] = None      # custom(x, y, z) -> (rho, u, v, w, p)
    # flux kernel (Sec. "Numerical Scheme"): roe_weno5 (the standard configuration),
    # roe_teno5, llf_weno5, hllc_wao53
    scheme: str = "roe_weno5"
    # gravity vector of the source term of eq:Euler (zero: no source)
    gravity: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    # equation of state: "stiffened" (eq:StiffenedGas with gamma, B) or "tait"
    # (p = B ((rho/rho0)^gamma - 1) + A; the energy is not evolved and the IC pressure unused)
    eos: str = "stiffened"
    tait_A: float = 1.0
    tait_rho0: float = 1.0
    # dynamic viscosity of the Navier-Stokes form (0: Euler equations)
    mu: float = 0.0

    @property
    def adapt(self) -> int:
        return 1 if self.lmax > 0 else 0

    def dx(self, level: int) -> float:
        return self.dx0 / (1 << level)

    def cell_centres(self, level: int, bx: int, by: int, bz: int):
        """Global cell indices and centre coordinates of a block's interior, shape (16,)*3
        in [z][y][x] order."""
        ar = np.arange(IC)
        gz, gy, gx = np.meshgrid(bz * IC + ar, by * IC + ar, bx * IC + ar, indexing="ij")
        h = self.dx(level)
        return (gx, gy, gz), ((gx + 0.5) * h, (gy + 0.5) * h, (gz + 0.5) * h)

    def bc_fixed_states(self) -> Optional[np.ndarray]:
        """Halo states of the fixed-value boundaries: the initial condition (without noise)
        at the halo cell centres beyond each side of the axes with bc 3, taken on the
        line through the middle of the boundary plane (such problems are uniform along
        their fixed boundaries).  [6 sides x-, x+, y-, y+, z-, z+][lmax + 1][4 layers, the
        one at the face first][5 primitives]; None if no axis has bc 3."""
        if 3 not in tuple(self.bc):
            return None
        out = np.zeros((6, self.lmax + 1, 4, 5))
        ext = [self.n0[a] * IC * self.dx0 for a in range(3)]
        for a in range(3):
            if self.bc[a] != 3:
                continue
            for side in range(2):
                for lvl in range(self.lmax + 1):
                    h = self.dx(lvl)
                    c = [np.full(4, 0.5 * ext[b]) for b in range(3)]
                    lay = np.arange(4) + 0.5
                    c[a] = ext[a] + lay * h if side else -lay * h
                    st = _STATES[self.kind](self, *c)
                    for q in range(5):
                        out[2 * a + side, lvl, :, q] = np.broadcast_to(st[q], (4,))
        return out

    def primitives(self, level: int, bx: int, by: int, bz: int) -> np.ndarray:
        """Initial primitive state (rho, u, v, w, p) of one block interior, [5][16][16][16]."""
        (gx, gy, gz), (x, y, z) = self.cell_centres(level, bx, by, bz)
        rho, u, v, w, p = _STATES[self.kind](self, x, y, z)
        if self.noise:
            r = uniform01(self.seed, self.instance, level, gx, gy, gz)
            rho = rho + self.noise * (2.0 * r - 1.0)
        out = np.empty((5, IC, IC, IC), dtype=np.float64)
        for q, f in enumerate((rho, u, v, w, p)):
            out[q] = f
        return out


def _full(x, val):
    return np.full(np.shape(x), float(val), dtype=np.float64)


def _sod(pb: Problem, x, y, z):
    prm = pb.params
    axis = prm.get("axis", 0)
    pos = prm.get("pos", 0.5)
    c = (x, y, z)[axis]
    left = c < pos
    rl, pl = prm.get("left", (1.0, 1.0))
    rr, pr = prm.get("right", (0.125, 0.1))
    rho = np.where(left, rl, rr)
    p = np.where(left, pl, pr)
    zero = _full(x, 0.0)
    return rho, zero, zero.copy(), zero.copy(), p


def _blast(pb: Problem, x, y, z):
    prm = pb.params
    cx, cy, cz = prm.get("centre", (0.5, 0.5, 0.5))
    r0 = prm.get("radius", 0.1)
    ri, pi = prm.get("inner", (1.0, 10.0))
    ro, po = prm.get("outer", (0.125, 0.1))
    inside = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 < r0 * r0
    rho = np.where(inside, ri, ro)
    p = np.where(inside, pi, po)
    zero = _full(x, 0.0)
    return rho, zero, zero.copy(), zero.copy(), p


def _kh(pb: Problem, x, y, z):
    """Shear layer: |y-1/2| < 1/4 carries rho=2, u=+0.5, else rho=1, u=-0.5; p = 2.5;
    v = sum over modes m=1..8 of (A/8) sin(2 pi m x + phi_m) [G(y-1/4) + G(y-3/4)]."""
    prm = pb.params
    amp = prm.get("amp", 0.01)
    modes = prm.get("modes", 8)
    width = prm.get("width", 0.05)
    rng = np.random.default_rng(pb.seed)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=modes)
    band = np.abs(y - 0.5) < 0.25
    rho = np.where(band, 2.0, 1.0)
    u = np.where(band, 0.5, -0.5)
    g = np.exp(-((y - 0.25) ** 2) / (2 * width * width)) + np.exp(-((y - 0.75) ** 2) / (2 * width * width))
    v = np.zeros_like(x)
    for m in range(1, modes + 1):
        v = v + (amp / modes) * np.sin(2.0 * math.pi * m * x + phi[m - 1]) * g
    return rho, u, v, _full(x, 0.0), _full(x, 2.5)


def _shock_blobs(pb: Problem, x, y, z):
    """Mach-2 shock at x = x_s moving +x into gas at rest (p = 1) whose density carries
    32 seeded Gaussian blobs.  Post-shock state from the Rankine-Hugoniot relations for
    gamma = 1.4, M = 2 (tabulated values, not computed here)."""
    prm = pb.params
    xs = prm.get("x_shock", 0.1)
    post = prm.get("post", (8.0 / 3.0, 1.479019945774904, 4.5))
    nblob = prm.get("blobs", 32)
    amp = prm.get("amp", 0.5)
    wid = prm.get("width", 0.02)
    rng = np.random.default_rng(pb.seed)
    cs = np.stack([rng.uniform(0.2, 0.9, nblob), rng.uniform(0.1, 0.9, nblob),
                   rng.uniform(0.1, 0.9, nblob)], axis=1)
    rho = np.ones_like(x)
    for c in cs:
        rho = rho + amp * np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2 * wid * wid))
    behind = x < xs
    rho = np.where(behind, post[0], rho)
    u = np.where(behind, post[1], 0.0)
    p = np.where(behind, post[2], 1.0)
    return rho, u, _full(x, 0.0), _full(x, 0.0), p


def _rti(pb: Problem, x, y, z):
    """Heavy fluid (rho_h) above a light one (rho_l) under gravity -g along y, interface
    y_i(x) = y0 + a cos(k x) smoothed as a tanh of thickness delta, at rest; pressure in
    hydrostatic balance with the unperturbed (flat) profile, p0 at y0:
    p(y) = p0 - g (rho_m (y - y0) + (rho_h - rho_l)/2 delta ln cosh((y - y0)/delta))."""
    prm = pb.params
    rh, rl, g = prm["rho_h"], prm["rho_l"], prm["g"]
    k, a, y0, dl, p0 = prm["k"], prm["amp"], prm["y0"], prm["delta"], prm["p0"]
    yi = y0 + a * np.cos(k * x)
    rho = rl + (rh - rl) * 0.5 * (1.0 + np.tanh((y - yi) / dl))
    s = (y - y0) / dl
    lncosh = np.abs(s) + np.log1p(np.exp(-2.0 * np.abs(s))) - math.log(2.0)
    p = p0 - g * (0.5 * (rh + rl) * (y - y0) + 0.5 * (rh - rl) * dl * lncosh)
    zero = _full(x, 0.0)
    return rho, zero, zero.copy(), zero.copy(), p


def _wc_blast(pb: Problem, x, y, z):
    """Woodward and Colella's interacting blast waves along y: gas at rest, rho = 1,
    p = 1000 below y = 0.1, 0.01 in between, 100 above y = 0.9."""
    prm = pb.params
    lo, hi = prm.get("lo", 0.1), prm.get("hi", 0.9)
    p = np.where(y < lo, prm.get("p_left", 1000.0), np.where(y > hi, prm.get("p_right", 100.0),
                                                              prm.get("p_mid", 0.01)))
    zero = _full(x, 0.0)
    return _full(x, 1.0), zero, zero.copy(), zero.copy(), p


def _uniform(pb: Problem, x, y, z):
    r, u, v, w, p = pb.params.get("state", (1.3, 0.3, -0.2, 0.1, 0.9))
    return _full(x, r), _full(x, u), _full(x, v), _full(x, w), _full(x, p)


def _custom(pb: Problem, x, y, z):
    out = pb.custom(x, y, z)
    return tuple(np.broadcast_to(np.asarray(f, dtype=np.float64), np.shape(x)).copy() for f in out)


_STATES = {"sod": _sod, "blast": _blast, "kh": _kh, "shock_blobs": _shock_blobs,
           "uniform": _uniform, "custom": _custom, "rti": _rti, "wc_blast": _wc_blast}


# ---------------------------------------------------------------- named workloads -----

def sod_single_level(seed_k: int = 1) -> Problem:
    """Plain method, single level: 32^3 cells as 2^3 blocks of 16^3, x-direction Sod tube
    (rho,u,p) = (1,0,1) | (0.125,0,0.1) at x = 0.5, +-1e-3 density noise, periodic in y,z,
    zero-gradient in x, CFL 0.5, 10 steps (FP64)."""
    return Problem(name="sod_32c_1lvl", kind="sod", lmax=0, n0=(2, 2, 2), dx0=1.0 / 32,
                   bc=(1, 0, 0), steps=10, seed=BASE_SEED + seed_k, noise=1e-3,
                   scale_rho=1.0, scale_E=2.5, eps=1e-3,
                   params={"axis": 0, "pos": 0.5, "left": (1.0, 1.0), "right": (0.125, 0.1)})


def sod_tait_mr3(seed_k: int = 6, steps: int = 40, eos: str = "tait") -> Problem:
    """Sec. "Influence of Equation of State": Sod tube along x with l_max = 3 (2 level-0
    blocks in x, 256 cells effective), Tait's equation with gamma 1.4, A = 1, B = 0.937315,
    rho0 = 1 (eos = "stiffened": the same tube with the ideal gas), densities 1 | 0.125 at
    rest, pressures 1 | 0.1 for the ideal gas, zero-gradient in x, periodic in y and z."""
    return Problem(name=f"sod_{eos}_256e_4lvl", kind="sod", lmax=3, n0=(2, 1, 1), dx0=1.0 / 32,
                   bc=(1, 0, 0), steps=steps, seed=BASE_SEED + seed_k, noise=0.0,
                   scale_rho=1.0, scale_E=2.5, eps=1e-3, cfl=0.5, B=0.937315 if eos == "tait" else 0.0,
                   eos=eos, tait_A=1.0, tait_rho0=1.0,
                   params={"axis": 0, "pos": 0.5, "left": (1.0, 1.0), "right": (0.125, 0.1)})


def blast_mr3(seed_k: int = 2, steps: int = 50) -> Problem:
    """MR, 3 levels, 128^3 effective, 16^3 blocks: spherical blast in a unit periodic box,
    radius 0.1 at (rho,p) = (1,10) inside and (0.125,0.1) outside, +-1e-3 density noise,
    Harten threshold 1e-3 on the finest level, 50 steps."""
    return Problem(name="blast_128e_3lvl", kind="blast", lmax=2, n0=(2, 2, 2), dx0=1.0 / 32,
                   bc=(0, 0, 0), steps=steps, seed=BASE_SEED + seed_k, noise=1e-3, eps=1e-3,
                   scale_rho=1.0, scale_E=25.0,
                   params={"centre": (0.5, 0.5, 0.5), "radius": 0.1, "inner": (1.0, 10.0),
                           "outer": (0.125, 0.1)})


def local_blast_mr5(seed_k: int = 10, steps: int = 20) -> Problem:
    """A localised 3D feature on a 5-level tree, the kind of tree local time stepping is for:
    a blast of radius 0.05 at the centre of a periodic unit box, (rho, p) = (1, 10) inside
    and (0.125, 0.1) outside, at rest, no noise; l_max = 4, 4^3 level-0 blocks (256^3
    effective).  After algo:Init 1240 leaves, 512 of them on level 4."""
    return Problem(name="localblast_256e_5lvl", kind="blast", lmax=4, n0=(4, 4, 4), dx0=1.0 / 64,
                   bc=(0, 0, 0), steps=steps, seed=BASE_SEED + seed_k, noise=0.0, eps=1e-3,
                   scale_rho=1.0, scale_E=25.0,
                   params={"centre": (0.5, 0.5, 0.5), "radius": 0.05, "inner": (1.0, 10.0),
                           "outer": (0.125, 0.1)})


def kh_mr5(seed_k: int = 3, steps: int = 20) -> Problem:
    """5-level MR, 256^3 effective: Kelvin-Helmholtz shear layer (rho = 2|1, u = +-0.5,
    p = 2.5) with seeded sinusoidal v-perturbations of amplitude 0.01 over modes 1-8."""
    return Problem(name="kh_256e_5lvl", kind="kh", lmax=4, n0=(1, 1, 1), dx0=1.0 / 16,
                   bc=(0, 0, 0), steps=steps, seed=BASE_SEED + seed_k, noise=0.0, eps=1e-3,
                   scale_rho=2.0, scale_E=6.5, params={"amp": 0.01, "modes": 8, "width": 0.05})


def multi_instance(n: int = 256, seed_k: int = 4, steps: int = 20):
    """Uneven batch of independent MR problems: effective grid N in {32,64,128}^3 with
    2-4 levels (L <= 1 + log2(N/16)), each a blast or Sod tube with seeded centre/plane,
    radius in [0.05,0.2] and pressure ratio in [5,100]."""
    rng = np.random.default_rng(BASE_SEED + seed_k)
    out = []
    for i in range(n):
        N = int(rng.choice([32, 64, 128]))
        Lmax_levels = min(4, 1 + int(round(math.log2(N // 16))))
        L = int(rng.integers(2, Lmax_levels + 1))
        lmax = L - 1
        n0 = N // (16 << lmax)
        ratio = float(rng.uniform(5.0, 100.0))
        if rng.random() < 0.5:
            c = tuple(float(v) for v in rng.uniform(0.3, 0.7, 3))
            r0 = float(rng.uniform(0.05, 0.2))
            pb = Problem(name=f"blast{i}", kind="blast", lmax=lmax, n0=(n0,) * 3, dx0=1.0 / (16 * n0),
                         bc=(0, 0, 0), steps=steps, seed=BASE_SEED + seed_k, instance=i,
                         noise=1e-3, eps=1e-3, scale_rho=1.0, scale_E=0.25 * ratio,
                         params={"centre": c, "radius": r0, "inner": (1.0, 0.1 * ratio),
                                 "outer": (0.125, 0.1)})
        else:
            axis = int(rng.integers(0, 3))
            pos = float(rng.uniform(0.3, 0.7))
            bc = [0, 0, 0]
            bc[axis] = 1
            pb = Problem(name=f"sod{i}", kind="sod", lmax=lmax, n0=(n0,) * 3, dx0=1.0 / (16 * n0),
                         bc=tuple(bc), steps=steps, seed=BASE_SEED + seed_k, instance=i,
                         noise=1e-3, eps=1e-3, scale_rho=1.0, scale_E=0.25 * ratio,
                         params={"axis": axis, "pos": pos, "left": (1.0, 0.1 * ratio),
                                 "right": (0.125, 0.1)})
        out.append(pb)
    return out


def shock_blobs_mr6(seed_k: int = 5, steps: int = 30) -> Problem:
    """6-level MR, 512^3 effective: Mach-2 shock hitting 32 seeded Gaussian density blobs
    (amplitude 0.5, width 0.02); zero-gradient in x, periodic in y,z."""
    return Problem(name="shockblobs_512e_6lvl", kind="shock_blobs", lmax=5, n0=(1, 1, 1),
                   dx0=1.0 / 16, bc=(1, 0, 0), steps=steps, seed=BASE_SEED + seed_k, noise=0.0,
                   eps=1e-3, scale_rho=8.0 / 3.0, scale_E=12.0,
                   params={"x_shock": 0.1, "blobs": 32, "amp": 0.5, "width": 0.02})


def wc_blast_mr4(scheme: str = "roe_weno5", steps: int = 25, seed_k: int = 8) -> Problem:
    """The weak-scaling case of Sec. "Weak Scaling" in its one-core size: Woodward and
    Colella's interacting blast waves along y, l_max = 3, 128 x 512 x 128 cells effective
    (level 0: one block across x and z, four along y, dx0 = 1/64), reflecting (symmetry)
    walls at y = 0 and 1, periodic in x and z, CFL 0.9, 25 steps; flux kernel `scheme`."""
    return Problem(name=f"wcblast_128x512x128_4lvl_{scheme}", kind="wc_blast", lmax=3, n0=(1, 4, 1),
                   dx0=1.0 / 64, bc=(0, 2, 0), steps=steps, seed=BASE_SEED + seed_k, noise=0.0, eps=1e-3,
                   scale_rho=1.0, scale_E=2500.0, cfl=0.9, scheme=scheme, params={})


# fluid properties of the Rayleigh-Taylor growth-rate study per Atwood number:
# (rho_h, rho_l, mu); g = 1 for both
RTI_FLUIDS = {0.5: (1.5, 0.5, 0.1), 0.998: (99.9, 0.1, 0.5)}


def rti(k: float = 1.0, atwood: float = 0.5, lmax: int = 3, steps: int = 0, p0: Optional[float] = None,
        delta_cells: float = 1.0, amp: Optional[float] = None, eps: float = 1e-3,
        long_blocks: int = 10) -> Problem:
    """Sec. "Rayleigh-Taylor instability" with the fluids of its table of inputs: the short
    sides span one wavelength 2 pi / k, the long (vertical, y) side ten (1:10, one level-0
    block across, ten along y, 16 * 2^lmax cells per wavelength: 1280 cells along y at
    lmax = 3); interface at mid-height deflected by amp cos(k x), amp = 0.05 / k; gravity
    -g along y; symmetry planes on the sides, fixed values (the hydrostatic initial state
    continued) at top and bottom; one ideal gas (gamma 1.4) whose density
    jumps at the interface, both fluids with the same dynamic viscosity.  p0 (interface
    pressure) defaults to 15 wavelengths of heavy-fluid weight, which keeps the top at 10
    and the flow nearly incompressible (g / (k c^2) < 0.01 at k = 1)."""
    rh, rl, mu = RTI_FLUIDS[atwood]
    g = 1.0
    lam = 2.0 * math.pi / k
    dx0 = lam / 16.0
    return Problem(name=f"rti_at{atwood}_k{k:g}_{lmax + 1}lvl", kind="rti", lmax=lmax,
                   n0=(1, long_blocks, 1), dx0=dx0, bc=(2, 3, 2), steps=steps, noise=0.0, eps=eps,
                   scale_rho=rh, scale_E=(p0 or 15.0 * lam * rh * g) / 0.4, cfl=0.5,
                   gravity=(0.0, -g, 0.0), mu=mu,
                   params={"rho_h": rh, "rho_l": rl, "g": g, "k": k,
                           "amp": 0.05 / k if amp is None else amp,
                           "y0": 0.5 * long_blocks * lam, "delta": delta_cells * dx0 / (1 << lmax),
                           "p0": p0 or 15.0 * lam * rh * g})


def uniform_flow(lmax: int = 2, n0=(1, 1, 1), state=(1.3, 0.3, -0.2, 0.1, 0.9)) -> Problem:
    """Uniform free stream on a periodic box (free-stream preservation check)."""
    return Problem(name="uniform", kind="uniform", lmax=lmax, n0=tuple(n0), dx0=1.0 / (16 * n0[0]),
                   bc=(0, 0, 0), steps=20, noise=0.0, eps=1e-3, scale_rho=1.0, scale_E=1.0,
                   params={"state": state})
