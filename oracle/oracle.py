"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg import this
module.  The product path (the HIP library and its Python binding) never does.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

P, H, N = 24, 4, 16
MAX_LEVELS = 16


class _Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("B", C.c_double), ("cfl", C.c_double),
                ("eps", C.c_double), ("scale_rho", C.c_double), ("scale_E", C.c_double),
                ("dx0", C.c_double), ("lmax", C.c_int32), ("n0", C.c_int32 * 3),
                ("bc", C.c_int32 * 3), ("adapt", C.c_int32), ("scheme", C.c_int32),
                ("gravity", C.c_double * 3), ("eos", C.c_int32), ("tait_A", C.c_double),
                ("tait_rho0", C.c_double), ("mu", C.c_double), ("bc_fixed", C.POINTER(C.c_double))]


IC_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                    C.POINTER(C.c_double))


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liborc.so")
        if not os.path.exists(path):
            from . import build as _b  # noqa: F401  (package-relative when imported as oracle.oracle)
            _b.build()
        L = C.CDLL(path)
        d, i32, vp = C.c_double, C.c_int32, C.c_void_p
        pd = C.POINTER(C.c_double)
        L.orc_pressure.argtypes = [pd, d, d]
        L.orc_pressure.restype = d
        L.orc_flux_x.argtypes = [pd, d, d, pd]
        L.orc_roe_matrices.argtypes = [pd, pd, d, d, pd, pd]
        L.orc_weno5_minus.argtypes = [d] * 5
        L.orc_weno5_minus.restype = d
        L.orc_face_flux_x.argtypes = [pd, d, d, pd]
        L.orc_face_flux_x.restype = C.c_int
        L.orc_face_flux.argtypes = [C.c_int, pd, d, d, pd]
        L.orc_face_flux.restype = C.c_int
        L.orc_predict_cell.argtypes = [pd] + [C.c_int] * 6
        L.orc_predict_cell.restype = d
        L.orc_average8.argtypes = [pd]
        L.orc_average8.restype = d
        L.orc_ssprk3_stage.argtypes = [C.c_int, d, d, d, d]
        L.orc_ssprk3_stage.restype = d
        L.orc_exact_riemann.argtypes = [d] * 7 + [pd, C.c_int, pd]
        L.orc_exact_riemann.restype = C.c_int
        L.orc_sim_create.argtypes = [C.POINTER(_Params)]
        L.orc_sim_create.restype = vp
        L.orc_sim_free.argtypes = [vp]
        L.orc_sim_init.argtypes = [vp, IC_FN, vp]
        L.orc_sim_init.restype = C.c_int
        L.orc_sim_step.argtypes = [vp, pd]
        L.orc_sim_step.restype = C.c_int
        L.orc_sim_step_dt.argtypes = [vp, d]
        L.orc_sim_step_dt.restype = C.c_int
        L.orc_sim_step_lts_dt.argtypes = [vp, d]
        L.orc_sim_step_lts_dt.restype = C.c_int
        L.orc_sim_step_lts.argtypes = [vp, pd]
        L.orc_sim_step_lts.restype = C.c_int
        L.orc_sim_lts_steps.argtypes = [vp, C.POINTER(C.c_int64)]
        L.orc_lts_lowest_ending.argtypes = [i32, i32]
        L.orc_lts_lowest_ending.restype = i32
        L.orc_sim_nblocks.argtypes = [vp]
        L.orc_sim_nblocks.restype = i32
        L.orc_sim_blocks.argtypes = [vp, C.POINTER(C.c_int64)]
        L.orc_sim_get_block.argtypes = [vp, i32, pd]
        L.orc_sim_set_block.argtypes = [vp, i32, pd]
        L.orc_sim_detail.argtypes = [vp, i32]
        L.orc_sim_detail.restype = d
        L.orc_sim_refine.argtypes = [vp, i32, i32, i32, i32]
        L.orc_sim_refine.restype = C.c_int
        L.orc_sim_coarsen.argtypes = [vp, i32, i32, i32, i32]
        L.orc_sim_coarsen.restype = C.c_int
        L.orc_sim_project.argtypes = [vp]
        L.orc_sim_fill_halos.argtypes = [vp]
        L.orc_sim_rhs.argtypes = [vp, pd]
        L.orc_sim_rhs.restype = i32
        L.orc_sim_details.argtypes = [vp, pd, C.POINTER(C.c_int8)]
        L.orc_sim_dt.argtypes = [vp]
        L.orc_sim_dt.restype = d
        L.orc_sim_totals.argtypes = [vp, pd]
        L.orc_sim_time.argtypes = [vp]
        L.orc_sim_time.restype = d
        L.orc_sim_llf_fraction.argtypes = [vp]
        L.orc_sim_llf_fraction.restype = d
        L.orc_num_threads.restype = C.c_int
        L.orc_teno5_minus.argtypes = [d] * 5
        L.orc_teno5_minus.restype = d
        L.orc_wao53_minus.argtypes = [d] * 5
        L.orc_wao53_minus.restype = d
        L.orc_beta_quartic.argtypes = [d] * 5
        L.orc_beta_quartic.restype = d
        L.orc_hllc_flux_x.argtypes = [pd, pd, d, d, pd]
        L.orc_face_flux_scheme.argtypes = [C.c_int, C.c_int, pd, d, d, pd]
        L.orc_face_flux_scheme.restype = C.c_int
        L.orc_block_rhs_scheme.argtypes = [C.c_int, pd, d, d, d, pd]
        L.orc_morton_encode.argtypes = [i32] * 5
        L.orc_morton_encode.restype = C.c_uint64
        L.orc_morton_neighbor.argtypes = [C.c_uint64, i32, i32, C.POINTER(i32)]
        L.orc_morton_neighbor.restype = C.c_uint64
        L.orc_morton_level.argtypes = [C.c_uint64, i32]
        L.orc_morton_level.restype = i32
        L.orc_mlp_nparams.restype = C.c_int
        L.orc_bf16_round.argtypes = [d]
        L.orc_bf16_round.restype = d
        L.orc_mlp_forward.argtypes = [pd, pd, C.c_int, C.c_int, pd]
        L.orc_mlp_loss_grad.argtypes = [pd, pd, C.POINTER(C.c_int32), pd, C.c_int, C.c_int, pd]
        L.orc_mlp_loss_grad.restype = d
        L.orc_features.argtypes = [pd, d, d, d, d, d, pd]
        L.orc_block_rhs.argtypes = [pd, d, d, d, pd]
        L.orc_tait_pressure.argtypes = [d, d, d, d, d]
        L.orc_tait_pressure.restype = d
        L.orc_tait_sound_speed.argtypes = [d, d, d, d]
        L.orc_tait_sound_speed.restype = d
        L.orc_tait_flux_x.argtypes = [pd, d, d, d, d, pd]
        L.orc_tait_roe_matrices.argtypes = [pd, pd, d, d, d, d, pd, pd]
        L.orc_tait_face_flux.argtypes = [C.c_int, pd, d, d, d, d, pd]
        L.orc_tait_face_flux.restype = C.c_int
        L.orc_tait_exact_riemann.argtypes = [d, d, d, d, d, d, d, d, pd, C.c_int, pd]
        L.orc_tait_exact_riemann.restype = C.c_int
        L.orc_visc_face_flux.argtypes = [C.c_int, pd, d, C.c_int, d, pd]
        L.orc_visc_dt.argtypes = [d, d, d, d]
        L.orc_visc_dt.restype = d
        L.orc_rti_growth_rate.argtypes = [d, d, d, d, d]
        L.orc_rti_growth_rate.restype = d
        L.orc_block_rhs.restype = None
        L.orc_block_detail.argtypes = [pd, pd, C.c_int, C.c_int, C.c_int, d, d]
        L.orc_block_detail.restype = d
        _LIB = L
    return _LIB


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ------------------------------------------------------------------- pointwise -------

def pressure(U, gamma=1.4, B=0.0) -> float:
    U = np.ascontiguousarray(U, dtype=np.float64)
    return lib().orc_pressure(_dp(U), gamma, B)


def flux_x(U, gamma=1.4, B=0.0) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64)
    F = np.zeros(5)
    lib().orc_flux_x(_dp(U), gamma, B, _dp(F))
    return F


def roe_matrices(UL, UR, gamma=1.4, B=0.0):
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UR = np.ascontiguousarray(UR, dtype=np.float64)
    R = np.zeros(25)
    L = np.zeros(25)
    lib().orc_roe_matrices(_dp(UL), _dp(UR), gamma, B, _dp(R), _dp(L))
    return R.reshape(5, 5), L.reshape(5, 5)


def weno5_minus(a, b, c, d, e) -> float:
    return lib().orc_weno5_minus(float(a), float(b), float(c), float(d), float(e))


def face_flux(d: int, st, gamma=1.4, B=0.0):
    st = np.ascontiguousarray(st, dtype=np.float64).reshape(30)
    F = np.zeros(5)
    n = lib().orc_face_flux(d, _dp(st), gamma, B, _dp(F))
    return F, n


SCHEMES = {"roe_weno5": 0, "roe_teno5": 1, "llf_weno5": 2, "hllc_wao53": 3}


def teno5_minus(a, b, c, d, e) -> float:
    return lib().orc_teno5_minus(float(a), float(b), float(c), float(d), float(e))


def wao53_minus(a, b, c, d, e) -> float:
    return lib().orc_wao53_minus(float(a), float(b), float(c), float(d), float(e))


def beta_quartic(a, b, c, d, e) -> float:
    return lib().orc_beta_quartic(float(a), float(b), float(c), float(d), float(e))


def hllc_flux_x(UL, UR, gamma=1.4, B=0.0) -> np.ndarray:
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UR = np.ascontiguousarray(UR, dtype=np.float64)
    F = np.zeros(5)
    lib().orc_hllc_flux_x(_dp(UL), _dp(UR), gamma, B, _dp(F))
    return F


def face_flux_scheme(scheme: int, d: int, st, gamma=1.4, B=0.0):
    st = np.ascontiguousarray(st, dtype=np.float64).reshape(30)
    F = np.zeros(5)
    n = lib().orc_face_flux_scheme(scheme, d, _dp(st), gamma, B, _dp(F))
    return F, n


def block_rhs_scheme(scheme, u_padded, gamma, B, dx) -> np.ndarray:
    u = np.ascontiguousarray(u_padded, dtype=np.float64)
    assert u.shape == (5, P, P, P)
    out = np.zeros((5, 16, 16, 16))
    lib().orc_block_rhs_scheme(scheme, _dp(u), gamma, B, dx, _dp(out))
    return out


def predict_cell(parent_padded: np.ndarray, octant, i, j, k) -> float:
    a = np.ascontiguousarray(parent_padded, dtype=np.float64)
    assert a.shape == (P, P, P)
    return lib().orc_predict_cell(_dp(a), int(octant[0]), int(octant[1]), int(octant[2]), i, j, k)


def average8(c) -> float:
    c = np.ascontiguousarray(c, dtype=np.float64).reshape(8)
    return lib().orc_average8(_dp(c))


def ssprk3_stage(stage, u0, us, L, dt) -> float:
    return lib().orc_ssprk3_stage(stage, u0, us, L, dt)


def exact_riemann(left, right, gamma, s) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.float64)
    out = np.zeros((len(s), 3))
    rc = lib().orc_exact_riemann(*left, *right, gamma, _dp(s), len(s), _dp(out))
    if rc != 0:
        raise RuntimeError("exact Riemann solver did not converge")
    return out


EOS = {"stiffened": 0, "tait": 1}


def tait_pressure(rho, gamma, B, A, rho0) -> float:
    return lib().orc_tait_pressure(rho, gamma, B, A, rho0)


def tait_sound_speed(rho, gamma, B, rho0) -> float:
    return lib().orc_tait_sound_speed(rho, gamma, B, rho0)


def tait_flux_x(U, gamma, B, A, rho0) -> np.ndarray:
    u = np.ascontiguousarray(U, dtype=np.float64)
    F = np.zeros(5)
    lib().orc_tait_flux_x(_dp(u), gamma, B, A, rho0, _dp(F))
    return F


def tait_roe_matrices(UL, UR, gamma, B, A, rho0):
    a, b = np.ascontiguousarray(UL, dtype=np.float64), np.ascontiguousarray(UR, dtype=np.float64)
    R, L = np.zeros(16), np.zeros(16)
    lib().orc_tait_roe_matrices(_dp(a), _dp(b), gamma, B, A, rho0, _dp(R), _dp(L))
    return R.reshape(4, 4), L.reshape(4, 4)


def tait_face_flux(d: int, st, gamma, B, A, rho0):
    s = np.ascontiguousarray(st, dtype=np.float64).reshape(30)
    F = np.zeros(5)
    n = lib().orc_tait_face_flux(d, _dp(s), gamma, B, A, rho0, _dp(F))
    return F, n


def tait_exact_riemann(left, right, gamma, B, A, rho0, s) -> np.ndarray:
    """(rho, u) of the exact barotropic Riemann solution at x/t = s; left/right = (rho, u)."""
    s = np.ascontiguousarray(s, dtype=np.float64)
    out = np.zeros((len(s), 2))
    rc = lib().orc_tait_exact_riemann(left[0], left[1], right[0], right[1], gamma, B, A, rho0,
                                      _dp(s), len(s), _dp(out))
    if rc != 0:
        raise ValueError("vacuum")
    return out


def visc_face_flux(d: int, st, mu: float, dx: float, energy: bool = True) -> np.ndarray:
    """Viscous flux through a face normal to axis d; st[2][5][5] = (side, cell, q) with
    cell 0 the one sharing the face and 1..4 its tangential neighbours (-1/+1 along the
    lower other axis, then along the higher one)."""
    s = np.ascontiguousarray(st, dtype=np.float64).reshape(50)
    F = np.zeros(5)
    lib().orc_visc_face_flux(d, _dp(s), mu, 1 if energy else 0, dx, _dp(F))
    return F


def visc_dt(cfl: float, dx: float, mu: float, rinv_max: float) -> float:
    return lib().orc_visc_dt(cfl, dx, mu, rinv_max)


def rti_growth_rate(k: float, rho_h: float, rho_l: float, mu: float, g: float) -> float:
    """Root n of eq:SinglePhaseGrowth (equal dynamic viscosities, no surface tension)."""
    n = lib().orc_rti_growth_rate(k, rho_h, rho_l, mu, g)
    if n < 0:
        raise ValueError("no growing mode")
    return n


def lts_lowest_ending(lmax: int, r: int) -> int:
    """Lowest level that completes a step of its own at micro step r (algo:ComputeLoop)."""
    return lib().orc_lts_lowest_ending(lmax, r)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def morton_encode(shadow, level, bx, by, bz) -> int:
    return int(lib().orc_morton_encode(shadow, level, bx, by, bz))


def morton_neighbor(mid: int, d: int, direction: int):
    w = C.c_int32(0)
    n = lib().orc_morton_neighbor(C.c_uint64(mid), d, direction, C.byref(w))
    return int(n), bool(w.value)


def morton_level(mid: int, shadow: int) -> int:
    return int(lib().orc_morton_level(C.c_uint64(mid), shadow))


# ------------------------------------------------------------- learned proposer -------

def mlp_nparams() -> int:
    return lib().orc_mlp_nparams()


def bf16_round(x: float) -> float:
    return lib().orc_bf16_round(float(x))


def mlp_forward(params, X, bf16=True) -> np.ndarray:
    P_ = np.ascontiguousarray(params, dtype=np.float64)
    X_ = np.ascontiguousarray(X, dtype=np.float64)
    n = X_.shape[0]
    out = np.zeros((n, 3))
    lib().orc_mlp_forward(_dp(P_), _dp(X_), n, 1 if bf16 else 0, _dp(out))
    return out


def mlp_loss_grad(params, X, labels, class_w=(1.0, 1.0, 1.0), bf16=True):
    P_ = np.ascontiguousarray(params, dtype=np.float64)
    X_ = np.ascontiguousarray(X, dtype=np.float64)
    y = np.ascontiguousarray(labels, dtype=np.int32)
    w = np.ascontiguousarray(class_w, dtype=np.float64)
    g = np.zeros_like(P_)
    loss = lib().orc_mlp_loss_grad(_dp(P_), _dp(X_), y.ctypes.data_as(C.POINTER(C.c_int32)), _dp(w),
                                   X_.shape[0], 1 if bf16 else 0, _dp(g))
    return loss, g


def features(u_padded, gamma, B, s_rho, s_p, eps_l) -> np.ndarray:
    u = np.ascontiguousarray(u_padded, dtype=np.float64)
    assert u.shape == (5, P, P, P)
    out = np.zeros(192)
    lib().orc_features(_dp(u), gamma, B, s_rho, s_p, eps_l, _dp(out))
    return out


def block_rhs(u_padded, gamma, B, dx) -> np.ndarray:
    """-div F of one padded block [5,24,24,24] -> [5,16,16,16] (no jump correction)."""
    u = np.ascontiguousarray(u_padded, dtype=np.float64)
    assert u.shape == (5, P, P, P)
    out = np.zeros((5, 16, 16, 16))
    lib().orc_block_rhs(_dp(u), gamma, B, dx, _dp(out))
    return out


def block_detail(u_padded, parent_padded, octant, s_rho, s_E) -> float:
    u = np.ascontiguousarray(u_padded, dtype=np.float64)
    pu = np.ascontiguousarray(parent_padded, dtype=np.float64)
    assert u.shape == (5, P, P, P) and pu.shape == (5, P, P, P)
    return lib().orc_block_detail(_dp(u), _dp(pu), int(octant[0]), int(octant[1]), int(octant[2]),
                                  s_rho, s_E)


# ------------------------------------------------------------------ simulation -------

class Sim:
    """One oracle MR simulation of a workloads.Problem."""

    def __init__(self, problem, adapt=None):
        self.problem = problem
        p = _Params()
        p.gamma, p.B, p.cfl, p.eps = problem.gamma, problem.B, problem.cfl, problem.eps
        p.scale_rho, p.scale_E, p.dx0 = problem.scale_rho, problem.scale_E, problem.dx0
        p.lmax = problem.lmax
        for a in range(3):
            p.n0[a] = problem.n0[a]
            p.bc[a] = problem.bc[a]
        p.adapt = problem.adapt if adapt is None else int(adapt)
        p.scheme = SCHEMES[getattr(problem, "scheme", "roe_weno5")]
        for a, gv in enumerate(getattr(problem, "gravity", (0.0, 0.0, 0.0))):
            p.gravity[a] = gv
        p.eos = EOS[getattr(problem, "eos", "stiffened")]
        p.tait_A = getattr(problem, "tait_A", 1.0)
        p.tait_rho0 = getattr(problem, "tait_rho0", 1.0)
        p.mu = getattr(problem, "mu", 0.0)
        fixed = problem.bc_fixed_states() if hasattr(problem, "bc_fixed_states") else None
        if fixed is not None:
            self._fixed = np.ascontiguousarray(fixed, dtype=np.float64)   # copied by create
            p.bc_fixed = _dp(self._fixed)
        self._p = p
        self.h = lib().orc_sim_create(C.byref(p))
        self._cb = None

    def close(self):
        if self.h:
            lib().orc_sim_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, ic=None):
        """algo:Init with the problem's initial condition (or a custom ic(level,bx,by,bz))."""
        gen = ic if ic is not None else self.problem.primitives

        def cb(user, level, bx, by, bz, prim):
            arr = np.ctypeslib.as_array(prim, shape=(5 * N * N * N,))
            arr[:] = np.asarray(gen(level, bx, by, bz), dtype=np.float64).reshape(-1)

        self._cb = IC_FN(cb)
        rc = lib().orc_sim_init(self.h, self._cb, None)
        if rc != 0:
            raise RuntimeError(f"oracle init failed ({rc})")
        return self

    def step(self) -> float:
        dt = C.c_double(0.0)
        rc = lib().orc_sim_step(self.h, C.byref(dt))
        if rc != 0:
            raise RuntimeError(f"oracle step failed ({rc}): non-physical state")
        return dt.value

    def step_dt(self, dt: float):
        """One global step with a given dt."""
        if lib().orc_sim_step_dt(self.h, dt) != 0:
            raise RuntimeError("oracle step failed: non-physical state")

    def step_lts_dt(self, dt: float):
        """One LTS macro step with a given level-lmax step dt."""
        rc = lib().orc_sim_step_lts_dt(self.h, dt)
        if rc == -1:
            raise ValueError("local time stepping with viscosity is not supported")
        if rc != 0:
            raise RuntimeError("oracle LTS step failed: non-physical state")

    def step_lts(self) -> float:
        """One macro step of local time stepping (eq:LtsTimestep): 2^lmax micro steps of
        the returned dt (the eq:Cfl step of level lmax), level l stepping 2^(lmax-l) dt."""
        dt = C.c_double(0.0)
        rc = lib().orc_sim_step_lts(self.h, C.byref(dt))
        if rc == -1:
            raise ValueError("local time stepping with viscosity is not supported")
        if rc != 0:
            raise RuntimeError(f"oracle LTS step failed ({rc}): non-physical state")
        return dt.value

    def lts_steps(self) -> np.ndarray:
        """Own steps completed per level under local time stepping."""
        out = np.zeros(MAX_LEVELS, dtype=np.int64)
        lib().orc_sim_lts_steps(self.h, out.ctypes.data_as(C.POINTER(C.c_int64)))
        return out

    def blocks(self) -> np.ndarray:
        n = lib().orc_sim_nblocks(self.h)
        info = np.zeros((n, 8), dtype=np.int64)
        lib().orc_sim_blocks(self.h, info.ctypes.data_as(C.POINTER(C.c_int64)))
        return info

    def block_index(self):
        """dict (level, bx, by, bz) -> block index."""
        return {tuple(int(v) for v in r[:4]): n for n, r in enumerate(self.blocks())}

    def get_block(self, idx: int) -> np.ndarray:
        out = np.zeros((5, P, P, P))
        lib().orc_sim_get_block(self.h, idx, _dp(out))
        return out

    def set_block(self, idx: int, data: np.ndarray):
        a = np.ascontiguousarray(data, dtype=np.float64)
        assert a.shape == (5, P, P, P)
        lib().orc_sim_set_block(self.h, idx, _dp(a))

    def refine(self, level, bx, by, bz):
        if lib().orc_sim_refine(self.h, level, bx, by, bz) != 0:
            raise ValueError("cannot refine")

    def coarsen(self, level, bx, by, bz):
        if lib().orc_sim_coarsen(self.h, level, bx, by, bz) != 0:
            raise ValueError("cannot coarsen")

    def project(self):
        lib().orc_sim_project(self.h)

    def fill_halos(self):
        lib().orc_sim_fill_halos(self.h)

    def rhs(self) -> np.ndarray:
        nleaf = int((self.blocks()[:, 4] == 1).sum())
        out = np.zeros((nleaf, 5, N, N, N))
        lib().orc_sim_rhs(self.h, _dp(out))
        return out

    def details(self):
        n = lib().orc_sim_nblocks(self.h)
        det = np.zeros(n)
        fl = np.zeros(n, dtype=np.int8)
        lib().orc_sim_details(self.h, _dp(det), fl.ctypes.data_as(C.POINTER(C.c_int8)))
        return det, fl

    def dt(self) -> float:
        return lib().orc_sim_dt(self.h)

    def totals(self) -> np.ndarray:
        t = np.zeros(5)
        lib().orc_sim_totals(self.h, _dp(t))
        return t

    @property
    def time(self) -> float:
        return lib().orc_sim_time(self.h)

    @property
    def llf_fraction(self) -> float:
        return lib().orc_sim_llf_fraction(self.h)

    def leaf_states(self):
        """dict (level,bx,by,bz) -> interior state [5][16][16][16] of every leaf."""
        out = {}
        for n, r in enumerate(self.blocks()):
            if r[4] == 1:
                out[tuple(int(v) for v in r[:4])] = self.get_block(n)[:, H:H + N, H:H + N, H:H + N]
        return out
