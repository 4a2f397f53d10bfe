"""ctypes binding of libmrfv.so (the C ABI declared in include/mrfv.h).

Argument marshalling only: every step of the method runs in the library's HIP kernels
and host code.  PyTorch supplies device memory (tensor storage) and the stream.  There is
no fallback: if the library is missing or no HIP device is present, construction fails.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Callable, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrfv.so")

OK, EINVAL, EHIP, ENOMEM, ESTATE, ENONPHYS = 0, -1, -2, -3, -4, -5
F32, F64 = 0, 1
NI, HW, NP = 16, 4, 24


class MrfvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mrfv error {code}: {msg}")
        self.code = code


class Instance(C.Structure):
    _fields_ = [("gamma", C.c_double), ("B", C.c_double), ("cfl", C.c_double),
                ("eps", C.c_double), ("scale_rho", C.c_double), ("scale_E", C.c_double),
                ("dx0", C.c_double), ("lmax", C.c_int32), ("n0", C.c_int32 * 3),
                ("bc", C.c_int32 * 3), ("adapt", C.c_int32), ("gravity", C.c_double * 3),
                ("eos", C.c_int32), ("tait_A", C.c_double), ("tait_rho0", C.c_double),
                ("mu", C.c_double), ("bc_fixed", C.POINTER(C.c_double))]


class Config(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("n_instances", C.c_int32),
                ("slot_capacity", C.c_int32), ("batched", C.c_int32), ("scheme", C.c_int32)]


# flux kernels (mrfv_scheme)
SCHEMES = {"roe_weno5": 0, "roe_teno5": 1, "llf_weno5": 2, "hllc_wao53": 3}
EOS = {"stiffened": 0, "tait": 1}


IC_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                    C.POINTER(C.c_double))

_LIB = None


def lib():
    """Load libmrfv.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    pvp = C.POINTER(C.c_void_p)
    sig = {
        "mrfv_create": ([pvp, C.POINTER(Config), C.POINTER(Instance), vp], C.c_int),
        "mrfv_destroy": ([vp], C.c_int),
        "mrfv_last_error": ([vp], C.c_char_p),
        "mrfv_state_bytes": ([vp], i64),
        "mrfv_interior_bytes": ([vp], i64),
        "mrfv_init_blocks": ([vp, IC_FN, vp, vp], C.c_int),
        "mrfv_fill_halos": ([vp, vp], C.c_int),
        "mrfv_rhs_stage": ([vp, vp, vp], C.c_int),
        "mrfv_rk_update": ([vp, i32, vp, vp, vp, vp], C.c_int),
        "mrfv_mr_project": ([vp, vp], C.c_int),
        "mrfv_mr_predict": ([vp, vp, C.POINTER(i32), i32], C.c_int),
        "mrfv_mr_flag": ([vp, vp, vp, vp], C.c_int),
        "mrfv_set_detail_band": ([vp, d], C.c_int),
        "mrfv_cfl_dt": ([vp, vp, vp], C.c_int),
        "mrfv_totals": ([vp, vp, vp], C.c_int),
        "mrfv_totals_noalloc": ([vp, vp, vp], C.c_int),
        "mrfv_commit_flags": ([vp, C.POINTER(C.c_int8), C.POINTER(i32), C.POINTER(i32)], C.c_int),
        "mrfv_step": ([vp, vp, vp, vp, vp], C.c_int),
        "mrfv_run": ([vp, vp, vp, vp, vp, i32, C.POINTER(i64)], C.c_int),
        "mrfv_step_lts": ([vp, vp, vp, vp, vp, C.POINTER(i64)], C.c_int),
        "mrfv_check": ([vp], C.c_int),
        "mrfv_get_blocks": ([vp, C.POINTER(i64), C.POINTER(i32)], C.c_int),
        "mrfv_stats": ([vp, C.POINTER(i64)], C.c_int),
        "mrfv_refine_block": ([vp, vp, i32, i32, i32, i32, i32], C.c_int),
        "mrfv_coarsen_block": ([vp, i32, i32, i32, i32, i32], C.c_int),
        "mrfv_enable_kernel_timing": ([vp, i32], C.c_int),
        "mrfv_kernel_time": ([vp, C.POINTER(i64), C.POINTER(d), C.POINTER(i64)], C.c_int),
        "mrfv_morton_encode": ([i32, i32, i32, i32, i32], C.c_uint64),
        "mrfv_morton_neighbor": ([C.c_uint64, i32, i32, i32, C.POINTER(i32)], C.c_uint64),
        "mrfv_mlp_create": ([pvp, i32, vp], C.c_int),
        "mrfv_mlp_destroy": ([vp], C.c_int),
        "mrfv_mlp_last_error": ([vp], C.c_char_p),
        "mrfv_mlp_nparams": ([], i32),
        "mrfv_mlp_set_params": ([vp, C.POINTER(C.c_float)], C.c_int),
        "mrfv_mlp_get_params": ([vp, C.POINTER(C.c_float)], C.c_int),
        "mrfv_mlp_forward": ([vp, vp, i32, vp], C.c_int),
        "mrfv_mlp_loss_grad": ([vp, vp, C.POINTER(i32), C.POINTER(C.c_float), i32,
                                C.POINTER(C.c_float), C.POINTER(C.c_float)], C.c_int),
        "mrfv_mlp_adam_step": ([vp, C.c_float, C.c_float, C.c_float, C.c_float], C.c_int),
        "mrfv_features": ([vp, vp, vp, C.POINTER(i32), C.POINTER(i32)], C.c_int),
        "mrfv_set_proposer": ([vp, vp, i32], C.c_int),
        "mrfv_proposer_stats": ([vp, C.POINTER(i64), C.POINTER(d)], C.c_int),
        "mrfv_last_flags": ([vp, C.POINTER(C.c_int8)], C.c_int),
        "mrfv_step_timing": ([vp, C.POINTER(d)], C.c_int),
        "mrfv_rhs_variant": ([vp, i32, C.POINTER(i32), C.POINTER(i32)], C.c_int),
        "mrfv_fused_stage": ([vp, i32, vp, vp, vp, vp, i32], C.c_int),
        "mrfv_autotune": ([vp, vp, vp, vp, i32, C.POINTER(C.c_float), C.POINTER(i32)], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _LIB = L
    return L


def exported_symbols():
    return ["mrfv_create", "mrfv_destroy", "mrfv_last_error", "mrfv_state_bytes",
            "mrfv_interior_bytes", "mrfv_init_blocks", "mrfv_fill_halos", "mrfv_rhs_stage",
            "mrfv_rk_update", "mrfv_mr_project", "mrfv_mr_predict", "mrfv_mr_flag",
            "mrfv_cfl_dt", "mrfv_totals", "mrfv_commit_flags", "mrfv_step", "mrfv_check",
            "mrfv_get_blocks", "mrfv_stats", "mrfv_refine_block", "mrfv_coarsen_block",
            "mrfv_enable_kernel_timing", "mrfv_kernel_time", "mrfv_morton_encode",
            "mrfv_morton_neighbor", "mrfv_mlp_create", "mrfv_mlp_destroy",
            "mrfv_mlp_last_error", "mrfv_mlp_nparams", "mrfv_mlp_set_params",
            "mrfv_mlp_get_params", "mrfv_mlp_forward", "mrfv_mlp_loss_grad",
            "mrfv_mlp_adam_step", "mrfv_features", "mrfv_set_proposer", "mrfv_proposer_stats",
            "mrfv_last_flags", "mrfv_step_timing", "mrfv_rhs_variant", "mrfv_autotune",
            "mrfv_fused_stage", "mrfv_run", "mrfv_set_detail_band", "mrfv_totals_noalloc",
            "mrfv_step_lts"]


def morton_encode(shadow, level, bx, by, bz) -> int:
    return int(lib().mrfv_morton_encode(shadow, level, bx, by, bz))


def morton_neighbor(mid: int, shadow: int, d: int, direction: int):
    w = C.c_int32(0)
    n = lib().mrfv_morton_neighbor(C.c_uint64(mid), shadow, d, direction, C.byref(w))
    return int(n), bool(w.value)


def _instance(pb, keep: list) -> Instance:
    """The ABI struct of a problem; arrays it points to are appended to `keep` (they must
    outlive mrfv_create)."""
    inst = Instance()
    inst.gamma, inst.B, inst.cfl, inst.eps = pb.gamma, pb.B, pb.cfl, pb.eps
    inst.scale_rho, inst.scale_E, inst.dx0 = pb.scale_rho, pb.scale_E, pb.dx0
    inst.lmax = pb.lmax
    for a in range(3):
        inst.n0[a] = pb.n0[a]
        inst.bc[a] = pb.bc[a]
    inst.adapt = pb.adapt
    for a, gv in enumerate(getattr(pb, "gravity", (0.0, 0.0, 0.0))):
        inst.gravity[a] = gv
    inst.eos = EOS[getattr(pb, "eos", "stiffened")]
    inst.tait_A = getattr(pb, "tait_A", 1.0)
    inst.tait_rho0 = getattr(pb, "tait_rho0", 1.0)
    inst.mu = getattr(pb, "mu", 0.0)
    fixed = pb.bc_fixed_states() if hasattr(pb, "bc_fixed_states") else None
    if fixed is not None:
        fixed = np.ascontiguousarray(fixed, dtype=np.float64)
        keep.append(fixed)
        inst.bc_fixed = fixed.ctypes.data_as(C.POINTER(C.c_double))
    return inst


def slot_capacity_for(problems) -> int:
    """Upper bound of blocks: every instance fully refined."""
    tot = 0
    for pb in problems:
        n = pb.n0[0] * pb.n0[1] * pb.n0[2]
        tot += sum(n * 8 ** l for l in range(pb.lmax + 1))
    return tot


class Solver:
    """One library context plus caller-owned device buffers (torch tensors)."""

    def __init__(self, problems: Sequence, dtype: str = "f32", batched=True,
                 capacity: Optional[int] = None, device: str = "cuda:0", adapt=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the MR solver runs on the GPU only")
        self.torch = torch
        self.problems = list(problems)
        self.dtype = F64 if dtype in ("f64", "float64", "double") else F32
        self.tdtype = torch.float64 if self.dtype == F64 else torch.float32
        self.device = torch.device(device)
        cap = capacity or slot_capacity_for(self.problems)
        n = len(self.problems)
        arr = (Instance * n)()
        keep = []
        for i, pb in enumerate(self.problems):
            arr[i] = _instance(pb, keep)
            if adapt is not None:
                arr[i].adapt = int(adapt)
        schemes = {getattr(pb, "scheme", "roe_weno5") for pb in self.problems}
        if len(schemes) != 1:
            raise ValueError("all problems of one context use the same flux kernel")
        self.scheme = schemes.pop()
        cfg = Config(self.dtype, n, cap, int(batched), SCHEMES[self.scheme])
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = lib().mrfv_create(C.byref(h), C.byref(cfg), arr, C.c_void_p(self.stream.cuda_stream))
        if rc != OK:
            raise MrfvError(rc, "mrfv_create failed (bad configuration or out of memory)")
        self.h = h
        self.capacity = cap
        self.n_inst = n
        es = 8 if self.dtype == F64 else 4
        assert lib().mrfv_state_bytes(h) == cap * 5 * NP ** 3 * es
        self.U = torch.zeros((cap, 5, NP, NP, NP), dtype=self.tdtype, device=self.device)
        self.U0 = torch.zeros((cap, 5, NI, NI, NI), dtype=self.tdtype, device=self.device)
        self.L = torch.zeros((cap, 5, NI, NI, NI), dtype=self.tdtype, device=self.device)
        self.dt = torch.zeros(n, dtype=torch.float64, device=self.device)
        self.flags = torch.zeros(cap, dtype=torch.int8, device=self.device)
        self.det = torch.zeros(cap, dtype=torch.float64, device=self.device)
        self.tot = torch.zeros((n, 5), dtype=torch.float64, device=self.device)
        self._cb = None
        self.time = np.zeros(n)

    # -------------------------------------------------------------------- plumbing
    def _chk(self, rc: int):
        if rc != OK:
            msg = lib().mrfv_last_error(self.h)
            raise MrfvError(rc, msg.decode() if msg else "")

    @staticmethod
    def _p(t):
        return C.c_void_p(t.data_ptr())

    def close(self):
        if getattr(self, "h", None):
            lib().mrfv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ the ABI
    def init(self, ic: Optional[Callable] = None):
        """algo:Init; ic(inst, level, bx, by, bz) -> prim[5,16,16,16] (defaults to the
        problems' own generators)."""
        def default(inst, level, bx, by, bz):
            return self.problems[inst].primitives(level, bx, by, bz)
        gen = ic or default

        def cb(user, inst, level, bx, by, bz, prim):
            out = np.ctypeslib.as_array(prim, shape=(5 * NI ** 3,))
            out[:] = np.asarray(gen(inst, level, bx, by, bz), dtype=np.float64).reshape(-1)

        self._cb = IC_FN(cb)
        self._chk(lib().mrfv_init_blocks(self.h, self._cb, None, self._p(self.U)))
        return self

    def fill_halos(self):
        self._chk(lib().mrfv_fill_halos(self.h, self._p(self.U)))

    def rhs_stage(self):
        self._chk(lib().mrfv_rhs_stage(self.h, self._p(self.U), self._p(self.L)))
        return self.L

    def rk_update(self, stage: int):
        self._chk(lib().mrfv_rk_update(self.h, stage, self._p(self.dt), self._p(self.U),
                                       self._p(self.U0), self._p(self.L)))

    def mr_project(self):
        self._chk(lib().mrfv_mr_project(self.h, self._p(self.U)))

    def mr_predict(self, slots):
        a = np.ascontiguousarray(slots, dtype=np.int32)
        self._chk(lib().mrfv_mr_predict(self.h, self._p(self.U),
                                        a.ctypes.data_as(C.POINTER(C.c_int32)), len(a)))

    def mr_flag(self):
        self._chk(lib().mrfv_mr_flag(self.h, self._p(self.U), self._p(self.flags), self._p(self.det)))
        return self.flags, self.det

    def set_detail_band(self, band: float):
        self._chk(lib().mrfv_set_detail_band(self.h, float(band)))

    def cfl_dt(self):
        self._chk(lib().mrfv_cfl_dt(self.h, self._p(self.U), self._p(self.dt)))
        return self.dt

    def totals(self):
        self._chk(lib().mrfv_totals(self.h, self._p(self.U), self._p(self.tot)))
        return self.tot

    def commit_flags(self, flags_host: np.ndarray):
        f = np.ascontiguousarray(flags_host, dtype=np.int8)
        out = np.zeros(self.capacity, dtype=np.int32)
        n = C.c_int32(0)
        self._chk(lib().mrfv_commit_flags(self.h, f.ctypes.data_as(C.POINTER(C.c_int8)),
                                          out.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(n)))
        return out[: n.value]

    def step(self) -> np.ndarray:
        self._chk(lib().mrfv_step(self.h, self._p(self.U), self._p(self.U0), self._p(self.L),
                                  self._p(self.dt)))
        return self.dt

    def run(self, n: int) -> int:
        """n steps natively (mrfv_run: the same result as n calls of step, with the next
        step queued before the host reads the current step's flags).  Returns the leaf
        cells of the steps' trees, summed over the steps."""
        cells = C.c_int64(0)
        self._chk(lib().mrfv_run(self.h, self._p(self.U), self._p(self.U0), self._p(self.L),
                                 self._p(self.dt), int(n), C.byref(cells)))
        return int(cells.value)

    def step_lts(self) -> int:
        """One macro step of local time stepping (mrfv_step_lts): 2^lmax micro steps of
        dt (left in self.dt), level l advancing with 2^(lmax-l) dt.  Returns the cell
        updates of the macro step (leaf cells times their own steps)."""
        cells = C.c_int64(0)
        self._chk(lib().mrfv_step_lts(self.h, self._p(self.U), self._p(self.U0), self._p(self.L),
                                      self._p(self.dt), C.byref(cells)))
        return int(cells.value)

    def check(self):
        self._chk(lib().mrfv_check(self.h))

    def refine(self, inst, level, bx, by, bz):
        self._chk(lib().mrfv_refine_block(self.h, self._p(self.U), inst, level, bx, by, bz))

    def coarsen(self, inst, level, bx, by, bz):
        self._chk(lib().mrfv_coarsen_block(self.h, inst, level, bx, by, bz))

    def blocks(self) -> np.ndarray:
        n = C.c_int32(0)
        self._chk(lib().mrfv_get_blocks(self.h, None, C.byref(n)))
        info = np.zeros((n.value, 8), dtype=np.int64)
        self._chk(lib().mrfv_get_blocks(self.h, info.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(n)))
        return info

    def enable_kernel_timing(self, on: bool = True):
        self._chk(lib().mrfv_enable_kernel_timing(self.h, 1 if on else 0))

    def kernel_time(self):
        n, cells = C.c_int64(0), C.c_int64(0)
        ms = C.c_double(0.0)
        self._chk(lib().mrfv_kernel_time(self.h, C.byref(n), C.byref(ms), C.byref(cells)))
        return n.value, ms.value, cells.value

    # ------------------------------------------------------------- conveniences
    def advance(self, steps: int):
        """steps calls of step, accumulating the simulated time; checks the error word."""
        for _ in range(steps):
            self.step()
            self.time += self.dt.cpu().numpy()
        self.check()

    def leaf_states(self, inst: int = 0):
        """dict (level,bx,by,bz) -> float64 interior state [5,16,16,16] of every leaf."""
        self.torch.cuda.synchronize()
        info = self.blocks()
        sel = info[(info[:, 6] == 1) & (info[:, 1] == inst)]
        U = self.U[self.torch.as_tensor(sel[:, 0], device=self.device)]
        U = U[:, :, HW:HW + NI, HW:HW + NI, HW:HW + NI].double().cpu().numpy()
        return {tuple(int(v) for v in r[2:6]): U[k] for k, r in enumerate(sel)}

    def stats(self):
        """(blocks, leaves, leaf cells, finest level) from the host tree."""
        out = (C.c_int64 * 4)()
        self._chk(lib().mrfv_stats(self.h, out))
        return tuple(int(v) for v in out)

    def leaf_cells(self) -> int:
        return self.stats()[2]

    def fused_stage(self, stage: int, Uout, Uin=None, restrict_parents: bool = False):
        """One stage of the batched FP32 path from Uin (default: the state) into Uout;
        restrict_parents: jump-free leaves also restrict their result into their parents."""
        Uin = self.U if Uin is None else Uin
        self._chk(lib().mrfv_fused_stage(self.h, int(stage), self._p(self.dt), self._p(Uin),
                                         self._p(Uout), self._p(self.U0), int(bool(restrict_parents))))

    def rhs_variants(self):
        """[(z-planes per group, threads per workgroup, waves per SIMD aimed at, pointer
        loads)] of the fused kernel's variants; a negative thread count marks a persistent
        grid looping over the leaves, waves 1 the compiler's default register allocation,
        pointer loads 1 the per-lane pointer path for the stencils."""
        n = C.c_int32(0)
        lib().mrfv_rhs_variant(self.h, -1, C.byref(n), None)
        shp = (C.c_int32 * (4 * n.value))()
        lib().mrfv_rhs_variant(self.h, -1, None, shp)
        return [tuple(shp[4 * v + i] for i in range(4)) for v in range(n.value)]

    def set_rhs_variant(self, v: int) -> int:
        rc = lib().mrfv_rhs_variant(self.h, int(v), None, None)
        self._chk(min(rc, 0))
        return rc

    def autotune(self, reps: int = 5):
        """Times every fused-kernel variant on the current state and keeps the fastest;
        returns (choice, [ms per variant])."""
        nv = len(self.rhs_variants())
        ms = (C.c_float * nv)()
        ch = C.c_int32(-1)
        self._chk(lib().mrfv_autotune(self.h, self._p(self.U), self._p(self.U0), self._p(self.dt),
                                      int(reps), ms, C.byref(ch)))
        return ch.value, list(ms)

    def step_timing(self) -> dict:
        """Host clock of the adaptation phase, summed over adaptive steps (ms)."""
        out = (C.c_double * 4)()
        self._chk(lib().mrfv_step_timing(self.h, out))
        return dict(steps=int(out[0]), wait_ms=out[1], commit_ms=out[2], predict_ms=out[3])


# --------------------------------------------------------------------- proposer
N_FEATURES = 192
CLASS_REFINE, CLASS_KEEP, CLASS_COARSEN = 0, 1, 2


def flags_to_classes(flags: np.ndarray) -> np.ndarray:
    """Judge flags (+1 refine, 0 keep, -1 coarsen) -> class labels (0, 1, 2)."""
    f = np.asarray(flags)
    return np.where(f > 0, CLASS_REFINE, np.where(f < 0, CLASS_COARSEN, CLASS_KEEP)).astype(np.int32)


class MLP:
    """The refinement proposer's network on the device (bfloat16 products, FP32 master
    parameters and Adam moments)."""

    def __init__(self, max_rows: int, device: str = "cuda:0"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the proposer network runs on the GPU only")
        self.torch = torch
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self.max_rows = int(max_rows)
        h = C.c_void_p()
        rc = lib().mrfv_mlp_create(C.byref(h), self.max_rows, C.c_void_p(self.stream.cuda_stream))
        if rc != OK:
            raise MrfvError(rc, "mrfv_mlp_create failed")
        self.h = h
        self.nparams = int(lib().mrfv_mlp_nparams())

    def _chk(self, rc: int):
        if rc != OK:
            msg = lib().mrfv_mlp_last_error(self.h)
            raise MrfvError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            lib().mrfv_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p: np.ndarray):
        a = np.ascontiguousarray(p, dtype=np.float32)
        assert a.size == self.nparams
        self._chk(lib().mrfv_mlp_set_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float))))

    def get_params(self) -> np.ndarray:
        a = np.zeros(self.nparams, dtype=np.float32)
        self._chk(lib().mrfv_mlp_get_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float))))
        return a

    def init_params(self, seed: int) -> np.ndarray:
        """He-uniform weights, zero biases (layout W1, b1, W2, b2, W3, b3)."""
        rng = np.random.default_rng(seed)
        parts = []
        for fi, fo in ((192, 64), (64, 64), (64, 3)):
            lim = np.sqrt(6.0 / fi)
            parts += [rng.uniform(-lim, lim, fi * fo), np.zeros(fo)]
        p = np.concatenate(parts).astype(np.float32)
        self.set_params(p)
        return p

    def forward(self, X):
        """X: device float32 [N, 192] -> device float32 logits [N, 3]."""
        X = X.contiguous()
        out = self.torch.empty((X.shape[0], 3), dtype=self.torch.float32, device=self.device)
        self._chk(lib().mrfv_mlp_forward(self.h, C.c_void_p(X.data_ptr()), int(X.shape[0]),
                                         C.c_void_p(out.data_ptr())))
        return out

    def loss_grad(self, X, labels: np.ndarray, class_w, want_grad: bool = True):
        X = X.contiguous()
        y = np.ascontiguousarray(labels, dtype=np.int32)
        cw = np.ascontiguousarray(class_w, dtype=np.float32)
        loss = C.c_float(0.0)
        g = np.zeros(self.nparams, dtype=np.float32) if want_grad else None
        self._chk(lib().mrfv_mlp_loss_grad(
            self.h, C.c_void_p(X.data_ptr()), y.ctypes.data_as(C.POINTER(C.c_int32)),
            cw.ctypes.data_as(C.POINTER(C.c_float)), int(X.shape[0]), C.byref(loss),
            g.ctypes.data_as(C.POINTER(C.c_float)) if want_grad else None))
        return float(loss.value), g

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self._chk(lib().mrfv_mlp_adam_step(self.h, lr, beta1, beta2, eps))

    def train(self, X, labels: np.ndarray, epochs: int, lr: float = 3e-3, batch: int = 4096,
              seed: int = 0, class_w=None):
        """Mini-batch Adam on the device; class weights default to inverse frequencies."""
        torch = self.torch
        y = np.asarray(labels, dtype=np.int32)
        if class_w is None:
            cnt = np.bincount(y, minlength=3).astype(np.float64)
            class_w = np.where(cnt > 0, cnt.sum() / np.maximum(cnt, 1) / 3.0, 0.0)
        rng = np.random.default_rng(seed)
        n = X.shape[0]
        losses = []
        for _ in range(epochs):
            perm = rng.permutation(n)
            for a in range(0, n, batch):
                idx = perm[a:a + batch]
                Xb = X[torch.as_tensor(idx, device=self.device)]
                loss, _ = self.loss_grad(Xb, y[idx], class_w, want_grad=False)
                self.adam_step(lr)
                losses.append(loss)
        return losses


def solver_features(solver: "Solver"):
    """Proposer features of every current leaf: (device float32 [n, 192], slots)."""
    torch = solver.torch
    X = torch.zeros((solver.capacity, N_FEATURES), dtype=torch.float32, device=solver.device)
    slots = np.zeros(solver.capacity, dtype=np.int32)
    n = C.c_int32(0)
    solver._chk(lib().mrfv_features(solver.h, solver._p(solver.U), C.c_void_p(X.data_ptr()),
                                    slots.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(n)))
    return X[: n.value], slots[: n.value]


def set_proposer(solver: "Solver", mlp: Optional[MLP], mode: int):
    solver._chk(lib().mrfv_set_proposer(solver.h, mlp.h if mlp is not None else None, int(mode)))
    solver._proposer = mlp   # keep the network alive while the solver uses it


def last_flags(solver: "Solver") -> np.ndarray:
    """Judged flags (int8 by slot) of the last adaptive step."""
    f = np.zeros(solver.capacity, dtype=np.int8)
    solver._chk(lib().mrfv_last_flags(solver.h, f.ctypes.data_as(C.POINTER(C.c_int8))))
    return f


def collect_training_data(solver: "Solver", steps: int, with_steps: bool = False):
    """Run steps and record, for every step, the features of the leaves at its start and
    the judge's class for each of them at its end: (device X [n, 192], int32 labels), and
    with_steps the step index of every row."""
    torch = solver.torch
    Xs, ys, ks = [], [], []
    for k in range(steps):
        X, slots = solver_features(solver)
        X = X.clone()
        solver.step()
        ys.append(flags_to_classes(last_flags(solver)[slots]))
        Xs.append(X)
        ks.append(np.full(len(slots), k, dtype=np.int64))
    if with_steps:
        return torch.cat(Xs), np.concatenate(ys), np.concatenate(ks)
    return torch.cat(Xs), np.concatenate(ys)


def proposer_stats(solver: "Solver") -> dict:
    out = (C.c_int64 * 14)()
    ms = C.c_double(0.0)
    solver._chk(lib().mrfv_proposer_stats(solver.h, out, C.byref(ms)))
    v = list(out)
    per = {name: dict(tp=v[2 + 3 * c], fp=v[3 + 3 * c], fn=v[4 + 3 * c])
           for c, name in enumerate(("refine", "keep", "coarsen"))}
    return dict(steps=v[0], hits=v[1], staged=v[11], adopted=v[12], net_runs=v[13], build_ms=ms.value,
                **per)
