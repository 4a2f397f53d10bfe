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
                ("bc", C.c_int32 * 3), ("adapt", C.c_int32)]


class Config(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("n_instances", C.c_int32),
                ("slot_capacity", C.c_int32), ("batched", C.c_int32)]


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
        "mrfv_cfl_dt": ([vp, vp, vp], C.c_int),
        "mrfv_totals": ([vp, vp, vp], C.c_int),
        "mrfv_commit_flags": ([vp, C.POINTER(C.c_int8), C.POINTER(i32), C.POINTER(i32)], C.c_int),
        "mrfv_step": ([vp, vp, vp, vp, vp], C.c_int),
        "mrfv_check": ([vp], C.c_int),
        "mrfv_get_blocks": ([vp, C.POINTER(i64), C.POINTER(i32)], C.c_int),
        "mrfv_stats": ([vp, C.POINTER(i64)], C.c_int),
        "mrfv_refine_block": ([vp, vp, i32, i32, i32, i32, i32], C.c_int),
        "mrfv_coarsen_block": ([vp, i32, i32, i32, i32, i32], C.c_int),
        "mrfv_enable_kernel_timing": ([vp, i32], C.c_int),
        "mrfv_kernel_time": ([vp, C.POINTER(i64), C.POINTER(d), C.POINTER(i64)], C.c_int),
        "mrfv_morton_encode": ([i32, i32, i32, i32, i32], C.c_uint64),
        "mrfv_morton_neighbor": ([C.c_uint64, i32, i32, i32, C.POINTER(i32)], C.c_uint64),
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
            "mrfv_morton_neighbor"]


def morton_encode(shadow, level, bx, by, bz) -> int:
    return int(lib().mrfv_morton_encode(shadow, level, bx, by, bz))


def morton_neighbor(mid: int, shadow: int, d: int, direction: int):
    w = C.c_int32(0)
    n = lib().mrfv_morton_neighbor(C.c_uint64(mid), shadow, d, direction, C.byref(w))
    return int(n), bool(w.value)


def _instance(pb) -> Instance:
    inst = Instance()
    inst.gamma, inst.B, inst.cfl, inst.eps = pb.gamma, pb.B, pb.cfl, pb.eps
    inst.scale_rho, inst.scale_E, inst.dx0 = pb.scale_rho, pb.scale_E, pb.dx0
    inst.lmax = pb.lmax
    for a in range(3):
        inst.n0[a] = pb.n0[a]
        inst.bc[a] = pb.bc[a]
    inst.adapt = pb.adapt
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

    def __init__(self, problems: Sequence, dtype: str = "f32", batched: bool = True,
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
        for i, pb in enumerate(self.problems):
            arr[i] = _instance(pb)
            if adapt is not None:
                arr[i].adapt = int(adapt)
        cfg = Config(self.dtype, n, cap, 1 if batched else 0)
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
    def run(self, steps: int):
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
