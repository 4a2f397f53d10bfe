"""CPU checks of the C ABI library: it loads, exports every symbol the public header
declares, validates arguments without touching a device, and its host Morton logic
matches the paper's worked example and brute force."""
import itertools
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2012_04385_amd import mrfv
    if not os.path.exists(mrfv.LIB_PATH):
        from paper_2012_04385_amd import build
        build.build()
    return mrfv


def test_header_symbols_exported():
    mrfv = _lib()
    hdr = open(os.path.join(ROOT, "include", "mrfv.h")).read()
    declared = set(re.findall(r"^\s*(?:int|int32_t|int64_t|uint64_t|const char \*)\s*(mrfv_\w+)\s*\(", hdr, re.M))
    assert len(declared) >= 20
    L = mrfv.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(mrfv.exported_symbols())


def test_create_rejects_bad_config_without_device():
    import ctypes as C
    mrfv = _lib()
    inst = (mrfv.Instance * 1)()
    inst[0].gamma, inst[0].cfl, inst[0].dx0 = 1.4, 0.5, 1 / 32
    inst[0].scale_rho = inst[0].scale_E = 1.0
    for a in range(3):
        inst[0].n0[a] = 1
    h = C.c_void_p()
    bad = [mrfv.Config(7, 1, 10, 0), mrfv.Config(0, 0, 10, 0), mrfv.Config(0, 1, 0, 0),
           mrfv.Config(0, 1, 10, 0, 4)]
    for cfg in bad:
        assert mrfv.lib().mrfv_create(C.byref(h), C.byref(cfg), inst, None) == mrfv.EINVAL
    inst[0].gamma = 1.0
    assert mrfv.lib().mrfv_create(C.byref(h), C.byref(mrfv.Config(0, 1, 10, 0)), inst, None) == mrfv.EINVAL
    inst[0].gamma = 1.4
    ok_cfg = mrfv.Config(1, 1, 10, 0)
    # viscosity, boundary kinds and fixed-value states are validated before any device call
    inst[0].mu = -1.0
    assert mrfv.lib().mrfv_create(C.byref(h), C.byref(ok_cfg), inst, None) == mrfv.EINVAL
    inst[0].mu = 0.0
    inst[0].bc[1] = 4
    assert mrfv.lib().mrfv_create(C.byref(h), C.byref(ok_cfg), inst, None) == mrfv.EINVAL
    inst[0].bc[1] = 3   # fixed values without states
    assert mrfv.lib().mrfv_create(C.byref(h), C.byref(ok_cfg), inst, None) == mrfv.EINVAL
    import numpy as np
    states = np.ones((6, 1, 4, 5))
    states[3, 0, 2, 0] = 0.0   # rho = 0 in one layer of the y+ side
    inst[0].bc_fixed = states.ctypes.data_as(C.POINTER(C.c_double))
    assert mrfv.lib().mrfv_create(C.byref(h), C.byref(ok_cfg), inst, None) == mrfv.EINVAL
    states[3, 0, 2, 0] = 1.0
    states[2, 0, 0, 4] = -2.0  # negative pressure on the y- side
    assert mrfv.lib().mrfv_create(C.byref(h), C.byref(ok_cfg), inst, None) == mrfv.EINVAL
    states[2, 0, 0, 4] = 1.0   # all valid now: only the missing device stops the context
    assert mrfv.lib().mrfv_create(C.byref(h), C.byref(ok_cfg), inst, None) not in (mrfv.OK, mrfv.EINVAL)
    assert mrfv.lib().mrfv_destroy(None) == mrfv.EINVAL
    assert mrfv.lib().mrfv_step(None, None, None, None, None) == mrfv.EINVAL


def test_morton_worked_example():
    mrfv = _lib()
    # +z neighbour of 001 111 is 101 011 (headbit prepended; one group above level 0)
    mid = int("1001111", 2)
    n, w = mrfv.morton_neighbor(mid, 1, 2, +1)
    assert n == int("1101011", 2) and not w
    assert mrfv.morton_encode(1, 0, 0, 0, 1) == int("1100", 2)
    assert mrfv.morton_encode(1, 1, 3, 1, 2) >> 3 == mrfv.morton_encode(1, 0, 1, 0, 1)


@pytest.mark.parametrize("shadow", [0, 1, 2])
def test_morton_brute_force(shadow):
    mrfv = _lib()
    for level in range(3):
        n = 1 << (shadow + level)
        for bx, by, bz in itertools.product(range(n), repeat=3):
            mid = mrfv.morton_encode(shadow, level, bx, by, bz)
            c = [bx, by, bz]
            for d in range(3):
                for s in (1, -1):
                    got, w = mrfv.morton_neighbor(mid, shadow, d, s)
                    cc = list(c)
                    cc[d] += s
                    out = not (0 <= cc[d] < n)
                    cc[d] %= n
                    assert got == mrfv.morton_encode(shadow, level, *cc)
                    assert w == out
