"""The C-ABI library loads and exports every entry point include/ugks.h
declares; argument validation runs before any device call (CPU only)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ugks.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    from paper_2604_09984_amd import ugks
    L = ugks.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(ugks.exported_symbols())


def _problem(ugks, case, **over):
    vx = np.ascontiguousarray(case.vx, dtype=np.float64)
    vy = np.ascontiguousarray(case.vy, dtype=np.float64)
    bint, bdbl, nodes = case.block_ints(), case.block_dbls(), case.node_array()
    p = ugks._Problem()
    p.dim = over.get("dim", case.dim)
    p.pr, p.omega, p.mu_ref, p.rt_ref = case.pr, case.omega, case.mu_ref, case.rt_ref
    p.nvx, p.nvy = over.get("nvx", case.nvx), case.nvy
    p.vx, p.vy = ugks._dp(vx), ugks._dp(vy)
    for m in range(4):
        p.vrange[m] = case.vrange[m]
    p.cfl_s, p.cfl_p = case.cfl_s, case.cfl_p
    p.nblock = len(case.blocks)
    p.bint = bint.ctypes.data_as(C.POINTER(C.c_int32))
    p.bdbl = ugks._dp(bdbl)
    p.nodes = ugks._dp(nodes)
    p.prec = over.get("prec", 0)
    return p, (vx, vy, bint, bdbl, nodes)


@pytest.mark.parametrize("bad,code", [({"dim": 3}, -1), ({"prec": 7}, -1), ({"nvx": 1}, -2)])
def test_create_rejects_bad_arguments_without_device(bad, code):
    from paper_2604_09984_amd import ugks, workloads as wl
    p, keep = _problem(ugks, wl.sod_1d(20, 9), **bad)
    ctx = C.c_void_p()
    rc = ugks.lib().ugks_create(C.byref(p), 0, C.byref(ctx))
    assert rc == code
    assert ugks.lib().ugks_last_error().decode() != ""
    assert not ctx.value


def test_null_context_is_an_argument_error():
    from paper_2604_09984_amd import ugks
    L = ugks.lib()
    assert L.ugks_flux(None, 1.0, None, None, None, None, None, None, None, None, None) == -1
    assert L.ugks_destroy(None) == 0


def test_workspace_size_without_device():
    """ugks_workspace_size is host arithmetic on the problem: the scratch
    holds at least the two [ncell][nv] divergence / residual arrays and the
    adjoint workspace at least its 14 FP64 [ncell][nv] arrays; bad problems
    are rejected as by ugks_create."""
    from paper_2604_09984_amd import ugks, workloads as wl
    case = wl.cylinder(ni=16, nj=8, nvx=12)
    n = case.ncell * case.nv
    s64, a64 = ugks.workspace_size(case, ugks.F64)
    s32, a32 = ugks.workspace_size(case, ugks.F32)
    assert s64 >= 2 * 8 * n and s32 >= 2 * 4 * n and s32 < s64
    assert a64 == a32 >= 14 * 8 * n
    p, keep = _problem(ugks, case, dim=3)
    a, b = C.c_size_t(), C.c_size_t()
    assert ugks.lib().ugks_workspace_size(C.byref(p), C.byref(a), C.byref(b)) == -1


def test_create_with_workspace_rejects_bad_buffers_without_device():
    from paper_2604_09984_amd import ugks, workloads as wl
    case = wl.sod_1d(20, 9)
    p, keep = _problem(ugks, case)
    ctx = C.c_void_p()
    L = ugks.lib()
    assert L.ugks_create_with_workspace(C.byref(p), 0, None, 1 << 20, C.byref(ctx)) == -1
    assert L.ugks_create_with_workspace(C.byref(p), 0, C.c_void_p(4096 + 8), 1 << 20, C.byref(ctx)) == -1
    s, _ = ugks.workspace_size(case, ugks.F64)
    assert L.ugks_create_with_workspace(C.byref(p), 0, C.c_void_p(4096), s - 1, C.byref(ctx)) == -2
    assert not ctx.value
