"""Thin Python binding of libugks (C ABI of include/ugks.h).

Argument marshalling only: every step of the method runs in the HIP
library.  PyTorch provides device memory and streams.  The binding raises if
the library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libugks.so")

F64, F32 = 0, 1

_lib = None


class _Problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("pr", C.c_double), ("omega", C.c_double), ("mu_ref", C.c_double),
                ("rt_ref", C.c_double), ("nvx", C.c_int32), ("nvy", C.c_int32),
                ("vx", C.POINTER(C.c_double)), ("vy", C.POINTER(C.c_double)),
                ("vrange", C.c_double * 4), ("winf", C.c_double * 4), ("cfl_s", C.c_double),
                ("cfl_p", C.c_double), ("nblock", C.c_int32), ("bint", C.POINTER(C.c_int32)),
                ("bdbl", C.POINTER(C.c_double)), ("nodes", C.POINTER(C.c_double)), ("prec", C.c_int32),
                ("nvu", C.c_int32), ("vu", C.POINTER(C.c_double)), ("wu", C.POINTER(C.c_double))]


class UgksError(RuntimeError):
    pass


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise UgksError(f"libugks.so not built ({LIB_PATH}); run paper_2604_09984_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        d = C.c_double
        i32 = C.c_int32
        L.ugks_last_error.restype = C.c_char_p
        L.ugks_create.argtypes = [C.POINTER(_Problem), C.c_int, C.POINTER(vp)]
        L.ugks_destroy.argtypes = [vp]
        L.ugks_sizes.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.ugks_set_poses.argtypes = [vp, C.POINTER(d), C.POINTER(d)]
        L.ugks_set_types.argtypes = [vp, C.POINTER(C.c_int8)]
        L.ugks_set_farfield.argtypes = [vp, C.POINTER(d)]
        L.ugks_get_types.argtypes = [vp, C.POINTER(C.c_int8)]
        L.ugks_set_overset.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(d)]
        L.overset_assemble.argtypes = [vp, i32, i32, C.POINTER(i32)]
        L.overset_assemble_device.argtypes = [vp, i32, i32, C.POINTER(i32)]
        L.ugks_get_overset.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32),
                                       C.POINTER(i32), C.POINTER(d)]
        L.ugks_maxwellian.argtypes = [vp, vp, vp, vp, vp]
        L.ugks_moments.argtypes = [vp, vp, vp, vp, vp, vp]
        L.ugks_heatflux.argtypes = [vp, vp, vp, vp, vp, vp]
        L.ugks_flux.argtypes = [vp, d, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.overset_interp.argtypes = [vp, vp, vp, vp, vp, vp]
        L.ugks_begin_step.argtypes = [vp, d, vp, vp, vp, vp, vp, vp, vp, vp]
        L.ugks_step.argtypes = [vp, d, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.ugks_timesteps.argtypes = [vp, C.POINTER(d), C.POINTER(d)]
        L.ugks_step_profile.argtypes = [vp, d, i32, vp, vp, vp, vp, vp, vp, vp, vp, C.POINTER(d), vp]
        L.ugks_step_graph.argtypes = [vp, d, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        pa = C.POINTER(vp)
        L.ugks_batch_create.argtypes = [i32, pa, C.POINTER(vp)]
        L.ugks_batch_destroy.argtypes = [vp]
        L.ugks_batch_step.argtypes = [vp, C.POINTER(d), i32, pa, pa, pa, pa, pa, pa, pa, pa, pa, vp]
        L.ugks_batch_set_mode.argtypes = [vp, i32]
        L.ugks_batch_get_mode.argtypes = [vp, C.POINTER(i32)]
        L.ugks_set_tuning.argtypes = [vp, i32, i32, i32]
        L.ugks_get_tuning.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.ugks_micro_shape.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.ugks_autotune.argtypes = [vp, d, i32, vp, vp, vp, vp, vp, vp, vp, vp, C.POINTER(i32), C.POINTER(d), vp]
        L.ugks_set_wall_rt.argtypes = [vp, i32, i32, d]
        L.ugks_set_block_velocity.argtypes = [vp, i32, d, d, d]
        L.ugks_face_geometry.argtypes = [vp, C.POINTER(d)]
        L.ugks_overset_rows.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.ugks_last_flux.argtypes = [vp, vp, vp]
        L.ugks_flux_adjoint.argtypes = [vp] + [vp] * 12 + [vp]
        L.ugks_step_adjoint.argtypes = [vp, d] + [vp] * 22 + [vp]
        L.ugks_begin_step_adjoint.argtypes = [vp, d, vp, vp, vp, vp, i32] + [vp] * 12 + [vp]
        L.ugks_workspace_size.argtypes = [C.POINTER(_Problem), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
        L.ugks_create_with_workspace.argtypes = [C.POINTER(_Problem), C.c_int, vp, C.c_size_t, C.POINTER(vp)]
        L.ugks_status.argtypes = [vp, vp]
        L.ugks_set_checks.argtypes = [vp, i32, i32]
        L.ugks_wall_loads.argtypes = [vp, vp, vp, vp, vp]
        L.ugks_wall_loads_adjoint.argtypes = [vp, vp, vp, vp, vp]
        L.ugks_param_bars.argtypes = [vp, vp, vp, vp, vp]
        L.ugks_newton_euler.argtypes = [vp, i32, C.POINTER(d), d, vp, C.POINTER(d), vp]
        L.ugks_flux_noalloc.argtypes = [vp, d, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def exported_symbols():
    return ["ugks_create", "ugks_destroy", "ugks_sizes", "ugks_set_poses", "ugks_set_types",
            "ugks_get_types", "ugks_set_overset", "overset_assemble", "overset_assemble_device", "ugks_get_overset", "ugks_maxwellian",
            "ugks_moments", "ugks_heatflux", "ugks_flux", "overset_interp", "ugks_begin_step", "ugks_step",
            "ugks_timesteps", "ugks_step_profile", "ugks_step_graph", "ugks_batch_create", "ugks_batch_step",
            "ugks_batch_destroy", "ugks_batch_set_mode", "ugks_batch_get_mode", "ugks_set_tuning", "ugks_get_tuning", "ugks_micro_shape", "ugks_autotune", "ugks_set_wall_rt",
            "ugks_last_flux", "ugks_set_block_velocity", "ugks_set_farfield", "ugks_face_geometry", "ugks_overset_rows",
            "ugks_flux_adjoint", "ugks_step_adjoint", "ugks_begin_step_adjoint",
            "ugks_workspace_size", "ugks_create_with_workspace", "ugks_status", "ugks_set_checks",
            "ugks_wall_loads", "ugks_wall_loads_adjoint", "ugks_param_bars", "ugks_newton_euler",
            "ugks_flux_noalloc", "ugks_last_error"]


def _check(rc):
    if rc != 0:
        msg = lib().ugks_last_error().decode()
        raise UgksError(f"libugks error {rc}: {msg}")


def _p(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return C.c_void_p(t.data_ptr())


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _problem(case, prec):
    """The ugks_problem of a case and the host arrays it points to."""
    vx = np.ascontiguousarray(case.vx, dtype=np.float64)
    vy = np.ascontiguousarray(case.vy, dtype=np.float64)
    bint = case.block_ints()
    bdbl = case.block_dbls()
    nodes = case.node_array()
    p = _Problem()
    p.dim = case.dim
    p.pr, p.omega, p.mu_ref, p.rt_ref = case.pr, case.omega, case.mu_ref, case.rt_ref
    p.nvx, p.nvy = case.nvx, case.nvy
    p.vx, p.vy = _dp(vx), _dp(vy)
    for m in range(4):
        p.vrange[m] = float(case.vrange[m])
        p.winf[m] = float(case.winf[m]) if m < case.nw else 0.0
    p.cfl_s, p.cfl_p = case.cfl_s, case.cfl_p
    p.nblock = len(case.blocks)
    p.bint = bint.ctypes.data_as(C.POINTER(C.c_int32))
    p.bdbl = _dp(bdbl)
    p.nodes = _dp(nodes)
    p.prec = prec
    keep = (vx, vy, bint, bdbl, nodes)
    dvs = getattr(case, "dvs", None)
    if dvs is not None:
        # unstructured velocity mesh: points (x then y) and cell areas
        vu = np.ascontiguousarray(np.concatenate([dvs[0], dvs[1]]), dtype=np.float64)
        wu = np.ascontiguousarray(dvs[2], dtype=np.float64)
        p.nvu, p.vu, p.wu = len(dvs[0]), _dp(vu), _dp(wu)
        keep = keep + (vu, wu)
    return p, keep


def workspace_size(case, prec: int = F64):
    """(scratch bytes, adjoint workspace bytes) of a case (ugks_workspace_size)."""
    p, keep = _problem(case, prec)
    a, b = C.c_size_t(), C.c_size_t()
    _check(lib().ugks_workspace_size(C.byref(p), C.byref(a), C.byref(b)))
    return a.value, b.value


class Solver:
    """A libugks context for one case (see workloads.Case).  With
    workspace="scratch" or "all" the context's scratch (and with "all" also
    the reverse-mode workspace) lives in a torch-allocated device buffer
    (ugks_create_with_workspace) that the Solver keeps."""

    def __init__(self, case, prec: int = F64, device: int = 0, workspace: Optional[str] = None):
        L = lib()
        self.case = case
        self.prec = prec
        self.device = torch.device("cuda", device)
        self.dtype = torch.float64 if prec == F64 else torch.float32
        p, self._keep = _problem(case, prec)
        ctx = C.c_void_p()
        if workspace is None:
            _check(L.ugks_create(C.byref(p), device, C.byref(ctx)))
            self.workspace = None
        else:
            sb, ab = workspace_size(case, prec)
            nbytes = sb + (ab if workspace == "all" else 0)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            off = (-base) % 256
            _check(L.ugks_create_with_workspace(C.byref(p), device, C.c_void_p(base + off), C.c_size_t(nbytes),
                                                C.byref(ctx)))
        self.ctx = ctx
        n = [C.c_int32() for _ in range(4)]
        _check(L.ugks_sizes(ctx, *[C.byref(x) for x in n]))
        self.ncell, self.nface, self.nv = n[0].value, n[1].value, n[2].value
        self.dim, self.nw = case.dim, case.nw

    def close(self):
        if getattr(self, "ctx", None):
            lib().ugks_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ setup
    def set_poses(self, poses) -> float:
        a = np.ascontiguousarray(np.asarray(poses, dtype=np.float64).reshape(-1, 6))
        dts = C.c_double()
        _check(lib().ugks_set_poses(self.ctx, _dp(a), C.byref(dts)))
        self.poses = a.copy()
        return dts.value

    def timesteps(self):
        dts = C.c_double()
        dtp = np.zeros(self.ncell)
        _check(lib().ugks_timesteps(self.ctx, C.byref(dts), _dp(dtp)))
        return dts.value, dtp

    def set_types(self, t):
        t = np.ascontiguousarray(t, dtype=np.int8)
        _check(lib().ugks_set_types(self.ctx, t.ctypes.data_as(C.POINTER(C.c_int8))))

    def types(self):
        t = np.zeros(self.ncell, np.int8)
        _check(lib().ugks_get_types(self.ctx, t.ctypes.data_as(C.POINTER(C.c_int8))))
        return t

    def set_overset(self, rec, ptr, don, w):
        rec = np.ascontiguousarray(rec, np.int32); ptr = np.ascontiguousarray(ptr, np.int32)
        don = np.ascontiguousarray(don, np.int32); w = np.ascontiguousarray(w, np.float64)
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        _check(lib().ugks_set_overset(self.ctx, len(rec), ip(rec), ip(ptr), ip(don), _dp(w)))

    def assemble(self, wrule=0, overlap=2, device=False) -> int:
        """Overset assembly at the installed poses (on the GPU with
        device=True; identical results); returns the receptor count."""
        n = C.c_int32()
        fn = lib().overset_assemble_device if device else lib().overset_assemble
        _check(fn(self.ctx, int(wrule), int(overlap), C.byref(n)))
        return n.value

    def overset(self):
        """Installed donor table: (rec, ptr, don, w) host arrays."""
        nrec, nd = C.c_int32(), C.c_int32()
        _check(lib().ugks_get_overset(self.ctx, C.byref(nrec), C.byref(nd), None, None, None, None))
        rec = np.zeros(max(nrec.value, 1), np.int32); ptr = np.zeros(nrec.value + 1, np.int32)
        don = np.zeros(max(nd.value, 1), np.int32); w = np.zeros(max(nd.value, 1))
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        _check(lib().ugks_get_overset(self.ctx, None, None, ip(rec), ip(ptr), ip(don), _dp(w)))
        return rec[:nrec.value], ptr, don[:nd.value], w[:nd.value]

    # -------------------------------------------------------------- tensors
    def empty_f(self):
        return torch.empty((self.ncell, self.nv), dtype=self.dtype, device=self.device)

    def zeros_w(self):
        return torch.zeros((self.ncell, self.nw), dtype=torch.float64, device=self.device)

    def zeros_q(self):
        return torch.zeros((self.ncell, self.dim), dtype=torch.float64, device=self.device)

    def zeros_face(self, width):
        return torch.zeros((self.nface, width), dtype=torch.float64, device=self.device)

    def _stream(self, stream):
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return C.c_void_p(s.cuda_stream)

    # ------------------------------------------------------------ compute
    def maxwellian(self, W, stream=None):
        h, b = self.empty_f(), self.empty_f()
        _check(lib().ugks_maxwellian(self.ctx, _p(W), _p(h), _p(b), self._stream(stream)))
        return h, b

    def moments(self, h, b, stream=None):
        W, q = self.zeros_w(), self.zeros_q()
        _check(lib().ugks_moments(self.ctx, _p(h), _p(b), _p(W), _p(q), self._stream(stream)))
        return W, q

    def flux(self, dts, h, b, W, q, stream=None):
        Dh, Db = self.empty_f(), self.empty_f()
        F, wall = self.zeros_face(self.nw), self.zeros_face(self.nw + 1)
        _check(lib().ugks_flux(self.ctx, float(dts), _p(h), _p(b), _p(W), _p(q), _p(Dh), _p(Db), _p(F),
                               _p(wall), self._stream(stream)))
        return Dh, Db, F, wall

    def interp(self, h, b, W, q, stream=None):
        _check(lib().overset_interp(self.ctx, _p(h), _p(b), _p(W), _p(q), self._stream(stream)))

    def begin_step(self, dt, h, b, W, q, Sh=None, Sb=None, Fn=None, stream=None):
        Sh = self.empty_f() if Sh is None else Sh
        Sb = self.empty_f() if Sb is None else Sb
        Fn = self.zeros_face(self.nw) if Fn is None else Fn
        _check(lib().ugks_begin_step(self.ctx, float(dt), _p(h), _p(b), _p(W), _p(q), _p(Sh), _p(Sb), _p(Fn),
                                     self._stream(stream)))
        return Sh, Sb, Fn

    def step(self, dt, n_inner, h, b, W, Wn, q, Sh, Sb, Fn, resid=None, stream=None):
        _check(lib().ugks_step(self.ctx, float(dt), int(n_inner), _p(h), _p(b), _p(W), _p(Wn), _p(q), _p(Sh),
                               _p(Sb), _p(Fn), _p(resid), self._stream(stream)))
        return resid

    def step_graph(self, dt, n_inner, h, b, W, Wn, q, Sh, Sb, Fn, resid=None, stream=None):
        """ugks_step through the context's captured graph (same results)."""
        _check(lib().ugks_step_graph(self.ctx, float(dt), int(n_inner), _p(h), _p(b), _p(W), _p(Wn), _p(q),
                                     _p(Sh), _p(Sb), _p(Fn), _p(resid), self._stream(stream)))
        return resid

    def set_tuning(self, kc_max=16, rg_eq=8, rg_flux=8):
        _check(lib().ugks_set_tuning(self.ctx, int(kc_max), int(rg_eq), int(rg_flux)))

    def tuning(self):
        v = [C.c_int32() for _ in range(3)]
        _check(lib().ugks_get_tuning(self.ctx, *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def micro_shape(self):
        """(chunk width, rows per thread, ring depth, fused residual) of the
        micro sweep under the current tuning."""
        v = [C.c_int32() for _ in range(4)]
        _check(lib().ugks_micro_shape(self.ctx, *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def autotune(self, dt, n_inner, h, b, W, Wn, q, Sh, Sb, Fn, stream=None):
        """Time the launch shapes on copies of the state; keeps and returns
        the fastest ((kc_max, rg_eq, rg_flux), ms per pseudo-iteration)."""
        ch = (C.c_int32 * 3)()
        ms = C.c_double()
        _check(lib().ugks_autotune(self.ctx, float(dt), int(n_inner), _p(h), _p(b), _p(W), _p(Wn), _p(q),
                                   _p(Sh), _p(Sb), _p(Fn), ch, C.byref(ms), self._stream(stream)))
        return tuple(ch), ms.value

    def set_wall_rt(self, blk, side, rtw):
        """RT of the isothermal wall on one side of a block."""
        _check(lib().ugks_set_wall_rt(self.ctx, int(blk), int(side), float(rtw)))

    def set_farfield(self, winf):
        """Far-field conservative state (nw values) and its Maxwellian
        (ugks_set_farfield)."""
        a = np.zeros(4)
        a[:self.nw] = np.asarray(winf, dtype=np.float64).reshape(-1)[:self.nw]
        _check(lib().ugks_set_farfield(self.ctx, _dp(a)))

    def set_block_velocity(self, blk, ux, uy, om=0.0):
        """Rigid velocity of a block; geometry, dt_s and dt' stay fixed."""
        _check(lib().ugks_set_block_velocity(self.ctx, int(blk), float(ux), float(uy), float(om)))

    def face_geometry(self):
        """Host [nface][8]: normal (2), area, grid velocity (2), wall velocity
        (2), wall RT."""
        g = np.zeros((self.nface, 8))
        _check(lib().ugks_face_geometry(self.ctx, _dp(g)))
        return g

    def overset_rows(self):
        """(receptor rows, refill rows, refills pending) of the donor table."""
        v = [C.c_int32() for _ in range(3)]
        _check(lib().ugks_overset_rows(self.ctx, *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def status(self, stream=None):
        """Waits for the stream and raises UgksError if a device-side check
        failed (ugks_status: -3 a sweep's wait ran out, -4 a non-physical
        state)."""
        _check(lib().ugks_status(self.ctx, self._stream(stream)))

    def status_code(self, stream=None) -> int:
        """ugks_status's return code (0 when no check failed)."""
        return int(lib().ugks_status(self.ctx, self._stream(stream)))

    def set_checks(self, sync=False, wait_limit=-1):
        """ugks_set_checks: synchronising status checks; bound of the micro
        sweep's neighbour wait (negative: default)."""
        _check(lib().ugks_set_checks(self.ctx, int(bool(sync)), int(wait_limit)))

    def wall_loads(self, F, stream=None):
        """(face loads [nface][dim+3], side loads [nblock][4][4]) of a face
        macro flux F (ugks_wall_loads)."""
        fo = self.zeros_face(self.dim + 3)
        so = torch.zeros((len(self.case.blocks), 4, 4), dtype=torch.float64, device=self.device)
        _check(lib().ugks_wall_loads(self.ctx, _p(F.contiguous()), _p(fo), _p(so), self._stream(stream)))
        return fo, so

    def wall_loads_adjoint(self, face_bar=None, side_bar=None, stream=None):
        """F_bar [nface][nw] from cotangents of the wall loads."""
        Fb = self.zeros_face(self.nw)
        _check(lib().ugks_wall_loads_adjoint(self.ctx, _p(None if face_bar is None else face_bar.contiguous()),
                                             _p(None if side_bar is None else side_bar.contiguous()), _p(Fb),
                                             self._stream(stream)))
        return Fb

    def param_bars(self, face_bar, stream=None):
        """(U_bar [nblock][2], rtw_bar [nblock][4]) from per-face
        cotangents [nface][5] (ugks_param_bars)."""
        nb = len(self.case.blocks)
        U = torch.zeros((nb, 2), dtype=torch.float64, device=self.device)
        R = torch.zeros((nb, 4), dtype=torch.float64, device=self.device)
        _check(lib().ugks_param_bars(self.ctx, _p(face_bar.contiguous()), _p(U), _p(R), self._stream(stream)))
        return U, R

    def newton_euler(self, blk, body, dt, F, pose, stream=None):
        """The block's pose [6] after one Newton-Euler step driven by the wall
        loads of F and the external load in body = (m, I, Fx, Fy, Mz)
        (ugks_newton_euler); returns the new pose (host)."""
        p = np.ascontiguousarray(np.array(pose, dtype=np.float64))
        bd = np.ascontiguousarray(np.array(body, dtype=np.float64))
        _check(lib().ugks_newton_euler(self.ctx, int(blk), _dp(bd), float(dt), _p(F.contiguous()), _dp(p),
                                       self._stream(stream)))
        return p

    def last_flux(self, stream=None):
        """Face macro flux [nface][nw] of the last flux evaluation."""
        F = self.zeros_face(self.nw)
        _check(lib().ugks_last_flux(self.ctx, _p(F), self._stream(stream)))
        return F

    # ------------------------------------------------ reverse mode (adjoint)
    def _bar(self, t, shape):
        if t is None:
            return None
        assert t.dtype == torch.float64 and tuple(t.shape) == shape, (t.dtype, t.shape, shape)
        return t.contiguous()

    def flux_adjoint(self, h, b, W, q, Dh_bar=None, Db_bar=None, F_bar=None, stream=None):
        """Cotangents (h, b, W, q, face[nface][5]) of ugks_flux at dt_s."""
        f, fw = (self.ncell, self.nv), (self.nface, self.nw)
        Dh_bar, Db_bar, F_bar = self._bar(Dh_bar, f), self._bar(Db_bar, f), self._bar(F_bar, fw)
        out = [torch.empty(f, dtype=torch.float64, device=self.device) for _ in range(2)]
        out += [self.zeros_w(), self.zeros_q(), self.zeros_face(5)]
        _check(lib().ugks_flux_adjoint(self.ctx, _p(h), _p(b), _p(W), _p(q), _p(Dh_bar), _p(Db_bar), _p(F_bar),
                                       *[_p(t) for t in out], self._stream(stream)))
        return tuple(out)

    def step_adjoint(self, dt, h, b, W, Wn, q, Sh, Sb, Fn, h1_bar=None, b1_bar=None, W1_bar=None, q1_bar=None,
                     F_bar=None, stream=None):
        """Cotangents of one inner iteration at its inputs: returns
        (h, b, W, Wn, q, Sh, Sb, Fn, face[nface][5]) bars."""
        f, w, qq, fw = (self.ncell, self.nv), (self.ncell, self.nw), (self.ncell, self.dim), (self.nface, self.nw)
        bars = [self._bar(h1_bar, f), self._bar(b1_bar, f), self._bar(W1_bar, w), self._bar(q1_bar, qq),
                self._bar(F_bar, fw)]
        out = [torch.empty(f, dtype=torch.float64, device=self.device) for _ in range(2)]
        out += [self.zeros_w(), self.zeros_w(), self.zeros_q()]
        out += [torch.empty(f, dtype=torch.float64, device=self.device) for _ in range(2)]
        out += [self.zeros_face(self.nw), self.zeros_face(5)]
        _check(lib().ugks_step_adjoint(self.ctx, float(dt), _p(h), _p(b), _p(W), _p(Wn), _p(q), _p(Sh), _p(Sb),
                                       _p(Fn), *[_p(t) for t in bars], *[_p(t) for t in out],
                                       self._stream(stream)))
        return tuple(out)

    def begin_step_adjoint(self, dt, h, b, W, q, h1_bar=None, b1_bar=None, W1_bar=None, q1_bar=None,
                           Sh_bar=None, Sb_bar=None, Fn_bar=None, refill=False, stream=None):
        """Cotangents of Steps 1-2 at their inputs: (h, b, W, q, face) bars."""
        f, w, qq, fw = (self.ncell, self.nv), (self.ncell, self.nw), (self.ncell, self.dim), (self.nface, self.nw)
        Sh_bar = torch.zeros(f, dtype=torch.float64, device=self.device) if Sh_bar is None else Sh_bar
        Sb_bar = torch.zeros(f, dtype=torch.float64, device=self.device) if Sb_bar is None else Sb_bar
        bars = [self._bar(h1_bar, f), self._bar(b1_bar, f), self._bar(W1_bar, w), self._bar(q1_bar, qq),
                self._bar(Sh_bar, f), self._bar(Sb_bar, f), self._bar(Fn_bar, fw)]
        out = [torch.empty(f, dtype=torch.float64, device=self.device) for _ in range(2)]
        out += [self.zeros_w(), self.zeros_q(), self.zeros_face(5)]
        _check(lib().ugks_begin_step_adjoint(self.ctx, float(dt), _p(h), _p(b), _p(W), _p(q), int(bool(refill)),
                                             *[_p(t) for t in bars], *[_p(t) for t in out], self._stream(stream)))
        return tuple(out)

    STAGES = ["interp", "gradW_wall", "face_eq", "face_fin", "flux", "flux_fin", "macro_lusgs", "cell_rec",
              "micro_rhs", "micro_sweep", "step7"]

    def step_profile(self, dt, n_inner, h, b, W, Wn, q, Sh, Sb, Fn, stream=None):
        """Run n_inner pseudo-iterations with stage timing; returns
        {stage: mean ms per pseudo-iteration} (synchronous)."""
        ms = (C.c_double * len(self.STAGES))()
        _check(lib().ugks_step_profile(self.ctx, float(dt), int(n_inner), _p(h), _p(b), _p(W), _p(Wn), _p(q),
                                       _p(Sh), _p(Sb), _p(Fn), ms, self._stream(stream)))
        return dict(zip(self.STAGES, list(ms)))

    # ------------------------------------------------------------- driver
    def init_state(self):
        W = torch.tensor(np.asarray(self.case.w_init, dtype=np.float64), device=self.device).contiguous()
        h, b = self.maxwellian(W)
        q = self.heatflux(h, b, W)
        return h, b, W, q

    def heatflux(self, h, b, W, stream=None):
        """Heat flux of (h, b) about the velocity of W."""
        q = self.zeros_q()
        _check(lib().ugks_heatflux(self.ctx, _p(h), _p(b), _p(W), _p(q), self._stream(stream)))
        return q

    def physical_step(self, dt, h, b, W, q, n_inner=None, resid=None):
        Wn = W.clone()
        Sh, Sb, Fn = self.begin_step(dt, h, b, W, q)
        n = self.case.n_inner if n_inner is None else n_inner
        self.step(dt, n, h, b, W, Wn, q, Sh, Sb, Fn, resid)
        return Wn


class Batch:
    """Independent cases (one Solver each, ragged sizes) advanced together
    from one captured graph: mode 1, one launch per stage for all cases
    (persistent march and micro-sweep grids over work items); mode 0, each
    case's own kernel chain on concurrent branches."""

    def __init__(self, solvers, mode=None):
        self.solvers = list(solvers)
        arr = (C.c_void_p * len(self.solvers))(*[s.ctx for s in self.solvers])
        h = C.c_void_p()
        _check(lib().ugks_batch_create(len(self.solvers), arr, C.byref(h)))
        self.handle = h
        if mode is not None:
            self.set_mode(mode)

    def set_mode(self, mode):
        _check(lib().ugks_batch_set_mode(self.handle, int(mode)))

    @property
    def mode(self):
        m = C.c_int32()
        _check(lib().ugks_batch_get_mode(self.handle, C.byref(m)))
        return int(m.value)

    def close(self):
        if getattr(self, "handle", None):
            lib().ugks_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()

    def step(self, dts, n_inner, states, resid=None, stream=None):
        """states: per case (h, b, W, Wn, q, Sh, Sb, Fn) device tensors."""
        n = len(self.solvers)
        cols = list(zip(*states))
        ptrs = [(C.c_void_p * n)(*[t.data_ptr() for t in col]) for col in cols]
        rp = None if resid is None else (C.c_void_p * n)(*[0 if r is None else r.data_ptr() for r in resid])
        dt = (C.c_double * n)(*[float(x) for x in dts])
        st = self.solvers[0]._stream(stream)
        _check(lib().ugks_batch_step(self.handle, dt, int(n_inner), *ptrs, rp, st))
