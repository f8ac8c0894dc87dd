"""ctypes wrapper of the plain-C FP64 oracle.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark; never by the product path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

D = C.POINTER(C.c_double)
I = C.POINTER(C.c_int)
I8 = C.POINTER(C.c_int8)


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "libugks_oracle.so")
        if not os.path.exists(path):
            from . import build as _b  # type: ignore
            _b.build()
        L = C.CDLL(path)
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.c_int, D, I, D, D, D, D, D, C.c_int, I, D, D]
        L.or_free.argtypes = [C.c_void_p]
        for n in ("or_ncell", "or_nface", "or_nv"):
            getattr(L, n).argtypes = [C.c_void_p]
            getattr(L, n).restype = C.c_int
        L.or_set_pose.argtypes = [C.c_void_p, C.c_int] + [C.c_double] * 6
        L.or_update_geometry.argtypes = [C.c_void_p]
        L.or_dvs.argtypes = [C.c_void_p, D, D, D]
        L.or_nc_weights.argtypes = [C.c_int, C.c_double, C.c_double, D]
        L.or_geometry.argtypes = [C.c_void_p, D, D, D, I, I, D, D, D, D]
        L.or_face_ids.argtypes = [C.c_void_p, I, I, I, I]
        L.or_set_types.argtypes = [C.c_void_p, I8]
        L.or_get_types.argtypes = [C.c_void_p, I8]
        L.or_set_overset.argtypes = [C.c_void_p, C.c_int, I, I, I, D]
        L.or_get_overset.argtypes = [C.c_void_p, I, I, I, D]
        L.or_get_overset.restype = C.c_int
        L.or_overset_count.argtypes = [C.c_void_p]
        L.or_nodes.argtypes = [C.c_void_p, D, D]
        L.or_refill_count.argtypes = [C.c_void_p]
        L.or_refill_count.restype = C.c_int
        L.or_overset_count.restype = C.c_int
        L.or_maxwellian.argtypes = [C.c_void_p, D, D, D]
        L.or_moments.argtypes = [C.c_void_p, D, D, D, D]
        L.or_heatflux.argtypes = [C.c_void_p, D, D, D, D]
        L.or_timesteps.argtypes = [C.c_void_p, D]
        L.or_timesteps.restype = C.c_double
        L.or_time_coeffs.argtypes = [C.c_double, C.c_double, D]
        L.or_slope_coeffs.argtypes = [C.c_int, C.c_double, D, C.c_double, D, D, D, D]
        L.or_shakhov.argtypes = [C.c_int, C.c_double, C.c_double, D, C.c_double, D, D, D, D]
        L.or_flux.argtypes = [C.c_void_p, C.c_double, D, D, D, D, D, D, D, D]
        L.or_interp.argtypes = [C.c_void_p, D, D, D, D]
        L.or_begin_step.argtypes = [C.c_void_p, C.c_double, C.c_double, D, D, D, D, D, D, D]
        L.or_pseudo_step.argtypes = [C.c_void_p, C.c_double, C.c_double, D, D, D, D, D, D, D, D, D, D]
        L.or_macro_lusgs.argtypes = [C.c_void_p, C.c_double, D, D, D, D, D, D, D]
        L.or_micro_lusgs.argtypes = [C.c_void_p, C.c_double, D, D, D, D, D, D, D, D, D]
        L.or_step7.argtypes = [C.c_void_p, D, D, D, D]
        L.or_assemble.argtypes = [C.c_void_p, C.c_int, C.c_int, I]
        L.or_assemble.restype = C.c_int
        _LIB = L
    return _LIB


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(D)


def _i(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(I)


def nc_weights(n, a, b):
    w = np.zeros(n)
    lib().or_nc_weights(n, a, b, _d(w))
    return w


def time_coeffs(dts, tau):
    q = np.zeros(5)
    lib().or_time_coeffs(dts, tau, _d(q))
    return q


def slope_coeffs(dim, rho, u, lam, uf, dW):
    u = np.ascontiguousarray(np.resize(np.asarray(u, float), 2))
    uf = np.ascontiguousarray(np.resize(np.asarray(uf, float), 2))
    dW = np.ascontiguousarray(np.asarray(dW, float).reshape(dim, dim + 2))
    a = np.zeros((dim, dim + 2))
    A = np.zeros(dim + 2)
    lib().or_slope_coeffs(dim, rho, _d(u), lam, _d(uf), _d(dW), _d(a), _d(A))
    return a, A


def shakhov(dim, pr, rho, u, lam, q, v):
    u = np.ascontiguousarray(np.resize(np.asarray(u, float), 2))
    q = np.ascontiguousarray(np.resize(np.asarray(q, float), 2))
    v = np.ascontiguousarray(np.resize(np.asarray(v, float), 2))
    hp = np.zeros(1)
    bp = np.zeros(1)
    lib().or_shakhov(dim, pr, rho, _d(u), lam, _d(q), _d(v), _d(hp), _d(bp))
    return hp[0], bp[0]


class Oracle:
    """One case held by the C oracle; state arrays stay in numpy."""

    def __init__(self, case):
        self.case = case
        L = lib()
        gas = np.array([case.pr, case.omega, case.mu_ref, case.rt_ref], dtype=np.float64)
        nv = np.array([case.nvx, case.nvy], dtype=np.int32)
        vr = np.array(case.vrange, dtype=np.float64)
        vx = np.ascontiguousarray(case.vx, dtype=np.float64)
        vy = np.ascontiguousarray(case.vy, dtype=np.float64)
        winf = np.zeros(4)
        winf[:case.nw] = case.winf
        cfl = np.array([case.cfl_s, case.cfl_p], dtype=np.float64)
        bint = case.block_ints()
        bdbl = case.block_dbls()
        nodes = case.node_array()
        self._keep = (gas, nv, vr, vx, vy, winf, cfl, bint, bdbl, nodes)
        self.ptr = L.or_create(case.dim, _d(gas), _i(nv), _d(vr), _d(vx), _d(vy), _d(winf),
                               _d(cfl), len(case.blocks), _i(bint), _d(bdbl), _d(nodes))
        if not self.ptr:
            raise ValueError("oracle rejected the case")
        self.ncell = L.or_ncell(self.ptr)
        self.nface = L.or_nface(self.ptr)
        self.nv = L.or_nv(self.ptr)
        self.dim = case.dim
        self.nw = case.nw

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().or_free(self.ptr)
            self.ptr = None

    # setup ----------------------------------------------------------------
    def set_poses(self, poses):
        for b, p in enumerate(poses):
            lib().or_set_pose(self.ptr, b, *[float(x) for x in p])
        lib().or_update_geometry(self.ptr)

    def dvs(self):
        vx = np.zeros(self.nv); vy = np.zeros(self.nv); w = np.zeros(self.nv)
        lib().or_dvs(self.ptr, _d(vx), _d(vy), _d(w))
        return vx, vy, w

    def geometry(self):
        cx = np.zeros((self.ncell, 2)); vol = np.zeros(self.ncell); g = np.zeros((self.ncell, 4))
        fl = np.zeros(self.nface, np.int32); fr = np.zeros(self.nface, np.int32)
        fn = np.zeros((self.nface, 2)); fs = np.zeros(self.nface)
        fx = np.zeros((self.nface, 2)); fu = np.zeros((self.nface, 2))
        lib().or_geometry(self.ptr, _d(cx), _d(vol), _d(g), _i(fl), _i(fr), _d(fn), _d(fs),
                          _d(fx), _d(fu))
        return dict(cx=cx, vol=vol, g=g, fl=fl, fr=fr, fn=fn, fs=fs, fx=fx, fu=fu)

    def refill_count(self):
        return int(lib().or_refill_count(self.ptr))

    def nodes(self):
        nn = sum((b.ni + 1) * (b.nj + 1) for b in self.case.blocks)
        x = np.zeros(nn); y = np.zeros(nn)
        lib().or_nodes(self.ptr, _d(x), _d(y))
        return x, y

    def face_ids(self):
        a = [np.zeros(self.nface, np.int32) for _ in range(4)]
        lib().or_face_ids(self.ptr, *[_i(x) for x in a])
        return a

    def product_face_index(self):
        """Index of each oracle face in the face numbering of include/ugks.h
        (per block the (ni+1)*nj i-faces, then the ni*(nj+1) j-faces)."""
        blk, dr, fi, fj = self.face_ids()
        offs_i, offs_j, nf = [], [], 0
        for b in self.case.blocks:
            offs_i.append(nf); nf += (b.ni + 1) * b.nj
            offs_j.append(nf)
            if self.case.dim == 2:
                nf += b.ni * (b.nj + 1)
        out = np.zeros(self.nface, np.int64)
        for f in range(self.nface):
            B = self.case.blocks[blk[f]]
            out[f] = (offs_i[blk[f]] + fi[f] + (B.ni + 1) * fj[f]) if dr[f] == 0 else \
                     (offs_j[blk[f]] + fi[f] + B.ni * fj[f])
        return out

    def set_types(self, t):
        t = np.ascontiguousarray(t, dtype=np.int8)
        lib().or_set_types(self.ptr, t.ctypes.data_as(I8))

    def types(self):
        t = np.zeros(self.ncell, np.int8)
        lib().or_get_types(self.ptr, t.ctypes.data_as(I8))
        return t

    def set_overset(self, rec, ptr, don, w):
        rec = np.ascontiguousarray(rec, np.int32); ptr = np.ascontiguousarray(ptr, np.int32)
        don = np.ascontiguousarray(don, np.int32); w = np.ascontiguousarray(w, np.float64)
        lib().or_set_overset(self.ptr, len(rec), _i(rec), _i(ptr), _i(don), _d(w))

    def assemble(self, wrule=0, overlap=2):
        n = np.zeros(1, np.int32)
        rc = lib().or_assemble(self.ptr, int(wrule), int(overlap), _i(n))
        return rc, int(n[0])

    def overset(self):
        """Installed donor table: (rec, ptr, don, w)."""
        L = lib()
        ptr = np.zeros(self.ncell + 1, np.int32)
        rec = np.zeros(self.ncell, np.int32)
        nd = L.or_get_overset(self.ptr, _i(rec), _i(ptr), None, None)
        nrec = int(L.or_overset_count(self.ptr))
        don = np.zeros(max(nd, 1), np.int32); w = np.zeros(max(nd, 1))
        L.or_get_overset(self.ptr, None, None, _i(don), _d(w))
        return rec[:nrec], ptr[:nrec + 1], don[:nd], w[:nd]

    # physics --------------------------------------------------------------
    def maxwellian(self, W):
        h = np.zeros((self.ncell, self.nv)); b = np.zeros((self.ncell, self.nv))
        lib().or_maxwellian(self.ptr, _d(np.ascontiguousarray(W, float)), _d(h), _d(b))
        return h, b

    def moments(self, h, b):
        W = np.zeros((self.ncell, self.nw)); q = np.zeros((self.ncell, self.dim))
        lib().or_moments(self.ptr, _d(h), _d(b), _d(W), _d(q))
        return W, q

    def heatflux(self, h, b, W):
        q = np.zeros((self.ncell, self.dim))
        lib().or_heatflux(self.ptr, _d(h), _d(b), _d(np.ascontiguousarray(W, float)), _d(q))
        return q

    def timesteps(self):
        dtp = np.zeros(self.ncell)
        dts = lib().or_timesteps(self.ptr, _d(dtp))
        return dts, dtp

    def flux(self, dts, h, b, W, q):
        Dh = np.zeros((self.ncell, self.nv)); Db = np.zeros((self.ncell, self.nv))
        F = np.zeros((max(self.nface, 1), self.nw)); wall = np.zeros((max(self.nface, 1), 1 + self.nw))
        lib().or_flux(self.ptr, dts, _d(h), _d(b), _d(W), _d(q), _d(Dh), _d(Db), _d(F), _d(wall))
        return Dh, Db, F, wall

    def interp(self, h, b, W, q):
        lib().or_interp(self.ptr, _d(h), _d(b), _d(W), _d(q))

    def begin_step(self, dt, dts, h, b, W, q):
        Sh = np.zeros_like(h); Sb = np.zeros_like(b); Fn = np.zeros((max(self.nface, 1), self.nw))
        lib().or_begin_step(self.ptr, dt, dts, _d(h), _d(b), _d(W), _d(q), _d(Sh), _d(Sb), _d(Fn))
        return Sh, Sb, Fn

    def pseudo_step(self, dt, dts, dtp, h, b, W, Wn, q, Sh, Sb, Fn):
        resid = np.zeros(self.nw)
        lib().or_pseudo_step(self.ptr, dt, dts, _d(dtp), _d(h), _d(b), _d(W), _d(Wn), _d(q),
                             _d(Sh), _d(Sb), _d(Fn), _d(resid))
        return resid

    def macro_lusgs(self, dt, dtp, W, Wn, F, Fn):
        Wp = np.zeros_like(W); resid = np.zeros(self.nw)
        lib().or_macro_lusgs(self.ptr, dt, _d(dtp), _d(W), _d(Wn), _d(F), _d(Fn), _d(Wp), _d(resid))
        return Wp, resid

    def micro_lusgs(self, dt, dtp, Wp, qp, h, b, Sh, Sb, Dh, Db):
        lib().or_micro_lusgs(self.ptr, dt, _d(dtp), _d(Wp), _d(qp), _d(h), _d(b), _d(Sh), _d(Sb),
                             _d(Dh), _d(Db))

    def step7(self, Wp, h, b):
        W = np.zeros_like(Wp)
        lib().or_step7(self.ptr, _d(Wp), _d(h), _d(b), _d(W))
        return W

    # drivers ----------------------------------------------------------------
    def init_state(self):
        W = np.ascontiguousarray(self.case.w_init, dtype=np.float64).copy()
        h, b = self.maxwellian(W)
        q = self.heatflux(h, b, W)
        return h, b, W, q

    def physical_step(self, t, h, b, W, q, n_inner=None):
        """Steps 1-8 of one physical step from t to t + dt (poses at t + dt)."""
        case = self.case
        dts, dtp = self.timesteps()
        dt = case.dt if case.dt is not None else case.dt_over_dts * dts
        Wn = W.copy()
        Sh, Sb, Fn = self.begin_step(dt, dts, h, b, W, q)
        res = []
        for _ in range(case.n_inner if n_inner is None else n_inner):
            res.append(self.pseudo_step(dt, dts, dtp, h, b, W, Wn, q, Sh, Sb, Fn))
        return dt, np.array(res)
