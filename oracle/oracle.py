"""ctypes wrapper of the plain-C FP64 oracle.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark; never by the product path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIBS = {}

D = C.POINTER(C.c_double)
I = C.POINTER(C.c_int)
I8 = C.POINTER(C.c_int8)


class Dual(C.Structure):
    """A scalar of the tangent build: value and directional derivative."""
    _fields_ = [("v", C.c_double), ("d", C.c_double)]


def _bind(L, S):
    """Argument types of every entry point; S is the scalar type (double, or
    Dual in the tangent build, whose arrays are (value, tangent) pairs)."""
    L.or_create.restype = C.c_void_p
    L.or_create.argtypes = [C.c_int, D, I, D, D, D, D, D, C.c_int, I, D, D]
    L.or_free.argtypes = [C.c_void_p]
    L.or_set_dvs.argtypes = [C.c_void_p, C.c_int, D, D, D]
    L.or_set_dvs.restype = C.c_int
    for n in ("or_ncell", "or_nface", "or_nv"):
        getattr(L, n).argtypes = [C.c_void_p]
        getattr(L, n).restype = C.c_int
    L.or_set_pose.argtypes = [C.c_void_p, C.c_int] + [S] * 6
    L.or_set_wall_rt.argtypes = [C.c_void_p, C.c_int, C.c_int, S]
    L.or_set_farfield.argtypes = [C.c_void_p, D]
    L.or_update_geometry.argtypes = [C.c_void_p]
    L.or_dvs.argtypes = [C.c_void_p, D, D, D]
    L.or_nc_weights.argtypes = [C.c_int, S, S, D]
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
    L.or_timesteps.restype = S
    L.or_time_coeffs.argtypes = [S, S, D]
    L.or_slope_coeffs.argtypes = [C.c_int, S, D, S, D, D, D, D]
    L.or_shakhov.argtypes = [C.c_int, S, S, D, S, D, D, D, D]
    L.or_flux.argtypes = [C.c_void_p, S, D, D, D, D, D, D, D, D]
    L.or_interp.argtypes = [C.c_void_p, D, D, D, D]
    L.or_wall_loads.argtypes = [C.c_void_p, D, D, D]
    L.or_newton_euler.argtypes = [C.c_void_p, C.c_int, D, S, D, D]
    L.or_begin_step.argtypes = [C.c_void_p, S, S, D, D, D, D, D, D, D]
    L.or_begin_step_cells.argtypes = [C.c_void_p, S, S, D, D, D, D, C.c_int, I, D, D, D]
    L.or_pseudo_step.argtypes = [C.c_void_p, S, S, D, D, D, D, D, D, D, D, D, D, D]
    L.or_macro_lusgs.argtypes = [C.c_void_p, S, D, D, D, D, D, D, D]
    L.or_micro_lusgs.argtypes = [C.c_void_p, S, D, D, D, D, D, D, D, D, D]
    L.or_step7.argtypes = [C.c_void_p, D, D, D, D]
    L.or_assemble.argtypes = [C.c_void_p, C.c_int, C.c_int, I]
    L.or_assemble.restype = C.c_int
    return L


def lib(tangent=False):
    """The double build, or with tangent=True the dual-number build."""
    if tangent not in _LIBS:
        name = "libugks_oracle_tl.so" if tangent else "libugks_oracle.so"
        path = os.path.join(HERE, name)
        if not os.path.exists(path):
            from . import build as _b  # type: ignore
            _b.build()
        _LIBS[tangent] = _bind(C.CDLL(path), Dual if tangent else C.c_double)
    return _LIBS[tangent]


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


def dual(v, t=None):
    """(value, tangent) pairs of the tangent build from a value array and an
    optional tangent array of the same shape (zero if omitted)."""
    v = np.asarray(v, dtype=np.float64)
    out = np.zeros(v.shape + (2,))
    out[..., 0] = v
    if t is not None:
        out[..., 1] = t
    return out


class Oracle:
    """One case held by the C oracle; state arrays stay in numpy.

    With tangent=True the case lives in the dual-number build: every float
    array argument and result carries a trailing axis of two (value, tangent;
    see dual()), scalars may be given as (value, tangent) tuples, and each
    result's tangent is the directional derivative along the seeded inputs."""

    def __init__(self, case, tangent=False):
        self.case = case
        self.tangent = tangent
        self.L = L = lib(tangent)
        gas = self._in(np.array([case.pr, case.omega, case.mu_ref, case.rt_ref], dtype=np.float64))
        nv = np.array([case.nvx, case.nvy], dtype=np.int32)
        vr = self._in(np.array(case.vrange, dtype=np.float64))
        vx = self._in(np.ascontiguousarray(case.vx, dtype=np.float64))
        vy = self._in(np.ascontiguousarray(case.vy, dtype=np.float64))
        winf = np.zeros(4)
        winf[:case.nw] = case.winf
        winf = self._in(winf)
        cfl = self._in(np.array([case.cfl_s, case.cfl_p], dtype=np.float64))
        bint = case.block_ints()
        bdbl = self._in(case.block_dbls())
        nodes = self._in(case.node_array())
        self._keep = (gas, nv, vr, vx, vy, winf, cfl, bint, bdbl, nodes)
        self.ptr = L.or_create(case.dim, _d(gas), _i(nv), _d(vr), _d(vx), _d(vy), _d(winf),
                               _d(cfl), len(case.blocks), _i(bint), _d(bdbl), _d(nodes))
        if not self.ptr:
            raise ValueError("oracle rejected the case")
        if getattr(case, "dvs", None) is not None:
            dx, dy, dw = (self._in(np.ascontiguousarray(a, dtype=np.float64)) for a in case.dvs)
            if L.or_set_dvs(self.ptr, len(case.dvs[0]), _d(dx), _d(dy), _d(dw)) != 0:
                raise ValueError("oracle rejected the velocity mesh")
        self.ncell = L.or_ncell(self.ptr)
        self.nface = L.or_nface(self.ptr)
        self.nv = L.or_nv(self.ptr)
        self.dim = case.dim
        self.nw = case.nw

    def __del__(self):
        if getattr(self, "ptr", None):
            self.L.or_free(self.ptr)
            self.ptr = None

    # scalar and array conventions of the two builds
    def _in(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        return dual(a) if self.tangent else a

    def _z(self, *shape):
        return np.zeros(shape + ((2,) if self.tangent else ()))

    def _s(self, x):
        if not self.tangent:
            return float(x)
        if isinstance(x, (tuple, list, np.ndarray)):
            return Dual(float(x[0]), float(x[1]))
        return Dual(float(x), 0.0)

    def _val(self, a):
        return a[..., 0] if self.tangent else a

    # setup ----------------------------------------------------------------
    def set_poses(self, poses):
        for b, p in enumerate(poses):
            self.L.or_set_pose(self.ptr, b, *[self._s(x) for x in p])
        self.L.or_update_geometry(self.ptr)

    def set_wall_rt(self, blk, side, rtw):
        """RT of the isothermal wall on one block side (scalar or (v, t))."""
        self.L.or_set_wall_rt(self.ptr, int(blk), int(side), self._s(rtw))

    def set_farfield(self, winf):
        """Far-field conservative state (nw values; held fixed in the tangent
        build) and its Maxwellian."""
        w = self._in(np.asarray(winf, dtype=np.float64).reshape(-1)[:self.case.nw].copy())
        self._keep_farfield = w
        self.L.or_set_farfield(self.ptr, _d(w))

    def dvs(self):
        vx = self._z(self.nv); vy = self._z(self.nv); w = self._z(self.nv)
        self.L.or_dvs(self.ptr, _d(vx), _d(vy), _d(w))
        return self._val(vx), self._val(vy), self._val(w)

    def geometry(self):
        z = self._z
        cx = z(self.ncell, 2); vol = z(self.ncell); g = z(self.ncell, 4)
        fl = np.zeros(self.nface, np.int32); fr = np.zeros(self.nface, np.int32)
        fn = z(self.nface, 2); fs = z(self.nface)
        fx = z(self.nface, 2); fu = z(self.nface, 2)
        self.L.or_geometry(self.ptr, _d(cx), _d(vol), _d(g), _i(fl), _i(fr), _d(fn), _d(fs),
                           _d(fx), _d(fu))
        v = self._val
        return dict(cx=v(cx), vol=v(vol), g=v(g), fl=fl, fr=fr, fn=v(fn), fs=v(fs), fx=v(fx), fu=v(fu))

    def refill_count(self):
        return int(self.L.or_refill_count(self.ptr))

    def nodes(self):
        nn = sum((b.ni + 1) * (b.nj + 1) for b in self.case.blocks)
        x = self._z(nn); y = self._z(nn)
        self.L.or_nodes(self.ptr, _d(x), _d(y))
        return self._val(x), self._val(y)

    def face_ids(self):
        a = [np.zeros(self.nface, np.int32) for _ in range(4)]
        self.L.or_face_ids(self.ptr, *[_i(x) for x in a])
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
        self.L.or_set_types(self.ptr, t.ctypes.data_as(I8))

    def types(self):
        t = np.zeros(self.ncell, np.int8)
        self.L.or_get_types(self.ptr, t.ctypes.data_as(I8))
        return t

    def set_overset(self, rec, ptr, don, w):
        rec = np.ascontiguousarray(rec, np.int32); ptr = np.ascontiguousarray(ptr, np.int32)
        don = np.ascontiguousarray(don, np.int32); w = self._in(w)
        self.L.or_set_overset(self.ptr, len(rec), _i(rec), _i(ptr), _i(don), _d(w))

    def assemble(self, wrule=0, overlap=2):
        n = np.zeros(1, np.int32)
        rc = self.L.or_assemble(self.ptr, int(wrule), int(overlap), _i(n))
        return rc, int(n[0])

    def overset(self):
        """Installed donor table: (rec, ptr, don, w)."""
        L = self.L
        ptr = np.zeros(self.ncell + 1, np.int32)
        rec = np.zeros(self.ncell, np.int32)
        nd = L.or_get_overset(self.ptr, _i(rec), _i(ptr), None, None)
        nrec = int(L.or_overset_count(self.ptr))
        don = np.zeros(max(nd, 1), np.int32); w = self._z(max(nd, 1))
        L.or_get_overset(self.ptr, None, None, _i(don), _d(w))
        return rec[:nrec], ptr[:nrec + 1], don[:nd], self._val(w)[:nd]

    # physics --------------------------------------------------------------
    # (tangent build: float arrays in and out carry the trailing (value,
    # tangent) axis)
    def maxwellian(self, W):
        h = self._z(self.ncell, self.nv); b = self._z(self.ncell, self.nv)
        self.L.or_maxwellian(self.ptr, _d(np.ascontiguousarray(W, float)), _d(h), _d(b))
        return h, b

    def moments(self, h, b):
        W = self._z(self.ncell, self.nw); q = self._z(self.ncell, self.dim)
        self.L.or_moments(self.ptr, _d(h), _d(b), _d(W), _d(q))
        return W, q

    def heatflux(self, h, b, W):
        q = self._z(self.ncell, self.dim)
        self.L.or_heatflux(self.ptr, _d(h), _d(b), _d(np.ascontiguousarray(W, float)), _d(q))
        return q

    def timesteps(self):
        dtp = self._z(self.ncell)
        dts = self.L.or_timesteps(self.ptr, _d(dtp))
        if self.tangent:
            return (dts.v, dts.d), dtp
        return dts, dtp

    def flux(self, dts, h, b, W, q):
        z = self._z
        Dh = z(self.ncell, self.nv); Db = z(self.ncell, self.nv)
        F = z(max(self.nface, 1), self.nw); wall = z(max(self.nface, 1), 1 + self.nw)
        self.L.or_flux(self.ptr, self._s(dts), _d(h), _d(b), _d(W), _d(q), _d(Dh), _d(Db), _d(F), _d(wall))
        return Dh, Db, F, wall

    def wall_loads(self, F):
        """(face_out [nface][dim+3], side_out [nblock][4][4]) from a face
        macro flux F [nface][nw] (oracle face order)."""
        fo = self._z(max(self.nface, 1), self.dim + 3)
        so = self._z(len(self.case.blocks), 4, 4)
        self.L.or_wall_loads(self.ptr, _d(np.ascontiguousarray(F)), _d(fo), _d(so))
        return fo[:self.nface], so

    def newton_euler(self, blk, body, dt, F, pose):
        """The block's pose [6] advanced by one Newton-Euler step from the
        wall loads of F (oracle face order) and the external load in body =
        (m, I, Fx_ext, Fy_ext, M_ext); returns the new pose."""
        assert not self.tangent
        p = np.array(pose, dtype=np.float64)
        bd = np.array(body, dtype=np.float64)
        self.L.or_newton_euler(self.ptr, int(blk), _d(bd), float(dt), _d(np.ascontiguousarray(F)), _d(p))
        return p

    def interp(self, h, b, W, q):
        self.L.or_interp(self.ptr, _d(h), _d(b), _d(W), _d(q))

    def begin_step(self, dt, dts, h, b, W, q):
        Sh = np.zeros_like(h); Sb = np.zeros_like(b); Fn = self._z(max(self.nface, 1), self.nw)
        self.L.or_begin_step(self.ptr, self._s(dt), self._s(dts), _d(h), _d(b), _d(W), _d(q),
                             _d(Sh), _d(Sb), _d(Fn))
        return Sh, Sb, Fn

    def begin_step_cells(self, dt, dts, h, b, W, q, cells):
        """Steps 1-2 at the listed cells only (h, b, W, q interpolated in
        place over the whole field as in begin_step): rows of Sh and Sb
        [ns][nv] and the macro flux of each face slot of each cell
        [ns][4][nw]."""
        cells = np.ascontiguousarray(cells, dtype=np.int32)
        ns = len(cells)
        Sh = self._z(max(ns, 1), self.nv); Sb = self._z(max(ns, 1), self.nv)
        Fc = self._z(max(ns, 1), 4, self.nw)
        self.L.or_begin_step_cells(self.ptr, self._s(dt), self._s(dts), _d(h), _d(b), _d(W), _d(q), ns,
                                   _i(cells), _d(Sh), _d(Sb), _d(Fc))
        return Sh[:ns], Sb[:ns], Fc[:ns]

    def pseudo_step(self, dt, dts, dtp, h, b, W, Wn, q, Sh, Sb, Fn, F=None):
        """One inner iteration in place; F (optional, [nface][nw]) receives the
        face macro flux of Step 3."""
        resid = self._z(self.nw)
        self.L.or_pseudo_step(self.ptr, self._s(dt), self._s(dts), _d(dtp), _d(h), _d(b), _d(W), _d(Wn),
                              _d(q), _d(Sh), _d(Sb), _d(Fn), _d(resid), _d(F))
        return resid

    def macro_lusgs(self, dt, dtp, W, Wn, F, Fn):
        Wp = np.zeros_like(W); resid = self._z(self.nw)
        self.L.or_macro_lusgs(self.ptr, self._s(dt), _d(dtp), _d(W), _d(Wn), _d(F), _d(Fn), _d(Wp), _d(resid))
        return Wp, resid

    def micro_lusgs(self, dt, dtp, Wp, qp, h, b, Sh, Sb, Dh, Db):
        self.L.or_micro_lusgs(self.ptr, self._s(dt), _d(dtp), _d(Wp), _d(qp), _d(h), _d(b), _d(Sh), _d(Sb),
                              _d(Dh), _d(Db))

    def step7(self, Wp, h, b):
        W = np.zeros_like(Wp)
        self.L.or_step7(self.ptr, _d(Wp), _d(h), _d(b), _d(W))
        return W

    # drivers ----------------------------------------------------------------
    def init_state(self):
        W = self._in(np.ascontiguousarray(self.case.w_init, dtype=np.float64).copy())
        h, b = self.maxwellian(W)
        q = self.heatflux(h, b, W)
        return h, b, W, q

    def physical_step(self, t, h, b, W, q, n_inner=None):
        """Steps 1-8 of one physical step from t to t + dt (poses at t + dt)."""
        assert not self.tangent
        case = self.case
        dts, dtp = self.timesteps()
        dt = case.dt if case.dt is not None else case.dt_over_dts * dts
        Wn = W.copy()
        Sh, Sb, Fn = self.begin_step(dt, dts, h, b, W, q)
        res = []
        for _ in range(case.n_inner if n_inner is None else n_inner):
            res.append(self.pseudo_step(dt, dts, dtp, h, b, W, Wn, q, Sh, Sb, Fn))
        return dt, np.array(res)
