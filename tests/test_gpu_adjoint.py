"""Parity of the hand-written adjoint of the HIP library (reverse mode,
through the C ABI) with the oracle's reference gradient, and with central
finite differences of the HIP forward path.

The reference gradient is the dual-number (forward-mode) build of the FP64
oracle: for random input directions v and random output cotangents y it
gives y . (J v) exactly up to rounding, and the adjoint gives (J^T y) . v.
The two must agree to rounding level (relative 1e-9 here; observed 1e-16 to
4e-14).
Element by element, the full gradient of y . Phi with respect to sampled
inputs is compared to oracle Jacobian-vector products along unit vectors.

Directions cover the distribution (h, b), W, q, the dual-time inputs (Wn,
S, Fn), the rigid velocity of a block (the face grid velocity and the wall
velocity of its faces) and the wall temperature.  dt, dt_s and dt' are held
fixed (the oracle gets them as plain inputs).
"""
import numpy as np
import pytest
import torch

from oracle.oracle import Oracle, dual
from paper_2604_09984_amd import ugks, workloads as wl
from tests.parity import dev, host, say

pytestmark = pytest.mark.gpu

TOL = 1e-9


def cases():
    cav = wl.cavity(6, 8, kn=0.1, lid=0.5)
    cyl = wl.cylinder(ni=16, nj=6, nvx=12, vmax=5.0, kn=0.05, mach=0.6, r_out=1.5, ratio=1.1,
                      dt_over_dts=5.0)
    cyl.name = "moving_cylinder"
    cyl.motion = lambda t: [(0.0, 0.02, 0.1, 0.05, 0.03, 0.2)]
    mix = wl.periodic_box(2, 7, 9, 10)
    mix.blocks[0].bc = (wl.COPY, wl.FARFIELD, wl.WALL, wl.COPY)
    mix.name = "mixed_box"
    ov = wl.overset_cylinder(ni_bg=28, nb=20, njb=8, nv=8, kn=0.05)
    ov.motion = lambda t: [(0.0, 0.0, 0.0, 0.0, 0.0, 0.0), (0.0, 0.03, 0.1, 0.02, 0.08, 0.3)]
    return [cav, cyl, mix, ov]


CASES = cases()
IDS = [c.name for c in CASES]


class Setup:
    """Oracle (double and tangent builds) and library on the same case,
    pose and state; maps between the two face numberings."""

    def __init__(self, case, seed=5):
        self.case = case
        self.poses = case.poses(0.0) if case.motion is not None else None
        self.o = Oracle(case)
        self.s = ugks.Solver(case, ugks.F64)
        if self.poses is not None:
            self.o.set_poses(self.poses)
            self.s.set_poses(self.poses)
        if case.overset is not None:
            self.o.assemble(case.overset["wrule"], case.overset["overlap"])
            self.s.assemble(case.overset["wrule"], case.overset["overlap"])
        self.field = self.o.types() == 1
        self.live = self.o.types() != 0
        self.idx = self.o.product_face_index()
        blk, dr, fi, fj = self.o.face_ids()
        self.fblk = np.zeros(self.s.nface, np.int64)
        self.fblk[self.idx] = blk
        h, b, W = wl.synthetic_f(case, seed=seed, amp=0.02)
        q = self.o.heatflux(h, b, W)
        self.dts, self.dtp = self.o.timesteps()
        self.dt = case.dt if case.dt is not None else case.dt_over_dts * self.dts
        # a state inside a physical step: Steps 1-2, then one inner iteration
        self.Wn = W.copy()
        self.Sh, self.Sb, self.Fn = self.o.begin_step(self.dt, self.dts, h, b, W, q)
        self.o.pseudo_step(self.dt, self.dts, self.dtp, h, b, W, self.Wn, q, self.Sh, self.Sb, self.Fn)
        self.h, self.b, self.W, self.q = h, b, W, q
        self.rng = np.random.default_rng(seed + 11)

    # tangent-build oracle at the same pose, with block velocity / wall RT seeds
    def tangent(self, dU=None, drtw=None):
        ot = Oracle(self.case, tangent=True)
        if self.poses is not None or dU is not None:
            poses = [list(p) for p in (self.poses or [(0.0,) * 6] * len(self.case.blocks))]
            tp = []
            for bi, p in enumerate(poses):
                row = [(x, 0.0) for x in p]
                if dU is not None and dU[0] == bi:
                    row[3] = (p[3], dU[1])
                    row[4] = (p[4], dU[2])
                tp.append(row)
            ot.set_poses(tp)
        if drtw is not None:
            bi, d = drtw
            B = self.case.blocks[bi]
            for side in range(4):
                if B.bc[side] == wl.WALL:
                    ot.set_wall_rt(bi, side, (B.rtw[side], d))
        if self.case.overset is not None:
            ot.set_types(self.o.types())
            ot.set_overset(*self.o.overset())
        return ot

    def rand_like(self, a, rel=None, mask=None):
        r = self.rng.standard_normal(a.shape)
        if rel is not None:
            r = r * np.abs(a) * rel
        if mask is not None:
            r = r * mask.reshape((-1,) + (1,) * (a.ndim - 1))
        return r

    def face_param_bars(self, face_bar, blk):
        """Block velocity bar (sum over the block's faces of U_f and wall
        velocity bars) and block wall-RT bar."""
        fb = host(face_bar)
        sel = self.fblk == blk
        return (fb[sel, 0] + fb[sel, 2]).sum(), (fb[sel, 1] + fb[sel, 3]).sum(), fb[sel, 4].sum()


def body_block(case):
    for bi, B in enumerate(case.blocks):
        if any(bc == wl.WALL for bc in B.bc):
            return bi
    return 0


def dot(a, b):
    return float(np.sum(np.asarray(a, dtype=np.float64) * np.asarray(b, dtype=np.float64)))


def check(name, lhs, rhs, tol=TOL):
    rel = abs(lhs - rhs) / max(abs(lhs), abs(rhs), 1e-300)
    say(f"  {name}: oracle J v . y = {lhs:.15e}  adjoint (J^T y) . v = {rhs:.15e}  rel {rel:.2e}")
    assert abs(lhs) > 1e-8, (name, lhs)
    assert rel <= tol, (name, lhs, rhs, rel)


# --------------------------------------------------------------------------
# the flux (Sec. 2.1): (h, b, W, q; U, T_w) -> (Dh, Db, F)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_flux_adjoint_dot(case):
    say("flux adjoint", case.name)
    S = Setup(case)
    bi = body_block(case)
    dh = S.rand_like(S.h, 0.1, S.live); db = S.rand_like(S.b, 0.1, S.live)
    dW = S.rand_like(S.W, 0.01, S.live); dq = S.rand_like(S.q, 0.1, S.live)
    dU = (bi, 0.7, -0.4)
    has_wall = any(bc == wl.WALL for bc in case.blocks[bi].bc)
    drt = (bi, 0.3) if has_wall else None
    ot = S.tangent(dU=dU, drtw=drt)
    Dh, Db, F, _ = ot.flux((S.dts, 0.0), dual(S.h, dh), dual(S.b, db), dual(S.W, dW), dual(S.q, dq))
    yDh = S.rand_like(S.h, None, S.field); yDb = S.rand_like(S.b, None, S.field)
    yF = np.zeros((S.s.nface, case.nw)); yF[S.idx] = S.rng.standard_normal((S.o.nface, case.nw))
    lhs = dot(yDh, Dh[..., 1]) + dot(yDb, Db[..., 1]) + dot(yF[S.idx], F[:S.o.nface, :, 1])
    hb, bb, Wb, qb, fb = S.s.flux_adjoint(dev(S.h), dev(S.b), dev(S.W), dev(S.q), dev(yDh), dev(yDb), dev(yF))
    Ux, Uy, Rt = S.face_param_bars(fb, bi)
    rhs = dot(host(hb), dh) + dot(host(bb), db) + dot(host(Wb), dW) + dot(host(qb), dq) + Ux * dU[1] + Uy * dU[2]
    if drt is not None:
        rhs += Rt * drt[1]
    check("flux", lhs, rhs)


# --------------------------------------------------------------------------
# one inner iteration (Sec. 2.2, Steps 3-7)
# --------------------------------------------------------------------------
def step_dot(S, parts, seed_params=True):
    case = S.case
    bi = body_block(case)
    z = lambda a: np.zeros_like(a)
    d = dict(h=z(S.h), b=z(S.b), W=z(S.W), Wn=z(S.Wn), q=z(S.q), Sh=z(S.Sh), Sb=z(S.Sb), Fn=z(S.Fn))
    if "f" in parts:
        d["h"] = S.rand_like(S.h, 0.1, S.live); d["b"] = S.rand_like(S.b, 0.1, S.live)
    if "W" in parts:
        d["W"] = S.rand_like(S.W, 0.01, S.live); d["q"] = S.rand_like(S.q, 0.1, S.live)
    if "src" in parts:
        d["Wn"] = S.rand_like(S.Wn, 0.01, S.field)
        d["Sh"] = S.rand_like(S.Sh, 0.1, S.field); d["Sb"] = S.rand_like(S.Sb, 0.1, S.field)
        d["Fn"] = np.zeros_like(S.Fn); d["Fn"][:S.o.nface] = S.rng.standard_normal((S.o.nface, case.nw)) * 0.1
    dU = (bi, 0.5, 0.8) if "U" in parts else None
    has_wall = any(bc == wl.WALL for bc in case.blocks[bi].bc)
    drt = (bi, 0.4) if ("T" in parts and has_wall) else None
    ot = S.tangent(dU=dU, drtw=drt)
    hd, bd, Wd, qd = dual(S.h, d["h"]), dual(S.b, d["b"]), dual(S.W, d["W"]), dual(S.q, d["q"])
    Fo = ot._z(max(S.o.nface, 1), case.nw)
    ot.pseudo_step((S.dt, 0.0), (S.dts, 0.0), dual(S.dtp), hd, bd, Wd, dual(S.Wn, d["Wn"]), qd,
                   dual(S.Sh, d["Sh"]), dual(S.Sb, d["Sb"]), dual(S.Fn, d["Fn"]), Fo)
    yh = S.rand_like(S.h, None, S.live); yb = S.rand_like(S.b, None, S.live)
    yW = S.rand_like(S.W, None, S.live); yq = S.rand_like(S.q, None, S.live)
    yF = np.zeros((S.s.nface, case.nw)); yF[S.idx] = S.rng.standard_normal((S.o.nface, case.nw))
    lhs = (dot(yh, hd[..., 1]) + dot(yb, bd[..., 1]) + dot(yW, Wd[..., 1]) + dot(yq, qd[..., 1])
           + dot(yF[S.idx], Fo[:S.o.nface, :, 1]))
    # product face numbering of Fn
    Fn_p = np.zeros((S.s.nface, case.nw)); Fn_p[S.idx] = S.Fn[:S.o.nface]
    out = S.s.step_adjoint(S.dt, dev(S.h), dev(S.b), dev(S.W), dev(S.Wn), dev(S.q), dev(S.Sh), dev(S.Sb),
                           dev(Fn_p), dev(yh), dev(yb), dev(yW), dev(yq), dev(yF))
    hb, bb, Wb, Wnb, qb, Shb, Sbb, Fnb, fb = [host(t) for t in out]
    rhs = (dot(hb, d["h"]) + dot(bb, d["b"]) + dot(Wb, d["W"]) + dot(Wnb, d["Wn"]) + dot(qb, d["q"])
           + dot(Shb, d["Sh"]) + dot(Sbb, d["Sb"]) + dot(Fnb[S.idx], d["Fn"][:S.o.nface]))
    Ux, Uy, Rt = S.face_param_bars(out[8], bi)
    if dU is not None:
        rhs += Ux * dU[1] + Uy * dU[2]
    if drt is not None:
        rhs += Rt * drt[1]
    return lhs, rhs


@pytest.mark.parametrize("case", CASES, ids=IDS)
@pytest.mark.parametrize("parts", ["f", "W", "src", "U", "T", "f+W+src+U+T"])
def test_step_adjoint_dot(case, parts):
    say("step adjoint", case.name, parts)
    S = Setup(case)
    if parts == "T" and not any(bc == wl.WALL for bc in case.blocks[body_block(case)].bc):
        pytest.skip("no wall")
    lhs, rhs = step_dot(S, parts.split("+"))
    check(f"step[{parts}]", lhs, rhs)


# --------------------------------------------------------------------------
# Steps 1-2
# --------------------------------------------------------------------------
@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_begin_step_adjoint_dot(case):
    say("begin-step adjoint", case.name)
    S = Setup(case)
    bi = body_block(case)
    dh = S.rand_like(S.h, 0.1, S.live); db = S.rand_like(S.b, 0.1, S.live)
    dW = S.rand_like(S.W, 0.01, S.live); dq = S.rand_like(S.q, 0.1, S.live)
    dU = (bi, -0.3, 0.6)
    has_wall = any(bc == wl.WALL for bc in case.blocks[bi].bc)
    drt = (bi, 0.5) if has_wall else None
    ot = S.tangent(dU=dU, drtw=drt)
    hd, bd, Wd, qd = dual(S.h, dh), dual(S.b, db), dual(S.W, dW), dual(S.q, dq)
    Sh, Sb, Fn = ot.begin_step((S.dt, 0.0), (S.dts, 0.0), hd, bd, Wd, qd)
    y = dict(h=S.rand_like(S.h, None, S.live), b=S.rand_like(S.b, None, S.live),
             W=S.rand_like(S.W, None, S.live), q=S.rand_like(S.q, None, S.live),
             Sh=S.rand_like(S.h, None, S.field), Sb=S.rand_like(S.b, None, S.field))
    yF = np.zeros((S.s.nface, case.nw)); yF[S.idx] = S.rng.standard_normal((S.o.nface, case.nw))
    lhs = (dot(y["h"], hd[..., 1]) + dot(y["b"], bd[..., 1]) + dot(y["W"], Wd[..., 1]) + dot(y["q"], qd[..., 1])
           + dot(y["Sh"], Sh[..., 1]) + dot(y["Sb"], Sb[..., 1]) + dot(yF[S.idx], Fn[:S.o.nface, :, 1]))
    out = S.s.begin_step_adjoint(S.dt, dev(S.h), dev(S.b), dev(S.W), dev(S.q), dev(y["h"]), dev(y["b"]),
                                 dev(y["W"]), dev(y["q"]), dev(y["Sh"]), dev(y["Sb"]), dev(yF))
    hb, bb, Wb, qb, fb = out
    Ux, Uy, Rt = S.face_param_bars(fb, bi)
    rhs = dot(host(hb), dh) + dot(host(bb), db) + dot(host(Wb), dW) + dot(host(qb), dq) + Ux * dU[1] + Uy * dU[2]
    if drt is not None:
        rhs += Rt * drt[1]
    check("begin", lhs, rhs)


# --------------------------------------------------------------------------
# element by element: gradient of y . Phi for sampled inputs
# --------------------------------------------------------------------------
def test_step_gradient_elements():
    case = CASES[0]
    say("step gradient elements", case.name)
    S = Setup(case)
    yh = S.rand_like(S.h, None, S.live); yb = S.rand_like(S.b, None, S.live)
    yW = S.rand_like(S.W, None, S.live); yq = S.rand_like(S.q, None, S.live)
    yF = np.zeros((S.s.nface, case.nw)); yF[S.idx] = S.rng.standard_normal((S.o.nface, case.nw))
    Fn_p = np.zeros((S.s.nface, case.nw)); Fn_p[S.idx] = S.Fn[:S.o.nface]
    out = S.s.step_adjoint(S.dt, dev(S.h), dev(S.b), dev(S.W), dev(S.Wn), dev(S.q), dev(S.Sh), dev(S.Sb),
                           dev(Fn_p), dev(yh), dev(yb), dev(yW), dev(yq), dev(yF))
    hb, Wb = host(out[0]), host(out[2])
    ot = S.tangent()
    cells = np.flatnonzero(S.field)
    picks = [(int(c), int(k)) for c, k in zip(S.rng.choice(cells, 12), S.rng.integers(0, case.nvx ** 2, 12))]
    for which, (c, k) in [("h", p) for p in picks] + [("W", (int(c), int(m))) for c, m in
                                                       zip(S.rng.choice(cells, 6), S.rng.integers(0, case.nw, 6))]:
        d = {"h": np.zeros_like(S.h), "W": np.zeros_like(S.W)}
        d[which][c, k] = 1.0
        hd, bd, Wd, qd = dual(S.h, d["h"]), dual(S.b), dual(S.W, d["W"]), dual(S.q)
        Fo = ot._z(max(S.o.nface, 1), case.nw)
        ot.pseudo_step((S.dt, 0.0), (S.dts, 0.0), dual(S.dtp), hd, bd, Wd, dual(S.Wn), qd, dual(S.Sh),
                       dual(S.Sb), dual(S.Fn), Fo)
        ref = (dot(yh, hd[..., 1]) + dot(yb, bd[..., 1]) + dot(yW, Wd[..., 1]) + dot(yq, qd[..., 1])
               + dot(yF[S.idx], Fo[:S.o.nface, :, 1]))
        got = hb[c, k] if which == "h" else Wb[c, k]
        scale = max(abs(ref), 1e-3 * np.abs(hb if which == "h" else Wb).max())
        say(f"  d/d{which}[{c},{k}]: oracle {ref:.15e} adjoint {got:.15e}")
        assert abs(got - ref) <= 1e-9 * scale


# --------------------------------------------------------------------------
# central differences of the HIP forward path
# --------------------------------------------------------------------------
@pytest.mark.parametrize("case", CASES[:2], ids=IDS[:2])
def test_step_adjoint_finite_difference(case):
    say("step adjoint vs finite differences", case.name)
    S = Setup(case)
    s = S.s
    Fn_p = np.zeros((s.nface, case.nw)); Fn_p[S.idx] = S.Fn[:S.o.nface]
    dh = S.rand_like(S.h, 0.1, S.live); db = S.rand_like(S.b, 0.1, S.live)
    dW = S.rand_like(S.W, 0.01, S.live)
    yh = S.rand_like(S.h, None, S.field); yW = S.rand_like(S.W, None, S.field)
    yF = np.zeros((s.nface, case.nw)); yF[S.idx] = S.rng.standard_normal((S.o.nface, case.nw))

    def J(eps):
        h, b, W, q = dev(S.h + eps * dh), dev(S.b + eps * db), dev(S.W + eps * dW), dev(S.q)
        s.step(S.dt, 1, h, b, W, dev(S.Wn), q, dev(S.Sh), dev(S.Sb), dev(Fn_p))
        F = s.last_flux()
        return dot(yh, host(h)) + dot(yW, host(W)) + dot(yF, host(F))

    eps = 1e-6
    fd = (J(eps) - J(-eps)) / (2 * eps)
    out = s.step_adjoint(S.dt, dev(S.h), dev(S.b), dev(S.W), dev(S.Wn), dev(S.q), dev(S.Sh), dev(S.Sb),
                         dev(Fn_p), dev(yh), None, dev(yW), None, dev(yF))
    ad = dot(host(out[0]), dh) + dot(host(out[1]), db) + dot(host(out[2]), dW)
    rel = abs(fd - ad) / max(abs(ad), 1e-300)
    say(f"  finite difference {fd:.12e} adjoint {ad:.12e} rel {rel:.2e}")
    assert rel <= 1e-6


# --------------------------------------------------------------------------
# Steps 1-2 with the cells uncovered from holes refilled (after a jump)
# --------------------------------------------------------------------------
def test_begin_step_adjoint_with_refill():
    case = wl.overset_patch(ni_bg=16, npatch=14, half=0.55, nv=8)
    say("begin-step adjoint with refill", case.name)
    jump = [(0.0,) * 6, (0.18, 0.3, 0.09, 0.0, 0.0, 0.0)]
    o, ot, s = Oracle(case), Oracle(case, tangent=True), ugks.Solver(case, ugks.F64)
    for x in (o, ot, s):
        x.set_poses(case.poses(0.0))
        x.assemble(0, 2)
        x.set_poses(jump)
        x.assemble(0, 2)
    nrec, nref, pending = s.overset_rows()
    assert nref > 0 and pending == 1 and o.refill_count() == nref
    h, b, W = wl.synthetic_f(case, amp=0.02)
    q = o.heatflux(h, b, W)
    dts, _ = o.timesteps()
    dt = case.dt
    rng = np.random.default_rng(21)
    live = o.types() != 0
    dh = rng.standard_normal(h.shape) * h * 0.1
    db = rng.standard_normal(b.shape) * b * 0.1
    dW = rng.standard_normal(W.shape) * 0.01
    dq = rng.standard_normal(q.shape) * 0.05
    hd, bd, Wd, qd = dual(h, dh), dual(b, db), dual(W, dW), dual(q, dq)
    Sh, Sb, Fn = ot.begin_step((dt, 0.0), (dts, 0.0), hd, bd, Wd, qd)
    idx = o.product_face_index()
    y = {k: rng.standard_normal(a.shape) * live.reshape((-1,) + (1,) * (a.ndim - 1))
         for k, a in (("h", h), ("b", b), ("W", W), ("q", q))}
    field = (o.types() == 1)[:, None]
    ySh = rng.standard_normal(h.shape) * field
    ySb = rng.standard_normal(b.shape) * field
    yF = np.zeros((s.nface, case.nw)); yF[idx] = rng.standard_normal((o.nface, case.nw))
    lhs = (dot(y["h"], hd[..., 1]) + dot(y["b"], bd[..., 1]) + dot(y["W"], Wd[..., 1]) + dot(y["q"], qd[..., 1])
           + dot(ySh, Sh[..., 1]) + dot(ySb, Sb[..., 1]) + dot(yF[idx], Fn[:o.nface, :, 1]))
    out = s.begin_step_adjoint(dt, dev(h), dev(b), dev(W), dev(q), dev(y["h"]), dev(y["b"]), dev(y["W"]),
                               dev(y["q"]), dev(ySh), dev(ySb), dev(yF), refill=True)
    rhs = dot(host(out[0]), dh) + dot(host(out[1]), db) + dot(host(out[2]), dW) + dot(host(out[3]), dq)
    check("begin with refill", lhs, rhs)
