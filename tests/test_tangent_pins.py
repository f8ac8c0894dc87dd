"""Pins of the oracle's reference gradient (the dual-number tangent build of
the FP64 oracle, test infrastructure for the adjoint).

Independent references: the double build itself (the tangent build's values
must be bit-identical to it), central finite differences of the double build
(with dt, dt_s and dt' held fixed), exact linearity of the maps that are
linear in the distribution, and a high-precision numerical derivative of the
time-integral coefficients of Eq. fullSolution (mpmath).
"""
import ctypes as C

import mpmath
import numpy as np
import pytest

from oracle.oracle import Dual, Oracle, dual, lib
from paper_2604_09984_amd import workloads as wl


def small_cases():
    cav = wl.cavity(5, 8, kn=0.1, lid=0.5)
    cyl = wl.cylinder(ni=12, nj=5, nvx=10, vmax=5.0, kn=0.05, mach=0.6, r_out=1.5, ratio=1.1, dt_over_dts=5.0)
    cyl.name = "moving_cylinder"
    cyl.motion = lambda t: [(0.0, 0.02, 0.1, 0.05, 0.03, 0.2)]
    ov = wl.overset_cylinder(ni_bg=28, nb=20, njb=8, nv=6, kn=0.05)
    ov.motion = lambda t: [(0.0, 0.0, 0.0, 0.0, 0.0, 0.0), (0.0, 0.03, 0.1, 0.02, 0.08, 0.3)]
    return [cav, cyl, ov]


CASES = small_cases()
IDS = [c.name for c in CASES]


def setup(case, tangent=False, dU=None, drt=None):
    """Oracle at the case's pose (optionally with a block velocity and wall RT
    seed in the tangent build), assembled if overset."""
    o = Oracle(case, tangent=tangent)
    poses = case.poses(0.0) if case.motion is not None else [(0.0,) * 6] * len(case.blocks)
    if dU is not None or case.motion is not None:
        ps = []
        for bi, p in enumerate(poses):
            row = list(p)
            if dU is not None and bi == dU[0]:
                if tangent:
                    row = [(x, 0.0) for x in row]
                    row[3] = (p[3], dU[1]); row[4] = (p[4], dU[2])
                else:
                    row[3] += dU[1]; row[4] += dU[2]
            ps.append(row)
        o.set_poses(ps)
    if drt is not None:
        bi, d = drt
        B = case.blocks[bi]
        for side in range(4):
            if B.bc[side] == wl.WALL:
                o.set_wall_rt(bi, side, (B.rtw[side], d) if tangent else B.rtw[side] + d)
    if case.overset is not None:
        ref = Oracle(case)
        ref.set_poses(poses)
        ref.assemble(case.overset["wrule"], case.overset["overlap"])
        o.set_types(ref.types())
        o.set_overset(*ref.overset())
    return o


def base_state(case):
    o = setup(case)
    h, b, W = wl.synthetic_f(case, amp=0.02)
    q = o.heatflux(h, b, W)
    dts, dtp = o.timesteps()
    dt = case.dt if case.dt is not None else case.dt_over_dts * dts
    Wn = W.copy()
    Sh, Sb, Fn = o.begin_step(dt, dts, h, b, W, q)
    o.pseudo_step(dt, dts, dtp, h, b, W, Wn, q, Sh, Sb, Fn)
    return dict(h=h, b=b, W=W, q=q, Wn=Wn, Sh=Sh, Sb=Sb, Fn=Fn, dt=dt, dts=dts, dtp=dtp, live=o.types() != 0)


def run_step(o, st, d=None):
    """One inner iteration from the base state; with the tangent build the
    inputs carry the directions d."""
    d = d or {}
    t = o.tangent
    g = lambda k: dual(st[k], d.get(k)) if t else (st[k] + d.get(k, 0.0)).copy()
    h, b, W, q, Wn, Sh, Sb, Fn = (g(k) for k in ("h", "b", "W", "q", "Wn", "Sh", "Sb", "Fn"))
    F = o._z(max(o.nface, 1), o.case.nw)
    dtp = dual(st["dtp"]) if t else st["dtp"]
    o.pseudo_step(st["dt"], st["dts"], dtp, h, b, W, Wn, q, Sh, Sb, Fn, F)
    return h, b, W, q, F


def directions(case, st, rng):
    m = st["live"][:, None]
    return dict(h=rng.standard_normal(st["h"].shape) * st["h"] * 0.1 * m,
                b=rng.standard_normal(st["b"].shape) * st["b"] * 0.1 * m,
                W=rng.standard_normal(st["W"].shape) * 0.01 * m,
                q=rng.standard_normal(st["q"].shape) * 0.05 * m,
                Wn=rng.standard_normal(st["W"].shape) * 0.01 * m,
                Sh=rng.standard_normal(st["Sh"].shape) * np.abs(st["Sh"]) * 0.1 * m,
                Sb=rng.standard_normal(st["Sb"].shape) * np.abs(st["Sb"]) * 0.1 * m,
                Fn=rng.standard_normal(st["Fn"].shape) * 0.05)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_tangent_values_match_double_build_bitwise(case):
    st = base_state(case)
    o, ot = setup(case), setup(case, tangent=True)
    r0 = run_step(o, st)
    r1 = run_step(ot, st)
    for a, b in zip(r0, r1):
        assert np.array_equal(a, b[..., 0])
    Dh0, Db0, F0, w0 = o.flux(st["dts"], st["h"], st["b"], st["W"], st["q"])
    Dh1, Db1, F1, w1 = ot.flux(st["dts"], dual(st["h"]), dual(st["b"]), dual(st["W"]), dual(st["q"]))
    assert np.array_equal(Dh0, Dh1[..., 0]) and np.array_equal(F0, F1[..., 0]) and np.array_equal(w0, w1[..., 0])


def _fd_check(case, which, eps_rel=1e-6, tol=5e-6):
    st = base_state(case)
    rng = np.random.default_rng(3)
    bi = 1 if case.overset is not None else 0
    if which == "state":
        d = directions(case, st, rng)
        ot = setup(case, tangent=True)
        tl = run_step(ot, st, d)
        fd = [(a - c) / (2 * eps_rel) for a, c in zip(run_step(setup(case), st, {k: eps_rel * v for k, v in d.items()}),
                                                       run_step(setup(case), st, {k: -eps_rel * v for k, v in d.items()}))]
    elif which == "U":
        ot = setup(case, tangent=True, dU=(bi, 1.0, -0.5))
        tl = run_step(ot, st)
        fd = [(a - c) / (2 * eps_rel) for a, c in zip(run_step(setup(case, dU=(bi, eps_rel, -0.5 * eps_rel)), st),
                                                       run_step(setup(case, dU=(bi, -eps_rel, 0.5 * eps_rel)), st))]
    else:
        ot = setup(case, tangent=True, drt=(bi, 1.0))
        tl = run_step(ot, st)
        fd = [(a - c) / (2 * eps_rel) for a, c in zip(run_step(setup(case, drt=(bi, eps_rel)), st),
                                                       run_step(setup(case, drt=(bi, -eps_rel)), st))]
    for name, a, f in zip(("h", "b", "W", "q", "F"), tl, fd):
        t = a[..., 1]
        nrm = np.linalg.norm(t)
        err = np.linalg.norm(t - f) / max(nrm, 1e-300)
        assert nrm > 0 and err <= tol, (which, name, err)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_tangent_state_direction_matches_finite_differences(case):
    _fd_check(case, "state")


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_tangent_block_velocity_matches_finite_differences(case):
    _fd_check(case, "U")


@pytest.mark.parametrize("case", CASES[:2], ids=IDS[:2])
def test_tangent_wall_temperature_matches_finite_differences(case):
    _fd_check(case, "T")


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_tangent_of_micro_lusgs_is_its_exact_increment(case):
    """Steps 5-6 are linear in (f, S, D) for a fixed (W~, q~): the tangent
    equals the exact difference of two double-build solves."""
    st = base_state(case)
    rng = np.random.default_rng(9)
    o, ot = setup(case), setup(case, tangent=True)
    Wp, qp = st["W"], st["q"]
    Dh = rng.standard_normal(st["h"].shape) * 0.01
    Db = rng.standard_normal(st["b"].shape) * 0.01
    d = directions(case, st, rng)
    dD = rng.standard_normal(Dh.shape) * 0.01
    h0, b0 = st["h"].copy(), st["b"].copy()
    o.micro_lusgs(st["dt"], st["dtp"], Wp, qp, h0, b0, st["Sh"], st["Sb"], Dh, Db)
    h1, b1 = st["h"] + d["h"], st["b"] + d["b"]
    o.micro_lusgs(st["dt"], st["dtp"], Wp, qp, h1, b1, st["Sh"] + d["Sh"], st["Sb"] + d["Sb"], Dh + dD, Db)
    ht, bt = dual(st["h"], d["h"]), dual(st["b"], d["b"])
    ot.micro_lusgs((st["dt"], 0.0), dual(st["dtp"]), dual(Wp), dual(qp), ht, bt, dual(st["Sh"], d["Sh"]),
                   dual(st["Sb"], d["Sb"]), dual(Dh, dD), dual(Db))
    ref = np.concatenate([(h1 - h0).ravel(), (b1 - b0).ravel()])
    got = np.concatenate([ht[..., 1].ravel(), bt[..., 1].ravel()])
    assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)


def test_tangent_of_time_coefficients_against_mpmath():
    """d q_i / d tau of Eq. fullSolution's time integrals, both branches
    (Taylor series for dt_s/tau < 1, closed forms above)."""
    L = lib(True)
    dts = 0.37
    for tau in (0.05, 0.2, 0.37, 0.9, 3.0, 40.0):
        q = (Dual * 5)()
        L.or_time_coeffs(Dual(dts, 0.0), Dual(tau, 1.0), C.cast(q, C.POINTER(C.c_double)))
        mpmath.mp.dps = 40
        x = lambda t: mpmath.mpf(dts) / t
        e = lambda t: mpmath.exp(-x(t))
        ref = [lambda t: t * (1 - e(t)),
               lambda t: t * t * (-1 + (1 + x(t)) * e(t)),
               lambda t: dts - t * (1 - e(t)),
               lambda t: t * t * (2 - x(t) - (2 + x(t)) * e(t)),
               lambda t: t * t * (x(t) ** 2 / 2 - x(t) + 1 - e(t))]
        for i in range(5):
            dref = float(mpmath.diff(ref[i], mpmath.mpf(tau)))
            assert abs(q[i].d - dref) <= 1e-12 * max(abs(dref), 1e-8), (tau, i, q[i].d, dref)
