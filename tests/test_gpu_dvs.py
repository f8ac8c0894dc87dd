"""The HIP path on unstructured velocity meshes (Sec. 2.1: V_k is the volume
of the k-th velocity cell), through the C ABI, against the FP64 oracle on
the same meshes: polar meshes (annular sectors, turned from ring to ring,
the sector areas as weights; workloads.polar_dvs) and a disk cut out of a
uniform grid.  Velocity counts are not multiples of the kernels' 64-wide
chunks.

FP64: moments, flux (D, face macro flux, wall output) and Steps 1-2 plus
three inner iterations to relative L2 <= 1e-10, with a per-cell bound on
max |f - f_oracle| / max |f_oracle|; FP32 storage to 1e-5.  Also the moving
overset case (interpolation of every velocity), and the errors of a bad
mesh.
"""
import numpy as np
import pytest
import torch

from paper_2604_09984_amd import ugks, workloads as wl
from tests.parity import both, dev, host, rel_l2, say

pytestmark = pytest.mark.gpu


def _disk(n, vmax):
    """Uniform n x n grid on [-vmax, vmax]^2 cut to the disk |v| <= vmax
    (cell areas dv^2)."""
    v = np.linspace(-vmax, vmax, n)
    X, Y = np.meshgrid(v, v)
    keep = np.hypot(X, Y) <= vmax
    dv = v[1] - v[0]
    return X[keep], Y[keep], np.full(int(keep.sum()), dv * dv)


def _cases():
    cyl = wl.with_dvs(wl.cylinder(ni=16, nj=8, nvx=16, vmax=8.0), wl.polar_dvs(9, 20, 8.0))
    cav = wl.with_dvs(wl.cavity(8, 12), wl.polar_dvs(8, 18, 3.6))
    box = wl.with_dvs(wl.periodic_box(2, 8, 6, 10), _disk(15, 5.0))
    mix = wl.periodic_box(2, 7, 9, 10)
    mix.blocks[0].bc = (wl.COPY, wl.FARFIELD, wl.WALL, wl.COPY)
    mix.name = "mixed_box"
    mix = wl.with_dvs(mix, wl.polar_dvs(7, 17, 5.0))
    return [cyl, cav, box, mix]


CASES = _cases()
IDS = [c.name for c in CASES]


def _cell_max_rel(a, b):
    d = np.abs(a - b).max(axis=1)
    m = np.abs(b).max(axis=1)
    return float((d / m).max())


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_dvs_moments_and_flux(case):
    o, s = both(case)
    assert s.nv == o.nv == len(case.dvs[0])
    h, b, W = wl.synthetic_f(case)
    Wo, qo = o.moments(h, b)
    Ws, qs = s.moments(dev(h), dev(b))
    assert rel_l2(host(Ws), Wo) <= 1e-13 and rel_l2(host(qs), qo) <= 1e-12
    q = o.heatflux(h, b, W)
    dts, _ = o.timesteps()
    assert abs(s.timesteps()[0] - dts) <= 1e-14 * dts
    Dho, Dbo, Fo, wo = o.flux(dts, h, b, W, q)
    Dhs, Dbs, Fs, ws = (host(t) for t in s.flux(dts, dev(h), dev(b), dev(W), dev(q)))
    idx = o.product_face_index()
    e = (rel_l2(Dhs, Dho), rel_l2(Dbs, Dbo), rel_l2(Fs[idx], Fo[:o.nface]), rel_l2(ws[idx], wo[:o.nface]))
    say("dvs flux", case.name, o.nv, "velocities: D_h D_b F wall", e)
    assert max(e) <= 1e-10
    s.close()


@pytest.mark.parametrize("prec", [ugks.F64, ugks.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_dvs_physical_step(case, prec):
    o, s = both(case, prec=prec)
    h, b, W = wl.synthetic_f(case, amp=0.02)
    q = o.heatflux(h, b, W)
    dts, dtp = o.timesteps()
    dt = case.dt if case.dt is not None else case.dt_over_dts * dts
    dt_t = torch.float64 if prec == ugks.F64 else torch.float32
    hd, bd, Wd, qd = dev(h, dt_t), dev(b, dt_t), dev(W), dev(q)
    Wn = W.copy()
    Sh, Sb, Fn = o.begin_step(dt, dts, h, b, W, q)
    for _ in range(3):
        o.pseudo_step(dt, dts, dtp, h, b, W, Wn, q, Sh, Sb, Fn)
    Wnd = Wd.clone()
    Shd, Sbd, Fnd = s.begin_step(dt, hd, bd, Wd, qd)
    s.step(dt, 3, hd, bd, Wd, Wnd, qd, Shd, Sbd, Fnd)
    f = o.types() == 1
    hh, bb = host(hd), host(bd)
    e = (rel_l2(hh[f], h[f]), rel_l2(bb[f], b[f]), rel_l2(host(Wd)[f], W[f]))
    c = max(_cell_max_rel(hh[f], h[f]), _cell_max_rel(bb[f], b[f]))
    say("dvs step", case.name, "f64" if prec == ugks.F64 else "f32", "h b W", e, "per-cell max rel", c)
    assert max(e) <= (1e-10 if prec == ugks.F64 else 1e-5)
    assert c <= (1e-12 if prec == ugks.F64 else 1e-4)
    s.close()


def test_dvs_moving_overset():
    case = wl.with_dvs(wl.overset_cylinder(ni_bg=28, nb=20, njb=8, nv=8), wl.polar_dvs(6, 14, 5.0))
    o, s = both(case)
    h, b, W = wl.synthetic_f(case, amp=0.02)
    q = o.heatflux(h, b, W)
    hd, bd, Wd, qd = dev(h), dev(b), dev(W), dev(q)
    t = 0.0
    for n in range(2):
        t += 0.05
        for x in (o, s):
            x.set_poses(case.poses(t))
        assert o.assemble(0, 2)[0] == 0
        s.assemble(0, 2, device=True)
        assert np.array_equal(s.types(), o.types())
        dts, dtp = o.timesteps()
        dt = case.dt_over_dts * dts
        Wn = W.copy()
        Sh, Sb, Fn = o.begin_step(dt, dts, h, b, W, q)
        for _ in range(2):
            o.pseudo_step(dt, dts, dtp, h, b, W, Wn, q, Sh, Sb, Fn)
        Wnd = Wd.clone()
        Shd, Sbd, Fnd = s.begin_step(dt, hd, bd, Wd, qd)
        s.step(dt, 2, hd, bd, Wd, Wnd, qd, Shd, Sbd, Fnd)
    live = o.types() != 0
    e = (rel_l2(host(hd)[live], h[live]), rel_l2(host(bd)[live], b[live]), rel_l2(host(Wd)[live], W[live]))
    say("dvs moving overset h b W", e)
    assert max(e) <= 1e-10
    s.close()


def test_dvs_bad_mesh_rejected():
    vx, vy, w = wl.polar_dvs(3, 6, 2.0)
    w[2] = -1.0
    with pytest.raises(ugks.UgksError, match="-1"):
        ugks.Solver(wl.with_dvs(wl.cavity(4, 4), (vx, vy, w)), ugks.F64)
    sod = wl.sod_1d(ncell=10, nv=9)
    sod.dvs = wl.polar_dvs(3, 6, 2.0)
    with pytest.raises(ugks.UgksError, match="-6"):
        ugks.Solver(sod, ugks.F64)
