"""Overset assembly and moving-overset physical steps of the HIP path
(through the C ABI) against the oracle.

Assembly (host code of the library): cell kinds, receptors and donor
indices bit-exact, weights to 1e-15.  Physical steps with the meshes
re-assembled at every step: relative L2 <= 1e-10 over the non-hole cells
(FP64), 1e-5 (FP32 storage), and per cell (receptors and refilled cells
included) max |f - f_oracle| / max |f_oracle| <= 1e-12 (FP64), 1e-4 (FP32).
"""
import numpy as np
import pytest
import torch

from paper_2604_09984_amd import ugks, workloads as wl
from tests.parity import cell_max_rel, both, dev, host, rel_l2, say

pytestmark = pytest.mark.gpu

OV_CASES = [
    ("patch_idw", lambda: wl.overset_patch(ni_bg=16, npatch=14, half=0.55, nv=8, wrule=0)),
    ("patch_bilinear", lambda: wl.overset_patch(ni_bg=16, npatch=14, half=0.55, nv=8, wrule=1)),
    ("cyl_idw", lambda: wl.overset_cylinder(ni_bg=28, nb=20, njb=8, nv=8, wrule=0)),
    ("cyl_bilinear", lambda: wl.overset_cylinder(ni_bg=28, nb=20, njb=8, nv=8, wrule=1)),
    ("cyl_default", lambda: wl.overset_cylinder(nv=8)),
]


def _same_tables(o, s):
    assert np.array_equal(s.types(), o.types())
    orec, optr, odon, ow = o.overset()
    srec, sptr, sdon, sw = s.overset()
    assert np.array_equal(srec, orec) and np.array_equal(sptr, optr) and np.array_equal(sdon, odon)
    assert np.abs(sw - ow).max(initial=0.0) <= 1e-15


@pytest.mark.parametrize("name,mk", OV_CASES, ids=[c[0] for c in OV_CASES])
def test_assembly_parity(name, mk):
    case = mk()
    say("assembly", name, case.ncell)
    o, s = both(case)
    for t in (0.0, 0.37, 1.3):
        poses = case.poses(t)
        o.set_poses(poses)
        s.set_poses(poses)
        rc, n_o = o.assemble(case.overset["wrule"], case.overset["overlap"])
        assert rc == 0
        n_s = s.assemble(case.overset["wrule"], case.overset["overlap"])
        assert n_s == n_o
        _same_tables(o, s)
    s.close()


def test_assembly_errors():
    case = wl.overset_patch(ni_bg=16, npatch=14, half=0.55, nv=4)
    o, s = both(case)
    with pytest.raises(ugks.UgksError):
        s.assemble(2, 2)  # wrule
    with pytest.raises(ugks.UgksError):
        s.assemble(0, -1)  # overlap
    assert s.assemble(0, 2) > 0
    before = s.types()
    # the patch moved out of the box: its fringe has no donor, nothing installed
    s.set_poses([(0.0,) * 6, (5.0, 0.0, 0.0, 0.0, 0.0, 0.0)])
    with pytest.raises(ugks.UgksError, match="-5"):
        s.assemble(0, 2)
    assert np.array_equal(s.types(), before)
    s.close()


def _moving_steps(case, prec, nsteps=2, n_inner=3, jump=None, device=False):
    o, s = both(case, prec=prec)
    h, b, W = wl.synthetic_f(case, amp=0.02)
    q = o.heatflux(h, b, W)
    dt_t = torch.float64 if prec == ugks.F64 else torch.float32
    hd, bd, Wd = dev(h, dt_t), dev(b, dt_t), dev(W)
    qd = dev(q)
    wr, ov = case.overset["wrule"], case.overset["overlap"]
    t = 0.0
    for n in range(nsteps):
        t += case.dt if case.dt is not None else 0.05
        poses = case.poses(t) if jump is None or n == 0 else jump
        if case.motion is not None or jump is not None:
            o.set_poses(poses)
            s.set_poses(poses)
        assert o.assemble(wr, ov)[0] == 0
        s.assemble(wr, ov, device=device)
        _same_tables(o, s)
        dts, dtp = o.timesteps()
        dt = case.dt if case.dt is not None else case.dt_over_dts * dts
        Wn = W.copy()
        Sh, Sb, Fn = o.begin_step(dt, dts, h, b, W, q)
        for _ in range(n_inner):
            o.pseudo_step(dt, dts, dtp, h, b, W, Wn, q, Sh, Sb, Fn)
        Wnd = Wd.clone()
        Shd, Sbd, Fnd = s.begin_step(dt, hd, bd, Wd, qd)
        s.step(dt, n_inner, hd, bd, Wd, Wnd, qd, Shd, Sbd, Fnd)
    live = o.types() != 0
    hh, bb, WW = host(hd), host(bd), host(Wd)
    e = (rel_l2(hh[live], h[live]), rel_l2(bb[live], b[live]), rel_l2(WW[live], W[live]))
    # per cell (receptors and refilled cells included): max |f - f_oracle| /
    # max |f_oracle| within the cell
    c = max(cell_max_rel(hh, h, live), cell_max_rel(bb, b, live), cell_max_rel(WW, W, live))
    say("  per-cell max rel", c)
    s.close()
    return e, c


@pytest.mark.parametrize("name,mk", OV_CASES[:4], ids=[c[0] for c in OV_CASES[:4]])
def test_moving_overset_steps(name, mk):
    case = mk()
    say("moving overset", name)
    e, c = _moving_steps(case, ugks.F64)
    say("  h b W", e)
    assert max(e) <= 1e-10 and c <= 1e-12


def test_static_overset_steps():
    """The cylinder overset case at rest (assembly once)."""
    case = wl.overset_cylinder(ni_bg=28, nb=20, njb=8, nv=8)
    case.motion = None
    e, c = _moving_steps(case, ugks.F64, nsteps=1)
    say("static overset h b W", e)
    assert max(e) <= 1e-10 and c <= 1e-12


def test_moving_overset_refill():
    """A jump of the patch uncovers hole cells straight into field cells,
    which the next begin_step fills by the donor rule on both sides."""
    case = wl.overset_patch(ni_bg=16, npatch=14, half=0.55, nv=8)
    jump = [(0.0,) * 6, (0.18, 0.3, 0.09, 0.0, 0.0, 0.0)]
    e, c = _moving_steps(case, ugks.F64, nsteps=2, jump=jump)
    say("refill h b W", e)
    assert max(e) <= 1e-10 and c <= 1e-12


@pytest.mark.parametrize("name,mk", [OV_CASES[0], OV_CASES[3]], ids=[OV_CASES[0][0], OV_CASES[3][0]])
def test_moving_overset_steps_f32(name, mk):
    case = mk()
    e, c = _moving_steps(case, ugks.F32)
    say("f32 moving overset", name, e)
    assert max(e) <= 1e-5 and c <= 1e-4


# ----------------------------------------------------------------------------
# The assembly on the GPU (overset_assemble_device): the same tables as the
# oracle and, weights included, bit for bit as the host assembly.

def _tables(s):
    return (s.types(), *s.overset())


@pytest.mark.parametrize("name,mk", OV_CASES, ids=[c[0] for c in OV_CASES])
def test_device_assembly_parity(name, mk):
    case = mk()
    o, s = both(case)
    h = ugks.Solver(case, ugks.F64)
    for t in (0.0, 0.37, 1.3):
        poses = case.poses(t)
        for x in (o, s, h):
            x.set_poses(poses)
        rc, n_o = o.assemble(case.overset["wrule"], case.overset["overlap"])
        assert rc == 0
        n_d = s.assemble(case.overset["wrule"], case.overset["overlap"], device=True)
        n_h = h.assemble(case.overset["wrule"], case.overset["overlap"])
        assert n_d == n_o == n_h
        _same_tables(o, s)
        td, th = _tables(s), _tables(h)
        assert all(np.array_equal(a, b) for a, b in zip(td, th))
    s.close()
    h.close()


def test_device_assembly_orphan():
    case = wl.overset_patch(ni_bg=16, npatch=14, half=0.55, nv=4)
    s = ugks.Solver(case, ugks.F64)
    assert s.assemble(0, 2, device=True) > 0
    before = s.types()
    s.set_poses([(0.0,) * 6, (5.0, 0.0, 0.0, 0.0, 0.0, 0.0)])
    with pytest.raises(ugks.UgksError, match="-5"):
        s.assemble(0, 2, device=True)
    assert np.array_equal(s.types(), before)
    with pytest.raises(ugks.UgksError):
        s.assemble(2, 2, device=True)
    s.close()


def test_device_assembly_refill_steps():
    """A jump uncovers hole cells: the device assembly's refill rows drive
    the same moving steps as the oracle's."""
    case = wl.overset_patch(ni_bg=16, npatch=14, half=0.55, nv=8)
    jump = [(0.0,) * 6, (0.18, 0.3, 0.09, 0.0, 0.0, 0.0)]
    e, c = _moving_steps(case, ugks.F64, nsteps=2, jump=jump, device=True)
    say("device assembly, refill h b W", e)
    assert max(e) <= 1e-10 and c <= 1e-12


@pytest.mark.parametrize("mk", [lambda: wl.mems_plate(kn=0.1), lambda: wl.two_body(nv=4)], ids=["mems_plate", "two_body"])
def test_device_assembly_full_size(mk):
    """Full-size meshes (256^2 + 128 x 64; 512 x 256 + 2 x 128 x 96) at a
    moving pose: device tables equal the host's bit for bit; both timed."""
    import time
    case = mk()
    s, h = ugks.Solver(case, ugks.F32), ugks.Solver(case, ugks.F32)
    for t in (0.025, 0.3):
        for x in (s, h):
            x.set_poses(case.poses(t))
        t1 = time.perf_counter()
        n_h = h.assemble(case.overset["wrule"], case.overset["overlap"])
        t2 = time.perf_counter()
        n_d = s.assemble(case.overset["wrule"], case.overset["overlap"], device=True)
        t0 = t1 - (time.perf_counter() - t2)
        td, th = _tables(s), _tables(h)
        say(f"  {case.name} t={t}: {n_d} receptors; device {1e3 * (t1 - t0):.1f} ms, host {1e3 * (t2 - t1):.1f} ms")
        assert n_d == n_h
        assert all(np.array_equal(a, b) for a, b in zip(td, th))
    s.close()
    h.close()
