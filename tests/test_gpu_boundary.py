"""The library's boundary beyond the step itself, on the GPU through the C ABI:
device-side failure reports (ugks_status, ugks_set_checks), the caller
workspace (ugks_create_with_workspace), the wall loads and their reverse
(ugks_wall_loads, ugks_wall_loads_adjoint) and the parameter cotangents
(ugks_param_bars)."""
import numpy as np
import pytest
import torch

from paper_2604_09984_amd import ugks, workloads as wl
from tests.parity import both, dev, host, rel_l2, say

pytestmark = pytest.mark.gpu


def _stepped(case, s, n_inner=2, h=None):
    """Steps 1-2 and n_inner inner iterations from the synthetic state; returns
    the device state after them."""
    hh, bb, W = wl.synthetic_f(case, amp=0.02)
    hd = dev(hh if h is None else h, s.dtype)
    bd, Wd = dev(bb, s.dtype), dev(W)
    qd = s.heatflux(hd, bd, Wd)
    dts, _ = s.timesteps()
    dt = 10.0 * dts
    Wn = Wd.clone()
    Sh, Sb, Fn = s.begin_step(dt, hd, bd, Wd, qd)
    s.step(dt, n_inner, hd, bd, Wd, Wn, qd, Sh, Sb, Fn)
    return hd, bd, Wd, qd


def test_nonphysical_state_is_reported():
    """A NaN planted in one pair of f reaches W through Step 7: the step
    reports UGKS_E_NONPHYS (synchronising mode), or ugks_status does after an
    asynchronous step; the word is cleared once read."""
    case = wl.cylinder(ni=16, nj=8, nvx=12, vmax=6.0, kn=0.05, mach=1.0)
    s = ugks.Solver(case, ugks.F64)
    h, _, _ = wl.synthetic_f(case, amp=0.02)
    bad = h.copy()
    bad[37, 5] = np.nan
    say("nonphys: clean run")
    _stepped(case, s)
    assert s.status_code() == 0
    say("nonphys: asynchronous, then ugks_status")
    _stepped(case, s, h=bad)
    assert s.status_code() == -4
    assert s.status_code() == 0  # cleared
    say("nonphys: synchronising mode")
    s.set_checks(sync=True)
    with pytest.raises(ugks.UgksError, match="-4"):
        _stepped(case, s, h=bad)
    _stepped(case, s)  # clean again: no error raised
    s.close()


@pytest.mark.parametrize("case", [wl.cylinder(ni=16, nj=64, nvx=16, vmax=6.0, kn=0.05, mach=1.0),
                                  wl.channel(4, 96, 6)], ids=["cylinder64", "channel96"])
def test_micro_wait_limit_is_reported(case):
    """With the bound of the micro sweep's neighbour wait forced to zero
    sleeps from the host, every kernel still ends; a wavefront that finds a
    neighbour behind gives up and the step reports UGKS_E_DEVICE.  A run in
    which no wavefront had to wait must equal the normal run bit for bit, so
    no wrong f is ever returned silently."""
    ref = ugks.Solver(case, ugks.F64)
    h0, b0, W0, _ = _stepped(case, ref)
    s = ugks.Solver(case, ugks.F64)
    kc, rows, depth, fused = s.micro_shape()
    say("wait limit", case.name, "micro shape", kc, rows, depth, fused)
    s.set_checks(sync=False, wait_limit=0)
    h1, b1, W1, _ = _stepped(case, s)
    code = s.status_code()
    say("wait limit 0: status", code)
    if code == 0:
        assert torch.equal(h1, h0) and torch.equal(W1, W0)
    else:
        assert code == -3
    # the default bound again: normal results, no report
    s.set_checks(sync=True, wait_limit=-1)
    h2, b2, W2, _ = _stepped(case, s)
    assert torch.equal(h2, h0) and torch.equal(b2, b0) and torch.equal(W2, W0)
    s.close()
    ref.close()


@pytest.mark.parametrize("prec", [ugks.F64, ugks.F32])
def test_caller_workspace_gives_identical_results(prec):
    """Scratch (and, with "all", the reverse-mode workspace) in the caller's
    buffer: the step equals that of a context with its own allocations bit
    for bit, the flux adjoint to the rounding of its atomic accumulation."""
    case = wl.cylinder(ni=16, nj=8, nvx=12, vmax=6.0, kn=0.05, mach=1.0)
    sb, ab = ugks.workspace_size(case, prec)
    assert sb > 0 and ab > 0
    a = ugks.Solver(case, prec)
    b = ugks.Solver(case, prec, workspace="all")
    ra = _stepped(case, a)
    rb = _stepped(case, b)
    for x, y in zip(ra, rb):
        assert torch.equal(x, y)
    if prec == ugks.F64:
        h, bb, W, q = ra
        dts, _ = a.timesteps()
        Dh = torch.ones_like(h)
        ga = a.flux_adjoint(h, bb, W, q, Dh_bar=Dh)
        gb = b.flux_adjoint(h, bb, W, q, Dh_bar=Dh)
        for x, y in zip(ga, gb):
            assert rel_l2(host(x), host(y)) <= 1e-13
    a.close()
    b.close()


def _load_cases():
    cav = wl.cavity(8, 12, kn=0.1, lid=0.5)
    cyl = wl.cylinder(ni=16, nj=8, nvx=16)
    mov = wl.cylinder(ni=16, nj=6, nvx=12, vmax=6.0, kn=0.02, mach=1.2, r_out=2.0, ratio=1.15)
    mov.name = "moving_cylinder"
    mov.motion = lambda t: [(0.1, 0.03, 0.2, 0.05, 0.03, 0.4)]
    ov = wl.overset_cylinder(ni_bg=28, nb=20, njb=8, nv=8)
    return [cav, cyl, mov, ov]


@pytest.mark.parametrize("case", _load_cases(), ids=lambda c: c.name)
def test_wall_loads_parity_and_transpose(case):
    """Face and side wall loads from the same face macro flux against the
    oracle's or_wall_loads (1e-13), the reverse map against the forward one
    by the dot-product identity (the map is linear in F), and the parameter
    cotangents against sums of the per-face cotangents over each block and
    wall side."""
    say("wall loads", case.name)
    poses = case.poses(0.05) if case.motion is not None else None
    o, s = both(case, poses=poses)
    if case.overset is not None:
        s.assemble(case.overset["wrule"], case.overset["overlap"])
        o.set_types(s.types())
        o.set_overset(*s.overset())
    h, b, W = wl.synthetic_f(case, amp=0.02)
    q = o.heatflux(h, b, W)
    dts, _ = o.timesteps()
    _, _, Fo, _ = o.flux(dts, h, b, W, q)
    idx = o.product_face_index()
    Fs = np.zeros((s.nface, case.nw))
    Fs[idx] = Fo[:o.nface]
    face, side = s.wall_loads(dev(Fs))
    face_o, side_o = o.wall_loads(Fo[:o.nface])
    assert np.abs(host(side) - side_o).max() <= 1e-13 * max(np.abs(side_o).max(), 1e-300)
    fs = host(face)
    assert np.abs(fs[idx] - face_o).max() <= 1e-13 * max(np.abs(face_o).max(), 1e-300)
    rest = np.ones(s.nface, bool)
    rest[idx] = False
    assert np.all(fs[rest] == 0.0)
    # transpose
    rng = np.random.default_rng(4)
    gb_face = rng.standard_normal(fs.shape)
    gb_side = rng.standard_normal((len(case.blocks), 4, 4))
    Fb = host(s.wall_loads_adjoint(dev(gb_face), dev(gb_side)))
    lhs = np.sum(gb_face * fs) + np.sum(gb_side * host(side))
    rhs = np.sum(Fb * Fs)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.abs(Fb * Fs).sum())
    # parameter cotangents: U_bar sums the grid- and wall-velocity entries
    # over a block's faces, rtw_bar the wall RT entries over a wall side's
    fbar = rng.standard_normal((s.nface, 5))
    U, R = s.param_bars(dev(fbar))
    U, R = host(U), host(R)
    f0 = 0
    for bi, B in enumerate(case.blocks):
        fi0, fj0 = f0, f0 + (B.ni + 1) * B.nj
        nf = (B.ni + 1) * B.nj + B.ni * (B.nj + 1)
        sl = slice(f0, f0 + nf)
        want = [fbar[sl, 0].sum() + fbar[sl, 2].sum(), fbar[sl, 1].sum() + fbar[sl, 3].sum()]
        assert np.allclose(U[bi], want, rtol=1e-12, atol=1e-12)
        sides = [fi0 + (B.ni + 1) * np.arange(B.nj), fi0 + B.ni + (B.ni + 1) * np.arange(B.nj),
                 fj0 + np.arange(B.ni), fj0 + B.ni * B.nj + np.arange(B.ni)]
        for sd in range(4):
            want = fbar[sides[sd], 4].sum() if B.bc[sd] == wl.WALL else 0.0
            assert abs(R[bi, sd] - want) <= 1e-12 * max(1.0, np.abs(fbar[sides[sd], 4]).sum())
        f0 += nf
