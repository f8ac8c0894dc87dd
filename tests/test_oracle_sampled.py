"""The oracle's sampled Steps 1-2 (used for parity at sizes where the whole
field is too costly on the CPU) against its full Steps 1-2: the same cells'
rows of S and face fluxes, bit for bit, on a fixed mesh, a moving overset
case and an overset case whose assembly leaves cells to refill."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2604_09984_amd import workloads as wl


def cell_faces(o):
    """[ncell * 4] oracle face of each slot 2 dir + (1 on the cell's + side)
    of each cell, -1 where the slot has no face."""
    g = o.geometry()
    _, dr, _, _ = o.face_ids()
    cf = -np.ones(4 * o.ncell, np.int64)
    for f in range(o.nface):
        if g["fl"][f] >= 0:
            cf[4 * g["fl"][f] + 2 * dr[f] + 1] = f
        if g["fr"][f] >= 0:
            cf[4 * g["fr"][f] + 2 * dr[f]] = f
    return cf


def _check(case, poses=None, prev_poses=None):
    full, samp = Oracle(case), Oracle(case)
    for o in (full, samp):
        if prev_poses is not None:
            o.set_poses(prev_poses)
            assert o.assemble(case.overset["wrule"], case.overset["overlap"])[0] == 0
        if poses is not None:
            o.set_poses(poses)
            assert o.assemble(case.overset["wrule"], case.overset["overlap"])[0] == 0
    nref = full.refill_count()
    h, b, W = wl.synthetic_f(case, amp=0.02)
    q = full.heatflux(h, b, W)
    dts, _ = full.timesteps()
    dt = 10.0 * dts
    x = [a.copy() for a in (h, b, W, q)]
    Sh, Sb, Fn = full.begin_step(dt, dts, h, b, W, q)
    rng = np.random.default_rng(5)
    cells = np.sort(rng.choice(case.ncell, size=min(40, case.ncell), replace=False)).astype(np.int32)
    sh, sb, fc = samp.begin_step_cells(dt, dts, *x, cells)
    assert np.array_equal(sh, Sh[cells]) and np.array_equal(sb, Sb[cells])
    assert np.array_equal(x[0], h) and np.array_equal(x[2], W)  # same interpolation
    cface = cell_faces(full)
    for i, n in enumerate(cells):
        for s in range(4):
            f = cface[4 * n + s]
            want = Fn[f] if f >= 0 else np.zeros(case.nw)
            assert np.array_equal(fc[i, s], want)
    assert full.refill_count() == 0 and samp.refill_count() == 0
    return nref


def test_sampled_fixed_mesh():
    _check(wl.cylinder(ni=16, nj=8, nvx=12))


def test_sampled_moving_overset():
    case = wl.overset_cylinder(ni_bg=28, nb=20, njb=8, nv=8)
    _check(case, poses=case.poses(0.3))


def test_sampled_refill():
    case = wl.overset_patch(ni_bg=16, npatch=14, half=0.55, nv=8)
    nref = _check(case, prev_poses=case.poses(0.0), poses=[(0.0,) * 6, (0.18, 0.3, 0.09, 0.0, 0.0, 0.0)])
    assert nref > 0
