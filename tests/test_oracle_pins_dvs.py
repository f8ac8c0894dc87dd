"""Pins of the oracle on an unstructured velocity mesh (Sec. 2.1: the
quadrature weight V_k of a velocity point is the volume of its cell of the
velocity mesh).  The mesh here is polar: rings of equal width on the disk
|v| <= vmax, sectors turned from ring to ring, a point at the centre of each
annular sector with the sector's area as weight (workloads.polar_dvs).

- the discrete moments of a Maxwellian (density, momentum, energy) converge
  to the continuous ones at the second order of the midpoint rule in the
  radius (the angular sums of a smooth periodic integrand converge far
  faster);
- a uniform resting Maxwellian of a periodic box, on a mesh symmetric under
  v -> -v, is a fixed point of whole physical steps: the face fluxes of
  every velocity telescope whatever the weights, the odd moments (heat
  flux) of f = g(W) vanish, so the Shakhov source is g(W) itself and the
  collision term vanishes (a moving Maxwellian is not: the quadrature's
  error in the heat flux drives a Shakhov correction);
- the micro LU-SGS sweeps solve their factorised system for every velocity
  of the mesh.
"""
import numpy as np
import pytest

from paper_2604_09984_amd import workloads as wl
from tests.test_oracle_pins import _lower_upper, _micro_system


def _box(nr, nth, vmax=6.0, twist=0.5):
    case = wl.periodic_box(2, 6, 5, 8, vmax=vmax)
    return wl.with_dvs(case, wl.polar_dvs(nr, nth, vmax, twist=twist))


def test_polar_mesh_weights_are_sector_areas():
    vx, vy, w = wl.polar_dvs(7, 12, 3.0)
    assert len(w) == 84
    assert abs(w.sum() - np.pi * 9.0) <= 1e-12 * np.pi * 9.0      # the disk's area
    r = np.hypot(vx, vy)
    assert np.allclose(np.unique(np.round(r, 12)), (np.arange(7) + 0.5) * 3.0 / 7)


def test_maxwellian_moments_converge_at_second_order(oracle_lib):
    """W of the discrete reduced Maxwellian of (rho, U, RT) against the
    exact (rho, rho U, rho E): the error falls by about 4 when the ring
    width halves."""
    rho, u, rt = 1.2, np.array([0.4, -0.3]), 0.55
    Wx = wl.cons(2, rho, u, rt)
    errs = []
    for nr in (16, 32, 64):
        case = _box(nr, 48, vmax=7.0)
        o = oracle_lib.Oracle(case)
        W = np.tile(Wx, (o.ncell, 1))
        h, b = o.maxwellian(W)
        Wd, _ = o.moments(h, b)
        errs.append(np.abs(Wd[0] - Wx).max() / np.abs(Wx).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0, errs
    assert errs[-1] < 1e-3, errs


def test_uniform_maxwellian_is_a_fixed_point(oracle_lib):
    case = _box(10, 24, twist=0.0)
    case.w_init = np.tile(wl.cons(2, 1.1, [0.0, 0.0], 0.5), (case.ncell, 1))
    o = oracle_lib.Oracle(case)
    h, b, W, q = o.init_state()
    h0, b0, W0 = h.copy(), b.copy(), W.copy()
    o.physical_step(0.0, h, b, W, q, n_inner=3)
    assert np.abs(h - h0).max() <= 1e-13 * h0.max()
    assert np.abs(b - b0).max() <= 1e-13 * b0.max()
    assert np.abs(W - W0).max() <= 1e-13 * np.abs(W0).max()


def test_micro_lusgs_on_polar_mesh(oracle_lib):
    case = wl.with_dvs(wl.cavity(5, 4), wl.polar_dvs(4, 10, 3.5))
    case.mu_ref = 0.0
    o = oracle_lib.Oracle(case)
    assert o.nv == 40
    rng = np.random.default_rng(12)
    h = rng.uniform(0.5, 1.5, size=(o.ncell, o.nv))
    b = rng.uniform(0.5, 1.5, size=(o.ncell, o.nv))
    Sh = rng.normal(size=(o.ncell, o.nv)); Sb = rng.normal(size=(o.ncell, o.nv))
    Dh = rng.normal(size=(o.ncell, o.nv)); Db = rng.normal(size=(o.ncell, o.nv))
    W = np.tile(case.winf, (o.ncell, 1))
    qp = np.zeros((o.ncell, 2))
    dts, dtp = o.timesteps()
    dt = 0.05
    hs = h.copy()
    hn = h.copy(); bn = b.copy()
    o.micro_lusgs(dt, dtp, W, qp, hn, bn, Sh, Sb, Dh, Db)
    for k in range(o.nv):
        A = _micro_system(o, dt, dtp, k)
        r = Sh[:, k] - hs[:, k] / dt + 0.5 * Dh[:, k]
        Dg, Lw, Up = _lower_upper(A)
        df = hn[:, k] - hs[:, k]
        lhs = (Dg + Lw) @ np.linalg.solve(Dg, (Dg + Up) @ df)
        assert np.allclose(lhs, r, rtol=1e-12, atol=1e-12 * np.abs(r).max())


def test_rejects_bad_mesh(oracle_lib):
    vx, vy, w = wl.polar_dvs(3, 6, 2.0)
    w[4] = 0.0
    with pytest.raises(ValueError):
        oracle_lib.Oracle(wl.with_dvs(wl.cavity(4, 4), (vx, vy, w)))
