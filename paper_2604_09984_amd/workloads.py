"""Seeded synthetic inputs shaped like the paper's workloads.

This module is the only code the oracle and the HIP path both use.  It holds
no arithmetic of the method: it builds structured meshes (node coordinates,
boundary kinds), uniform velocity points, gas parameters, initial
macroscopic states, prescribed rigid-body poses and positive synthetic
distributions.  Quadrature weights, geometry, equilibria, fluxes and the
dual-time solver are computed independently on each side.

Units: rho_ref = 1, RT_ref = 1/2 (so sqrt(2 RT_ref) = 1), L_ref = 1, unless a
case says otherwise.  Seeds derive from 260409984.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np

SEED = 260409984

# boundary kinds of a block side (values are part of both C interfaces)
PERIODIC, FARFIELD, COPY, WALL, NONE = 0, 1, 2, 3, 4
# cell kinds
HOLE, FIELD, RECEPTOR = 0, 1, 2


@dataclass
class Block:
    ni: int
    nj: int
    bc: Sequence[int]                 # i-min, i-max, j-min, j-max
    x: np.ndarray                     # nodes, shape (nj+1, ni+1) (1D: (ni+1,))
    y: Optional[np.ndarray] = None
    rtw: Sequence[float] = (0.5, 0.5, 0.5, 0.5)   # wall RT per side
    vwx: Sequence[float] = (0.0, 0.0, 0.0, 0.0)   # wall velocity beyond the mesh's
    vwy: Sequence[float] = (0.0, 0.0, 0.0, 0.0)
    xc0: float = 0.0                  # rotation centre, reference pose
    yc0: float = 0.0
    body: bool = False                # body-fitted block (walls on j-min)

    @property
    def ncell(self) -> int:
        return self.ni * self.nj


@dataclass
class Case:
    name: str
    dim: int
    pr: float
    omega: float
    mu_ref: float          # tau = mu_ref (RT/rt_ref)^omega / p ; <= 0: collisionless
    rt_ref: float
    vx: np.ndarray         # velocity points per axis
    vy: np.ndarray
    vrange: Sequence[float]
    winf: np.ndarray       # far-field conservative state
    blocks: List[Block]
    w_init: np.ndarray     # [ncell, dim+2]
    cfl_s: float = 0.5
    cfl_p: float = 100.0
    dt: Optional[float] = None          # physical step, absolute ...
    dt_over_dts: Optional[float] = None  # ... or as a multiple of dt_s
    n_inner: int = 10
    n_phys: int = 1
    motion: Optional[Callable[[float], list]] = None  # t -> [(dx,dy,th,ux,uy,om)] per block
    overset: Optional[dict] = None      # {"wrule": 0|1, "overlap": int}
    notes: str = ""
    # unstructured velocity mesh (2D): (vx_k, vy_k, area_k) of every point;
    # vx then holds vx_k and vy = [0] so that nvx = nv, nvy = 1
    dvs: Optional[tuple] = None

    @property
    def nvx(self) -> int:
        return len(self.vx)

    @property
    def nvy(self) -> int:
        return len(self.vy) if self.dim == 2 else 1

    @property
    def nv(self) -> int:
        return self.nvx * self.nvy

    @property
    def nw(self) -> int:
        return self.dim + 2

    @property
    def ncell(self) -> int:
        return sum(b.ncell for b in self.blocks)

    def poses(self, t: float) -> list:
        if self.motion is None:
            return [(0.0, 0.0, 0.0, 0.0, 0.0, 0.0)] * len(self.blocks)
        return self.motion(t)

    # flat arrays for the C interfaces -------------------------------------
    def block_ints(self) -> np.ndarray:
        return np.array([[b.ni, b.nj, *b.bc] for b in self.blocks], dtype=np.int32).ravel()

    def block_dbls(self) -> np.ndarray:
        return np.array([[*b.rtw, *b.vwx, *b.vwy, b.xc0, b.yc0] for b in self.blocks],
                        dtype=np.float64).ravel()

    def node_array(self) -> np.ndarray:
        parts = []
        for b in self.blocks:
            parts.append(np.ascontiguousarray(b.x, dtype=np.float64).ravel())
            if self.dim == 2:
                parts.append(np.ascontiguousarray(b.y, dtype=np.float64).ravel())
        return np.concatenate(parts)

    def node_centres(self) -> np.ndarray:
        """Mean of each cell's corner nodes (used only to lay out initial data)."""
        out = []
        for b in self.blocks:
            if self.dim == 1:
                xc = 0.5 * (b.x[:-1] + b.x[1:])
                out.append(np.stack([xc, np.zeros_like(xc)], 1))
            else:
                xc = 0.25 * (b.x[:-1, :-1] + b.x[:-1, 1:] + b.x[1:, :-1] + b.x[1:, 1:])
                yc = 0.25 * (b.y[:-1, :-1] + b.y[:-1, 1:] + b.y[1:, :-1] + b.y[1:, 1:])
                out.append(np.stack([xc.ravel(), yc.ravel()], 1))
        return np.concatenate(out)


# --------------------------------------------------------------------------
# helpers (problem statement only)
# --------------------------------------------------------------------------
def polar_dvs(nr: int, nth: int, vmax: float, twist: float = 0.5):
    """Polar velocity mesh on the disk |v| <= vmax: nr rings of width
    vmax/nr, nth sectors, a point at the centre of each annular sector
    (radius (m + 1/2) dr; the sectors of ring m turned by twist * m * dth so
    that rings do not line up), its area r dr dth as the weight.  Points in
    ring-major order."""
    dr, dth = vmax / nr, 2.0 * math.pi / nth
    vx, vy, w = [], [], []
    for m in range(nr):
        r = (m + 0.5) * dr
        for n in range(nth):
            th = (n + 0.5 + twist * m) * dth
            vx.append(r * math.cos(th))
            vy.append(r * math.sin(th))
            w.append(r * dr * dth)
    return np.array(vx), np.array(vy), np.array(w)


def with_dvs(case: "Case", dvs) -> "Case":
    """The case on an unstructured velocity mesh dvs = (vx_k, vy_k, area_k)."""
    case.dvs = tuple(np.asarray(a, dtype=np.float64) for a in dvs)
    case.vx = case.dvs[0].copy()
    case.vy = np.zeros(1)
    case.name = case.name + f"_dvs{len(case.dvs[0])}"
    return case


def uniform_points(n: int, a: float, b: float) -> np.ndarray:
    if n == 1:
        return np.zeros(1)
    return np.array([a + (b - a) * i / (n - 1) for i in range(n)], dtype=np.float64)


def mu_ref_from_kn(kn: float, omega: float, rho_ref: float = 1.0, rt_ref: float = 0.5,
                   length: float = 1.0) -> float:
    """Variable-hard-sphere reference viscosity for a Knudsen number
    (Bird's mean-free-path definition): mu = 15 sqrt(2 pi RT) rho lambda / (2(5-2w)(7-2w))."""
    return 15.0 * math.sqrt(2.0 * math.pi * rt_ref) * rho_ref * length * kn / (
        2.0 * (5.0 - 2.0 * omega) * (7.0 - 2.0 * omega))


def cons(dim: int, rho, u, rt) -> np.ndarray:
    """Conservative variables of a monatomic gas (3 translational degrees of freedom)."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    rt = np.asarray(rt, dtype=np.float64)
    ke = 0.5 * rho * np.sum(u[..., :dim] ** 2, axis=-1)
    e = ke + 1.5 * rho * rt
    parts = [rho[..., None], (rho[..., None] * u[..., :dim]), e[..., None]]
    return np.concatenate(parts, axis=-1)


def cartesian_block(ni, nj, x0, x1, y0, y1, bc, **kw) -> Block:
    xs = uniform_points(ni + 1, x0, x1)
    ys = uniform_points(nj + 1, y0, y1)
    X, Y = np.meshgrid(xs, ys)
    return Block(ni, nj, bc, X, Y, **kw)


def line_block(ni, x0, x1, bc) -> Block:
    return Block(ni, 1, bc, uniform_points(ni + 1, x0, x1), None)


def o_block(ni, nj, radii, centre=(0.0, 0.0), bc=(PERIODIC, PERIODIC, WALL, FARFIELD),
            shape=None, **kw) -> Block:
    """O-mesh around a closed body; i runs clockwise (right-handed (i, j)),
    j outward.  `radii` are the nj+1 radial stations (scale factors when a
    body `shape` is given: shape(theta) -> (x, y) of the wall point)."""
    th = np.array([-2.0 * math.pi * i / ni for i in range(ni + 1)])
    X = np.empty((nj + 1, ni + 1))
    Y = np.empty((nj + 1, ni + 1))
    for j, r in enumerate(radii):
        if shape is None:
            X[j] = centre[0] + r * np.cos(th)
            Y[j] = centre[1] + r * np.sin(th)
        else:
            for i, t in enumerate(th):
                px, py = shape(t, r)
                X[j, i] = centre[0] + px
                Y[j, i] = centre[1] + py
    X[:, ni] = X[:, 0]
    Y[:, ni] = Y[:, 0]
    return Block(ni, nj, bc, X, Y, xc0=centre[0], yc0=centre[1], **kw)


def geometric_radii(r0, r1, n, ratio):
    d0 = (r1 - r0) * (ratio - 1.0) / (ratio ** n - 1.0)
    r = [r0]
    for k in range(n):
        r.append(r[-1] + d0 * ratio ** k)
    r[-1] = r1
    return np.array(r)


# --------------------------------------------------------------------------
# synthetic states
# --------------------------------------------------------------------------
def smooth_state(case: Case, seed: int = SEED, amp: float = 0.1) -> np.ndarray:
    """Smooth positive macroscopic field: a random low-order Fourier perturbation
    of the far-field state."""
    rng = np.random.default_rng(seed)
    xc = case.node_centres()
    rho0 = case.winf[0]
    u0 = case.winf[1:1 + case.dim] / rho0
    rt0 = (case.winf[-1] - 0.5 * rho0 * np.sum(u0 ** 2)) / (1.5 * rho0)
    k = rng.uniform(0.5, 2.0, size=(4, 2)) * 2 * math.pi
    ph = rng.uniform(0, 2 * math.pi, size=4)
    w = [np.sin(xc[:, 0] * k[m, 0] + xc[:, 1] * k[m, 1] + ph[m]) for m in range(4)]
    rho = rho0 * (1 + amp * w[0])
    rt = rt0 * (1 + amp * w[1])
    u = np.zeros((len(xc), 2))
    u[:, 0] = u0[0] + amp * math.sqrt(2 * rt0) * w[2]
    if case.dim == 2:
        u[:, 1] = u0[1] + amp * math.sqrt(2 * rt0) * w[3]
    return cons(case.dim, rho, u, rt)


def synthetic_f(case: Case, seed: int = SEED, amp: float = 0.05):
    """Positive smooth synthetic reduced distributions (h, b), shape [ncell, nv],
    not an equilibrium: a skewed Gaussian bump per cell with a smooth
    velocity-space ripple.  Used to exercise every term at arbitrary states."""
    rng = np.random.default_rng(seed + 1)
    W = smooth_state(case, seed)
    rho = W[:, 0]
    u = np.zeros((case.ncell, 2))
    u[:, :case.dim] = W[:, 1:1 + case.dim] / rho[:, None]
    rt = (W[:, -1] - 0.5 * rho * np.sum(u ** 2, 1)) / (1.5 * rho)
    if case.dvs is not None:
        vx, vy = case.dvs[0][None, :], case.dvs[1][None, :]
    else:
        VX, VY = np.meshgrid(case.vx, case.vy if case.dim == 2 else np.zeros(1))
        vx = VX.ravel()[None, :]
        vy = VY.ravel()[None, :]
    a1 = rng.uniform(-1, 1, size=(case.ncell, 1))
    a2 = rng.uniform(-1, 1, size=(case.ncell, 1))
    nxi = 3 - case.dim
    h = np.empty((case.ncell, vx.shape[1]))
    b = np.empty_like(h)
    rows = max(1, (1 << 20) // vx.shape[1])  # bounded temporaries for large cases

    def fill(r0):
        c = slice(r0, r0 + rows)
        s = 1.0 / (2.0 * rt[c, None])
        uc = u[c]
        r2 = (vx - uc[:, 0:1]) ** 2 + ((vy - uc[:, 1:2]) ** 2 if case.dim == 2 else 0.0)
        base = rho[c, None] * (s / math.pi) ** (case.dim / 2) * np.exp(-s * r2)
        rip = 1 + amp * np.tanh(a1[c] * (vx - uc[:, 0:1]) + a2[c] * (vy - uc[:, 1:2]))
        h[c] = base * rip
        b[c] = h[c] * (nxi * rt[c, None]) * (1 + 0.5 * amp * np.cos(a2[c] * vx + a1[c] * vy))

    starts = range(0, case.ncell, rows)
    if len(starts) > 1:
        # element-wise work on disjoint rows: threads give the same values
        with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
            list(ex.map(fill, starts))
    else:
        fill(0)
    return h, b, W


# --------------------------------------------------------------------------
# cases
# --------------------------------------------------------------------------
def sod_1d(ncell: int = 200, nv: int = 101, kn: float = 1e-3, dt: float = 1.5e-3,
           n_inner: int = 10, n_phys: int = 100) -> Case:
    """1D Sod-type tube on [0,1]: (rho,p) = (1,1) | (0.125,0.1), zero-gradient
    ends, 101-point grid on [-8,8], Kn referred to the left state (RT = 1)."""
    blk = line_block(ncell, 0.0, 1.0, (COPY, COPY, NONE, NONE))
    case = Case("sod1d", 1, 2.0 / 3.0, 0.5, mu_ref_from_kn(kn, 0.5, 1.0, 1.0), 1.0,
                uniform_points(nv, -8.0, 8.0), np.zeros(1), (-8.0, 8.0, 0.0, 0.0),
                cons(1, 1.0, [0.0], 1.0), [blk], None, dt=dt, n_inner=n_inner, n_phys=n_phys)
    xc = case.node_centres()[:, 0]
    left = xc < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    case.w_init = cons(1, rho, np.zeros((ncell, 1)), p / rho)
    return case


def cylinder(ni: int = 128, nj: int = 64, nvx: int = 64, vmax: float = 15.0, kn: float = 0.01,
             mach: float = 5.0, r_out: float = 8.0, ratio: float = 1.06,
             n_inner: int = 10, n_phys: int = 50, dt_over_dts: float = 20.0,
             start: str = "potential") -> Case:
    """Ma 5 flow over a stationary cylinder (diameter 1): O-mesh ni x nj
    (periodic around, geometric radial spacing to r_out), isothermal wall at
    the free-stream temperature, far field outside, hard-sphere gas.
    start = "potential": the initial velocity is the incompressible potential
    flow around the cylinder (no flow through the wall) at the free-stream
    density and temperature; "uniform": an impulsive uniform start."""
    radii = geometric_radii(0.5, r_out, nj, ratio)
    blk = o_block(ni, nj, radii, bc=(PERIODIC, PERIODIC, WALL, FARFIELD),
                  rtw=(0.5, 0.5, 0.5, 0.5), body=True)
    rt = 0.5
    u = mach * math.sqrt(5.0 / 3.0 * rt)
    winf = cons(2, 1.0, [u, 0.0], rt)
    v = uniform_points(nvx, -vmax, vmax)
    case = Case("cylinder", 2, 2.0 / 3.0, 0.5, mu_ref_from_kn(kn, 0.5), 0.5, v, v.copy(),
                (-vmax, vmax, -vmax, vmax), winf, [blk],
                np.tile(winf, (ni * nj, 1)), dt_over_dts=dt_over_dts,
                n_inner=n_inner, n_phys=n_phys)
    if start == "potential" and mach > 0:
        xc = case.node_centres()
        r2 = np.sum(xc ** 2, 1)
        a2 = 0.25
        ux = u * (1.0 - a2 * (xc[:, 0] ** 2 - xc[:, 1] ** 2) / r2 ** 2)
        uy = u * (-a2 * 2.0 * xc[:, 0] * xc[:, 1] / r2 ** 2)
        case.w_init = cons(2, np.ones(len(xc)), np.stack([ux, uy], 1), np.full(len(xc), rt))
    return case


def periodic_box(dim: int = 2, ni: int = 8, nj: int = 6, nv: int = 12, vmax: float = 5.0,
                 kn: float = 0.05, seed: int = SEED) -> Case:
    """Doubly periodic box (unit cell, slightly skewed nodes) for conservation pins."""
    if dim == 1:
        blk = line_block(ni, 0.0, 1.0, (PERIODIC, PERIODIC, NONE, NONE))
        v = uniform_points(nv, -vmax, vmax)
        case = Case("box1d", 1, 2.0 / 3.0, 0.5, mu_ref_from_kn(kn, 0.5), 0.5, v, np.zeros(1),
                    (-vmax, vmax, 0, 0), cons(1, 1.0, [0.3], 0.5), [blk], None, dt=0.01)
    else:
        blk = cartesian_block(ni, nj, 0.0, 1.0, 0.0, 1.0, (PERIODIC, PERIODIC, PERIODIC, PERIODIC))
        rng = np.random.default_rng(seed + 7)
        # interior node jitter keeps periodic images identical
        jx = rng.uniform(-0.15, 0.15, size=(nj, ni)) / ni
        jy = rng.uniform(-0.15, 0.15, size=(nj, ni)) / nj
        jx = np.pad(jx, ((0, 1), (0, 1)), mode="wrap")
        jy = np.pad(jy, ((0, 1), (0, 1)), mode="wrap")
        blk.x = blk.x + jx
        blk.y = blk.y + jy
        v = uniform_points(nv, -vmax, vmax)
        case = Case("box2d", 2, 2.0 / 3.0, 0.5, mu_ref_from_kn(kn, 0.5), 0.5, v, v.copy(),
                    (-vmax, vmax, -vmax, vmax), cons(2, 1.0, [0.3, -0.2], 0.5), [blk], None,
                    dt=0.01)
    case.w_init = smooth_state(case, seed)
    return case


def cavity(n: int = 16, nv: int = 16, kn: float = 0.1, lid: float = 0.5, periodic_x: bool = False,
           seed: int = SEED) -> Case:
    """Square cavity [0,1]^2 with diffuse walls at RT = 1/2; the top wall moves
    along +x at `lid` (in units of sqrt(2 RT_0)).  periodic_x gives the
    moving-plate (Couette-type) variant."""
    bc = (PERIODIC, PERIODIC, WALL, WALL) if periodic_x else (WALL, WALL, WALL, WALL)
    blk = cartesian_block(n, n, 0.0, 1.0, 0.0, 1.0, bc, vwx=(0.0, 0.0, 0.0, lid))
    vmax = 5.0 * math.sqrt(0.5)
    v = uniform_points(nv, -vmax, vmax)
    winf = cons(2, 1.0, [0.0, 0.0], 0.5)
    return Case("plate" if periodic_x else "cavity", 2, 2.0 / 3.0, 0.5, mu_ref_from_kn(kn, 0.5),
                0.5, v, v.copy(), (-vmax, vmax, -vmax, vmax), winf, [blk],
                np.tile(winf, (n * n, 1)), dt_over_dts=10.0)


def channel(ni: int = 6, nj: int = 70, nv: int = 8, kn: float = 0.1, lid: float = 0.4) -> Case:
    """Periodic channel [0, 1] x [0, nj/ni]: diffuse walls below and above, the
    upper wall moving along +x (a tall block for the sweep variants)."""
    blk = cartesian_block(ni, nj, 0.0, 1.0, 0.0, nj / ni, (PERIODIC, PERIODIC, WALL, WALL),
                          vwx=(0.0, 0.0, 0.0, lid))
    vmax = 5.0 * math.sqrt(0.5)
    v = uniform_points(nv, -vmax, vmax)
    winf = cons(2, 1.0, [0.0, 0.0], 0.5)
    return Case(f"channel{nj}", 2, 2.0 / 3.0, 0.5, mu_ref_from_kn(kn, 0.5), 0.5, v, v.copy(),
                (-vmax, vmax, -vmax, vmax), winf, [blk], np.tile(winf, (ni * nj, 1)), dt_over_dts=10.0)


def overset_patch(ni_bg: int = 32, npatch: int = 16, half: float = 0.5, nv: int = 12, kn: float = 0.1,
                  wrule: int = 0) -> Case:
    """Overset case without walls: a periodic background box [-1, 1]^2 and a
    square patch grid [-half, half]^2 (all four sides overset) translating and
    rotating rigidly over it (free-stream preservation on moving overset
    meshes)."""
    bg = cartesian_block(ni_bg, ni_bg, -1.0, 1.0, -1.0, 1.0, (PERIODIC, PERIODIC, PERIODIC, PERIODIC))
    patch = cartesian_block(npatch, npatch, -half, half, -half, half, (NONE, NONE, NONE, NONE))
    vmax = 4.0
    v = uniform_points(nv, -vmax, vmax)
    winf = cons(2, 1.0, [0.4, 0.1], 0.5)
    ncell = bg.ncell + patch.ncell

    def motion(t):
        return [(0.0, 0.0, 0.0, 0.0, 0.0, 0.0),
                (0.05 * t, 0.02 * t * t, 0.3 * t, 0.05, 0.04 * t, 0.3)]
    return Case("patch", 2, 2.0 / 3.0, 0.5, mu_ref_from_kn(kn, 0.5), 0.5, v, v.copy(),
                (-vmax, vmax, -vmax, vmax), winf, [bg, patch], np.tile(winf, (ncell, 1)),
                dt=0.02, motion=motion, overset={"wrule": wrule, "overlap": 2})


def overset_cylinder(ni_bg: int = 40, nb: int = 40, njb: int = 12, nv: int = 12, kn: float = 0.05,
                     mach: float = 0.5, wrule: int = 0) -> Case:
    """Moving body on an overset mesh: far-field box [-2, 2]^2 and an O-grid
    (diameter 0.5, isothermal wall, outer side overset out to r = 1) that
    plunges and pitches rigidly through a uniform stream."""
    bg = cartesian_block(ni_bg, ni_bg, -2.0, 2.0, -2.0, 2.0, (FARFIELD, FARFIELD, FARFIELD, FARFIELD))
    radii = geometric_radii(0.25, 1.0, njb, 1.08)
    body = o_block(nb, njb, radii, bc=(PERIODIC, PERIODIC, WALL, NONE), rtw=(0.5, 0.5, 0.55, 0.5),
                   body=True)
    vmax = 5.0
    v = uniform_points(nv, -vmax, vmax)
    u = mach * math.sqrt(5.0 / 3.0 * 0.5)
    winf = cons(2, 1.0, [u, 0.0], 0.5)
    ncell = bg.ncell + body.ncell

    def motion(t):
        # plunge y = 0.1 sin(2 pi t / 2), pitch 0.2 sin(2 pi t / 2)
        w = math.pi
        return [(0.0, 0.0, 0.0, 0.0, 0.0, 0.0),
                (0.0, 0.1 * math.sin(w * t), 0.2 * math.sin(w * t), 0.0, 0.1 * w * math.cos(w * t),
                 0.2 * w * math.cos(w * t))]
    return Case("ovcyl", 2, 2.0 / 3.0, 0.5, mu_ref_from_kn(kn, 0.5), 0.5, v, v.copy(),
                (-vmax, vmax, -vmax, vmax), winf, [bg, body], np.tile(winf, (ncell, 1)),
                dt_over_dts=5.0, motion=motion, overset={"wrule": wrule, "overlap": 2})


def rounded_rect_point(phi: float, a: float, b: float, d: float) -> tuple:
    """Point at polar angle phi on the boundary of the set of points within
    distance d of the rectangle [-a, a] x [-b, b] (bisection along the ray)."""
    ux, uy = math.cos(phi), math.sin(phi)
    lo, hi = 0.0, a + b + d + 1.0
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        px, py = mid * ux, mid * uy
        dist = math.hypot(max(abs(px) - a, 0.0), max(abs(py) - b, 0.0))
        if dist > d:
            hi = mid
        else:
            lo = mid
    return lo * ux, lo * uy


def mems_plate(n_bg: int = 256, ni: int = 128, nj: int = 64, nv: int = 48, kn: float = 0.1,
               wrule: int = 1) -> Case:
    """Thermal MEMS plate: a 1 x 0.1 plate, 10 % hotter than the gas, heaving
    as y = 0.2 sin(2 pi t / T) (T = 10) inside a closed box [-2, 2]^2 with
    diffuse walls at T0; background 256 x 256 Cartesian cells, body-fitted
    O-mesh 128 x 64 extending 0.25 from the plate (rays through the points of
    the ellipse of the plate's half-widths, geometric spacing), overset with
    bilinear donors; 48 x 48 velocities on [-6, 6]^2; gas at rest (rho 1,
    RT 1/2); dt = T/400."""
    bg = cartesian_block(n_bg, n_bg, -2.0, 2.0, -2.0, 2.0, (WALL, WALL, WALL, WALL))
    a, bh = 0.5, 0.05
    offs = geometric_radii(0.0, 0.25, nj, 1.05)
    shape = lambda t, r: rounded_rect_point(math.atan2(bh * math.sin(t), a * math.cos(t)), a, bh, r)
    body = o_block(ni, nj, offs, shape=shape, bc=(PERIODIC, PERIODIC, WALL, NONE),
                   rtw=(0.5, 0.5, 0.55, 0.5), body=True)
    v = uniform_points(nv, -6.0, 6.0)
    winf = cons(2, 1.0, [0.0, 0.0], 0.5)
    ncell = bg.ncell + body.ncell
    period = 10.0
    w = 2.0 * math.pi / period

    def motion(t):
        return [(0.0, 0.0, 0.0, 0.0, 0.0, 0.0),
                (0.0, 0.2 * math.sin(w * t), 0.0, 0.0, 0.2 * w * math.cos(w * t), 0.0)]
    return Case("mems_plate", 2, 2.0 / 3.0, 0.5, mu_ref_from_kn(kn, 0.5), 0.5, v, v.copy(),
                (-6.0, 6.0, -6.0, 6.0), winf, [bg, body], np.tile(winf, (ncell, 1)),
                dt=period / 400.0, n_inner=10, n_phys=20, motion=motion,
                overset={"wrule": wrule, "overlap": 2})


def two_body(nx: int = 512, ny: int = 256, ni: int = 128, nj: int = 96, nv: int = 100, kn: float = 1e-3,
             mach: float = 6.0, vmax: float = 20.0) -> Case:
    """Two-body separation: background [-3, 13] x [-4, 4] (512 x 256,
    far field); a circle of diameter 1 at the origin inside a 128 x 96 O-mesh
    out to radius 1.5 (radial ratio 1.02), and one of diameter 0.3 at
    (0.5, 2.55) inside a 128 x 96 O-mesh out to radius 1.0 (ratio 1.03); the
    small body moves as dy = t^2 / 2, dtheta = t / 5 about its centre;
    isothermal walls at the free-stream temperature; Ma 6 along +x;
    100 x 100 velocities on [-vmax, vmax]^2 (vmax = 20); dt = 10 dt_s.

    The two body meshes overlap the background only: where two body-fitted
    meshes of like spacing overlap, the wall-distance rule switches both at
    the same line and leaves receptors without a field donor.  The outer
    spacing of each O-mesh is close to the background's, so that its
    receptors fall in field cells of the background at any pose (with
    fewer radial cells the radial ratios grow so that the outer spacing
    stays the same)."""
    bg = cartesian_block(nx, ny, -3.0, 13.0, -4.0, 4.0, (FARFIELD, FARFIELD, FARFIELD, FARFIELD))
    big = o_block(ni, nj, geometric_radii(0.5, 1.5, nj, 1.02 ** (96 / nj)), bc=(PERIODIC, PERIODIC, WALL, NONE),
                  rtw=(0.5, 0.5, 0.5, 0.5), body=True)
    small = o_block(ni, nj, geometric_radii(0.15, 1.0, nj, 1.03 ** (96 / nj)), centre=(0.5, 2.55),
                    bc=(PERIODIC, PERIODIC, WALL, NONE), rtw=(0.5, 0.5, 0.5, 0.5), body=True)
    rt = 0.5
    u = mach * math.sqrt(5.0 / 3.0 * rt)
    winf = cons(2, 1.0, [u, 0.0], rt)
    v = uniform_points(nv, -vmax, vmax)
    ncell = bg.ncell + big.ncell + small.ncell

    def motion(t):
        return [(0.0,) * 6, (0.0,) * 6, (0.0, 0.5 * t * t, 0.2 * t, 0.0, t, 0.2)]
    return Case("two_body", 2, 2.0 / 3.0, 0.5, mu_ref_from_kn(kn, 0.5), rt, v, v.copy(),
                (-vmax, vmax, -vmax, vmax), winf, [bg, big, small], np.tile(winf, (ncell, 1)),
                dt_over_dts=10.0, n_inner=15, n_phys=20, motion=motion, overset={"wrule": 0, "overlap": 2})


def batch_cases(count: int = 64, seed: int = SEED) -> list:
    """Seeded batch of ragged cavity / plate cases: case i has n x n cells
    (n uniform in 32..128) and m x m velocities on [-5 sqrt(RT0), 5 sqrt(RT0)]^2
    (m uniform in 24..64), Kn = 10^U(-4, 1), an even case is a lid-driven
    cavity and an odd one a plate (periodic in x, moving top wall), wall speed
    U(0.1, 1) times sqrt(2 RT0); dt = 10 dt_s."""
    rng = np.random.default_rng(seed + 97)
    out = []
    for i in range(count):
        n = int(rng.integers(32, 129))
        m = int(rng.integers(24, 65))
        kn = float(10.0 ** rng.uniform(-4.0, 1.0))
        lid = float(rng.uniform(0.1, 1.0))
        c = cavity(n, m, kn=kn, lid=lid, periodic_x=(i % 2 == 1))
        c.name = f"batch{i:02d}_{c.name}_{n}x{n}_v{m}"
        out.append(c)
    return out
