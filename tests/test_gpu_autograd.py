"""Gradients through torch.autograd (the library's hand-written adjoint behind
torch.autograd.Function, checkpointed across dual-time steps) against the
oracle's reference gradient (the dual-number tangent build run through the
same physical steps) and against central differences of the HIP forward
path.

Objective: wall heat flux and force on a body (the side loads the library
forms from the face macro flux of the last inner iteration of each physical
step, ugks_wall_loads; the oracle's or_wall_loads on its side) plus a random
linear functional of the final distribution.  Parameters: the rigid
velocity of a block (dt_s and dt' held at the pose's values) and the wall
temperature; and the initial distribution.
"""
import numpy as np
import pytest
import torch

from oracle.oracle import Oracle, dual
from paper_2604_09984_amd import adjoint, ugks, workloads as wl
from tests.parity import dev, host, say

pytestmark = pytest.mark.gpu


def cavity():
    return wl.cavity(6, 8, kn=0.1, lid=0.5)


def moving_overset():
    ov = wl.overset_cylinder(ni_bg=28, nb=20, njb=8, nv=8, kn=0.05)
    w = np.pi
    ov.motion = lambda t: [(0.0, 0.0, 0.0, 0.0, 0.0, 0.0),
                           (0.0, 0.04 * np.sin(w * t), 0.1 * np.sin(w * t), 0.0, 0.04 * w * np.cos(w * t),
                            0.1 * w * np.cos(w * t))]
    return ov


class Run:
    """A short differentiable run: n_phys physical steps of n_inner inner
    iterations, objective J, on the library; and the same sequence on the
    oracle's tangent build."""

    def __init__(self, case, n_phys, n_inner, body, sides, seed=3, c=(1.0, 0.3, -0.2), yh_scale=0.1,
                 times=None, prec=ugks.F64):
        self.case, self.n_phys, self.n_inner, self.body, self.sides = case, n_phys, n_inner, body, sides
        self.s = ugks.Solver(case, prec)
        self.o = Oracle(case)
        self.idx = self.o.product_face_index()
        h, b, W = wl.synthetic_f(case, seed=seed, amp=0.02)
        self.h0, self.b0, self.W0 = h, b, W
        self.q0 = self.o.heatflux(h, b, W)  # held fixed (not a function of h0)
        rng = np.random.default_rng(seed + 1)
        self.yh = rng.standard_normal(h.shape) * yh_scale
        self.c = c  # weights of energy flux, x force, y force
        self.dt_over = case.dt_over_dts
        self.times = [0.05 * (k + 1) for k in range(n_phys)] if times is None else list(times)

    def setup_fn(self, k, types_prev):
        """Restores step k's geometry: the kinds before its assembly, the
        pose and the assembly (None for a fixed mesh)."""
        case, s = self.case, self.s
        if case.motion is None:
            return None

        def setup(solver):
            solver.set_types(types_prev)
            solver.set_poses(case.poses(self.times[k]))
            if case.overset is not None:
                solver.assemble(case.overset["wrule"], case.overset["overlap"])
        return setup

    def gpu(self, U, rtw, checkpoint=True, h0=None):
        s, case = self.s, self.case
        # initial geometry and kinds
        s.set_types(np.ones(case.ncell, np.int8))
        s.set_poses(case.poses(0.0))
        if case.overset is not None:
            s.assemble(case.overset["wrule"], case.overset["overlap"])
        h = dev(self.h0, s.dtype) if h0 is None else h0
        b, W, q = dev(self.b0, s.dtype), dev(self.W0), dev(self.q0)
        J = 0.0
        self.dts, self.dtps, self.dtk = [], [], []
        for k in range(self.n_phys):
            setup = self.setup_fn(k, s.types())
            if setup is not None:
                setup(s)
            dts, dtp = s.timesteps()
            dt = self.dt_over * dts
            self.dts.append(dts); self.dtps.append(dtp); self.dtk.append(dt)
            h, b, W, q, F, L = adjoint.physical_step(s, dt, self.n_inner, h, b, W, q, U, rtw, setup=setup,
                                                     checkpoint=checkpoint, loads=True)
            L = L[self.body, list(self.sides)]
            J = J + (self.c[0] * L[:, 3] + self.c[1] * L[:, 0] + self.c[2] * L[:, 1]).sum()
        J = J + (dev(self.yh) * h).sum()
        return J

    def gpu_rollout(self, U, rtw, snapshots, inner_snapshots=None, h0=None, stats=None):
        """The same objective through one adjoint.rollout node (binomial
        checkpointing over the physical steps)."""
        s, case = self.s, self.case
        s.set_types(np.ones(case.ncell, np.int8))
        s.set_poses(case.poses(0.0))
        if case.overset is not None:
            s.assemble(case.overset["wrule"], case.overset["overlap"])
        h = dev(self.h0, s.dtype) if h0 is None else h0
        b, W, q = dev(self.b0, s.dtype), dev(self.W0), dev(self.q0)

        def setup_at(k):
            if case.motion is None:
                return None

            def setup(solver):
                solver.set_poses(case.poses(self.times[k]))
                if case.overset is not None:
                    solver.assemble(case.overset["wrule"], case.overset["overlap"])
            return setup
        dt_of = lambda solver: self.dt_over * solver.timesteps()[0]
        steps = [(dt_of, self.n_inner, setup_at(k)) for k in range(self.n_phys)]
        h, b, W, q, F, Ls = adjoint.rollout(s, steps, h, b, W, q, U, rtw, snapshots=snapshots,
                                            inner_snapshots=inner_snapshots, stats=stats)
        J = 0.0
        for k in range(self.n_phys):
            L = Ls[k][self.body, list(self.sides)]
            J = J + (self.c[0] * L[:, 3] + self.c[1] * L[:, 0] + self.c[2] * L[:, 1]).sum()
        return J + (dev(self.yh) * h).sum()

    def oracle(self, U, rtw, dU=None, drt=None, dh0=None):
        """J and its directional derivative from the tangent build, with the
        library's dt_s and dt' of each step."""
        case = self.case
        ot = Oracle(case, tangent=True)
        h = dual(self.h0, dh0); b = dual(self.b0); W = dual(self.W0)
        nb = len(case.blocks)

        def pose(t):
            out = []
            for bi, p in enumerate(case.poses(t)):
                row = [(x, 0.0) for x in p]
                row[3] = (float(U[bi, 0]), dU[bi, 0] if dU is not None else 0.0)
                row[4] = (float(U[bi, 1]), dU[bi, 1] if dU is not None else 0.0)
                out.append(row)
            return out
        for bi, B in enumerate(case.blocks):
            for sd in range(4):
                if B.bc[sd] == wl.WALL:
                    ot.set_wall_rt(bi, sd, (float(rtw[bi, sd]), drt[bi, sd] if drt is not None else 0.0))
        ot.set_poses(pose(0.0))
        if case.overset is not None:
            ot.assemble(case.overset["wrule"], case.overset["overlap"])
        q = dual(self.q0)
        Jv, Jd = 0.0, 0.0
        for k in range(self.n_phys):
            if case.motion is not None:
                ot.set_poses(pose(self.times[k]))
                if case.overset is not None:
                    ot.assemble(case.overset["wrule"], case.overset["overlap"])
            dts, dt = self.dts[k], self.dtk[k]
            Wn = W.copy()
            Sh, Sb, Fn = ot.begin_step((dt, 0.0), (dts, 0.0), h, b, W, q)
            F = ot._z(max(ot.nface, 1), case.nw)
            for _ in range(self.n_inner):
                ot.pseudo_step((dt, 0.0), (dts, 0.0), dual(self.dtps[k]), h, b, W, Wn, q, Sh, Sb, Fn, F)
            _, side = ot.wall_loads(F[:ot.nface])
            L = side[self.body, list(self.sides)]
            G = self.c[0] * L[:, 3] + self.c[1] * L[:, 0] + self.c[2] * L[:, 1]
            Jv += float(np.sum(G[..., 0])); Jd += float(np.sum(G[..., 1]))
        Jv += float(np.sum(self.yh * h[..., 0])); Jd += float(np.sum(self.yh * h[..., 1]))
        return Jv, Jd


def _params(run):
    U, R = adjoint.default_params(run.s)
    for bi, p in enumerate(run.case.poses(0.0)):
        U[bi, 0], U[bi, 1] = p[3], p[4]
    return U, R


def _close(a, b, tol, what):
    rel = abs(a - b) / max(abs(a), abs(b), 1e-300)
    say(f"  {what}: reference {a:.15e} autograd {b:.15e} rel {rel:.2e}")
    assert rel <= tol, (what, a, b, rel)


@pytest.mark.parametrize("make,body,sides", [(cavity, 0, (0, 1, 2, 3)), (moving_overset, 1, (2,))],
                         ids=["cavity", "moving_overset"])
def test_checkpointed_gradient_matches_oracle(make, body, sides):
    case = make()
    say("autograd vs oracle", case.name)
    R = Run(case, n_phys=2, n_inner=2, body=body, sides=sides)
    U, rt = _params(R)
    Ug = U.clone().requires_grad_(True)
    rtg = rt.clone().requires_grad_(True)
    h0 = dev(R.h0).requires_grad_(True)
    J = R.gpu(Ug, rtg, h0=h0)
    gU, gR, gh = torch.autograd.grad(J, [Ug, rtg, h0])
    Jv, _ = R.oracle(U, rt)
    _close(Jv, float(J), 1e-9, "J")
    nb = len(case.blocks)
    for comp in range(2):
        dU = np.zeros((nb, 2)); dU[body, comp] = 1.0
        _, Jd = R.oracle(U, rt, dU=dU)
        _close(Jd, float(gU[body, comp]), 1e-8, f"dJ/dU[{body},{comp}]")
    wall_sides = [sd for sd in sides if case.blocks[body].bc[sd] == wl.WALL]
    drt = np.zeros((nb, 4)); drt[body, wall_sides[0]] = 1.0
    _, Jd = R.oracle(U, rt, drt=drt)
    _close(Jd, float(gR[body, wall_sides[0]]), 1e-8, f"dJ/dRTw[{body},{wall_sides[0]}]")
    rng = np.random.default_rng(7)
    dh = rng.standard_normal(R.h0.shape) * R.h0 * 0.1
    _, Jd = R.oracle(U, rt, dh0=dh)
    _close(Jd, float((gh * dev(dh)).sum()), 1e-8, "dJ/dh0 . v")


def test_checkpointed_equals_stored_graph():
    case = cavity()
    say("checkpointed vs stored", case.name)
    R = Run(case, n_phys=2, n_inner=3, body=0, sides=(3,))
    U, rt = _params(R)
    grads = []
    for ck in (True, False):
        Ug = U.clone().requires_grad_(True)
        rtg = rt.clone().requires_grad_(True)
        h0 = dev(R.h0).requires_grad_(True)
        J = R.gpu(Ug, rtg, checkpoint=ck, h0=h0)
        grads.append([t.detach().cpu().numpy() for t in torch.autograd.grad(J, [Ug, rtg, h0])])
    for a, b in zip(*grads):
        assert np.allclose(a, b, rtol=1e-12, atol=1e-14 * np.abs(a).max())


def test_autograd_gradient_matches_finite_differences():
    case = cavity()
    say("autograd vs finite differences", case.name)
    R = Run(case, n_phys=2, n_inner=2, body=0, sides=(3,))
    U, rt = _params(R)
    Ug = U.clone().requires_grad_(True)
    rtg = rt.clone().requires_grad_(True)
    gU, gR = torch.autograd.grad(R.gpu(Ug, rtg), [Ug, rtg])
    eps = 1e-6
    with torch.no_grad():
        for what, P, G, i in (("U[0,0]", U, gU, (0, 0)), ("U[0,1]", U, gU, (0, 1)), ("RTw[0,3]", rt, gR, (0, 3))):
            Pp, Pm = P.clone(), P.clone()
            Pp[i] += eps; Pm[i] -= eps
            if P is U:
                fd = (float(R.gpu(Pp, rt)) - float(R.gpu(Pm, rt))) / (2 * eps)
            else:
                fd = (float(R.gpu(U, Pp)) - float(R.gpu(U, Pm))) / (2 * eps)
            _close(fd, float(G[i]), 1e-6, what)


@pytest.mark.timeout(400)
def test_two_body_lift_gradient():
    """The two-body separation, reduced (96 x 48 background, two 24 x 10
    O-meshes, 16 x 16 velocities on [-6, 6]^2): gradient of the small body's
    lift (y force on its wall, summed over the steps) through 20 checkpointed
    physical steps with re-assembly at each, with respect to the small body's
    velocity and wall temperature; against the oracle's tangent build and
    central differences of the HIP forward path.  Ma 0.5 and Kn 0.1 at this
    resolution: an impulsive start at Ma 6 empties the thin lee-side wall
    cells within a few large implicit steps."""
    case = wl.two_body(nx=96, ny=48, ni=24, nj=10, nv=16, vmax=6.0, mach=0.5, kn=0.1)
    say("two-body lift gradient", case.ncell * case.nv, "pairs, 20 physical steps")
    R = Run(case, n_phys=20, n_inner=2, body=2, sides=(2,), c=(0.0, 0.0, 1.0), yh_scale=0.0,
            times=[0.02 * (k + 1) for k in range(20)])
    U, rt = _params(R)
    Ug = U.clone().requires_grad_(True)
    rtg = rt.clone().requires_grad_(True)
    J = R.gpu(Ug, rtg)
    gU, gR = torch.autograd.grad(J, [Ug, rtg])
    nb = len(case.blocks)
    dU = np.zeros((nb, 2)); dU[2, 1] = 1.0
    Jv, Jd = R.oracle(U, rt, dU=dU)
    _close(Jv, float(J), 1e-9, "lift")
    _close(Jd, float(gU[2, 1]), 1e-8, "dlift/dU_y")
    dU = np.zeros((nb, 2)); dU[2, 0] = 1.0
    _, Jd = R.oracle(U, rt, dU=dU)
    _close(Jd, float(gU[2, 0]), 1e-8, "dlift/dU_x")
    drt = np.zeros((nb, 4)); drt[2, 2] = 1.0
    _, Jd = R.oracle(U, rt, drt=drt)
    _close(Jd, float(gR[2, 2]), 1e-8, "dlift/dRTw")
    eps = 1e-6
    with torch.no_grad():
        for what, i in (("U_y", (2, 1)), ("RTw", (2, 2))):
            P = U if what == "U_y" else rt
            Pp, Pm = P.clone(), P.clone()
            Pp[i] += eps; Pm[i] -= eps
            if P is U:
                fd = (float(R.gpu(Pp, rt)) - float(R.gpu(Pm, rt))) / (2 * eps)
            else:
                fd = (float(R.gpu(U, Pp)) - float(R.gpu(U, Pm))) / (2 * eps)
            _close(fd, float((gU if P is U else gR)[i]), 1e-6, "finite difference " + what)


@pytest.mark.timeout(300)
def test_batch_cases_wall_heat_flux_gradient():
    """The adjoint of the wall heat flux (energy flux through the moving top
    wall, summed over two checkpointed physical steps of two inner
    iterations) for the two smallest cases of the seeded 64-case batch, with
    respect to the top wall's temperature and the initial distribution,
    against the oracle's tangent build."""
    cases = wl.batch_cases(64)
    pairs = [c.ncell * c.nv for c in cases]
    for i in np.argsort(pairs, kind="stable")[:2]:
        case = cases[int(i)]
        say("batch case heat-flux gradient", case.name)
        R = Run(case, n_phys=2, n_inner=2, body=0, sides=(3,), c=(1.0, 0.0, 0.0), yh_scale=0.0)
        U, rt = _params(R)
        rtg = rt.clone().requires_grad_(True)
        h0 = dev(R.h0).requires_grad_(True)
        J = R.gpu(U, rtg, h0=h0)
        gR, gh = torch.autograd.grad(J, [rtg, h0])
        nb = len(case.blocks)
        drt = np.zeros((nb, 4)); drt[0, 3] = 1.0
        Jv, Jd = R.oracle(U, rt, drt=drt)
        _close(Jv, float(J), 1e-9, "heat flux")
        _close(Jd, float(gR[0, 3]), 1e-8, "d/dRTw")
        rng = np.random.default_rng(int(i))
        dh = rng.standard_normal(R.h0.shape) * R.h0 * 0.1
        _, Jd = R.oracle(U, rt, dh0=dh)
        _close(Jd, float((gh * dev(dh)).sum()), 1e-8, "d/dh0 . v")
        R.s.close()


@pytest.mark.parametrize("make,body,sides", [(cavity, 0, (0, 1, 2, 3)), (moving_overset, 1, (2,))],
                         ids=["cavity", "moving_overset"])
def test_fp32_storage_gradient(make, body, sides):
    """A solver with FP32 storage differentiated through checkpointed
    physical steps (its reverse passes run on an FP64 twin context): the
    objective and its gradients agree with the FP64 solver's to the FP32
    storage error, and the block-velocity derivative with the oracle's
    tangent build."""
    case = make()
    say("FP32-storage gradient", case.name)
    out = []
    for prec in (ugks.F64, ugks.F32):
        R = Run(case, n_phys=2, n_inner=2, body=body, sides=sides, prec=prec)
        U, rt = _params(R)
        Ug = U.clone().requires_grad_(True)
        rtg = rt.clone().requires_grad_(True)
        h0 = dev(R.h0, R.s.dtype).requires_grad_(True)
        J = R.gpu(Ug, rtg, h0=h0)
        g = torch.autograd.grad(J, [Ug, rtg, h0])
        assert g[2].dtype == R.s.dtype
        out.append((float(J.detach()), [t.detach().double().cpu().numpy() for t in g], R, U, rt))
    (J64, g64, R64, U, rt), (J32, g32, _, _, _) = out
    _close(J64, J32, 1e-5, "J (FP32 storage vs FP64)")
    for a, b_, what in zip(g64[:2], g32[:2], ("dJ/dU", "dJ/dRTw")):
        err = np.abs(a - b_).max() / max(np.abs(a).max(), 1e-300)
        say(f"  {what}: max relative difference FP32 vs FP64 {err:.2e}")
        assert err <= 1e-4, (what, err)
    # dJ/dh0 is evaluated at the FP32-rounded state, which flushes the far
    # velocity tails (below FP32's range) to zero; there the limiters take
    # other branches, so entries of those tails differ: the gradient is
    # compared along directions scaled like the state (tails weigh little)
    a, b_ = g64[2], g32[2]
    l2 = float(np.linalg.norm(a - b_) / np.linalg.norm(a))
    v = np.random.default_rng(9).standard_normal(a.shape) * R64.h0
    dd = abs(float(np.sum(a * v)) - float(np.sum(b_ * v))) / abs(float(np.sum(a * v)))
    say(f"  dJ/dh0: relative L2 {l2:.2e}, along a random direction {dd:.2e}, "
        f"max entry {np.abs(a - b_).max() / np.abs(a).max():.2e}")
    assert dd <= 1e-4
    dU = np.zeros((len(case.blocks), 2)); dU[body, 0] = 1.0
    _, Jd = R64.oracle(U, rt, dU=dU)
    _close(Jd, float(g32[0][body, 0]), 1e-4, f"dJ/dU[{body},0] FP32 vs oracle")


@pytest.mark.timeout(300)
def test_rollout_binomial_checkpointing_same_bits():
    """Six physical steps of the moving overset cylinder (re-assembly at each
    step) as one rollout node: for every number of kept states (1: each step
    re-run from the input; 2, 3; 5: each state computed once) and with the
    inner iterations of a step re-run from Steps 1-2's output (inner
    snapshots 1), the gradients equal, bit for bit, those of the chain of
    checkpointed physical steps, and the re-run steps number
    revolve_cost(6, snapshots)."""
    case = moving_overset()
    R = Run(case, n_phys=6, n_inner=2, body=1, sides=(2,))
    U, rt = _params(R)

    def grads(fn):
        Ug = U.clone().requires_grad_(True)
        rtg = rt.clone().requires_grad_(True)
        h0 = dev(R.h0).requires_grad_(True)
        J = fn(Ug, rtg, h0)
        return [float(J)] + [t.detach().clone() for t in torch.autograd.grad(J, [Ug, rtg, h0])]

    ref = grads(lambda u, r, h0: R.gpu(u, r, h0=h0))
    for snaps, inner in ((1, None), (2, None), (3, 1), (5, None)):
        stats = {}
        got = grads(lambda u, r, h0: R.gpu_rollout(u, r, snaps, inner, h0=h0, stats=stats))
        say("rollout", "snapshots", snaps, "inner", inner, "re-run steps", stats["recomputed_steps"],
            "J", got[0], "|dJ/dU|", float(got[1].abs().max()))
        for name, a, b in zip(("U", "RTw", "h0"), ref[1:], got[1:]):
            d = (a - b).abs().max().item()
            say("  ", name, "max |difference|", d, "max |gradient|", a.abs().max().item(),
                "equal" if torch.equal(a, b) else "differ")
        assert got[0] == ref[0]
        for a, b in zip(ref[1:], got[1:]):
            assert torch.equal(a, b)
        assert stats["recomputed_steps"] == adjoint.revolve_cost(6, snaps)


def test_wall_loads_reverse_refuses_another_pose():
    """adjoint.wall_loads reverses at the solver's current geometry, so it
    refuses to run after the pose moved (the loads of a moving step come
    from physical_step(loads=True) or rollout instead)."""
    case = moving_overset()
    s = ugks.Solver(case, ugks.F64)
    s.set_poses(case.poses(0.1))
    F = torch.ones((s.nface, case.nw), dtype=torch.float64, device="cuda", requires_grad=True)
    L = adjoint.wall_loads(s, F)
    s.set_poses(case.poses(0.2))
    with pytest.raises(ValueError, match="another pose"):
        L.sum().backward()
    s.set_poses(case.poses(0.1))
    L = adjoint.wall_loads(s, F)
    L.sum().backward()
    assert float(F.grad.abs().sum()) > 0
    s.close()


@pytest.mark.timeout(900)
def test_batch_all_cases_heat_flux_gradient_fd():
    """All 64 cases of the seeded batch (cavities and plates, 32^2 to 128^2
    cells, 24^2 to 64^2 velocities, Kn 1e-4 to 10): the energy flux into the
    moving top wall through one checkpointed physical step of two inner
    iterations, differentiated with respect to that wall's temperature by the
    library's adjoint, against central differences of the HIP forward path
    (FP64 storage; relative 1e-6)."""
    cases = wl.batch_cases(64)
    worst = 0.0
    for case in cases:
        s = ugks.Solver(case, ugks.F64)
        h0, b0, W0 = wl.synthetic_f(case, seed=5, amp=0.02)
        hd, bd, Wd = dev(h0), dev(b0), dev(W0)
        qd = s.heatflux(hd, bd, Wd)
        dts, _ = s.timesteps()
        dt = case.dt if case.dt is not None else case.dt_over_dts * dts
        U, R = adjoint.default_params(s)

        def J(rt):
            _, _, _, _, _, L = adjoint.physical_step(s, dt, 2, hd, bd, Wd, qd, U, rt, loads=True)
            return L[0, 3, 3]
        Rg = R.clone().requires_grad_(True)
        g = torch.autograd.grad(J(Rg), [Rg])[0][0, 3].item()
        eps = 1e-6 * float(R[0, 3])
        with torch.no_grad():
            Rp, Rm = R.clone(), R.clone()
            Rp[0, 3] += eps; Rm[0, 3] -= eps
            fd = (float(J(Rp)) - float(J(Rm))) / (2 * eps)
        rel = abs(fd - g) / max(abs(fd), abs(g), 1e-300)
        worst = max(worst, rel)
        say(f"  {case.name}: dq/dRTw adjoint {g:.12e} central differences {fd:.12e} rel {rel:.2e}")
        assert abs(g) > 0 and rel <= 1e-6, (case.name, g, fd, rel)
        s.close()
    say("worst relative difference over the 64 cases", worst)
