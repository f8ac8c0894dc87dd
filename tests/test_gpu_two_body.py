"""The two-body separation at its stated physics (Ma 6 along +x, Kn 1e-3,
100 x 100-style velocity range [-20, 20]^2, small body moving as
dy = t^2 / 2, dtheta = t / 5), on a down-scaled mesh whose whole field the
oracle computes in seconds: background [-3, 13] x [-4, 4] of 256 x 128 cells,
two 64 x 48 O-meshes, 24 x 24 velocities (22.4 M pairs).

Two physical steps from t = 0.5 (the small body moving at 0.5 upward and
0.2 rad per unit time), each with the pose at the step's end, the overset
assembly (bit-exact), Steps 1-2 and three inner iterations through the
autotuned captured graph, against the FP64 oracle's whole field: relative
L2 <= 1e-10 (FP64) and 1e-5 (FP32 storage) over h, b and W of the live
cells, and per cell max |f - f_oracle| / max |f_oracle| on the cells beside
a wall and on the overset fringe (receptors and their index neighbours),
where an error confined to a few cells would hide inside a global norm.

The survey's smaller down-scale (128 x 64 background, 32 x 24 O-meshes)
leaves receptors of the small body's overset layers without a field donor
under the assembly rules of Sec. 3.1 (its outer O-mesh cells are coarser
than the overlap the rules need), so the O-meshes here keep the full-size
mesh's relative spacing at half its resolution.
"""
import numpy as np
import pytest
import torch

from oracle.oracle import Oracle, dual
from paper_2604_09984_amd import adjoint, ugks, workloads as wl
from tests.parity import dev, host, rel_l2, say

pytestmark = pytest.mark.gpu

T0 = 0.5
NPHYS = 2
NINNER = 3


def _case():
    return wl.two_body(nx=256, ny=128, ni=64, nj=48, nv=24)


def _cell_sets(case, types, rec):
    """Cells beside a wall (j = 0 of the body blocks) and the fringe:
    receptors and their index neighbours within the same block."""
    wall, fringe = [], set()
    off = 0
    index = {}
    for bi, blk in enumerate(case.blocks):
        if blk.body:
            wall.extend(off + i for i in range(blk.ni))
        for j in range(blk.nj):
            for i in range(blk.ni):
                index[off + i + blk.ni * j] = (bi, i, j, off)
        off += blk.ncell
    for r in rec:
        bi, i, j, o = index[int(r)]
        blk = case.blocks[bi]
        for di, dj in ((0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)):
            ii, jj = i + di, j + dj
            if blk.bc[0] == wl.PERIODIC:
                ii %= blk.ni
            if 0 <= ii < blk.ni and 0 <= jj < blk.nj:
                c = o + ii + blk.ni * jj
                if types[c] != 0:
                    fringe.add(c)
    return np.array(sorted(wall)), np.array(sorted(fringe))


def _cell_max_rel(a, b, cells):
    """max over the cells of max_k |a - b| / max_k |b|."""
    d = np.abs(a[cells] - b[cells]).max(axis=1)
    m = np.abs(b[cells]).max(axis=1)
    return float((d / m).max())


@pytest.fixture(scope="module")
def two_body_ref():
    case = _case()
    o = Oracle(case)
    h, b, W, q = o.init_state()
    inputs = dict(h=h.copy(), b=b.copy(), W=W.copy(), q=q.copy())
    t = T0
    steps = []
    for n in range(NPHYS):
        dts, _ = o.timesteps()
        t += case.dt_over_dts * dts
        o.set_poses(case.poses(t))
        rc, _ = o.assemble(case.overset["wrule"], case.overset["overlap"])
        assert rc == 0
        tables = (o.types(), *o.overset())
        dts, dtp = o.timesteps()
        dt = case.dt_over_dts * dts
        Wn = W.copy()
        Sh, Sb, Fn = o.begin_step(dt, dts, h, b, W, q)
        for _ in range(NINNER):
            o.pseudo_step(dt, dts, dtp, h, b, W, Wn, q, Sh, Sb, Fn)
        steps.append(dict(t=t, dt=dt, tables=tables))
    live = o.types() == 1
    rho = W[live, 0]
    say("two-body (Ma 6, Kn 1e-3) down-scale:", case.ncell * case.nv, "pairs; oracle density after",
        NPHYS, "steps in", float(rho.min()), float(rho.max()))
    assert rho.min() > 0.1
    return dict(case=case, inputs=inputs, steps=steps, out=dict(h=h, b=b, W=W), live=live,
                types=o.types(), rec=o.overset()[0])


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec,tol,ctol", [(ugks.F64, 1e-10, 1e-12), (ugks.F32, 1e-5, 1e-5)], ids=["f64", "f32"])
def test_two_body_ma6_steps(two_body_ref, prec, tol, ctol):
    ref = two_body_ref
    case = ref["case"]
    s = ugks.Solver(case, prec)
    dt_t = torch.float64 if prec == ugks.F64 else torch.float32
    x = ref["inputs"]
    h, b, W, q = dev(x["h"], dt_t), dev(x["b"], dt_t), dev(x["W"]), dev(x["q"])
    for n, st in enumerate(ref["steps"]):
        s.set_poses(case.poses(st["t"]))
        s.assemble(case.overset["wrule"], case.overset["overlap"])
        types, rec, ptr, don, w = st["tables"]
        srec, sptr, sdon, sw = s.overset()
        assert np.array_equal(s.types(), types)
        assert np.array_equal(srec, rec) and np.array_equal(sptr, ptr) and np.array_equal(sdon, don)
        assert np.abs(sw - w).max(initial=0.0) <= 1e-15
        dts, _ = s.timesteps()
        dt = case.dt_over_dts * dts
        assert abs(dt - st["dt"]) <= 1e-15 * st["dt"]
        Wn = W.clone()
        Sh, Sb, Fn = s.begin_step(dt, h, b, W, q)
        if n == 0:
            work = [t.clone() for t in (h, b, W, Wn, q, Sh, Sb, Fn)]
            tuning, _ = s.autotune(dt, NINNER, *work)
            say("  launch shapes", tuning)
        s.step_graph(dt, NINNER, h, b, W, Wn, q, Sh, Sb, Fn)
    torch.cuda.synchronize()
    live = ref["live"]
    out = ref["out"]
    hh, bb, WW = host(h), host(b), host(W)
    e = [rel_l2(hh[live], out["h"][live]), rel_l2(bb[live], out["b"][live]), rel_l2(WW[live], out["W"][live])]
    wall, fringe = _cell_sets(case, ref["types"], ref["rec"])
    cw = max(_cell_max_rel(hh, out["h"], wall), _cell_max_rel(bb, out["b"], wall))
    cf = max(_cell_max_rel(hh, out["h"], fringe), _cell_max_rel(bb, out["b"], fringe))
    say("  ", "f64" if prec == ugks.F64 else "f32", "rel L2 h b W", e, "per-cell max rel: wall", cw,
        f"({len(wall)} cells)", "fringe", cf, f"({len(fringe)} cells)")
    assert max(e) <= tol
    assert max(cw, cf) <= ctol
    s.close()


# ----------------------------------------------------------------------------
# Full shape (512 x 256 background, two 128 x 96 O-meshes, 100 x 100
# velocities: 1.56 G pairs): Steps 1-2 and one inner iteration against the
# oracle's whole field.  The oracle needs about 100 GB of host memory and
# minutes of host time for it (149 s on 16 host threads), so the test runs
# on request only (UGKS_FULL_ORACLE=1); its last result is quoted with the
# design notes.

@pytest.mark.timeout(1500)
@pytest.mark.skipif(__import__("os").environ.get("UGKS_FULL_ORACLE") != "1",
                    reason="needs ~100 GB of host memory and minutes of oracle time (UGKS_FULL_ORACLE=1)")
@pytest.mark.parametrize("prec,tol", [(ugks.F64, 1e-10)], ids=["f64"])
def test_two_body_full_shape_whole_step(prec, tol):
    import time
    case = wl.two_body()
    o = Oracle(case)
    s = ugks.Solver(case, prec)
    h, b, W, q = o.init_state()
    dts, _ = o.timesteps()
    t = T0 + case.dt_over_dts * dts
    o.set_poses(case.poses(t))
    s.set_poses(case.poses(t))
    rc, _ = o.assemble(case.overset["wrule"], case.overset["overlap"])
    assert rc == 0
    s.assemble(case.overset["wrule"], case.overset["overlap"])
    assert np.array_equal(s.types(), o.types())
    dts, dtp = o.timesteps()
    dt = case.dt_over_dts * dts
    dt_t = torch.float64 if prec == ugks.F64 else torch.float32
    hd, bd, Wd, qd = dev(h, dt_t), dev(b, dt_t), dev(W), dev(q)
    Wnd = Wd.clone()
    Shd, Sbd, Fnd = s.begin_step(dt, hd, bd, Wd, qd)
    s.step_graph(dt, 1, hd, bd, Wd, Wnd, qd, Shd, Sbd, Fnd)
    torch.cuda.synchronize()
    del Shd, Sbd, Fnd, Wnd
    say("full-shape two-body:", case.ncell * case.nv, "pairs; library step done, oracle running")
    t0 = time.time()
    Wn = W.copy()
    Sh, Sb, Fn = o.begin_step(dt, dts, h, b, W, q)
    o.pseudo_step(dt, dts, dtp, h, b, W, Wn, q, Sh, Sb, Fn)
    del Sh, Sb, Fn
    say("  oracle Steps 1-2 and one inner iteration:", round(time.time() - t0, 1), "s")
    live = o.types() == 1
    err = []
    for name, ref, d in (("h", h, hd), ("b", b, bd)):
        num = den = 0.0
        for c0 in range(0, case.ncell, 8192):
            c1 = min(case.ncell, c0 + 8192)
            m = live[c0:c1]
            x = d[c0:c1].double().cpu().numpy()[m]
            y = ref[c0:c1][m]
            num += float(np.sum((x - y) ** 2))
            den += float(np.sum(y ** 2))
        err.append((num / den) ** 0.5)
    err.append(rel_l2(host(Wd)[live], W[live]))
    say("  rel L2 h b W", err)
    assert max(err) <= tol
    s.close()


# --------------------------------------------------------------------------
# the adjoint at Ma 6, Kn 1e-3 after a ramped inflow
# --------------------------------------------------------------------------
NRAMP, NDIFF, NIN = 20, 20, 2


def _winf(mach, rt=0.5):
    return wl.cons(2, 1.0, [mach * np.sqrt(5.0 / 3.0 * rt), 0.0], rt)


@pytest.mark.timeout(900)
def test_ma6_adjoint_after_ramped_inflow():
    """The separation's gradient at Ma 6 and Kn 1e-3: a 96 x 48 background
    with two 24 x 10 O-meshes and 24 x 24 velocities on [-10, 10]^2 (a
    range that still resolves the Ma 6 Maxwellian), started at rest and
    brought to Ma 6 by 20 non-differentiated steps of the oracle with the
    far-field Mach number raised by 0.3 per step (an impulsive Ma 6 start
    empties the lee-side wall cells at this resolution); from that state,
    20 differentiated physical steps (two inner iterations each, the small
    body moving as dy = t^2 / 2, dtheta = t / 5 with re-assembly at every
    step, through adjoint.rollout with 3 kept states) of the small body's
    lift summed over the steps, with respect to its (constant) block
    velocity and wall temperature: against the oracle's tangent build run
    through the same 20 steps (its own assembly and time steps at each
    pose) and central differences of the HIP forward path."""
    case = wl.two_body(nx=96, ny=48, ni=24, nj=10, nv=24, vmax=10.0, mach=6.0, kn=1e-3)
    o = Oracle(case)
    o.set_poses(case.poses(0.0))
    assert o.assemble(0, 2)[0] == 0
    W = np.tile(_winf(0.0), (case.ncell, 1))
    h, b = o.maxwellian(W)
    q = o.heatflux(h, b, W)
    for k in range(NRAMP):
        o.set_farfield(_winf(6.0 * (k + 1) / NRAMP))
        dts, dtp = o.timesteps()
        dt = case.dt_over_dts * dts
        Wn = W.copy()
        Sh, Sb, Fn = o.begin_step(dt, dts, h, b, W, q)
        for _ in range(NIN):
            o.pseudo_step(dt, dts, dtp, h, b, W, Wn, q, Sh, Sb, Fn)
    field = o.types() == 1
    say("Ma 6 ramp: field rho min", float(W[field, 0].min()), "max", float(W[field, 0].max()))
    assert np.isfinite(h).all() and W[field, 0].min() > 0.3
    times = [0.02 * (k + 1) for k in range(NDIFF)]
    body, side = 2, 2  # the small body's wall (its O-mesh's j-min side)

    s = ugks.Solver(case, ugks.F64)
    s.set_farfield(_winf(6.0))
    U, R = adjoint.default_params(s)
    U[body, 1] = 0.4

    def J_gpu(Ug, Rg, stats=None):
        s.set_types(np.ones(case.ncell, np.int8))
        s.set_poses(case.poses(0.0))
        s.assemble(0, 2)

        def setup_at(t):
            def setup(solver):
                solver.set_poses(case.poses(t))
                solver.assemble(0, 2)
            return setup
        dt_of = lambda solver: case.dt_over_dts * solver.timesteps()[0]
        steps = [(dt_of, NIN, setup_at(t)) for t in times]
        hN, bN, WN, qN, F, L = adjoint.rollout(s, steps, dev(h), dev(b), dev(W), dev(q), Ug, Rg, snapshots=3,
                                               stats=stats)
        assert bool(torch.isfinite(WN).all())
        return L[:, body, side, 1].sum()

    Ug = U.clone().requires_grad_(True)
    Rg = R.clone().requires_grad_(True)
    stats = {}
    J = J_gpu(Ug, Rg, stats)
    gU, gR = torch.autograd.grad(J, [Ug, Rg])
    assert stats["recomputed_steps"] == adjoint.revolve_cost(NDIFF, 3)

    # the oracle's tangent build along the small body's y velocity
    ot = Oracle(case, tangent=True)
    ot.set_farfield(_winf(6.0))

    def pose(t):
        out = []
        for bi, p in enumerate(case.poses(t)):
            row = [(x, 0.0) for x in p]
            row[3] = (float(U[bi, 0]), 0.0)
            row[4] = (float(U[bi, 1]), 1.0 if bi == body else 0.0)
            out.append(row)
        return out
    ot.set_poses(pose(0.0))
    assert ot.assemble(0, 2)[0] == 0
    hd, bd, Wd, qd = dual(h), dual(b), dual(W), dual(q)
    Jv = Jd = 0.0
    for t in times:
        # as the library: the pose's geometry, assembly and time steps,
        # then the block velocity parameter on the faces (dt_s, dt' kept)
        ot.set_poses([[(x, 0.0) for x in p] for p in case.poses(t)])
        assert ot.assemble(0, 2)[0] == 0
        dts, dtp = ot.timesteps()
        ot.set_poses(pose(t))
        dt = case.dt_over_dts * dts[0]
        Wn = Wd.copy()
        Sh, Sb, Fn = ot.begin_step((dt, 0.0), (dts[0], 0.0), hd, bd, Wd, qd)
        F = ot._z(max(ot.nface, 1), case.nw)
        for _ in range(NIN):
            ot.pseudo_step((dt, 0.0), (dts[0], 0.0), dtp, hd, bd, Wd, Wn, qd, Sh, Sb, Fn, F)
        _, sl = ot.wall_loads(F[:ot.nface])
        Jv += float(sl[body, side, 1, 0])
        Jd += float(sl[body, side, 1, 1])

    def close(ref, got, tol, what):
        rel = abs(ref - got) / max(abs(ref), abs(got), 1e-300)
        say(f"  {what}: reference {ref:.15e} gpu {got:.15e} rel {rel:.2e}")
        assert rel <= tol, (what, ref, got, rel)
    close(Jv, float(J), 1e-9, "lift over 20 steps")
    close(Jd, float(gU[body, 1]), 1e-8, "dlift/dU_y (oracle tangent)")
    eps = 1e-6
    with torch.no_grad():
        Up, Um = U.clone(), U.clone()
        Up[body, 1] += eps; Um[body, 1] -= eps
        fd = (float(J_gpu(Up, R)) - float(J_gpu(Um, R))) / (2 * eps)
        close(fd, float(gU[body, 1]), 1e-6, "dlift/dU_y (central differences)")
        Rp, Rm = R.clone(), R.clone()
        Rp[body, side] += eps; Rm[body, side] -= eps
        fd = (float(J_gpu(U, Rp)) - float(J_gpu(U, Rm))) / (2 * eps)
        close(fd, float(gR[body, side]), 1e-6, "dlift/dRTw (central differences)")
    s.close()


def test_set_farfield_rejects_a_bad_state():
    s = ugks.Solver(wl.cavity(4, 4), ugks.F64)
    for bad in ([0.0, 0.0, 0.0, 1.0], [1.0, 2.0, 0.0, 1.0], [1.0, float("nan"), 0.0, 1.0]):
        with pytest.raises(ugks.UgksError):
            s.set_farfield(bad)
    s.set_farfield(_winf(0.5))
    s.close()
