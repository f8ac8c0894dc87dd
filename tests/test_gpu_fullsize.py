"""Parity at the workloads' full sizes, in the launch configuration bench.py
times (autotuned launch shapes, the captured graph), element by element
against the FP64 oracle: FP64 to relative L2 1e-10, the FP32-storage path
to 1e-5.

- Ma 5 cylinder: O-mesh 128 x 64 cells, 64 x 64 velocities (33.6 M pairs),
  Steps 1-2 and one inner iteration from the potential-flow start.
- Thermal MEMS plate: 256 x 256 background plus a 128 x 64 overset O-mesh,
  48 x 48 velocities (169.9 M pairs), Kn 0.1 and 1: the plate's pose at the
  first step, the overset assembly bit-exact, then Steps 1-2 and one inner
  iteration from a perturbed state (every cell carries a non-equilibrium f).
- Two-body separation: 512 x 256 background plus two 128 x 96 O-meshes,
  100 x 100 velocities (1.56 G pairs): the assembly whole, Steps 1-2 at a
  sample of cells, then one inner iteration run whole.
"""
import numpy as np
import pytest
import torch

from oracle.oracle import Oracle
from paper_2604_09984_amd import ugks, workloads as wl
from tests.parity import dev, host, rel_l2, say

pytestmark = pytest.mark.gpu


def _oracle_step(case, state, t):
    """Oracle: pose at t and assembly (moving overset), Steps 1-2, one inner
    iteration.  Returns the inputs, the outputs and the donor tables."""
    o = Oracle(case)
    tables = None
    if case.motion is not None:
        o.set_poses(case.poses(t))
        rc, _ = o.assemble(case.overset["wrule"], case.overset["overlap"])
        assert rc == 0
        tables = (o.types(), *o.overset())
    h, b, W, q = state(o)
    inputs = dict(h=h.copy(), b=b.copy(), W=W.copy(), q=q.copy())
    dts, dtp = o.timesteps()
    dt = case.dt if case.dt is not None else case.dt_over_dts * dts
    Wn = W.copy()
    Sh, Sb, Fn = o.begin_step(dt, dts, h, b, W, q)
    o.pseudo_step(dt, dts, dtp, h, b, W, Wn, q, Sh, Sb, Fn)
    return dict(case=case, t=t, inputs=inputs, out=dict(h=h, b=b, W=W, q=q), tables=tables,
                live=o.types() == 1)


def _gpu_step(ref, prec, tol):
    case = ref["case"]
    s = ugks.Solver(case, prec)
    if case.motion is not None:
        s.set_poses(case.poses(ref["t"]))
        s.assemble(case.overset["wrule"], case.overset["overlap"])
        types, rec, ptr, don, w = ref["tables"]
        srec, sptr, sdon, sw = s.overset()
        assert np.array_equal(s.types(), types)
        assert np.array_equal(srec, rec) and np.array_equal(sptr, ptr) and np.array_equal(sdon, don)
        assert np.abs(sw - w).max(initial=0.0) <= 1e-15
        say("  assembly bit-exact:", len(rec), "receptors,", int(np.sum(types == 0)), "holes")
    dt_t = torch.float64 if prec == ugks.F64 else torch.float32
    x = ref["inputs"]
    h, b, W, q = dev(x["h"], dt_t), dev(x["b"], dt_t), dev(x["W"]), dev(x["q"])
    dts, _ = s.timesteps()
    dt = case.dt if case.dt is not None else case.dt_over_dts * dts
    Wn = W.clone()
    Sh, Sb, Fn = s.begin_step(dt, h, b, W, q)
    # the benchmark's launch shapes, chosen on copies of this state
    tuning, _ = s.autotune(dt, 1, h, b, W, Wn, q, Sh, Sb, Fn)
    s.step_graph(dt, 1, h, b, W, Wn, q, Sh, Sb, Fn)
    torch.cuda.synchronize()
    f = ref["live"]
    out = ref["out"]
    e = [rel_l2(host(t)[f], out[k][f]) for k, t in (("h", h), ("b", b), ("W", W), ("q", q))]
    # the change over the step alone (a stricter measure where the step
    # moves f little)
    ch = rel_l2(host(h)[f] - x["h"][f], out["h"][f] - x["h"][f])
    say("  launch shapes", tuning, " rel L2 h b W q", e, " change of h", ch)
    s.close()
    assert max(e[:3]) <= tol
    assert e[3] <= max(tol, 1e-9)
    if prec == ugks.F64:
        assert ch <= 1e-9


@pytest.fixture(scope="module")
def cylinder_ref():
    return _oracle_step(wl.cylinder(), lambda o: o.init_state(), 0.0)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec,tol", [(ugks.F64, 1e-10), (ugks.F32, 1e-5)], ids=["f64", "f32"])
def test_cylinder_full_size_step(cylinder_ref, prec, tol):
    case = cylinder_ref["case"]
    say("full-size cylinder", "f64" if prec == ugks.F64 else "f32", case.ncell * case.nv, "pairs")
    _gpu_step(cylinder_ref, prec, tol)


def _perturbed(case):
    def state(o):
        h, b, W = wl.synthetic_f(case, amp=0.02)
        return h, b, W, o.heatflux(h, b, W)
    return state


@pytest.fixture(scope="module", params=[0.1, 1.0], ids=["kn0.1", "kn1"])
def plate_ref(request):
    case = wl.mems_plate(kn=request.param)
    return _oracle_step(case, _perturbed(case), case.dt)


@pytest.mark.timeout(400)
@pytest.mark.parametrize("prec,tol", [(ugks.F64, 1e-10), (ugks.F32, 1e-5)], ids=["f64", "f32"])
def test_mems_plate_full_size_step(plate_ref, prec, tol):
    case = plate_ref["case"]
    say("full-size MEMS plate", case.mu_ref, "f64" if prec == ugks.F64 else "f32", case.ncell * case.nv, "pairs")
    _gpu_step(plate_ref, prec, tol)


# ----------------------------------------------------------------------------
# Two-body separation at full size (512 x 256 background, two 128 x 96
# O-meshes, 100 x 100 velocities: 1.56 G pairs).  The whole oracle step would
# take minutes on the host, so Steps 1-2 (interpolation, flux, source) are
# compared at a sample of cells, each computed by the oracle on its own, and
# the level-n face flux at the sample's faces; the assembly is compared whole.

def _sample_cells(case, types, rec, don, rng):
    cell0 = np.cumsum([0] + [B.ncell for B in case.blocks])
    pick = []
    for b in range(len(case.blocks)):  # anywhere in each block
        field = np.nonzero(types[cell0[b]:cell0[b + 1]] == 1)[0] + cell0[b]
        pick.append(rng.choice(field, 64, replace=False))
    for b in (1, 2):  # beside each wall (j = 0 ring)
        ring = cell0[b] + np.arange(case.blocks[b].ni)
        pick.append(rng.choice(ring[types[ring] == 1], 32, replace=False))
    # donors of receptors: field cells whose stencils reach the overset rows
    d = np.unique(don)
    pick.append(rng.choice(d[types[d] == 1], 64, replace=False))
    return np.unique(np.concatenate(pick)).astype(np.int32)


@pytest.fixture(scope="module")
def two_body_ref():
    case = wl.two_body()
    t = 0.25
    o = Oracle(case)
    o.set_poses(case.poses(t))
    rc, _ = o.assemble(case.overset["wrule"], case.overset["overlap"])
    assert rc == 0
    types = o.types()
    rec, ptr, don, w = o.overset()
    h, b, W = wl.synthetic_f(case, amp=0.02)
    q = o.heatflux(h, b, W)
    dts, _ = o.timesteps()
    dt = case.dt_over_dts * dts
    cells = _sample_cells(case, types, rec, don, np.random.default_rng(11))
    # the oracle interpolates into the table's rows in place: keep the inputs
    keep = [a[rec].copy() for a in (h, b, W, q)]
    sh, sb, fc = o.begin_step_cells(dt, dts, h, b, W, q, cells)
    for a, k in zip((h, b, W, q), keep):
        a[rec] = k
    return dict(case=case, t=t, h=h, b=b, W=W, q=q, dt=dt, cells=cells, sh=sh, sb=sb, fc=fc,
                tables=(types, rec, ptr, don, w), face_index=o.product_face_index(), cface=_cell_faces(o))


def _cell_faces(o):
    g = o.geometry()
    _, dr, _, _ = o.face_ids()
    cf = -np.ones((o.ncell, 4), np.int64)
    L, R = g["fl"], g["fr"]
    f = np.arange(o.nface)
    cf[L[L >= 0], 2 * dr[L >= 0] + 1] = f[L >= 0]
    cf[R[R >= 0], 2 * dr[R >= 0]] = f[R >= 0]
    return cf


@pytest.mark.timeout(400)
@pytest.mark.parametrize("prec,tol", [(ugks.F64, 1e-10), (ugks.F32, 1e-5)], ids=["f64", "f32"])
def test_two_body_full_size_sampled(two_body_ref, prec, tol):
    ref = two_body_ref
    case = ref["case"]
    say("full-size two-body", "f64" if prec == ugks.F64 else "f32", case.ncell * case.nv, "pairs,",
        len(ref["cells"]), "sampled cells")
    s = ugks.Solver(case, prec)
    s.set_poses(case.poses(ref["t"]))
    s.assemble(case.overset["wrule"], case.overset["overlap"])
    types, rec, ptr, don, w = ref["tables"]
    srec, sptr, sdon, sw = s.overset()
    assert np.array_equal(s.types(), types)
    assert np.array_equal(srec, rec) and np.array_equal(sptr, ptr) and np.array_equal(sdon, don)
    assert np.abs(sw - w).max(initial=0.0) <= 1e-15
    say("  assembly bit-exact:", len(rec), "receptors,", int(np.sum(types == 0)), "holes")
    dt_t = torch.float64 if prec == ugks.F64 else torch.float32
    h, b = dev(ref["h"], dt_t), dev(ref["b"], dt_t)
    W, q = dev(ref["W"]), dev(ref["q"])
    Sh, Sb, Fn = s.begin_step(ref["dt"], h, b, W, q)
    idx = torch.tensor(ref["cells"], dtype=torch.int64, device="cuda")
    e_sh = rel_l2(host(Sh.index_select(0, idx)), ref["sh"])
    e_sb = rel_l2(host(Sb.index_select(0, idx)), ref["sb"])
    cf = ref["cface"][ref["cells"]]
    have = cf >= 0
    Fg = host(Fn)[ref["face_index"][cf[have]]]
    e_f = rel_l2(Fg, ref["fc"][have])
    say("  Steps 1-2 at the sample: rel L2 Sh", e_sh, "Sb", e_sb, "face flux", e_f)
    assert max(e_sh, e_sb, e_f) <= tol
    # one inner iteration through the autotuned captured graph at this size:
    # the path runs whole and keeps the state physical
    Wn = W.clone()
    tuning, ms = s.autotune(ref["dt"], 1, h, b, W, Wn, q, Sh, Sb, Fn)
    resid = torch.zeros(case.nw, dtype=torch.float64, device="cuda")
    s.step_graph(ref["dt"], 1, h, b, W, Wn, q, Sh, Sb, Fn, resid=resid)
    torch.cuda.synchronize()
    Wh = host(W)[types == 1]
    r = host(resid)
    say("  launch shapes", tuning, f"{ms:.1f} ms per inner iteration, residual", r)
    assert np.all(np.isfinite(r)) and np.all(np.isfinite(Wh)) and Wh[:, 0].min() > 0
    assert bool(torch.isfinite(h).all())
    s.close()


# ----------------------------------------------------------------------------
# The 64-case batch (ragged cavities and plates, 0.97 G pairs in all): every
# case advanced by the batch graph equals its own captured-graph step bit for
# bit, and three cases (the smallest, the median and the largest) equal the
# oracle's Steps 1-2 and one inner iteration.

@pytest.fixture(scope="module")
def batch_ref():
    cases = wl.batch_cases(64)
    pairs = np.array([c.ncell * c.nv for c in cases])
    order = np.argsort(pairs, kind="stable")
    pick = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    refs = {i: _oracle_step(cases[i], _perturbed(cases[i]), 0.0) for i in pick}
    return cases, refs, int(pairs.sum())


@pytest.mark.timeout(400)
@pytest.mark.parametrize("prec,tol", [(ugks.F32, 1e-5), (ugks.F64, 1e-10)], ids=["f32", "f64"])
def test_batch_full_size(batch_ref, prec, tol):
    cases, refs, total = batch_ref
    say("full-size batch", len(cases), "cases,", total, "pairs,", "f64" if prec == ugks.F64 else "f32")
    dt_t = torch.float64 if prec == ugks.F64 else torch.float32
    solvers = [ugks.Solver(c, prec) for c in cases]
    dts, states = [], []
    for i, (c, s) in enumerate(zip(cases, solvers)):
        if i in refs:
            x = refs[i]["inputs"]
            h, b, W, q = dev(x["h"], dt_t), dev(x["b"], dt_t), dev(x["W"]), dev(x["q"])
        else:
            h, b, W, q = s.init_state()
        d, _ = s.timesteps()
        dt = c.dt_over_dts * d
        Wn = W.clone()
        Sh, Sb, Fn = s.begin_step(dt, h, b, W, q)
        s.autotune(dt, 1, h, b, W, Wn, q, Sh, Sb, Fn)
        dts.append(dt)
        states.append([h, b, W, Wn, q, Sh, Sb, Fn])
    own = [[t.clone() for t in st] for st in states]
    batch = ugks.Batch(solvers)
    batch.step(dts, 1, states)
    for s, st, dt in zip(solvers, own, dts):
        s.step_graph(dt, 1, *st)
    torch.cuda.synchronize()
    for i in range(len(cases)):
        assert all(torch.equal(a, b) for a, b in zip(states[i][:5], own[i][:5])), cases[i].name
    for i, ref in refs.items():
        f = ref["live"]
        out = ref["out"]
        e = [rel_l2(host(t)[f], out[k][f]) for k, t in zip("hbW", states[i][:3])]
        say(" ", cases[i].name, "rel L2 h b W", e)
        assert max(e) <= tol
    batch.close()
    for s in solvers:
        s.close()
