"""Captured pseudo-iterations, batches of cases and launch-shape tuning of
the HIP path (through the C ABI): all give results bit-identical to the
eager ugks_step, which the other GPU tests hold to the oracle.

Graph replays are checked replay by replay, with eager work and
synchronisations of the program between them."""
import numpy as np
import pytest
import torch

from paper_2604_09984_amd import ugks, workloads as wl
from tests.parity import dev, host, say

pytestmark = pytest.mark.gpu


def _state(s, case, prec):
    h, b, W = wl.synthetic_f(case, amp=0.02)
    dt_t = torch.float64 if prec == ugks.F64 else torch.float32
    hd, bd, Wd = dev(h, dt_t), dev(b, dt_t), dev(W)
    qd = s.heatflux(hd, bd, Wd)
    dts, _ = s.timesteps()
    dt = case.dt if case.dt is not None else case.dt_over_dts * dts
    Wn = Wd.clone()
    Sh, Sb, Fn = s.begin_step(dt, hd, bd, Wd, qd)
    return dt, [hd, bd, Wd, Wn, qd, Sh, Sb, Fn]


def _clone(st):
    return [t.clone() for t in st]


def _equal(a, b):
    torch.cuda.synchronize()
    assert all(bool(torch.isfinite(x).all()) for x in a), "non-finite state"
    return all(torch.equal(x, y) for x, y in zip(a, b))


def _cyl():
    c = wl.cylinder(ni=16, nj=8, nvx=16)
    c.dt_over_dts = 5.0  # stays smooth over the repeated replays
    return c


CASES = [_cyl(), wl.cavity(8, 12), wl.periodic_box(2, 8, 6, 10)]


@pytest.mark.parametrize("prec", [ugks.F64, ugks.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("case", CASES, ids=[c.name for c in CASES])
def test_graph_replays_match_eager(case, prec):
    say("graph", case.name, prec)
    s = ugks.Solver(case, prec)
    dt, st0 = _state(s, case, prec)
    eager, graph = _clone(st0), _clone(st0)
    re = torch.zeros((3, case.nw), dtype=torch.float64, device="cuda")
    rg = torch.zeros_like(re)
    for rep in range(3):
        s.step(dt, 3, *eager[:3], eager[3], eager[4], *eager[5:], re)
        s.step_graph(dt, 3, *graph[:3], graph[3], graph[4], *graph[5:], rg)
        # eager work of the program between replays
        junk = torch.ones(1000, device="cuda").cumsum(0)
        torch.cuda.synchronize()
        assert _equal(eager, graph), f"replay {rep}"
        assert torch.equal(re, rg)
        del junk
    # a changed dt is captured again
    s.step(0.5 * dt, 2, *eager[:3], eager[3], eager[4], *eager[5:])
    s.step_graph(0.5 * dt, 2, *graph[:3], graph[3], graph[4], *graph[5:])
    assert _equal(eager, graph)
    s.close()


def test_graph_after_motion_and_assembly():
    """Geometry and donor tables change between replays: the graph follows."""
    case = wl.overset_patch(ni_bg=16, npatch=14, half=0.55, nv=8)
    s = ugks.Solver(case, ugks.F64)
    eager = graph = None
    t = 0.0
    for n in range(3):
        t += case.dt
        s.set_poses(case.poses(t))
        s.assemble(0, 2)
        if eager is None:
            dt, st0 = _state(s, case, ugks.F64)
            eager, graph = _clone(st0), _clone(st0)
        s.step(case.dt, 2, *eager[:3], eager[3], eager[4], *eager[5:])
        s.step_graph(case.dt, 2, *graph[:3], graph[3], graph[4], *graph[5:])
        assert _equal(eager, graph), f"step {n}"
    s.close()


@pytest.mark.parametrize("mode,prec", [(1, ugks.F64), (1, ugks.F32), (0, ugks.F64)],
                         ids=["one_launch_per_stage_f64", "one_launch_per_stage_f32", "branches_f64"])
def test_batch_matches_individual_steps(mode, prec):
    """Ragged cases (cylinder, cavities, a box periodic in both directions,
    a 70-row channel) advanced by the batch graph equal each case's own
    pseudo-iterations bit for bit, over two replays."""
    cases = [_cyl(), wl.cavity(8, 12), wl.periodic_box(2, 8, 6, 10),
             wl.cavity(6, 10, periodic_x=True), wl.channel(6, 70, 8)]
    solvers = [ugks.Solver(c, prec) for c in cases]
    states, dts, ref = [], [], []
    for c, s in zip(cases, solvers):
        dt, st = _state(s, c, prec)
        dts.append(dt)
        states.append(_clone(st))
        ref.append(_clone(st))
    batch = ugks.Batch(solvers, mode=mode)
    assert batch.mode == mode
    resid = [torch.zeros((3, c.nw), dtype=torch.float64, device="cuda") for c in cases]
    rref = [torch.zeros_like(r) for r in resid]
    for rep in range(2):
        for s, st, dt, r in zip(solvers, ref, dts, rref):
            s.step(dt, 3, *st[:3], st[3], st[4], *st[5:], r)
        batch.step(dts, 3, states, resid)
        torch.cuda.synchronize()
        for i in range(len(cases)):
            assert _equal(states[i], ref[i]), f"case {cases[i].name} replay {rep}"
            assert torch.equal(resid[i], rref[i])
    batch.close()
    for s in solvers:
        s.close()


@pytest.mark.parametrize("prec", [ugks.F64, ugks.F32], ids=["f64", "f32"])
def test_tuning_does_not_change_results(prec):
    case = _cyl()
    s = ugks.Solver(case, prec)
    dt, st0 = _state(s, case, prec)
    out = None
    for kc in (16, 8, 4):
        for re_ in (10, 8, 6):
            for rf in (10, 8, 6):
                s.set_tuning(kc, re_, rf)
                assert s.tuning() == (kc, re_, rf)
                # 128 x 64 cells: one row per thread; chunks of 8 or more
                # velocities form the residual inside the forward sweep
                assert s.micro_shape() == ((kc, 1, 2, 1) if kc >= 8 else (kc, 1, 3, 0))
                st = _clone(st0)
                s.step(dt, 2, *st[:3], st[3], st[4], *st[5:])
                if out is None:
                    out = st
                else:
                    assert _equal(out, st), (kc, re_, rf)
    with pytest.raises(ugks.UgksError):
        s.set_tuning(32, 8, 8)
    with pytest.raises(ugks.UgksError):
        s.set_tuning(16, 12, 8)
    with pytest.raises(ugks.UgksError):
        s.set_tuning(16, 8, 4)
    st = _clone(st0)
    choice, ms = s.autotune(dt, 2, *st[:3], st[3], st[4], *st[5:])
    say("autotune", choice, ms)
    assert choice[0] in (16, 8, 4) and choice[1] in (10, 8, 6) and choice[2] in (10, 8, 6) and ms > 0
    assert s.tuning() == choice
    assert _equal(st, st0)  # the caller's state is not written
    s.close()


def test_batch_mode_rules():
    """One launch per stage needs 2D cases of one storage type; a batch with
    a 1D case keeps the branch graph."""
    s1 = ugks.Solver(wl.sod_1d(ncell=20, nv=13), ugks.F64)
    s2 = ugks.Solver(wl.cavity(6, 8), ugks.F64)
    s3 = ugks.Solver(wl.cavity(6, 8), ugks.F32)
    for group in ([s1, s2], [s2, s3]):
        b = ugks.Batch(group)
        assert b.mode == 0
        with pytest.raises(ugks.UgksError):
            b.set_mode(1)
        with pytest.raises(ugks.UgksError):
            b.set_mode(2)
        b.close()
    for s in (s1, s2, s3):
        s.close()
