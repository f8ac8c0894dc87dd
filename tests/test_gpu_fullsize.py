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
