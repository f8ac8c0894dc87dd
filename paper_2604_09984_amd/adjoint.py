"""Differentiable dual-time stepping: torch.autograd.Function wrappers of the
library's hand-written adjoint (reverse mode of Sec. 2.2's Steps 1-2 and of
the inner iteration, Steps 3-7) and checkpointed recomputation across
dual-time steps.

Argument marshalling only: every forward and reverse pass runs in the HIP
library (ugks_begin_step, ugks_step, ugks_begin_step_adjoint,
ugks_step_adjoint).  Differentiable inputs are the state (h, b, W, q), the
dual-time inputs of an inner iteration (Wn, Sh, Sb, Fn) and two sets of
parameters of the prescribed motion and boundaries:

  U    [nblock][2]  rigid velocity of each block (the face grid velocity and
                    wall velocity of its faces; node positions, dt_s and dt'
                    are those of the block's pose and are not differentiated),
  rtw  [nblock][4]  RT of the isothermal wall on each side of each block
                    (entries of sides that are not walls are ignored).

U and rtw are float64 tensors on any device; their gradients come back on the
same device.  Objectives are functions of the returned states and of F, the
face macro flux of the last inner iteration (wall force, moment and heat
flux per block side: wall_loads(), computed by the library).

Checkpointing: physical_step() stores only its inputs; its backward re-runs
the step's forward (Steps 1-2 and the n_inner inner iterations) and then
the reverse passes, keeping all inner states or, with inner_snapshots=c, at
most c of them at a time (binomial checkpointing over the inner
iterations).  rollout() runs a whole sequence of physical steps as one node
that keeps only its inputs and, in its backward, at most `snapshots` states
of the sequence at a time: the steps are re-run from the nearest kept state
in the order of a binomial checkpointing schedule (revolve_schedule), which
re-runs the fewest steps any schedule with that many kept states can
(Griewank and Walther's bound, revolve_cost).  The kernels sum in a fixed
order, so every schedule gives the same bits.  A `setup` callable restores the
step's geometry (poses, overset assembly) before the forward and before the
recomputation, so moving-mesh runs are differentiated step by step; it is
called as setup(solver) when it takes an argument, else as setup().

FP32 storage: the library's reverse passes work on FP64 storage, so the
backward of a solver with FP32 storage runs on an FP64 twin context of the
same case: the checkpointed step is recomputed there from the (exactly
representable) FP32 inputs, and the gradients are those of the FP64 map at
those inputs, returned in the inputs' dtypes.  The twin takes the solver's
poses, cell kinds and donor table (or, with a setup, runs setup(twin), so a
moving FP32 run needs a setup that takes the solver).
"""
from __future__ import annotations

import inspect
from math import comb

import numpy as np
import torch

from . import ugks


# --------------------------------------------------------------------------
# wall loads (computed by the library) as a differentiable function of F
# --------------------------------------------------------------------------
def _positions(solver):
    poses = getattr(solver, "poses", None)
    return None if poses is None else poses[:, :3].copy()


class WallLoads(torch.autograd.Function):
    """F [nface][dim+2] -> side loads [nblock][4][4] (force x, y, moment,
    energy flux into the walls of each block side; ugks_wall_loads).  The
    map depends on the wall faces' areas, normals and moment arms at the
    solver's pose; its reverse uses the solver's geometry when it runs, so
    the pose must not have changed in between (on moving meshes take the
    loads from physical_step(loads=True) or rollout, whose reverse restores
    each step's geometry)."""

    @staticmethod
    def forward(ctx, solver, F):
        _, side = solver.wall_loads(F)
        ctx.solver = solver
        ctx.pos = _positions(solver)
        return side

    @staticmethod
    def backward(ctx, g):
        pos = _positions(ctx.solver)
        if (pos is None) != (ctx.pos is None) or (pos is not None and not np.array_equal(pos, ctx.pos)):
            raise ValueError("wall loads differentiated at another pose than they were formed at: take them "
                             "from physical_step(loads=True) or rollout")
        return None, ctx.solver.wall_loads_adjoint(side_bar=g.contiguous())


def wall_loads(solver, F):
    """Differentiable side loads of a face macro flux (see WallLoads)."""
    return WallLoads.apply(solver, F)


def _param_grads(solver, face_bar):
    """Block velocity and wall-RT cotangents from per-face cotangents
    (ugks_param_bars)."""
    return solver.param_bars(face_bar)


def apply_params(solver, U, rtw):
    """Set the block velocities and wall temperatures (angular velocities from
    the current poses are kept; dt_s and dt' stay fixed)."""
    if U is not None:
        Uh = U.detach().double().cpu().numpy()
        poses = getattr(solver, "poses", None)
        for b in range(len(solver.case.blocks)):
            solver.set_block_velocity(b, Uh[b, 0], Uh[b, 1], 0.0 if poses is None else poses[b, 5])
    if rtw is not None:
        Rh = rtw.detach().double().cpu().numpy()
        for b, B in enumerate(solver.case.blocks):
            for s in range(4):
                if B.bc[s] == 3:
                    solver.set_wall_rt(b, s, Rh[b, s])


def _out_grad(U, g):
    return None if U is None else g.to(U.device, U.dtype)


def _run_setup(setup, solver):
    if setup is None:
        return
    try:
        takes = len(inspect.signature(setup).parameters) > 0
    except (TypeError, ValueError):
        takes = False
    if takes:
        setup(solver)
    elif getattr(solver, "_adj_owner", None) is not None:
        raise ValueError("the FP64 twin of an FP32 solver needs a setup(solver) that takes the solver")
    else:
        setup()


def _twin(solver):
    """The context that runs the reverse passes: the solver itself (FP64
    storage) or its FP64 twin (FP32 storage)."""
    if solver.prec == ugks.F64:
        return solver
    t = getattr(solver, "_adj_twin", None)
    if t is None:
        t = ugks.Solver(solver.case, ugks.F64, device=solver.device.index)
        t._adj_owner = solver
        solver._adj_twin = t
    return t


def _mirror(src, dst):
    """dst takes src's poses, cell kinds and receptor donor table."""
    if dst is src:
        return
    poses = getattr(src, "poses", None)
    if poses is not None:
        dst.set_poses(poses)
    dst.set_types(src.types())
    rec, ptr, don, w = src.overset()
    if len(rec) > 0:
        dst.set_overset(rec, ptr, don, w)


def _f64(t):
    return None if t is None else t.double().contiguous()


def _as(t, like):
    return t if t.dtype == like.dtype else t.to(like.dtype)


def _clone(*ts):
    return [t.clone() for t in ts]


# --------------------------------------------------------------------------
# one inner iteration and Steps 1-2
# --------------------------------------------------------------------------
class PseudoStep(torch.autograd.Function):
    """(h, b, W, q, Wn, Sh, Sb, Fn, U, rtw) -> (h', b', W', q', F): one inner
    iteration (Steps 3-7); F is the face macro flux of its Step 3."""

    @staticmethod
    def forward(ctx, solver, dt, setup, h, b, W, q, Wn, Sh, Sb, Fn, U, rtw):
        _run_setup(setup, solver)
        apply_params(solver, U, rtw)
        h1, b1, W1, q1 = _clone(h, b, W, q)
        solver.step(dt, 1, h1, b1, W1, Wn, q1, Sh, Sb, Fn)
        F = solver.last_flux()
        ctx.solver, ctx.dt, ctx.setup = solver, dt, setup
        ctx.save_for_backward(h, b, W, q, Wn, Sh, Sb, Fn, U, rtw)
        return h1, b1, W1, q1, F

    @staticmethod
    def backward(ctx, gh, gb, gW, gq, gF):
        h, b, W, q, Wn, Sh, Sb, Fn, U, rtw = ctx.saved_tensors
        s = ctx.solver
        _run_setup(ctx.setup, s)
        t = _twin(s)
        _mirror(s, t)
        apply_params(t, U, rtw)
        hb, bb, Wb, Wnb, qb, Shb, Sbb, Fnb, fb = t.step_adjoint(ctx.dt, _f64(h), _f64(b), W, Wn, q, _f64(Sh),
                                                                 _f64(Sb), Fn, _f64(gh), _f64(gb), _c(gW),
                                                                 _c(gq), _c(gF))
        gU, gR = _param_grads(t, fb)
        return (None, None, None, _as(hb, h), _as(bb, b), Wb, qb, Wnb, _as(Shb, Sh), _as(Sbb, Sb), Fnb,
                _out_grad(U, gU), _out_grad(rtw, gR))


class BeginStep(torch.autograd.Function):
    """(h, b, W, q, U, rtw) -> (h', b', W', q', Sh, Sb, Fn): Steps 1-2 (the
    primed state has its receptor rows, and once after an assembly the cells
    uncovered from holes, interpolated)."""

    @staticmethod
    def forward(ctx, solver, dt, setup, h, b, W, q, U, rtw):
        _run_setup(setup, solver)
        apply_params(solver, U, rtw)
        ctx.refill = solver.overset_rows()[2] != 0
        if ctx.refill and solver.prec != ugks.F64:
            raise ValueError("cells to refill with FP32 storage: use the checkpointed physical_step")
        h1, b1, W1, q1 = _clone(h, b, W, q)
        Sh, Sb, Fn = solver.begin_step(dt, h1, b1, W1, q1)
        ctx.solver, ctx.dt, ctx.setup = solver, dt, setup
        ctx.save_for_backward(h, b, W, q, U, rtw)
        return h1, b1, W1, q1, Sh, Sb, Fn

    @staticmethod
    def backward(ctx, gh, gb, gW, gq, gSh, gSb, gFn):
        h, b, W, q, U, rtw = ctx.saved_tensors
        s = ctx.solver
        _run_setup(ctx.setup, s)
        t = _twin(s)
        _mirror(s, t)
        apply_params(t, U, rtw)
        hb, bb, Wb, qb, fb = t.begin_step_adjoint(ctx.dt, _f64(h), _f64(b), W, q, _f64(gh), _f64(gb), _c(gW),
                                                  _c(gq), _f64(gSh), _f64(gSb), _c(gFn), refill=ctx.refill)
        gU, gR = _param_grads(t, fb)
        return None, None, None, _as(hb, h), _as(bb, b), Wb, qb, _out_grad(U, gU), _out_grad(rtw, gR)


def _c(t):
    return None if t is None else t.contiguous()


# --------------------------------------------------------------------------
# binomial checkpointing schedules
# --------------------------------------------------------------------------
def revolve_cost(n, c):
    """Fewest forward steps that reverse a chain of n steps when at most c
    states beyond the chain's input are held at once: r n - C(c + r, c + 1)
    with r the least integer such that C(c + r, c) >= n (for c >= 2; c <= 1:
    every step re-run from the input, n (n - 1) / 2)."""
    if n <= 1:
        return 0
    if c <= 1:
        return n * (n - 1) // 2
    r = 0
    while comb(c + r, c) < n:
        r += 1
    return r * n - comb(c + r, c + 1)


def revolve_schedule(n, c):
    """Actions that reverse steps n-1, ..., 0 of a chain whose input (state
    0) is held, keeping at most max(c, 1) further states:
    ("advance", a, m): run steps a .. m-1 from the held state a and hold
    state m; ("reverse", k): reverse step k from the held state k;
    ("free", m): drop state m.  Each split is chosen so that the schedule's
    forward steps equal revolve_cost(n, c)."""
    acts = []

    def rev(a, n, c):
        while True:
            if n == 1:
                acts.append(("reverse", a))
                return
            if c <= 1:
                for k in range(a + n - 1, a, -1):
                    acts.extend((("advance", a, k), ("reverse", k), ("free", k)))
                acts.append(("reverse", a))
                return
            m = min(range(1, n), key=lambda m: (m + revolve_cost(n - m, c - 1) + revolve_cost(m, c), -m))
            acts.append(("advance", a, a + m))
            rev(a + m, n - m, c - 1)
            acts.append(("free", a + m))
            n = m

    if n > 0:
        rev(0, n, c)
    return acts


def _run_schedule(n, c, state0, advance, reverse):
    """Execute revolve_schedule(n, c): advance(a, state_a, m) returns state
    m (a new object), reverse(k, state_k) reverses step k.  Returns the
    number of forward steps re-run."""
    held = {0: state0}
    steps = 0
    for act in revolve_schedule(n, c):
        if act[0] == "advance":
            _, a, m = act
            held[m] = advance(a, held[a], m)
            steps += m - a
        elif act[0] == "reverse":
            reverse(act[1], held[act[1]])
        else:
            del held[act[1]]
    return steps


# --------------------------------------------------------------------------
# one physical step, checkpointed
# --------------------------------------------------------------------------
def _prepare(solver, setup, types0, U, rtw):
    """A step's geometry on solver: the cell kinds it started from (types0,
    when re-running it), its setup, the parameters."""
    if setup is not None and types0 is not None:
        solver.set_types(types0)
    _run_setup(setup, solver)
    apply_params(solver, U, rtw)


def _forward_step(solver, dt, n_inner, h, b, W, q):
    """Steps 1-2 and n_inner inner iterations, in place; returns F of the
    last inner iteration."""
    Wn = W.clone()
    Sh, Sb, Fn = solver.begin_step(dt, h, b, W, q)
    for _ in range(n_inner):
        solver.step(dt, 1, h, b, W, Wn, q, Sh, Sb, Fn)
    return solver.last_flux()


def _step_reverse(solver, dt, n_inner, setup, types0, refill, state, U, rtw, g, gF, gL, inner_snapshots):
    """Reverse of one physical step from its input state: the step is re-run
    (on the FP64 context) and its inner iterations reversed in the order of
    revolve_schedule(n_inner, inner_snapshots) (None: all inner states
    kept), then Steps 1-2.  g: cotangents of the step's output state
    (entries may be None), gF: of F, gL: of the side loads of F (taken at
    the step's geometry).  Returns the input-state cotangents and the
    parameter cotangents."""
    h, b, W, q = state
    s = _twin(solver)
    if setup is not None:
        s.set_types(types0)
        _run_setup(setup, s)
    else:
        _mirror(solver, s)
    apply_params(s, U, rtw)
    if gL is not None:
        gFl = s.wall_loads_adjoint(side_bar=gL.contiguous())
        gF = gFl if gF is None else gF + gFl
    h_in, b_in = h, b
    h, b = _f64(h), _f64(b)
    x0 = _clone(h, b, W, q)
    Wn = W.clone()
    Sh, Sb, Fn = s.begin_step(dt, *x0)
    cur = [_f64(g[0]), _f64(g[1]), _c(g[2]), _c(g[3])]
    gSh = torch.zeros_like(Sh); gSb = torch.zeros_like(Sb)
    gFn = torch.zeros_like(Fn); gWn = torch.zeros_like(W)
    faces = torch.zeros((s.nface, 5), dtype=torch.float64, device=h.device)

    def advance(a, st, m):
        x = _clone(*st)
        for _ in range(a, m):
            s.step(dt, 1, x[0], x[1], x[2], Wn, x[3], Sh, Sb, Fn)
        return x

    def reverse(k, st):
        out = s.step_adjoint(dt, st[0], st[1], st[2], Wn, st[3], Sh, Sb, Fn, *cur,
                             _c(gF) if k == n_inner - 1 else None)
        cur[:] = out[0], out[1], out[2], out[4]
        gWn.add_(out[3]); gSh.add_(out[5]); gSb.add_(out[6]); gFn.add_(out[7]); faces.add_(out[8])

    c = n_inner if inner_snapshots is None else inner_snapshots
    _run_schedule(n_inner, c, x0, advance, reverse)
    del x0
    # Steps 1-2 (Wn is the input W)
    hb, bb, Wb, qb, fb = s.begin_step_adjoint(dt, h, b, W, q, *cur, gSh, gSb, gFn, refill=refill)
    faces += fb
    Wb = Wb + gWn
    gU, gR = _param_grads(s, faces)
    return _as(hb, h_in), _as(bb, b_in), Wb, qb, gU, gR


class PhysicalStep(torch.autograd.Function):
    """(h, b, W, q, U, rtw) -> (h', b', W', q', F, L): Steps 1-8 of one
    physical step (Steps 1-2, then n_inner inner iterations); F is the face
    macro flux of the last inner iteration, L its side loads at the step's
    geometry (ugks_wall_loads).  Only the inputs are kept; the backward pass
    recomputes the step."""

    @staticmethod
    def forward(ctx, solver, dt, n_inner, setup, inner_snapshots, h, b, W, q, U, rtw):
        # the cell kinds before the step's setup decide which cells an
        # overset assembly refills; the recomputation restores them
        ctx.types0 = solver.types() if setup is not None else None
        _prepare(solver, setup, None, U, rtw)
        ctx.refill = solver.overset_rows()[2] != 0
        h1, b1, W1, q1 = _clone(h, b, W, q)
        F = _forward_step(solver, dt, n_inner, h1, b1, W1, q1)
        L = solver.wall_loads(F)[1]
        ctx.solver, ctx.dt, ctx.n_inner, ctx.setup, ctx.inner = solver, dt, n_inner, setup, inner_snapshots
        ctx.save_for_backward(h, b, W, q, U, rtw)
        return h1, b1, W1, q1, F, L

    @staticmethod
    def backward(ctx, gh, gb, gW, gq, gF, gL):
        h, b, W, q, U, rtw = ctx.saved_tensors
        hb, bb, Wb, qb, gU, gR = _step_reverse(ctx.solver, ctx.dt, ctx.n_inner, ctx.setup, ctx.types0, ctx.refill,
                                               (h, b, W, q), U, rtw, (gh, gb, gW, gq), gF, gL, ctx.inner)
        return None, None, None, None, None, hb, bb, Wb, qb, _out_grad(U, gU), _out_grad(rtw, gR)


class Rollout(torch.autograd.Function):
    """(h, b, W, q, U, rtw) -> (h_N, b_N, W_N, q_N, F[N], L[N]): a sequence
    of N physical steps (each as PhysicalStep; F[k] the face macro flux of
    step k's last inner iteration, L[k] its side loads).  Only the inputs and each step's time step,
    cell kinds and refill flag are kept; the backward pass re-runs steps
    from the nearest kept state, holding at most `snapshots` states of the
    sequence at once (revolve_schedule)."""

    @staticmethod
    def forward(ctx, solver, steps, snapshots, inner_snapshots, stats, h, b, W, q, U, rtw):
        recs = []
        x = _clone(h, b, W, q)
        Fs, Ls = [], []
        for dt, n_inner, setup in steps:
            types0 = solver.types() if setup is not None else None
            _prepare(solver, setup, None, U, rtw)
            dt = float(dt(solver)) if callable(dt) else float(dt)
            refill = solver.overset_rows()[2] != 0
            Fs.append(_forward_step(solver, dt, n_inner, *x))
            Ls.append(solver.wall_loads(Fs[-1])[1])
            recs.append((dt, int(n_inner), setup, types0, refill))
        ctx.solver, ctx.recs, ctx.snapshots, ctx.inner, ctx.stats = solver, recs, snapshots, inner_snapshots, stats
        ctx.save_for_backward(h, b, W, q, U, rtw)
        return x[0], x[1], x[2], x[3], torch.stack(Fs), torch.stack(Ls)

    @staticmethod
    def backward(ctx, gh, gb, gW, gq, gFs, gLs):
        h, b, W, q, U, rtw = ctx.saved_tensors
        solver, recs = ctx.solver, ctx.recs
        g = [gh, gb, gW, gq]
        par = [None, None]

        def advance(a, st, m):
            x = _clone(*st)
            for k in range(a, m):
                dt, n_inner, setup, types0, _ = recs[k]
                _prepare(solver, setup, types0, U, rtw)
                _forward_step(solver, dt, n_inner, *x)
            return x

        def reverse(k, st):
            dt, n_inner, setup, types0, refill = recs[k]
            gF = None if gFs is None else gFs[k]
            gL = None if gLs is None else gLs[k]
            hb, bb, Wb, qb, gU, gR = _step_reverse(solver, dt, n_inner, setup, types0, refill, st, U, rtw, g, gF, gL,
                                                   ctx.inner)
            g[:] = hb, bb, Wb, qb
            par[0] = gU if par[0] is None else par[0] + gU
            par[1] = gR if par[1] is None else par[1] + gR

        n = _run_schedule(len(recs), ctx.snapshots, (h, b, W, q), advance, reverse)
        if ctx.stats is not None:
            ctx.stats["recomputed_steps"] = n
        gU = None if par[0] is None else _out_grad(U, par[0])
        gR = None if par[1] is None else _out_grad(rtw, par[1])
        return None, None, None, None, None, g[0], g[1], g[2], g[3], gU, gR


def rollout(solver, steps, h, b, W, q, U=None, rtw=None, snapshots=2, inner_snapshots=None, stats=None):
    """N differentiable physical steps with binomial checkpointing; returns
    (h_N, b_N, W_N, q_N, F, L) with F [N][nface][dim+2] (F[k]: the face
    macro flux of step k's last inner iteration) and L [N][nblock][4][4]
    (its side loads at step k's geometry, as ugks_wall_loads forms them).  steps: one (dt, n_inner, setup)
    per physical step; dt may be a callable dt(solver), evaluated once after
    the step's setup.  The backward pass holds at most `snapshots` states of
    the sequence besides its input and re-runs revolve_cost(N, snapshots)
    steps; within a step, inner_snapshots bounds the inner states the same
    way (None: all kept).  stats (a dict) receives "recomputed_steps"."""
    return Rollout.apply(solver, list(steps), int(snapshots), inner_snapshots, stats, h, b, W, q, U, rtw)


def physical_step(solver, dt, n_inner, h, b, W, q, U=None, rtw=None, setup=None, checkpoint=True,
                  inner_snapshots=None, loads=False):
    """One differentiable physical step; returns (h', b', W', q', F), and
    with loads=True also L, the side loads of F at the step's geometry
    [nblock][4][4] (ugks_wall_loads; their reverse runs at that geometry).
    With checkpoint=False the step is composed of BeginStep and PseudoStep
    nodes whose inputs autograd keeps (n_inner states of f; fixed geometry).
    inner_snapshots bounds the inner states the checkpointed backward holds
    (None: all)."""
    if checkpoint:
        out = PhysicalStep.apply(solver, dt, n_inner, setup, inner_snapshots, h, b, W, q, U, rtw)
        return out if loads else out[:5]
    if setup is not None:
        raise ValueError("checkpoint=False keeps every node of the step for one geometry: no setup")
    Wn = W
    h, b, W, q, Sh, Sb, Fn = BeginStep.apply(solver, dt, setup, h, b, W, q, U, rtw)
    F = None
    for _ in range(n_inner):
        h, b, W, q, F = PseudoStep.apply(solver, dt, setup, h, b, W, q, Wn, Sh, Sb, Fn, U, rtw)
    return (h, b, W, q, F, wall_loads(solver, F)) if loads else (h, b, W, q, F)


def default_params(solver):
    """U and rtw tensors holding the block velocities of the solver's current
    poses (zero before any set_poses) and the case's wall temperatures (1 on
    sides that are not walls)."""
    case = solver.case
    nb = len(case.blocks)
    U = torch.zeros((nb, 2), dtype=torch.float64)
    poses = getattr(solver, "poses", None)
    if poses is not None:
        U[:] = torch.tensor(poses[:, 3:5])
    R = torch.ones((nb, 4), dtype=torch.float64)
    for bi, B in enumerate(case.blocks):
        for s in range(4):
            if B.bc[s] == 3:
                R[bi, s] = float(B.rtw[s])
    return U, R
