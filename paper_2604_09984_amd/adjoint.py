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
the step's forward (Steps 1-2 and the n_inner inner iterations, keeping the
inner states) and then the reverse passes.  A `setup` callable restores the
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

import torch

from . import ugks


# --------------------------------------------------------------------------
# wall loads (computed by the library) as a differentiable function of F
# --------------------------------------------------------------------------
class WallLoads(torch.autograd.Function):
    """F [nface][dim+2] -> side loads [nblock][4][4] (force x, y, moment,
    energy flux into the walls of each block side; ugks_wall_loads)."""

    @staticmethod
    def forward(ctx, solver, F):
        _, side = solver.wall_loads(F)
        ctx.solver = solver
        return side

    @staticmethod
    def backward(ctx, g):
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
# one physical step, checkpointed
# --------------------------------------------------------------------------
class PhysicalStep(torch.autograd.Function):
    """(h, b, W, q, U, rtw) -> (h', b', W', q', F): Steps 1-8 of one physical
    step (Steps 1-2, then n_inner inner iterations); F is the face macro flux
    of the last inner iteration.  Only the inputs are kept; the backward pass
    recomputes the step."""

    @staticmethod
    def forward(ctx, solver, dt, n_inner, setup, h, b, W, q, U, rtw):
        # the cell kinds before the step's setup decide which cells an
        # overset assembly refills; the recomputation restores them
        ctx.types0 = solver.types() if setup is not None else None
        _run_setup(setup, solver)
        apply_params(solver, U, rtw)
        ctx.refill = solver.overset_rows()[2] != 0
        h1, b1, W1, q1 = _clone(h, b, W, q)
        Wn = W1.clone()
        Sh, Sb, Fn = solver.begin_step(dt, h1, b1, W1, q1)
        solver.step(dt, n_inner, h1, b1, W1, Wn, q1, Sh, Sb, Fn)
        F = solver.last_flux()
        ctx.solver, ctx.dt, ctx.n_inner, ctx.setup = solver, dt, n_inner, setup
        ctx.save_for_backward(h, b, W, q, U, rtw)
        return h1, b1, W1, q1, F

    @staticmethod
    def backward(ctx, gh, gb, gW, gq, gF):
        h, b, W, q, U, rtw = ctx.saved_tensors
        dt = ctx.dt
        s = _twin(ctx.solver)
        if ctx.setup is not None:
            s.set_types(ctx.types0)
            _run_setup(ctx.setup, s)
        else:
            _mirror(ctx.solver, s)
        apply_params(s, U, rtw)
        # recomputation: Steps 1-2, then the inner iterations, keeping their
        # inputs (FP64 storage: the twin's, from the FP32 inputs if need be)
        h_in, b_in = h, b
        h, b = _f64(h), _f64(b)
        hs, bs, Ws, qs = _clone(h, b, W, q)
        Wn = W.clone()
        Sh, Sb, Fn = s.begin_step(dt, hs, bs, Ws, qs)
        states = []
        for _ in range(ctx.n_inner):
            states.append(_clone(hs, bs, Ws, qs))
            s.step(dt, 1, hs, bs, Ws, Wn, qs, Sh, Sb, Fn)
        del hs, bs, Ws, qs
        # reverse through the inner iterations
        gh, gb, gW, gq = _f64(gh), _f64(gb), _c(gW), _c(gq)
        gSh = torch.zeros_like(Sh); gSb = torch.zeros_like(Sb)
        gFn = torch.zeros_like(Fn); gWn = torch.zeros_like(W)
        faces = torch.zeros((s.nface, 5), dtype=torch.float64, device=h.device)
        for it in range(ctx.n_inner - 1, -1, -1):
            hi, bi, Wi, qi = states.pop()
            out = s.step_adjoint(dt, hi, bi, Wi, Wn, qi, Sh, Sb, Fn, gh, gb, gW, gq,
                                 _c(gF) if it == ctx.n_inner - 1 else None)
            gh, gb, gW, gWn_i, gq, gSh_i, gSb_i, gFn_i, fb = out
            gWn += gWn_i; gSh += gSh_i; gSb += gSb_i; gFn += gFn_i; faces += fb
        # Steps 1-2 (Wn is the input W)
        hb, bb, Wb, qb, fb = s.begin_step_adjoint(dt, h, b, W, q, gh, gb, gW, gq, gSh, gSb, gFn,
                                                  refill=ctx.refill)
        faces += fb
        Wb = Wb + gWn
        gU, gR = _param_grads(s, faces)
        return None, None, None, None, _as(hb, h_in), _as(bb, b_in), Wb, qb, _out_grad(U, gU), _out_grad(rtw, gR)


def physical_step(solver, dt, n_inner, h, b, W, q, U=None, rtw=None, setup=None, checkpoint=True):
    """One differentiable physical step; returns (h', b', W', q', F).  With
    checkpoint=False the step is composed of BeginStep and PseudoStep nodes
    whose inputs autograd keeps (n_inner states of f; fixed geometry)."""
    if checkpoint:
        return PhysicalStep.apply(solver, dt, n_inner, setup, h, b, W, q, U, rtw)
    if setup is not None:
        raise ValueError("checkpoint=False keeps every node of the step for one geometry: no setup")
    Wn = W
    h, b, W, q, Sh, Sb, Fn = BeginStep.apply(solver, dt, setup, h, b, W, q, U, rtw)
    F = None
    for _ in range(n_inner):
        h, b, W, q, F = PseudoStep.apply(solver, dt, setup, h, b, W, q, Wn, Sh, Sb, Fn, U, rtw)
    return h, b, W, q, F


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
