"""Differentiable evolution: the GRMHD update as a ``torch.autograd.Function``.

``evolve(solver, P0, dt, nsteps, every)`` returns the primitives after
``nsteps`` Runge-Kutta steps from the primitives ``P0``; its backward pass
gives the vector-Jacobian product with respect to ``P0`` through the
library's hand-written adjoint (``grmhd_step_adjoint``, ``grmhd_prim_adjoint``,
``grmhd_cons_adjoint``).  This is the building block of the gradient-based
source-parameter inverse problems the paper motivates (section 1).

Memory: the forward pass keeps the conserved state only every ``every``
steps (checkpoints).  The backward pass walks the segments from the last to
the first and recomputes each segment from its checkpoint.  With a solver
created with ``tape_steps >= every`` the recomputation records every step's
stages (``grmhd_step_record``) and the reverse sweep uses them
(``grmhd_step_adjoint_recorded``): a gradient costs one forward evolution
(the recomputation) plus ``nsteps`` reverse sweeps, and the tape holds
``every`` steps' stages.  The forward pass records the last segment's steps
itself, so the backward pass reverses them without recomputing them (unless
the tape was used by another call in between).  Otherwise the recomputation keeps the segment's
states and each ``grmhd_step_adjoint`` recomputes its step's stages again.

Argument marshalling only: every operation runs in the library's kernels.
"""
from __future__ import annotations

import torch


class _Evolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P0, solver, dt, nsteps, every):
        s = solver
        U = s.cons(P0.detach().contiguous())
        checkpoints = {0: U.clone()}
        # with a tape, the steps of the last segment (the first one the
        # backward pass reverses) are recorded now instead of recomputed then
        last = ((nsteps - 1) // every) * every
        taped = s.tape_steps >= every
        token = object()
        for k in range(1, nsteps + 1):
            if taped and k > last:
                s.step_record(U, dt, k - 1 - last)
            else:
                s.step(U, dt)
            if k % every == 0 and k < nsteps:
                checkpoints[k] = U.clone()
        s.tape_owner = token if taped else None
        P = s.prim(U)
        ctx.solver, ctx.dt, ctx.nsteps, ctx.every = s, dt, nsteps, every
        ctx.checkpoints, ctx.token, ctx.last = checkpoints, token, last
        ctx.save_for_backward(P0, U)
        return P

    @staticmethod
    def backward(ctx, Pbar):
        s, dt, nsteps, every = ctx.solver, ctx.dt, ctx.nsteps, ctx.every
        P0, U_end = ctx.saved_tensors
        Ubar = s.prim_adjoint(U_end, Pbar.contiguous())
        starts = sorted(ctx.checkpoints)
        taped = s.tape_steps >= every
        for c in reversed(starts):
            stop = min(c + every, nsteps)
            if taped and c == ctx.last and getattr(s, "tape_owner", None) is ctx.token:
                # recorded by the forward pass, and the tape not used since
                for k in range(stop - 1, c - 1, -1):
                    s.step_adjoint_recorded(k - c, Ubar)
                continue
            s.tape_owner = None
            # recompute the segment from its checkpoint
            U = ctx.checkpoints[c].clone()
            if c == 0:
                s.cons(P0.detach().contiguous(), U)   # the step cache exactly as in the forward pass
            else:
                s.prim(U)                   # the primitives of U_c into the step cache
            if taped:
                # every step of the segment recorded once, then reversed
                for k in range(c, stop):
                    s.step_record(U, dt, k - c)
                for k in range(stop - 1, c - 1, -1):
                    s.step_adjoint_recorded(k - c, Ubar)
                continue
            states = [U.clone()]
            for _ in range(c + 1, stop):
                s.step(U, dt)
                states.append(U.clone())
            for Uk in reversed(states):
                s.step_adjoint(Uk, Ubar, dt)
            del states
        Pbar0 = s.cons_adjoint(P0.detach().contiguous(), Ubar)
        return Pbar0, None, None, None, None


def evolve(solver, P0: torch.Tensor, dt: float, nsteps: int, every: int = 10) -> torch.Tensor:
    """Primitives after ``nsteps`` steps of size ``dt`` from ``P0`` (float64,
    shape (9, nz, ny, nx), on the solver's device), differentiable in ``P0``.
    The solver must have been created with ``adjoint=True`` (and
    ``tape_steps >= every`` to record the recomputed steps); ``every`` is the
    checkpoint interval of the backward pass."""
    if nsteps < 1 or every < 1:
        raise ValueError("nsteps and every must be >= 1")
    return _Evolve.apply(P0, solver, float(dt), int(nsteps), int(every))
