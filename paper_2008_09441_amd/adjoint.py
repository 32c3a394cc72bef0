"""Differentiable receiver traces: the discrete adjoint of libdg behind a
torch.autograd.Function.

``receiver_traces(m, solver, zp, zs, q0, t0, dt, nsteps, every)`` returns
the receiver velocities [nsteps, nrec, 3] (CPU float64 tensor) of an
LSRK(5,4) run whose weight-adjusted material weights are
m = (1/rho, lam, mu) at the quadrature points ([3, K, Nq], CPU float64
tensor); the flux impedances zp, zs [K, Np] are held fixed.  Its backward
is libdg's reverse sweep (``dg_adjoint_forward`` keeps a checkpoint every
``every`` steps, ``dg_adjoint_backward`` recomputes each interval from its
checkpoint and runs the transposed stage kernels), so any torch expression
of the traces (a misfit) and of the parameters behind m (nodal rho, lam,
mu mapped to the quadrature points, for instance) differentiates through
it.  The solver must have its mesh, sources and receivers set; its state is
reset to q0 by every forward call.
"""
from __future__ import annotations

import numpy as np

from . import _binding as B


def _autograd_function():
    import torch

    class _Traces(torch.autograd.Function):
        @staticmethod
        def forward(ctx, m, solver, zp, zs, q0, t0, dt, nsteps, every):
            mm = m.detach().cpu().numpy().astype(np.float64)
            B.dg_material_set_weights(solver.ctx, mm[0], mm[1], mm[2], zp, zs)
            solver.set_state(q0)
            tr = np.empty((nsteps, solver.nrec, 3), dtype=solver.dtype)
            B.dg_adjoint_forward(solver.ctx, t0, dt, nsteps, every, tr)
            ctx.solver = solver
            ctx.shape = tuple(m.shape)
            return torch.from_numpy(tr.astype(np.float64))

        @staticmethod
        def backward(ctx, g):
            s = ctx.solver
            resid = np.ascontiguousarray(g.detach().cpu().numpy(), dtype=s.dtype)
            grad = np.empty(ctx.shape, dtype=np.float64)
            B.dg_adjoint_backward(s.ctx, resid, grad)
            return (torch.from_numpy(grad),) + (None,) * 8

    return _Traces


_FN = None


def receiver_traces(m, solver, zp, zs, q0, t0, dt, nsteps, every=20):
    global _FN
    if _FN is None:
        _FN = _autograd_function()
    return _FN.apply(m, solver, zp, zs, q0, t0, dt, nsteps, every)
