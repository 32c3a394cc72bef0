"""Differentiable receiver traces: the discrete adjoint of libdg behind a
torch.autograd.Function.

``receiver_traces(m, solver, zp, zs, q0, t0, dt, nsteps, every)`` returns
the receiver velocities [nsteps, nrec, 3] (CPU float64 tensor) of an
LSRK(5,4) run whose weight-adjusted material weights are
m = (1/rho, lam, mu) at the quadrature points ([3, K, Nq], CPU float64
tensor) and whose upwind flux reads the impedances zp = rho cp and
zs = rho cs at the nodes ([K, Np] each, CPU float64 tensors or arrays).
Its backward is libdg's reverse sweep (``dg_adjoint_forward`` keeps a
checkpoint every ``every`` steps, ``dg_adjoint_backward`` recomputes each
interval from its checkpoint and runs the transposed stage kernels), which
returns dJ/dm and, for tensors zp, zs, dJ/dzp and dJ/dzs; so any torch
expression of the traces (a misfit) and of the fields behind m and z
(rho, lam, mu at the quadrature points and nodes, with zp = sqrt(rho (lam +
2 mu)), zs = sqrt(rho mu)) differentiates through it.  The solver must have
its mesh, sources and receivers set; its state is reset to q0 by every
forward call.  A solver holds one recorded run: the backward of a run
refuses (RuntimeError) once a later forward has run on the same solver, and
the library refuses (DG_ESTATE) once the material, sources or receivers
have changed since the run.
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
            z = [x.detach().cpu().numpy() if torch.is_tensor(x) else np.asarray(x)
                 for x in (zp, zs)]
            B.dg_material_set_weights(solver.ctx, mm[0], mm[1], mm[2], z[0], z[1])
            solver.set_state(q0)
            tr = np.empty((nsteps, solver.nrec, 3), dtype=solver.dtype)
            B.dg_adjoint_forward(solver.ctx, t0, dt, nsteps, every, tr)
            # the library keeps one recorded run per context: a later forward
            # on the same solver replaces it, and this backward must refuse
            solver._adjoint_run = getattr(solver, "_adjoint_run", 0) + 1
            ctx.run = solver._adjoint_run
            ctx.solver = solver
            ctx.shape = tuple(m.shape)
            ctx.zshape = z[0].shape
            return torch.from_numpy(tr.astype(np.float64))

        @staticmethod
        def backward(ctx, g):
            s = ctx.solver
            if getattr(s, "_adjoint_run", None) != ctx.run:
                raise RuntimeError(
                    "receiver_traces: another forward run on this solver replaced the "
                    "checkpoints this backward needs; differentiate each run before "
                    "starting the next on the same solver")
            resid = np.ascontiguousarray(g.detach().cpu().numpy(), dtype=s.dtype)
            grad = np.empty(ctx.shape, dtype=np.float64)
            want_z = ctx.needs_input_grad[2] or ctx.needs_input_grad[3]
            gz = np.empty((2,) + ctx.zshape, dtype=np.float64) if want_z else None
            B.dg_adjoint_backward(s.ctx, resid, grad, gz)
            gzp = torch.from_numpy(gz[0].copy()) if ctx.needs_input_grad[2] else None
            gzs = torch.from_numpy(gz[1].copy()) if ctx.needs_input_grad[3] else None
            return (torch.from_numpy(grad), None, gzp, gzs) + (None,) * 5

    return _Traces


_FN = None


def receiver_traces(m, solver, zp, zs, q0, t0, dt, nsteps, every=20):
    global _FN
    if _FN is None:
        _FN = _autograd_function()
    return _FN.apply(m, solver, zp, zs, q0, t0, dt, nsteps, every)
