"""MI355X-native nodal DG elastic-wave hot path (libdg, HIP for gfx950).

The C-ABI (include/dg.h) is mirrored one to one in ``_binding`` (dg_create,
dg_mesh_upload, dg_material_upload, dg_rhs, dg_step, dg_run, ...).
``Solver`` is a thin convenience wrapper over those calls; torch provides
device memory and the stream, nothing else.
"""
from __future__ import annotations

import numpy as np

from . import _binding as B
from ._binding import (DG_FLUX_CENTRAL, DG_FLUX_UPWIND, DG_FP32, DG_FP32_BF16X3,
                       DG_FP64, DGError)

PRECISIONS = {"fp64": DG_FP64, "fp32": DG_FP32, "bf16x3": DG_FP32_BF16X3}
FLUXES = {"upwind": DG_FLUX_UPWIND, "central": DG_FLUX_CENTRAL}

__all__ = ["Solver", "DGError", "PRECISIONS", "FLUXES", "B"]


class Solver:
    """One DG context: mesh, media and state resident on one GPU."""

    def __init__(self, order, precision="fp32", flux="upwind", device=0,
                 stream=None, hbm_budget_bytes=0):
        self.precision = precision
        self.order = order
        self.device = device
        self._torch_stream = None
        if device >= 0 and stream is None:
            import torch
            self._torch_stream = torch.cuda.current_stream(device)
            stream = self._torch_stream.cuda_stream
        self.ctx = B.dg_create(order, PRECISIONS[precision], FLUXES[flux], device,
                               stream, hbm_budget_bytes)

    def close(self):
        if self.ctx is not None:
            B.dg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    @property
    def dtype(self):
        return np.float64 if self.precision == "fp64" else np.float32

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.precision == "fp64" else torch.float32

    def sizes(self):
        return B.dg_sizes(self.ctx)

    def upload_mesh(self, vxyz, period=(1.0, 1.0, 1.0)):
        B.dg_mesh_upload(self.ctx, vxyz, np.asarray(period, dtype=np.float64))

    def node_coords(self):
        return B.dg_node_coords(self.ctx)

    def quad_coords(self):
        return B.dg_quad_coords(self.ctx)

    def upload_media(self, media):
        """media(x[..., 3]) -> (rho, cp, cs), sampled at quadrature points and
        nodes."""
        rq, pq, sq = media(self.quad_coords())
        rn, pn, sn = media(self.node_coords())
        B.dg_material_upload(self.ctx, rq, pq, sq, rn, pn, sn)

    def project(self, fq):
        return B.dg_project(self.ctx, fq)

    def project_function(self, fun):
        return self.project(fun(self.quad_coords()))

    # ------------------------------------------------------------------
    def set_state(self, q):
        """q: host array or device tensor [9, K, Np] (cast to the working
        precision)."""
        if isinstance(q, np.ndarray):
            B.dg_state_set(self.ctx, np.ascontiguousarray(q, dtype=self.dtype), False)
        else:
            q = q.to(device=f"cuda:{self.device}", dtype=self.torch_dtype).contiguous()
            B.dg_state_set(self.ctx, q, True)
            self._keep = q

    def get_state(self):
        K, Np, _, _ = self.sizes()
        out = np.empty((9, K, Np), dtype=self.dtype)
        B.dg_state_get(self.ctx, out, False)
        return out

    def state_tensor(self):
        """A new device tensor holding a copy of the state."""
        import torch
        K, Np, _, _ = self.sizes()
        out = torch.empty((9, K, Np), dtype=self.torch_dtype, device=f"cuda:{self.device}")
        B.dg_state_get(self.ctx, out, True)
        return out

    def rhs(self, q, out=None, t=0.0):
        """dq/dt at time t of the device tensor q [9, K, Np] into out
        (allocated if None)."""
        import torch
        if out is None:
            out = torch.empty_like(q)
        B.dg_rhs(self.ctx, q, out, t, self.torch_dtype)
        return out

    def step(self, t, dt):
        B.dg_step(self.ctx, t, dt)

    def run(self, t0, dt, nsteps):
        B.dg_run(self.ctx, t0, dt, nsteps)

    def set_sources(self, xyz, dirs, f0, t0, amp=1.0):
        """Point forces with Ricker signals (see dg_sources_set)."""
        B.dg_sources_set(self.ctx, xyz, dirs, f0, t0, amp)

    def set_receivers(self, xyz):
        B.dg_receivers_set(self.ctx, xyz)
        self.nrec = int(np.asarray(xyz).reshape(-1, 3).shape[0])

    def sample_receivers(self):
        """Velocity at the receivers for the current state: host [nrec, 3]."""
        out = np.empty((self.nrec, 3), dtype=self.dtype)
        B.dg_receivers_sample(self.ctx, out, False)
        return out

    def run_record(self, t0, dt, nsteps, out=None):
        """nsteps steps recording the receivers after each: returns
        [nsteps, nrec, 3] (a device tensor if out is one, else host)."""
        if out is not None:
            B.dg_run_record(self.ctx, t0, dt, nsteps, out, True)
            return out
        tr = np.empty((nsteps, self.nrec, 3), dtype=self.dtype)
        B.dg_run_record(self.ctx, t0, dt, nsteps, tr, False)
        return tr

    def synchronize(self):
        B.dg_synchronize(self.ctx)
