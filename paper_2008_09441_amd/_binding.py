"""ctypes binding of libdg (include/dg.h): argument marshalling only.

Every computation of the DG path runs in the HIP library; this module only
converts NumPy arrays and torch device tensors to pointers.  Importing it
raises if libdg.so has not been built: there is no fallback."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdg.so")

DG_OK, DG_EINVAL, DG_ENOMEM, DG_EDEVICE, DG_ESTATE, DG_ENONFINITE = range(6)
DG_FP64, DG_FP32, DG_FP32_BF16X3 = 0, 1, 2
DG_FLUX_UPWIND, DG_FLUX_CENTRAL = 0, 1
STATUS_NAMES = {0: "DG_OK", 1: "DG_EINVAL", 2: "DG_ENOMEM", 3: "DG_EDEVICE",
                4: "DG_ESTATE", 5: "DG_ENONFINITE"}

EXPORTS = [
    "dg_create", "dg_destroy", "dg_last_error", "dg_sizes", "dg_mesh_upload",
    "dg_node_coords", "dg_quad_coords", "dg_material_upload", "dg_project",
    "dg_state_set", "dg_state_get", "dg_state_device_ptr", "dg_rhs", "dg_step",
    "dg_batch_create", "dg_batch_destroy", "dg_batch_advance", "dg_batch_advance_noalloc",
    "dg_run", "dg_synchronize", "dg_ref_operator", "dg_face_nodes",
    "dg_connectivity", "dg_geometry", "dg_tile_order", "dg_sources_set", "dg_receivers_set",
    "dg_receivers_sample", "dg_run_record", "dg_time_set", "dg_time_get",
    "dg_trace_reserve", "dg_trace_copy", "dg_advance", "dg_graph_advance", "dg_memory",
    "dg_footprint", "dg_state_zero", "dg_material_set_weights", "dg_adjoint_forward",
    "dg_adjoint_backward", "dg_measure_copy", "dg_measure_mfma",
]


class dg_options(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("flux", ctypes.c_int32), ("device", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("hbm_budget_bytes", ctypes.c_uint64)]


class DGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    # torch ships its own HIP runtime; loading it first makes libdg bind to
    # the same runtime instead of bringing in a second one
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libdg.so is not built ({LIB_PATH}); run "
                          "python -m paper_2008_09441_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, U64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                           ctypes.c_double, ctypes.c_uint64)
    sig = {
        "dg_create": ([ctypes.POINTER(P), ctypes.POINTER(dg_options)], I32),
        "dg_destroy": ([P], None),
        "dg_last_error": ([P], ctypes.c_char_p),
        "dg_sizes": ([P, P, P, P, P], I32),
        "dg_mesh_upload": ([P, I64, P, P], I32),
        "dg_node_coords": ([P, P], I32),
        "dg_quad_coords": ([P, P], I32),
        "dg_material_upload": ([P, P, P, P, P, P, P], I32),
        "dg_project": ([P, I32, P, P], I32),
        "dg_state_set": ([P, P, I32], I32),
        "dg_state_get": ([P, P, I32], I32),
        "dg_state_device_ptr": ([P, ctypes.POINTER(P)], I32),
        "dg_rhs": ([P, P, P, D], I32),
        "dg_step": ([P, D, D], I32),
        "dg_run": ([P, D, D, I64], I32),
        "dg_synchronize": ([P], I32),
        "dg_ref_operator": ([P, I32, P], I32),
        "dg_face_nodes": ([P, P], I32),
        "dg_connectivity": ([P, P, P, P], I32),
        "dg_tile_order": ([P, P], I32),
        "dg_geometry": ([P, P, P, P], I32),
        "dg_sources_set": ([P, I32, P, P, P, P, P], I32),
        "dg_receivers_set": ([P, I32, P], I32),
        "dg_receivers_sample": ([P, P, I32], I32),
        "dg_run_record": ([P, D, D, I64, P, I32], I32),
        "dg_time_set": ([P, D], I32),
        "dg_time_get": ([P, P, P], I32),
        "dg_trace_reserve": ([P, I64], I32),
        "dg_trace_copy": ([P, P, I64], I32),
        "dg_advance": ([P, D, I64], I32),
        "dg_graph_advance": ([P, D, I64], I32),
        "dg_memory": ([P, P], I32),
        "dg_footprint": ([I32, I32, I64, I32, I32, I64, P], I32),
        "dg_state_zero": ([P], I32),
        "dg_material_set_weights": ([P, P, P, P, P, P], I32),
        "dg_adjoint_forward": ([P, D, D, I64, I64, P], I32),
        "dg_adjoint_backward": ([P, P, P, P], I32),
        "dg_batch_create": ([ctypes.POINTER(P), I32, I32], I32),
        "dg_batch_destroy": ([P], None),
        "dg_batch_advance": ([P, P, P, I32, P, I64], I32),
        "dg_batch_advance_noalloc": ([P, P, I32, P, I64], I32),
        "dg_measure_copy": ([I32, I64, I32, P], I32),
        "dg_measure_mfma": ([I32, I32, P], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def _ptr(a):
    """Pointer of a C-contiguous NumPy array or a contiguous torch tensor."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return a.ctypes.data
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr()
    raise TypeError(type(a))


def _f64(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a


def check(ctx, status):
    if status != DG_OK:
        msg = lib.dg_last_error(ctx).decode() if ctx else ""
        raise DGError(status, msg)


# ----------------------------------------------------------- C-ABI mirror --

def dg_create(order, precision=DG_FP32, flux=DG_FLUX_UPWIND, device=0,
              stream=None, hbm_budget_bytes=0):
    opt = dg_options(order, precision, flux, device, stream or None, hbm_budget_bytes)
    h = ctypes.c_void_p()
    st = lib.dg_create(ctypes.byref(h), ctypes.byref(opt))
    if st != DG_OK:
        raise DGError(st, "dg_create failed")
    return h


def dg_destroy(ctx):
    lib.dg_destroy(ctx)


def dg_sizes(ctx):
    K, Np, Nfp, Nq = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(ctx, lib.dg_sizes(ctx, ctypes.byref(K), ctypes.byref(Np), ctypes.byref(Nfp),
                            ctypes.byref(Nq)))
    return K.value, Np.value, Nfp.value, Nq.value


def dg_mesh_upload(ctx, vxyz, period):
    vxyz = np.ascontiguousarray(vxyz, dtype=np.float64)
    K = vxyz.shape[0]
    vxyz = _f64(vxyz, (K, 4, 3))
    period = _f64(period, (3,))
    check(ctx, lib.dg_mesh_upload(ctx, K, _ptr(vxyz), _ptr(period)))


def dg_node_coords(ctx):
    K, Np, _, _ = dg_sizes(ctx)
    out = np.empty((K, Np, 3))
    check(ctx, lib.dg_node_coords(ctx, _ptr(out)))
    return out


def dg_quad_coords(ctx):
    K, _, _, Nq = dg_sizes(ctx)
    out = np.empty((K, Nq, 3))
    check(ctx, lib.dg_quad_coords(ctx, _ptr(out)))
    return out


def dg_material_upload(ctx, rho_q, cp_q, cs_q, rho_n, cp_n, cs_n):
    K, Np, _, Nq = dg_sizes(ctx)
    arrs = [_f64(a, (K, Nq)) for a in (rho_q, cp_q, cs_q)] + \
           [_f64(a, (K, Np)) for a in (rho_n, cp_n, cs_n)]
    check(ctx, lib.dg_material_upload(ctx, *[_ptr(a) for a in arrs]))


def dg_project(ctx, fq):
    K, Np, _, Nq = dg_sizes(ctx)
    fq = np.ascontiguousarray(fq, dtype=np.float64)
    nf = fq.shape[0]
    fq = _f64(fq, (nf, K, Nq))
    out = np.empty((nf, K, Np))
    check(ctx, lib.dg_project(ctx, nf, _ptr(fq), _ptr(out)))
    return out


def _check_host_state(ctx, a):
    K, Np, _, _ = dg_sizes(ctx)
    if a.size != 9 * K * Np:
        raise ValueError(f"state: expected 9*K*Np = {9 * K * Np} values, got {a.shape}")


def dg_state_set(ctx, q, on_device):
    if on_device:
        _check_device_state(ctx, q, "state")
    else:
        _check_host_state(ctx, q)
    check(ctx, lib.dg_state_set(ctx, _ptr(q), 1 if on_device else 0))


def dg_state_get(ctx, out, on_device):
    if on_device:
        _check_device_state(ctx, out, "state")
    else:
        _check_host_state(ctx, out)
    check(ctx, lib.dg_state_get(ctx, _ptr(out), 1 if on_device else 0))
    return out


def dg_state_device_ptr(ctx):
    p = ctypes.c_void_p()
    check(ctx, lib.dg_state_device_ptr(ctx, ctypes.byref(p)))
    return p.value


def _check_device_state(ctx, t, what):
    """The C-ABI takes raw device pointers: check size, dtype and placement
    here so that a wrong tensor is rejected before any kernel runs."""
    K, Np, _, _ = dg_sizes(ctx)
    if not hasattr(t, "is_cuda") or not t.is_cuda:
        raise ValueError(f"{what}: expected a device tensor")
    if not t.is_contiguous() or t.numel() != 9 * K * Np:
        raise ValueError(f"{what}: expected a contiguous tensor of 9*K*Np = "
                         f"{9 * K * Np} elements, got {tuple(t.shape)}")


def dg_rhs(ctx, q_dev, rhs_dev, t=0.0, dtype=None):
    _check_device_state(ctx, q_dev, "q")
    _check_device_state(ctx, rhs_dev, "rhs")
    if q_dev.dtype != rhs_dev.dtype or (dtype is not None and q_dev.dtype != dtype):
        raise ValueError("q and rhs must have the context's working precision")
    check(ctx, lib.dg_rhs(ctx, _ptr(q_dev), _ptr(rhs_dev), float(t)))


def dg_step(ctx, t, dt):
    check(ctx, lib.dg_step(ctx, float(t), float(dt)))


def dg_run(ctx, t0, dt, nsteps):
    check(ctx, lib.dg_run(ctx, float(t0), float(dt), int(nsteps)))


def dg_sources_set(ctx, xyz, dirs, f0, t0, amp):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    n = xyz.shape[0]
    dirs = _f64(np.asarray(dirs, dtype=np.float64).reshape(-1, 3), (n, 3))
    f0, t0, amp = (_f64(np.broadcast_to(np.asarray(v, dtype=np.float64), (n,)), (n,))
                   for v in (f0, t0, amp))
    check(ctx, lib.dg_sources_set(ctx, n, _ptr(xyz), _ptr(dirs), _ptr(f0), _ptr(t0),
                                  _ptr(amp)))


def dg_receivers_set(ctx, xyz):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    check(ctx, lib.dg_receivers_set(ctx, xyz.shape[0], _ptr(xyz)))


def dg_receivers_sample(ctx, out, on_device):
    check(ctx, lib.dg_receivers_sample(ctx, _ptr(out), 1 if on_device else 0))


def dg_run_record(ctx, t0, dt, nsteps, trace, on_device):
    check(ctx, lib.dg_run_record(ctx, float(t0), float(dt), int(nsteps), _ptr(trace),
                                 1 if on_device else 0))


def dg_material_set_weights(ctx, irho_q, lam_q, mu_q, zp_n, zs_n):
    K, Np, _, Nq = dg_sizes(ctx)
    a = [_f64(x, (K, Nq)) for x in (irho_q, lam_q, mu_q)] + \
        [_f64(x, (K, Np)) for x in (zp_n, zs_n)]
    check(ctx, lib.dg_material_set_weights(ctx, *[_ptr(x) for x in a]))


def dg_adjoint_forward(ctx, t0, dt, nsteps, every, trace):
    if not isinstance(trace, np.ndarray) or not trace.flags["C_CONTIGUOUS"]:
        raise ValueError("trace must be a C-contiguous host array")
    check(ctx, lib.dg_adjoint_forward(ctx, float(t0), float(dt), int(nsteps), int(every),
                                      _ptr(trace)))


def dg_adjoint_backward(ctx, resid, grad, grad_z=None):
    K, Np, _, Nq = dg_sizes(ctx)
    for a, shape in ((grad, (3, K, Nq)), (grad_z, (2, K, Np))):
        if a is None:
            continue
        if a.dtype != np.float64 or not a.flags["C_CONTIGUOUS"] or a.size != int(np.prod(shape)):
            raise ValueError(f"gradients must be C-contiguous float64 host arrays of {shape}")
    check(ctx, lib.dg_adjoint_backward(ctx, _ptr(np.ascontiguousarray(resid)), _ptr(grad),
                                       _ptr(grad_z) if grad_z is not None else None))


def dg_batch_create(device, max_slots):
    h = ctypes.c_void_p()
    st = lib.dg_batch_create(ctypes.byref(h), int(device), int(max_slots))
    if st != DG_OK:
        raise DGError(st, "dg_batch_create failed")
    return h


def dg_batch_destroy(b):
    lib.dg_batch_destroy(b)


def _ctx_array(ctxs):
    vals = [c.value if isinstance(c, ctypes.c_void_p) else c for c in ctxs]
    return (ctypes.c_void_p * len(vals))(*vals)


def dg_batch_advance(b, stream, ctxs, dts, nsteps):
    """Advance the contexts ctxs (a list of dg_create handles) by nsteps steps
    of their own time steps dts on `stream` (an int hipStream_t or None)."""
    dts = np.ascontiguousarray(dts, dtype=np.float64)
    if dts.shape != (len(ctxs),):
        raise ValueError("one time step per context")
    check(ctxs[0], lib.dg_batch_advance(b, stream or None, _ctx_array(ctxs), len(ctxs),
                                        _ptr(dts), int(nsteps)))


def dg_batch_advance_noalloc(stream, ctxs, dts, nsteps):
    """dg_batch_advance without a batch object: the slot table lives in the
    library's static device array (at most 64 contexts, no allocation)."""
    dts = np.ascontiguousarray(dts, dtype=np.float64)
    if dts.shape != (len(ctxs),):
        raise ValueError("one time step per context")
    check(ctxs[0], lib.dg_batch_advance_noalloc(stream or None, _ctx_array(ctxs), len(ctxs),
                                                _ptr(dts), int(nsteps)))


def dg_measure_copy(device, nbytes, reps=10):
    v = ctypes.c_double()
    st = lib.dg_measure_copy(int(device), int(nbytes), int(reps), ctypes.byref(v))
    if st != DG_OK:
        raise DGError(st, "dg_measure_copy failed")
    return v.value


def dg_measure_mfma(device, reps=10):
    v = ctypes.c_double()
    st = lib.dg_measure_mfma(int(device), int(reps), ctypes.byref(v))
    if st != DG_OK:
        raise DGError(st, "dg_measure_mfma failed")
    return v.value


def dg_state_zero(ctx):
    check(ctx, lib.dg_state_zero(ctx))


def dg_time_set(ctx, t):
    check(ctx, lib.dg_time_set(ctx, float(t)))


def dg_time_get(ctx):
    t, step = ctypes.c_double(), ctypes.c_int64()
    check(ctx, lib.dg_time_get(ctx, ctypes.byref(t), ctypes.byref(step)))
    return t.value, step.value


def dg_trace_reserve(ctx, max_steps):
    check(ctx, lib.dg_trace_reserve(ctx, int(max_steps)))


def dg_trace_copy(ctx, out, nrows):
    check(ctx, lib.dg_trace_copy(ctx, _ptr(out), int(nrows)))


def dg_advance(ctx, dt, nsteps):
    check(ctx, lib.dg_advance(ctx, float(dt), int(nsteps)))


def dg_graph_advance(ctx, dt, nsteps):
    check(ctx, lib.dg_graph_advance(ctx, float(dt), int(nsteps)))


def dg_memory(ctx):
    b = ctypes.c_uint64()
    check(ctx, lib.dg_memory(ctx, ctypes.byref(b)))
    return b.value


def dg_footprint(order, precision, K, nsrc=0, nrec=0, trace_steps=0):
    b = ctypes.c_uint64()
    st = lib.dg_footprint(int(order), int(precision), int(K), int(nsrc), int(nrec),
                          int(trace_steps), ctypes.byref(b))
    if st != DG_OK:
        raise DGError(st, "dg_footprint: bad arguments")
    return b.value


def dg_synchronize(ctx):
    check(ctx, lib.dg_synchronize(ctx))


def dg_ref_operator(ctx, which):
    _, Np, Nfp, Nq = dg_sizes(ctx)
    shapes = {0: (Np, Np), 1: (Np, Np), 2: (Np, Np), 3: (Np, 4 * Nfp),
              4: (Nq, Np), 5: (Np, Nq), 6: (Np, 3), 7: (Nq, 4)}
    out = np.empty(shapes[which])
    check(ctx, lib.dg_ref_operator(ctx, which, _ptr(out)))
    return out


def dg_face_nodes(ctx):
    _, _, Nfp, _ = dg_sizes(ctx)
    out = np.empty((4, Nfp), dtype=np.int32)
    check(ctx, lib.dg_face_nodes(ctx, _ptr(out)))
    return out


def dg_connectivity(ctx):
    K, _, Nfp, _ = dg_sizes(ctx)
    etoe = np.empty((K, 4), dtype=np.int32)
    etof = np.empty((K, 4), dtype=np.int32)
    nbn = np.empty((K, 4, Nfp), dtype=np.int32)
    check(ctx, lib.dg_connectivity(ctx, _ptr(etoe), _ptr(etof), _ptr(nbn)))
    return etoe, etof, nbn


def dg_tile_order(ctx):
    K, _, _, _ = dg_sizes(ctx)
    out = np.empty((K + 15) // 16, dtype=np.int32)
    check(ctx, lib.dg_tile_order(ctx, _ptr(out)))
    return out


def dg_geometry(ctx):
    K, _, _, _ = dg_sizes(ctx)
    geo = np.empty((K, 9))
    fgeo = np.empty((K, 4, 4))
    J = np.empty(K)
    check(ctx, lib.dg_geometry(ctx, _ptr(geo), _ptr(fgeo), _ptr(J)))
    return geo, fgeo, J
