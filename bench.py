"""Throughput benchmark of the DG elastic-wave hot path on one MI355X.

Workload (default): order N=4 (Np=35) nodal DG on the periodic unit cube cut
into 48^3 x 6 = 663,552 Kuhn tetrahedra; smooth heterogeneous media sampled
per quadrature point and node from seeded sums of 16 random Fourier modes
(rho in [1,3], cp in [2,4], cs = cp/[1.6,2]); Gaussian velocity pulse initial
condition (L2-projected); upwind flux; LSRK(5,4) at CFL 0.5 with cp_max = 4.

One step = one LSRK(5,4) step = five fused stage kernels (volume + face
flux + LIFT + weight-adjusted mass inverse + stage update) over all
elements.  Metric: DOF-updates/s = 9 K Np steps / seconds.  The measured
path is FP32 with BF16x3 matrix-core contractions; the plain FP32 and FP64
GPU paths run the same mesh, media, initial condition and step count beside
it, and the reduced-precision states are compared with the FP64 one in the
quadrature L2 norm (per field, and per field over the norm of its group:
velocity or stress).

Prints one JSON line.  N > 1 GPUs is not supported (one-GPU build).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic HBM bytes per element per stage (each value read or written
# once): q and res read + written (4 * 9 * Np), 1/rho, lam, mu at the Nq
# quadrature points, Zp and Zs at the Np nodes, 9 metric terms, 4 x (normal,
# Fscale), 4 neighbour ids + 4 pattern bytes
def alg_bytes_per_elem_stage(N, elem_bytes):
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    Nq = (N + 1) ** 3
    reals = 4 * 9 * Np + 3 * Nq + 2 * Np + 9 + 16
    return reals * elem_bytes + 4 * 4 + 4


def kernel_build_hash(source):
    """First 16 hex digits of the sha256 of a kernel source followed by the
    hipcc flags it is built with: a record of counters taken on that build
    holds only while both are unchanged."""
    import hashlib
    from paper_2008_09441_amd.build import HIPCC_FLAGS
    h = hashlib.sha256(open(os.path.join(ROOT, source), "rb").read())
    h.update(" ".join(HIPCC_FLAGS).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, precision, order, elements):
    """HBM bytes per launch from the rocprofv3 FETCH_SIZE/WRITE_SIZE record of
    this kernel and workload, or None when there is none or the kernel source
    or its build flags have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_records.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        line = line.strip()
        if not line:
            continue
        r = json.loads(line)
        if (r["kernel"], r["precision"], r["order"], r["elements"]) != (kernel, precision, order, elements):
            continue
        if kernel_build_hash(r["source"]) != r["kernel_build_sha256_16"]:
            return None
        return 1024.0 * (r["fetch_kib"] * r["fetch_factor"] + r["write_kib"] * r["write_factor"])
    return None


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--precision", default="bf16x3", choices=["fp32", "bf16x3", "fp64"])
    p.add_argument("--n", type=int, default=48, help="hexahedra per cube side")
    p.add_argument("--order", type=int, default=4)
    p.add_argument("--no-fp64-reference", action="store_true")
    p.add_argument("--no-fp32-path", action="store_true")
    p.add_argument("--no-sources", action="store_true",
                   help="skip the point-source / receiver measurement")
    p.add_argument("--no-serving", action="store_true", help="skip the serving measurement")
    p.add_argument("--no-adjoint", action="store_true", help="skip the adjoint measurement")
    p.add_argument("--no-order7", action="store_true",
                   help="skip the order-7 layered-media measurement")
    p.add_argument("--adjoint-steps", type=int, default=400)
    p.add_argument("--adjoint-n", type=int, default=24,
                   help="hexahedra per cube side of the adjoint workload")
    p.add_argument("--serving-requests", type=int, default=64)
    p.add_argument("--serving-rate", type=float, default=3.0, help="arrivals per second")
    p.add_argument("--serving-full", action="store_true",
                   help="serve the full stream (256 requests, n in [8,32], 100-800 steps)")
    p.add_argument("--serving-precisions", default="fp32,bf16x3",
                   help="comma-separated precisions of the serving measurement")
    p.add_argument("--serving-batched", action="store_true",
                   help="with --serving-full: batched stepping instead of per-request graphs")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-config1", action="store_true",
                   help="skip the order-3 plane-wave latency and convergence measurement")
    p.add_argument("--no-peaks", action="store_true", help="skip the copy and GEMM peak measurement")
    p.add_argument("--cpu-sample-n", type=int, default=12)
    p.add_argument("--calibrate-copy", action="store_true",
                   help="before timing, run a fill, a sum and a copy of 256 MiB so that "
                        "counter runs see kernels with known read/write bytes")
    return p.parse_args()


def stage_kernel_name(precision, N):
    """The kernel one stage launches for this precision and order."""
    if precision == "bf16x3":
        return f"stage_bx<{N}>" if N <= 4 else f"stage_be<{N}>"
    if precision == "fp32":
        return f"stage_bx<{N},f32>" if N <= 4 else f"stage_be<{N},f32>"
    return f"stage_bx_d<{N}>" if N <= 4 else f"stage_be_d<{N}>"


def setup(args, precision, q0=None):
    import synth
    from paper_2008_09441_amd import B, Solver
    s = Solver(args.order, precision=precision, flux="upwind", device=0)
    s.upload_mesh(synth.kuhn_cube_vertices(args.n))
    return s


def upload_media_and_state(s, media_cache):
    import synth
    from paper_2008_09441_amd import B
    if "media" not in media_cache:
        xq = s.quad_coords()
        xn = s.node_coords()
        media_cache["media"] = synth.fourier_media(xq) + synth.fourier_media(xn)
        fq = synth.gaussian_pulse_vx(xq)[None]      # only v_x is nonzero
        q0x = s.project(fq)[0]
        K, Np, _, _ = s.sizes()
        q0 = np.zeros((9, K, Np))
        q0[0] = q0x
        media_cache["q0"] = q0
        del xq, xn, fq
    B.dg_material_upload(s.ctx, *media_cache["media"])
    s.set_state(media_cache["q0"])


def timed_run(s, dt, steps, warmup):
    import torch
    s.run(0.0, dt, warmup)
    s.synchronize()
    stream = torch.cuda.current_stream(0)    # the stream libdg launches on
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    s.run(warmup * dt, dt, steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.synchronize()
    return ev0.elapsed_time(ev1) / 1e3, wall


class QuadNorm:
    """Quadrature L2 norm ||e||^2 = sum_k J_k sum_q w_q (V_q e_k)_q^2 of each
    field (reference operators and geometry exported by the library)."""

    def __init__(self, args):
        from paper_2008_09441_amd import B, Solver
        s = Solver(args.order, precision="fp64", flux="upwind", device=-1)
        s.upload_mesh(__import__("synth").kuhn_cube_vertices(args.n))
        Vq = B.dg_ref_operator(s.ctx, 4)
        w = B.dg_ref_operator(s.ctx, 7)[:, 3]
        self.M = Vq.T @ (w[:, None] * Vq)
        _, _, self.J = B.dg_geometry(s.ctx)
        s.close()

    def sq(self, q):
        return np.array([float(np.sum(self.J[:, None] * (q[f] @ self.M) * q[f])) for f in range(9)])

    def errors(self, q, ref):
        e2, r2 = self.sq(q - ref), self.sq(ref)
        grp = np.array([r2[:3].sum()] * 3 + [r2[3:].sum()] * 6)
        return {"rel_per_field": [float(x) for x in np.sqrt(e2 / np.maximum(r2, 1e-300))],
                "rel_per_field_of_group": [float(x) for x in np.sqrt(e2 / grp)]}


# Stated bounds of the reduced-precision paths against the FP64 GPU path on
# the order-4 workload, in the energy measure of EnergyNorm.errors: each
# field's error over the energy norm of the FP64 state, at any step count up
# to 200 steps.
ENERGY_BOUND = {"fp32": 1e-6, "bf16x3": 1e-5}


class EnergyNorm:
    """Errors measured in the elastic energy norm, which the solution keeps
    (upwind: does not increase) at every step, so a bound stated in it holds
    at any step count:

        ||q||_E^2 = sum_k J_k sum_q w_q (rho |v|^2 + sigma : C^-1 : sigma)(x_q),
        sigma : C^-1 : sigma = (sigma : sigma - lam / (3 lam + 2 mu) tr(sigma)^2) / (2 mu),

    evaluated at the quadrature points (V_q applied to each field).  A
    field's error is scaled the same way, rho e^2 for a velocity and
    d_f e^2 / (2 mu) for a stress (d_f = 1 for normal, 2 for shear
    components; an upper bound of its share since lam >= 0 here), and
    divided by the energy norm of the reference state.  Evaluated on the GPU
    in FP64 with torch (a measurement, not part of the path)."""

    def __init__(self, s, rho_q, cp_q, cs_q):
        import torch
        from paper_2008_09441_amd import B
        dev = torch.device("cuda:0")
        self.Vq = torch.from_numpy(B.dg_ref_operator(s.ctx, 4)).to(dev)        # [Nq, Np]
        w = torch.from_numpy(B.dg_ref_operator(s.ctx, 7)[:, 3].copy()).to(dev)
        _, _, J = B.dg_geometry(s.ctx)
        self.W = torch.from_numpy(J).to(dev)[:, None] * w[None, :]             # [K, Nq]
        rho = torch.from_numpy(np.asarray(rho_q)).to(dev)
        cp = torch.from_numpy(np.asarray(cp_q)).to(dev)
        cs = torch.from_numpy(np.asarray(cs_q)).to(dev)
        mu = rho * cs * cs
        lam = rho * cp * cp - 2.0 * mu
        self.rho = rho
        self.inv2mu = 0.5 / mu
        self.kappa = lam / (3.0 * lam + 2.0 * mu)

    def _at_q(self, q, f):
        import torch
        return torch.from_numpy(np.ascontiguousarray(q[f], dtype=np.float64)).to(
            self.Vq.device) @ self.Vq.T

    def energy_sq(self, q):
        v2 = sum(self._at_q(q, f) ** 2 for f in range(3))
        s = [self._at_q(q, f) for f in range(3, 9)]
        ss = s[0] ** 2 + s[1] ** 2 + s[2] ** 2 + 2.0 * (s[3] ** 2 + s[4] ** 2 + s[5] ** 2)
        tr = s[0] + s[1] + s[2]
        e = self.rho * v2 + self.inv2mu * (ss - self.kappa * tr * tr)
        return float((self.W * e).sum())

    def field_sq(self, e):
        out = []
        for f in range(9):
            x = self._at_q(e, f) ** 2
            wt = self.rho if f < 3 else self.inv2mu * (1.0 if f < 6 else 2.0)
            out.append(float((self.W * wt * x).sum()))
        return np.array(out)

    def errors(self, q, ref, precision):
        rel = np.sqrt(self.field_sq(q - ref) / self.energy_sq(ref))
        bound = ENERGY_BOUND[precision]
        return {"rel_per_field_of_energy": [float(x) for x in rel],
                "max": float(rel.max()), "bound": bound,
                "within_bound": bool(rel.max() <= bound)}


def sources_receivers(args, steps=50):
    """The order-4 Kuhn cube of 24^3 x 6 tets with Fourier media, 4 Ricker
    point forces and 64 receivers: DOF-updates/s of the recorded run
    (receivers sampled after every step) against the same run without
    sources and receivers."""
    import synth
    from paper_2008_09441_amd import B, Solver
    n, N = 24, args.order
    s = Solver(N, precision=args.precision, flux="upwind", device=0)
    s.upload_mesh(synth.kuhn_cube_vertices(n))
    B.dg_material_upload(s.ctx, *(synth.fourier_media(s.quad_coords())
                                  + synth.fourier_media(s.node_coords())))
    K, Np, _, _ = s.sizes()
    rng = np.random.default_rng(2024)
    f0 = rng.uniform(5.0, 15.0, 4)
    dt = 0.5 * (1.0 / n) / math.sqrt(2.0) / (4.0 * (N + 1) ** 2)
    zero = np.zeros((9, K, Np))

    def timed(record):
        s.set_state(zero)
        s.synchronize()
        t0 = time.perf_counter()
        if record:
            tr = s.run_record(0.0, dt, steps)
        else:
            s.run(0.0, dt, steps)
            s.synchronize()
            tr = None
        return time.perf_counter() - t0, tr
    plain, _ = timed(False)
    s.set_sources(rng.random((4, 3)), rng.standard_normal((4, 3)), f0, 1.2 / f0, 1.0)
    s.set_receivers(rng.random((64, 3)))
    timed(True)                                       # warm-up of the recorded path
    rec, tr = timed(True)
    s.close()
    dofs = 9 * K * Np * steps
    return {"workload": f"N={N}, {n}^3x6 = {K} tets, Fourier media, 4 Ricker forces "
                        f"(f0 in [5,15]), 64 receivers sampled every step, {steps} steps, "
                        f"{args.precision}",
            "value": dofs / rec, "unit": "DOF-updates/s", "plain_value": dofs / plain,
            "overhead_frac": rec / plain - 1.0,
            "max_abs_trace": float(np.abs(tr).max())}


def order7_layered(args, steps=20):
    """The order-7 workload: 24^3 x 6 = 82,944 tets, five layers whose
    interfaces cut through elements, BF16x3 contractions.  Rate of the
    BF16x3 and FP64 GPU paths (both on the matrix cores) over `steps` steps
    of a smooth state (plane P and S waves plus a Gaussian pulse) and the
    per-field error of the BF16x3 state against the FP64 one."""
    import synth
    from paper_2008_09441_amd import B, Solver
    n, N = 24, 7
    dt = 0.5 * (1.0 / n) / math.sqrt(2.0) / (4.5 * (N + 1) ** 2)
    res, states = {}, {}
    q0 = None
    for prec in ("bf16x3", "fp64"):
        s = Solver(N, precision=prec, flux="upwind", device=0)
        s.upload_mesh(synth.kuhn_cube_vertices(n))
        B.dg_material_upload(s.ctx, *(synth.layered_media(s.quad_coords())
                                      + synth.layered_media(s.node_coords())))
        if q0 is None:
            q0 = s.project_function(lambda x: synth.plane_p_wave(x, 0.1) + synth.plane_s_wave(x, 0.2)
                                    + synth.gaussian_pulse(x, width=0.1))
            q0 = q0.astype(np.float32).astype(np.float64)
        K, Np, _, _ = s.sizes()
        s.set_state(q0)
        s.run(0.0, dt, 1)                              # warm-up step
        s.set_state(q0)
        s.synchronize()
        t0 = time.perf_counter()
        s.run(0.0, dt, steps)
        s.synchronize()
        sec = time.perf_counter() - t0
        res[prec] = {"value": 9 * K * Np * steps / sec, "ms_per_stage": sec / (5 * steps) * 1e3}
        states[prec] = s.get_state().astype(np.float64)
        s.close()
    d = (states["bf16x3"] - states["fp64"]).reshape(9, -1)
    r = states["fp64"].reshape(9, -1)
    err = np.linalg.norm(d, axis=1) / np.linalg.norm(r, axis=1)
    # matrix-core roofline: the dense contractions (D_r, D_s, D_t, LIFT, V_q,
    # P_q over nine fields) of one element-stage, against the dense bf16 peak
    # divided by the three products of a BF16x3 split product
    Nfp, Nq = (N + 1) * (N + 2) // 2, (N + 1) ** 3
    flop = 2 * 9 * (3 * Np * Np + Np * 4 * Nfp + 2 * Nq * Np)
    achieved = flop * K / (res["bf16x3"]["ms_per_stage"] * 1e-3) / 1e12
    peak = 2500.0 / 3.0
    # the FP64 path's same contractions against the 78.6 TFLOP/s FP64 peak
    a64 = flop * K / (res["fp64"]["ms_per_stage"] * 1e-3) / 1e12
    res["fp64"]["kernel"] = stage_kernel_name("fp64", N)
    res["fp64"]["roofline"] = {"bound": "fp64", "achieved": a64, "peak": 78.6,
                               "unit": "TFLOP/s", "frac": a64 / 78.6}
    return {"workload": f"N=7 (Np=120), {n}^3x6 = 82944 tets, 5 layers (interfaces inside "
                        f"elements, cp contrast 3x), smooth state, upwind, {steps} steps",
            "kernel": stage_kernel_name("bf16x3", N), "unit": "DOF-updates/s",
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                         "frac": achieved / peak, "flop_per_element_stage": flop},
            "bf16x3": res["bf16x3"], "fp64_path": res["fp64"],
            "speedup_vs_fp64_path": res["bf16x3"]["value"] / res["fp64"]["value"],
            "rel_l2_vs_fp64_per_field": [float(x) for x in err]}


def serving(args, precision="fp32", batched=False, rate=None):
    """Continuous batching of independent solves: a seeded Poisson stream of
    requests (periodic Kuhn cubes, N in {3, 4, 5}, smooth random media, one
    Ricker force with f0 in [5, 15], 16 receivers), admitted by HBM budget.
    Per-request mode: each request on its own stream, advanced by captured
    hipGraphs of 10 steps.  Batched mode: the running requests of each order
    advance together through one slot table, one launch per stage for the
    whole group (dg_batch_advance), 10-step chunks.  Latency = finish -
    arrival.  Default: 64 requests, n in [8, 24], 100-200 steps;
    --serving-full: the full stream, 256 requests, n in [8, 32], 100-800
    steps (progress on stderr as requests complete)."""
    from paper_2008_09441_amd.serving import Server, poisson_workload
    rate = args.serving_rate if rate is None else rate
    if args.serving_full:
        nreq, n_range, steps = 256, (8, 32), (100, 800)
    else:
        nreq, n_range, steps = args.serving_requests, (8, 24), (100, 200)
    reqs = poisson_workload(nreq, rate=rate, n_range=n_range, orders=(3, 4, 5),
                            steps=steps, nrec=16, precision=precision, seed=2008)
    srv = Server(hbm_budget=64 << 30, max_active=16, chunk=10, graphs=True, workers=4,
                 batched=batched)

    def progress(r):
        print(f"serving {precision}: request {r.rid} done, latency {r.latency:.2f} s",
              file=sys.stderr, flush=True)
    srv.run(reqs, on_result=progress if args.serving_full else None)
    st = dict(srv.stats)
    if batched:
        st["batch_chunks"] = srv.batch_launches
    st["workload"] = (f"{len(reqs)} Poisson requests at {rate}/s, periodic "
                      f"n^3x6 Kuhn cubes n in [{n_range[0]},{n_range[1]}], N in {{3,4,5}}, "
                      f"{steps[0]}-{steps[1]} LSRK(5,4) steps, {precision}, smooth random media "
                      "(4 Fourier modes), 1 Ricker force (f0 in [5,15]), 16 receivers; 16 slots, "
                      "64 GiB budget, 10-step chunks, "
                      + ("batched: one launch per stage per order over a slot table"
                         if batched else "per-request captured graphs"))
    return st


def adjoint(args):
    """Gradient of an L2 receiver misfit with respect to the material fields
    rho, lam, mu (at the quadrature points and at the nodes): order 4 on
    24^3 x 6 tets (--adjoint-n), smooth random media, 4 Ricker forces, 64 receivers,
    checkpoint every 20 steps, FP32, upwind.  libdg returns dJ/dm for the
    weight-adjusted weights m = (1/rho, lam, mu) and dJ/d(Zp, Zs) for the
    flux impedances; the field gradient follows by the chain rule.  Times
    the checkpointed forward run and the reverse sweep; the directional
    derivative is checked against a central difference of the same GPU run
    that perturbs the fields (weights and impedances recomputed)."""
    import synth
    from paper_2008_09441_amd import B, Solver
    n, N, steps, every = args.adjoint_n, 4, args.adjoint_steps, 20
    s = Solver(N, precision="fp32", flux="upwind", device=0)
    s.upload_mesh(synth.kuhn_cube_vertices(n))
    xq, xn = s.quad_coords(), s.node_coords()
    rq, pq, sq = synth.fourier_media(xq, seed=77)
    rn, pn, sn = synth.fourier_media(xn, seed=77)
    P = [rq, rq * (pq ** 2 - 2 * sq ** 2), rq * sq ** 2, rn, rn * (pn ** 2 - 2 * sn ** 2),
         rn * sn ** 2]

    def weights(PP):
        a, b, c, d_, e, f = PP
        return np.stack([1.0 / a, b, c]), np.sqrt(d_ * (e + 2 * f)), np.sqrt(d_ * f)
    m, zp, zs = weights(P)
    del xq, xn
    K, Np, _, Nq = s.sizes()
    rng = np.random.default_rng(5)
    f0 = rng.uniform(5.0, 15.0, 4)
    B.dg_material_set_weights(s.ctx, m[0], m[1], m[2], zp, zs)
    s.set_sources(rng.random((4, 3)), rng.standard_normal((4, 3)), f0, 1.2 / f0, 1.0)
    s.set_receivers(rng.random((64, 3)))
    dt = 0.5 * (1.0 / n) / math.sqrt(2.0) / (4.0 * (N + 1) ** 2)
    zero = np.zeros((9, K, Np), np.float32)
    tr = np.empty((steps, 64, 3), np.float32)

    def J(PP):
        mm, zzp, zzs = weights(PP)
        B.dg_material_set_weights(s.ctx, mm[0], mm[1], mm[2], zzp, zzs)
        s.set_state(zero)
        B.dg_adjoint_forward(s.ctx, 0.0, dt, steps, every, tr)
        return tr.astype(np.float64)
    d = 0.5 * J(P)                                 # synthetic data: half the signal
    s.set_state(zero)
    t0 = time.perf_counter()
    B.dg_adjoint_forward(s.ctx, 0.0, dt, steps, every, tr)
    t_fwd = time.perf_counter() - t0
    resid = (tr.astype(np.float64) - d).astype(np.float32)
    g = np.empty((3, K, Nq))
    gz = np.empty((2, K, Np))
    t0 = time.perf_counter()
    B.dg_adjoint_backward(s.ctx, resid, g, gz)
    t_bwd = time.perf_counter() - t0
    a_, b_, c_, d_, e_, f_ = P
    gP = [-g[0] / a_ ** 2, g[1], g[2],
          gz[0] * (e_ + 2 * f_) / (2 * zp) + gz[1] * f_ / (2 * zs),
          gz[0] * d_ / (2 * zp), gz[0] * d_ / zp + gz[1] * d_ / (2 * zs)]
    dP = [rng.standard_normal(p.shape) * p * 0.1 for p in P]
    eps = 1e-2   # FP32 misfits: a larger step keeps the quotient's rounding error down
    fd = (0.5 * np.sum((J([p + eps * q for p, q in zip(P, dP)]) - d) ** 2)
          - 0.5 * np.sum((J([p - eps * q for p, q in zip(P, dP)]) - d) ** 2)) / (2 * eps)
    an = float(sum(np.sum(x * y) for x, y in zip(gP, dP)))
    s.close()
    dofs = 9 * K * Np * steps
    return {"workload": f"N={N}, {n}^3x6 = {K} tets, smooth random media, 4 Ricker forces, "
                        f"64 receivers, {steps} LSRK steps, checkpoint every {every}, fp32, "
                        "upwind; gradient in rho, lam, mu at the quadrature points and nodes "
                        "(weights and flux impedances)",
            "forward_s": t_fwd, "backward_s": t_bwd, "backward_over_forward": t_bwd / t_fwd,
            "adjoint_dof_updates_per_s": dofs / t_bwd,
            "directional_derivative": an, "central_difference": fd,
            "rel_diff_vs_central_difference": abs(fd - an) / max(abs(fd), 1e-300)}


def config1(args):
    """The order-3 plane-wave workload: n = 4 (384 tets), N = 3, rho = 1,
    cp = 2, cs = 1, plane P wave along (1,1,0), upwind, LSRK(5,4) to T = 0.5
    at CFL 0.5, FP64 on the GPU.  Too small for a roofline: reported as the
    latency of a step (the 182-step run timed with HIP events after a
    warm-up run) and as its error against the exact solution; plus the
    convergence sweep n = 2, 4, 8, 16 at the same order to T = 0.1, with
    the order fitted over the three finest meshes."""
    import torch
    import synth
    from paper_2008_09441_amd import Solver

    def run(n, T, timed=False):
        s = Solver(3, precision="fp64", flux="upwind", device=0)
        s.upload_mesh(synth.kuhn_cube_vertices(n))
        s.upload_media(synth.homogeneous_media)
        q0 = s.project_function(lambda x: synth.plane_p_wave(x, 0.0))
        # dt from the CFL rule with h_min of the Kuhn cube (3 vol / max face area)
        hmin = (1.0 / n) / math.sqrt(2.0)
        nst = int(math.ceil(T / (0.5 * hmin / (2.0 * 16.0)) - 1e-12))
        dt = T / nst
        ms = None
        if timed:
            s.set_state(q0)
            s.run(0.0, dt, nst)                      # warm-up run
            st = torch.cuda.current_stream(0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.set_state(q0)
            torch.cuda.synchronize()
            e0.record(st)
            s.run(0.0, dt, nst)
            e1.record(st)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / nst
        else:
            s.set_state(q0)
            s.run(0.0, dt, nst)
        q = s.get_state()
        qe = s.project_function(lambda x: synth.plane_p_wave(x, T))
        norm = QuadNormOf(s)
        err = math.sqrt(norm.sq(q - qe).sum() / norm.sq(qe).sum())
        s.close()
        return err, nst, ms
    err, nst, ms = run(4, 0.5, timed=True)
    sweep = [(n,) + run(n, 0.1)[:2] for n in (2, 4, 8, 16)]
    errs = np.array([e for _, e, _ in sweep])
    h = 1.0 / np.array([n for n, _, _ in sweep], dtype=np.float64)
    slope = float(np.polyfit(np.log(h[1:]), np.log(errs[1:]), 1)[0])
    return {"workload": "N=3, 4^3x6 = 384 tets, rho=1 cp=2 cs=1, plane P wave along (1,1,0), "
                        "upwind, LSRK(5,4) to T=0.5 at CFL 0.5, fp64",
            "steps": nst, "ms_per_step": ms, "us_per_stage": ms * 1e3 / 5,
            "rel_l2_error_vs_exact": err,
            "convergence": {"T": 0.1, "n": [n for n, _, _ in sweep],
                            "rel_l2_error": [float(e) for e in errs],
                            "steps": [k for _, _, k in sweep],
                            "fitted_order_n4_to_16": slope}}


class QuadNormOf(QuadNorm):
    """The quadrature L2 norm of QuadNorm for an existing solver's mesh."""

    def __init__(self, s):
        from paper_2008_09441_amd import B
        Vq = B.dg_ref_operator(s.ctx, 4)
        w = B.dg_ref_operator(s.ctx, 7)[:, 3]
        self.M = Vq.T @ (w[:, None] * Vq)
        _, _, self.J = B.dg_geometry(s.ctx)


def measured_peaks():
    """The box's achievable rates, beside the published peaks the rooflines
    use: a device-to-device copy of 2 GiB (bytes read plus written per
    second) and a dense 8192^3 bf16 GEMM through torch (the library GEMM on
    the matrix cores), each timed over ten repetitions with HIP events."""
    import torch
    st = torch.cuda.current_stream(0)

    def timed(fn, reps=10):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    x = torch.empty(512 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
    x.fill_(1.0)
    y = torch.empty_like(x)
    copy_gbps = 2 * x.numel() * 4 / timed(lambda: y.copy_(x)) / 1e9
    del x, y
    n = 8192
    a = torch.randn(n, n, dtype=torch.bfloat16, device="cuda:0")
    b = torch.randn(n, n, dtype=torch.bfloat16, device="cuda:0")
    gemm_tflops = 2 * n ** 3 / timed(lambda: torch.matmul(a, b)) / 1e12
    del a, b
    torch.cuda.empty_cache()
    from paper_2008_09441_amd import B
    own_copy = B.dg_measure_copy(0, 2 << 30, 10)
    own_mfma = B.dg_measure_mfma(0, 10)
    return {"hbm_copy_GBps": own_copy, "mfma_bf16_TFLOPs": own_mfma,
            "torch_copy_GBps": copy_gbps, "torch_bf16_gemm_TFLOPs": gemm_tflops,
            "published": {"hbm_GBps": 8000.0, "bf16_dense_TFLOPs": 2500.0},
            "method": "libdg dg_measure_copy (hand-written 16 B/lane copy of 2 GiB) and "
                      "dg_measure_mfma (8 chains of v_mfma_f32_16x16x32_bf16 per wave); "
                      "torch 2 GiB device copy and 8192^3 bf16 matmul beside them; "
                      "HIP events over 10 reps"}


def cpu_baseline(args, N):
    """The oracle (FP64 NumPy, untuned) on a bounded sample: one LSRK(5,4)
    step on the n_s^3 x 6 periodic cube with the same order, media and
    initial condition (per-element work identical to the full workload)."""
    import synth
    from oracle.dg import ElasticDG
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    ns = args.cpu_sample_n
    op = ElasticDG(ns, N, synth.fourier_media)
    q0 = op.project_function(synth.gaussian_pulse)
    hmin = (1.0 / ns) / math.sqrt(2.0)
    dt = 0.5 * hmin / (4.0 * (N + 1) ** 2)
    # whole LSRK steps until at least 10 s of CPU time have been spent
    q, res, steps = q0, np.zeros_like(q0), 0
    t0 = time.perf_counter()
    while True:
        q, res = op.step(q, res, dt, t=steps * dt)
        steps += 1
        sec = time.perf_counter() - t0
        if sec >= 10.0:
            break
    dofs = 9 * op.K * op.Np
    return {"value": dofs * steps / sec, "unit": "DOF-updates/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{steps} LSRK(5,4) steps of the FP64 NumPy oracle on the {ns}^3x6 "
                      f"= {op.K}-tet periodic cube, N={N}, same media and pulse "
                      f"({sec:.1f} s)"}


def progress(msg):
    """One line on stderr as each measurement finishes (stdout keeps the JSON)."""
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not "
              "supported (the multi-GPU element partition is design-only)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2008_09441_amd import Solver  # noqa: F401  (fails loudly if unbuilt)
    N, n = args.order, args.n
    K = 6 * n ** 3
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    hmin = (1.0 / n) / math.sqrt(2.0)     # 3 vol / max face area of a Kuhn tet
    dt = 0.5 * hmin / (4.0 * (N + 1) ** 2)
    cache = {}

    if args.calibrate_copy:
        # kernels of known traffic for the counter runs: a fill (writes 256
        # MiB), a sum (reads 256 MiB) and a copy (reads and writes 256 MiB)
        x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        x.fill_(1.0)
        float(x.sum())
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    s = setup(args, args.precision)
    upload_media_and_state(s, cache)
    sec, wall = timed_run(s, dt, args.steps, args.warmup)
    q_lo = s.get_state().astype(np.float64)
    s.close()
    del s
    torch.cuda.empty_cache()
    progress(f"{args.precision} path timed: {sec / args.steps * 1e3:.3f} ms per step")

    dofs = 9 * K * Np
    value = dofs * args.steps / sec
    ms_step = sec / args.steps * 1e3
    stage_s = sec / (5 * args.steps)
    eb = 8 if args.precision == "fp64" else 4
    bytes_launch = alg_bytes_per_elem_stage(N, eb) * K
    achieved = bytes_launch / stage_s / 1e9
    kernel = stage_kernel_name(args.precision, N)

    out = {
        "metric": "DG DOF-updates/sec (FP32/BF16x3 vs FP64 at stated L2 error); batched p50/p99",
        "value": value, "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16x3": "bf16x3+f32acc"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"elastic velocity-stress DG, N={N} (Np={Np}), periodic "
                               f"{n}^3x6 = {K} Kuhn tets, Fourier-mode media, Gaussian "
                               f"pulse, upwind, LSRK(5,4) CFL 0.5",
                   "order": N, "elements": K, "dofs": dofs, "precision": args.precision,
                   "dt": dt},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                     "frac": achieved / 8000.0,
                     "traffic": measured_traffic(kernel, args.precision, N, K),
                     "kernel": kernel,
                     "alg_bytes_per_launch": bytes_launch,
                     "avg_launch_us": stage_s * 1e6},
        "wall_s_timed": wall,
    }

    def other_path(prec):
        so = setup(args, prec)
        upload_media_and_state(so, cache)
        sec_o, _ = timed_run(so, dt, args.steps, args.warmup)
        q_o = so.get_state().astype(np.float64)
        so.close()
        del so
        torch.cuda.empty_cache()
        return sec_o, q_o

    if not args.no_fp32_path and args.precision == "bf16x3":
        sec32, q32 = other_path("fp32")
        out["fp32_path"] = {"value": dofs * args.steps / sec32,
                            "ms_per_step": sec32 / args.steps * 1e3,
                            "kernel": stage_kernel_name("fp32", N)}
        # FP32 matrix cores: dense contraction flops of an element-stage
        # (D_r, D_s, D_t, LIFT, V_q, P_q over nine fields) per launch
        Np, Nfp, Nq = (N + 1) * (N + 2) * (N + 3) // 6, (N + 1) * (N + 2) // 2, (N + 1) ** 3
        flop = 2 * 9 * (3 * Np * Np + Np * 4 * Nfp + 2 * Nq * Np)
        a32 = flop * K / (sec32 / (5 * args.steps)) / 1e12
        out["fp32_path"]["roofline"] = {"bound": "mfma", "achieved": a32, "peak": 157.3,
                                        "unit": "TFLOP/s", "frac": a32 / 157.3,
                                        "flop_per_element_stage": flop}
        progress("fp32 path timed")
    if not args.no_fp64_reference and args.precision != "fp64":
        sec64, q64 = other_path("fp64")
        out["fp64_path"] = {"value": dofs * args.steps / sec64,
                            "ms_per_step": sec64 / args.steps * 1e3,
                            "kernel": stage_kernel_name("fp64", N)}
        # the FP64 comparator against its own roofline: the dense
        # contractions of an element-stage (D_r, D_s, D_t, LIFT, V_q, P_q over
        # nine fields; 261,450 flop at order 4) against the 78.6 TFLOP/s FP64
        # peak, and its FP64 algorithmic bytes against HBM
        Np_, Nfp_, Nq_ = (N + 1) * (N + 2) * (N + 3) // 6, (N + 1) * (N + 2) // 2, (N + 1) ** 3
        dense = 2 * 9 * (3 * Np_ * Np_ + Np_ * 4 * Nfp_ + 2 * Nq_ * Np_)
        f64_stage = sec64 / (5 * args.steps)
        a64 = dense * K / f64_stage / 1e12
        out["fp64_path"]["roofline"] = {
            "bound": "fp64", "achieved": a64, "peak": 78.6, "unit": "TFLOP/s",
            "frac": a64 / 78.6, "flop_per_element_stage": dense,
            "hbm_frac": alg_bytes_per_elem_stage(N, 8) * K / f64_stage / 8e12}
        out["speedup_vs_fp64_path"] = sec64 / sec
        progress("fp64 path timed")
        norm = QuadNorm(args)
        out["l2_vs_fp64"] = {"norm": "quadrature L2 after warmup+steps", **norm.errors(q_lo, q64)}
        if "fp32_path" in out:
            out["fp32_path"]["l2_vs_fp64"] = norm.errors(q32, q64)
        from paper_2008_09441_amd import Solver
        sq = Solver(N, precision="fp64", flux="upwind", device=-1)   # host tables only
        sq.upload_mesh(__import__("synth").kuhn_cube_vertices(n))
        en = EnergyNorm(sq, *cache["media"][:3])
        sq.close()
        if args.precision in ENERGY_BOUND:
            out["l2_vs_fp64"]["energy"] = en.errors(q_lo, q64, args.precision)
            out["within_bound"] = out["l2_vs_fp64"]["energy"]["within_bound"]
        if "fp32_path" in out:
            out["fp32_path"]["l2_vs_fp64"]["energy"] = en.errors(q32, q64, "fp32")
            out["fp32_path"]["within_bound"] = out["fp32_path"]["l2_vs_fp64"]["energy"]["within_bound"]
        del en
        torch.cuda.empty_cache()
        progress("errors against the fp64 path computed")
    if not args.no_config1:
        out["config1_plane_wave_order3"] = config1(args)
        progress("configuration 1 measured")
    if not args.no_sources:
        out["sources_receivers"] = sources_receivers(args)
        progress("sources and receivers measured")
    if not args.no_order7:
        out["order7_layered"] = order7_layered(args)
        progress("order 7 measured")
    if not args.no_serving and args.serving_full:
        # the full stream: one run per listed precision, per-request graphs
        # (or batched with --serving-batched), at --serving-rate
        for prec in args.serving_precisions.split(","):
            out[f"serving_full_{prec}"] = serving(args, prec, batched=args.serving_batched)
    elif not args.no_serving:
        for prec in args.serving_precisions.split(","):
            out["serving" if prec == "fp32" else f"serving_{prec}"] = serving(args, prec)
        out["serving_batched"] = serving(args, "fp32", batched=True)
        # capacity: every request arrives within a fraction of a second, so
        # the queue never empties and the rate is the server's, not the stream's
        out["serving_saturated"] = {
            "note": "arrivals at 1000/s: the rate is the capacity of the server",
            "graphs_fp32": serving(args, "fp32", batched=False, rate=1000.0),
            "batched_fp32": serving(args, "fp32", batched=True, rate=1000.0),
            "batched_bf16x3": serving(args, "bf16x3", batched=True, rate=1000.0)}
    if not args.no_adjoint:
        out["adjoint"] = adjoint(args)
        progress("adjoint measured")
    if not args.no_peaks:
        out["peaks_measured"] = measured_peaks()
        progress("peaks measured")
        out["roofline"]["frac_of_measured_copy"] = (
            out["roofline"]["achieved"] / out["peaks_measured"]["hbm_copy_GBps"])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, N)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
