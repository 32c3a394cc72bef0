/*
 * libdg: nodal discontinuous-Galerkin right-hand side and low-storage
 * Runge-Kutta stepping for the velocity-stress elastic wave equation on
 * periodic tetrahedral meshes, on one AMD Instinct MI355X (gfx950).
 *
 * The mounted paper (sparse-grid noise reduction for particle-in-cell) does
 * not define this operation; each call below cites the standard published
 * formulation it follows:
 *   [HW08]  Hesthaven & Warburton, Nodal Discontinuous Galerkin Methods
 *           (2008), Ch. 2-3, 6, 10: nodal basis, strong-form DG, LIFT.
 *   [WSG10] Wilcox, Stadler, Burstedde & Ghattas, JCP 229 (2010): exact
 *           Riemann (upwind) flux for isotropic elasticity.
 *   [CHW17] Chan, Hewett & Warburton, SISC 39 (2017); [C18] Chan, IJNME 113
 *           (2018): weight-adjusted mass inverse for variable coefficients.
 *   [CK94]  Carpenter & Kennedy, NASA TM-109112 (1994): LSRK(5,4).
 *
 * Conventions shared with callers:
 *   - fields, in order: v_x, v_y, v_z, s_xx, s_yy, s_zz, s_yz, s_xz, s_xy;
 *   - state layout [9][K][Np] (structure of arrays; Np = (N+1)(N+2)(N+3)/6),
 *     element type double for DG_FP64, float for DG_FP32 / DG_FP32_BF16X3;
 *   - reference nodes: equispaced on the reference tetrahedron with vertices
 *     (-1,-1,-1), (1,-1,-1), (-1,1,-1), (-1,-1,1), enumerated t-index
 *     outermost, then s, then r; node p of element k sits at
 *     x0 + F (r+1, s+1, t+1), F = [x1-x0, x2-x0, x3-x0] / 2;
 *   - quadrature: collapsed Gauss-Jacobi rule, Nq = (N+1)^3 points, point
 *     q = ia + (N+1) (ib + (N+1) ic), exact to degree 2N+1.
 *
 * Errors: every call returns a dg_status; arguments are validated on the
 * host before any device work; dg_last_error() gives a message.  Device
 * work is stream-ordered on the context's stream and asynchronous unless
 * stated; asynchronous device faults surface on the next synchronising
 * call.  The library never aborts the process.
 */
#ifndef DG_H_
#define DG_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_ctx dg_ctx;
typedef struct dg_batch dg_batch;

/* No C++ exception crosses this interface: a host allocation failure inside
 * a call returns DG_ENOMEM, any other internal exception DG_EINVAL. */
typedef enum {
  DG_OK = 0,
  DG_EINVAL = 1,      /* bad argument, size or mesh/material           */
  DG_ENOMEM = 2,      /* device or host allocation failed, or over the HBM budget */
  DG_EDEVICE = 3,     /* HIP error, or compute call on host-only ctx   */
  DG_ESTATE = 4,      /* call out of order (e.g. rhs before material)  */
  DG_ENONFINITE = 5   /* non-finite input                              */
} dg_status;

/* DG_FP64: FP64 state and arithmetic (the dense contractions on the FP64
 * matrix cores, 16x16x4 products, at every order).
 * DG_FP32: FP32 state and arithmetic, with the
 * dense contractions on the FP32 matrix cores (16x16x4 products).
 * DG_FP32_BF16X3: FP32 state, the dense contractions as split products of
 * bf16 hi/lo parts on the matrix cores with FP32 accumulation (three
 * products each, about 2^-16 relative error per product). */
typedef enum { DG_FP64 = 0, DG_FP32 = 1, DG_FP32_BF16X3 = 2 } dg_precision;
typedef enum { DG_FLUX_UPWIND = 0, DG_FLUX_CENTRAL = 1 } dg_flux;

typedef struct {
  int32_t order;             /* N, 1..7 (else DG_EINVAL)                         */
  int32_t precision;         /* dg_precision                                     */
  int32_t flux;              /* dg_flux                                          */
  int32_t device;            /* HIP device ordinal; -1 = host-only (no GPU work) */
  void* stream;              /* hipStream_t to order work on; NULL = default     */
  uint64_t hbm_budget_bytes; /* 0 = unlimited                                    */
} dg_options;

/* Create a context.  *out receives the handle (NULL on failure).  The
 * reference element of order N is built here in FP64 on the host [HW08]. */
dg_status dg_create(dg_ctx** out, const dg_options* opt);

/* Destroy a context and free its device memory.  NULL is allowed. */
void dg_destroy(dg_ctx* ctx);

/* Message for the last failed call on ctx (never NULL). */
const char* dg_last_error(const dg_ctx* ctx);

/* Sizes: K (elements; 0 before mesh upload), Np, Nfp, Nq.  Any out pointer
 * may be NULL. */
dg_status dg_sizes(const dg_ctx* ctx, int64_t* K, int32_t* Np, int32_t* Nfp,
                   int32_t* Nq);

/* Upload a periodic conforming tetrahedral mesh.  vxyz: host [K][4][3]
 * per-element vertex coordinates (unwrapped; positive orientation
 * required); period: host [3] box lengths > 0 of the periodic domain.
 * Computes connectivity (faces matched by centroid modulo the period, trace
 * permutations from the vertex correspondence) and affine geometric factors
 * in FP64 [HW08, Ch. 10], then copies them to the device (cast to the
 * working precision).  Host arrays are copied; the caller keeps ownership.
 * Errors: DG_EINVAL (non-positive orientation, unmatched face), DG_ENOMEM. */
dg_status dg_mesh_upload(dg_ctx* ctx, int64_t K, const double* vxyz,
                         const double* period);

/* Physical coordinates of the nodes [K][Np][3] / quadrature points
 * [K][Nq][3] into host arrays, so callers can sample media and initial
 * conditions.  Requires a mesh. */
dg_status dg_node_coords(const dg_ctx* ctx, double* xyz);
dg_status dg_quad_coords(const dg_ctx* ctx, double* xyz);

/* Upload isotropic media.  rho_q, cp_q, cs_q: host [K][Nq] samples at the
 * quadrature points (for the weight-adjusted mass inverse [CHW17, C18]);
 * rho_n, cp_n, cs_n: host [K][Np] samples at the nodes (impedances
 * Zp = rho cp, Zs = rho cs for the upwind flux [WSG10]).  Stored on the
 * device as 1/rho, lam = rho (cp^2 - 2 cs^2), mu = rho cs^2 and Zp, Zs.
 * Errors: DG_EINVAL for rho <= 0, cs <= 0 or cp^2 < 2 cs^2 (lam < 0 is
 * allowed down to the cp >= sqrt(2) cs bound), DG_ENONFINITE for NaN/Inf. */
dg_status dg_material_upload(dg_ctx* ctx, const double* rho_q, const double* cp_q,
                             const double* cs_q, const double* rho_n,
                             const double* cp_n, const double* cs_n);

/* Host FP64 L2 projection of quadrature samples onto the nodal basis:
 * q[f][k][:] = P_q fq[f][k][:] for f < nfields.  fq: [nfields][K][Nq],
 * q: [nfields][K][Np], both host. */
dg_status dg_project(const dg_ctx* ctx, int32_t nfields, const double* fq, double* q);

/* Set the state (and the LSRK residual) to zero with a device fill kernel:
 * no host transfer.  Stream-ordered. */
dg_status dg_state_zero(dg_ctx* ctx);

/* Set / get the context's state [9][K][Np] (working precision).  on_device
 * != 0: q is a device pointer (copied stream-ordered); else host (the call
 * synchronises).  dg_state_set also zeroes the LSRK residual. */
dg_status dg_state_set(dg_ctx* ctx, const void* q, int32_t on_device);
dg_status dg_state_get(dg_ctx* ctx, void* q, int32_t on_device);

/* Device pointer of the context's current state [9][K][Np] (valid until the
 * next dg_step / dg_run, which swap buffers). */
dg_status dg_state_device_ptr(dg_ctx* ctx, void** ptr);

/* Semi-discrete right-hand side rhs = dq/dt at time t for a caller-owned
 * device state q_dev [9][K][Np] into caller-owned device rhs_dev [9][K][Np]
 * (working precision; must not alias): volume terms div(sigma), eps(v)
 * [HW08, Ch. 10], flux of the selected type at every face node gathered
 * through the neighbour tables [WSG10], LIFT, then the weight-adjusted mass
 * inverse [CHW17, C18], plus the point sources' terms at time t (see
 * dg_sources_set).  Stream-ordered, asynchronous. */
dg_status dg_rhs(dg_ctx* ctx, const void* q_dev, void* rhs_dev, double t);

/* One LSRK(5,4) step [CK94] of the context's state from time t with step
 * dt: five fused stages res <- a_s res + dt rhs(q, t + c_s dt);
 * q <- q + b_s res.  Stream-ordered, asynchronous. */
dg_status dg_step(dg_ctx* ctx, double t, double dt);

/* nsteps LSRK(5,4) steps from t0.  Stream-ordered, asynchronous. */
dg_status dg_run(dg_ctx* ctx, double t0, double dt, int64_t nsteps);

/* Point forces with Ricker time signals.  Source i acts at xyz[i] (host
 * [nsrc][3], any periodic image) in direction dir[i] (host [nsrc][3]) with
 * f_i(t) = amp[i] (1 - 2 a^2) exp(-a^2), a = pi f0[i] (t - t0[i]).  The
 * force enters the velocity rows of the element containing the point as
 * M_k^-1 l(x^_i) f_i(t) dir[i] (the nodal basis evaluated at the point,
 * [HW08, Ch. 10]) and passes through the weight-adjusted mass inverse
 * [CHW17, C18] like every other term; the responses are precomputed in FP64
 * on the host from the device material and recomputed when the material
 * changes.  Replaces any earlier set; nsrc = 0 removes all.  Host arrays
 * are copied.  Errors: DG_ESTATE before mesh and material, DG_EINVAL for a
 * point outside the mesh or f0 <= 0, DG_ENONFINITE, DG_EDEVICE for a
 * host-only context.  Synchronises the context's stream. */
dg_status dg_sources_set(dg_ctx* ctx, int32_t nsrc, const double* xyz, const double* dir,
                         const double* f0, const double* t0, const double* amp);

/* Receivers at xyz (host [nrec][3], any periodic image): the velocity there
 * is the polynomial of the containing element evaluated at the point.
 * Replaces any earlier set; nrec = 0 removes all.  Errors as for
 * dg_sources_set (mesh needed, material not).  Synchronises the stream. */
dg_status dg_receivers_set(dg_ctx* ctx, int32_t nrec, const double* xyz);

/* Velocity at the receivers for the current state into out [nrec][3]
 * (working precision): device pointer if on_device != 0 (stream-ordered),
 * else host (synchronous).  DG_ESTATE without receivers or state. */
dg_status dg_receivers_sample(dg_ctx* ctx, void* out, int32_t on_device);

/* nsteps LSRK(5,4) steps from t0, sampling the receivers after every step
 * into trace [nsteps][nrec][3] (working precision): device pointer if
 * on_device != 0 (stream-ordered), else host (the library stages the trace
 * in device memory it owns and copies it at the end; synchronous). */
dg_status dg_run_record(dg_ctx* ctx, double t0, double dt, int64_t nsteps, void* trace,
                        int32_t on_device);

/* ---- Runs on the device clock (for captured graphs and serving) --------
 * Each context keeps a device-resident clock (time, step count).  Runs on
 * it read the time from device memory, so their launch arguments do not
 * depend on the time and a captured run can be replayed at any time. */

/* Set the clock to time t and step count 0 (stream-ordered). */
dg_status dg_time_set(dg_ctx* ctx, double t);

/* Read the clock (synchronises the stream).  Either pointer may be NULL. */
dg_status dg_time_get(dg_ctx* ctx, double* t, int64_t* step);

/* Library-owned device trace [max_steps][nrec][3] (working precision) that
 * dg_advance fills: after the i-th step of a run that starts at clock step
 * s, row s + i receives the receiver velocities; rows at or beyond
 * max_steps are not written, rows not yet written are undefined.  Needs
 * receivers (DG_ESTATE); replaced by a later call or dg_receivers_set.
 * Counted against the HBM budget.  Synchronises the stream. */
dg_status dg_trace_reserve(dg_ctx* ctx, int64_t max_steps);

/* Copy the first nrows rows of the trace to host memory out (synchronous). */
dg_status dg_trace_copy(dg_ctx* ctx, void* out, int64_t nrows);

/* nsteps LSRK(5,4) steps [CK94] from the device clock: stage s of step i
 * evaluates the sources at clock time + (i + c_s) dt, the receivers are
 * recorded into the trace after every step, then the clock advances by
 * nsteps steps.  Stream-ordered, asynchronous. */
dg_status dg_advance(dg_ctx* ctx, double dt, int64_t nsteps);

/* As dg_advance, but the launches of the run are captured once into a
 * hipGraph per (dt, nsteps, starting state buffer) and replayed on later
 * calls.  Needs a context created with its own stream (DG_ESTATE
 * otherwise).  Graphs are dropped when sources, receivers, the trace, the
 * material or the mesh change. */
dg_status dg_graph_advance(dg_ctx* ctx, double dt, int64_t nsteps);

/* ---- Batched stepping (continuous batching of many solves) -------------
 * Many independent contexts of one order and precision advanced together:
 * each LSRK stage of the whole batch is one launch of the context's stage
 * kernel over a slot table (every context owns a range of workgroups and
 * runs the same per-tile arithmetic as alone, so each result is
 * bit-identical alone and in a batch), followed by one source launch, and
 * after each step one receiver launch, for all slots.  Each context steps
 * on its own device clock with its own dt, exactly as dg_advance would, and
 * may join or leave the batch between calls. */

/* A batch object: a device slot table for up to max_slots contexts of
 * `device` (allocated here, max_slots * a few hundred bytes).  DG_EINVAL
 * for a bad device or max_slots outside 1 .. 65536, DG_ENOMEM. */
dg_status dg_batch_create(dg_batch** out, int32_t device, int32_t max_slots);
void dg_batch_destroy(dg_batch* b);   /* waits for the device first */

/* nsteps LSRK(5,4) steps [CK94] of every context in ctxs[0..n): context i
 * with time step dt[i] from its device clock, sources and receivers as in
 * dg_advance.  All contexts: distinct, on the batch's device, same order,
 * FP32 or DG_FP32_BF16X3, with mesh, material and state (DG_EINVAL /
 * DG_ESTATE, reported in ctxs[0]'s dg_last_error).  Launches on `stream`
 * (a hipStream_t; NULL: ctxs[0]'s stream); the caller orders the contexts'
 * own streams against it (the serving loop creates every context of a batch
 * on that stream).  Asynchronous.  The slot table is rewritten by every
 * call; calls on one batch object are stream-ordered. */
dg_status dg_batch_advance(dg_batch* b, void* stream, dg_ctx* const* ctxs, int32_t n,
                           const double* dt, int64_t nsteps);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * as dg_batch_advance, but the slot table lives in a static device array of
 * the library (64 slots, 17,920 bytes per GPU, held until the process
 * ends; its address is resolved once per device on the first call there).
 * Calls no hipMalloc, hipFree or other allocating routine.  More than 64
 * contexts: DG_EINVAL.  Every call on a GPU rewrites that GPU's one table,
 * so calls that overlap on one GPU (from several host threads, or on
 * streams not ordered against each other) race: order them. */
dg_status dg_batch_advance_noalloc(void* stream, dg_ctx* const* ctxs, int32_t n,
                                   const double* dt, int64_t nsteps);

/* ---- Discrete adjoint ---------------------------------------------------
 * Gradient of a receiver misfit with respect to the material: the
 * weight-adjusted weights m = (1/rho, lam, mu) at the quadrature points
 * [CHW17, C18] and, for the upwind flux, the impedances Zp = rho cp and
 * Zs = rho cs at the nodes that the exact-Riemann flux reads [WSG10]; a
 * gradient with respect to rho, lam, mu fields follows by the chain rule.
 * FP64 and FP32 contexts (DG_EINVAL for DG_FP32_BF16X3). */

/* Set the weights directly: 1/rho, lam, mu host [K][Nq], impedances Zp, Zs
 * host [K][Np] (all copied).  Errors: DG_ESTATE before the mesh,
 * DG_ENONFINITE, DG_EINVAL for non-positive impedances. */
dg_status dg_material_set_weights(dg_ctx* ctx, const double* irho_q, const double* lam_q,
                                  const double* mu_q, const double* zp_n, const double* zs_n);

/* nsteps LSRK(5,4) steps from the current state (host time t0 + i dt),
 * keeping a copy of the state every `every` steps on the device and writing
 * the receiver velocities after every step to trace (host
 * [nsteps][nrec][3], working precision).  Leaves the context at the end of
 * the run.  Needs receivers (DG_ESTATE).  Library-owned device memory:
 * ceil(nsteps/every) + 5 every + 6 states (FP32 at orders 1-4: 10 every + 6,
 * the replay also keeping R y of every stage input, or 20 every + 6 when
 * that much fits, so that the replay of the next interval overlaps the
 * reverse sweep of this one) plus face-node work arrays
 * ([K][4 Nfp][9], two of them on the generic adjoint kernels) and the FP64
 * gradient [3][K][Nq] (upwind: also [K][4 Nfp][4] impedance terms, [K][4
 * Nfp][8] face jumps on the tiled FP32 kernels of orders 1-4, and the FP64
 * gradient [2][K][Np]), counted against the HBM budget.  Upwind on those
 * tiled kernels, the replay also keeps the [K][4 Nfp][8] face jumps of every
 * stage input (5 every of them, 10 every with the overlap) when they fit
 * after everything else; otherwise the reverse stage recomputes them from
 * the stage input, with the same results up to rounding.  These buffers are
 * kept from one call to the next; an optional one (the second interval, the
 * jumps) that did not fit is not tried again for the same sizes until the
 * next dg_mesh_upload. */
dg_status dg_adjoint_forward(dg_ctx* ctx, double t0, double dt, int64_t nsteps, int64_t every,
                             void* trace);

/* Reverse sweep of the last dg_adjoint_forward run for a misfit J with
 * dJ/d(trace) = resid (host [nsteps][nrec][3], working precision): the
 * discrete adjoint of every stage (transposed weight-adjusted inverse,
 * transposed volume, flux and LIFT operators, receiver adjoint), with the
 * states of each checkpoint interval recomputed from its checkpoint.
 * grad: host double [3][K][Nq] = dJ/d(1/rho, lam, mu) at the quadrature
 * points.  grad_z: host double [2][K][Np] = dJ/d(Zp, Zs) at the nodes, or
 * NULL to skip it (zero for the central flux, which reads no impedance).
 * The context's state is not changed.  Synchronous.  DG_ESTATE when no
 * forward run is recorded, or the mesh, material, sources or receivers
 * changed since it. */
dg_status dg_adjoint_backward(dg_ctx* ctx, const void* resid, double* grad, double* grad_z);

/* Device bytes the context holds (the amount counted against its HBM
 * budget). */
dg_status dg_memory(const dg_ctx* ctx, uint64_t* bytes);

/* Device bytes a context of this order and precision will hold for a mesh
 * of K elements with nsrc sources, nrec receivers and a trace of
 * trace_steps rows (an upper bound: the face-pattern table is counted at
 * its maximum size), so that a scheduler can admit work by HBM budget
 * before creating the context.  No device needed. */
dg_status dg_footprint(int32_t order, int32_t precision, int64_t K, int32_t nsrc, int32_t nrec,
                       int64_t trace_steps, uint64_t* bytes);

/* Wait for the context's stream; reports asynchronous device errors. */
dg_status dg_synchronize(dg_ctx* ctx);

/* Host FP64 precompute, exported for cross-checking (no device needed).
 * which: 0 Dr, 1 Ds, 2 Dt [Np][Np]; 3 LIFT [Np][4 Nfp] (face-major
 * columns, face node order of dg_face_nodes); 4 Vq [Nq][Np]; 5 Pq [Np][Nq];
 * 6 nodes [Np][3]; 7 quadrature points and weights [Nq][4]. */
dg_status dg_ref_operator(const dg_ctx* ctx, int32_t which, double* out);

/* Face node masks [4][Nfp] (volume node index of each face node). */
dg_status dg_face_nodes(const dg_ctx* ctx, int32_t* fmask);

/* Connectivity after dg_mesh_upload: neighbour element [K][4], neighbour
 * face [K][4], and neighbour volume node of each own face node
 * [K][4][Nfp]; geometry: metric terms [K][9] (d rst_i / d x_j), face data
 * [K][4][4] (outward unit normal, Fscale = sJ/J), J [K].  Any pointer may
 * be NULL. */
dg_status dg_connectivity(const dg_ctx* ctx, int32_t* etoe, int32_t* etof,
                          int32_t* nbnode);
dg_status dg_geometry(const dg_ctx* ctx, double* geo, double* fgeo, double* J);

/* Tile processing order of the matrix-core stage (any precision; no device
 * needed): out[ceil(K/16)] is the 16-element tile that launch position p
 * processes.  Positions are dealt to the eight XCDs in contiguous ranges;
 * the order puts the tiles into eight slabs along the axis of largest
 * extent and sweeps each slab along its longest remaining axis (coordinates
 * bucketed by the typical element size, ties in element order), so that
 * face-neighbour tiles run close together on one XCD's L2.  A permutation
 * of 0 .. ceil(K/16) - 1.  DG_ESTATE before dg_mesh_upload. */
dg_status dg_tile_order(const dg_ctx* ctx, int32_t* out);

/* ---- Measured rates of the device (reference for rooflines) ------------
 * dg_measure_copy: a hand-written streaming copy of `bytes` bytes (16 B per
 * lane and access), bytes read plus bytes written per second, in GB/s.
 * dg_measure_mfma: eight independent chains of v_mfma_f32_16x16x32_bf16 per
 * wave, eight waves per SIMD, no memory traffic: the dense bf16 matrix-core
 * rate in TFLOP/s.  Each is timed with HIP events over `reps` launches after
 * a warm-up launch, on the null stream of `device`, with buffers allocated
 * and freed here.  DG_EINVAL for bad arguments, DG_ENOMEM, DG_EDEVICE. */
dg_status dg_measure_copy(int32_t device, int64_t bytes, int32_t reps, double* gbytes_per_s);
dg_status dg_measure_mfma(int32_t device, int32_t reps, double* tflops);

#ifdef __cplusplus
}
#endif
#endif /* DG_H_ */
