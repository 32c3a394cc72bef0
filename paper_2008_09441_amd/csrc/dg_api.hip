// C-ABI of libdg: context, uploads, right-hand side, LSRK(5,4) stepping.
// The function contracts are documented in include/dg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/dg.h"
#include "dg_host.hpp"
#include "dg_kernels.hpp"
#include "dg_be.hpp"
#include "dg_bx.hpp"
#include "dg_src.hpp"
#include "dg_adj.hpp"
#include "dg_adjt.hpp"
#include "dg_batch.hpp"
#include "dg_peaks.hpp"
#include "dg_mfma_host.hpp"

namespace {

// LSRK(5,4) coefficients [CK94]
const double kRkA[5] = {0.0,
                        -567301805773.0 / 1357537059087.0,
                        -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0,
                        -1275806237668.0 / 842570457699.0};
const double kRkB[5] = {1432997174477.0 / 9575080441755.0,
                        5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0,
                        3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};
const double kRkC[5] = {0.0,
                        1432997174477.0 / 9575080441755.0,
                        2526269341429.0 / 6820363962896.0,
                        2006345519317.0 / 3224310063776.0,
                        2802321613138.0 / 2924317926251.0};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

// a batch: the device slot table of dg_batch_advance and its host image
struct dg_batch {
  int device = 0;
  int max_slots = 0;
  void* table = nullptr;
  std::vector<dgb::BatchSlot> host;
};

struct dg_ctx {
  dg_options opt{};
  std::string err;
  dgh::RefElement re;
  dgh::MeshData mesh;
  bool has_mesh = false, has_mat = false, has_state = false;
  hipStream_t stream = nullptr;
  size_t elem = 8;          // bytes of the working precision
  size_t allocated = 0;     // device bytes held
  // device arrays
  DevBuf ops;               // Dr | Ds | Dt | LIFT | Vq | Pq
  DevBuf opsT;              // transposed: DrT | DsT | DtT | LIFTT | VqT | PqT
  DevBuf fmask, geo, fgeo, etoe, etop, pat;
  DevBuf irho, lam, mu, zp, zs;
  DevBuf q[2], res;
  DevBuf frags;             // BF16x3: operator hi/lo fragments
  DevBuf matblk;            // BF16x3: material blocked by 16-element tile
  DevBuf nbn;               // BF16x3: neighbour volume node of each face node
  DevBuf torder;            // BF16x3: tile processed at each launch position
  int cur = 0;
  // point sources: specification (host) and device arrays
  struct Source {
    double x[3], d[3], f0, t0, amp;
  };
  std::vector<Source> src;
  DevBuf src_elem;          // int64 [nsrc]
  DevBuf src_w;             // working precision [nsrc][3][Np]
  DevBuf src_par;           // double [nsrc][3]: f0, t0, amplitude
  // receivers
  int32_t nrec = 0;
  DevBuf rec_elem;          // int64 [nrec]
  DevBuf rec_w;             // working precision [nrec][Np]
  DevBuf rec_buf;           // working precision scratch for host-side traces
  // device clock (time, step count) and the receiver trace it indexes
  DevBuf clk;               // double [2]
  DevBuf trace;             // working precision [trace_cap][nrec][3]
  int64_t trace_cap = 0;
  // captured runs: (dt, steps, starting state buffer) -> executable graph
  struct Graph {
    double dt;
    int64_t nsteps;
    int cur;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
  DevBuf src_wraw;          // raw source vectors (before the mass inverse)
  // discrete adjoint: tables, checkpoints and work arrays
  DevBuf adj_nbface, adj_invf;
  DevBuf adj_ck;            // checkpoints [nck][9][K][Np]
  DevBuf adj_seg;           // stage inputs of one segment [every][5][9][K][Np]
  DevBuf adj_v;             // ly, lres, mu, nu, r, res [6][9][K][Np]
  DevBuf adj_gb, adj_hb;    // face-node work [K][4 Nfp][9]
  DevBuf adj_grad;          // double [3][K][Nq]
  DevBuf adj_zb;            // upwind: impedance terms per face node [K][4 Nfp][4]
                            // (tiled adjoint: face-node jumps [K][4 Nfp][8])
  DevBuf adj_gradz;         // upwind: double [2][K][Np]
  DevBuf adj_frag;          // FP32 orders 1-4: fragments of the tiled adjoint kernel
  DevBuf adj_r;             // FP32 orders 1-4: R y of every stage input of a segment,
                            // [every][5][9][K][Np] (stored by the replay)
  bool adj_ov = false;      // adj_seg and adj_r hold two segments: the replay of
                            // the next segment overlaps the reverse sweep
  DevBuf adj_j;             // FP32 orders 1-4, upwind, when it fits: the face-node
                            // jumps of every stage input of a segment (as adj_r),
                            // [every][5][K][4 Nfp][8], stored by the replay
  size_t adj_ov_failed = 0; // interval sizes (bytes of one segment, of the jumps) whose
  size_t adj_j_failed = 0;  // optional buffers did not fit: not tried again for this mesh
  DevBuf adj_trace;         // [nsteps][nrec][3]
  bool adj_ready = false;
  double adj_t0 = 0.0, adj_dt = 0.0;
  int64_t adj_nsteps = 0, adj_every = 0;
  int32_t adj_nrec = 0;     // receivers of the recorded forward run
};

namespace {

dg_status fail(dg_ctx* c, dg_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define DG_HIP(ctx, call)                                                        \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      return fail(ctx, DG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

bool device_ctx(const dg_ctx* c) { return c->opt.device >= 0; }

// The 16-element-tile matrix-core stage (dg_bx.hpp) runs every precision at
// orders 1-4 (BF16x3, FP32 and FP64 products); it reads the blocked
// material, the neighbour-node table and the tile order.  The [K][Nq]
// material is held by every other context and by FP32 and FP64 ones too
// (adjoint, sources).
bool tiled_kernel(int32_t precision, int order) {
  return order <= 4 &&
         (precision == DG_FP32_BF16X3 || precision == DG_FP32 || precision == DG_FP64);
}
bool plain_material(int32_t precision, int order) {
  return !(precision == DG_FP32_BF16X3 && order <= 4);
}
// FP32 and BF16x3 contexts (launch_mfma: the tiled kernel at orders 1-4, one
// element per workgroup at 5-7); FP64 contexts run the FP64 matrix-core
// kernels through launch_stage.
bool tiled_mfma(const dg_ctx* c) {
  return c->opt.precision == DG_FP32_BF16X3 || c->opt.precision == DG_FP32;
}
// FP32 contexts of orders 1-4 run the reverse stage on the tiled adjoint
// kernel (matrix cores); the others on the generic adjoint kernels
bool adj_tiled(const dg_ctx* c) { return c->opt.precision == DG_FP32 && c->re.N <= 4; }

dg_status set_device(dg_ctx* c) {
  if (!device_ctx(c)) return fail(c, DG_EDEVICE, "host-only context: no device work");
  DG_HIP(c, hipSetDevice(c->opt.device));
  return DG_OK;
}

void release(dg_ctx* c, DevBuf& b) {
  if (b.p) {
    (void)hipFree(b.p);
    c->allocated -= b.bytes;
  }
  b = DevBuf();
}

dg_status alloc(dg_ctx* c, DevBuf& b, size_t bytes) {
  release(c, b);
  if (bytes == 0) return DG_OK;
  if (c->opt.hbm_budget_bytes && c->allocated + bytes > c->opt.hbm_budget_bytes)
    return fail(c, DG_ENOMEM, "allocation of " + std::to_string(bytes) +
                                  " bytes exceeds the HBM budget");
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess)
    return fail(c, DG_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  b.p = p;
  b.bytes = bytes;
  c->allocated += bytes;
  return DG_OK;
}

// synchronous copy ordered on the context's own stream: the library never
// uses the legacy null stream when the context has a stream of its own, so
// other contexts' captures and non-blocking streams are not disturbed
hipError_t copy_sync(const dg_ctx* c, void* dst, const void* src, size_t bytes,
                     hipMemcpyKind kind) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, c->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(c->stream);
}

// upload an FP64 host array cast to the working precision
dg_status upload_real(dg_ctx* c, DevBuf& b, const double* src, size_t n) {
  dg_status s = alloc(c, b, n * c->elem);
  if (s != DG_OK) return s;
  if (c->elem == 8) {
    DG_HIP(c, copy_sync(c, b.p, src, n * 8, hipMemcpyHostToDevice));
  } else {
    std::vector<float> tmp(n);
    for (size_t i = 0; i < n; ++i) tmp[i] = float(src[i]);
    DG_HIP(c, copy_sync(c, b.p, tmp.data(), n * 4, hipMemcpyHostToDevice));
  }
  return DG_OK;
}

template <typename U>
dg_status upload_raw(dg_ctx* c, DevBuf& b, const U* src, size_t n) {
  dg_status s = alloc(c, b, n * sizeof(U));
  if (s != DG_OK) return s;
  DG_HIP(c, copy_sync(c, b.p, src, n * sizeof(U), hipMemcpyHostToDevice));
  return DG_OK;
}

// ---------------------------------------------------------------- launch --
// FP64 stage on the matrix cores at orders 1-4: the tiled kernel with FP64
// fragments and v_mfma_f64_16x16x4f64 (dg_bx.hpp)
template <int N>
hipError_t launch_mfma_d(const dg_ctx* c, const double* q_in, double* q_out, double* res,
                         double* rhs_out, double a, double b, double dt, int lsrk) {
  dgb::BxArgsT<double> A{};
  A.q_in = q_in;
  A.q_out = q_out;
  A.res = res;
  A.rhs_out = rhs_out;
  A.geo = static_cast<const double*>(c->geo.p);
  A.fgeo = static_cast<const double*>(c->fgeo.p);
  A.nbn = static_cast<const int32_t*>(c->nbn.p);
  A.torder = static_cast<const int32_t*>(c->torder.p);
  A.fmask = static_cast<const int32_t*>(c->fmask.p);
  A.mat = static_cast<const double*>(c->matblk.p);
  A.zp = static_cast<const double*>(c->zp.p);
  A.zs = static_cast<const double*>(c->zs.p);
  A.frags = static_cast<const dgb::u32x4*>(c->frags.p);
  A.K = c->mesh.K;
  A.a = a;
  A.b = b;
  A.dt = dt;
  A.lsrk = lsrk;
  A.upwind = c->opt.flux == DG_FLUX_UPWIND ? 1 : 0;
  const int64_t tiles = (c->mesh.K + dgb::kTile - 1) / dgb::kTile;
  if (tiles > 0x7fffffff) return hipErrorInvalidValue;
  dgb::stage_bx_d<N><<<dim3(unsigned(tiles)), dim3(dgb::kThreads), 0, c->stream>>>(A);
  return hipGetLastError();
}

// FP64 stage on the matrix cores at orders 5-7: one element per workgroup
// with FP64 fragments and v_mfma_f64_16x16x4f64 (dg_be.hpp)
template <int N>
hipError_t launch_be_d(const dg_ctx* c, const double* q_in, double* q_out, double* res,
                       double* rhs_out, double a, double b, double dt, int lsrk) {
  dgb::BeArgsT<double> A;
  A.q_in = q_in;
  A.q_out = q_out;
  A.res = res;
  A.rhs_out = rhs_out;
  A.geo = static_cast<const double*>(c->geo.p);
  A.fgeo = static_cast<const double*>(c->fgeo.p);
  A.nbn = static_cast<const int32_t*>(c->nbn.p);
  A.fmask = static_cast<const int32_t*>(c->fmask.p);
  A.irho = static_cast<const double*>(c->irho.p);
  A.lam = static_cast<const double*>(c->lam.p);
  A.mu = static_cast<const double*>(c->mu.p);
  A.zp = static_cast<const double*>(c->zp.p);
  A.zs = static_cast<const double*>(c->zs.p);
  A.frags = static_cast<const dgb::u32x4*>(c->frags.p);
  A.K = c->mesh.K;
  A.a = a;
  A.b = b;
  A.dt = dt;
  A.lsrk = lsrk;
  A.upwind = c->opt.flux == DG_FLUX_UPWIND ? 1 : 0;
  if (c->mesh.K > 0x7fffffff) return hipErrorInvalidValue;
  dgb::stage_be_d<N><<<dim3(unsigned(c->mesh.K)), dim3(dgb::kThreads), 0, c->stream>>>(A);
  return hipGetLastError();
}

// FP64 contexts: the matrix-core kernels in double precision (the tiled
// kernel at orders 1-4, one element per workgroup at 5-7), as FP32 and
// BF16x3 contexts run on the matrix cores at every order (launch_mfma)
hipError_t launch_stage_f64(const dg_ctx* c, const double* q_in, double* q_out, double* res,
                            double* rhs_out, double a, double b, double dt, int lsrk) {
  switch (c->re.N) {
    case 1: return launch_mfma_d<1>(c, q_in, q_out, res, rhs_out, a, b, dt, lsrk);
    case 2: return launch_mfma_d<2>(c, q_in, q_out, res, rhs_out, a, b, dt, lsrk);
    case 3: return launch_mfma_d<3>(c, q_in, q_out, res, rhs_out, a, b, dt, lsrk);
    case 4: return launch_mfma_d<4>(c, q_in, q_out, res, rhs_out, a, b, dt, lsrk);
    case 5: return launch_be_d<5>(c, q_in, q_out, res, rhs_out, a, b, dt, lsrk);
    case 6: return launch_be_d<6>(c, q_in, q_out, res, rhs_out, a, b, dt, lsrk);
    case 7: return launch_be_d<7>(c, q_in, q_out, res, rhs_out, a, b, dt, lsrk);
    default: return hipErrorInvalidValue;
  }
}

dg_status launch_stage(dg_ctx* c, const void* q_in, void* q_out, void* res, void* rhs_out,
                       double a, double b, double dt, int lsrk) {
  if (c->elem != 8) return fail(c, DG_EDEVICE, "stage launch: not an FP64 context");
  const hipError_t e = launch_stage_f64(
      c, static_cast<const double*>(q_in), static_cast<double*>(q_out),
      static_cast<double*>(res), static_cast<double*>(rhs_out), a, b, dt, lsrk);
  if (e != hipSuccess) return fail(c, DG_EDEVICE, std::string("stage launch: ") + hipGetErrorString(e));
  return DG_OK;
}

template <int N, bool F32, bool RST = false>
hipError_t launch_mfma_n(dg_ctx* c, const float* q_in, float* q_out, float* res, float* rhs_out,
                         double a, double b, double dt, int lsrk, float* r_out = nullptr,
                         float* j_out = nullptr) {
  dgb::BxArgs A{};
  A.q_in = q_in;
  A.q_out = q_out;
  A.res = res;
  A.rhs_out = rhs_out;
  A.geo = static_cast<const float*>(c->geo.p);
  A.fgeo = static_cast<const float*>(c->fgeo.p);
  A.nbn = static_cast<const int32_t*>(c->nbn.p);
  A.torder = static_cast<const int32_t*>(c->torder.p);
  A.fmask = static_cast<const int32_t*>(c->fmask.p);
  A.mat = static_cast<const float*>(c->matblk.p);
  A.zp = static_cast<const float*>(c->zp.p);
  A.zs = static_cast<const float*>(c->zs.p);
  A.frags = static_cast<const dgb::u32x4*>(c->frags.p);
  A.K = c->mesh.K;
  A.a = float(a);
  A.b = float(b);
  A.dt = float(dt);
  A.lsrk = lsrk;
  A.upwind = c->opt.flux == DG_FLUX_UPWIND ? 1 : 0;
  // one workgroup per tile of 16 elements
  const int64_t tiles = (c->mesh.K + dgb::kTile - 1) / dgb::kTile;
  if (tiles > 0x7fffffff) return hipErrorInvalidValue;
  A.r_out = r_out;
  A.j_out = j_out;
  if constexpr (RST)
    dgb::stage_bx_r<N><<<dim3(unsigned(tiles)), dim3(dgb::kThreads), 0, c->stream>>>(A);
  else
    dgb::stage_bx<N, F32><<<dim3(unsigned(tiles)), dim3(dgb::kThreads), 0, c->stream>>>(A);
  return hipGetLastError();
}

template <int N, bool F32>
hipError_t launch_mfma_e(dg_ctx* c, const float* q_in, float* q_out, float* res, float* rhs_out,
                         double a, double b, double dt, int lsrk) {
  dgb::BeArgs A;
  A.q_in = q_in;
  A.q_out = q_out;
  A.res = res;
  A.rhs_out = rhs_out;
  A.geo = static_cast<const float*>(c->geo.p);
  A.fgeo = static_cast<const float*>(c->fgeo.p);
  A.nbn = static_cast<const int32_t*>(c->nbn.p);
  A.fmask = static_cast<const int32_t*>(c->fmask.p);
  A.irho = static_cast<const float*>(c->irho.p);
  A.lam = static_cast<const float*>(c->lam.p);
  A.mu = static_cast<const float*>(c->mu.p);
  A.zp = static_cast<const float*>(c->zp.p);
  A.zs = static_cast<const float*>(c->zs.p);
  A.frags = static_cast<const dgb::u32x4*>(c->frags.p);
  A.K = c->mesh.K;
  A.a = float(a);
  A.b = float(b);
  A.dt = float(dt);
  A.lsrk = lsrk;
  A.upwind = c->opt.flux == DG_FLUX_UPWIND ? 1 : 0;
  // one workgroup per element
  if (c->mesh.K > 0x7fffffff) return hipErrorInvalidValue;
  dgb::stage_be<N, F32><<<dim3(unsigned(c->mesh.K)), dim3(dgb::kThreads), 0, c->stream>>>(A);
  return hipGetLastError();
}

dg_status launch_mfma(dg_ctx* c, const void* q_in, void* q_out, void* res, void* rhs_out,
                      double a, double b, double dt, int lsrk) {
  const float* qi = static_cast<const float*>(q_in);
  float* qo = static_cast<float*>(q_out);
  float* rs = static_cast<float*>(res);
  float* ro = static_cast<float*>(rhs_out);
  hipError_t e;
  const bool f32 = c->opt.precision == DG_FP32;
  switch (c->re.N) {
    case 1: e = f32 ? launch_mfma_n<1, true>(c, qi, qo, rs, ro, a, b, dt, lsrk)
                    : launch_mfma_n<1, false>(c, qi, qo, rs, ro, a, b, dt, lsrk); break;
    case 2: e = f32 ? launch_mfma_n<2, true>(c, qi, qo, rs, ro, a, b, dt, lsrk)
                    : launch_mfma_n<2, false>(c, qi, qo, rs, ro, a, b, dt, lsrk); break;
    case 3: e = f32 ? launch_mfma_n<3, true>(c, qi, qo, rs, ro, a, b, dt, lsrk)
                    : launch_mfma_n<3, false>(c, qi, qo, rs, ro, a, b, dt, lsrk); break;
    case 4: e = f32 ? launch_mfma_n<4, true>(c, qi, qo, rs, ro, a, b, dt, lsrk)
                    : launch_mfma_n<4, false>(c, qi, qo, rs, ro, a, b, dt, lsrk); break;
    case 5: e = f32 ? launch_mfma_e<5, true>(c, qi, qo, rs, ro, a, b, dt, lsrk)
                    : launch_mfma_e<5, false>(c, qi, qo, rs, ro, a, b, dt, lsrk); break;
    case 6: e = f32 ? launch_mfma_e<6, true>(c, qi, qo, rs, ro, a, b, dt, lsrk)
                    : launch_mfma_e<6, false>(c, qi, qo, rs, ro, a, b, dt, lsrk); break;
    case 7: e = f32 ? launch_mfma_e<7, true>(c, qi, qo, rs, ro, a, b, dt, lsrk)
                    : launch_mfma_e<7, false>(c, qi, qo, rs, ro, a, b, dt, lsrk); break;
    default: e = hipErrorInvalidValue;
  }
  if (e != hipSuccess)
    return fail(c, DG_EDEVICE, std::string("matrix-core stage launch: ") + hipGetErrorString(e));
  return DG_OK;
}

dg_status stage(dg_ctx* c, const void* q_in, void* q_out, void* res, void* rhs_out, double a,
                double b, double dt, int lsrk) {
  if (tiled_mfma(c)) return launch_mfma(c, q_in, q_out, res, rhs_out, a, b, dt, lsrk);
  return launch_stage(c, q_in, q_out, res, rhs_out, a, b, dt, lsrk);
}

dg_status fill_zero(dg_ctx* c, void* p, int64_t n) {
  const int64_t nb = (n + 255) / 256;
  if (c->elem == 8)
    hipLaunchKernelGGL(dgk::fill_kernel<double>, dim3(unsigned(nb)), dim3(256), 0, c->stream,
                       static_cast<double*>(p), n, 0.0);
  else
    hipLaunchKernelGGL(dgk::fill_kernel<float>, dim3(unsigned(nb)), dim3(256), 0, c->stream,
                       static_cast<float*>(p), n, 0.0f);
  DG_HIP(c, hipGetLastError());
  return DG_OK;
}

// 1/rho at the quadrature points of element k, read back from the device
// material in the layout of the context's precision
dg_status device_irho(dg_ctx* c, int64_t k, std::vector<double>& out) {
  const int Nq = c->re.Nq;
  out.assign(Nq, 0.0);
  if (!plain_material(c->opt.precision, c->re.N)) {
    for (int p = 0; p < Nq; ++p) {
      float v = 0.f;
      const size_t idx = dgh::mfma_material_index(c->re.N, k, p, 0);
      DG_HIP(c, copy_sync(c, &v, static_cast<const float*>(c->matblk.p) + idx, 4,
                          hipMemcpyDeviceToHost));
      out[p] = v;
    }
  } else if (c->elem == 8) {
    DG_HIP(c, copy_sync(c, out.data(), static_cast<const double*>(c->irho.p) + k * Nq, 8 * Nq,
                        hipMemcpyDeviceToHost));
  } else {
    std::vector<float> tmp(Nq);
    DG_HIP(c, copy_sync(c, tmp.data(), static_cast<const float*>(c->irho.p) + k * Nq, 4 * Nq,
                        hipMemcpyDeviceToHost));
    for (int p = 0; p < Nq; ++p) out[p] = tmp[p];
  }
  return DG_OK;
}

// Device arrays of the point sources: element, response after the mass
// inverse P_q[(1/rho) V_q (V psi(x^_s) / J_k)] d (FP64 on the host, from the
// device material), Ricker parameters.
dg_status upload_sources(dg_ctx* c) {
  const int Np = c->re.Np, Nq = c->re.Nq;
  const size_t ns = c->src.size();
  release(c, c->src_elem);
  release(c, c->src_w);
  release(c, c->src_wraw);
  release(c, c->src_par);
  if (ns == 0) return DG_OK;
  std::vector<int64_t> elem(ns);
  std::vector<double> w(ns * 3 * Np), wraw(ns * 3 * Np), par(ns * 3);
  std::vector<double> psi(Np), raw(Np), rq(Nq), irho;
  for (size_t i = 0; i < ns; ++i) {
    const dg_ctx::Source& S = c->src[i];
    int64_t k = -1;
    double rst[3];
    if (!dgh::locate_point(c->re, c->mesh, S.x, k, rst))
      return fail(c, DG_EINVAL, "sources: point outside the mesh");
    elem[i] = k;
    dgh::basis_at(c->re, rst[0], rst[1], rst[2], psi.data());
    for (int n = 0; n < Np; ++n) {
      double acc = 0.0;
      for (int m = 0; m < Np; ++m) acc += c->re.V[size_t(n) * Np + m] * psi[m];
      raw[n] = acc / c->mesh.J[k];
      for (int d = 0; d < 3; ++d) wraw[(i * 3 + d) * Np + n] = S.d[d] * raw[n];
    }
    dg_status st = device_irho(c, k, irho);
    if (st != DG_OK) return st;
    for (int p = 0; p < Nq; ++p) {
      double acc = 0.0;
      for (int n = 0; n < Np; ++n) acc += c->re.Vq[size_t(p) * Np + n] * raw[n];
      rq[p] = irho[p] * acc;
    }
    for (int n = 0; n < Np; ++n) {
      double acc = 0.0;
      for (int p = 0; p < Nq; ++p) acc += c->re.Pq[size_t(n) * Nq + p] * rq[p];
      for (int d = 0; d < 3; ++d) w[(i * 3 + d) * Np + n] = S.d[d] * acc;
    }
    par[3 * i] = S.f0;
    par[3 * i + 1] = S.t0;
    par[3 * i + 2] = S.amp;
  }
  dg_status st;
  if ((st = upload_raw(c, c->src_elem, elem.data(), ns)) != DG_OK) return st;
  if ((st = upload_real(c, c->src_w, w.data(), w.size())) != DG_OK) return st;
  if ((st = upload_real(c, c->src_wraw, wraw.data(), wraw.size())) != DG_OK) return st;
  if ((st = upload_raw(c, c->src_par, par.data(), par.size())) != DG_OK) return st;
  return DG_OK;
}

// out1 += alpha f(t) w, out2 += beta f(t) w for every source
dg_status launch_sources(dg_ctx* c, void* out1, void* out2, double t, double alpha,
                         double beta) {
  const int ns = int(c->src.size());
  if (ns == 0) return DG_OK;
  const int Np = c->re.Np;
  const int64_t KNp = c->mesh.K * Np;
  const unsigned nb = unsigned((3 * Np + 255) / 256);
  const int64_t* el = static_cast<const int64_t*>(c->src_elem.p);
  const double* par = static_cast<const double*>(c->src_par.p);
  if (c->elem == 8)
    dgs::source_add<double><<<nb, 256, 0, c->stream>>>(
        static_cast<double*>(out1), static_cast<double*>(out2), el,
        static_cast<const double*>(c->src_w.p), par, ns, Np, KNp, t, alpha, beta);
  else
    dgs::source_add<float><<<nb, 256, 0, c->stream>>>(
        static_cast<float*>(out1), static_cast<float*>(out2), el,
        static_cast<const float*>(c->src_w.p), par, ns, Np, KNp, t, alpha, beta);
  DG_HIP(c, hipGetLastError());
  return DG_OK;
}

// velocity at the receivers of the current state into out (device, [nrec][3])
dg_status launch_receivers(dg_ctx* c, void* out) {
  if (c->nrec == 0) return DG_OK;
  const int Np = c->re.Np;
  const int64_t KNp = c->mesh.K * Np;
  const unsigned nb = unsigned((3 * c->nrec + 255) / 256);
  const int64_t* el = static_cast<const int64_t*>(c->rec_elem.p);
  if (c->elem == 8)
    dgs::receiver_sample<double><<<nb, 256, 0, c->stream>>>(
        static_cast<double*>(out), static_cast<const double*>(c->q[c->cur].p), el,
        static_cast<const double*>(c->rec_w.p), c->nrec, Np, KNp);
  else
    dgs::receiver_sample<float><<<nb, 256, 0, c->stream>>>(
        static_cast<float*>(out), static_cast<const float*>(c->q[c->cur].p), el,
        static_cast<const float*>(c->rec_w.p), c->nrec, Np, KNp);
  DG_HIP(c, hipGetLastError());
  return DG_OK;
}

// captured graphs hold buffer addresses and source/receiver counts: drop
// them whenever those change
void drop_graphs(dg_ctx* c) {
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  c->graphs.clear();
}

// nsteps LSRK(5,4) steps from the device clock: sources read the clock,
// receivers (if a trace is reserved) write row clk_step + i after step i,
// and the clock advances at the end.  Every launch argument is independent
// of the time, so the sequence can be captured once and replayed.
dg_status advance_impl(dg_ctx* c, double dt, int64_t nsteps) {
  const int Np = c->re.Np;
  const int64_t KNp = c->mesh.K * Np;
  double* clk = static_cast<double*>(c->clk.p);
  const int ns = int(c->src.size());
  for (int64_t i = 0; i < nsteps; ++i) {
    for (int st = 0; st < 5; ++st) {
      dg_status s = stage(c, c->q[c->cur].p, c->q[1 - c->cur].p, c->res.p, nullptr, kRkA[st],
                          kRkB[st], dt, 1);
      if (s != DG_OK) return s;
      if (ns > 0) {
        const unsigned nb = unsigned((3 * Np + 255) / 256);
        const int64_t* el = static_cast<const int64_t*>(c->src_elem.p);
        const double* par = static_cast<const double*>(c->src_par.p);
        const double toff = (double(i) + kRkC[st]) * dt;
        if (c->elem == 8)
          dgs::source_add_clk<double><<<nb, 256, 0, c->stream>>>(
              static_cast<double*>(c->res.p), static_cast<double*>(c->q[1 - c->cur].p), el,
              static_cast<const double*>(c->src_w.p), par, ns, Np, KNp, clk, toff, dt,
              kRkB[st] * dt);
        else
          dgs::source_add_clk<float><<<nb, 256, 0, c->stream>>>(
              static_cast<float*>(c->res.p), static_cast<float*>(c->q[1 - c->cur].p), el,
              static_cast<const float*>(c->src_w.p), par, ns, Np, KNp, clk, toff, dt,
              kRkB[st] * dt);
        DG_HIP(c, hipGetLastError());
      }
      c->cur = 1 - c->cur;
    }
    if (c->nrec > 0 && c->trace_cap > 0) {
      const unsigned nb = unsigned((3 * c->nrec + 255) / 256);
      const int64_t* el = static_cast<const int64_t*>(c->rec_elem.p);
      if (c->elem == 8)
        dgs::receiver_sample_clk<double><<<nb, 256, 0, c->stream>>>(
            static_cast<double*>(c->trace.p), c->trace_cap, clk, i,
            static_cast<const double*>(c->q[c->cur].p), el,
            static_cast<const double*>(c->rec_w.p), c->nrec, Np, KNp);
      else
        dgs::receiver_sample_clk<float><<<nb, 256, 0, c->stream>>>(
            static_cast<float*>(c->trace.p), c->trace_cap, clk, i,
            static_cast<const float*>(c->q[c->cur].p), el,
            static_cast<const float*>(c->rec_w.p), c->nrec, Np, KNp);
      DG_HIP(c, hipGetLastError());
    }
  }
  dgs::clock_advance<<<1, 64, 0, c->stream>>>(clk, dt, nsteps);
  DG_HIP(c, hipGetLastError());
  return DG_OK;
}

// ------------------------------------------------------------ adjoint ---
template <typename T>
dga::AdjArgs<T> adj_args(const dg_ctx* c) {
  const dgh::RefElement& re = c->re;
  const int Np = re.Np, NF4 = 4 * re.Nfp, Nq = re.Nq;
  const T* ops = static_cast<const T*>(c->ops.p);   // Dr | Ds | Dt | LIFT | Vq | Pq
  dga::AdjArgs<T> A;
  A.geo = static_cast<const T*>(c->geo.p);
  A.fgeo = static_cast<const T*>(c->fgeo.p);
  A.etoe = static_cast<const int32_t*>(c->etoe.p);
  A.etop = static_cast<const uint8_t*>(c->etop.p);
  A.pat = static_cast<const int32_t*>(c->pat.p);
  A.fmask = static_cast<const int32_t*>(c->fmask.p);
  A.nbface = static_cast<const int32_t*>(c->adj_nbface.p);
  A.invf = static_cast<const int32_t*>(c->adj_invf.p);
  A.zp = static_cast<const T*>(c->zp.p);
  A.zs = static_cast<const T*>(c->zs.p);
  A.Dr = ops;
  A.Ds = ops + size_t(Np) * Np;
  A.Dt = ops + 2 * size_t(Np) * Np;
  A.LIFT = ops + 3 * size_t(Np) * Np;
  A.Vq = A.LIFT + size_t(Np) * NF4;
  A.Pq = A.Vq + size_t(Nq) * Np;
  // the transposed operator pack: DrT | DsT | DtT | LIFTT | VqT | PqT
  A.NpP = 4 * ((Np + 3) / 4);
  A.QP = 32 * ((Nq + 31) / 32);
  const T* opsT = static_cast<const T*>(c->opsT.p);
  A.DrT = opsT;
  A.DsT = opsT + size_t(Np) * A.NpP;
  A.DtT = opsT + 2 * size_t(Np) * A.NpP;
  A.LIFTT = opsT + 3 * size_t(Np) * A.NpP;
  A.VqT = A.LIFTT + size_t(NF4) * A.NpP;
  A.irho = static_cast<const T*>(c->irho.p);
  A.lam = static_cast<const T*>(c->lam.p);
  A.mu = static_cast<const T*>(c->mu.p);
  A.K = c->mesh.K;
  A.Np = Np;
  A.Nfp = re.Nfp;
  A.Nq = Nq;
  A.upwind = c->opt.flux == DG_FLUX_UPWIND ? 1 : 0;
  return A;
}

inline unsigned nblocks(int64_t n) { return unsigned((n + 255) / 256); }

// tables of the flux transpose: for every face node, the neighbour's face
// node that reads it (flat index nb * 4 Nfp + j'), and for every volume node
// the face nodes that lie on it
dg_status adj_tables(dg_ctx* c) {
  if (c->adj_nbface.p) return DG_OK;
  const dgh::RefElement& re = c->re;
  const dgh::MeshData& m = c->mesh;
  const int NF4 = 4 * re.Nfp;
  if (m.K * NF4 >= (int64_t(1) << 31)) return fail(c, DG_EINVAL, "adjoint: mesh too large");
  std::vector<int32_t> nbf, invf;
  std::string err;
  if (!dgh::adjoint_face_tables(re, m, nbf, invf, err)) return fail(c, DG_EINVAL, err);
  dg_status st;
  if (adj_tiled(c)) {
    const std::vector<float> fr = dgh::adj_fragments_f32(re);
    if ((st = upload_raw(c, c->adj_frag, fr.data(), fr.size())) != DG_OK) return st;
  }
  if ((st = upload_raw(c, c->adj_nbface, nbf.data(), nbf.size())) != DG_OK) return st;
  return upload_raw(c, c->adj_invf, invf.data(), invf.size());
}

// one reverse stage on the tiled adjoint kernels (FP32, orders 1-4): lres
// = a lres + b ly, the gradient terms, then ly += dt R^T W^T lres and the
// impedance gradient
template <int N>
void launch_adj_tile(dg_ctx* c, const dgt::TileArgs& A) {
  const unsigned tiles = unsigned((A.K + 15) / 16);
  hipLaunchKernelGGL((dgt::adj_tile<N, true>), dim3(tiles), dim3(dgt::kThreads), 0, c->stream, A);
}

// one FP32 stage of the replay (fused LSRK update) that also stores R q_in
// and, if j_out is not null, the jumps at its face nodes
dg_status stage_raw(dg_ctx* c, const void* q_in, void* q_out, void* res, void* r_out,
                    float* j_out, double a, double b, double dt) {
  const float* qi = static_cast<const float*>(q_in);
  float* qo = static_cast<float*>(q_out);
  float* rs = static_cast<float*>(res);
  float* ro = static_cast<float*>(r_out);
  float* jo = j_out;   // may be null
  hipError_t e;
  switch (c->re.N) {
    case 1: e = launch_mfma_n<1, true, true>(c, qi, qo, rs, nullptr, a, b, dt, 1, ro, jo); break;
    case 2: e = launch_mfma_n<2, true, true>(c, qi, qo, rs, nullptr, a, b, dt, 1, ro, jo); break;
    case 3: e = launch_mfma_n<3, true, true>(c, qi, qo, rs, nullptr, a, b, dt, 1, ro, jo); break;
    case 4: e = launch_mfma_n<4, true, true>(c, qi, qo, rs, nullptr, a, b, dt, 1, ro, jo); break;
    default: return fail(c, DG_EINVAL, "adjoint: no tiled kernel at this order");
  }
  if (e != hipSuccess) return fail(c, DG_EDEVICE, std::string("stage launch: ") + hipGetErrorString(e));
  return DG_OK;
}

// jin: the stage input's face-node jumps as the replay stored them, or null
// (the tile kernel then computes them from y into adj_zb)
dg_status adj_stage_tiled(dg_ctx* c, const float* y, const float* r, const float* jin,
                          float* lres, float* ly, float* nu, double* grad, double* gradz,
                          float a, float b, double dt, double ts) {
  const int64_t K = c->mesh.K;
  const int Np = c->re.Np;
  dgt::TileArgs A{};
  A.y = y;
  A.r = r;
  A.lres = lres;
  A.ly = ly;
  A.nu = nu;
  A.gf = static_cast<float*>(c->adj_gb.p);
  A.jmp = static_cast<float*>(c->adj_zb.p);
  A.grad = grad;
  A.geo = static_cast<const float*>(c->geo.p);
  A.fgeo = static_cast<const float*>(c->fgeo.p);
  A.nbn = static_cast<const int32_t*>(c->nbn.p);
  A.fmask = static_cast<const int32_t*>(c->fmask.p);
  A.mat = static_cast<const float*>(c->matblk.p);
  A.zp = static_cast<const float*>(c->zp.p);
  A.zs = static_cast<const float*>(c->zs.p);
  A.frags = static_cast<const float*>(c->adj_frag.p);
  A.src_elem = static_cast<const int64_t*>(c->src_elem.p);
  A.src_w = static_cast<const float*>(c->src_wraw.p);
  A.src_par = static_cast<const double*>(c->src_par.p);
  A.nsrc = int(c->src.size());
  A.ts = ts;
  A.K = K;
  A.a = a;
  A.b = b;
  A.s = dt;
  A.upwind = c->opt.flux == DG_FLUX_UPWIND ? 1 : 0;
  A.jumps = jin ? 0 : 1;
  if (!A.nbn || !A.mat || !A.frags || !A.fmask || !A.r)
    return fail(c, DG_ESTATE, "adjoint: tiled kernel tables missing");
  switch (c->re.N) {
    case 1: launch_adj_tile<1>(c, A); break;
    case 2: launch_adj_tile<2>(c, A); break;
    case 3: launch_adj_tile<3>(c, A); break;
    case 4: launch_adj_tile<4>(c, A); break;
    default: return fail(c, DG_EINVAL, "adjoint: no tiled kernel at this order");
  }
  DG_HIP(c, hipGetLastError());
  dgt::NodeArgs B{};
  B.nu = nu;
  B.gf = A.gf;
  B.jmp = jin ? jin : A.jmp;
  B.ly = ly;
  B.gradz = gradz;
  B.fgeo = A.fgeo;
  B.zp = A.zp;
  B.zs = A.zs;
  B.nbn = A.nbn;
  B.nbface = static_cast<const int32_t*>(c->adj_nbface.p);
  B.invf = static_cast<const int32_t*>(c->adj_invf.p);
  B.K = K;
  B.Np = Np;
  B.Nfp = c->re.Nfp;
  B.s = dt;
  B.upwind = A.upwind;
  hipLaunchKernelGGL(dgt::adj_nodes, dim3(nblocks(K * Np)), dim3(256), 0, c->stream, B);
  DG_HIP(c, hipGetLastError());
  return DG_OK;
}

// The tiled FP32 sweep (orders 1-4).  Per segment: the replay, whose FP32
// stages store every stage input and its R y, then the reverse stages on the
// tiled adjoint kernels.  With two segment buffers (adj_ov) the replay of
// the next segment runs on a second stream while this one is reversed; the
// results are the same bit for bit.
dg_status adj_backward_tiled(dg_ctx* c, const float* resid) {
  const int Np = c->re.Np, Nq = c->re.Nq;
  const int64_t K = c->mesh.K, n = int64_t(9) * K * Np, KNp = K * Np;
  const float* ck = static_cast<const float*>(c->adj_ck.p);
  float* seg0 = static_cast<float*>(c->adj_seg.p);
  float* rr0 = static_cast<float*>(c->adj_r.p);
  float* jj0 = static_cast<float*>(c->adj_j.p);   // null: the replay keeps no jumps
  float* v = static_cast<float*>(c->adj_v.p);
  // res and res2 (a scratch output for a segment's last stage) are the
  // replay's; ly, lres and nu the reverse sweep's
  float *ly = v, *lres = v + n, *res2 = v + 2 * n, *nu = v + 3 * n, *res = v + 5 * n;
  double* grad = static_cast<double*>(c->adj_grad.p);
  double* gradz = static_cast<double*>(c->adj_gradz.p);
  const double t0 = c->adj_t0, dt = c->adj_dt;
  const int64_t nsteps = c->adj_nsteps, every = c->adj_every;
  const int64_t nck = (nsteps + every - 1) / every;
  const size_t segn = size_t(every) * 5 * size_t(n);
  const size_t jn = size_t(K) * 4 * c->re.Nfp * 8, segj = size_t(every) * 5 * jn;
  const hipStream_t st = c->stream;
  dg_status s;
  if ((s = fill_zero(c, ly, n)) != DG_OK) return s;
  if ((s = fill_zero(c, lres, n)) != DG_OK) return s;
  dgk::fill_kernel<double><<<nblocks(3 * K * Nq), 256, 0, st>>>(grad, 3 * K * Nq, 0.0);
  DG_HIP(c, hipGetLastError());
  if (c->opt.flux == DG_FLUX_UPWIND) {
    dgk::fill_kernel<double><<<nblocks(2 * KNp), 256, 0, st>>>(gradz, 2 * KNp, 0.0);
    DG_HIP(c, hipGetLastError());
  }
  // the replay of segment sg into buffer b, on the context's current stream
  auto replay = [&](int64_t sg, int b) -> dg_status {
    float* seg = seg0 + b * segn;
    float* rr = rr0 + b * segn;
    float* jj = jj0 ? jj0 + b * segj : nullptr;
    const int64_t n0 = sg * every, n1 = std::min(n0 + every, nsteps);
    DG_HIP(c, hipMemcpyAsync(seg, ck + sg * n, n * sizeof(float), hipMemcpyDeviceToDevice,
                             c->stream));
    // the residual is cleared once per segment: as in the forward run, the
    // first stage's a_0 = 0 discards the previous step's (finite) residual
    dg_status e;
    if ((e = fill_zero(c, res, n)) != DG_OK) return e;
    for (int64_t i = n0; i < n1; ++i) {
      float* y = seg + (i - n0) * 5 * n;
      const double ti = t0 + double(i) * dt;
      for (int q = 0; q < 5; ++q) {
        float* out = q < 4 ? y + (q + 1) * n : (i + 1 < n1 ? y + 5 * n : res2);
        const int64_t sl = (i - n0) * 5 + q;
        if ((e = stage_raw(c, y + q * n, out, res, rr + sl * n, jj ? jj + sl * jn : nullptr,
                           kRkA[q], kRkB[q], dt)) != DG_OK)
          return e;
        if ((e = launch_sources(c, res, out, ti + kRkC[q] * dt, dt, kRkB[q] * dt)) != DG_OK)
          return e;
      }
    }
    return DG_OK;
  };
  // the reverse stages of segment sg from buffer b, on the context's stream
  auto reverse = [&](int64_t sg, int b) -> dg_status {
    const float* seg = seg0 + b * segn;
    const float* rr = rr0 + b * segn;
    const float* jj = jj0 ? jj0 + b * segj : nullptr;
    const int64_t n0 = sg * every, n1 = std::min(n0 + every, nsteps);
    dg_status e;
    for (int64_t i = n1 - 1; i >= n0; --i) {
      const float* ys = seg + (i - n0) * 5 * n;
      // misfit sensitivity of the trace row of step i (state after step i)
      if (c->nrec > 0) {
        dga::receiver_adjoint<float><<<nblocks(3 * Np), 256, 0, st>>>(
            ly, resid + i * c->nrec * 3, static_cast<const int64_t*>(c->rec_elem.p),
            static_cast<const float*>(c->rec_w.p), c->nrec, Np, KNp);
        DG_HIP(c, hipGetLastError());
      }
      const double ti = t0 + double(i) * dt;
      // the residual scaling of the stage after (a_{q+1}; for q = 4 the a_0
      // = 0 of the next step's first stage) is applied in the kernel
      for (int q = 4; q >= 0; --q) {
        const int64_t sl = (i - n0) * 5 + q;
        if ((e = adj_stage_tiled(c, ys + q * n, rr + sl * n, jj ? jj + sl * jn : nullptr, lres,
                                 ly, nu, grad, gradz, float(kRkA[q == 4 ? 0 : q + 1]),
                                 float(kRkB[q]), dt, ti + kRkC[q] * dt)) != DG_OK)
          return e;
      }
    }
    return DG_OK;
  };
  if (!c->adj_ov) {
    for (int64_t sg = nck - 1; sg >= 0; --sg) {
      if ((s = replay(sg, 0)) != DG_OK) return s;
      if ((s = reverse(sg, 0)) != DG_OK) return s;
    }
    return DG_OK;
  }
  // overlapped: a second stream (default priority) for the replays; events
  // order each reverse sweep after its replay, and each replay after the
  // reverse sweep that last read its buffer.  The guard restores the
  // context's stream and waits for the replay stream on every exit.
  struct Side {
    dg_ctx* c;
    hipStream_t main, s2 = nullptr;
    hipEvent_t ev0 = nullptr, rep[2] = {nullptr, nullptr}, rev[2] = {nullptr, nullptr};
    ~Side() {
      c->stream = main;
      if (s2) {
        (void)hipStreamSynchronize(s2);
        (void)hipStreamDestroy(s2);
      }
      for (hipEvent_t e : {ev0, rep[0], rep[1], rev[0], rev[1]})
        if (e) (void)hipEventDestroy(e);
    }
  } side{c, st};
  DG_HIP(c, hipStreamCreateWithFlags(&side.s2, hipStreamNonBlocking));
  for (hipEvent_t* e : {&side.ev0, &side.rep[0], &side.rep[1], &side.rev[0], &side.rev[1]})
    DG_HIP(c, hipEventCreateWithFlags(e, hipEventDisableTiming));
  DG_HIP(c, hipEventRecord(side.ev0, st));   // the forward run and the fills above
  DG_HIP(c, hipStreamWaitEvent(side.s2, side.ev0, 0));
  c->stream = side.s2;
  if ((s = replay(nck - 1, 0)) != DG_OK) return s;
  DG_HIP(c, hipEventRecord(side.rep[0], side.s2));
  c->stream = st;
  for (int64_t sg = nck - 1; sg >= 0; --sg) {
    const int b = int((nck - 1 - sg) & 1);
    if (sg > 0) {
      // buffer 1 - b was last read by the reverse sweep of segment sg + 1
      if (sg + 1 <= nck - 1) DG_HIP(c, hipStreamWaitEvent(side.s2, side.rev[1 - b], 0));
      c->stream = side.s2;
      if ((s = replay(sg - 1, 1 - b)) != DG_OK) return s;
      DG_HIP(c, hipEventRecord(side.rep[1 - b], side.s2));
      c->stream = st;
    }
    DG_HIP(c, hipStreamWaitEvent(st, side.rep[b], 0));
    if ((s = reverse(sg, b)) != DG_OK) return s;
    DG_HIP(c, hipEventRecord(side.rev[b], st));
  }
  return DG_OK;
}

template <typename T>
dg_status adj_backward_t(dg_ctx* c, const T* resid) {
  if constexpr (std::is_same_v<T, float>)
    if (adj_tiled(c)) return adj_backward_tiled(c, resid);
  const int Np = c->re.Np, NF4 = 4 * c->re.Nfp, Nq = c->re.Nq;
  const int64_t K = c->mesh.K, n = int64_t(9) * K * Np, KNp = K * Np;
  const dga::AdjArgs<T> A = adj_args<T>(c);
  T* ck = static_cast<T*>(c->adj_ck.p);
  T* seg = static_cast<T*>(c->adj_seg.p);
  T* v = static_cast<T*>(c->adj_v.p);
  T *ly = v, *lres = v + n, *mu = v + 2 * n, *nu = v + 3 * n, *r = v + 4 * n, *res = v + 5 * n;
  T* gb = static_cast<T*>(c->adj_gb.p);
  T* hb = static_cast<T*>(c->adj_hb.p);
  double* grad = static_cast<double*>(c->adj_grad.p);
  // per-element kernels: one workgroup per element, the element's vectors in LDS
  if (K > 0x7fffffff) return fail(c, DG_EINVAL, "adjoint: too many elements for one grid");
  const dim3 eg(static_cast<unsigned>(K)), et(static_cast<unsigned>(dga::kAdjThreads));
  const size_t lraw = size_t(dga::raw_lds_elems(Np, c->re.Nfp)) * sizeof(T);
  const size_t lgw = size_t(dga::gradw_lds_elems(Np, Nq)) * sizeof(T);
  const size_t l9 = size_t(9) * Np * sizeof(T);
  const double t0 = c->adj_t0, dt = c->adj_dt;
  const int64_t nsteps = c->adj_nsteps, every = c->adj_every;
  const int64_t nck = (nsteps + every - 1) / every;
  const int ns = int(c->src.size());
  hipStream_t st = c->stream;
  dg_status s;
  if ((s = fill_zero(c, ly, n)) != DG_OK) return s;
  if ((s = fill_zero(c, lres, n)) != DG_OK) return s;
  dgk::fill_kernel<double><<<nblocks(3 * K * Nq), 256, 0, st>>>(grad, 3 * K * Nq, 0.0);
  DG_HIP(c, hipGetLastError());
  const bool upwind = c->opt.flux == DG_FLUX_UPWIND;
  T* zb = static_cast<T*>(c->adj_zb.p);
  double* gradz = static_cast<double*>(c->adj_gradz.p);
  if (upwind) {
    dgk::fill_kernel<double><<<nblocks(2 * KNp), 256, 0, st>>>(gradz, 2 * KNp, 0.0);
    DG_HIP(c, hipGetLastError());
  }
  for (int64_t sg = nck - 1; sg >= 0; --sg) {
    const int64_t n0 = sg * every, n1 = std::min(n0 + every, nsteps);
    // the stage inputs y_0 .. y_4 of every step of the segment, recomputed
    // from its checkpoint by the forward stages (so bit for bit those of the
    // forward run); step i's inputs at seg + (i - n0) 5 n
    DG_HIP(c, hipMemcpyAsync(seg, ck + sg * n, n * sizeof(T), hipMemcpyDeviceToDevice, st));
    for (int64_t i = n0; i < n1; ++i) {
      T* y = seg + (i - n0) * 5 * n;
      const double ti = t0 + double(i) * dt;
      if ((s = fill_zero(c, res, n)) != DG_OK) return s;
      for (int q = 0; q < 5 && (q < 4 || i + 1 < n1); ++q) {
        T* out = q < 4 ? y + (q + 1) * n : y + 5 * n;   // stage 5: the next step's y_0
        if ((s = stage(c, y + q * n, out, res, nullptr, kRkA[q], kRkB[q], dt, 1)) != DG_OK)
          return s;
        if ((s = launch_sources(c, res, out, ti + kRkC[q] * dt, dt, kRkB[q] * dt)) != DG_OK)
          return s;
      }
    }
    for (int64_t i = n1 - 1; i >= n0; --i) {
      const T* ys = seg + (i - n0) * 5 * n;
      // misfit sensitivity of the trace row of step i (state after step i)
      if (c->nrec > 0) {
        dga::receiver_adjoint<T><<<nblocks(3 * Np), 256, 0, st>>>(
            ly, resid + i * c->nrec * 3, static_cast<const int64_t*>(c->rec_elem.p),
            static_cast<const T*>(c->rec_w.p), c->nrec, Np, KNp);
        DG_HIP(c, hipGetLastError());
      }
      const double ti = t0 + double(i) * dt;
      for (int q = 4; q >= 0; --q) {
        const double ts = ti + kRkC[q] * dt;
        dga::axpby<T><<<nblocks(n), 256, 0, st>>>(lres, ly, kRkB[q], 1.0, n);
        // gradient: dt d/dm <lres, W(m) (R y_q + raw sources(ts))>
        dga::raw_rhs<T><<<eg, et, lraw, st>>>(A, ys + q * n, r);
        if (ns > 0) {
          dgs::source_add<T><<<nblocks(3 * Np), 256, 0, st>>>(
              r, static_cast<T*>(nullptr), static_cast<const int64_t*>(c->src_elem.p),
              static_cast<const T*>(c->src_wraw.p), static_cast<const double*>(c->src_par.p),
              ns, Np, KNp, ts, 1.0, 0.0);
        }
        // and mu = W^T lres (one kernel); then ly += dt R^T mu
        dga::grad_wadgT<T><<<eg, et, lgw, st>>>(A, lres, r, grad, dt, mu);
        dga::liftT_faces<T><<<eg, et, l9, st>>>(A, mu, gb);
        if (upwind) {
          // and the impedance gradient dt d/dZ <mu, R(Z) y_q>
          dga::zgrad_faces<T><<<nblocks(K * NF4), 256, 0, st>>>(A, ys + q * n, gb, zb);
          dga::zgrad_nodes<T><<<nblocks(KNp), 256, 0, st>>>(A, zb, gradz, dt);
        }
        dga::fluxT_faces<T><<<nblocks(K * NF4), 256, 0, st>>>(A, gb, hb);
        dga::volT_nodes<T><<<eg, et, l9, st>>>(A, mu, hb, nu);
        dga::axpby<T><<<nblocks(n), 256, 0, st>>>(ly, nu, dt, 1.0, n);
        dga::axpby<T><<<nblocks(n), 256, 0, st>>>(lres, lres, 0.0, kRkA[q], n);
        DG_HIP(c, hipGetLastError());
      }
    }
  }
  return DG_OK;
}

dg_status ready(dg_ctx* c, bool need_state) {
  if (!c) return DG_EINVAL;
  if (!device_ctx(c)) return fail(c, DG_EDEVICE, "host-only context: no device work");
  if (!c->has_mesh) return fail(c, DG_ESTATE, "no mesh uploaded");
  if (!c->has_mat) return fail(c, DG_ESTATE, "no material uploaded");
  if (need_state && !c->has_state) return fail(c, DG_ESTATE, "no state set");
  return set_device(c);
}

// No C++ exception crosses the C boundary: host allocation failures (the
// precompute's containers) become DG_ENOMEM, anything else DG_EINVAL.
dg_status exception_status() {
  try {
    throw;
  } catch (const std::bad_alloc&) {
    return DG_ENOMEM;
  } catch (const std::length_error&) {
    return DG_ENOMEM;
  } catch (...) {
    return DG_EINVAL;
  }
}

// ------------------------------------------------------------- batches ---
// One launch per stage over many contexts (dg_batch.hpp): the slot table is
// built on the host and written to device memory (the batch object's buffer,
// or the library's static scratch array) by launches that carry it as
// arguments, then each step runs five stage launches, five source launches
// and one receiver launch for the whole batch.

template <int N, bool F32>
hipError_t launch_batch_stage(const dgb::BatchSlot* table, int n, int64_t grid, hipStream_t st,
                              int par, double a, double b) {
  if constexpr (N <= 4)
    dgb::stage_bx_batch<N, F32><<<dim3(unsigned(grid)), dim3(dgb::kThreads), 0, st>>>(
        table, n, par, float(a), float(b));
  else
    dgb::stage_be_batch<N, F32><<<dim3(unsigned(grid)), dim3(dgb::kThreads), 0, st>>>(
        table, n, par, float(a), float(b));
  return hipGetLastError();
}

hipError_t batch_stage(int N, bool f32, const dgb::BatchSlot* table, int n, int64_t grid,
                       hipStream_t st, int par, double a, double b) {
  switch (N) {
#define DG_BATCH_CASE(NN)                                                                  \
  case NN:                                                                                 \
    return f32 ? launch_batch_stage<NN, true>(table, n, grid, st, par, a, b)              \
               : launch_batch_stage<NN, false>(table, n, grid, st, par, a, b);
    DG_BATCH_CASE(1)
    DG_BATCH_CASE(2)
    DG_BATCH_CASE(3)
    DG_BATCH_CASE(4)
    DG_BATCH_CASE(5)
    DG_BATCH_CASE(6)
    DG_BATCH_CASE(7)
#undef DG_BATCH_CASE
    default: return hipErrorInvalidValue;
  }
}

// the slot of context c (state buffers in the order of its current parity)
dgb::BatchSlot batch_slot_of(const dg_ctx* c, double dt, int64_t first) {
  dgb::BatchSlot S;
  std::memset(&S, 0, sizeof(S));
  const int Np = c->re.Np;
  float* q0 = static_cast<float*>(c->q[c->cur].p);
  float* q1 = static_cast<float*>(c->q[1 - c->cur].p);
  float* res = static_cast<float*>(c->res.p);
  if (c->re.N <= 4) {
    dgb::BxArgs& A = S.k.bx;
    A.q_in = q0;
    A.q_out = q1;
    A.res = res;
    A.rhs_out = nullptr;
    A.geo = static_cast<const float*>(c->geo.p);
    A.fgeo = static_cast<const float*>(c->fgeo.p);
    A.nbn = static_cast<const int32_t*>(c->nbn.p);
    A.torder = static_cast<const int32_t*>(c->torder.p);
    A.fmask = static_cast<const int32_t*>(c->fmask.p);
    A.mat = static_cast<const float*>(c->matblk.p);
    A.zp = static_cast<const float*>(c->zp.p);
    A.zs = static_cast<const float*>(c->zs.p);
    A.frags = static_cast<const dgb::u32x4*>(c->frags.p);
    A.K = c->mesh.K;
    A.dt = float(dt);
    A.lsrk = 1;
    A.upwind = c->opt.flux == DG_FLUX_UPWIND ? 1 : 0;
    S.nwg = (c->mesh.K + dgb::kTile - 1) / dgb::kTile;
  } else {
    dgb::BeArgs& A = S.k.be;
    A.q_in = q0;
    A.q_out = q1;
    A.res = res;
    A.rhs_out = nullptr;
    A.geo = static_cast<const float*>(c->geo.p);
    A.fgeo = static_cast<const float*>(c->fgeo.p);
    A.nbn = static_cast<const int32_t*>(c->nbn.p);
    A.fmask = static_cast<const int32_t*>(c->fmask.p);
    A.irho = static_cast<const float*>(c->irho.p);
    A.lam = static_cast<const float*>(c->lam.p);
    A.mu = static_cast<const float*>(c->mu.p);
    A.zp = static_cast<const float*>(c->zp.p);
    A.zs = static_cast<const float*>(c->zs.p);
    A.frags = static_cast<const dgb::u32x4*>(c->frags.p);
    A.K = c->mesh.K;
    A.dt = float(dt);
    A.lsrk = 1;
    A.upwind = c->opt.flux == DG_FLUX_UPWIND ? 1 : 0;
    S.nwg = c->mesh.K;
  }
  S.first = first;
  S.q[0] = q0;
  S.q[1] = q1;
  S.res = res;
  S.KNp = c->mesh.K * Np;
  S.Np = Np;
  S.nsrc = int(c->src.size());
  S.src_elem = static_cast<const int64_t*>(c->src_elem.p);
  S.src_w = static_cast<const float*>(c->src_w.p);
  S.src_par = static_cast<const double*>(c->src_par.p);
  S.nrec = c->nrec;
  S.rec_elem = static_cast<const int64_t*>(c->rec_elem.p);
  S.rec_w = static_cast<const float*>(c->rec_w.p);
  S.trace = static_cast<float*>(c->trace.p);
  S.trace_cap = c->trace_cap;
  S.clk = static_cast<double*>(c->clk.p);
  S.dt = dt;
  return S;
}

// Checks the batch, builds its slot table in the host array `slots` and
// writes it to the device array `table` (both with room for max_slots),
// then advances every context by nsteps steps on the stream.  Errors are
// reported on the first context.
dg_status batch_advance_impl(void* table, dgb::BatchSlot* slots, int max_slots, void* stream,
                             dg_ctx* const* cs, int n, const double* dt, int64_t nsteps) {
  if (!cs || n < 1 || !cs[0]) return DG_EINVAL;
  dg_ctx* c0 = cs[0];
  if (!dt) return fail(c0, DG_EINVAL, "batch: null time steps");
  if (n > max_slots)
    return fail(c0, DG_EINVAL, "batch: " + std::to_string(n) + " contexts, more than the " +
                                   std::to_string(max_slots) + " slots of the table");
  if (nsteps < 0) return fail(c0, DG_EINVAL, "batch: negative step count");
  for (int i = 0; i < n; ++i) {
    dg_ctx* c = cs[i];
    if (!c) return fail(c0, DG_EINVAL, "batch: null context");
    for (int j = 0; j < i; ++j)
      if (cs[j] == c) return fail(c0, DG_EINVAL, "batch: a context appears twice");
    if (c->opt.device != c0->opt.device || c->re.N != c0->re.N ||
        c->opt.precision != c0->opt.precision)
      return fail(c0, DG_EINVAL, "batch: contexts differ in device, order or precision");
    if (c->opt.precision != DG_FP32 && c->opt.precision != DG_FP32_BF16X3)
      return fail(c0, DG_EINVAL, "batch: FP32 and BF16x3 contexts only");
    if (!std::isfinite(dt[i])) return fail(c0, DG_EINVAL, "batch: non-finite time step");
    dg_status s = ready(c, true);
    if (s != DG_OK) return fail(c0, s, "batch: context " + std::to_string(i) + ": " + c->err);
  }
  dg_status s = set_device(c0);
  if (s != DG_OK) return s;
  hipStream_t st = stream ? static_cast<hipStream_t>(stream) : c0->stream;
  int64_t pos = 0;
  bool any_src = false, any_rec = false;
  int max_np3 = 0, max_rec3 = 0;
  for (int i = 0; i < n; ++i) {
    slots[i] = batch_slot_of(cs[i], dt[i], pos);
    pos += (slots[i].nwg + 7) / 8 * 8;
    any_src = any_src || slots[i].nsrc > 0;
    any_rec = any_rec || (slots[i].nrec > 0 && slots[i].trace_cap > 0);
    max_np3 = std::max(max_np3, 3 * slots[i].Np);
    max_rec3 = std::max(max_rec3, 3 * slots[i].nrec);
  }
  if (pos > 0x7fffffff) return fail(c0, DG_EINVAL, "batch: too many workgroups for one grid");
  // the slot table, written by launches that carry it
  const size_t words = size_t(n) * sizeof(dgb::BatchSlot) / 4;
  static_assert(sizeof(dgb::BatchSlot) % 4 == 0, "whole words");
  const uint32_t* src = reinterpret_cast<const uint32_t*>(slots);
  uint32_t* dst = static_cast<uint32_t*>(table);
  for (size_t w0 = 0; w0 < words; w0 += dgb::kSlotWords) {
    dgb::SlotChunk ch;
    const int nw = int(std::min<size_t>(dgb::kSlotWords, words - w0));
    std::memcpy(ch.w, src + w0, size_t(nw) * 4);
    dgb::slot_write<<<1, 256, 0, st>>>(dst + w0, ch, nw);
    DG_HIP(c0, hipGetLastError());
  }
  const dgb::BatchSlot* tab = static_cast<const dgb::BatchSlot*>(table);
  const bool f32 = c0->opt.precision == DG_FP32;
  const dim3 gsrc(unsigned((max_np3 + 255) / 256), unsigned(n));
  const dim3 grec(unsigned((max_rec3 + 255) / 256), unsigned(n));
  for (int64_t i = 0; i < nsteps; ++i) {
    for (int stg = 0; stg < 5; ++stg) {
      const int par = int((5 * i + stg) & 1);
      const hipError_t e = batch_stage(c0->re.N, f32, tab, n, pos, st, par, kRkA[stg], kRkB[stg]);
      if (e != hipSuccess)
        return fail(c0, DG_EDEVICE, std::string("batch stage launch: ") + hipGetErrorString(e));
      if (any_src) {
        dgb::source_add_batch<<<gsrc, 256, 0, st>>>(tab, par, double(i) + kRkC[stg], kRkB[stg]);
        DG_HIP(c0, hipGetLastError());
      }
    }
    if (any_rec && max_rec3 > 0) {
      dgb::receiver_sample_batch<<<grec, 256, 0, st>>>(tab, int((5 * (i + 1)) & 1), i);
      DG_HIP(c0, hipGetLastError());
    }
  }
  if (nsteps > 0) {
    dgb::clock_advance_batch<<<unsigned((n + 63) / 64), 64, 0, st>>>(tab, n, nsteps);
    DG_HIP(c0, hipGetLastError());
  }
  // five stages per step: the current buffer flips once per odd step count
  if (nsteps & 1)
    for (int i = 0; i < n; ++i) cs[i]->cur = 1 - cs[i]->cur;
  return DG_OK;
}

// The allocation-free variant's slot table: a static device array, one copy
// per GPU, whose address each device resolves once (hipGetSymbolAddress) the
// first time the entry point runs on it; host code uses only that address.
constexpr int kBatchStaticSlots = 64;
static __device__ __align__(256) unsigned char scratch[kBatchStaticSlots * sizeof(dgb::BatchSlot)];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// ====================================================================== ABI
extern "C" {

dg_status dg_create(dg_ctx** out, const dg_options* opt) {
  dg_ctx* c = nullptr;   // freed here if an exception escapes the set-up
  try {
    if (!out) return DG_EINVAL;
    *out = nullptr;
    if (!opt) return DG_EINVAL;
    if (opt->order < 1 || opt->order > 7) return DG_EINVAL;
    if (opt->precision != DG_FP64 && opt->precision != DG_FP32 &&
        opt->precision != DG_FP32_BF16X3)
      return DG_EINVAL;
    if (opt->flux != DG_FLUX_UPWIND && opt->flux != DG_FLUX_CENTRAL) return DG_EINVAL;
    if (opt->precision == DG_FP32_BF16X3 && !dgh::mfma_supported(opt->order)) return DG_EINVAL;
    c = new (std::nothrow) dg_ctx();
    if (!c) return DG_ENOMEM;
    c->opt = *opt;
    c->elem = (opt->precision == DG_FP64) ? 8 : 4;
    c->stream = static_cast<hipStream_t>(opt->stream);
    std::string err;
    if (!dgh::build_ref_element(opt->order, c->re, err)) {
      delete c;
      return DG_EINVAL;
    }
    if (device_ctx(c)) {
      int ndev = 0;
      if (hipGetDeviceCount(&ndev) != hipSuccess || opt->device >= ndev) {
        delete c;
        return DG_EDEVICE;
      }
      if (hipSetDevice(opt->device) != hipSuccess) {
        delete c;
        return DG_EDEVICE;
      }
      // reference operators and face masks, cast to the working precision
      std::vector<double> ops;
      const dgh::RefElement& re = c->re;
      for (const auto* v : {&re.Dr, &re.Ds, &re.Dt, &re.LIFT, &re.Vq, &re.Pq})
        ops.insert(ops.end(), v->begin(), v->end());
      // transposed, padded operators (generic FP64 kernel, adjoint)
      const std::vector<double> opsT = dgh::col_operators(re);
      if (upload_real(c, c->opsT, opsT.data(), opsT.size()) != DG_OK ||
          upload_real(c, c->ops, ops.data(), ops.size()) != DG_OK ||
          upload_raw(c, c->fmask, re.Fmask.data(), re.Fmask.size()) != DG_OK) {
        dg_destroy(c);
        return DG_ENOMEM;
      }
      if (opt->precision == DG_FP32_BF16X3) {
        const std::vector<uint16_t> fr = dgh::mfma_fragments(re);
        if (upload_raw(c, c->frags, fr.data(), fr.size()) != DG_OK) {
          dg_destroy(c);
          return DG_ENOMEM;
        }
      } else if (opt->precision == DG_FP32) {
        const std::vector<float> fr = dgh::mfma_fragments_f32(re);
        if (upload_raw(c, c->frags, fr.data(), fr.size()) != DG_OK) {
          dg_destroy(c);
          return DG_ENOMEM;
        }
      } else {   // FP64 on the matrix cores
        const std::vector<double> fr = dgh::mfma_fragments_f64(re);
        if (upload_raw(c, c->frags, fr.data(), fr.size()) != DG_OK) {
          dg_destroy(c);
          return DG_ENOMEM;
        }
      }
    }
    *out = c;
    return DG_OK;
  } catch (...) {
    const dg_status st = exception_status();
    if (c) dg_destroy(c);
    if (out) *out = nullptr;
    return st;
  }
}

void dg_destroy(dg_ctx* c) {
  if (!c) return;
  if (device_ctx(c) && hipSetDevice(c->opt.device) == hipSuccess) {
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    release(c, c->clk);
    release(c, c->trace);
    for (DevBuf* b : {&c->ops, &c->opsT, &c->fmask, &c->geo, &c->fgeo, &c->etoe, &c->etop, &c->pat,
                      &c->irho, &c->lam, &c->mu, &c->zp, &c->zs, &c->q[0], &c->q[1],
                      &c->res, &c->frags, &c->matblk, &c->nbn, &c->torder, &c->src_elem, &c->src_w,
                      &c->src_par, &c->rec_elem, &c->rec_w, &c->rec_buf, &c->src_wraw,
                      &c->adj_nbface, &c->adj_invf, &c->adj_ck, &c->adj_seg, &c->adj_r,
                      &c->adj_j, &c->adj_v, &c->adj_gb, &c->adj_hb, &c->adj_grad, &c->adj_zb,
                      &c->adj_gradz, &c->adj_frag, &c->adj_trace})
      release(c, *b);
  }
  delete c;
}

const char* dg_last_error(const dg_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

dg_status dg_sizes(const dg_ctx* c, int64_t* K, int32_t* Np, int32_t* Nfp, int32_t* Nq) {
  try {
    if (!c) return DG_EINVAL;
    if (K) *K = c->has_mesh ? c->mesh.K : 0;
    if (Np) *Np = c->re.Np;
    if (Nfp) *Nfp = c->re.Nfp;
    if (Nq) *Nq = c->re.Nq;
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_mesh_upload(dg_ctx* c, int64_t K, const double* vxyz, const double* period) {
  try {
    if (!c) return DG_EINVAL;
    if (!vxyz || !period || K <= 0) return fail(c, DG_EINVAL, "mesh: bad arguments");
    for (int64_t i = 0; i < K * 12; ++i)
      if (!std::isfinite(vxyz[i])) return fail(c, DG_ENONFINITE, "mesh: non-finite vertex");
    std::string err;
    dgh::MeshData m;
    if (!dgh::build_mesh(c->re, K, vxyz, period, m, err)) return fail(c, DG_EINVAL, err);
    c->mesh = std::move(m);
    c->has_mesh = true;
    c->has_mat = false;
    c->has_state = false;
    c->src.clear();           // sources and receivers belong to the old mesh
    c->nrec = 0;
    if (!device_ctx(c)) return DG_OK;
    dg_status s = set_device(c);
    if (s != DG_OK) return s;
    drop_graphs(c);
    for (DevBuf* b : {&c->src_elem, &c->src_w, &c->src_par, &c->rec_elem, &c->rec_w, &c->rec_buf,
                      &c->trace, &c->src_wraw, &c->adj_nbface, &c->adj_invf, &c->adj_ck,
                      &c->adj_seg, &c->adj_r, &c->adj_j, &c->adj_v, &c->adj_gb, &c->adj_hb,
                      &c->adj_grad, &c->adj_zb, &c->adj_gradz, &c->adj_frag, &c->adj_trace})
      release(c, *b);
    c->adj_ready = false;
    c->adj_ov_failed = c->adj_j_failed = 0;
    c->trace_cap = 0;
    if (!c->clk.p) {
      if ((s = alloc(c, c->clk, 2 * sizeof(double))) != DG_OK) return s;
    }
    dgs::clock_set<<<1, 64, 0, c->stream>>>(static_cast<double*>(c->clk.p), 0.0);
    DG_HIP(c, hipGetLastError());
    const dgh::MeshData& md = c->mesh;
    if ((s = upload_real(c, c->geo, md.geo.data(), md.geo.size())) != DG_OK) return s;
    if ((s = upload_real(c, c->fgeo, md.fgeo.data(), md.fgeo.size())) != DG_OK) return s;
    if ((s = upload_raw(c, c->etoe, md.EToE.data(), md.EToE.size())) != DG_OK) return s;
    if ((s = upload_raw(c, c->etop, md.EToP.data(), md.EToP.size())) != DG_OK) return s;
    if ((s = upload_raw(c, c->pat, md.pat.data(), md.pat.size())) != DG_OK) return s;
    {   // every stage kernel gathers through the neighbour-node table
      if (K * c->re.Np >= (int64_t(1) << 31)) return fail(c, DG_EINVAL, "mesh: K Np too large");
      const std::vector<int32_t> nbn = dgh::neighbour_nodes(c->re, md);
      if ((s = upload_raw(c, c->nbn, nbn.data(), nbn.size())) != DG_OK) return s;
      if (tiled_kernel(c->opt.precision, c->re.N)) {
        const std::vector<int32_t> tord = dgh::tile_order(md, dgb::kTile, 8);
        if ((s = upload_raw(c, c->torder, tord.data(), tord.size())) != DG_OK) return s;
      }
    }
    const size_t nstate = size_t(9) * K * c->re.Np * c->elem;
    for (DevBuf* b : {&c->q[0], &c->q[1], &c->res})
      if ((s = alloc(c, *b, nstate)) != DG_OK) return s;
    c->cur = 0;
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_node_coords(const dg_ctx* c, double* xyz) {
  try {
    if (!c || !xyz) return DG_EINVAL;
    if (!c->has_mesh) return DG_ESTATE;
    dgh::node_coords(c->re, c->mesh, xyz);
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_quad_coords(const dg_ctx* c, double* xyz) {
  try {
    if (!c || !xyz) return DG_EINVAL;
    if (!c->has_mesh) return DG_ESTATE;
    dgh::quad_coords(c->re, c->mesh, xyz);
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_material_upload(dg_ctx* c, const double* rho_q, const double* cp_q,
                             const double* cs_q, const double* rho_n, const double* cp_n,
                             const double* cs_n) {
  try {
    if (!c) return DG_EINVAL;
    if (!c->has_mesh) return fail(c, DG_ESTATE, "material: no mesh uploaded");
    if (!rho_q || !cp_q || !cs_q || !rho_n || !cp_n || !cs_n)
      return fail(c, DG_EINVAL, "material: null array");
    const int64_t K = c->mesh.K;
    const size_t nq = size_t(K) * c->re.Nq, nn = size_t(K) * c->re.Np;
    auto check = [&](const double* r, const double* p, const double* s, size_t n) -> dg_status {
      for (size_t i = 0; i < n; ++i) {
        if (!std::isfinite(r[i]) || !std::isfinite(p[i]) || !std::isfinite(s[i]))
          return fail(c, DG_ENONFINITE, "material: non-finite sample");
        if (!(r[i] > 0.0) || !(s[i] > 0.0) || p[i] * p[i] < 2.0 * s[i] * s[i])
          return fail(c, DG_EINVAL, "material: need rho > 0, cs > 0, cp >= sqrt(2) cs");
      }
      return DG_OK;
    };
    dg_status s = check(rho_q, cp_q, cs_q, nq);
    if (s != DG_OK) return s;
    if ((s = check(rho_n, cp_n, cs_n, nn)) != DG_OK) return s;
    c->has_mat = false;
    c->adj_ready = false;
    if (!device_ctx(c)) {
      c->has_mat = true;
      return DG_OK;
    }
    if ((s = set_device(c)) != DG_OK) return s;
    std::vector<double> a(nq), b(nq), d(nq);
    for (size_t i = 0; i < nq; ++i) {
      const double r = rho_q[i], p = cp_q[i], v = cs_q[i];
      a[i] = 1.0 / r;
      b[i] = r * (p * p - 2.0 * v * v);
      d[i] = r * v * v;
    }
    if (tiled_kernel(c->opt.precision, c->re.N)) {
      const std::vector<double> blk =
          dgh::mfma_material(c->re.N, K, a.data(), b.data(), d.data(), c->opt.precision == DG_FP64);
      if ((s = upload_real(c, c->matblk, blk.data(), blk.size())) != DG_OK) return s;
    }
    if (plain_material(c->opt.precision, c->re.N)) {
      if ((s = upload_real(c, c->irho, a.data(), nq)) != DG_OK) return s;
      if ((s = upload_real(c, c->lam, b.data(), nq)) != DG_OK) return s;
      if ((s = upload_real(c, c->mu, d.data(), nq)) != DG_OK) return s;
    }
    std::vector<double> zp(nn), zs(nn);
    for (size_t i = 0; i < nn; ++i) {
      zp[i] = rho_n[i] * cp_n[i];
      zs[i] = rho_n[i] * cs_n[i];
    }
    if ((s = upload_real(c, c->zp, zp.data(), nn)) != DG_OK) return s;
    if ((s = upload_real(c, c->zs, zs.data(), nn)) != DG_OK) return s;
    c->has_mat = true;
    drop_graphs(c);
    if (!c->src.empty()) return upload_sources(c);   // source responses depend on 1/rho
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_project(const dg_ctx* c, int32_t nfields, const double* fq, double* q) {
  try {
    if (!c || !fq || !q || nfields < 1) return DG_EINVAL;
    if (!c->has_mesh) return DG_ESTATE;
    const int Np = c->re.Np, Nq = c->re.Nq;
    const int64_t K = c->mesh.K;
    for (int64_t fk = 0; fk < int64_t(nfields) * K; ++fk) {
      const double* src = fq + fk * Nq;
      double* dst = q + fk * Np;
      for (int n = 0; n < Np; ++n) {
        double acc = 0.0;
        const double* P = &c->re.Pq[size_t(n) * Nq];
        for (int j = 0; j < Nq; ++j) acc += P[j] * src[j];
        dst[n] = acc;
      }
    }
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_state_set(dg_ctx* c, const void* q, int32_t on_device) {
  try {
    if (!c || !q) return DG_EINVAL;
    dg_status s = ready(c, false);
    if (s != DG_OK) return s;
    const size_t n = size_t(9) * c->mesh.K * c->re.Np;
    if (on_device)
      DG_HIP(c, hipMemcpyAsync(c->q[c->cur].p, q, n * c->elem, hipMemcpyDeviceToDevice,
                               c->stream));
    else {
      DG_HIP(c, copy_sync(c, c->q[c->cur].p, q, n * c->elem, hipMemcpyHostToDevice));
    }
    if ((s = fill_zero(c, c->res.p, int64_t(n))) != DG_OK) return s;
    c->has_state = true;
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_state_zero(dg_ctx* c) {
  try {
    if (!c) return DG_EINVAL;
    dg_status s = ready(c, false);
    if (s != DG_OK) return s;
    const int64_t n = int64_t(9) * c->mesh.K * c->re.Np;
    if ((s = fill_zero(c, c->q[c->cur].p, n)) != DG_OK) return s;
    if ((s = fill_zero(c, c->res.p, n)) != DG_OK) return s;
    c->has_state = true;
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_state_get(dg_ctx* c, void* q, int32_t on_device) {
  try {
    if (!c || !q) return DG_EINVAL;
    dg_status s = ready(c, true);
    if (s != DG_OK) return s;
    const size_t n = size_t(9) * c->mesh.K * c->re.Np * c->elem;
    if (on_device)
      DG_HIP(c, hipMemcpyAsync(q, c->q[c->cur].p, n, hipMemcpyDeviceToDevice, c->stream));
    else {
      DG_HIP(c, hipMemcpyAsync(q, c->q[c->cur].p, n, hipMemcpyDeviceToHost, c->stream));
      DG_HIP(c, hipStreamSynchronize(c->stream));
    }
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_state_device_ptr(dg_ctx* c, void** ptr) {
  try {
    if (!c || !ptr) return DG_EINVAL;
    dg_status s = ready(c, false);
    if (s != DG_OK) return s;
    *ptr = c->q[c->cur].p;
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_rhs(dg_ctx* c, const void* q_dev, void* rhs_dev, double t) {
  try {
    if (!c || !q_dev || !rhs_dev) return DG_EINVAL;
    if (q_dev == rhs_dev) return fail(c, DG_EINVAL, "rhs: q and rhs must not alias");
    if (!std::isfinite(t)) return fail(c, DG_EINVAL, "rhs: non-finite t");
    dg_status s = ready(c, false);
    if (s != DG_OK) return s;
    if ((s = stage(c, q_dev, nullptr, nullptr, rhs_dev, 0.0, 0.0, 0.0, 0)) != DG_OK) return s;
    return launch_sources(c, rhs_dev, nullptr, t, 1.0, 0.0);
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_step(dg_ctx* c, double t, double dt) {
  try {
    if (!c) return DG_EINVAL;
    if (!std::isfinite(t) || !std::isfinite(dt)) return fail(c, DG_EINVAL, "step: non-finite t/dt");
    dg_status s = ready(c, true);
    if (s != DG_OK) return s;
    for (int st = 0; st < 5; ++st) {
      s = stage(c, c->q[c->cur].p, c->q[1 - c->cur].p, c->res.p, nullptr, kRkA[st], kRkB[st],
                dt, 1);
      if (s != DG_OK) return s;
      s = launch_sources(c, c->res.p, c->q[1 - c->cur].p, t + kRkC[st] * dt, dt, kRkB[st] * dt);
      if (s != DG_OK) return s;
      c->cur = 1 - c->cur;
    }
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_run(dg_ctx* c, double t0, double dt, int64_t nsteps) {
  try {
    if (!c) return DG_EINVAL;
    if (nsteps < 0) return fail(c, DG_EINVAL, "run: negative step count");
    for (int64_t i = 0; i < nsteps; ++i) {
      dg_status s = dg_step(c, t0 + double(i) * dt, dt);
      if (s != DG_OK) return s;
    }
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_sources_set(dg_ctx* c, int32_t nsrc, const double* xyz, const double* dir,
                         const double* f0, const double* t0, const double* amp) {
  try {
    if (!c) return DG_EINVAL;
    if (nsrc < 0 || (nsrc > 0 && (!xyz || !dir || !f0 || !t0 || !amp)))
      return fail(c, DG_EINVAL, "sources: bad arguments");
    if (!device_ctx(c)) return fail(c, DG_EDEVICE, "host-only context: no device work");
    if (!c->has_mesh) return fail(c, DG_ESTATE, "sources: no mesh uploaded");
    if (!c->has_mat) return fail(c, DG_ESTATE, "sources: no material uploaded");
    std::vector<dg_ctx::Source> src(nsrc);
    for (int i = 0; i < nsrc; ++i) {
      for (int d = 0; d < 3; ++d) {
        src[i].x[d] = xyz[3 * i + d];
        src[i].d[d] = dir[3 * i + d];
        if (!std::isfinite(src[i].x[d]) || !std::isfinite(src[i].d[d]))
          return fail(c, DG_ENONFINITE, "sources: non-finite position or direction");
      }
      src[i].f0 = f0[i];
      src[i].t0 = t0[i];
      src[i].amp = amp[i];
      if (!std::isfinite(f0[i]) || !std::isfinite(t0[i]) || !std::isfinite(amp[i]))
        return fail(c, DG_ENONFINITE, "sources: non-finite wavelet parameter");
      if (!(f0[i] > 0.0)) return fail(c, DG_EINVAL, "sources: need f0 > 0");
      int64_t k;
      double rst[3];
      if (!dgh::locate_point(c->re, c->mesh, src[i].x, k, rst))
        return fail(c, DG_EINVAL, "sources: point outside the mesh");
    }
    dg_status s = set_device(c);
    if (s != DG_OK) return s;
    DG_HIP(c, hipStreamSynchronize(c->stream));   // the old arrays may be in use
    drop_graphs(c);
    c->adj_ready = false;
    c->src = std::move(src);
    return upload_sources(c);
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_receivers_set(dg_ctx* c, int32_t nrec, const double* xyz) {
  try {
    if (!c) return DG_EINVAL;
    if (nrec < 0 || (nrec > 0 && !xyz)) return fail(c, DG_EINVAL, "receivers: bad arguments");
    if (!device_ctx(c)) return fail(c, DG_EDEVICE, "host-only context: no device work");
    if (!c->has_mesh) return fail(c, DG_ESTATE, "receivers: no mesh uploaded");
    const int Np = c->re.Np;
    std::vector<int64_t> elem(nrec);
    std::vector<double> w(size_t(nrec) * Np), psi(Np);
    for (int r = 0; r < nrec; ++r) {
      for (int d = 0; d < 3; ++d)
        if (!std::isfinite(xyz[3 * r + d]))
          return fail(c, DG_ENONFINITE, "receivers: non-finite position");
      double rst[3];
      if (!dgh::locate_point(c->re, c->mesh, xyz + 3 * r, elem[r], rst))
        return fail(c, DG_EINVAL, "receivers: point outside the mesh");
      // Lagrange basis at the point: l = V^-T psi, i.e. solve V^T l = psi
      dgh::basis_at(c->re, rst[0], rst[1], rst[2], psi.data());
      std::vector<double> VT(size_t(Np) * Np), l(Np);
      for (int i = 0; i < Np; ++i)
        for (int j = 0; j < Np; ++j) VT[size_t(i) * Np + j] = c->re.V[size_t(j) * Np + i];
      // Gaussian elimination with partial pivoting
      std::vector<double> b(psi);
      for (int col = 0; col < Np; ++col) {
        int piv = col;
        for (int i = col + 1; i < Np; ++i)
          if (std::fabs(VT[size_t(i) * Np + col]) > std::fabs(VT[size_t(piv) * Np + col])) piv = i;
        if (piv != col) {
          for (int j = 0; j < Np; ++j) std::swap(VT[size_t(col) * Np + j], VT[size_t(piv) * Np + j]);
          std::swap(b[col], b[piv]);
        }
        for (int i = col + 1; i < Np; ++i) {
          const double f = VT[size_t(i) * Np + col] / VT[size_t(col) * Np + col];
          for (int j = col; j < Np; ++j) VT[size_t(i) * Np + j] -= f * VT[size_t(col) * Np + j];
          b[i] -= f * b[col];
        }
      }
      for (int i = Np - 1; i >= 0; --i) {
        double acc = b[i];
        for (int j = i + 1; j < Np; ++j) acc -= VT[size_t(i) * Np + j] * l[j];
        l[i] = acc / VT[size_t(i) * Np + i];
      }
      for (int n = 0; n < Np; ++n) w[size_t(r) * Np + n] = l[n];
    }
    dg_status s = set_device(c);
    if (s != DG_OK) return s;
    DG_HIP(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    c->adj_ready = false;
    c->nrec = 0;
    c->trace_cap = 0;
    for (DevBuf* b : {&c->rec_elem, &c->rec_w, &c->rec_buf, &c->trace}) release(c, *b);
    if (nrec == 0) return DG_OK;
    if ((s = upload_raw(c, c->rec_elem, elem.data(), elem.size())) != DG_OK) return s;
    if ((s = upload_real(c, c->rec_w, w.data(), w.size())) != DG_OK) return s;
    c->nrec = nrec;
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_receivers_sample(dg_ctx* c, void* out, int32_t on_device) {
  try {
    if (!c || !out) return DG_EINVAL;
    dg_status s = ready(c, true);
    if (s != DG_OK) return s;
    if (c->nrec == 0) return fail(c, DG_ESTATE, "receivers: none set");
    const size_t bytes = size_t(c->nrec) * 3 * c->elem;
    if (on_device) return launch_receivers(c, out);
    if (c->rec_buf.bytes < bytes && (s = alloc(c, c->rec_buf, bytes)) != DG_OK) return s;
    if ((s = launch_receivers(c, c->rec_buf.p)) != DG_OK) return s;
    DG_HIP(c, hipMemcpyAsync(out, c->rec_buf.p, bytes, hipMemcpyDeviceToHost, c->stream));
    DG_HIP(c, hipStreamSynchronize(c->stream));
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_run_record(dg_ctx* c, double t0, double dt, int64_t nsteps, void* trace,
                        int32_t on_device) {
  try {
    if (!c || !trace) return DG_EINVAL;
    if (nsteps < 0) return fail(c, DG_EINVAL, "run: negative step count");
    dg_status s = ready(c, true);
    if (s != DG_OK) return s;
    if (c->nrec == 0) return fail(c, DG_ESTATE, "receivers: none set");
    const size_t per = size_t(c->nrec) * 3 * c->elem;
    char* dst = static_cast<char*>(trace);
    if (!on_device) {
      const size_t bytes = per * size_t(nsteps);
      if (c->rec_buf.bytes < bytes && (s = alloc(c, c->rec_buf, bytes)) != DG_OK) return s;
      dst = static_cast<char*>(c->rec_buf.p);
    }
    for (int64_t i = 0; i < nsteps; ++i) {
      if ((s = dg_step(c, t0 + double(i) * dt, dt)) != DG_OK) return s;
      if ((s = launch_receivers(c, dst + per * size_t(i))) != DG_OK) return s;
    }
    if (!on_device && nsteps > 0) {
      DG_HIP(c, hipMemcpyAsync(trace, c->rec_buf.p, per * size_t(nsteps), hipMemcpyDeviceToHost,
                               c->stream));
      DG_HIP(c, hipStreamSynchronize(c->stream));
    }
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_time_set(dg_ctx* c, double t) {
  try {
    if (!c) return DG_EINVAL;
    if (!std::isfinite(t)) return fail(c, DG_EINVAL, "time: non-finite");
    dg_status s = ready(c, false);
    if (s != DG_OK) return s;
    dgs::clock_set<<<1, 64, 0, c->stream>>>(static_cast<double*>(c->clk.p), t);
    DG_HIP(c, hipGetLastError());
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_time_get(dg_ctx* c, double* t, int64_t* step) {
  try {
    if (!c) return DG_EINVAL;
    dg_status s = ready(c, false);
    if (s != DG_OK) return s;
    double h[2];
    DG_HIP(c, hipMemcpyAsync(h, c->clk.p, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    DG_HIP(c, hipStreamSynchronize(c->stream));
    if (t) *t = h[0];
    if (step) *step = int64_t(h[1]);
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_trace_reserve(dg_ctx* c, int64_t max_steps) {
  try {
    if (!c) return DG_EINVAL;
    if (max_steps < 0) return fail(c, DG_EINVAL, "trace: negative capacity");
    if (!device_ctx(c)) return fail(c, DG_EDEVICE, "host-only context: no device work");
    if (c->nrec == 0) return fail(c, DG_ESTATE, "trace: no receivers set");
    dg_status s = set_device(c);
    if (s != DG_OK) return s;
    DG_HIP(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    c->trace_cap = 0;
    if ((s = alloc(c, c->trace, size_t(max_steps) * c->nrec * 3 * c->elem)) != DG_OK) return s;
    c->trace_cap = max_steps;
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_trace_copy(dg_ctx* c, void* out, int64_t nrows) {
  try {
    if (!c || !out) return DG_EINVAL;
    if (nrows < 0 || nrows > c->trace_cap) return fail(c, DG_EINVAL, "trace: rows out of range");
    dg_status s = set_device(c);
    if (s != DG_OK) return s;
    const size_t bytes = size_t(nrows) * c->nrec * 3 * c->elem;
    if (bytes) DG_HIP(c, hipMemcpyAsync(out, c->trace.p, bytes, hipMemcpyDeviceToHost, c->stream));
    DG_HIP(c, hipStreamSynchronize(c->stream));
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_advance(dg_ctx* c, double dt, int64_t nsteps) {
  try {
    if (!c) return DG_EINVAL;
    if (!std::isfinite(dt) || nsteps < 0) return fail(c, DG_EINVAL, "advance: bad dt or steps");
    dg_status s = ready(c, true);
    if (s != DG_OK) return s;
    return advance_impl(c, dt, nsteps);
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_graph_advance(dg_ctx* c, double dt, int64_t nsteps) {
  try {
    if (!c) return DG_EINVAL;
    if (!std::isfinite(dt) || nsteps < 1) return fail(c, DG_EINVAL, "graph: bad dt or steps");
    dg_status s = ready(c, true);
    if (s != DG_OK) return s;
    if (!c->stream) return fail(c, DG_ESTATE, "graph: the context needs its own stream");
    const int cur0 = c->cur;
    const int cur1 = int((cur0 + 5 * nsteps) & 1);
    const dg_ctx::Graph* g = nullptr;
    for (const auto& x : c->graphs)
      if (x.dt == dt && x.nsteps == nsteps && x.cur == cur0) g = &x;
    if (!g) {
      hipGraph_t graph = nullptr;
      // relaxed: other threads (other requests' set-up) keep calling HIP
      DG_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
      s = advance_impl(c, dt, nsteps);
      const hipError_t ec = hipStreamEndCapture(c->stream, &graph);
      c->cur = cur0;   // capture recorded the launches without running them
      if (s != DG_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
      }
      if (ec != hipSuccess)
        return fail(c, DG_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
      hipGraphExec_t exec = nullptr;
      const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess)
        return fail(c, DG_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
      c->graphs.push_back({dt, nsteps, cur0, exec});
      g = &c->graphs.back();
    }
    DG_HIP(c, hipGraphLaunch(g->exec, c->stream));
    c->cur = cur1;
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_memory(const dg_ctx* c, uint64_t* bytes) {
  try {
    if (!c || !bytes) return DG_EINVAL;
    *bytes = c->allocated;
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_footprint(int32_t order, int32_t precision, int64_t K, int32_t nsrc, int32_t nrec,
                       int64_t trace_steps, uint64_t* bytes) {
  try {
    if (!bytes || order < 1 || order > 7 || K < 1 || nsrc < 0 || nrec < 0 || trace_steps < 0)
      return DG_EINVAL;
    if (precision != DG_FP64 && precision != DG_FP32 && precision != DG_FP32_BF16X3)
      return DG_EINVAL;
    if (precision == DG_FP32_BF16X3 && !dgh::mfma_supported(order)) return DG_EINVAL;
    const uint64_t N = uint64_t(order), Np = (N + 1) * (N + 2) * (N + 3) / 6;
    const uint64_t Nfp = (N + 1) * (N + 2) / 2, Nq = (N + 1) * (N + 1) * (N + 1), NF4 = 4 * Nfp;
    const uint64_t NpP = 4 * ((Np + 3) / 4), QP = 32 * ((Nq + 31) / 32);
    const uint64_t e = precision == DG_FP64 ? 8 : 4, k = uint64_t(K);
    uint64_t b = 0;
    b += (3 * Np * Np + Np * NF4 + Nq * Np + Np * Nq) * e;              // operators
    b += (3 * Np * NpP + NF4 * NpP + Np * QP + QP * NpP) * e;           // transposed operators
    b += NF4 * 4;                                                       // face masks
    if (precision == DG_FP32_BF16X3) b += uint64_t(dgh::mfma_frag_count(order)) * 64 * 8 * 2;
    else if (precision == DG_FP32) b += uint64_t(dgh::mfma_f32_frag_count(order)) * 16;
    else b += uint64_t(dgh::mfma_f32_frag_count(order)) * 32;   // FP64 fragments
    b += k * (9 + 16) * e + k * 4 * 4 + k * 4 + 96 * Nfp * 4;          // geometry, tables
    b += 3 * 9 * k * Np * e + 2 * sizeof(double);                      // q[2], res, clock
    b += k * NF4 * 4;                                                   // neighbour nodes
    if (tiled_kernel(precision, order)) {
      b += ((k + 15) / 16) * 3 * uint64_t(dgh::mfma_mats(order)) * e;   // blocked material
      b += (k + 15) / 16 * 4;                                           // tile order
    }
    if (plain_material(precision, order)) b += 3 * k * Nq * e;          // 1/rho, lam, mu
    b += 2 * k * Np * e;                                                // impedances
    b += uint64_t(nsrc) * (8 + 3 * Np * e + 3 * 8);                     // sources
    b += uint64_t(nrec) * (8 + Np * e) + uint64_t(trace_steps) * nrec * 3 * e;   // receivers
    *bytes = b;
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_material_set_weights(dg_ctx* c, const double* irho_q, const double* lam_q,
                                  const double* mu_q, const double* zp_n, const double* zs_n) {
  try {
    if (!c) return DG_EINVAL;
    if (!c->has_mesh) return fail(c, DG_ESTATE, "weights: no mesh uploaded");
    if (!irho_q || !lam_q || !mu_q || !zp_n || !zs_n) return fail(c, DG_EINVAL, "weights: null");
    const int64_t K = c->mesh.K;
    const size_t nq = size_t(K) * c->re.Nq, nn = size_t(K) * c->re.Np;
    for (size_t i = 0; i < nq; ++i)
      if (!std::isfinite(irho_q[i]) || !std::isfinite(lam_q[i]) || !std::isfinite(mu_q[i]))
        return fail(c, DG_ENONFINITE, "weights: non-finite value");
    for (size_t i = 0; i < nn; ++i) {
      if (!std::isfinite(zp_n[i]) || !std::isfinite(zs_n[i]))
        return fail(c, DG_ENONFINITE, "weights: non-finite impedance");
      if (!(zp_n[i] > 0.0) || !(zs_n[i] > 0.0))
        return fail(c, DG_EINVAL, "weights: impedances must be positive");
    }
    c->has_mat = false;
    c->adj_ready = false;
    if (!device_ctx(c)) {
      c->has_mat = true;
      return DG_OK;
    }
    dg_status s = set_device(c);
    if (s != DG_OK) return s;
    DG_HIP(c, hipStreamSynchronize(c->stream));
    if (tiled_kernel(c->opt.precision, c->re.N)) {
      const std::vector<double> blk =
          dgh::mfma_material(c->re.N, K, irho_q, lam_q, mu_q, c->opt.precision == DG_FP64);
      if ((s = upload_real(c, c->matblk, blk.data(), blk.size())) != DG_OK) return s;
    }
    if (plain_material(c->opt.precision, c->re.N)) {
      if ((s = upload_real(c, c->irho, irho_q, nq)) != DG_OK) return s;
      if ((s = upload_real(c, c->lam, lam_q, nq)) != DG_OK) return s;
      if ((s = upload_real(c, c->mu, mu_q, nq)) != DG_OK) return s;
    }
    if ((s = upload_real(c, c->zp, zp_n, nn)) != DG_OK) return s;
    if ((s = upload_real(c, c->zs, zs_n, nn)) != DG_OK) return s;
    c->has_mat = true;
    drop_graphs(c);
    if (!c->src.empty()) return upload_sources(c);
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_adjoint_forward(dg_ctx* c, double t0, double dt, int64_t nsteps, int64_t every,
                             void* trace) {
  try {
    if (!c || !trace) return DG_EINVAL;
    if (!std::isfinite(t0) || !std::isfinite(dt) || nsteps < 1 || every < 1)
      return fail(c, DG_EINVAL, "adjoint: bad t0, dt, step count or checkpoint interval");
    dg_status s = ready(c, true);
    if (s != DG_OK) return s;
    if (c->opt.precision == DG_FP32_BF16X3)
      return fail(c, DG_EINVAL, "adjoint: FP64 and FP32 contexts only");
    if (c->nrec == 0) return fail(c, DG_ESTATE, "adjoint: no receivers set");
    if ((s = adj_tables(c)) != DG_OK) return s;
    const int64_t K = c->mesh.K, n = int64_t(9) * K * c->re.Np;
    const int NF4 = 4 * c->re.Nfp, Nq = c->re.Nq;
    const size_t S = size_t(n) * c->elem;
    const int64_t nck = (nsteps + every - 1) / every;
    const size_t tb = size_t(nsteps) * c->nrec * 3 * c->elem;
    const bool upwind = c->opt.flux == DG_FLUX_UPWIND, tiled = adj_tiled(c);
    DG_HIP(c, hipStreamSynchronize(c->stream));
    c->adj_ready = false;
    // the tiled adjoint keeps two segments when the memory allows, so that
    // the replay of one overlaps the reverse sweep of the other
    const size_t segb = S * size_t(every) * 5;
    c->adj_ov = false;
    if (tiled && nck > 1) {
      if (c->adj_seg.bytes == 2 * segb && c->adj_r.bytes == 2 * segb) {
        c->adj_ov = true;   // kept from the last run with this interval
      } else if (c->adj_ov_failed != segb) {
        release(c, c->adj_seg);
        release(c, c->adj_r);
        if (alloc(c, c->adj_seg, 2 * segb) == DG_OK && alloc(c, c->adj_r, 2 * segb) == DG_OK) {
          c->adj_ov = true;
        } else {
          // one segment then; the failed allocation is not an error
          release(c, c->adj_seg);
          release(c, c->adj_r);
          c->adj_ov_failed = segb;
          c->err.clear();
          (void)hipGetLastError();
        }
      }
    }
    const int nseg = c->adj_ov ? 2 : 1;
    struct Need {
      DevBuf* b;
      size_t bytes;
    } need[] = {{&c->adj_ck, S * nck},
                {&c->adj_seg, segb * nseg},
                {&c->adj_r, tiled ? segb * nseg : 0},
                {&c->adj_v, S * 6},
                {&c->adj_gb, size_t(K) * NF4 * 9 * c->elem},
                {&c->adj_hb, tiled ? 0 : size_t(K) * NF4 * 9 * c->elem},
                {&c->adj_grad, size_t(K) * Nq * 3 * sizeof(double)},
                {&c->adj_zb, upwind ? size_t(K) * NF4 * (tiled ? 8 : 4) * c->elem : 0},
                {&c->adj_gradz, upwind ? size_t(K) * c->re.Np * 2 * sizeof(double) : 0},
                {&c->adj_trace, tb}};
    for (auto& x : need)
      if (x.b->bytes != x.bytes && (s = alloc(c, *x.b, x.bytes)) != DG_OK) return s;
    // tiled and upwind: the replay also stores the face-node jumps of every
    // stage input when the memory holds them (else the tile kernel computes
    // them from the stage input); the failed allocation is not an error
    const size_t jb =
        tiled && upwind ? size_t(K) * NF4 * 8 * sizeof(float) * size_t(every) * 5 * nseg : 0;
    if (c->adj_j.bytes != jb) {
      release(c, c->adj_j);
      if (jb && jb != c->adj_j_failed && alloc(c, c->adj_j, jb) != DG_OK) {
        release(c, c->adj_j);
        c->adj_j_failed = jb;
        c->err.clear();
        (void)hipGetLastError();
      }
    }
    char* ck = static_cast<char*>(c->adj_ck.p);
    char* tr = static_cast<char*>(c->adj_trace.p);
    const size_t per = size_t(c->nrec) * 3 * c->elem;
    for (int64_t i = 0; i < nsteps; ++i) {
      if (i % every == 0)
        DG_HIP(c, hipMemcpyAsync(ck + S * size_t(i / every), c->q[c->cur].p, S,
                                 hipMemcpyDeviceToDevice, c->stream));
      if ((s = dg_step(c, t0 + double(i) * dt, dt)) != DG_OK) return s;
      if ((s = launch_receivers(c, tr + per * size_t(i))) != DG_OK) return s;
    }
    DG_HIP(c, copy_sync(c, trace, tr, tb, hipMemcpyDeviceToHost));
    c->adj_t0 = t0;
    c->adj_dt = dt;
    c->adj_nsteps = nsteps;
    c->adj_every = every;
    c->adj_nrec = c->nrec;
    c->adj_ready = true;
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_adjoint_backward(dg_ctx* c, const void* resid, double* grad, double* grad_z) {
  try {
    if (!c || !resid || !grad) return DG_EINVAL;
    dg_status s = ready(c, true);
    if (s != DG_OK) return s;
    if (!c->adj_ready)
      return fail(c, DG_ESTATE,
                  "adjoint: no checkpointed forward run since the last change of mesh, "
                  "material, sources or receivers");
    if (c->adj_nrec != c->nrec)
      return fail(c, DG_ESTATE, "adjoint: receivers changed since the forward run");
    const size_t tb = size_t(c->adj_nsteps) * c->adj_nrec * 3 * c->elem;
    DG_HIP(c, copy_sync(c, c->adj_trace.p, resid, tb, hipMemcpyHostToDevice));
    // the sweep recomputes states in its own buffers: the context's state (the
    // end of the forward run) is left as it is
    if (c->elem == 8)
      s = adj_backward_t<double>(c, static_cast<const double*>(c->adj_trace.p));
    else
      s = adj_backward_t<float>(c, static_cast<const float*>(c->adj_trace.p));
    if (s != DG_OK) return s;
    const size_t gb = size_t(c->mesh.K) * c->re.Nq * 3 * sizeof(double);
    DG_HIP(c, copy_sync(c, grad, c->adj_grad.p, gb, hipMemcpyDeviceToHost));
    if (grad_z) {
      const size_t nz = size_t(c->mesh.K) * c->re.Np * 2;
      if (c->opt.flux == DG_FLUX_UPWIND)
        DG_HIP(c, copy_sync(c, grad_z, c->adj_gradz.p, nz * sizeof(double),
                            hipMemcpyDeviceToHost));
      else
        std::fill(grad_z, grad_z + nz, 0.0);   // the central flux reads no impedance
    }
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_synchronize(dg_ctx* c) {
  try {
    if (!c) return DG_EINVAL;
    dg_status s = set_device(c);
    if (s != DG_OK) return s;
    DG_HIP(c, hipStreamSynchronize(c->stream));
    DG_HIP(c, hipGetLastError());
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_ref_operator(const dg_ctx* c, int32_t which, double* out) {
  try {
    if (!c || !out) return DG_EINVAL;
    const dgh::RefElement& re = c->re;
    const std::vector<double>* src = nullptr;
    switch (which) {
      case 0: src = &re.Dr; break;
      case 1: src = &re.Ds; break;
      case 2: src = &re.Dt; break;
      case 3: src = &re.LIFT; break;
      case 4: src = &re.Vq; break;
      case 5: src = &re.Pq; break;
      case 6:
        for (int i = 0; i < re.Np; ++i) {
          out[i * 3 + 0] = re.r[i];
          out[i * 3 + 1] = re.s[i];
          out[i * 3 + 2] = re.t[i];
        }
        return DG_OK;
      case 7:
        for (int i = 0; i < re.Nq; ++i) {
          out[i * 4 + 0] = re.rq[i];
          out[i * 4 + 1] = re.sq[i];
          out[i * 4 + 2] = re.tq[i];
          out[i * 4 + 3] = re.wq[i];
        }
        return DG_OK;
      default: return DG_EINVAL;
    }
    std::memcpy(out, src->data(), src->size() * sizeof(double));
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_face_nodes(const dg_ctx* c, int32_t* fmask) {
  try {
    if (!c || !fmask) return DG_EINVAL;
    for (size_t i = 0; i < c->re.Fmask.size(); ++i) fmask[i] = c->re.Fmask[i];
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_connectivity(const dg_ctx* c, int32_t* etoe, int32_t* etof, int32_t* nbnode) {
  try {
    if (!c) return DG_EINVAL;
    if (!c->has_mesh) return DG_ESTATE;
    const dgh::MeshData& m = c->mesh;
    const int Nfp = c->re.Nfp;
    for (int64_t i = 0; i < m.K * 4; ++i) {
      if (etoe) etoe[i] = m.EToE[i];
      if (etof) etof[i] = m.EToF[i];
      if (nbnode)
        for (int j = 0; j < Nfp; ++j) nbnode[i * Nfp + j] = m.pat[size_t(m.EToP[i]) * Nfp + j];
    }
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_tile_order(const dg_ctx* c, int32_t* out) {
  try {
    if (!c || !out) return DG_EINVAL;
    if (!c->has_mesh) return DG_ESTATE;
    const std::vector<int32_t> t = dgh::tile_order(c->mesh, dgb::kTile, 8);
    std::memcpy(out, t.data(), t.size() * sizeof(int32_t));
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_geometry(const dg_ctx* c, double* geo, double* fgeo, double* J) {
  try {
    if (!c) return DG_EINVAL;
    if (!c->has_mesh) return DG_ESTATE;
    const dgh::MeshData& m = c->mesh;
    if (geo) std::memcpy(geo, m.geo.data(), m.geo.size() * sizeof(double));
    if (fgeo) std::memcpy(fgeo, m.fgeo.data(), m.fgeo.size() * sizeof(double));
    if (J) std::memcpy(J, m.J.data(), m.J.size() * sizeof(double));
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_batch_create(dg_batch** out, int32_t device, int32_t max_slots) {
  try {
    if (!out || device < 0 || max_slots < 1 || max_slots > (1 << 16)) return DG_EINVAL;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return DG_EDEVICE;
    dg_batch* b = new dg_batch();
    b->device = device;
    b->max_slots = max_slots;
    b->host.resize(size_t(max_slots));
    if (hipMalloc(&b->table, size_t(max_slots) * sizeof(dgb::BatchSlot)) != hipSuccess) {
      delete b;
      return DG_ENOMEM;
    }
    *out = b;
    return DG_OK;
  } catch (...) {
    return exception_status();
  }
}

void dg_batch_destroy(dg_batch* b) {
  if (!b) return;
  if (b->table && hipSetDevice(b->device) == hipSuccess) {
    (void)hipDeviceSynchronize();   // launches of the batch may still read the table
    (void)hipFree(b->table);
  }
  delete b;
}

dg_status dg_batch_advance(dg_batch* b, void* stream, dg_ctx* const* ctxs, int32_t n,
                           const double* dt, int64_t nsteps) {
  try {
    if (!b || !ctxs || n < 1 || !ctxs[0]) return DG_EINVAL;
    if (ctxs[0]->opt.device != b->device)
      return fail(ctxs[0], DG_EINVAL, "batch: contexts on another device than the batch");
    return batch_advance_impl(b->table, b->host.data(), b->max_slots, stream, ctxs, n, dt,
                              nsteps);
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_batch_advance_noalloc(void* stream, dg_ctx* const* ctxs, int32_t n,
                                   const double* dt, int64_t nsteps) {
  try {
    if (!ctxs || n < 1 || !ctxs[0]) return DG_EINVAL;
    dg_ctx* c0 = ctxs[0];
    if (n > kBatchStaticSlots)
      return fail(c0, DG_EINVAL, "batch (no allocation): " + std::to_string(n) +
                                     " contexts, at most " + std::to_string(kBatchStaticSlots));
    dg_status s = set_device(c0);
    if (s != DG_OK) return s;
    const int dev = c0->opt.device;
    if (dev >= kMaxDevices) return fail(c0, DG_EINVAL, "batch (no allocation): device index");
    void* tab = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_scratch_mu);
      if (!g_scratch_ptr[dev]) {
        // with the device current: each GPU holds its own copy of the array
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
          return fail(c0, DG_EDEVICE, std::string("batch (no allocation): scratch address: ") +
                                          hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
      }
      tab = g_scratch_ptr[dev];
    }
    dgb::BatchSlot host[kBatchStaticSlots];
    return batch_advance_impl(tab, host, kBatchStaticSlots, stream, ctxs, n, dt, nsteps);
  } catch (...) {
    return exception_status();
  }
}

dg_status dg_measure_copy(int32_t device, int64_t bytes, int32_t reps, double* gbytes_per_s) {
  if (device < 0 || bytes < 16 || reps < 1 || !gbytes_per_s) return DG_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return DG_EDEVICE;
  const int64_t n = bytes / 16;
  void *src = nullptr, *dst = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  dg_status st = DG_OK;
  int cus = 0;
  float ms = 0.f;
  if (hipMalloc(&src, size_t(n) * 16) != hipSuccess || hipMalloc(&dst, size_t(n) * 16) != hipSuccess) {
    st = DG_ENOMEM;
  } else if (hipMemset(src, 0, size_t(n) * 16) != hipSuccess ||
             hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) !=
                 hipSuccess ||
             hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    st = DG_EDEVICE;
  } else {
    const unsigned grid = unsigned(cus) * 16;
    const auto* s4 = static_cast<const dgp::f32x4*>(src);
    auto* d4 = static_cast<dgp::f32x4*>(dst);
    dgp::copy16<<<grid, 256>>>(s4, d4, n);
    (void)hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps; ++r) dgp::copy16<<<grid, 256>>>(s4, d4, n);
    (void)hipEventRecord(e1, nullptr);
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
        ms <= 0.f)
      st = DG_EDEVICE;
    else
      *gbytes_per_s = 2.0 * double(n) * 16.0 * reps / (double(ms) * 1e-3) / 1e9;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (src) (void)hipFree(src);
  if (dst) (void)hipFree(dst);
  return st;
}

dg_status dg_measure_mfma(int32_t device, int32_t reps, double* tflops) {
  if (device < 0 || reps < 1 || !tflops) return DG_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return DG_EDEVICE;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return DG_EDEVICE;
  const unsigned grid = unsigned(cus) * 8;   // eight waves per SIMD
  const int iters = 2048;
  float* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  dg_status st = DG_OK;
  float ms = 0.f;
  if (hipMalloc(&out, size_t(grid) * 256 * sizeof(float)) != hipSuccess) {
    st = DG_ENOMEM;
  } else if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    st = DG_EDEVICE;
  } else {
    dgp::mfma_loop<<<grid, 256>>>(out, iters);
    (void)hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps; ++r) dgp::mfma_loop<<<grid, 256>>>(out, iters);
    (void)hipEventRecord(e1, nullptr);
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
        ms <= 0.f) {
      st = DG_EDEVICE;
    } else {
      const double flop = double(grid) * 4.0 * iters * 8.0 * 2.0 * 16 * 16 * 32 * reps;
      *tflops = flop / (double(ms) * 1e-3) / 1e12;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (out) (void)hipFree(out);
  return st;
}

}  // extern "C"
