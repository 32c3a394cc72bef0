// Tiled discrete adjoint of the FP32 stage at orders 1-4 on the matrix
// cores (v_mfma_f32_16x16x4_f32).  One reverse stage is two kernels:
//
// adj_tile<N, RIN>: one workgroup per 16 consecutive elements (the MFMA
//   columns).  With y the stage input and l = a lres + b ly the adjoint of
//   the stage's residual (written back to lres), it computes per element
//     r  = R y + raw sources                 (volume terms, fluxes, LIFT;
//                                             with RIN, R y is an input: the
//                                             replay's forward stage stores
//                                             it, dgb::stage_bx_r),
//     w  = V_q r,   p = P_q^T l              at the quadrature points,
//     grad += s d/dm <l, W(m) r>             (d/d(1/rho) = sum_v p w,
//                                             d/d lam = tr p tr w,
//                                             d/d mu = 2 sum_s p w),
//     mu = W^T l = V_q^T [weights . p],
//     nu = volume^T mu = sum_d D_d^T (geometry-weighted mu),
//     g  = LIFT^T mu at the face nodes,
//   [CHW17, C18] for W(m) r = P_q[weights . V_q r], [HW08, Ch. 10] for R.
//   Waves 0-2 each own one group of three components (velocities, normal
//   stresses, shear stresses) from R y to nu and g; the material operator
//   and the gradient terms then stay inside a wave except the stress sum of
//   d/d mu, whose two partial sums meet in LDS.  Every product's B operand
//   comes from LDS (y, fluxes, mu) or from registers in the K order of AOrd:
//   the previous product's accumulators, or l and R y loaded in that order
//   (with RIN the nodes of a last node tile of at most four go in one packed
//   step).  All waves compute the face fluxes (with RIN only the face
//   jumps); wave 3 also adds the stress term of the gradient.
//
//   For the upwind flux it also keeps the velocity and traction jumps of
//   every face node (the state the impedance gradient needs), unless they
//   are given (the replay's stage kernel, dgb::stage_bx_r, stores them
//   beside R y): then the tile reads no y at all.
//
// adj_nodes: one thread per volume node.  Adds the flux transposes of the
//   face nodes on the node (its own side, plus the side of the neighbour's
//   face node that reads it) to nu, and ly += s (nu + face terms); for the
//   upwind flux also the impedance gradient (own-side and neighbour-side
//   terms of the same face nodes, from their jumps), as the generic adjoint
//   kernels do.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dg_adj_flux.hpp"
#include "dg_bx_layout.hpp"

namespace dgt {

typedef float f4 __attribute__((ext_vector_type(4)));

struct TileArgs {
  const float* y;        // stage input [9][K][Np]
  const float* r;        // adj_tile<N, true>: its raw right-hand side R y [9][K][Np]
  float* lres;           // [9][K][Np]: in the residual adjoint before this stage, out l
  const float* ly;       // [9][K][Np]
  float* nu;             // out: volume transpose of mu [9][K][Np]
  float* gf;             // out: LIFT^T mu at the face nodes [K][4 Nfp][9]
  float* jmp;            // out (upwind): face-node jumps (jv, jt) [K][4 Nfp][8]
  double* grad;          // [3][K][Nq] += s d/dm <l, W(m) r>
  const float* geo;      // [K][9]
  const float* fgeo;     // [K][4][4]
  const int32_t* nbn;    // [K][4 Nfp] neighbour node, flat (element * Np + node)
  const int32_t* fmask;  // [4 Nfp] volume node of each face node
  const float* mat;      // blocked material (1/rho, lam, mu) [ceil(K/16)][3][MATS]
  const float* zp;       // [K][Np]
  const float* zs;
  const float* frags;    // [NG][64][4]
  const int64_t* src_elem;  // point sources: element, raw response [nsrc][3][Np],
  const float* src_w;       // Ricker parameters (f0, t0, amplitude)
  const double* src_par;
  int nsrc;
  double ts;             // time of the stage (sources)
  int64_t K;
  float a, b;            // l = a lres + b ly
  double s;              // gradient scale
  int upwind;
  int jumps;             // adj_tile<N, true>, upwind: 1 computes the face-node jumps
                         // into jmp; 0 skips them (the replay's stage stored them)
};

constexpr int kThreads = 256;

__device__ __forceinline__ f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// volume-term map: output component c reads field vfield(c, j) with weight
// vweight(c, j) times the metric term G_dj [HW08, Ch. 10]
__host__ __device__ constexpr int vfield(int c, int j) {
  return c == 0 ? (j == 0 ? 3 : j == 1 ? 8 : 7)
       : c == 1 ? (j == 0 ? 8 : j == 1 ? 4 : 6)
       : c == 2 ? (j == 0 ? 7 : j == 1 ? 6 : 5)
       : c == 3 ? 0
       : c == 4 ? 1
       : c == 5 ? 2
       : c == 6 ? (j == 1 ? 2 : 1)
       : c == 7 ? (j == 0 ? 2 : 0)
       : (j == 0 ? 1 : 0);
}
__host__ __device__ constexpr float vweight(int c, int j) {
  return c < 3 ? 1.f : c < 6 ? (j == c - 3 ? 1.f : 0.f) : (j == c - 6 ? 0.f : 0.5f);
}

// Ricker wavelet value of source i at time t (the forward source term)
__device__ inline double ricker(const double* par, int i, double t) {
  const double x = 3.14159265358979323846 * par[3 * i] * (t - par[3 * i + 1]);
  return par[3 * i + 2] * (1.0 - 2.0 * x * x) * exp(-x * x);
}

// The node held by lane group g in item j of node tile t: the chained K
// order 16 t + 4 g + j, except (packed, PK) for the last tile, whose nodes
// 16 t + g sit in item 0 (-1: no node)
template <int N, bool PK>
__device__ __forceinline__ int chained_node(int t, int g, int j) {
  using O = AOrd<N>;
  if (PK && t == O::RT - 1) return j == 0 && g < O::VLAST ? 16 * t + g : -1;
  const int n = 16 * t + 4 * g + j;
  return n < O::Np ? n : -1;
}

// l = a lres + b ly for components c0 .. c0 + 2 of element k0 + e at the
// rows the lane holds in the chained K order (chained_node)
template <int N, bool PK>
__device__ __forceinline__ void load_l(const TileArgs& A, int64_t k0, int c0,
                                       float (&lv)[3][AOrd<N>::RT][4]) {
  using O = AOrd<N>;
  constexpr int Np = O::Np;
  const int lane = threadIdx.x & 63, e = lane & 15, g = lane >> 4;
  const int64_t KNp = A.K * Np, kc = k0 + e < A.K ? k0 + e : A.K - 1;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int t = 0; t < O::RT; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = chained_node<N, PK>(t, g, j);
        const int64_t i = (c0 + c) * KNp + kc * Np + (n >= 0 ? n : 0);
        lv[c][t][j] = n >= 0 ? A.a * A.lres[i] + A.b * A.ly[i] : 0.f;
      }
}

// Waves 0-2: everything from R y to nu and g for components 3W .. 3W + 2.
template <int N, int W, bool RIN>
__device__ __forceinline__ void tile_group(const TileArgs& A, int64_t k0, float* sy,
                                           const float* sf, double* sg, const float (&G)[9],
                                           const float (&lv)[3][AOrd<N>::RT][4]) {
  using O = AOrd<N>;
  constexpr int RT = O::RT, QT = O::QT, FT = O::FT, KN = O::KN, KF = O::KF, KF4 = O::KF4;
  constexpr int Np = O::Np, Nq = O::Nq, NF4 = O::NF4, LN = 4 * KN, LFN = 4 * KF, CS = O::CS;
  constexpr int C0 = 3 * W;
  constexpr bool PK = RIN && O::PACK;   // the last node tile packed in one step
  const int lane = threadIdx.x & 63, e = lane & 15, g = lane >> 4;
  const int64_t K = A.K, KNp = K * Np;
  const int64_t k = k0 + e;
  const bool ok = k < K;
  const int64_t kc = ok ? k : K - 1;
  const f4* fr = reinterpret_cast<const f4*>(A.frags) + lane;
  auto frag = [&](int grp) { return fr[grp * 64]; };

  // r = R y: sum_d D_d (sum_j G_dj w(c, j) y_f(c, j)) + LIFT flux_c
  f4 r[RT][3];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int c = 0; c < 3; ++c) r[t][c] = f4{0.f, 0.f, 0.f, 0.f};
  if constexpr (RIN) {
    // R y given (stored by the forward stage that produced this stage's
    // output), at the chained rows
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int n = chained_node<N, PK>(t, g, j);
          r[t][c][j] = n >= 0 ? A.r[(C0 + c) * KNp + kc * Np + n] : 0.f;
        }
  } else {
  {
    // fragments two steps ahead
    f4 fa[3][RT];
#pragma unroll
    for (int s = 0; s < 2 && s < KN; ++s)
#pragma unroll
      for (int t = 0; t < RT; ++t) fa[s][t] = frag(O::G_D + t * KN + s);
#pragma unroll
    for (int s = 0; s < KN; ++s) {
      if (s + 2 < KN) {
#pragma unroll
        for (int t = 0; t < RT; ++t) fa[(s + 2) % 3][t] = frag(O::G_D + t * KN + s + 2);
      }
      const int m = 4 * s + g;
      float z[3][3];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          float acc = 0.f;
#pragma unroll
          for (int j = 0; j < 3; ++j)
            if (vweight(C0 + c, j) != 0.f)
              acc += vweight(C0 + c, j) * G[3 * d + j] * sy[(vfield(C0 + c, j) * LN + m) * CS + e];
          z[c][d] = acc;
        }
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
          for (int c = 0; c < 3; ++c) r[t][c] = mma(fa[s % 3][t][d], z[c][d], r[t][c]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  {
    f4 fa[2][RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) fa[0][t] = frag(O::G_L + t * KF4);
#pragma unroll
    for (int s4 = 0; s4 < KF4; ++s4) {
      if (s4 + 1 < KF4) {
#pragma unroll
        for (int t = 0; t < RT; ++t) fa[(s4 + 1) & 1][t] = frag(O::G_L + t * KF4 + s4 + 1);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int s = 4 * s4 + i;
        if (s < KF) {
          float b[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) b[c] = sf[((C0 + c) * LFN + 4 * s + g) * CS + e];
#pragma unroll
          for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int c = 0; c < 3; ++c) r[t][c] = mma(fa[s4 & 1][t][i], b[c], r[t][c]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  }
  // raw point sources (velocity rows) of the elements in this tile
  int64_t sel[8];
  if (W == 0 && A.nsrc > 0) {
    for (int i = 0; i < A.nsrc; ++i) {
      if (i % 8 == 0) {
        // the elements of the next eight sources, loaded together
#pragma unroll
        for (int q = 0; q < 8; ++q) sel[q] = i + q < A.nsrc ? A.src_elem[i + q] : -1;
      }
      if (sel[i % 8] != k || !ok) continue;
      const float f = float(ricker(A.src_par, i, A.ts));
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int n = chained_node<N, PK>(t, g, j);
            if (n >= 0) r[t][c][j] += f * A.src_w[(i * 3 + c) * Np + n];
          }
    }
  }
  // write l back
  if (ok) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int n = chained_node<N, PK>(t, g, j);
          if (n >= 0) A.lres[(C0 + c) * KNp + k * Np + n] = lv[c][t][j];
        }
  }
  __syncthreads();   // (1) every wave is done with the fluxes: sg may be written

  // per quadrature tile u: w = V_q r and p = P_q^T l, the gradient terms,
  // the material, and mu += V_q^T [weights . p]
  f4 mu[RT][3];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int c = 0; c < 3; ++c) mu[t][c] = f4{0.f, 0.f, 0.f, 0.f};
  {
    constexpr int MATS = 2 * ((QT + 1) / 2) * 64 * 4;   // BOrd<N>::MATS
    const float* mb = A.mat + (k0 / 16) * 3 * MATS + lane * 4;
    auto matv = [&](int f, int u) { return *reinterpret_cast<const f4*>(mb + f * MATS + u * 256); };
    f4 fv[RT], fp[RT], fvt[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      if (!PK || t < RT - 1) {
        fv[t] = frag(O::G_V + t);
        fp[t] = frag(O::G_P + t);
      } else {
        fv[t] = frag(O::G_VX);   // item 0: V_q, item 1: P_q of the packed tile
      }
      fvt[t] = frag(O::G_VT + t);
    }
    f4 m0 = matv(W == 0 ? 0 : 2, 0), m1 = W == 1 ? matv(1, 0) : f4{0.f, 0.f, 0.f, 0.f};
    // the gradient values of the quadrature tile after this one are read
    // while this one's products run
    double* gr = A.grad + (W == 2 ? 0 : W) * K * Nq + kc * Nq;
    double gnext[4];
    if (W < 2) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = 4 * g + j;
        gnext[j] = gr[p < Nq ? p : Nq - 1];
      }
    }
#pragma unroll
    for (int u = 0; u < QT; ++u) {
      double gold[4];
      if (W < 2) {
#pragma unroll
        for (int j = 0; j < 4; ++j) gold[j] = gnext[j];
        if (u + 1 < QT) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int p = 16 * (u + 1) + 4 * g + j;
            gnext[j] = gr[p < Nq ? p : Nq - 1];
          }
        }
      }
      f4 w[3], p[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) w[c] = p[c] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        if (PK && t == RT - 1) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            w[c] = mma(fv[t][0], r[t][c][0], w[c]);
            p[c] = mma(fv[t][1], lv[c][t][0], p[c]);
          }
          if (u + 1 < QT) fv[t] = frag(O::G_VX + u + 1);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              w[c] = mma(fv[t][j], r[t][c][j], w[c]);
              p[c] = mma(fp[t][j], lv[c][t][j], p[c]);
            }
          if (u + 1 < QT) {
            fv[t] = frag(O::G_V + (u + 1) * RT + t);
            fp[t] = frag(O::G_P + (u + 1) * RT + t);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      const f4 cm0 = m0, cm1 = m1;
      if (u + 1 < QT) {
        m0 = matv(W == 0 ? 0 : 2, u + 1);
        if (W == 1) m1 = matv(1, u + 1);
      }
      // gradient terms at points 16 u + 4 g + j of element k
      float uu[3][4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int pt = 16 * u + 4 * g + j;
        const bool live = ok && pt < Nq;
        if (W == 0) {
          const double g0 = double(p[0][j]) * double(w[0][j]) + double(p[1][j]) * double(w[1][j]) +
                            double(p[2][j]) * double(w[2][j]);
          if (live) gr[pt] = gold[j] + A.s * g0;
#pragma unroll
          for (int c = 0; c < 3; ++c) uu[c][j] = cm0[j] * p[c][j];
        } else if (W == 1) {
          const double g1 = (double(p[0][j]) + double(p[1][j]) + double(p[2][j])) *
                            (double(w[0][j]) + double(w[1][j]) + double(w[2][j]));
          if (live) gr[pt] = gold[j] + A.s * g1;
          sg[(16 * u + 4 * g + j) * 16 + e] = double(p[0][j]) * double(w[0][j]) +
                                              double(p[1][j]) * double(w[1][j]) +
                                              double(p[2][j]) * double(w[2][j]);
          const float tr = p[0][j] + p[1][j] + p[2][j];
          const float m2 = 2.f * cm0[j];
#pragma unroll
          for (int c = 0; c < 3; ++c) uu[c][j] = cm1[j] * tr + m2 * p[c][j];
        } else {
          sg[(16 * QT + 16 * u + 4 * g + j) * 16 + e] = double(p[0][j]) * double(w[0][j]) +
                                                        double(p[1][j]) * double(w[1][j]) +
                                                        double(p[2][j]) * double(w[2][j]);
          const float m2 = 2.f * cm0[j];
#pragma unroll
          for (int c = 0; c < 3; ++c) uu[c][j] = m2 * p[c][j];
        }
      }
#pragma unroll
      for (int t = 0; t < RT; ++t) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int c = 0; c < 3; ++c) mu[t][c] = mma(fvt[t][j], uu[c][j], mu[t][c]);
        if (u + 1 < QT) fvt[t] = frag(O::G_VT + (u + 1) * RT + t);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  __syncthreads();   // (2) y is no longer read: mu may overwrite it
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = 16 * t + 4 * g + j;
      if (n < LN) {
#pragma unroll
        for (int c = 0; c < 3; ++c) sy[((C0 + c) * LN + n) * CS + e] = mu[t][c][j];
      }
    }
  __syncthreads();   // (3) mu complete

  // nu_f = sum_d D_d^T (sum over (c, j) with vfield(c, j) = f of
  // vweight(c, j) G_dj mu_c), for the components f of this group
  {
    f4 o[RT][3];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int c = 0; c < 3; ++c) o[t][c] = f4{0.f, 0.f, 0.f, 0.f};
    f4 fa[3][RT];
#pragma unroll
    for (int s = 0; s < 2 && s < KN; ++s)
#pragma unroll
      for (int t = 0; t < RT; ++t) fa[s][t] = frag(O::G_DT + t * KN + s);
#pragma unroll
    for (int s = 0; s < KN; ++s) {
      if (s + 2 < KN) {
#pragma unroll
        for (int t = 0; t < RT; ++t) fa[(s + 2) % 3][t] = frag(O::G_DT + t * KN + s + 2);
      }
      const int m = 4 * s + g;
      float mv[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        bool used = false;
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
          for (int j = 0; j < 3; ++j) used |= vweight(c, j) != 0.f && vfield(c, j) == C0 + f;
        mv[c] = used ? sy[(c * LN + m) * CS + e] : 0.f;
      }
      float z[3][3];
#pragma unroll
      for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          float acc = 0.f;
#pragma unroll
          for (int c = 0; c < 9; ++c)
#pragma unroll
            for (int j = 0; j < 3; ++j)
              if (vweight(c, j) != 0.f && vfield(c, j) == C0 + f)
                acc += vweight(c, j) * G[3 * d + j] * mv[c];
          z[f][d] = acc;
        }
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
          for (int f = 0; f < 3; ++f) o[t][f] = mma(fa[s % 3][t][d], z[f][d], o[t][f]);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (ok) {
#pragma unroll
      for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int n = 16 * t + 4 * g + j;
            if (n < Np) A.nu[(C0 + f) * KNp + k * Np + n] = o[t][f][j];
          }
    }
  }
  // g_c = LIFT^T mu_c at the face nodes, K from the mu accumulators
  {
    f4 fa[2][RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) fa[0][t] = frag(O::G_LT + t);
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) {
      if (ft + 1 < FT) {
#pragma unroll
        for (int t = 0; t < RT; ++t) fa[(ft + 1) & 1][t] = frag(O::G_LT + (ft + 1) * RT + t);
      }
      f4 o[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) o[c] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int c = 0; c < 3; ++c) o[c] = mma(fa[ft & 1][t][j], mu[t][c][j], o[c]);
      if (ok) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int jf = 16 * ft + 4 * g + j;
          if (jf < NF4) {
#pragma unroll
            for (int c = 0; c < 3; ++c) A.gf[(k * NF4 + jf) * 9 + C0 + c] = o[c][j];
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <int N, bool RIN>
__global__ __launch_bounds__(kThreads, 2) void adj_tile(TileArgs A) {
  using O = AOrd<N>;
  constexpr int Np = O::Np, Nfp = O::Nfp, NF4 = O::NF4, Nq = O::Nq, QT = O::QT, CS = O::CS;
  constexpr int LN = 4 * O::KN, LFN = 4 * O::KF;
  constexpr int NT = (16 * NF4 + kThreads - 1) / kThreads;   // face-node tasks per thread
  static_assert(LFN == NF4, "the face-node steps cover the face nodes exactly");
  __shared__ __align__(16) float smem[O::BYTES / 4];
  float* sy = smem;                                   // y, later mu
  float* sf = smem + O::LY;                           // fluxes
  double* sg = reinterpret_cast<double*>(smem + O::LY);   // stress sums (after the fluxes)
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t K = A.K, KNp = K * Np;
  // XCD-aware tile order: each XCD takes one contiguous range of tiles
  const int64_t Gd = gridDim.x, bid = blockIdx.x;
  const int64_t xcd = bid & 7, per = Gd >> 3, rem8 = Gd & 7;
  const int64_t tile = xcd * per + (xcd < rem8 ? xcd : rem8) + (bid >> 3);
  const int64_t k0 = 16 * tile;

  float G[9];
  {
    const int64_t k = k0 + (tid & 15) < K ? k0 + (tid & 15) : K - 1;
#pragma unroll
    for (int i = 0; i < 9; ++i) G[i] = A.geo[k * 9 + i];
  }
  // the group waves' l (loaded at the start of their phases: issued here,
  // beside the neighbour gathers, it cost registers that then spilled)
  float lv[3][O::RT][4];
  if constexpr (RIN) {
    // R y is given: only the upwind flux's face-node jumps are needed here,
    // from the own and the neighbour's state gathered straight from HBM,
    // unless the replay's stage kernel stored them too
    if (A.upwind && A.jumps) {
      float qM[NT][9], qP[NT][9];
      f4 fg[NT];
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        const int task = tid + kThreads * i;
        const int tk = task < 16 * NF4 ? task : 16 * NF4 - 1;
        const int e = tk / NF4, jf = tk - e * NF4;
        const int64_t k = k0 + e < K ? k0 + e : K - 1;
        const int64_t nb = A.nbn[k * NF4 + jf];
        const int64_t own = k * Np + A.fmask[jf];
        fg[i] = reinterpret_cast<const f4*>(A.fgeo)[k * 4 + jf / Nfp];
#pragma unroll
        for (int f = 0; f < 9; ++f) {
          qM[i][f] = A.y[f * KNp + own];
          qP[i][f] = A.y[f * KNp + nb];
        }
      }
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        const int task = tid + kThreads * i;
        const int e = task / NF4, jf = task - e * NF4;
        if (task < 16 * NF4 && k0 + e < K) {
          float jm[6];
          dga::face_jumps<float>(qM[i], qP[i], fg[i][0], fg[i][1], fg[i][2], jm);
          f4* jo = reinterpret_cast<f4*>(A.jmp + ((k0 + e) * NF4 + jf) * 8);
          jo[0] = f4{jm[0], jm[1], jm[2], jm[3]};
          jo[1] = f4{jm[4], jm[5], 0.f, 0.f};
        }
      }
    }
  } else {
    // the tile's y into LDS (rows past Np and elements past K are zero): all
    // of a thread's loads are issued before the first store
    {
      constexpr int NY = (9 * 16 * LN + kThreads - 1) / kThreads;
      float yv[NY];
  #pragma unroll
      for (int r = 0; r < NY; ++r) {
        const int i = tid + kThreads * r;
        const int c = i / (16 * LN), rem = i - c * 16 * LN, e = rem / LN, m = rem - e * LN;
        const int64_t k = k0 + e;
        const bool live = i < 9 * 16 * LN && m < Np && k < K;
        yv[r] = live ? A.y[c * KNp + k * Np + m] : 0.f;
      }
  #pragma unroll
      for (int r = 0; r < NY; ++r) {
        const int i = tid + kThreads * r;
        const int c = i / (16 * LN), rem = i - c * 16 * LN, e = rem / LN, m = rem - e * LN;
        if (i < 9 * 16 * LN) sy[(c * LN + m) * CS + e] = yv[r];
      }
    }
    // face-node tasks (element e, face node jf): the neighbour's state and
    // impedances, then (after the barrier) the flux from the own side in LDS
    float qP[NT][9], zpP[NT], zsP[NT];
    int vMt[NT];
    f4 fg[NT];
  #pragma unroll
    for (int i = 0; i < NT; ++i) {
      const int task = tid + kThreads * i;
      const int tk = task < 16 * NF4 ? task : 16 * NF4 - 1;
      const int e = tk / NF4, jf = tk - e * NF4;
      const int64_t k = k0 + e < K ? k0 + e : K - 1;
      const int64_t nb = A.nbn[k * NF4 + jf];
      vMt[i] = A.fmask[jf];
      fg[i] = reinterpret_cast<const f4*>(A.fgeo)[k * 4 + jf / Nfp];
      zpP[i] = A.zp[nb];
      zsP[i] = A.zs[nb];
  #pragma unroll
      for (int f = 0; f < 9; ++f) qP[i][f] = A.y[f * KNp + nb];
    }
    __syncthreads();
  #pragma unroll
    for (int i = 0; i < NT; ++i) {
      const int task = tid + kThreads * i;
      if (task >= 16 * NF4) break;
      const int e = task / NF4, jf = task - e * NF4;
      const int64_t k = k0 + e < K ? k0 + e : K - 1;
      const int vM = vMt[i];
      float qM[9], fl[9];
  #pragma unroll
      for (int f = 0; f < 9; ++f) qM[f] = sy[(f * LN + vM) * CS + e];
      dga::flux<float>(qM, qP[i], fg[i][0], fg[i][1], fg[i][2], fg[i][3], A.zp[k * Np + vM],
                       A.zs[k * Np + vM], zpP[i], zsP[i], A.upwind, fl);
  #pragma unroll
      for (int c = 0; c < 9; ++c) sf[(c * LFN + jf) * CS + e] = fl[c];
      if (A.upwind && k0 + e < K) {
        float jm[6];
        dga::face_jumps<float>(qM, qP[i], fg[i][0], fg[i][1], fg[i][2], jm);
        f4* jo = reinterpret_cast<f4*>(A.jmp + (k * NF4 + jf) * 8);
        jo[0] = f4{jm[0], jm[1], jm[2], jm[3]};
        jo[1] = f4{jm[4], jm[5], 0.f, 0.f};
      }
    }
    __syncthreads();
  }

  if (wave == 0) {
    load_l<N, RIN && AOrd<N>::PACK>(A, k0, 0, lv);
    tile_group<N, 0, RIN>(A, k0, sy, sf, sg, G, lv);
  } else if (wave == 1) {
    load_l<N, RIN && AOrd<N>::PACK>(A, k0, 3, lv);
    tile_group<N, 1, RIN>(A, k0, sy, sf, sg, G, lv);
  } else if (wave == 2) {
    load_l<N, RIN && AOrd<N>::PACK>(A, k0, 6, lv);
    tile_group<N, 2, RIN>(A, k0, sy, sf, sg, G, lv);
  } else {
    __syncthreads();   // (1)
    __syncthreads();   // (2): the partial stress sums are complete
    __syncthreads();   // (3): nothing writes them any more
    // d/d mu = 2 (stress sum of the normal stresses + of the shear stresses),
    // while the other waves run their last products; in batches whose loads
    // are all issued before the first store
    const int lane = tid & 63;
    double* g2 = A.grad + 2 * K * Nq;
    constexpr int NB = 16, NI = (16 * Nq + 63) / 64;
#pragma unroll
    for (int r0 = 0; r0 < NI; r0 += NB) {
      double old[NB];
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        const int i = lane + 64 * (r0 + r);
        const int e = i / Nq, p = i - e * Nq;
        const bool live = r0 + r < NI && i < 16 * Nq && k0 + e < K;
        old[r] = live ? g2[(k0 + e) * Nq + p] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        const int i = lane + 64 * (r0 + r);
        const int e = i / Nq, p = i - e * Nq;
        if (r0 + r < NI && i < 16 * Nq && k0 + e < K)
          g2[(k0 + e) * Nq + p] = old[r] + A.s * 2.0 * (sg[p * 16 + e] + sg[(16 * QT + p) * 16 + e]);
      }
    }
  }
}

// The face terms of R^T mu and of the impedance gradient, gathered onto the
// volume nodes, and ly += s (nu + face terms).
struct NodeArgs {
  const float* nu;        // [9][K][Np]
  const float* gf;        // [K][4 Nfp][9]
  const float* jmp;       // [K][4 Nfp][8] face-node jumps (upwind)
  float* ly;              // [9][K][Np]
  double* gradz;          // [2][K][Np] (upwind)
  const float* fgeo;      // [K][4][4]
  const float* zp;        // [K][Np]
  const float* zs;
  const int32_t* nbn;     // [K][4 Nfp] neighbour node (flat)
  const int32_t* nbface;  // [K][4 Nfp] neighbour's face node (flat, element * 4 Nfp + j)
  const int32_t* invf;    // [Np][3] face nodes on each volume node (-1 padded)
  int64_t K;
  int Np, Nfp;
  double s;
  int upwind;
};

__global__ __launch_bounds__(256) void adj_nodes(NodeArgs A) {
  const int Np = A.Np, Nfp = A.Nfp, NF4 = 4 * Nfp;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t K = A.K, KNp = K * Np;
  if (i >= KNp) return;
  const int64_t k = i / Np;
  const int n = int(i - k * Np);
  float h[9];
#pragma unroll
  for (int f = 0; f < 9; ++f) h[f] = A.nu[f * KNp + i];
  const float ZpM = A.zp[i], ZsM = A.zs[i];
  double gp = 0.0, gs = 0.0;
  for (int t = 0; t < 3; ++t) {
    const int jf = A.invf[n * 3 + t];
    if (jf < 0) continue;
    const int64_t own = k * NF4 + jf, jn = A.nbface[own], nb = jn / NF4;
    const int jfn = int(jn - nb * NF4);
    const int64_t nP = A.nbn[own];
    const float ZpP = A.zp[nP], ZsP = A.zs[nP];
    const f4 fo = reinterpret_cast<const f4*>(A.fgeo)[k * 4 + jf / Nfp];
    const f4 fn = reinterpret_cast<const f4*>(A.fgeo)[nb * 4 + jfn / Nfp];
    float go[9], gn[9], a[9], b[9];
#pragma unroll
    for (int f = 0; f < 9; ++f) {
      go[f] = A.gf[own * 9 + f];
      gn[f] = A.gf[jn * 9 + f];
    }
    // own flux (this node on its "-" side), then the neighbour's flux at
    // its face node jn, which reads this node as its "+" side
    dga::rev_flux<float>(go, fo[0], fo[1], fo[2], fo[3], ZpM, ZsM, ZpP, ZsP, A.upwind, a, b);
#pragma unroll
    for (int f = 0; f < 9; ++f) h[f] += a[f];
    dga::rev_flux<float>(gn, fn[0], fn[1], fn[2], fn[3], ZpP, ZsP, ZpM, ZsM, A.upwind, a, b);
#pragma unroll
    for (int f = 0; f < 9; ++f) h[f] += b[f];
    if (A.upwind) {
      const f4* jo = reinterpret_cast<const f4*>(A.jmp + own * 8);
      const f4* jq = reinterpret_cast<const f4*>(A.jmp + jn * 8);
      const f4 o0 = jo[0], o1 = jo[1], q0 = jq[0], q1 = jq[1];
      const float jmo[6] = {o0[0], o0[1], o0[2], o0[3], o1[0], o1[1]};
      const float jmn[6] = {q0[0], q0[1], q0[2], q0[3], q1[0], q1[1]};
      float zo[4], zn[4];
      dga::zgrad_from_jumps<float>(jmo, fo[0], fo[1], fo[2], fo[3], ZpM, ZsM, ZpP, ZsP, go, zo);
      dga::zgrad_from_jumps<float>(jmn, fn[0], fn[1], fn[2], fn[3], ZpP, ZsP, ZpM, ZsM, gn, zn);
      gp += double(zo[0]) + double(zn[2]);
      gs += double(zo[1]) + double(zn[3]);
    }
  }
  const float sf = float(A.s);
#pragma unroll
  for (int f = 0; f < 9; ++f) A.ly[f * KNp + i] += sf * h[f];
  if (A.upwind) {
    A.gradz[i] += A.s * gp;
    A.gradz[KNp + i] += A.s * gs;
  }
}

}  // namespace dgt
