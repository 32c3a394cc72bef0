// Fused DG elastic-wave stage with BF16x3 matrix-core contractions for
// orders 5-7 (gfx950): one element per workgroup.
//
// At these orders the state and fluxes of a 16-element tile no longer fit in
// LDS, so the MFMA columns are the element's nine fields (and then its nine
// output components) instead of sixteen elements; columns 9-15 carry zeros.
// Every dense contraction runs on v_mfma_f32_16x16x32_bf16 as a BF16x3
// split product with FP32 accumulation, exactly as in the 16-element kernel
// (dg_bx.hpp): the reference derivatives D_r, D_s, D_t and LIFT [HW08,
// Ch. 10], and V_q and P_q of the weight-adjusted mass inverse [CHW17, C18].
// Operator rows (nodes or quadrature points) are split over the four waves;
// each wave streams its operator fragments from L2 several products ahead.
// Phases, with a workgroup barrier after each shared one:
//   1  stage q [Np][9] in LDS; issue the face-node loads, the material and
//      residual loads of phases 6 and 7, and the neighbour gathers;
//   2  D_d q for d = r, s, t (rows split by wave) into LDS;
//   3  face fluxes [WSG10] into LDS, one thread per face node;
//   4  chain rule with the element's metric terms: r = div(sigma), eps(v);
//   5  r += LIFT f (rows split by wave);
//   6  V_q r, the pointwise material operator (the trace of the normal
//      stresses is gathered across the lanes of a row), into LDS;
//   7  P_q (rows split by wave), then the right-hand side store or the
//      LSRK(5,4) stage update [CK94] straight from the accumulators.
// The FP32 variant (stage_be<N, true>) runs the same phases on
// v_mfma_f32_16x16x4_f32 with FP32 fragments (EFOrd), and stage_be_d<N> in
// double precision on v_mfma_f64_16x16x4f64.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dg_bx.hpp"

namespace dgb {

constexpr int kCS = 17;   // LDS row stride of a [rows][16 columns] buffer

// kernel arguments in the working precision T (float; double for the FP64
// matrix-core kernel)
template <typename T>
struct BeArgsT {
  const T* q_in;         // [9][K][Np]
  T* q_out;              // [9][K][Np] (LSRK mode)
  T* res;                // [9][K][Np] (LSRK mode)
  T* rhs_out;            // [9][K][Np] (rhs mode)
  const T* geo;          // [K][9]: d(r,s,t)_i / d(x,y,z)_j at i*3+j
  const T* fgeo;         // [K][4][4]: outward unit normal, Fscale
  const int32_t* nbn;    // [K][4 Nfp]: neighbour volume node nb * Np + vP of each face node
  const int32_t* fmask;  // [4][Nfp]
  const T* irho;         // [K][Nq]
  const T* lam;          // [K][Nq]
  const T* mu;           // [K][Nq]
  const T* zp;           // [K][Np]
  const T* zs;
  const u32x4* frags;    // [NFRAG][64]
  int64_t K;
  T a, b, dt;
  int lsrk;              // 0: write rhs_out; 1: fused LSRK update
  int upwind;            // 1 upwind, 0 central
};
typedef BeArgsT<float> BeArgs;

// LDS use of one workgroup, in elements of T, and its padded allocation in
// bytes
template <int N, typename T = float>
struct BeLds {
  using O = EOrd<N>;
  static constexpr int NK = 32 * O::KN, FK = 32 * O::KF, QK = 32 * O::KQ;
  static constexpr int SQ = NK * kCS;                 // q        [NK][17]
  static constexpr int SR = NK * kCS;                 // r        [NK][17]
  static constexpr int SD = 3 * O::Np * kCS;          // D_d q    [3][Np][17]  (phases 2-4)
  static constexpr int SF = FK * kCS;                 // fluxes   [FK][17]     (phases 3-5)
  static constexpr int SW = QK * kCS;                 // weighted V_q r [QK][17] (phases 6-7)
  static constexpr int OFF_U = ((SQ + SR) + 3) & ~3;
  static constexpr int SU = SD + SF > SW ? SD + SF : SW;
  static constexpr int USED = (OFF_U + SU) * int(sizeof(T));
  // Padded so that the workgroups one CU can hold (160 KiB of LDS) never use
  // more than 128 KiB together (at most 3 per CU at >40 KiB each, 2 at
  // >53.3 KiB each, or 1 at >80 KiB each).
  static constexpr int FLOOR =
      USED <= 43690 ? 40976 : USED <= 65536 ? 54630 : USED <= 81920 ? 81936 : 0;
  static constexpr int BYTES = USED > FLOOR ? USED : FLOOR;
};

// Operator fragments in flight per wave: each BF16x3 product waits for its
// two fragments (an L2 round trip), so they are loaded this many products
// ahead
constexpr int kBePD = 4;

// LDS rows of the B operand of K step s from a buffer [rows][17]: lane
// (column e, group g) takes rows 32 s + 8 g + j (j < 8) of column e
__device__ __forceinline__ void be_bread(const float* buf, int s, int g, int e, float (&v)[8]) {
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = buf[(32 * s + 8 * g + j) * kCS + e];
}

__device__ __forceinline__ void be_fload(const BeArgs& A, int frag, int lane, u32x4& ah,
                                         u32x4& al) {
  ah = A.frags[(frag + 0) * 64 + lane];
  al = A.frags[(frag + 1) * 64 + lane];
}

// acc[i] += A_{frag(s, i)} B_s for K steps s < NS and targets i < JS, in the
// order (s, i): the fragments of a product are loaded PD products ahead and
// the LDS rows of B_{s+1} while step s runs
template <int NS, int JS, typename Frag, typename BRead>
__device__ __forceinline__ void be_pipe(const BeArgs& A, int lane, Frag frag, BRead bread,
                                        f32x4 (&acc)[JS]) {
  constexpr int NJ = NS * JS, P = kBePD < NJ ? kBePD : NJ;
  u32x4 fh[P], fl[P];
#pragma unroll
  for (int j = 0; j < P; ++j) be_fload(A, frag(j / JS, j % JS), lane, fh[j], fl[j]);
  float vn[8];
  bread(0, vn);
  bf16x8 bh, bl;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int s = j / JS, i = j % JS;
    if (i == 0) {
      split8(vn, bh, bl);
      if (s + 1 < NS) bread(s + 1, vn);
    }
    acc[i] = mma3(fh[j % P], fl[j % P], bh, bl, acc[i]);
    if (j + P < NJ) be_fload(A, frag((j + P) / JS, (j + P) % JS), lane, fh[j % P], fl[j % P]);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// FP32 variant (v_mfma_f32_16x16x4_f32, fragments in the layout of EFOrd):
// K group s is 16 operator columns; lane (column e, group g) takes rows
// 16 s + 4 j + g of column e as the B operand of the group's product j
template <typename T>
__device__ __forceinline__ void be_bread4(const T* buf, int s, int g, int e, T (&v)[4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = buf[(16 * s + 4 * j + g) * kCS + e];
}

template <int NS, int JS, typename T, typename Frag, typename BRead>
__device__ __forceinline__ void be_pipe_f(const BeArgsT<T>& A, int lane, Frag frag, BRead bread,
                                          v4_t<T> (&acc)[JS]) {
  constexpr int NJ = NS * JS, P = kBePD < NJ ? kBePD : NJ;
  const v4_t<T>* fr = reinterpret_cast<const v4_t<T>*>(A.frags);
  v4_t<T> fa[P];
#pragma unroll
  for (int j = 0; j < P; ++j) fa[j] = fr[frag(j / JS, j % JS) * 64 + lane];
  T vn[4], b[4];
  bread(0, vn);
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int s = j / JS, i = j % JS;
    if (i == 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = vn[q];
      if (s + 1 < NS) bread(s + 1, vn);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[i] = mma_f(fa[j % P][q], b[q], acc[i]);
    if (j + P < NJ) fa[j % P] = fr[frag((j + P) / JS, (j + P) % JS) * 64 + lane];
    __builtin_amdgcn_sched_barrier(0);
  }
}

// The stage of one element: launch position bid of a grid of Gd positions
// over the context's elements (Gd = K); the kernels below call it for a
// single context or for one slot of a batch.
template <int N, bool F32, typename T = float>
__device__ __forceinline__ void stage_be_run(const BeArgsT<T>& A, int64_t Gd, int64_t bid) {
  static_assert(F32 || sizeof(T) == 4, "the BF16x3 kernel works in FP32");
  using V4 = v4_t<T>;
  constexpr bool D64 = sizeof(T) == 8;   // accumulator rows as acc_row(D64, g, j)
  using O = EOrd<N>;
  using OF = EFOrd<N>;
  using L = BeLds<N, T>;
  constexpr int Np = O::Np, Nfp = O::Nfp, NF4 = O::NF4, Nq = O::Nq;
  constexpr int RT = O::RT, KN = O::KN, KF = O::KF, KQ = O::KQ, QT = O::QT;
  static_assert(OF::RT == RT && OF::QT == QT && 16 * OF::KN <= L::NK && 16 * OF::KF <= L::FK &&
                16 * OF::KQ <= 32 * KQ, "FP32 K groups within the zero-padded LDS rows");
  constexpr int NK = L::NK, FK = L::FK;
  constexpr int TW = (RT + 3) / 4;   // node tiles per wave (at most)
  constexpr int QW = (QT + 3) / 4;   // quadrature tiles per wave (at most)
  constexpr int ML = (QW + 3) / 4;   // material loads per lane and field
  static_assert(NF4 <= kThreads && NK <= kThreads && FK <= kThreads, "one item per thread");
  __shared__ __align__(16) T smem[L::BYTES / sizeof(T)];
  T* sq = smem;                  // [NK][17]: q, columns = fields
  T* sr = smem + L::SQ;          // [NK][17]: r, columns = components
  T* sd = smem + L::OFF_U;       // [3][Np][17]
  T* sf = sd + L::SD;            // [FK][17]
  T* sw = smem + L::OFF_U;       // [QK][17]  (over sd, sf)

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int e = lane & 15, g = lane >> 4;
  // XCD-aware element order: each XCD takes one contiguous range of elements
  const int64_t xcd = bid & 7, per = Gd >> 3, rem8 = Gd & 7;
  const int64_t k = xcd * per + (xcd < rem8 ? xcd : rem8) + (bid >> 3);
  const int64_t K = A.K, KNp = K * Np;
  // the wave's node tiles t = wave + 4 i (clamped: a tile past RT repeats the
  // last one and is never stored)
  int tn[TW];
#pragma unroll
  for (int i = 0; i < TW; ++i) tn[i] = min(wave + 4 * i, RT - 1);

  // 1: level-1 loads (face-node tables, state, and everything later phases
  // read from HBM: the wave's material values and residual rows), then the
  // neighbour gathers.  The load counter is in order, so an HBM load issued
  // among the operator-fragment loads of phases 2-7 would stall them.
  const bool ft = tid < NF4;                       // face-node task of this thread
  const int jf = ft ? tid : NF4 - 1;
  const int vM = A.fmask[jf];
  const unsigned nbi = unsigned(A.nbn[k * NF4 + jf]);
  const V4 fg = reinterpret_cast<const V4*>(A.fgeo)[k * 4 + jf / Nfp];
  T qv[16];
  {
    const int n = tid < NK ? tid : NK - 1;
    const unsigned nc = unsigned(n < Np ? n : Np - 1);
#pragma unroll
    for (int f = 0; f < 9; ++f) qv[f] = (A.q_in + k * Np + f * KNp)[nc];
  }
  // material: lane l holds quadrature point 16 t + l % 16 of the wave's
  // quadrature tile t = wave + 4 (4 m + l / 16), for m < ML
  T mt[3][ML];
#pragma unroll
  for (int m = 0; m < ML; ++m) {
    const int t = min(wave + 4 * (4 * m + g), QT - 1);
    const int p = min(16 * t + e, Nq - 1);
    mt[0][m] = (A.irho + k * Nq)[p];
    mt[1][m] = (A.lam + k * Nq)[p];
    mt[2][m] = (A.mu + k * Nq)[p];
  }
  // residual of component e at the lane's output rows 16 t + acc_row(g, j) (read
  // from the state in right-hand-side mode, where it is not used)
  const int ec = e < 9 ? e : 8;
  T rv[TW][4];
  {
    const T* rb = (A.lsrk ? A.res : A.q_in) + ec * KNp + k * Np;
#pragma unroll
    for (int i = 0; i < TW; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) rv[i][j] = rb[min(16 * tn[i] + acc_row(D64, g, j), Np - 1)];
  }
  __builtin_amdgcn_sched_barrier(0);
  const T zpM = A.zp[k * Np + vM], zsM = A.zs[k * Np + vM];
  const T zpP = A.zp[nbi], zsP = A.zs[nbi];
  T qP[9];
#pragma unroll
  for (int f = 0; f < 9; ++f) qP[f] = (A.q_in + f * KNp)[nbi];
  if (tid < NK) {
#pragma unroll
    for (int c = 0; c < 16; ++c) sq[tid * kCS + c] = (c < 9 && tid < Np) ? qv[c] : T(0);
  }
  __syncthreads();

  // 2: D_d q for the wave's node tiles (target i = 3 tile + d)
  {
    V4 acc[3 * TW];
#pragma unroll
    for (int i = 0; i < 3 * TW; ++i) acc[i] = V4{T(0), T(0), T(0), T(0)};
    if constexpr (F32)
      be_pipe_f<OF::KN, 3 * TW>(
          A, lane,
          [&](int s, int i) { return OF::OFF_D + ((i % 3) * RT + tn[i / 3]) * OF::KN + s; },
          [&](int s, T(&v)[4]) { be_bread4(sq, s, g, e, v); }, acc);
    else
      be_pipe<KN, 3 * TW>(
          A, lane,
          [&](int s, int i) { return O::OFF_D + (((i % 3) * RT + tn[i / 3]) * KN + s) * 2; },
          [&](int s, T(&v)[8]) { be_bread(sq, s, g, e, v); }, acc);
#pragma unroll
    for (int i = 0; i < TW; ++i) {
      const int t = wave + 4 * i;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = 16 * t + acc_row(D64, g, j);
        if (t < RT && n < Np) {
#pragma unroll
          for (int d = 0; d < 3; ++d) sd[(d * Np + n) * kCS + e] = acc[3 * i + d][j];
        }
      }
    }
  }

  // 3: face fluxes, exact-Riemann upwind or central [WSG10], scaled by Fscale
  if (tid < FK) {
    T fl[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) fl[c] = T(0);
    if (ft) {
      T qM[9];
#pragma unroll
      for (int f = 0; f < 9; ++f) qM[f] = sq[vM * kCS + f];
      const T nx = fg[0], ny = fg[1], nz = fg[2], fs = fg[3];
      const T* P = qP;
      const T jtx = (P[3] - qM[3]) * nx + (P[8] - qM[8]) * ny + (P[7] - qM[7]) * nz;
      const T jty = (P[8] - qM[8]) * nx + (P[4] - qM[4]) * ny + (P[6] - qM[6]) * nz;
      const T jtz = (P[7] - qM[7]) * nx + (P[6] - qM[6]) * ny + (P[5] - qM[5]) * nz;
      const T jvx = P[0] - qM[0], jvy = P[1] - qM[1], jvz = P[2] - qM[2];
      T dvx, dvy, dvz, dtx, dty, dtz;
      if (A.upwind) {
        const T jvn = jvx * nx + jvy * ny + jvz * nz;
        const T jtn = jtx * nx + jty * ny + jtz * nz;
        // reciprocals (FP32: the hardware one, 1 ulp; FP64: a division): the
        // impedance sums are positive
        const T dvn = (zpP * jvn + jtn) * rcp_t(zpM + zpP);
        const T ivs = rcp_t(zsM + zsP);
        const T dvtx = (zsP * (jvx - jvn * nx) + (jtx - jtn * nx)) * ivs;
        const T dvty = (zsP * (jvy - jvn * ny) + (jty - jtn * ny)) * ivs;
        const T dvtz = (zsP * (jvz - jvn * nz) + (jtz - jtn * nz)) * ivs;
        dvx = dvn * nx + dvtx;
        dvy = dvn * ny + dvty;
        dvz = dvn * nz + dvtz;
        const T dtn = zpM * dvn;
        dtx = dtn * nx + zsM * dvtx;
        dty = dtn * ny + zsM * dvty;
        dtz = dtn * nz + zsM * dvtz;
      } else {
        dvx = T(0.5) * jvx; dvy = T(0.5) * jvy; dvz = T(0.5) * jvz;
        dtx = T(0.5) * jtx; dty = T(0.5) * jty; dtz = T(0.5) * jtz;
      }
      fl[0] = fs * dtx;
      fl[1] = fs * dty;
      fl[2] = fs * dtz;
      fl[3] = fs * dvx * nx;
      fl[4] = fs * dvy * ny;
      fl[5] = fs * dvz * nz;
      fl[6] = fs * T(0.5) * (dvy * nz + dvz * ny);
      fl[7] = fs * T(0.5) * (dvx * nz + dvz * nx);
      fl[8] = fs * T(0.5) * (dvx * ny + dvy * nx);
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) sf[tid * kCS + c] = c < 9 ? fl[c] : T(0);
  }
  __syncthreads();

  // 4: chain rule, r_c(n) = sum_d sum_j G_dj w(c, j) (D_d q_{f(c,j)})(n),
  // one node row per thread (rows past Np and columns past 8 are zero)
  if (tid < NK) {
    T G[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) G[i] = A.geo[k * 9 + i];
    const int n = tid < Np ? tid : Np - 1;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      T r = T(0);
      if (c < 9) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
          for (int j = 0; j < 3; ++j)
            if (comp_weight(c, j) != T(0))
              r += G[d * 3 + j] * comp_weight(c, j) * sd[(d * Np + n) * kCS + comp_field(c, j)];
      }
      sr[tid * kCS + c] = tid < Np ? r : T(0);
    }
  }
  __syncthreads();

  // 5: r += LIFT f for the wave's node tiles, in place
  {
    V4 acc[TW];
#pragma unroll
    for (int i = 0; i < TW; ++i) {
      acc[i] = V4{T(0), T(0), T(0), T(0)};
      if (wave + 4 * i < RT) {
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = sr[(16 * tn[i] + acc_row(D64, g, j)) * kCS + e];
      }
    }
    if constexpr (F32)
      be_pipe_f<OF::KF, TW>(
          A, lane, [&](int s, int i) { return OF::OFF_L + tn[i] * OF::KF + s; },
          [&](int s, T(&v)[4]) { be_bread4(sf, s, g, e, v); }, acc);
    else
      be_pipe<KF, TW>(
          A, lane, [&](int s, int i) { return O::OFF_L + (tn[i] * KF + s) * 2; },
          [&](int s, T(&v)[8]) { be_bread(sf, s, g, e, v); }, acc);
#pragma unroll
    for (int i = 0; i < TW; ++i) {
      if (wave + 4 * i < RT) {
#pragma unroll
        for (int j = 0; j < 4; ++j) sr[(16 * tn[i] + acc_row(D64, g, j)) * kCS + e] = acc[i][j];
      }
    }
  }
  __syncthreads();

  // 6: V_q r at the wave's quadrature tiles t = wave + 4 u, then the
  // weight-adjusted material operator: v rows times 1/rho, normal stresses
  // lam tr + 2 mu, shear stresses 2 mu
  {
    // the weight-adjusted material operator on tile u's V_q r (w) into sw
    auto weigh = [&](int u, const V4& w) {
      const int t = wave + 4 * u;
      if (t < QT) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int p = 16 * t + acc_row(D64, g, j);
          const int src = ((u & 3) << 4) + acc_row(D64, g, j);   // holder of point p
          const T ir = __shfl(mt[0][u >> 2], src), la = __shfl(mt[1][u >> 2], src);
          const T m2 = T(2) * __shfl(mt[2][u >> 2], src);
          const T tr = __shfl(w[j], 16 * g + 3) + __shfl(w[j], 16 * g + 4) + __shfl(w[j], 16 * g + 5);
          const T v = e < 3 ? ir * w[j] : e < 6 ? la * tr + m2 * w[j] : e < 9 ? m2 * w[j] : T(0);
          sw[p * kCS + e] = p < Nq ? v : T(0);
        }
      }
    };
    if constexpr (F32) {
      constexpr int KG = OF::KN;
      T b[KG][4];
#pragma unroll
      for (int s = 0; s < KG; ++s) be_bread4(sr, s, g, e, b[s]);
      constexpr int NJ = QW * KG, P = kBePD < NJ ? kBePD : NJ;
      const V4* fr = reinterpret_cast<const V4*>(A.frags);
      auto frag = [&](int j) {
        const int t = min(wave + 4 * (j / KG), QT - 1);
        return OF::OFF_V + t * KG + j % KG;
      };
      V4 fa[P];
#pragma unroll
      for (int j = 0; j < P; ++j) fa[j] = fr[frag(j) * 64 + lane];
#pragma unroll
      for (int u = 0; u < QW; ++u) {
        V4 w = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int s = 0; s < KG; ++s) {
          const int j = u * KG + s;
#pragma unroll
          for (int q = 0; q < 4; ++q) w = mma_f(fa[j % P][q], b[s][q], w);
          if (j + P < NJ) fa[j % P] = fr[frag(j + P) * 64 + lane];
          __builtin_amdgcn_sched_barrier(0);
        }
        weigh(u, w);
      }
    } else {
      bf16x8 bh[KN], bl[KN];
#pragma unroll
      for (int s = 0; s < KN; ++s) {
        T v[8];
        be_bread(sr, s, g, e, v);
        split8(v, bh[s], bl[s]);
      }
      constexpr int NJ = QW * KN, P = kBePD < NJ ? kBePD : NJ;
      auto frag = [&](int j) {
        const int t = min(wave + 4 * (j / KN), QT - 1);
        return O::OFF_V + (t * KN + j % KN) * 2;
      };
      u32x4 fh[P], fl[P];
#pragma unroll
      for (int j = 0; j < P; ++j) be_fload(A, frag(j), lane, fh[j], fl[j]);
#pragma unroll
      for (int u = 0; u < QW; ++u) {
        V4 w = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int s = 0; s < KN; ++s) {
          const int j = u * KN + s;
          w = mma3(fh[j % P], fl[j % P], bh[s], bl[s], w);
          if (j + P < NJ) be_fload(A, frag(j + P), lane, fh[j % P], fl[j % P]);
          __builtin_amdgcn_sched_barrier(0);
        }
        weigh(u, w);
      }
    }
  }
  __syncthreads();

  // 7: P_q for the wave's node tiles, then the store or stage update of
  // component e at nodes 16 t + 4 g + j
  {
    V4 acc[TW];
#pragma unroll
    for (int i = 0; i < TW; ++i) acc[i] = V4{T(0), T(0), T(0), T(0)};
    if constexpr (F32)
      be_pipe_f<OF::KQ, TW>(
          A, lane, [&](int s, int i) { return OF::OFF_P + tn[i] * OF::KQ + s; },
          [&](int s, T(&v)[4]) { be_bread4(sw, s, g, e, v); }, acc);
    else
      be_pipe<KQ, TW>(
          A, lane, [&](int s, int i) { return O::OFF_P + (tn[i] * KQ + s) * 2; },
          [&](int s, T(&v)[8]) { be_bread(sw, s, g, e, v); }, acc);
#pragma unroll
    for (int i = 0; i < TW; ++i) {
      const int t = wave + 4 * i;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = 16 * t + acc_row(D64, g, j);
        if (t < RT && e < 9 && n < Np) {
          const int64_t gi = ec * KNp + k * Np + n;
          if (A.lsrk) {
            const T rr = A.a * rv[i][j] + A.dt * acc[i][j];
            A.res[gi] = rr;
            A.q_out[gi] = sq[n * kCS + ec] + A.b * rr;
          } else {
            A.rhs_out[gi] = acc[i][j];
          }
        }
      }
    }
  }
}

template <int N, bool F32>
__global__ __launch_bounds__(kThreads, 2) void stage_be(BeArgs A) {
  stage_be_run<N, F32>(A, gridDim.x, blockIdx.x);
}

// FP64 on the matrix cores (v_mfma_f64_16x16x4f64, FP64 fragments in the
// layout of EFOrd): the kernel above in double precision; its LDS (twice
// that of FP32) leaves one workgroup per CU at orders 6 and 7
template <int N>
__global__ __launch_bounds__(kThreads, 1) void stage_be_d(BeArgsT<double> A) {
  stage_be_run<N, true, double>(A, gridDim.x, blockIdx.x);
}

}  // namespace dgb
