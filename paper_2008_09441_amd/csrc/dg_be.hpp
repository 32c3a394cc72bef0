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
// Operator rows (nodes or quadrature points) are split over the four waves.
// Phases, with a workgroup barrier after each shared one:
//   1  stage q [Np][9] in LDS; issue the face-node loads and neighbour gathers;
//   2  D_d q for d = r, s, t (rows split by wave) into LDS;
//   3  face fluxes [WSG10] into LDS, one thread per face node;
//   4  chain rule with the element's metric terms: r = div(sigma), eps(v);
//   5  r += LIFT f (rows split by wave);
//   6  V_q r, the pointwise material operator (the trace of the normal
//      stresses is gathered across the lanes of a row), into LDS;
//   7  P_q (rows split by wave), then the right-hand side store or the
//      LSRK(5,4) stage update [CK94] straight from the accumulators.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dg_bx.hpp"

namespace dgb {

constexpr int kCS = 17;   // LDS row stride of a [rows][16 columns] buffer

struct BeArgs {
  const float* q_in;     // [9][K][Np]
  float* q_out;          // [9][K][Np] (LSRK mode)
  float* res;            // [9][K][Np] (LSRK mode)
  float* rhs_out;        // [9][K][Np] (rhs mode)
  const float* geo;      // [K][9]: d(r,s,t)_i / d(x,y,z)_j at i*3+j
  const float* fgeo;     // [K][4][4]: outward unit normal, Fscale
  const int32_t* nbn;    // [K][4 Nfp]: neighbour volume node nb * Np + vP of each face node
  const int32_t* fmask;  // [4][Nfp]
  const float* irho;     // [K][Nq]
  const float* lam;      // [K][Nq]
  const float* mu;       // [K][Nq]
  const float* zp;       // [K][Np]
  const float* zs;
  const u32x4* frags;    // [NFRAG][64]
  int64_t K;
  float a, b, dt;
  int lsrk;              // 0: write rhs_out; 1: fused LSRK update
  int upwind;            // 1 upwind, 0 central
};

// LDS use of one workgroup, in floats, and its padded allocation in bytes
template <int N>
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
  static constexpr int USED = (OFF_U + SU) * 4;
  // Padded so that the workgroups one CU can hold (160 KiB of LDS) never use
  // more than 128 KiB together (at most 3 per CU at >40 KiB each, or 2 at
  // >53.3 KiB each).
  static constexpr int FLOOR = USED <= 43690 ? 40976 : (USED <= 65536 ? 54630 : 0);
  static constexpr int BYTES = USED > FLOOR ? USED : FLOOR;
};

// B operand of K step s from an LDS buffer [rows][17]: lane (column e, group
// g) holds rows 32 s + 8 g + j (j < 8) of column e
__device__ __forceinline__ void be_bload(const float* buf, int s, int g, int e, bf16x8& bh,
                                         bf16x8& bl) {
  float v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = buf[(32 * s + 8 * g + j) * kCS + e];
  split8(v, bh, bl);
}

__device__ __forceinline__ f32x4 be_mma(const BeArgs& A, int frag, int lane, const bf16x8& bh,
                                        const bf16x8& bl, f32x4 c) {
  const u32x4 ah = A.frags[(frag + 0) * 64 + lane];
  const u32x4 al = A.frags[(frag + 1) * 64 + lane];
  return mma3(ah, al, bh, bl, c);
}

template <int N>
__global__ __launch_bounds__(kThreads, 2) void stage_be(BeArgs A) {
  using O = EOrd<N>;
  using L = BeLds<N>;
  constexpr int Np = O::Np, Nfp = O::Nfp, NF4 = O::NF4, Nq = O::Nq;
  constexpr int RT = O::RT, KN = O::KN, KF = O::KF, KQ = O::KQ, QT = O::QT;
  constexpr int NK = L::NK, FK = L::FK;
  constexpr int TW = (RT + 3) / 4;   // node tiles per wave (at most)
  static_assert(NF4 <= kThreads && NK <= kThreads && FK <= kThreads, "one item per thread");
  __shared__ __align__(16) float smem[L::BYTES / 4];
  float* sq = smem;                  // [NK][17]: q, columns = fields
  float* sr = smem + L::SQ;          // [NK][17]: r, columns = components
  float* sd = smem + L::OFF_U;       // [3][Np][17]
  float* sf = sd + L::SD;            // [FK][17]
  float* sw = smem + L::OFF_U;       // [QK][17]  (over sd, sf)

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int e = lane & 15, g = lane >> 4;
  // XCD-aware element order: each XCD takes one contiguous range of elements
  const int64_t Gd = gridDim.x, bid = blockIdx.x;
  const int64_t xcd = bid & 7, per = Gd >> 3, rem8 = Gd & 7;
  const int64_t k = xcd * per + (xcd < rem8 ? xcd : rem8) + (bid >> 3);
  const int64_t K = A.K, KNp = K * Np;

  // 1: level-1 loads (face-node tables, state), then the neighbour gathers
  const bool ft = tid < NF4;                       // face-node task of this thread
  const int jf = ft ? tid : NF4 - 1;
  const int vM = A.fmask[jf];
  const unsigned nbi = unsigned(A.nbn[k * NF4 + jf]);
  const f32x4 fg = reinterpret_cast<const f32x4*>(A.fgeo)[k * 4 + jf / Nfp];
  float qv[16];
  {
    const int n = tid < NK ? tid : NK - 1;
    const unsigned nc = unsigned(n < Np ? n : Np - 1);
#pragma unroll
    for (int f = 0; f < 9; ++f) qv[f] = (A.q_in + k * Np + f * KNp)[nc];
  }
  __builtin_amdgcn_sched_barrier(0);
  const float zpM = A.zp[k * Np + vM], zsM = A.zs[k * Np + vM];
  const float zpP = A.zp[nbi], zsP = A.zs[nbi];
  float qP[9];
#pragma unroll
  for (int f = 0; f < 9; ++f) qP[f] = (A.q_in + f * KNp)[nbi];
  if (tid < NK) {
#pragma unroll
    for (int c = 0; c < 16; ++c) sq[tid * kCS + c] = (c < 9 && tid < Np) ? qv[c] : 0.f;
  }
  __syncthreads();

  // 2: D_d q for the wave's node tiles t = wave + 4 i
  {
    f32x4 acc[3][TW];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int i = 0; i < TW; ++i) acc[d][i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KN; ++s) {
      bf16x8 bh, bl;
      be_bload(sq, s, g, e, bh, bl);
#pragma unroll
      for (int i = 0; i < TW; ++i) {
        const int t = wave + 4 * i;
        if (t < RT) {
#pragma unroll
          for (int d = 0; d < 3; ++d)
            acc[d][i] = be_mma(A, O::OFF_D + ((d * RT + t) * KN + s) * 2, lane, bh, bl, acc[d][i]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < TW; ++i) {
      const int t = wave + 4 * i;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = 16 * t + 4 * g + j;
        if (t < RT && n < Np) {
#pragma unroll
          for (int d = 0; d < 3; ++d) sd[(d * Np + n) * kCS + e] = acc[d][i][j];
        }
      }
    }
  }

  // 3: face fluxes, exact-Riemann upwind or central [WSG10], scaled by Fscale
  if (tid < FK) {
    float fl[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) fl[c] = 0.f;
    if (ft) {
      float qM[9];
#pragma unroll
      for (int f = 0; f < 9; ++f) qM[f] = sq[vM * kCS + f];
      const float nx = fg[0], ny = fg[1], nz = fg[2], fs = fg[3];
      const float* P = qP;
      const float jtx = (P[3] - qM[3]) * nx + (P[8] - qM[8]) * ny + (P[7] - qM[7]) * nz;
      const float jty = (P[8] - qM[8]) * nx + (P[4] - qM[4]) * ny + (P[6] - qM[6]) * nz;
      const float jtz = (P[7] - qM[7]) * nx + (P[6] - qM[6]) * ny + (P[5] - qM[5]) * nz;
      const float jvx = P[0] - qM[0], jvy = P[1] - qM[1], jvz = P[2] - qM[2];
      float dvx, dvy, dvz, dtx, dty, dtz;
      if (A.upwind) {
        const float jvn = jvx * nx + jvy * ny + jvz * nz;
        const float jtn = jtx * nx + jty * ny + jtz * nz;
        // hardware reciprocals (1 ulp): the impedance sums are positive
        const float dvn = (zpP * jvn + jtn) * __builtin_amdgcn_rcpf(zpM + zpP);
        const float ivs = __builtin_amdgcn_rcpf(zsM + zsP);
        const float dvtx = (zsP * (jvx - jvn * nx) + (jtx - jtn * nx)) * ivs;
        const float dvty = (zsP * (jvy - jvn * ny) + (jty - jtn * ny)) * ivs;
        const float dvtz = (zsP * (jvz - jvn * nz) + (jtz - jtn * nz)) * ivs;
        dvx = dvn * nx + dvtx;
        dvy = dvn * ny + dvty;
        dvz = dvn * nz + dvtz;
        const float dtn = zpM * dvn;
        dtx = dtn * nx + zsM * dvtx;
        dty = dtn * ny + zsM * dvty;
        dtz = dtn * nz + zsM * dvtz;
      } else {
        dvx = 0.5f * jvx; dvy = 0.5f * jvy; dvz = 0.5f * jvz;
        dtx = 0.5f * jtx; dty = 0.5f * jty; dtz = 0.5f * jtz;
      }
      fl[0] = fs * dtx;
      fl[1] = fs * dty;
      fl[2] = fs * dtz;
      fl[3] = fs * dvx * nx;
      fl[4] = fs * dvy * ny;
      fl[5] = fs * dvz * nz;
      fl[6] = fs * 0.5f * (dvy * nz + dvz * ny);
      fl[7] = fs * 0.5f * (dvx * nz + dvz * nx);
      fl[8] = fs * 0.5f * (dvx * ny + dvy * nx);
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) sf[tid * kCS + c] = c < 9 ? fl[c] : 0.f;
  }
  __syncthreads();

  // 4: chain rule, r_c(n) = sum_d sum_j G_dj w(c, j) (D_d q_{f(c,j)})(n),
  // one node row per thread (rows past Np and columns past 8 are zero)
  if (tid < NK) {
    float G[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) G[i] = A.geo[k * 9 + i];
    const int n = tid < Np ? tid : Np - 1;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      float r = 0.f;
      if (c < 9) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
          for (int j = 0; j < 3; ++j)
            if (comp_weight(c, j) != 0.f)
              r += G[d * 3 + j] * comp_weight(c, j) * sd[(d * Np + n) * kCS + comp_field(c, j)];
      }
      sr[tid * kCS + c] = tid < Np ? r : 0.f;
    }
  }
  __syncthreads();

  // 5: r += LIFT f for the wave's node tiles, in place
  {
#pragma unroll
    for (int i = 0; i < TW; ++i) {
      const int t = wave + 4 * i;
      if (t < RT) {
        f32x4 acc;
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = sr[(16 * t + 4 * g + j) * kCS + e];
#pragma unroll
        for (int s = 0; s < KF; ++s) {
          bf16x8 bh, bl;
          be_bload(sf, s, g, e, bh, bl);
          acc = be_mma(A, O::OFF_L + (t * KF + s) * 2, lane, bh, bl, acc);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) sr[(16 * t + 4 * g + j) * kCS + e] = acc[j];
      }
    }
  }
  __syncthreads();

  // 6: V_q r at the wave's quadrature tiles, then the weight-adjusted
  // material operator: v rows times 1/rho, normal stresses lam tr + 2 mu,
  // shear stresses 2 mu
  {
    bf16x8 bh[KN], bl[KN];
#pragma unroll
    for (int s = 0; s < KN; ++s) be_bload(sr, s, g, e, bh[s], bl[s]);
    for (int t = wave; t < QT; t += 4) {
      f32x4 w = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < KN; ++s) w = be_mma(A, O::OFF_V + (t * KN + s) * 2, lane, bh[s], bl[s], w);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = 16 * t + 4 * g + j;
        const unsigned pc = unsigned(p < Nq ? p : Nq - 1);
        const float ir = (A.irho + k * Nq)[pc], la = (A.lam + k * Nq)[pc], m2 = 2.f * (A.mu + k * Nq)[pc];
        const float tr = __shfl(w[j], 16 * g + 3) + __shfl(w[j], 16 * g + 4) + __shfl(w[j], 16 * g + 5);
        const float v = e < 3 ? ir * w[j] : e < 6 ? la * tr + m2 * w[j] : e < 9 ? m2 * w[j] : 0.f;
        sw[p * kCS + e] = p < Nq ? v : 0.f;
      }
    }
  }
  __syncthreads();

  // 7: P_q for the wave's node tiles, then the store or stage update of
  // component e at nodes 16 t + 4 g + j
#pragma unroll
  for (int i = 0; i < TW; ++i) {
    const int t = wave + 4 * i;
    if (t < RT) {
      f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < KQ; ++s) {
        bf16x8 bh, bl;
        be_bload(sw, s, g, e, bh, bl);
        acc = be_mma(A, O::OFF_P + (t * KQ + s) * 2, lane, bh, bl, acc);
      }
      const int ec = e < 9 ? e : 8;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = 16 * t + 4 * g + j;
        if (e < 9 && n < Np) {
          const int64_t gi = ec * KNp + k * Np + n;
          if (A.lsrk) {
            const float rr = A.a * A.res[gi] + A.dt * acc[j];
            A.res[gi] = rr;
            A.q_out[gi] = sq[n * kCS + ec] + A.b * rr;
          } else {
            A.rhs_out[gi] = acc[j];
          }
        }
      }
    }
  }
}

}  // namespace dgb
