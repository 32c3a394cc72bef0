// Fused DG elastic-wave stage with BF16x3 matrix-core contractions (gfx950).
//
// Every dense contraction of the stage -- reference derivatives plus LIFT,
// interpolation to quadrature points (V_q) and projection back (P_q) -- runs
// on v_mfma_f32_16x16x32_bf16 as a split product: each FP32 operand x is
// written x = hi + lo with hi = bf16(x), lo = bf16(x - hi), and
// A B ~ A_hi B_hi + A_hi B_lo + A_lo B_hi with FP32 accumulation (relative
// error ~2^-17 per product).  Everything else (chain rule, fluxes, material
// weights, LSRK update) is FP32.
//
// Mapping.  The MFMA column index is the element: a tile of 16 consecutive
// elements is one column block, so a lane holds the same (node, element)
// entries of every field and pointwise work (chain rule, material weights)
// needs no data exchange.  Operators are the A operand; their hi/lo fragments
// are precomputed on the host in lane order.  The accumulator layout of one
// contraction (row 4*(lane/16) + j of a 16-row tile) is the B-operand layout
// of the next after permuting the next operator's K index on the host, so
// a value stays in the lane that produced it.
//
// The stage is split as
//   r_c = sum_d D_d U_{c,d} + LIFT (Fscale f_c), one K loop over the
//   concatenated [D_r | D_s | D_t | LIFT] operator, where U_{c,d} folds the
//   element's metric terms into the inputs (the metric is constant on an
//   affine element, so sum_d D_d (G_dj u) = G_dj D_d u):
//     velocity rows:  U_{c,d} = sum_j G_dj sigma_cj          (div sigma)
//     stress rows:    U_{ij,d} = (G_dj v_i + G_di v_j) / 2    (eps(v))
//   then V_q r -> pointwise 1/rho and lam tr(e) I + 2 mu e -> P_q, then the
//   right-hand side store or the fused LSRK stage update.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dg_mfma_layout.hpp"

namespace dgm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;         // four waves per workgroup

struct MfmaArgs {
  const float* q_in;     // [9][K][Np]
  float* q_out;
  float* res;
  float* rhs_out;
  const float* geo;      // [K][9]
  const float* fgeo;     // [K][4][4]
  const int32_t* etoe;   // [K][4]
  const uint8_t* etop;   // [K][4]
  const int32_t* pat;    // [npat][Nfp]
  const int32_t* fmask;  // [4][Nfp]
  const float* mat;      // [ntiles][3][QP][16]: 1/rho, lam, mu (zero padded)
  const float* zp;       // [K][Np]
  const float* zs;
  const u32x4* frags;    // [NFRAG][64] bf16x8 operator fragments
  int64_t K;
  int64_t ntiles;
  float a, b, dt;
  int lsrk;
  int upwind;
};

__device__ __forceinline__ f32x4 mma(const u32x4& a, const bf16x8& b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), b, c, 0, 0, 0);
}

// hi/lo bf16 split of 8 floats
__device__ __forceinline__ void split8(const float* v, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const __bf16 h = (__bf16)v[j];
    hi[j] = h;
    lo[j] = (__bf16)(v[j] - (float)h);
  }
}

// acc += A B with A given as hi/lo fragments and B as hi/lo
__device__ __forceinline__ f32x4 mma3(const u32x4& ah, const u32x4& al, const bf16x8& bh,
                                      const bf16x8& bl, f32x4 c) {
  c = mma(ah, bh, c);
  c = mma(ah, bl, c);
  c = mma(al, bh, c);
  return c;
}

// ------------------------------------------------------------------------
// Workgroup-cooperative tile pipeline.  A workgroup of four waves owns one
// tile of 16 elements at a time (persistent over tiles) and moves it through
// phases separated by barriers, so that every global access of a phase is
// issued by all 256 threads at once:
//   P0  stage q[9][16][Np] in LDS (coalesced) and prefetch each lane's
//       material samples for phase P3 into registers;
//   P1  face fluxes: one thread per (element, face node), neighbour traces
//       gathered from global memory, own traces from LDS; the nine scaled
//       flux components go to LDS in the row order of the LIFT columns;
//   P2  [D_r|D_s|D_t|LIFT] contraction, wave w computing node tile w for all
//       nine rows; results are written to LDS already in the lane order of
//       the V_q B operand (the accumulator lane of a value is also its B lane);
//   P3  wave w interpolates all nine fields to quadrature tiles 2w, 2w+1,
//       weights them by the material and contracts them with K block w of P_q;
//   P4  the four partial P_q products are summed in LDS in a fixed wave order
//       (deterministic), then all threads apply the LSRK update with
//       coalesced accesses to res and q.
// Operator fragments are read from global memory (each once per tile and
// wave); with 16 columns per fragment they cost ~6 KB of L2 traffic per
// element and stage.
template <int N>
struct Tile {
  using O = MOrd<N>;
  static constexpr int NpS = O::Np + 1;            // padded LDS row of q
  static constexpr int FRS = 18;                    // LDS row stride of the flux rows (bank-conflict free)
  static constexpr int FROWS = 8 * O::CF;           // flux rows incl. padding
  static constexpr int SQ = 9 * 16 * NpS;           // floats
  static constexpr int SF = 9 * FROWS * FRS;        // flux buffer
  static constexpr int SR = 9 * O::KQB * 64 * 8;    // r in V_q B-lane order
  static constexpr int SP = 6 * O::MT * 64 * 4;     // P_q partial sums of one pass
  static constexpr int SU = SF > SR + SP ? SF : SR + SP;
  static constexpr int LDS_FLOATS = SQ + SU;
};

__device__ __forceinline__ u32x4 ldfrag(const u32x4* __restrict__ f, int idx, int lane) {
  return f[idx * 64 + lane];
}

template <int N, int C0, int NFL>
__device__ __forceinline__ void p3_pass(const MfmaArgs& A, float* su, const float* sq,
                                        const u32x4* __restrict__ fr, const float (&mat)[3][8],
                                        int64_t tile, int64_t e0, int ne, int tid, int lane,
                                        int wave) {
  using O = MOrd<N>;
  using T = Tile<N>;
  constexpr int Np = O::Np, MT = O::MT;
  const int64_t KNp = A.K * Np;
  float* sp = su + T::SR;    // partial-sum buffer [NFL][MT][64][4] (after r)
  f32x4 pacc[NFL][MT];
#pragma unroll
  for (int c = 0; c < NFL; ++c)
#pragma unroll
    for (int t = 0; t < MT; ++t) pacc[c][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  if (wave < O::PKB) {
    f32x4 vq[NFL][2];
#pragma unroll
    for (int c = 0; c < NFL; ++c) vq[c][0] = vq[c][1] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < O::KQB; ++kb) {
      u32x4 ah[2], al[2];
#pragma unroll
      for (int tt = 0; tt < 2; ++tt) {
        const int qt = 2 * wave + tt;
        const int qc = qt < O::QT ? qt : O::QT - 1;
        ah[tt] = ldfrag(fr, O::OFF_Q + (qc * O::KQB + kb) * 2 + 0, lane);
        al[tt] = ldfrag(fr, O::OFF_Q + (qc * O::KQB + kb) * 2 + 1, lane);
      }
#pragma unroll
      for (int c = 0; c < NFL; ++c) {
        const float* src = su + (((C0 + c) * O::KQB + kb) * 64 + lane) * 8;
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = src[j];
        bf16x8 bh, bl;
        split8(v, bh, bl);
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) vq[c][tt] = mma3(ah[tt], al[tt], bh, bl, vq[c][tt]);
      }
    }
    // a quadrature tile beyond QT (odd QT) has zero material: its weights vanish
    float tr[8];
#pragma unroll
    for (int s = 0; s < 8; ++s)
      tr[s] = (C0 == 3) ? vq[0][s / 4][s % 4] + vq[1][s / 4][s % 4] + vq[2][s / 4][s % 4] : 0.f;
    u32x4 ah[MT], al[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      ah[t] = ldfrag(fr, O::OFF_P + (t * O::PKB + wave) * 2 + 0, lane);
      al[t] = ldfrag(fr, O::OFF_P + (t * O::PKB + wave) * 2 + 1, lane);
    }
#pragma unroll
    for (int c = 0; c < NFL; ++c) {
      float w[8];
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const float v = vq[c][s / 4][s % 4];
        if (C0 == 0)
          w[s] = mat[0][s] * v;                                   // 1/rho v
        else if (c < 3)
          w[s] = mat[1][s] * tr[s] + 2.0f * mat[2][s] * v;        // lam tr + 2 mu e
        else
          w[s] = 2.0f * mat[2][s] * v;                            // 2 mu e (shear)
      }
      bf16x8 bh, bl;
      split8(w, bh, bl);
#pragma unroll
      for (int t = 0; t < MT; ++t) pacc[c][t] = mma3(ah[t], al[t], bh, bl, pacc[c][t]);
    }
  }
  constexpr int NW = O::PKB < 4 ? O::PKB : 4;
#pragma unroll 1
  for (int w = 0; w < NW; ++w) {
    if (wave == w) {
#pragma unroll
      for (int c = 0; c < NFL; ++c)
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            float* dst = sp + ((c * MT + t) * 64 + lane) * 4 + j;
            *dst = (w == 0) ? pacc[c][t][j] : *dst + pacc[c][t][j];
          }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < NFL * 16 * Np; idx += 256) {
    const int c = idx / (16 * Np);
    const int rem = idx - c * 16 * Np;
    const int el = rem / Np, node = rem - el * Np;
    if (el >= ne) continue;
    const int f = C0 + c;
    const int t = node >> 4, gg = (node & 15) >> 2, j = node & 3;
    const float r = sp[((c * MT + t) * 64 + gg * 16 + el) * 4 + j];
    const int64_t gi = f * KNp + e0 * Np + rem;
    if (A.lsrk) {
      const float rr = A.a * A.res[gi] + A.dt * r;
      A.res[gi] = rr;
      A.q_out[gi] = sq[(f * 16 + el) * T::NpS + node] + A.b * rr;
    } else {
      A.rhs_out[gi] = r;
    }
  }
  __syncthreads();   // partial-sum buffer reused
  (void)tile;
}

template <int N>
__global__ __launch_bounds__(256, 2) void stage_mfma(MfmaArgs A) {
  using O = MOrd<N>;
  using T = Tile<N>;
  constexpr int Np = O::Np, MT = O::MT, CV = O::CV, CF = O::CF, NF4 = O::NF4;
  __shared__ float lds[T::LDS_FLOATS];
  float* sq = lds;               // [9][16][NpS]
  float* su = lds + T::SQ;       // union: flux | r | partial sums

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int g = lane >> 4, e = lane & 15;
  const int64_t K = A.K;
  const int64_t KNp = K * Np;
  const u32x4* __restrict__ fr = A.frags;

  const int xcd = blockIdx.x & 7;
  const int nwg_x = gridDim.x >> 3;
  const int64_t t0 = A.ntiles * xcd / 8, t1 = A.ntiles * (xcd + 1) / 8;
  for (int64_t tile = t0 + (blockIdx.x >> 3); tile < t1; tile += nwg_x) {
    const int64_t e0 = tile * 16;
    const int ne = int((K - e0) < 16 ? (K - e0) : 16);

    // ---- P0: stage q; prefetch material for P3 (quad tiles 2w, 2w+1)
    for (int idx = tid; idx < 9 * 16 * Np; idx += 256) {
      const int f = idx / (16 * Np);
      const int rem = idx - f * 16 * Np;
      const int el = rem / Np, m = rem - el * Np;
      sq[(f * 16 + el) * T::NpS + m] = (el < ne) ? A.q_in[f * KNp + e0 * Np + rem] : 0.f;
    }
    float mat[3][8];
    {
      const float* mt = A.mat + tile * 3 * O::QP * 16;
#pragma unroll
      for (int tt = 0; tt < 2; ++tt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int qt = 2 * wave + tt;
          const int qp = 16 * qt + 4 * g + j;
          const bool ok = (wave < O::PKB) && (qt < O::QT);
#pragma unroll
          for (int fld = 0; fld < 3; ++fld)
            mat[fld][tt * 4 + j] = ok ? mt[(fld * O::QP + qp) * 16 + e] : 0.f;
        }
    }
    __syncthreads();

    // ---- P1: fluxes at the 16 x NF4 face nodes -> su[c][row][e] (stride FRS)
    for (int idx = tid; idx < 16 * T::FROWS; idx += 256) {
      const int el = idx / T::FROWS, jf = idx - el * T::FROWS;
      float fl[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) fl[c] = 0.f;
      if (jf < NF4 && el < ne) {
        const int64_t k = e0 + el;
        const int face = jf / O::Nfp, i = jf - face * O::Nfp;
        const int vM = A.fmask[face * O::Nfp + i];
        const int64_t nb = A.etoe[k * 4 + face];
        const int vP = A.pat[int(A.etop[k * 4 + face]) * O::Nfp + i];
        float qM[9], qP[9];
#pragma unroll
        for (int f = 0; f < 9; ++f) {
          qM[f] = sq[(f * 16 + el) * T::NpS + vM];
          qP[f] = A.q_in[f * KNp + nb * Np + vP];
        }
        const float* fg = A.fgeo + (k * 4 + face) * 4;
        const float nx = fg[0], ny = fg[1], nz = fg[2], fs = fg[3];
        const float jtx = (qP[3] - qM[3]) * nx + (qP[8] - qM[8]) * ny + (qP[7] - qM[7]) * nz;
        const float jty = (qP[8] - qM[8]) * nx + (qP[4] - qM[4]) * ny + (qP[6] - qM[6]) * nz;
        const float jtz = (qP[7] - qM[7]) * nx + (qP[6] - qM[6]) * ny + (qP[5] - qM[5]) * nz;
        const float jvx = qP[0] - qM[0], jvy = qP[1] - qM[1], jvz = qP[2] - qM[2];
        float dvx, dvy, dvz, dtx, dty, dtz;
        if (A.upwind) {
          const float ZpM = A.zp[k * Np + vM], ZsM = A.zs[k * Np + vM];
          const float ZpP = A.zp[nb * Np + vP], ZsP = A.zs[nb * Np + vP];
          const float jvn = jvx * nx + jvy * ny + jvz * nz;
          const float jtn = jtx * nx + jty * ny + jtz * nz;
          const float dvn = (ZpP * jvn + jtn) / (ZpM + ZpP);
          const float ivs = 1.0f / (ZsM + ZsP);
          const float dvtx = (ZsP * (jvx - jvn * nx) + (jtx - jtn * nx)) * ivs;
          const float dvty = (ZsP * (jvy - jvn * ny) + (jty - jtn * ny)) * ivs;
          const float dvtz = (ZsP * (jvz - jvn * nz) + (jtz - jtn * nz)) * ivs;
          dvx = dvn * nx + dvtx;
          dvy = dvn * ny + dvty;
          dvz = dvn * nz + dvtz;
          const float dtn = ZpM * dvn;
          dtx = dtn * nx + ZsM * dvtx;
          dty = dtn * ny + ZsM * dvty;
          dtz = dtn * nz + ZsM * dvtz;
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
      for (int c = 0; c < 9; ++c) su[(c * T::FROWS + jf) * T::FRS + el] = fl[c];
    }
    __syncthreads();

    // ---- P2: wave w < MT: r tile w = [Dr|Ds|Dt|LIFT] [U; F] for all 9 rows
    f32x4 acc[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (wave < MT) {
      float G[9];
      const int64_t kk = e0 + (e < ne ? e : ne - 1);
#pragma unroll
      for (int i = 0; i < 9; ++i) G[i] = A.geo[kk * 9 + i];
      const float* qe = sq + e * T::NpS;     // field f at qe[f * 16 * NpS + m]
#pragma unroll 1
      for (int kb = 0; kb < O::KVB; ++kb) {
        const int h = 4 * kb + g;
        float bv[9][8];
        if (h < 3 * CV) {
          const int d = h / CV;
          const int m0 = 8 * (h - d * CV);
          const float g0 = G[d * 3 + 0], g1 = G[d * 3 + 1], g2 = G[d * 3 + 2];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int m = m0 + j;
            float v[9];
#pragma unroll
            for (int f = 0; f < 9; ++f) v[f] = (m < Np) ? qe[f * 16 * T::NpS + m] : 0.f;
            // div sigma rows
            bv[0][j] = g0 * v[3] + g1 * v[8] + g2 * v[7];
            bv[1][j] = g0 * v[8] + g1 * v[4] + g2 * v[6];
            bv[2][j] = g0 * v[7] + g1 * v[6] + g2 * v[5];
            // eps(v) rows
            bv[3][j] = g0 * v[0];
            bv[4][j] = g1 * v[1];
            bv[5][j] = g2 * v[2];
            bv[6][j] = 0.5f * (g2 * v[1] + g1 * v[2]);
            bv[7][j] = 0.5f * (g2 * v[0] + g0 * v[2]);
            bv[8][j] = 0.5f * (g1 * v[0] + g0 * v[1]);
          }
        } else if (h < 3 * CV + CF) {
          const int j0 = 8 * (h - 3 * CV);
#pragma unroll
          for (int c = 0; c < 9; ++c)
#pragma unroll
            for (int j = 0; j < 8; ++j) bv[c][j] = su[(c * T::FROWS + j0 + j) * T::FRS + e];
        } else {
#pragma unroll
          for (int c = 0; c < 9; ++c)
#pragma unroll
            for (int j = 0; j < 8; ++j) bv[c][j] = 0.f;
        }
        const u32x4 ah = ldfrag(fr, O::OFF_V + (wave * O::KVB + kb) * 2 + 0, lane);
        const u32x4 al = ldfrag(fr, O::OFF_V + (wave * O::KVB + kb) * 2 + 1, lane);
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          bf16x8 bh, bl;
          split8(bv[c], bh, bl);
          acc[c] = mma3(ah, al, bh, bl, acc[c]);
        }
      }
    }
    __syncthreads();   // flux rows consumed
    if (wave < MT) {
      // node 16 w + 4 g + j  ->  V_q K block w/2, B slot 4 (w%2) + j, same lane
      const int kb = wave >> 1, jo = 4 * (wave & 1);
#pragma unroll
      for (int c = 0; c < 9; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j) su[((c * O::KQB + kb) * 64 + lane) * 8 + jo + j] = acc[c][j];
    }
    if ((MT & 1) && wave == MT) {
      // the odd last node tile leaves slots 4..7 of its K block empty
      const int kb = MT >> 1;
#pragma unroll
      for (int c = 0; c < 9; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j) su[((c * O::KQB + kb) * 64 + lane) * 8 + 4 + j] = 0.f;
    }
    __syncthreads();

    // ---- P3/P4 in two passes (velocity fields 0-2, then stress fields 3-8):
    // wave w < PKB interpolates the pass's fields to quadrature tiles 2w,
    // 2w+1, weights them by the material, contracts with K block w of P_q;
    // the partial products are summed in LDS in a fixed wave order
    // (deterministic), then all threads apply the update.
    p3_pass<N, 0, 3>(A, su, sq, fr, mat, tile, e0, ne, tid, lane, wave);
    p3_pass<N, 3, 6>(A, su, sq, fr, mat, tile, e0, ne, tid, lane, wave);
    __syncthreads();   // LDS reused by the next tile
  }
}

}  // namespace dgm
