// Fused DG elastic-wave stage with BF16x3 matrix-core contractions (gfx950),
// component-group design.
//
// Every dense contraction of the stage -- reference derivatives plus LIFT,
// interpolation to the quadrature points (V_q) and projection back (P_q) --
// runs on v_mfma_f32_16x16x32_bf16 as a split product: each FP32 operand x is
// written x = hi + lo with hi = bf16(x), lo = bf16(x - hi), and
// A B ~ A_hi B_hi + A_hi B_lo + A_lo B_hi with FP32 accumulation (relative
// error ~2^-16 per product).  Fluxes, the chain rule, material weights and
// the LSRK(5,4) update [CK94] are FP32.
//
// One workgroup (four waves) owns a tile of 16 consecutive elements; the
// MFMA column index is the element, so a lane keeps the same element through
// the whole stage.  Each wave owns a fixed set of output components of the
// right-hand side and carries them through every contraction without any
// exchange with the other waves:
//   wave 0: v_x, v_y          (1/rho weights)
//   wave 1: v_z, s_yz         (1/rho and 2 mu weights)
//   wave 2: s_xx, s_yy, s_zz  (lam tr(e) + 2 mu e: the trace couples them)
//   wave 3: s_xz, s_xy        (2 mu weights)
// Phases (barriers only between the shared ones):
//   A  stage q[9][Np][16] and the metric terms in LDS (coalesced reads);
//   B  face fluxes [9][4 Nfp][16] in LDS, one thread per element face node:
//      own trace from LDS, neighbour trace gathered through the (neighbour,
//      trace pattern) tables, exact-Riemann upwind or central flux [WSG10],
//      scaled by Fscale;
//   C  per wave: r_c = sum_d D_d U_{c,d} + LIFT f_c as one K loop over the
//      concatenated [D_r|D_s|D_t|LIFT] operator [HW08, Ch. 10], with
//      U_{c,d} = sum_j G_dj w_cj q_{f_cj} folding the element's constant
//      metric terms into the inputs (div sigma rows, eps(v) rows);
//   D  per wave, for each chunk of 32 quadrature points: V_q r, the pointwise
//      weight-adjusted material operator [CHW17, C18], accumulation of P_q;
//      the accumulators of one contraction are the B operand of the next
//      (K slots permuted on the host), so values never leave their lane;
//   E  right-hand side store or fused stage update, coalesced over [9][K][Np].
// Operator fragments (hi/lo, in lane order) are read from global memory and
// stay in the L2/L1 caches; the material is stored blocked by element tile in
// the lane order of phase D, so its loads are whole 1 KiB wave transactions.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dg_bx_layout.hpp"

namespace dgb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// four values of the working precision: the MFMA accumulator of a lane and
// one lane's entry of an FP32 / FP64 operator fragment
template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef f32x4 type; };
template <> struct Vec4<double> { typedef f64x4 type; };
template <typename T> using v4_t = typename Vec4<T>::type;

constexpr int kThreads = 256;   // four waves
constexpr int kTile = 16;       // elements per workgroup
constexpr int kES = 17;         // LDS stride of a row of 16 element values (odd)

// Arguments of the stage in working precision T (float: BF16x3 or FP32
// matrix-core products; double: FP64 matrix-core products)
template <typename T>
struct BxArgsT {
  const T* q_in;         // [9][K][Np]
  T* q_out;              // [9][K][Np] (LSRK mode)
  T* res;                // [9][K][Np] (LSRK mode)
  T* rhs_out;            // [9][K][Np] (rhs mode)
  const T* geo;          // [K][9]: d(r,s,t)_i / d(x,y,z)_j at i*3+j
  const T* fgeo;         // [K][4][4]: outward unit normal, Fscale
  const int32_t* nbn;    // [K][4 Nfp]: neighbour volume node nb * Np + vP of each face node
  const int32_t* fmask;  // [4][Nfp]
  const int32_t* torder; // [ceil(K/16)]: tile processed at each launch position
  const T* mat;          // [ceil(K/16)][3][MATS]: 1/rho, lam, mu blocked
  const T* zp;           // [K][Np]
  const T* zs;
  const u32x4* frags;    // BF16x3: [NFRAG][64] u32x4; FP32 / FP64: FOrd fragments of T
  int64_t K;
  T a, b, dt;
  int lsrk;              // 0: write rhs_out; 1: fused LSRK update
  int upwind;            // 1 upwind, 0 central
  T* r_out;              // stage_bx_r: the raw right-hand side R q [9][K][Np]
  T* j_out;              // stage_bx_r, if not null: velocity and traction jumps of
                         // every face node, [K][4 Nfp][8] (jv, jt, 0, 0)
};
typedef BxArgsT<float> BxArgs;


// Output component c (vx vy vz sxx syy szz syz sxz sxy) of the volume term
// is sum_d D_d U_{c,d} with U_{c,d} = sum_j G_dj w(c,j) q_{f(c,j)}: the stress
// row (sigma_{c x}, sigma_{c y}, sigma_{c z}) for the velocity components,
// the symmetrised velocity pattern for the strain components.
__host__ __device__ constexpr int comp_field(int c, int j) {
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
__host__ __device__ constexpr float comp_weight(int c, int j) {
  return c < 3 ? 1.f
       : c < 6 ? (j == c - 3 ? 1.f : 0.f)
       : (j == c - 6 ? 0.f : 0.5f);
}

// components owned by wave W
__host__ __device__ constexpr int wave_ncomp(int W) { return W == 2 ? 3 : 2; }
__host__ __device__ constexpr int wave_comp(int W, int i) {
  return W == 0 ? i : W == 1 ? (i == 0 ? 2 : 6) : W == 2 ? 3 + i : 7 + i;
}

__device__ __forceinline__ f32x4 mma(const u32x4& a, const bf16x8& b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mma3(const u32x4& ah, const u32x4& al, const bf16x8& bh,
                                      const bf16x8& bl, f32x4 c) {
  c = mma(ah, bh, c);
  c = mma(ah, bl, c);
  c = mma(al, bh, c);
  return c;
}

// hi = bf16(x) (round to nearest even), lo = bf16(x - hi), converted in
// pairs (one packed conversion per pair and part)
__device__ __forceinline__ void split8(const float* v, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const f32x2 x = {v[2 * p], v[2 * p + 1]};
    const bf16x2 h = __builtin_convertvector(x, bf16x2);
    const f32x2 r = x - __builtin_convertvector(h, f32x2);
    const bf16x2 l = __builtin_convertvector(r, bf16x2);
    hi[2 * p] = h[0];
    hi[2 * p + 1] = h[1];
    lo[2 * p] = l[0];
    lo[2 * p + 1] = l[1];
  }
}

// LDS use of one workgroup, in values of T, and its padded allocation in bytes
template <int N, typename T = float>
struct BLds {
  using O = BOrd<N>;
  static constexpr int SQ = 9 * O::Np * kES;             // q       [9][Np][17]
  static constexpr int SG = kTile * 9;                   // metric  [16][9]
  static constexpr int SZ = 2 * O::Np * kES;             // Z_p, Z_s [2][Np][17]
  static constexpr int SF = 9 * O::NF4 * kES;            // fluxes  [9][4 Nfp][17]
  static constexpr int SR = 9 * O::Np * kES;             // result  [9][Np][17] (over the fluxes)
  // the three-component wave keeps its V_q B operands (hi/lo, lane order)
  // in LDS behind the result rows during phase D
  static constexpr int RO = (SR + 3) & ~3;
  static constexpr int SRL = sizeof(T) == 4 ? 3 * O::SVQ * 2 * 64 * 4 : 0;
  static constexpr int SU = SF > RO + SRL ? SF : RO + SRL;
  static constexpr int OFF_U = (SQ + SG + SZ + 3) & ~3;  // 16-byte aligned union
  static constexpr int USED = (OFF_U + SU) * int(sizeof(T));
  // Padded so that the workgroups one CU can hold (160 KiB of LDS) never use
  // more than 128 KiB together (at most 3 per CU at >40 KiB each, 2 at
  // >53.3 KiB each, or 1 at >80 KiB each).
  static constexpr int FLOOR =
      USED <= 43690 ? 40976 : USED <= 65536 ? 54630 : USED <= 81920 ? 81936 : 0;
  static constexpr int BYTES = USED > FLOOR ? USED : FLOOR;
};

// Phase C for wave W: acc[i][t] = rows 16 t + 4 g + j of r_{comp i}
template <int N, int W>
__device__ __forceinline__ void vol_lift(const BxArgs& A, const float* sq, const float* sg,
                                         const float* sF, int lane, f32x4 (&acc)[3][BOrd<N>::RT]) {
  using O = BOrd<N>;
  constexpr int Np = O::Np, NF4 = O::NF4, RT = O::RT, SN = O::SN, SVL = O::SVL;
  constexpr int NC = wave_ncomp(W);
  const int e = lane & 15, g = lane >> 4;
  float G[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) G[i] = sg[e * 9 + i];
#pragma unroll
  for (int i = 0; i < NC; ++i)
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};

  // operator fragments are prefetched one K step ahead (the fragment reads
  // hit L2; without the prefetch each step waits for its own)
  u32x4 fc[RT][2], fn[RT][2];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int h = 0; h < 2; ++h) fc[t][h] = A.frags[(O::OFF_V + t * SVL * 2 + h) * 64 + lane];
#pragma unroll
  for (int s = 0; s < SVL; ++s) {
    if (s + 1 < SVL) {
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          fn[t][h] = A.frags[(O::OFF_V + (t * SVL + s + 1) * 2 + h) * 64 + lane];
    }
    __builtin_amdgcn_sched_barrier(0);
    float bv[NC][8];
    if (s < SN) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        // node slots: entries beyond Np meet zero operator columns, so the
        // clamped node only has to be a finite value
        const int m = min(g + 4 * (2 * s + h), Np - 1);
#pragma unroll
        for (int i = 0; i < NC; ++i) {
          const int c = wave_comp(W, i);
          float a[3];
#pragma unroll
          for (int j = 0; j < 3; ++j)
            a[j] = comp_weight(c, j) != 0.f
                       ? comp_weight(c, j) * sq[(comp_field(c, j) * Np + m) * kES + e]
                       : 0.f;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            float u = 0.f;
#pragma unroll
            for (int j = 0; j < 3; ++j)
              if (comp_weight(c, j) != 0.f) u += G[d * 3 + j] * a[j];
            bv[i][3 * h + d] = u;
          }
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int jf = min(g + 4 * (2 * s + h), NF4 - 1);
#pragma unroll
        for (int i = 0; i < NC; ++i) bv[i][6 + h] = sF[(wave_comp(W, i) * NF4 + jf) * kES + e];
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int jf = min(g + 4 * (2 * SN + 8 * (s - SN) + j), NF4 - 1);
#pragma unroll
        for (int i = 0; i < NC; ++i) bv[i][j] = sF[(wave_comp(W, i) * NF4 + jf) * kES + e];
      }
    }
    bf16x8 bh[NC], bl[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) split8(bv[i], bh[i], bl[i]);
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int i = 0; i < NC; ++i) acc[i][t] = mma3(fc[t][0], fc[t][1], bh[i], bl[i], acc[i][t]);
#pragma unroll
    for (int t = 0; t < RT; ++t) fc[t][0] = fn[t][0], fc[t][1] = fn[t][1];
  }
}

// Material samples of chunk ch for this lane: m[f][u] holds quadrature
// points 32 ch + 16 u + 4 g + j (j < 4) of field f (1/rho, lam, mu); only the
// fields wave W uses are loaded
template <int N, int W, typename T = float>
__device__ __forceinline__ void mat_chunk(const BxArgsT<T>& A, int64_t tile, int lane, int ch,
                                          v4_t<T> (&m)[3][2]) {
  using O = BOrd<N>;
  constexpr bool need[3] = {W == 0 || W == 1, W == 2, W != 0};
  const v4_t<T>* mat = reinterpret_cast<const v4_t<T>*>(A.mat) + tile * 3 * (O::MATS / 4);
#pragma unroll
  for (int f = 0; f < 3; ++f)
#pragma unroll
    for (int u = 0; u < 2; ++u)
      m[f][u] = need[f] ? mat[f * (O::MATS / 4) + (ch * 2 + u) * 64 + lane] : v4_t<T>{0, 0, 0, 0};
}

// Phase D for wave W: V_q, material, P_q; the nodal result goes to sr.  m0
// holds the material of chunk 0 (loaded before phase C).
template <int N, int W>
__device__ __forceinline__ void quad_proj(const BxArgs& A, int64_t tile, int lane,
                                          const f32x4 (&acc)[3][BOrd<N>::RT],
                                          const f32x4 (&m0)[3][2], float* sr, bf16x8* srl) {
  using O = BOrd<N>;
  constexpr int Np = O::Np, RT = O::RT, QT = O::QT, QC = O::QC, SVQ = O::SVQ;
  constexpr int NC = wave_ncomp(W);
  const int e = lane & 15, g = lane >> 4;

  // V_q B operands: K slot 8 g + j of step s holds row 4 g + j % 4 of node
  // tile 2 s + j / 4, which is where this lane's accumulator already has it.
  // The three-component wave parks them in LDS (register budget).
  constexpr bool park = (NC == 3);
  bf16x8 rh[NC][SVQ], rl[NC][SVQ];
#pragma unroll
  for (int i = 0; i < NC; ++i)
#pragma unroll
    for (int s = 0; s < SVQ; ++s) {
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int t = 2 * s + j / 4;
        v[j] = t < RT ? acc[i][t][j % 4] : 0.f;
      }
      split8(v, rh[i][s], rl[i][s]);
      if constexpr (park) {
        srl[((i * SVQ + s) * 2 + 0) * 64 + lane] = rh[i][s];
        srl[((i * SVQ + s) * 2 + 1) * 64 + lane] = rl[i][s];
      }
    }

  f32x4 out[NC][RT];
#pragma unroll
  for (int i = 0; i < NC; ++i)
#pragma unroll
    for (int t = 0; t < RT; ++t) out[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};

  // V_q fragments of chunk 0; inside the loop the P_q fragments and the next
  // chunk's material are issued at the top of a chunk, the next chunk's V_q
  // fragments after its V_q products, so every fetch is covered by MFMA work
  u32x4 fv[2][SVQ][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int s = 0; s < SVQ; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h)
        fv[u][s][h] = u < QT ? A.frags[(O::OFF_Q + (u * SVQ + s) * 2 + h) * 64 + lane]
                             : u32x4{0u, 0u, 0u, 0u};
  f32x4 m[3][2];
#pragma unroll
  for (int f = 0; f < 3; ++f) m[f][0] = m0[f][0], m[f][1] = m0[f][1];
#pragma unroll
  for (int ch = 0; ch < QC; ++ch) {
    u32x4 fp[RT][2];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int h = 0; h < 2; ++h) fp[t][h] = A.frags[(O::OFF_P + (t * QC + ch) * 2 + h) * 64 + lane];
    f32x4 mn[3][2];
    if (ch + 1 < QC) mat_chunk<N, W>(A, tile, lane, ch + 1, mn);
    __builtin_amdgcn_sched_barrier(0);
    const f32x4* mi = m[0];
    const f32x4* ml = m[1];
    const f32x4* mm = m[2];
    f32x4 w[NC][2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int i = 0; i < NC; ++i) w[i][u] = f32x4{0.f, 0.f, 0.f, 0.f};
      if (2 * ch + u < QT) {
#pragma unroll
        for (int s = 0; s < SVQ; ++s)
#pragma unroll
          for (int i = 0; i < NC; ++i) {
            if constexpr (park)
              w[i][u] = mma3(fv[u][s][0], fv[u][s][1], srl[((i * SVQ + s) * 2 + 0) * 64 + lane],
                             srl[((i * SVQ + s) * 2 + 1) * 64 + lane], w[i][u]);
            else
              w[i][u] = mma3(fv[u][s][0], fv[u][s][1], rh[i][s], rl[i][s], w[i][u]);
          }
      }
    }
    if (ch + 1 < QC) {
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int s = 0; s < SVQ; ++s)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            fv[u][s][h] = 2 * (ch + 1) + u < QT
                              ? A.frags[(O::OFF_Q + ((2 * (ch + 1) + u) * SVQ + s) * 2 + h) * 64 + lane]
                              : u32x4{0u, 0u, 0u, 0u};
    }
    __builtin_amdgcn_sched_barrier(0);
    // pointwise weight-adjusted material operator
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if constexpr (W == 0) {
        w[0][u] *= mi[u];
        w[1][u] *= mi[u];
      } else if constexpr (W == 1) {
        w[0][u] *= mi[u];
        w[1][u] *= 2.f * mm[u];
      } else if constexpr (W == 2) {
        const f32x4 tr = w[0][u] + w[1][u] + w[2][u];
        const f32x4 m2 = 2.f * mm[u];
#pragma unroll
        for (int i = 0; i < 3; ++i) w[i][u] = ml[u] * tr + m2 * w[i][u];
      } else {
        w[0][u] *= 2.f * mm[u];
        w[1][u] *= 2.f * mm[u];
      }
    }
    // P_q B operands: K slot 8 g + j of chunk ch is row 4 g + j % 4 of
    // quadrature tile 2 ch + j / 4
    bf16x8 ph[NC], pl[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = w[i][j / 4][j % 4];
      split8(v, ph[i], pl[i]);
    }
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int i = 0; i < NC; ++i) out[i][t] = mma3(fp[t][0], fp[t][1], ph[i], pl[i], out[i][t]);
    if (ch + 1 < QC) {
#pragma unroll
      for (int f = 0; f < 3; ++f) m[f][0] = mn[f][0], m[f][1] = mn[f][1];
    }
  }
#pragma unroll
  for (int i = 0; i < NC; ++i)
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = 16 * t + 4 * g + j;
        if (n < Np) sr[(wave_comp(W, i) * Np + n) * kES + e] = out[i][t][j];
      }
}

__device__ __forceinline__ f32x4 mma_f(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mma_f(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// 1 / x: the hardware reciprocal (1 ulp) in FP32, a division in FP64
__device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_t(double x) { return 1.0 / x; }

// Phase C of the FP32 / FP64 kernel for wave W: acc[i][t] = rows
// 16 t + 4 g + j of r_{comp i}, one K slot per lane and step (the order of
// FOrd); operator fragments are fetched one group of four steps ahead.
template <int N, int W, typename T>
__device__ __forceinline__ void vol_lift_f(const BxArgsT<T>& A, const T* sq, const T* sg,
                                           const T* sF, int lane,
                                           v4_t<T> (&acc)[3][BOrd<N>::RT]) {
  using O = FOrd<N>;
  using V4 = v4_t<T>;
  constexpr int Np = O::Np, NF4 = O::NF4, RT = O::RT, NB = O::NB, SV = O::SV, SV4 = O::SV4;
  constexpr int NC = wave_ncomp(W);
  const int e = lane & 15, g = lane >> 4;
  const V4* fr = reinterpret_cast<const V4*>(A.frags) + O::OFF_V;
  T G[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) G[i] = sg[e * 9 + i];
#pragma unroll
  for (int i = 0; i < NC; ++i)
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[i][t] = V4{0, 0, 0, 0};
  V4 fc[RT], fn[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) fc[t] = fr[(t * SV4) * 64 + lane];
#pragma unroll
  for (int q = 0; q < SV4; ++q) {
    if (q + 1 < SV4) {
#pragma unroll
      for (int t = 0; t < RT; ++t) fn[t] = fr[(t * SV4 + q + 1) * 64 + lane];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int s = 4 * q + j;
      if (s >= SV) break;
      T b[NC];
      if (s < 3 * NB) {
        // U_{c,d} at node 4 (s / 3) + g (clamped: beyond Np the operator is zero)
        const int d = s % 3, m = min(4 * (s / 3) + g, Np - 1);
#pragma unroll
        for (int i = 0; i < NC; ++i) {
          const int c = wave_comp(W, i);
          T u = 0;
#pragma unroll
          for (int jj = 0; jj < 3; ++jj)
            if (comp_weight(c, jj) != 0.f)
              u += G[d * 3 + jj] * T(comp_weight(c, jj)) * sq[(comp_field(c, jj) * Np + m) * kES + e];
          b[i] = u;
        }
      } else {
        const int jf = min(4 * (s - 3 * NB) + g, NF4 - 1);
#pragma unroll
        for (int i = 0; i < NC; ++i) b[i] = sF[(wave_comp(W, i) * NF4 + jf) * kES + e];
      }
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int i = 0; i < NC; ++i) acc[i][t] = mma_f(fc[t][j], b[i], acc[i][t]);
    }
#pragma unroll
    for (int t = 0; t < RT; ++t) fc[t] = fn[t];
  }
}

// The raw right-hand side R q (volume terms and LIFT, before the mass
// inverse) of wave W's components from its phase-C accumulators, rows
// 16 t + 4 g + j of element column e, to r_out (FP32 only)
template <int N, int W>
__device__ __forceinline__ void store_raw(const BxArgs& A, int64_t e0, int ne, int lane,
                                          const f32x4 (&acc)[3][BOrd<N>::RT]) {
  using O = BOrd<N>;
  constexpr int Np = O::Np, RT = O::RT, NC = wave_ncomp(W);
  const int e = lane & 15, g = lane >> 4;
  if (e >= ne) return;
  const int64_t KNp = A.K * Np;
  float* out = A.r_out + (e0 + e) * Np;
#pragma unroll
  for (int i = 0; i < NC; ++i)
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = 16 * t + 4 * g + j;
        if (n < Np) out[wave_comp(W, i) * KNp + n] = acc[i][t][j];
      }
}

// Phase D of the FP32 kernel for wave W: per chunk of two quadrature tiles,
// V_q with the node accumulators as the B operand (K step (t, j) is row
// 16 t + 4 g + j), the pointwise weight-adjusted material operator, and
// P_q with the weighted values as the B operand (K step (u, j) is point
// 16 u + 4 g + j); the nodal result goes to sr.
template <int N, int W, typename T>
__device__ __forceinline__ void quad_proj_f(const BxArgsT<T>& A, int64_t tile, int lane,
                                            const v4_t<T> (&acc)[3][BOrd<N>::RT],
                                            const v4_t<T> (&m0)[3][2], T* sr) {
  using O = FOrd<N>;
  using V4 = v4_t<T>;
  constexpr int Np = O::Np, RT = O::RT, QT = O::QT, QC = O::QC;
  constexpr int NC = wave_ncomp(W);
  const int e = lane & 15, g = lane >> 4;
  const V4* frq = reinterpret_cast<const V4*>(A.frags) + O::OFF_Q;
  const V4* frp = reinterpret_cast<const V4*>(A.frags) + O::OFF_P;
  V4 out[NC][RT];
#pragma unroll
  for (int i = 0; i < NC; ++i)
#pragma unroll
    for (int t = 0; t < RT; ++t) out[i][t] = V4{0, 0, 0, 0};
  V4 m[3][2];
#pragma unroll
  for (int f = 0; f < 3; ++f) m[f][0] = m0[f][0], m[f][1] = m0[f][1];
#pragma unroll
  for (int ch = 0; ch < QC; ++ch) {
    V4 fv[2][RT], fp[RT][2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int qt = 2 * ch + u < QT ? 2 * ch + u : QT - 1;
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        fv[u][t] = frq[(qt * RT + t) * 64 + lane];
        fp[t][u] = frp[(t * QT + qt) * 64 + lane];
      }
    }
    V4 mn[3][2];
    if (ch + 1 < QC) mat_chunk<N, W, T>(A, tile, lane, ch + 1, mn);
    __builtin_amdgcn_sched_barrier(0);
    V4 w[NC][2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        w[i][u] = V4{0, 0, 0, 0};
        if (2 * ch + u < QT) {
#pragma unroll
          for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) w[i][u] = mma_f(fv[u][t][j], acc[i][t][j], w[i][u]);
        }
      }
    }
    const V4* mi = m[0];
    const V4* ml = m[1];
    const V4* mm = m[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if constexpr (W == 0) {
        w[0][u] *= mi[u];
        w[1][u] *= mi[u];
      } else if constexpr (W == 1) {
        w[0][u] *= mi[u];
        w[1][u] *= T(2) * mm[u];
      } else if constexpr (W == 2) {
        const V4 tr = w[0][u] + w[1][u] + w[2][u];
        const V4 m2 = T(2) * mm[u];
#pragma unroll
        for (int i = 0; i < 3; ++i) w[i][u] = ml[u] * tr + m2 * w[i][u];
      } else {
        w[0][u] *= T(2) * mm[u];
        w[1][u] *= T(2) * mm[u];
      }
    }
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (2 * ch + u < QT) {
#pragma unroll
          for (int i = 0; i < NC; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) out[i][t] = mma_f(fp[t][u][j], w[i][u][j], out[i][t]);
        }
      }
    if (ch + 1 < QC) {
#pragma unroll
      for (int f = 0; f < 3; ++f) m[f][0] = mn[f][0], m[f][1] = mn[f][1];
    }
  }
#pragma unroll
  for (int i = 0; i < NC; ++i)
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = 16 * t + acc_row(sizeof(T) == 8, g, j);
        if (n < Np) sr[(wave_comp(W, i) * Np + n) * kES + e] = out[i][t][j];
      }
}

// Item map of the tile's state, shared by the staging loads and the final
// update: field f of the tile is TS = 16 Np consecutive floats.  Main items
// r = tid + 256 it (it < MI) cover rows below 256 MI of every field; the TT
// rows left per field form 9 TT tail items t = tid + 256 j, clamped to the
// last one (duplicates repeat its load and store).  Rows are clamped to the
// tile's last valid row.
template <int N>
struct TileMap {
  static constexpr int Np = BOrd<N>::Np;
  static constexpr int TS = kTile * Np;
  static constexpr int MI = TS / kThreads;
  static constexpr int TT = TS - MI * kThreads;
  static constexpr int IT = (9 * TT + kThreads - 1) / kThreads;
  static_assert(TT > 0, "tail items assume 16 Np is not a multiple of 256");
  int rmax;   // last valid row: ne Np - 1
  __device__ explicit TileMap(int ne) : rmax(ne * Np - 1) {}
  __device__ unsigned main_row(int tid, int it) const {
    return min(unsigned(tid + it * kThreads), unsigned(rmax));
  }
  __device__ int tail_item(int tid, int j) const { return min(tid + j * kThreads, 9 * TT - 1); }
  __device__ int tail_field(int tid, int j) const { return tail_item(tid, j) / TT; }
  __device__ unsigned tail_row(int tid, int j) const {
    const int t = tail_item(tid, j);
    return min(unsigned(MI * kThreads + t - (t / TT) * TT), unsigned(rmax));
  }
  // LDS offset of row r (element r / Np, node r % Np) in a [Np][17] field block
  __device__ static int lds_row(unsigned r) {
    const unsigned e = r / Np;
    return int((r - e * Np) * kES + e);
  }
};

// The stage of one tile: launch position bid of a grid of G positions over
// the context's tiles (G = ceil(K / 16)); the kernels below call it for a
// single context or for one slot of a batch.
template <int N, bool F32, typename T = float, bool RST = false>
__device__ __forceinline__ void stage_bx_run(const BxArgsT<T>& A, int64_t G, int64_t bid) {
  static_assert(F32 || sizeof(T) == 4, "BF16x3 products work on FP32 data");
  static_assert(!RST || (F32 && sizeof(T) == 4), "R q is stored by the FP32 kernel");
  using O = BOrd<N>;
  using L = BLds<N, T>;
  using V4 = v4_t<T>;
  constexpr int Np = O::Np, Nfp = O::Nfp, NF4 = O::NF4, RT = O::RT;
  __shared__ __align__(16) T smem[L::BYTES / sizeof(T)];
  T* sq = smem;                   // [9][Np][17]
  T* sg = sq + L::SQ;             // [16][9]
  T* sz = sg + L::SG;             // [2][Np][17]: Z_p, Z_s of the tile's nodes
  T* sF = smem + L::OFF_U;        // [9][NF4][17]  (phases B, C)
  T* sr = sF;                     // [9][Np][17]   (phases D, E)
  bf16x8* srl = reinterpret_cast<bf16x8*>(sF + L::RO);   // wave 2, phase D

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // XCD-aware tile order: consecutive workgroups go round-robin to the eight
  // XCDs, so give each XCD one contiguous range of launch positions; the
  // host's tile order sweeps each range so that face neighbours run close
  // together (neighbour traces then mostly hit that XCD's L2)
  const int64_t xcd = bid & 7, per = G >> 3, rem8 = G & 7;
  const int64_t tile = A.torder[xcd * per + (xcd < rem8 ? xcd : rem8) + (bid >> 3)];
  const int64_t K = A.K;
  const int64_t KNp = K * Np;
  const int64_t e0 = tile * kTile;
  const int ne = int((K - e0) < kTile ? (K - e0) : kTile);
  // component group of this wave, rotated with the tile: the waves of a
  // workgroup go to the CU's four SIMDs in order, so the three-component
  // group of two workgroups sharing a CU then mostly runs on different SIMDs
  const int grp = (wave + int(bid >> 3)) & 3;

  // A: stage q and the metric terms; every thread issues all its loads
  // before the first LDS store (the phase is latency bound otherwise).  The
  // tile's values of field f are the TS = 16 Np consecutive floats at
  // f K Np + e0 Np.  Rows r < 256 MI of every field are read as
  // r = tid + 256 it from a per-field uniform base (no per-item index
  // arithmetic); the TT values left per field are spread over the threads
  // (item t: field t / TT).  Rows past the last element of a ragged tile are
  // clamped to its last value: their columns never reach memory.
  const TileMap<N> tm(ne);
  // Face-node tasks of phase B: one thread per (element, face node),
  // consecutive threads on consecutive face nodes of one element (so that a
  // wave's neighbour gathers fall in a few neighbour elements' lines).  Their
  // loads (neighbour node, face geometry, impedances) are issued here, behind
  // the state loads, and the neighbour gathers right after the state is
  // stored, so that phase B waits for data already in flight.  Slots past
  // the tile (ragged last tile, idx beyond the count) read a valid element
  // and face node and store zero.
  constexpr int TF = kTile * NF4;
  constexpr int IF = (TF + kThreads - 1) / kThreads;
  int vM[IF];
  bool ok[IF];
  T fg[IF][4], qP[IF][9], zpP[IF], zsP[IF];
  unsigned nbi[IF];
  {
    // level 1: the face-node task tables (the gathers depend on nbn), the
    // state, the impedances and the metric terms; level 2: the neighbour
    // gathers.  Issue order matters: the load counter is in order, so the
    // gathers wait for nbn but not for the state loads.
    const int32_t* nbt = A.nbn + e0 * NF4;
    const V4* fgt = reinterpret_cast<const V4*>(A.fgeo) + e0 * 4;
    unsigned ecs[IF];
#pragma unroll
    for (int it = 0; it < IF; ++it) {
      const int idx = tid + it * kThreads;
      const unsigned ic = min(unsigned(idx), unsigned(TF - 1));
      const unsigned e = ic / NF4, jf = ic - e * NF4;
      ok[it] = idx < TF && int(e) < ne;
      ecs[it] = min(e, unsigned(ne - 1));   // a valid element of the tile
      nbi[it] = unsigned(nbt[ecs[it] * NF4 + jf]);
      vM[it] = A.fmask[jf];
      const V4 g4 = fgt[ecs[it] * 4 + jf / Nfp];
#pragma unroll
      for (int j = 0; j < 4; ++j) fg[it][j] = g4[j];
    }
    __builtin_amdgcn_sched_barrier(0);
    const T* qt = A.q_in + e0 * Np;
    T vm[TileMap<N>::MI > 0 ? TileMap<N>::MI : 1][9], vt[TileMap<N>::IT];
#pragma unroll
    for (int it = 0; it < TileMap<N>::MI; ++it)
#pragma unroll
      for (int f = 0; f < 9; ++f) vm[it][f] = (qt + f * KNp)[tm.main_row(tid, it)];
#pragma unroll
    for (int j = 0; j < TileMap<N>::IT; ++j) vt[j] = qt[tm.tail_field(tid, j) * KNp + tm.tail_row(tid, j)];
    const T gv = tid < kTile * 9 && tid / 9 < ne ? A.geo[e0 * 9 + tid] : T(0);
    constexpr int IZ = (kTile * Np + kThreads - 1) / kThreads;
    T zv[2][IZ];
#pragma unroll
    for (int it = 0; it < IZ; ++it) {
      const unsigned r = min(unsigned(tid + it * kThreads), unsigned(tm.rmax));
      zv[0][it] = (A.zp + e0 * Np)[r];
      zv[1][it] = (A.zs + e0 * Np)[r];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int it = 0; it < IF; ++it) {
      // a neighbour inside the tile is read from LDS in phase B; its lanes
      // load the tile's first row instead (one hot line for all of them)
      const unsigned lr = unsigned(nbi[it] - unsigned(e0 * Np)) < unsigned(kTile * Np)
                              ? unsigned(e0 * Np) : nbi[it];
#pragma unroll
      for (int f = 0; f < 9; ++f) qP[it][f] = (A.q_in + f * KNp)[lr];
      zpP[it] = A.zp[lr];
      zsP[it] = A.zs[lr];
    }
#pragma unroll
    for (int it = 0; it < TileMap<N>::MI; ++it) {
      const int li = tm.lds_row(tm.main_row(tid, it));
#pragma unroll
      for (int f = 0; f < 9; ++f) sq[f * Np * kES + li] = vm[it][f];
    }
#pragma unroll
    for (int j = 0; j < TileMap<N>::IT; ++j)   // clamped duplicates store equal values
      sq[tm.tail_field(tid, j) * Np * kES + tm.lds_row(tm.tail_row(tid, j))] = vt[j];
    if (tid < kTile * 9) sg[tid] = gv;
#pragma unroll
    for (int it = 0; it < IZ; ++it) {
      const int r = tid + it * kThreads;
      if (r < kTile * Np) {
        const int li = tm.lds_row(unsigned(r));
        sz[li] = zv[0][it];
        sz[Np * kES + li] = zv[1][it];
      }
    }
  }
  __syncthreads();

  // B: face fluxes
  {
#pragma unroll
    for (int it = 0; it < IF; ++it) {
      const int idx = tid + it * kThreads;
      const int e = min(idx / NF4, kTile - 1);
      const int jf = idx - (idx / NF4) * NF4;
      T qM[9];
#pragma unroll
      for (int f = 0; f < 9; ++f) qM[f] = sq[(f * Np + vM[it]) * kES + e];
      const T nx = fg[it][0], ny = fg[it][1], nz = fg[it][2], fs = fg[it][3];
      // neighbour trace: from LDS when the neighbour is in the tile
      const unsigned rl = nbi[it] - unsigned(e0 * Np);
      const bool inT = rl < unsigned(kTile * Np);
      {
        const unsigned rc = inT ? rl : 0u;
        const unsigned en = rc / Np;
        const int ln = int((rc - en * Np) * kES + en);
#pragma unroll
        for (int f = 0; f < 9; ++f) {
          const T x = sq[f * Np * kES + ln];
          qP[it][f] = inT ? x : qP[it][f];
        }
        const T zpl = sz[ln], zsl = sz[Np * kES + ln];
        zpP[it] = inT ? zpl : zpP[it];
        zsP[it] = inT ? zsl : zsP[it];
      }
      const T* P = qP[it];
      const T jtx = (P[3] - qM[3]) * nx + (P[8] - qM[8]) * ny + (P[7] - qM[7]) * nz;
      const T jty = (P[8] - qM[8]) * nx + (P[4] - qM[4]) * ny + (P[6] - qM[6]) * nz;
      const T jtz = (P[7] - qM[7]) * nx + (P[6] - qM[6]) * ny + (P[5] - qM[5]) * nz;
      const T jvx = P[0] - qM[0], jvy = P[1] - qM[1], jvz = P[2] - qM[2];
      if constexpr (RST) {
        // the jumps the adjoint's impedance gradient reads (jt = t(P) - t(M),
        // t = sigma n, the same expressions as the flux's)
        if (A.j_out && ok[it]) {
          V4* jo = reinterpret_cast<V4*>(A.j_out + ((e0 + e) * NF4 + jf) * 8);
          jo[0] = V4{jvx, jvy, jvz, jtx};
          jo[1] = V4{jty, jtz, T(0), T(0)};
        }
      }
      T dvx, dvy, dvz, dtx, dty, dtz;
      if (A.upwind) {
        const int lm = vM[it] * kES + e;
        const T ZpM = sz[lm], ZsM = sz[Np * kES + lm], ZpP = zpP[it], ZsP = zsP[it];
        const T jvn = jvx * nx + jvy * ny + jvz * nz;
        const T jtn = jtx * nx + jty * ny + jtz * nz;
        // reciprocals of the (positive) impedance sums: 1 ulp in FP32
        const T dvn = (ZpP * jvn + jtn) * rcp_t(ZpM + ZpP);
        const T ivs = rcp_t(ZsM + ZsP);
        const T dvtx = (ZsP * (jvx - jvn * nx) + (jtx - jtn * nx)) * ivs;
        const T dvty = (ZsP * (jvy - jvn * ny) + (jty - jtn * ny)) * ivs;
        const T dvtz = (ZsP * (jvz - jvn * nz) + (jtz - jtn * nz)) * ivs;
        dvx = dvn * nx + dvtx;
        dvy = dvn * ny + dvty;
        dvz = dvn * nz + dvtz;
        const T dtn = ZpM * dvn;
        dtx = dtn * nx + ZsM * dvtx;
        dty = dtn * ny + ZsM * dvty;
        dtz = dtn * nz + ZsM * dvtz;
      } else {
        dvx = T(0.5) * jvx; dvy = T(0.5) * jvy; dvz = T(0.5) * jvz;
        dtx = T(0.5) * jtx; dty = T(0.5) * jty; dtz = T(0.5) * jtz;
      }
      const T z = ok[it] ? fs : T(0);   // zero flux outside the tile
      T fl[9];
      fl[0] = z * dtx;
      fl[1] = z * dty;
      fl[2] = z * dtz;
      fl[3] = z * dvx * nx;
      fl[4] = z * dvy * ny;
      fl[5] = z * dvz * nz;
      fl[6] = z * T(0.5) * (dvy * nz + dvz * ny);
      fl[7] = z * T(0.5) * (dvx * nz + dvz * nx);
      fl[8] = z * T(0.5) * (dvx * ny + dvy * nx);
      if (idx < TF) {
#pragma unroll
        for (int c = 0; c < 9; ++c) sF[(c * NF4 + jf) * kES + e] = fl[c];
      }
    }
  }
  __syncthreads();

  // C: volume + LIFT per wave
  V4 acc[3][RT];
  V4 m0[3][2];   // chunk-0 material, in flight during phase C
  if constexpr (F32) {
    switch (grp) {
      case 0: mat_chunk<N, 0, T>(A, tile, lane, 0, m0); vol_lift_f<N, 0, T>(A, sq, sg, sF, lane, acc); break;
      case 1: mat_chunk<N, 1, T>(A, tile, lane, 0, m0); vol_lift_f<N, 1, T>(A, sq, sg, sF, lane, acc); break;
      case 2: mat_chunk<N, 2, T>(A, tile, lane, 0, m0); vol_lift_f<N, 2, T>(A, sq, sg, sF, lane, acc); break;
      default: mat_chunk<N, 3, T>(A, tile, lane, 0, m0); vol_lift_f<N, 3, T>(A, sq, sg, sF, lane, acc); break;
    }
    if constexpr (RST) {
      switch (grp) {
        case 0: store_raw<N, 0>(A, e0, ne, lane, acc); break;
        case 1: store_raw<N, 1>(A, e0, ne, lane, acc); break;
        case 2: store_raw<N, 2>(A, e0, ne, lane, acc); break;
        default: store_raw<N, 3>(A, e0, ne, lane, acc); break;
      }
    }
  } else {
    switch (grp) {
      case 0: mat_chunk<N, 0>(A, tile, lane, 0, m0); vol_lift<N, 0>(A, sq, sg, sF, lane, acc); break;
      case 1: mat_chunk<N, 1>(A, tile, lane, 0, m0); vol_lift<N, 1>(A, sq, sg, sF, lane, acc); break;
      case 2: mat_chunk<N, 2>(A, tile, lane, 0, m0); vol_lift<N, 2>(A, sq, sg, sF, lane, acc); break;
      default: mat_chunk<N, 3>(A, tile, lane, 0, m0); vol_lift<N, 3>(A, sq, sg, sF, lane, acc); break;
    }
  }
  __syncthreads();   // fluxes consumed: sr may overwrite them

  // D: quadrature and projection per wave
  if constexpr (F32) {
    switch (grp) {
      case 0: quad_proj_f<N, 0, T>(A, tile, lane, acc, m0, sr); break;
      case 1: quad_proj_f<N, 1, T>(A, tile, lane, acc, m0, sr); break;
      case 2: quad_proj_f<N, 2, T>(A, tile, lane, acc, m0, sr); break;
      default: quad_proj_f<N, 3, T>(A, tile, lane, acc, m0, sr); break;
    }
  } else {
    switch (grp) {
      case 0: quad_proj<N, 0>(A, tile, lane, acc, m0, sr, srl); break;
      case 1: quad_proj<N, 1>(A, tile, lane, acc, m0, sr, srl); break;
      case 2: quad_proj<N, 2>(A, tile, lane, acc, m0, sr, srl); break;
      default: quad_proj<N, 3>(A, tile, lane, acc, m0, sr, srl); break;
    }
  }

  // E: right-hand side store or fused stage update, coalesced, done by the
  // three waves other than the three-component one (whose phase D is the
  // longest).  Updater thread u (0..191) owns rows u + 192 it of every
  // field; rows past the tile's last valid row are clamped to it (a
  // duplicate writes the value the row's owner writes).  The residual loads
  // are issued before the barrier, so that they overlap the end of phase D.
  // The thread index is rebuilt from the lane count, which the compiler
  // cannot match with phase A's index arithmetic: otherwise it keeps phase
  // A's addresses alive through the whole kernel to reuse them.
  constexpr int EP = 3 * 64, EI = (kTile * Np + EP - 1) / EP;
  const int64_t t0 = e0 * Np;
  unsigned er[EI];
  T rs[9][EI];
  if (grp != 2) {
    const int u = (grp > 2 ? grp - 1 : grp) * 64 +
                  int(__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)));
#pragma unroll
    for (int it = 0; it < EI; ++it) er[it] = min(unsigned(u + it * EP), unsigned(tm.rmax));
    if (A.lsrk) {
#pragma unroll
      for (int f = 0; f < 9; ++f)
#pragma unroll
        for (int it = 0; it < EI; ++it) rs[f][it] = (A.res + t0 + f * KNp)[er[it]];
    }
  }
  __syncthreads();
  if (grp != 2) {
#pragma unroll
    for (int it = 0; it < EI; ++it) {
      const int li = tm.lds_row(er[it]);
#pragma unroll
      for (int f = 0; f < 9; ++f) {
        const int64_t fb = t0 + f * KNp;
        const T rv = sr[f * Np * kES + li];
        if (A.lsrk) {
          const T rr = A.a * rs[f][it] + A.dt * rv;
          (A.res + fb)[er[it]] = rr;
          (A.q_out + fb)[er[it]] = sq[f * Np * kES + li] + A.b * rr;
        } else {
          (A.rhs_out + fb)[er[it]] = rv;
        }
      }
    }
  }
}

template <int N, bool F32>
__global__ __launch_bounds__(kThreads, 2) void stage_bx(BxArgs A) {
  stage_bx_run<N, F32>(A, gridDim.x, blockIdx.x);
}

// The FP32 stage that also stores the raw right-hand side R q of its input
// (r_out) and, for the upwind flux, the jumps at its face nodes (j_out): the
// replay of a checkpoint interval in the discrete adjoint, whose reverse
// stage needs R y of every stage input and, for the impedance gradient, its
// face-node jumps
template <int N>
__global__ __launch_bounds__(kThreads, 2) void stage_bx_r(BxArgs A) {
  stage_bx_run<N, true, float, true>(A, gridDim.x, blockIdx.x);
}

// FP64 stage on the matrix cores (v_mfma_f64_16x16x4f64): the FP32 kernel's
// tiling in double precision.  At order 4 its LDS (124 KiB) holds one
// workgroup per CU, whose waves may then use all 512 registers of a lane.
template <int N>
__global__ __launch_bounds__(kThreads, 1) void stage_bx_d(BxArgsT<double> A) {
  stage_bx_run<N, true, double>(A, gridDim.x, blockIdx.x);
}

}  // namespace dgb
