// Device kernel of the FP64 DG elastic-wave stage at orders 5-7: the generic
// LDS-staged kernel, templated on the order N.  Every precision at orders
// 1-4, and FP32 and BF16x3 at 5-7, run on the matrix cores (dg_bx.hpp,
// dg_be.hpp).
//
// One workgroup owns a block of E consecutive elements and runs the whole
// stage for them in six phases separated by workgroup barriers:
//   A  stage the block's state q[9][E][Np] in LDS (coalesced: each field's
//      block of E*Np values is contiguous in the [9][K][Np] layout);
//   B  volume terms at each node: reference derivatives D_r, D_s, D_t of the
//      nine fields, chain rule with the element's metric terms, then
//      r_v = div(sigma), r_s = eps(v) [HW08, Ch. 10];
//   C  flux at each face node: own trace from LDS, neighbour trace gathered
//      from global memory through (neighbour element, trace pattern) tables,
//      exact-Riemann upwind or central flux [WSG10], scaled by Fscale;
//   D  LIFT of the face fluxes into r [HW08, Ch. 10];
//   E  interpolate r to the quadrature points, apply 1/rho and
//      C:e = lam tr(e) I + 2 mu e pointwise [CHW17, C18];
//   F  project back with P_q and either store the right-hand side or apply
//      the fused LSRK(5,4) stage update [CK94]:
//        res <- a res + dt rhs;  q_out <- q_in + b res.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgk {

constexpr int kNF = 9;
constexpr int kBlock = 256;

template <int N>
struct Order {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int Nq = (N + 1) * (N + 1) * (N + 1);
  static constexpr int NF4 = 4 * Nfp;
  static constexpr int Nbuf = NF4 > Nq ? NF4 : Nq;
};

// elements per workgroup: as many as fit in 60 KiB of LDS (state, volume
// result and the larger of the face / quadrature buffers), at most 64
template <typename T, int N>
constexpr int elems_per_block() {
  constexpr int per = int(sizeof(T)) * kNF * (2 * Order<N>::Np + Order<N>::Nbuf);
  constexpr int e = 61440 / per;
  return e < 1 ? 1 : (e > 64 ? 64 : e);
}

template <typename T, int N>
constexpr int lds_bytes() {
  constexpr int E = elems_per_block<T, N>();
  return int(sizeof(T)) * kNF * E * (2 * Order<N>::Np + Order<N>::Nbuf);
}

template <typename T>
struct StageArgs {
  // state
  const T* q_in;      // [9][K][Np]
  T* q_out;           // [9][K][Np] (LSRK mode)
  T* res;             // [9][K][Np] (LSRK mode)
  T* rhs_out;         // [9][K][Np] (rhs mode)
  // mesh
  const T* geo;       // [K][9]
  const T* fgeo;      // [K][4][4]
  const int32_t* etoe;   // [K][4]
  const uint8_t* etop;   // [K][4]
  const int32_t* pat;    // [npat][Nfp]
  const int32_t* fmask;  // [4][Nfp]
  // material
  const T* irho;      // [K][Nq]
  const T* lam;
  const T* mu;
  const T* zp;        // [K][Np]
  const T* zs;
  // transposed operators (zero padded, NpP = 4 ceil(Np/4), QP = 32 ceil(Nq/32)),
  // so that threads over output rows read consecutive entries:
  const T* DrT;       // [Np][NpP]: DrT[m][n] = Dr[n][m]
  const T* DsT;
  const T* DtT;
  const T* LIFTT;     // [4 Nfp][NpP]
  const T* VqT;       // [Np][QP]
  const T* PqT;       // [QP][NpP]
  int64_t K;
  T a, b, dt;
  int lsrk;           // 0: write rhs_out; 1: fused LSRK update
  int upwind;         // 1 upwind, 0 central
};

template <typename T, int N>
__global__ __launch_bounds__(kBlock) void stage_generic(StageArgs<T> A) {
  using O = Order<N>;
  constexpr int Np = O::Np, Nfp = O::Nfp, Nq = O::Nq, NF4 = O::NF4;
  constexpr int NpP = 4 * ((Np + 3) / 4), QP = 32 * ((Nq + 31) / 32);
  constexpr int E = elems_per_block<T, N>();
  __shared__ __align__(16) unsigned char smem_raw[lds_bytes<T, N>()];
  T* sq = reinterpret_cast<T*>(smem_raw);   // [9][E][Np]
  T* sr = sq + kNF * E * Np;                // [9][E][Np]
  T* sb = sr + kNF * E * Np;                // [9][E][Nbuf]

  const int64_t K = A.K;
  const int64_t e0 = int64_t(blockIdx.x) * E;
  const int ne = int((K - e0) < E ? (K - e0) : E);
  const int64_t KNp = K * Np;

  // A: stage the block's state
  for (int idx = threadIdx.x; idx < kNF * E * Np; idx += kBlock) {
    const int f = idx / (E * Np);
    const int rem = idx - f * E * Np;
    const int e = rem / Np;
    sq[idx] = (e < ne) ? A.q_in[f * KNp + e0 * Np + rem] : T(0);
  }
  __syncthreads();

  // B: volume terms
  for (int idx = threadIdx.x; idx < E * Np; idx += kBlock) {
    const int e = idx / Np, n = idx - e * Np;
    if (e >= ne) continue;
    T dq[3][kNF];
#pragma unroll
    for (int f = 0; f < kNF; ++f) dq[0][f] = dq[1][f] = dq[2][f] = T(0);
    for (int m = 0; m < Np; ++m) {
      const T dr = A.DrT[m * NpP + n], ds = A.DsT[m * NpP + n], dt = A.DtT[m * NpP + n];
#pragma unroll
      for (int f = 0; f < kNF; ++f) {
        const T v = sq[(f * E + e) * Np + m];
        dq[0][f] += dr * v;
        dq[1][f] += ds * v;
        dq[2][f] += dt * v;
      }
    }
    const T* G = A.geo + (e0 + e) * 9;   // G[i*3+j] = d rst_i / d x_j
    T g[3][kNF];                          // g[j][f] = d q_f / d x_j
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int f = 0; f < kNF; ++f)
        g[j][f] = G[0 * 3 + j] * dq[0][f] + G[1 * 3 + j] * dq[1][f] + G[2 * 3 + j] * dq[2][f];
    // fields: 0 vx 1 vy 2 vz 3 sxx 4 syy 5 szz 6 syz 7 sxz 8 sxy
    T r[kNF];
    r[0] = g[0][3] + g[1][8] + g[2][7];
    r[1] = g[0][8] + g[1][4] + g[2][6];
    r[2] = g[0][7] + g[1][6] + g[2][5];
    r[3] = g[0][0];
    r[4] = g[1][1];
    r[5] = g[2][2];
    r[6] = T(0.5) * (g[2][1] + g[1][2]);
    r[7] = T(0.5) * (g[2][0] + g[0][2]);
    r[8] = T(0.5) * (g[1][0] + g[0][1]);
#pragma unroll
    for (int f = 0; f < kNF; ++f) sr[(f * E + e) * Np + n] = r[f];
  }

  // C: face fluxes (reads sq and global only; writes sb)
  for (int idx = threadIdx.x; idx < E * NF4; idx += kBlock) {
    const int e = idx / NF4, j = idx - e * NF4;
    if (e >= ne) continue;
    const int face = j / Nfp, i = j - face * Nfp;
    const int64_t k = e0 + e;
    const int vM = A.fmask[face * Nfp + i];
    const int64_t nb = A.etoe[k * 4 + face];
    const int vP = A.pat[int(A.etop[k * 4 + face]) * Nfp + i];
    T qM[kNF], qP[kNF];
#pragma unroll
    for (int f = 0; f < kNF; ++f) {
      qM[f] = sq[(f * E + e) * Np + vM];
      qP[f] = A.q_in[f * KNp + nb * Np + vP];
    }
    const T* fg = A.fgeo + (k * 4 + face) * 4;
    const T nx = fg[0], ny = fg[1], nz = fg[2], fs = fg[3];
    // tractions t = sigma n
    const T tMx = qM[3] * nx + qM[8] * ny + qM[7] * nz;
    const T tMy = qM[8] * nx + qM[4] * ny + qM[6] * nz;
    const T tMz = qM[7] * nx + qM[6] * ny + qM[5] * nz;
    const T tPx = qP[3] * nx + qP[8] * ny + qP[7] * nz;
    const T tPy = qP[8] * nx + qP[4] * ny + qP[6] * nz;
    const T tPz = qP[7] * nx + qP[6] * ny + qP[5] * nz;
    const T jvx = qP[0] - qM[0], jvy = qP[1] - qM[1], jvz = qP[2] - qM[2];
    const T jtx = tPx - tMx, jty = tPy - tMy, jtz = tPz - tMz;
    T dvx, dvy, dvz, dtx, dty, dtz;
    if (A.upwind) {
      const T ZpM = A.zp[k * Np + vM], ZsM = A.zs[k * Np + vM];
      const T ZpP = A.zp[nb * Np + vP], ZsP = A.zs[nb * Np + vP];
      const T jvn = jvx * nx + jvy * ny + jvz * nz;
      const T jtn = jtx * nx + jty * ny + jtz * nz;
      const T dvn = (ZpP * jvn + jtn) / (ZpM + ZpP);
      const T ivs = T(1) / (ZsM + ZsP);
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
    T fl[kNF];
    fl[0] = dtx;
    fl[1] = dty;
    fl[2] = dtz;
    fl[3] = dvx * nx;
    fl[4] = dvy * ny;
    fl[5] = dvz * nz;
    fl[6] = T(0.5) * (dvy * nz + dvz * ny);
    fl[7] = T(0.5) * (dvx * nz + dvz * nx);
    fl[8] = T(0.5) * (dvx * ny + dvy * nx);
#pragma unroll
    for (int f = 0; f < kNF; ++f) sb[(f * E + e) * NF4 + j] = fs * fl[f];
  }
  __syncthreads();

  // D: lift
  for (int idx = threadIdx.x; idx < E * Np; idx += kBlock) {
    const int e = idx / Np, n = idx - e * Np;
    if (e >= ne) continue;
    T acc[kNF];
#pragma unroll
    for (int f = 0; f < kNF; ++f) acc[f] = sr[(f * E + e) * Np + n];
    for (int j = 0; j < NF4; ++j) {
      const T l = A.LIFTT[j * NpP + n];
#pragma unroll
      for (int f = 0; f < kNF; ++f) acc[f] += l * sb[(f * E + e) * NF4 + j];
    }
#pragma unroll
    for (int f = 0; f < kNF; ++f) sr[(f * E + e) * Np + n] = acc[f];
  }
  __syncthreads();

  // E: to quadrature points, weight by the material
  for (int idx = threadIdx.x; idx < E * Nq; idx += kBlock) {
    const int e = idx / Nq, qp = idx - e * Nq;
    if (e >= ne) continue;
    T v[kNF];
#pragma unroll
    for (int f = 0; f < kNF; ++f) v[f] = T(0);
    for (int n = 0; n < Np; ++n) {
      const T w = A.VqT[n * QP + qp];
#pragma unroll
      for (int f = 0; f < kNF; ++f) v[f] += w * sr[(f * E + e) * Np + n];
    }
    const int64_t mi = (e0 + e) * Nq + qp;
    const T ir = A.irho[mi], la = A.lam[mi], m2 = T(2) * A.mu[mi];
    const T tr = v[3] + v[4] + v[5];
    T o[kNF];
    o[0] = ir * v[0];
    o[1] = ir * v[1];
    o[2] = ir * v[2];
    o[3] = la * tr + m2 * v[3];
    o[4] = la * tr + m2 * v[4];
    o[5] = la * tr + m2 * v[5];
    o[6] = m2 * v[6];
    o[7] = m2 * v[7];
    o[8] = m2 * v[8];
#pragma unroll
    for (int f = 0; f < kNF; ++f) sb[(f * E + e) * Nq + qp] = o[f];
  }
  __syncthreads();

  // F: project back and store / update
  for (int idx = threadIdx.x; idx < E * Np; idx += kBlock) {
    const int e = idx / Np, n = idx - e * Np;
    if (e >= ne) continue;
    T acc[kNF];
#pragma unroll
    for (int f = 0; f < kNF; ++f) acc[f] = T(0);
    for (int qp = 0; qp < Nq; ++qp) {
      const T p = A.PqT[qp * NpP + n];
#pragma unroll
      for (int f = 0; f < kNF; ++f) acc[f] += p * sb[(f * E + e) * Nq + qp];
    }
    const int64_t base = (e0 + e) * Np + n;
    if (A.lsrk) {
#pragma unroll
      for (int f = 0; f < kNF; ++f) {
        const int64_t gi = f * KNp + base;
        const T rr = A.a * A.res[gi] + A.dt * acc[f];
        A.res[gi] = rr;
        A.q_out[gi] = sq[(f * E + e) * Np + n] + A.b * rr;
      }
    } else {
#pragma unroll
      for (int f = 0; f < kNF; ++f) A.rhs_out[f * KNp + base] = acc[f];
    }
  }
}

// fill kernel (used instead of hipMemsetAsync so that the calls stay
// graph-capturable)
template <typename T>
__global__ void fill_kernel(T* p, int64_t n, T v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace dgk
