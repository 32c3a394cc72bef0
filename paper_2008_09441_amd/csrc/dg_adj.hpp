// Device kernels of the discrete adjoint of the DG elastic-wave stage (FP64
// and FP32): the raw right-hand side R q (volume terms, face fluxes, LIFT,
// before the mass inverse), the transposes W^T and R^T, the gradient with
// respect to the weight-adjusted material weights, the receiver adjoint and
// vector updates, over runtime sizes; the adjoint sweep calls them a few
// times per stage.  The per-element kernels run one workgroup of kAdjThreads
// per element and stage the element's vectors in LDS (dynamic shared memory),
// so that their inner loops read LDS broadcasts and operator rows that
// consecutive threads read at consecutive addresses.
//
// Transposes, per element (W(m) r = P_q[weights . V_q r], [CHW17, C18]):
//   (W^T l)_v = V_q^T (1/rho) P_q^T l_v,
//   (W^T l)_s = V_q^T [lam tr(P_q^T l_s) I + 2 mu P_q^T l_s];
// R = volume + LIFT Fscale flux(q-, q+) [HW08, Ch. 10], [WSG10]:
//   R^T mu = volume^T mu + per face node: (d flux / d q-)^T g at the own node
//            plus (d flux_nb / d q+)^T g_nb from the neighbour's face node
//            that reads this node, with g = Fscale LIFT^T mu at face nodes.
// The flux transpose is the reverse-mode derivative of the flux formula
// written out step by step (rev_flux in dg_adj_flux.hpp).  With the upwind
// flux the operator also depends on the impedances Zp, Zs at the nodes;
// their sensitivity d/dZ <mu, R(Z) y> is differentiated by hand per face
// node (zgrad_terms, applied by zgrad_faces) and gathered onto the nodes
// (zgrad_nodes).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dg_adj_flux.hpp"

namespace dga {

template <typename T>
struct AdjArgs {
  const T* geo;          // [K][9]
  const T* fgeo;         // [K][4][4]
  const int32_t* etoe;   // [K][4]
  const uint8_t* etop;   // [K][4]
  const int32_t* pat;    // [npat][Nfp]
  const int32_t* fmask;  // [4][Nfp]
  const int32_t* nbface; // [K][4 Nfp]: neighbour element * 4 Nfp + its face node
  const int32_t* invf;   // [Np][3]: face nodes on each volume node (-1 padded)
  const T* zp;           // [K][Np]
  const T* zs;
  const T* Dr;           // [Np][Np]
  const T* Ds;
  const T* Dt;
  const T* LIFT;         // [Np][4 Nfp]
  const T* Vq;           // [Nq][Np]
  const T* Pq;           // [Np][Nq]
  // transposes (zero padded): DrT | DsT | DtT [Np][NpP], LIFTT [4 Nfp][NpP],
  // VqT [Np][QP], so that threads over output rows read consecutive entries
  const T* DrT;
  const T* DsT;
  const T* DtT;
  const T* LIFTT;
  const T* VqT;
  int NpP, QP;
  const T* irho;         // [K][Nq]
  const T* lam;
  const T* mu;
  int64_t K;
  int Np, Nfp, Nq;
  int upwind;
};

// output component c of the volume term: sum_d D_d sum_j G_dj w(c,j) q_f(c,j)
// (the stress row of c for the velocity components, the symmetrised
// velocity pattern for the strain components)
__device__ inline int vf(int c, int j) {
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
template <typename T>
__device__ inline T vw(int c, int j) {
  if (c < 3) return T(1);
  if (c < 6) return j == c - 3 ? T(1) : T(0);
  return j == c - 6 ? T(0) : T(0.5);
}

constexpr int kAdjThreads = 128;   // threads of the per-element kernels

template <typename T>
__device__ inline T* adj_lds() {
  extern __shared__ __align__(16) unsigned char adj_smem[];
  return reinterpret_cast<T*>(adj_smem);
}

// raw right-hand side r = R q of element blockIdx.x (volume terms plus LIFT of
// the Fscale fluxes), r[9][K][Np].  LDS: q of the element [9][Np], fluxes
// [4 Nfp][9] (raw_lds_elems values).
__host__ __device__ inline int raw_lds_elems(int Np, int Nfp) { return 9 * Np + 36 * Nfp; }

template <typename T>
__global__ __launch_bounds__(kAdjThreads) void raw_rhs(AdjArgs<T> A, const T* q, T* r) {
  const int Np = A.Np, Nfp = A.Nfp, NF4 = 4 * Nfp;
  const int64_t k = blockIdx.x, KNp = A.K * Np;
  T* sq = adj_lds<T>();
  T* sfl = sq + 9 * Np;
  for (int i = threadIdx.x; i < 9 * Np; i += blockDim.x) {
    const int f = i / Np, n = i - f * Np;
    sq[i] = q[f * KNp + k * Np + n];
  }
  __syncthreads();
  for (int j = threadIdx.x; j < NF4; j += blockDim.x) {
    const int face = j / Nfp, ii = j - face * Nfp;
    const int vM = A.fmask[j];
    const int64_t nb = A.etoe[k * 4 + face];
    const int vP = A.pat[int(A.etop[k * 4 + face]) * Nfp + ii];
    T qM[9], qP[9];
    for (int f = 0; f < 9; ++f) {
      qM[f] = sq[f * Np + vM];
      qP[f] = q[f * KNp + nb * Np + vP];
    }
    const T* fg = A.fgeo + (k * 4 + face) * 4;
    flux(qM, qP, fg[0], fg[1], fg[2], fg[3], A.zp[k * Np + vM], A.zs[k * Np + vM],
         A.zp[nb * Np + vP], A.zs[nb * Np + vP], A.upwind, sfl + j * 9);
  }
  __syncthreads();
  const T* G = A.geo + k * 9;
  for (int n = threadIdx.x; n < Np; n += blockDim.x) {
    T dq[3][9];
    for (int d = 0; d < 3; ++d)
      for (int f = 0; f < 9; ++f) dq[d][f] = T(0);
#pragma unroll 4
    for (int m = 0; m < Np; ++m) {
      const int64_t o = int64_t(m) * A.NpP + n;
      const T dr = A.DrT[o], ds = A.DsT[o], dt = A.DtT[o];
      for (int f = 0; f < 9; ++f) {
        const T v = sq[f * Np + m];
        dq[0][f] += dr * v;
        dq[1][f] += ds * v;
        dq[2][f] += dt * v;
      }
    }
    T out[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const T w = vw<T>(c, j);
        if (w == T(0)) continue;
        const int f = vf(c, j);
        for (int d = 0; d < 3; ++d) acc += w * G[d * 3 + j] * dq[d][f];
      }
      out[c] = acc;
    }
#pragma unroll 4
    for (int j = 0; j < NF4; ++j) {
      const T l = A.LIFTT[int64_t(j) * A.NpP + n];
      for (int c = 0; c < 9; ++c) out[c] += l * sfl[j * 9 + c];
    }
    for (int c = 0; c < 9; ++c) r[c * KNp + k * Np + n] = out[c];
  }
}

// For element blockIdx.x, with p = P_q^T l and w = V_q r at each quadrature
// point: the gradient grad[3][K][Nq] += s d/dm <l, W(m) r>, and the
// transpose out = W^T l = V_q^T [weights . p] (1/rho on the velocity rows,
// lam tr + 2 mu on the normal stresses, 2 mu on the shear stresses),
// out[9][K][Np].  LDS: l and r of the element [2][9][Np], weighted p
// [Nq][9] (gradw_lds_elems values).
__host__ __device__ inline int gradw_lds_elems(int Np, int Nq) { return 18 * Np + 9 * Nq; }

template <typename T>
__global__ __launch_bounds__(kAdjThreads) void grad_wadgT(AdjArgs<T> A, const T* l, const T* r, double* grad, double s,
                           T* out) {
  const int Np = A.Np, Nq = A.Nq;
  const int64_t k = blockIdx.x, KNp = A.K * Np, KNq = A.K * Nq;
  T* sl = adj_lds<T>();
  T* sr = sl + 9 * Np;
  T* sob = sr + 9 * Np;
  for (int i = threadIdx.x; i < 9 * Np; i += blockDim.x) {
    const int f = i / Np, n = i - f * Np;
    sl[i] = l[f * KNp + k * Np + n];
    sr[i] = r[f * KNp + k * Np + n];
  }
  __syncthreads();
  for (int qp = threadIdx.x; qp < Nq; qp += blockDim.x) {
    T p[9], w[9];
    for (int f = 0; f < 9; ++f) p[f] = w[f] = T(0);
#pragma unroll 4
    for (int n = 0; n < Np; ++n) {
      const T pq = A.Pq[n * Nq + qp], vq = A.VqT[int64_t(n) * A.QP + qp];
      for (int f = 0; f < 9; ++f) {
        p[f] += pq * sl[f * Np + n];
        w[f] += vq * sr[f * Np + n];
      }
    }
    double g0 = 0.0, g2 = 0.0;
    for (int f = 0; f < 3; ++f) g0 += double(p[f]) * double(w[f]);
    for (int f = 3; f < 9; ++f) g2 += double(p[f]) * double(w[f]);
    const double g1 = (double(p[3]) + double(p[4]) + double(p[5])) *
                      (double(w[3]) + double(w[4]) + double(w[5]));
    const int64_t i = k * Nq + qp;
    grad[i] += s * g0;
    grad[KNq + i] += s * g1;
    grad[2 * KNq + i] += s * 2.0 * g2;
    const T ir = A.irho[i], la = A.lam[i], m2 = T(2) * A.mu[i];
    const T tr = p[3] + p[4] + p[5];
    for (int f = 0; f < 3; ++f) sob[qp * 9 + f] = ir * p[f];
    for (int f = 3; f < 6; ++f) sob[qp * 9 + f] = la * tr + m2 * p[f];
    for (int f = 6; f < 9; ++f) sob[qp * 9 + f] = m2 * p[f];
  }
  __syncthreads();
  for (int n = threadIdx.x; n < Np; n += blockDim.x) {
    T acc[9];
    for (int f = 0; f < 9; ++f) acc[f] = T(0);
#pragma unroll 4
    for (int qp = 0; qp < Nq; ++qp) {
      const T w = A.Vq[qp * Np + n];
      for (int f = 0; f < 9; ++f) acc[f] += w * sob[qp * 9 + f];
    }
    for (int f = 0; f < 9; ++f) out[f * KNp + k * Np + n] = acc[f];
  }
}

// R^T, pass 1: g = LIFT^T mu at every face node of element blockIdx.x,
// gb[(k * NF4 + j) * 9 + f].  LDS: mu of the element [9][Np].
template <typename T>
__global__ __launch_bounds__(kAdjThreads) void liftT_faces(AdjArgs<T> A, const T* mu, T* gb) {
  const int Np = A.Np, NF4 = 4 * A.Nfp;
  const int64_t k = blockIdx.x, KNp = A.K * Np;
  T* sm = adj_lds<T>();
  for (int i = threadIdx.x; i < 9 * Np; i += blockDim.x) {
    const int f = i / Np, n = i - f * Np;
    sm[i] = mu[f * KNp + k * Np + n];
  }
  __syncthreads();
  for (int j = threadIdx.x; j < NF4; j += blockDim.x) {
    T acc[9];
    for (int f = 0; f < 9; ++f) acc[f] = T(0);
#pragma unroll 4
    for (int n = 0; n < Np; ++n) {
      const T l = A.LIFT[n * NF4 + j];
      for (int f = 0; f < 9; ++f) acc[f] += l * sm[f * Np + n];
    }
    for (int f = 0; f < 9; ++f) gb[(k * NF4 + j) * 9 + f] = acc[f];
  }
}

// R^T, pass 2: at every face node, own-side flux transpose plus the
// neighbour's other-side flux transpose, hb[(k * NF4 + j) * 9 + f]
template <typename T>
__global__ void fluxT_faces(AdjArgs<T> A, const T* gb, T* hb) {
  const int Np = A.Np, Nfp = A.Nfp, NF4 = 4 * Nfp;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= A.K * NF4) return;
  const int64_t k = i / NF4;
  const int j = int(i - k * NF4), face = j / Nfp, ii = j - face * Nfp;
  const int vM = A.fmask[j];
  const int64_t nb = A.etoe[k * 4 + face];
  const int vP = A.pat[int(A.etop[k * 4 + face]) * Nfp + ii];
  const int64_t jn = A.nbface[i];                // neighbour's face node (flat)
  const int fn = int(jn - nb * NF4) / Nfp;       // neighbour's face
  const T ZpM = A.zp[k * Np + vM], ZsM = A.zs[k * Np + vM];
  const T ZpP = A.zp[nb * Np + vP], ZsP = A.zs[nb * Np + vP];
  T a[9], b[9], h[9];
  const T* fg = A.fgeo + (k * 4 + face) * 4;
  rev_flux(gb + i * 9, fg[0], fg[1], fg[2], fg[3], ZpM, ZsM, ZpP, ZsP, A.upwind, a, b);
  for (int f = 0; f < 9; ++f) h[f] = a[f];
  // the neighbour's flux at its face node jn reads this node as its "+" side
  const T* fn4 = A.fgeo + (nb * 4 + fn) * 4;
  rev_flux(gb + jn * 9, fn4[0], fn4[1], fn4[2], fn4[3], ZpP, ZsP, ZpM, ZsM, A.upwind, a, b);
  for (int f = 0; f < 9; ++f) h[f] += b[f];
  for (int f = 0; f < 9; ++f) hb[i * 9 + f] = h[f];
}

// R^T, pass 3: volume transpose plus the face contributions gathered onto
// the volume nodes of element blockIdx.x, out[9][K][Np] (= R^T mu).  LDS: mu
// of the element [9][Np].
template <typename T>
__global__ __launch_bounds__(kAdjThreads) void volT_nodes(AdjArgs<T> A, const T* mu, const T* hb, T* out) {
  const int Np = A.Np, NF4 = 4 * A.Nfp;
  const int64_t k = blockIdx.x, KNp = A.K * Np;
  T* sm = adj_lds<T>();
  for (int i = threadIdx.x; i < 9 * Np; i += blockDim.x) {
    const int f = i / Np, n = i - f * Np;
    sm[i] = mu[f * KNp + k * Np + n];
  }
  __syncthreads();
  const T* G = A.geo + k * 9;
  for (int n = threadIdx.x; n < Np; n += blockDim.x) {
    // t[d][c] = (D_d^T mu_c)_n
    T t[3][9];
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 9; ++c) t[d][c] = T(0);
#pragma unroll 4
    for (int m = 0; m < Np; ++m) {
      const T dr = A.Dr[m * Np + n], ds = A.Ds[m * Np + n], dt = A.Dt[m * Np + n];
      for (int c = 0; c < 9; ++c) {
        const T v = sm[c * Np + m];
        t[0][c] += dr * v;
        t[1][c] += ds * v;
        t[2][c] += dt * v;
      }
    }
    T acc[9];
    for (int f = 0; f < 9; ++f) acc[f] = T(0);
#pragma unroll
    for (int c = 0; c < 9; ++c)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const T w = vw<T>(c, j);
        if (w == T(0)) continue;
        const int f = vf(c, j);
        for (int d = 0; d < 3; ++d) acc[f] += w * G[d * 3 + j] * t[d][c];
      }
    for (int s = 0; s < 3; ++s) {
      const int jf = A.invf[n * 3 + s];
      if (jf < 0) continue;
      for (int f = 0; f < 9; ++f) acc[f] += hb[(k * NF4 + jf) * 9 + f];
    }
    for (int f = 0; f < 9; ++f) out[f * KNp + k * Np + n] = acc[f];
  }
}

// Impedance sensitivity of the upwind flux, pass 1: zb[i * 4 + {0, 1, 2, 3}]
// = d phi_i / d(ZpM, ZsM, ZpP, ZsP) at every face node i (zgrad_terms).
template <typename T>
__global__ void zgrad_faces(AdjArgs<T> A, const T* y, const T* gb, T* zb) {
  const int Np = A.Np, Nfp = A.Nfp, NF4 = 4 * Nfp;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= A.K * NF4) return;
  const int64_t k = i / NF4, KNp = A.K * Np;
  const int j = int(i - k * NF4), face = j / Nfp, ii = j - face * Nfp;
  const int vM = A.fmask[j];
  const int64_t nb = A.etoe[k * 4 + face];
  const int vP = A.pat[int(A.etop[k * 4 + face]) * Nfp + ii];
  T qM[9], qP[9];
  for (int f = 0; f < 9; ++f) {
    qM[f] = y[f * KNp + k * Np + vM];
    qP[f] = y[f * KNp + nb * Np + vP];
  }
  const T* fg = A.fgeo + (k * 4 + face) * 4;
  zgrad_terms(qM, qP, fg[0], fg[1], fg[2], fg[3], A.zp[k * Np + vM], A.zs[k * Np + vM],
              A.zp[nb * Np + vP], A.zs[nb * Np + vP], gb + i * 9, zb + i * 4);
}

// Impedance sensitivity, pass 2: onto every volume node n of element k,
// gradz[{0: Zp, 1: Zs}][k][n] += s * (the own-side terms of the face nodes
// on n, plus the neighbour-side terms of the neighbours' face nodes that
// read n); one thread per (element, node)
template <typename T>
__global__ void zgrad_nodes(AdjArgs<T> A, const T* zb, double* gradz, double s) {
  const int Np = A.Np, NF4 = 4 * A.Nfp;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= A.K * Np) return;
  const int64_t k = i / Np;
  const int n = int(i - k * Np);
  double gp = 0.0, gs = 0.0;
  for (int t = 0; t < 3; ++t) {
    const int jf = A.invf[n * 3 + t];
    if (jf < 0) continue;
    const int64_t own = k * NF4 + jf, nbj = A.nbface[own];
    gp += double(zb[own * 4 + 0]) + double(zb[nbj * 4 + 2]);
    gs += double(zb[own * 4 + 1]) + double(zb[nbj * 4 + 3]);
  }
  gradz[i] += s * gp;
  gradz[A.K * Np + i] += s * gs;
}

// receiver adjoint: l[c][k_r][n] += w_r[n] resid[r][c] for every receiver;
// one thread per (component, node), looping over the receivers
template <typename T>
__global__ void receiver_adjoint(T* l, const T* resid, const int64_t* elem, const T* w,
                                 int nrec, int Np, int64_t KNp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * Np) return;
  const int c = i / Np, n = i - c * Np;
  for (int r = 0; r < nrec; ++r)
    l[c * KNp + elem[r] * Np + n] += w[int64_t(r) * Np + n] * resid[r * 3 + c];
}

// y = a x + b y
template <typename T>
__global__ void axpby(T* y, const T* x, double a, double b, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = T(a) * x[i] + T(b) * y[i];
}

}  // namespace dga
