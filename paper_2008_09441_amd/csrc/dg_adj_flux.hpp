// Face-node flux of the DG elastic-wave stage and its derivatives, for the
// adjoint kernels (FP64 and FP32): the exact-Riemann upwind or central flux
// [WSG10], its transpose, and its sensitivity to the four impedances the
// face node reads.  Plain device functions, no kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace dga {

// forward flux (times Fscale) at one face node, fl[9]
template <typename T>
__device__ inline void flux(const T* qM, const T* qP, T nx, T ny, T nz, T fs, T ZpM, T ZsM,
                            T ZpP, T ZsP, int upwind, T* fl) {
  const T tMx = qM[3] * nx + qM[8] * ny + qM[7] * nz;
  const T tMy = qM[8] * nx + qM[4] * ny + qM[6] * nz;
  const T tMz = qM[7] * nx + qM[6] * ny + qM[5] * nz;
  const T tPx = qP[3] * nx + qP[8] * ny + qP[7] * nz;
  const T tPy = qP[8] * nx + qP[4] * ny + qP[6] * nz;
  const T tPz = qP[7] * nx + qP[6] * ny + qP[5] * nz;
  const T jvx = qP[0] - qM[0], jvy = qP[1] - qM[1], jvz = qP[2] - qM[2];
  const T jtx = tPx - tMx, jty = tPy - tMy, jtz = tPz - tMz;
  T dvx, dvy, dvz, dtx, dty, dtz;
  if (upwind) {
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
    dtx = ZpM * dvn * nx + ZsM * dvtx;
    dty = ZpM * dvn * ny + ZsM * dvty;
    dtz = ZpM * dvn * nz + ZsM * dvtz;
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

// reverse of flux(): the flux is linear in (qM, qP); given g = adjoint of
// fl, returns qMbar = (d fl / d qM)^T g and qPbar = (d fl / d qP)^T g
template <typename T>
__device__ inline void rev_flux(const T* g, T nx, T ny, T nz, T fs, T ZpM, T ZsM, T ZpP, T ZsP,
                                int upwind, T* qMb, T* qPb) {
  // fl -> (dv, dt)
  const T dtbx = fs * g[0], dtby = fs * g[1], dtbz = fs * g[2];
  const T dvbx = fs * (g[3] * nx + T(0.5) * (g[7] * nz + g[8] * ny));
  const T dvby = fs * (g[4] * ny + T(0.5) * (g[6] * nz + g[8] * nx));
  const T dvbz = fs * (g[5] * nz + T(0.5) * (g[6] * ny + g[7] * nx));
  T jvbx, jvby, jvbz, jtbx, jtby, jtbz;
  if (upwind) {
    // dv = dvn n + dvt;  dt = ZpM dvn n + ZsM dvt
    const T dvnb = dvbx * nx + dvby * ny + dvbz * nz + ZpM * (dtbx * nx + dtby * ny + dtbz * nz);
    const T dvtbx = dvbx + ZsM * dtbx, dvtby = dvby + ZsM * dtby, dvtbz = dvbz + ZsM * dtbz;
    // dvn = (ZpP jvn + jtn) / (ZpM + ZpP);  dvt = (ZsP jvt + jtt) / (ZsM + ZsP)
    const T ip = T(1) / (ZpM + ZpP), is = T(1) / (ZsM + ZsP);
    const T jvnb = ZpP * ip * dvnb, jtnb = ip * dvnb;
    const T jvtbx = ZsP * is * dvtbx, jvtby = ZsP * is * dvtby, jvtbz = ZsP * is * dvtbz;
    const T jttbx = is * dvtbx, jttby = is * dvtby, jttbz = is * dvtbz;
    // jvt = jv - (jv.n) n, jvn = jv.n: jvbar = jvtbar + (jvnbar - n.jvtbar) n
    const T av = jvnb - (jvtbx * nx + jvtby * ny + jvtbz * nz);
    const T at = jtnb - (jttbx * nx + jttby * ny + jttbz * nz);
    jvbx = jvtbx + av * nx; jvby = jvtby + av * ny; jvbz = jvtbz + av * nz;
    jtbx = jttbx + at * nx; jtby = jttby + at * ny; jtbz = jttbz + at * nz;
  } else {
    jvbx = T(0.5) * dvbx; jvby = T(0.5) * dvby; jvbz = T(0.5) * dvbz;
    jtbx = T(0.5) * dtbx; jtby = T(0.5) * dtby; jtbz = T(0.5) * dtbz;
  }
  // jv = vP - vM; jt = t(P) - t(M), t = sigma n (Voigt xx yy zz yz xz xy)
  const T s[9] = {jvbx, jvby, jvbz, jtbx * nx, jtby * ny, jtbz * nz,
                  jtby * nz + jtbz * ny, jtbx * nz + jtbz * nx, jtbx * ny + jtby * nx};
  for (int f = 0; f < 9; ++f) {
    qPb[f] = s[f];
    qMb[f] = -s[f];
  }
}

// Impedance sensitivity of the upwind flux, pass 1: at every face node i,
// the derivatives of phi_i = g_i . fl_i (g = LIFT^T mu at the face node, fl
// the Fscale-scaled flux of the state y) with respect to the four
// impedances the node reads, zb[i * 4 + {0, 1, 2, 3}] = d phi / d(ZpM, ZsM,
// ZpP, ZsP).  Writing dv = dvn n + dvt and dt = ZpM dvn n + ZsM dvt,
//   phi = dvn alpha + dvt . beta,  alpha = ZpM (h . n) + k . n,
//   beta = ZsM h + k,
// with h = fs g_{0..2} (traction rows) and k = fs S n, S the symmetric
// tensor of the stress rows (off-diagonals halved), so that
//   d/dZpM = dvn (h . n) - alpha dvn / (ZpM + ZpP),
//   d/dZpP = alpha (jvn - dvn) / (ZpM + ZpP),
//   d/dZsM = dvt . h - (beta . dvt) / (ZsM + ZsP),
//   d/dZsP = beta . (jvt - dvt) / (ZsM + ZsP).
// zgrad_terms gives these four for one face node from its two states,
// normal, Fscale, impedances and g; zgrad_faces applies it at every face
// node.
// the velocity jump jv = vP - vM and traction jump jt = t(P) - t(M) of a
// face node (t = sigma n, Voigt xx yy zz yz xz xy), j[0..5] = (jv, jt)
template <typename T>
__device__ inline void face_jumps(const T* qM, const T* qP, T nx, T ny, T nz, T* j) {
  j[0] = qP[0] - qM[0];
  j[1] = qP[1] - qM[1];
  j[2] = qP[2] - qM[2];
  j[3] = (qP[3] - qM[3]) * nx + (qP[8] - qM[8]) * ny + (qP[7] - qM[7]) * nz;
  j[4] = (qP[8] - qM[8]) * nx + (qP[4] - qM[4]) * ny + (qP[6] - qM[6]) * nz;
  j[5] = (qP[7] - qM[7]) * nx + (qP[6] - qM[6]) * ny + (qP[5] - qM[5]) * nz;
}

// the same four derivatives from the face node's jumps (face_jumps)
template <typename T>
__device__ inline void zgrad_from_jumps(const T* jmp, T nx, T ny, T nz, T fs, T ZpM, T ZsM,
                                        T ZpP, T ZsP, const T* g, T* z) {
  const T jvx = jmp[0], jvy = jmp[1], jvz = jmp[2];
  const T jtx = jmp[3], jty = jmp[4], jtz = jmp[5];
  const T jvn = jvx * nx + jvy * ny + jvz * nz;
  const T jtn = jtx * nx + jty * ny + jtz * nz;
  const T sp = ZpM + ZpP, ss = ZsM + ZsP;
  const T dvn = (ZpP * jvn + jtn) / sp;
  const T jvtx = jvx - jvn * nx, jvty = jvy - jvn * ny, jvtz = jvz - jvn * nz;
  const T dvtx = (ZsP * jvtx + (jtx - jtn * nx)) / ss;
  const T dvty = (ZsP * jvty + (jty - jtn * ny)) / ss;
  const T dvtz = (ZsP * jvtz + (jtz - jtn * nz)) / ss;
  const T hx = fs * g[0], hy = fs * g[1], hz = fs * g[2];
  const T kx = fs * (g[3] * nx + T(0.5) * (g[8] * ny + g[7] * nz));
  const T ky = fs * (T(0.5) * g[8] * nx + g[4] * ny + T(0.5) * g[6] * nz);
  const T kz = fs * (T(0.5) * (g[7] * nx + g[6] * ny) + g[5] * nz);
  const T hn = hx * nx + hy * ny + hz * nz;
  const T alpha = ZpM * hn + (kx * nx + ky * ny + kz * nz);
  const T bx = ZsM * hx + kx, by = ZsM * hy + ky, bz = ZsM * hz + kz;
  const T bdvt = bx * dvtx + by * dvty + bz * dvtz;
  z[0] = dvn * hn - alpha * dvn / sp;
  z[1] = (dvtx * hx + dvty * hy + dvtz * hz) - bdvt / ss;
  z[2] = alpha * (jvn - dvn) / sp;
  z[3] = (bx * (jvtx - dvtx) + by * (jvty - dvty) + bz * (jvtz - dvtz)) / ss;
}

template <typename T>
__device__ inline void zgrad_terms(const T* qM, const T* qP, T nx, T ny, T nz, T fs, T ZpM,
                                   T ZsM, T ZpP, T ZsP, const T* g, T* z) {
  T jmp[6];
  face_jumps(qM, qP, nx, ny, nz, jmp);
  zgrad_from_jumps(jmp, nx, ny, nz, fs, ZpM, ZsM, ZpP, ZsP, g, z);
}

}  // namespace dga
