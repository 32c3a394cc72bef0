// Device kernels for point sources and receivers of the DG elastic-wave
// solver (all precisions).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgs {

// source_add: after a stage kernel, add the point-force contribution of every
// source, f_s(t) w_s, where w_s[3][Np] is the source's velocity-row response
// after the weight-adjusted mass inverse (precomputed on the host) and
// f_s(t) = A (1 - 2 a^2) exp(-a^2), a = pi f0 (t - t0), the Ricker wavelet:
//   out1 += alpha f w,  out2 += beta f w (out2 may be null).
// For a stage of LSRK(5,4), out1 = res (alpha = dt) and out2 = q_out
// (beta = b_s dt): res = a res + dt (rhs + f w) and q_out = q_in + b_s res
// are both linear in the added term.  One thread per (velocity component,
// node); each thread loops over the sources, so sources sharing an element
// never race.
template <typename T>
__global__ void source_add(T* out1, T* out2, const int64_t* elem, const T* w,
                           const double* par, int nsrc, int Np, int64_t KNp, double t,
                           double alpha, double beta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * Np) return;
  const int c = i / Np, n = i - c * Np;
  for (int s = 0; s < nsrc; ++s) {
    const double a = 3.14159265358979323846 * par[3 * s] * (t - par[3 * s + 1]);
    const double f = par[3 * s + 2] * (1.0 - 2.0 * a * a) * exp(-a * a);
    const int64_t idx = c * KNp + elem[s] * Np + n;
    const T v = T(f) * w[(s * 3 + c) * Np + n];
    out1[idx] += T(alpha) * v;
    if (out2) out2[idx] += T(beta) * v;
  }
}

// receiver_sample: velocity at each receiver, out[r][c] = w_r . q[c][k_r][:],
// one thread per (receiver, component)
template <typename T>
__global__ void receiver_sample(T* out, const T* q, const int64_t* elem, const T* w, int nrec,
                                int Np, int64_t KNp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * nrec) return;
  const int r = i / 3, c = i - 3 * r;
  const T* qe = q + c * KNp + elem[r] * Np;
  const T* wr = w + int64_t(r) * Np;
  T acc = T(0);
  for (int n = 0; n < Np; ++n) acc += wr[n] * qe[n];
  out[i] = acc;
}

}  // namespace dgs

namespace dgs {

// Device-resident clock of a context: clk[0] = time (double), clk[1] = step
// count (stored as a double holding an exact integer, < 2^53).  Launches that
// read it have arguments independent of the time, so a captured graph of a
// run can be replayed at any time.
__global__ void clock_set(double* clk, double t) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    clk[0] = t;
    clk[1] = 0.0;
  }
}

__global__ void clock_advance(double* clk, double dt, int64_t nsteps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    // t0 + n dt from the step count, not a running sum (no drift)
    clk[1] += double(nsteps);
    clk[0] += double(nsteps) * dt;
  }
}

// source_add with the time read from the clock: t = clk[0] + toff
template <typename T>
__global__ void source_add_clk(T* out1, T* out2, const int64_t* elem, const T* w,
                               const double* par, int nsrc, int Np, int64_t KNp,
                               const double* clk, double toff, double alpha, double beta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * Np) return;
  const double t = clk[0] + toff;
  const int c = i / Np, n = i - c * Np;
  for (int s = 0; s < nsrc; ++s) {
    const double a = 3.14159265358979323846 * par[3 * s] * (t - par[3 * s + 1]);
    const double f = par[3 * s + 2] * (1.0 - 2.0 * a * a) * exp(-a * a);
    const int64_t idx = c * KNp + elem[s] * Np + n;
    const T v = T(f) * w[(s * 3 + c) * Np + n];
    out1[idx] += T(alpha) * v;
    if (out2) out2[idx] += T(beta) * v;
  }
}

// receiver_sample into row (clk[1] + soff) of a trace with cap rows; rows
// beyond the capacity are not written
template <typename T>
__global__ void receiver_sample_clk(T* trace, int64_t cap, const double* clk, int64_t soff,
                                    const T* q, const int64_t* elem, const T* w, int nrec,
                                    int Np, int64_t KNp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * nrec) return;
  const int64_t row = int64_t(clk[1]) + soff;
  if (row < 0 || row >= cap) return;
  const int r = i / 3, c = i - 3 * r;
  const T* qe = q + c * KNp + elem[r] * Np;
  const T* wr = w + int64_t(r) * Np;
  T acc = T(0);
  for (int n = 0; n < Np; ++n) acc += wr[n] * qe[n];
  trace[(row * nrec + r) * 3 + c] = acc;
}

}  // namespace dgs
