// Batched stepping of many independent contexts of one order and precision
// (FP32 or FP32 + BF16x3 state) by one launch per stage: the serving path's
// continuous batching.  Every context is one slot of a table in device
// memory; a slot owns a range of launch positions and runs the same stage
// body as a single-context launch over its own tiles (orders 1-4) or
// elements (orders 5-7), so each context's result is bit-identical alone and
// in a batch.  Sources, receivers and the device clocks of all slots are
// handled by one launch each as well.
//
// Buffer parity: slot s keeps its two state buffers as q[0] (the current
// state when the batch call starts) and q[1].  Stage st of step i reads
// q[p] and writes q[1 - p] with p = (5 i + st) & 1, the same alternation a
// single context goes through.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dg_be.hpp"
#include "dg_bx.hpp"

namespace dgb {

struct BatchSlot {
  union {
    BxArgs bx;           // orders 1-4: q_in = q[0], q_out = q[1], lsrk, dt
    BeArgs be;           // orders 5-7
  } k;
  int64_t first;         // first launch position (a multiple of 8, so that
                         // position p of the slot runs on the XCD p & 7)
  int64_t nwg;           // launch positions: tiles (1-4) or elements (5-7)
  float* q[2];
  float* res;
  int64_t KNp;
  int Np;
  // point sources
  int nsrc;
  const int64_t* src_elem;
  const float* src_w;
  const double* src_par;
  // receivers and trace (rows indexed by the device clock's step count)
  int nrec;
  const int64_t* rec_elem;
  const float* rec_w;
  float* trace;
  int64_t trace_cap;
  // device clock (time, step count) and the context's time step
  double* clk;
  double dt;
};

// last slot whose first position is <= bid (slots sorted by first)
__device__ __forceinline__ int batch_slot(const BatchSlot* slots, int nslots, int64_t bid) {
  int lo = 0, hi = nslots - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (slots[mid].first <= bid) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int N, bool F32>
__global__ __launch_bounds__(kThreads, 2) void stage_bx_batch(const BatchSlot* slots, int nslots,
                                                              int par, float a, float b) {
  const int64_t bid = blockIdx.x;
  const int s = batch_slot(slots, nslots, bid);
  const int64_t p = bid - slots[s].first;
  if (p >= slots[s].nwg) return;   // positions padding a slot to a multiple of 8
  BxArgs A = slots[s].k.bx;
  A.q_in = slots[s].q[par];
  A.q_out = slots[s].q[1 - par];
  A.a = a;
  A.b = b;
  stage_bx_run<N, F32>(A, slots[s].nwg, p);
}

template <int N, bool F32>
__global__ __launch_bounds__(kThreads, 2) void stage_be_batch(const BatchSlot* slots, int nslots,
                                                              int par, float a, float b) {
  const int64_t bid = blockIdx.x;
  const int s = batch_slot(slots, nslots, bid);
  const int64_t p = bid - slots[s].first;
  if (p >= slots[s].nwg) return;
  BeArgs A = slots[s].k.be;
  A.q_in = slots[s].q[par];
  A.q_out = slots[s].q[1 - par];
  A.a = a;
  A.b = b;
  stage_be_run<N, F32>(A, slots[s].nwg, p);
}

// After stage st of step i (parity par): res += dt f(t) w and
// q_out += b_s dt f(t) w for every source of slot blockIdx.y, with
// t = clk[0] + frac dt, frac = i + c_s; one thread per (velocity component,
// node), each looping over its slot's sources (the single-context kernel's
// arithmetic, in the same order).
__global__ void source_add_batch(const BatchSlot* slots, int par, double frac, double bcoef) {
  const BatchSlot& S = slots[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (S.nsrc == 0 || i >= 3 * S.Np) return;
  const double t = S.clk[0] + frac * S.dt;
  const double alpha = S.dt, beta = bcoef * S.dt;
  float* out2 = S.q[1 - par];
  const int c = i / S.Np, n = i - c * S.Np;
  for (int s = 0; s < S.nsrc; ++s) {
    const double a = 3.14159265358979323846 * S.src_par[3 * s] * (t - S.src_par[3 * s + 1]);
    const double f = S.src_par[3 * s + 2] * (1.0 - 2.0 * a * a) * exp(-a * a);
    const int64_t idx = c * S.KNp + S.src_elem[s] * S.Np + n;
    const float v = float(f) * S.src_w[(s * 3 + c) * S.Np + n];
    S.res[idx] += float(alpha) * v;
    out2[idx] += float(beta) * v;
  }
}

// After step i, whose result is in q[par]: velocity at the receivers of slot
// blockIdx.y into trace row clk[1] + i (rows past the capacity are skipped)
__global__ void receiver_sample_batch(const BatchSlot* slots, int par, int64_t soff) {
  const BatchSlot& S = slots[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (S.nrec == 0 || S.trace_cap == 0 || i >= 3 * S.nrec) return;
  const int64_t row = int64_t(S.clk[1]) + soff;
  if (row < 0 || row >= S.trace_cap) return;
  const int r = i / 3, c = i - 3 * r;
  const float* qe = S.q[par] + c * S.KNp + S.rec_elem[r] * S.Np;
  const float* wr = S.rec_w + int64_t(r) * S.Np;
  float acc = 0.f;
  for (int n = 0; n < S.Np; ++n) acc += wr[n] * qe[n];
  S.trace[(row * S.nrec + r) * 3 + c] = acc;
}

// the device clocks of every slot advance by nsteps steps of their own dt
__global__ void clock_advance_batch(const BatchSlot* slots, int nslots, int64_t nsteps) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  double* clk = slots[s].clk;
  clk[1] += double(nsteps);
  clk[0] += double(nsteps) * slots[s].dt;
}

// The slot table is written by launches whose arguments carry it (no host
// staging buffer, ordered on the stream like the kernels that read it).
constexpr int kSlotWords = 960;   // 3,840 bytes of table per launch
struct SlotChunk {
  uint32_t w[kSlotWords];
};

__global__ void slot_write(uint32_t* dst, SlotChunk chunk, int nwords) {
  for (int i = threadIdx.x; i < nwords; i += blockDim.x) dst[i] = chunk.w[i];
}

}  // namespace dgb
