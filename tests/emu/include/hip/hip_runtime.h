// Host stand-in for the HIP device environment, used only to run the stage
// kernels on the CPU in tests (threads, barriers, matrix-core emulation).
#pragma once
#include <barrier>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
struct emu_dim3 { unsigned x = 0, y = 0, z = 0; };
extern thread_local emu_dim3 threadIdx, blockIdx;
extern emu_dim3 gridDim, blockDim;
void __syncthreads();
typedef __bf16 emu_bf16x8 __attribute__((ext_vector_type(8)));
typedef float emu_f32x4 __attribute__((ext_vector_type(4)));
emu_f32x4 emu_mfma_16x16x32_bf16(emu_bf16x8 a, emu_bf16x8 b, emu_f32x4 c, int, int, int);
#define __builtin_amdgcn_mfma_f32_16x16x32_bf16 emu_mfma_16x16x32_bf16
emu_f32x4 emu_mfma_16x16x4_f32(float a, float b, emu_f32x4 c, int, int, int);
#define __builtin_amdgcn_mfma_f32_16x16x4f32 emu_mfma_16x16x4_f32
typedef double emu_f64x4 __attribute__((ext_vector_type(4)));
emu_f64x4 emu_mfma_16x16x4_f64(double a, double b, emu_f64x4 c, int, int, int);
#define __builtin_amdgcn_mfma_f64_16x16x4f64 emu_mfma_16x16x4_f64
#define __align__(n) __attribute__((aligned(n)))
#define __builtin_amdgcn_readfirstlane(x) (x)
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
// lane count builtins: number of lanes below this one in the mask (low/high half)
inline unsigned emu_mbcnt_lo(unsigned m, unsigned a) {
  const unsigned l = threadIdx.x & 63;
  return a + __builtin_popcount(l >= 32 ? m : (m & ((1u << l) - 1u)));
}
inline unsigned emu_mbcnt_hi(unsigned m, unsigned a) {
  const unsigned l = threadIdx.x & 63;
  return a + (l < 32 ? 0u : __builtin_popcount(m & ((1u << (l - 32)) - 1u)));
}
#define __builtin_amdgcn_mbcnt_lo emu_mbcnt_lo
#define __builtin_amdgcn_mbcnt_hi emu_mbcnt_hi
inline int min(int a, int b) { return a < b ? a : b; }
inline long min(long a, long b) { return a < b ? a : b; }
inline unsigned min(unsigned a, unsigned b) { return a < b ? a : b; }
#define __builtin_amdgcn_rcpf(x) (1.f / (x))
float emu_shfl(float v, int src, int width);
double emu_shfl_d(double v, int src, int width);
inline float __shfl(float v, int src, int width = 64) { return emu_shfl(v, src, width); }
inline double __shfl(double v, int src, int width = 64) { return emu_shfl_d(v, src, width); }
