// Reference kernels for the rates the hardware reaches on this part, used
// beside the published peaks when rooflines are reported: a streaming copy
// (HBM bandwidth) and a loop of independent bf16 matrix-core products (the
// dense MFMA rate of v_mfma_f32_16x16x32_bf16, the instruction of the BF16x3
// stage kernels).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgp {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// dst[i] = src[i] over n 16-byte words, grid-stride, 16 bytes per lane and
// access (each wave moves whole 1 KiB lines)
__global__ __launch_bounds__(256) void copy16(const f32x4* __restrict__ src,
                                              f32x4* __restrict__ dst, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

// iters x 8 independent 16x16x32 bf16 products per wave (8 accumulator
// chains keep the matrix pipe busy); the sums are stored so that no product
// is dead code
__global__ __launch_bounds__(256) void mfma_loop(float* out, int iters) {
  bf16x8 a, b;
  for (int j = 0; j < 8; ++j) {
    a[j] = __bf16(float((threadIdx.x + j) & 7) * 0.125f);
    b[j] = __bf16(float((threadIdx.x * 3 + j) & 7) * 0.0625f);
  }
  f32x4 c[8];
  for (int j = 0; j < 8; ++j) c[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) c[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c[j], 0, 0, 0);
  }
  float s = 0.f;
  for (int j = 0; j < 8; ++j) s += c[j][0] + c[j][1] + c[j][2] + c[j][3];
  out[int64_t(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

}  // namespace dgp
