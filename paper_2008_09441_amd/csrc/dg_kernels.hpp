// Small device utilities shared by the library (every stage runs on a
// matrix-core kernel: dg_bx.hpp, dg_be.hpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgk {

// fill kernel (used instead of hipMemsetAsync so that the calls stay
// graph-capturable)
template <typename T>
__global__ void fill_kernel(T* p, int64_t n, T v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace dgk
