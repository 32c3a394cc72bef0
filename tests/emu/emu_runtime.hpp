// Host runtime of the kernel emulators: host threads as the lanes of a
// workgroup with real barriers, and the matrix-core products and lane
// shuffles emulated in their hardware lane layouts (A: row lane%16, k
// lane/16 (bf16: k 8(lane/16)+j); B: column lane%16, same k; D: column
// lane%16, row 4(lane/16)+j for f32 and bf16, 4j+lane/16 for f64).
// Included once per emulator executable.
#pragma once
#include <hip/hip_runtime.h>
#include <barrier>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

thread_local emu_dim3 threadIdx, blockIdx;
emu_dim3 gridDim, blockDim;
static std::unique_ptr<std::barrier<>> g_bar;
static std::unique_ptr<std::barrier<>> g_wbar[4];
struct Slot { emu_bf16x8 a[64], b[64]; float x[64], fa[64], fb[64]; double da[64], db[64], xd[64]; };
static Slot g_slot[4];

void __syncthreads() { g_bar->arrive_and_wait(); }

emu_f32x4 emu_mfma_16x16x32_bf16(emu_bf16x8 a, emu_bf16x8 b, emu_f32x4 c, int, int, int) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  g_slot[w].a[lane] = a;
  g_slot[w].b[lane] = b;
  g_wbar[w]->arrive_and_wait();
  emu_f32x4 d = c;
  const int n = lane % 16;
  for (int j = 0; j < 4; ++j) {
    const int i = 4 * (lane / 16) + j;
    float acc = c[j];
    for (int k = 0; k < 32; ++k) {
      const float av = (float)g_slot[w].a[i + 16 * (k / 8)][k % 8];
      const float bv = (float)g_slot[w].b[n + 16 * (k / 8)][k % 8];
      acc += av * bv;
    }
    d[j] = acc;
  }
  g_wbar[w]->arrive_and_wait();
  return d;
}

// lane shuffle: every lane of the wave publishes its value, then reads lane src's
float emu_shfl(float v, int src, int) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  g_slot[w].x[lane] = v;
  g_wbar[w]->arrive_and_wait();
  const float r = g_slot[w].x[src & 63];
  g_wbar[w]->arrive_and_wait();
  return r;
}

double emu_shfl_d(double v, int src, int) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  g_slot[w].xd[lane] = v;
  g_wbar[w]->arrive_and_wait();
  const double r = g_slot[w].xd[src & 63];
  g_wbar[w]->arrive_and_wait();
  return r;
}

// FP32 MFMA 16x16x4: A lane l holds row l % 16, k = l / 16; B lane l holds
// column l % 16, k = l / 16; D as for the bf16 form
emu_f32x4 emu_mfma_16x16x4_f32(float a, float b, emu_f32x4 c, int, int, int) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  g_slot[w].fa[lane] = a;
  g_slot[w].fb[lane] = b;
  g_wbar[w]->arrive_and_wait();
  emu_f32x4 d = c;
  const int n = lane % 16;
  for (int j = 0; j < 4; ++j) {
    const int i = 4 * (lane / 16) + j;
    float acc = c[j];
    for (int k = 0; k < 4; ++k) acc += g_slot[w].fa[i + 16 * k] * g_slot[w].fb[n + 16 * k];
    d[j] = acc;
  }
  g_wbar[w]->arrive_and_wait();
  return d;
}

// the 16x16x4 f64 product (A: row lane%16, k lane/16; B: column lane%16, k
// lane/16; D: column lane%16, row 4 j + lane/16 -- the interleaved row order
// measured on gfx950, unlike the f32 product's 4 (lane/16) + j)
emu_f64x4 emu_mfma_16x16x4_f64(double a, double b, emu_f64x4 c, int, int, int) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  g_slot[w].da[lane] = a;
  g_slot[w].db[lane] = b;
  g_wbar[w]->arrive_and_wait();
  emu_f64x4 d = c;
  const int n = lane % 16;
  for (int j = 0; j < 4; ++j) {
    const int i = 4 * j + lane / 16;
    double acc = c[j];
    for (int k = 0; k < 4; ++k) acc += g_slot[w].da[i + 16 * k] * g_slot[w].db[n + 16 * k];
    d[j] = acc;
  }
  g_wbar[w]->arrive_and_wait();
  return d;
}

template <typename F>
static void run_grid(int grid, F kern) {
  gridDim.x = grid; blockDim.x = 256;
  for (int b = 0; b < grid; ++b) {
    g_bar = std::make_unique<std::barrier<>>(256);
    for (int w = 0; w < 4; ++w) g_wbar[w] = std::make_unique<std::barrier<>>(64);
    std::vector<std::thread> th;
    for (int t = 0; t < 256; ++t)
      th.emplace_back([=]() { threadIdx.x = t; blockIdx.x = b; kern(); });
    for (auto& x : th) x.join();
  }
}

// 128-byte aligned, size rounded up to whole 128-byte lines (the device
// allocations the kernels see are aligned at least as much)
template <typename T> static T* alloc(size_t n) {
  const size_t bytes = ((n * sizeof(T) + 127) / 128) * 128;
  return static_cast<T*>(std::aligned_alloc(128, bytes ? bytes : 128));
}
template <typename T> static T* dup(const std::vector<T>& v) {
  T* p = alloc<T>(v.size());
  std::memcpy(p, v.data(), v.size() * sizeof(T));
  return p;
}
static float* dupf(const std::vector<double>& v) {
  float* p = alloc<float>(v.size());
  for (size_t i = 0; i < v.size(); ++i) p[i] = float(v[i]);
  return p;
}

template <typename T>
static T* dupT(const std::vector<double>& v) {
  T* p = alloc<T>(v.size());
  for (size_t i = 0; i < v.size(); ++i) p[i] = T(v[i]);
  return p;
}

