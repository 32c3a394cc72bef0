// Runs the stage kernels on the CPU, for tests (the matrix-core kernels
// dgb::stage_bx<N> in BF16x3 and FP32, dgb::stage_bx_d<N> in FP64,
// dgb::stage_be<N> in BF16x3 and FP32, and dgb::stage_be_d<N> in FP64):
// each workgroup is 256 host threads with real barriers; the 16x16x32 bf16
// MFMA is emulated with its hardware lane layout (A: row lane%16, k 8(lane/16)+j;
// B: column lane%16, k 8(lane/16)+j; D: column lane%16, row 4(lane/16)+j).
// Built with AddressSanitizer by the test, so any out-of-bounds access of the
// kernel source shows up on the CPU.  Reads a binary problem file, writes the
// right-hand side (or the LSRK increment q_out - q_in) as float64.
#include <hip/hip_runtime.h>
#include <thread>
#include <vector>
#include <memory>
#include <cstring>
#include <cstdlib>
#include <cmath>
#include "dg_be.hpp"
#include "dg_bx.hpp"
#include "dg_host.hpp"
#include "dg_mfma_host.hpp"

#include "emu_runtime.hpp"

template <int N, bool F32>
static void run(dgb::BxArgs A, int grid) {
  run_grid(grid, [=]() { dgb::stage_bx<N, F32>(A); });
}


static int emu_rhs(int N, int64_t K, const double* vxyz, const double* period,
                       const double* rho_q, const double* cp_q, const double* cs_q,
                       const double* rho_n, const double* cp_n, const double* cs_n,
                       const float* q, double* out, int upwind, int grid, int lsrk) {
  dgh::RefElement re; std::string err;
  if (!dgh::build_ref_element(N, re, err)) { fprintf(stderr, "%s\n", err.c_str()); return 1; }
  dgh::MeshData m;
  if (!dgh::build_mesh(re, K, vxyz, period, m, err)) { fprintf(stderr, "%s\n", err.c_str()); return 2; }
  const int Np = re.Np, Nq = re.Nq;
  std::vector<double> a(K * Nq), b(K * Nq), d(K * Nq), zp(K * Np), zs(K * Np);
  for (int64_t i = 0; i < K * Nq; ++i) {
    a[i] = 1.0 / rho_q[i]; b[i] = rho_q[i] * (cp_q[i] * cp_q[i] - 2 * cs_q[i] * cs_q[i]);
    d[i] = rho_q[i] * cs_q[i] * cs_q[i];
  }
  for (int64_t i = 0; i < K * Np; ++i) { zp[i] = rho_n[i] * cp_n[i]; zs[i] = rho_n[i] * cs_n[i]; }
  if (grid < 1 || grid > 4) return 3;
  if (grid == 3 && N >= 5) {   // FP64 matrix-core kernel, orders 5-7
    dgb::BeArgsT<double> E{};
    std::vector<double> qd(q, q + 9 * K * Np);
    E.q_in = dupT<double>(qd);
    E.rhs_out = alloc<double>(9 * K * Np);
    E.q_out = lsrk ? alloc<double>(9 * K * Np) : nullptr;
    E.res = nullptr;
    if (lsrk) { E.res = alloc<double>(9 * K * Np); for (int64_t i = 0; i < 9 * K * Np; ++i) E.res[i] = 0.0; }
    E.geo = dupT<double>(m.geo); E.fgeo = dupT<double>(m.fgeo);
    E.nbn = dup(dgh::neighbour_nodes(re, m));
    std::vector<int32_t> fmd(re.Fmask.begin(), re.Fmask.end());
    E.fmask = dup(fmd);
    E.irho = dupT<double>(a); E.lam = dupT<double>(b); E.mu = dupT<double>(d);
    E.zp = dupT<double>(zp); E.zs = dupT<double>(zs);
    E.frags = reinterpret_cast<const dgb::u32x4*>(dup(dgh::mfma_fragments_f64(re)));
    E.K = K; E.a = 0.0; E.b = 1.0; E.dt = 1.0; E.lsrk = lsrk; E.upwind = upwind;
    switch (N) {
      case 5: run_grid(int(K), [=]() { dgb::stage_be_d<5>(E); }); break;
      case 6: run_grid(int(K), [=]() { dgb::stage_be_d<6>(E); }); break;
      default: run_grid(int(K), [=]() { dgb::stage_be_d<7>(E); }); break;
    }
    for (int64_t i = 0; i < 9 * K * Np; ++i)
      out[i] = lsrk ? E.q_out[i] - E.q_in[i] : E.rhs_out[i];
    return 0;
  }
  if (grid == 3) {   // FP64 matrix-core tiled kernel, orders 1-4
    dgb::BxArgsT<double> D{};
    std::vector<double> qd(q, q + 9 * K * Np);
    D.q_in = dupT<double>(qd);
    D.rhs_out = alloc<double>(9 * K * Np);
    D.q_out = lsrk ? alloc<double>(9 * K * Np) : nullptr;
    D.res = nullptr;
    if (lsrk) { D.res = alloc<double>(9 * K * Np); for (int64_t i = 0; i < 9 * K * Np; ++i) D.res[i] = 0.0; }
    D.geo = dupT<double>(m.geo); D.fgeo = dupT<double>(m.fgeo);
    D.nbn = dup(dgh::neighbour_nodes(re, m));
    D.torder = dup(dgh::tile_order(m, dgb::kTile, 8));
    std::vector<int32_t> fmd(re.Fmask.begin(), re.Fmask.end());
    D.fmask = dup(fmd);
    D.mat = dupT<double>(dgh::mfma_material(N, K, a.data(), b.data(), d.data(), true));
    D.zp = dupT<double>(zp); D.zs = dupT<double>(zs);
    D.frags = reinterpret_cast<const dgb::u32x4*>(dup(dgh::mfma_fragments_f64(re)));
    D.K = K; D.a = 0.0; D.b = 1.0; D.dt = 1.0; D.lsrk = lsrk; D.upwind = upwind;
    const int tg = int((K + dgb::kTile - 1) / dgb::kTile);
    switch (N) {
      case 1: run_grid(tg, [=]() { dgb::stage_bx_d<1>(D); }); break;
      case 2: run_grid(tg, [=]() { dgb::stage_bx_d<2>(D); }); break;
      case 3: run_grid(tg, [=]() { dgb::stage_bx_d<3>(D); }); break;
      default: run_grid(tg, [=]() { dgb::stage_bx_d<4>(D); }); break;
    }
    for (int64_t i = 0; i < 9 * K * Np; ++i)
      out[i] = lsrk ? D.q_out[i] - D.q_in[i] : D.rhs_out[i];
    return 0;
  }
  std::vector<uint16_t> fr = dgh::mfma_fragments(re);
  if (N >= 5) {   // one element per workgroup (grid 2: the FP32 kernel)
    dgb::BeArgs E{};
    float* qe = alloc<float>(9 * K * Np);
    std::memcpy(qe, q, sizeof(float) * 9 * K * Np);
    E.q_in = qe;
    E.rhs_out = alloc<float>(9 * K * Np);
    E.q_out = lsrk ? alloc<float>(9 * K * Np) : nullptr;
    E.res = nullptr;
    if (lsrk) { E.res = alloc<float>(9 * K * Np); for (int64_t i = 0; i < 9 * K * Np; ++i) E.res[i] = 0.f; }
    E.geo = dupf(m.geo); E.fgeo = dupf(m.fgeo);
    E.nbn = dup(dgh::neighbour_nodes(re, m));
    std::vector<int32_t> fme(re.Fmask.begin(), re.Fmask.end());
    E.fmask = dup(fme);
    E.irho = dupf(a); E.lam = dupf(b); E.mu = dupf(d);
    E.zp = dupf(zp); E.zs = dupf(zs);
    const bool fe = grid == 2;
    if (fe) {
      const std::vector<float> ff = dgh::mfma_fragments_f32(re);
      E.frags = reinterpret_cast<const dgb::u32x4*>(dup(ff));
    } else {
      E.frags = reinterpret_cast<const dgb::u32x4*>(dup(fr));
    }
    E.K = K; E.a = 0.f; E.b = 1.f; E.dt = 1.f; E.lsrk = lsrk; E.upwind = upwind;
    switch (N) {
      case 5: fe ? run_grid(int(K), [=]() { dgb::stage_be<5, true>(E); })
                 : run_grid(int(K), [=]() { dgb::stage_be<5, false>(E); }); break;
      case 6: fe ? run_grid(int(K), [=]() { dgb::stage_be<6, true>(E); })
                 : run_grid(int(K), [=]() { dgb::stage_be<6, false>(E); }); break;
      default: fe ? run_grid(int(K), [=]() { dgb::stage_be<7, true>(E); })
                  : run_grid(int(K), [=]() { dgb::stage_be<7, false>(E); }); break;
    }
    for (int64_t i = 0; i < 9 * K * Np; ++i)
      out[i] = lsrk ? double(E.q_out[i]) - double(E.q_in[i]) : double(E.rhs_out[i]);
    return 0;
  }
  dgb::BxArgs A{};
  float* qin = alloc<float>(9 * K * Np);
  std::memcpy(qin, q, sizeof(float) * 9 * K * Np);
  A.q_in = qin;
  A.rhs_out = alloc<float>(9 * K * Np);
  A.q_out = lsrk ? alloc<float>(9 * K * Np) : nullptr;
  A.res = nullptr;
  if (lsrk) { A.res = alloc<float>(9 * K * Np); for (int64_t i = 0; i < 9 * K * Np; ++i) A.res[i] = 0.f; }
  A.geo = dupf(m.geo); A.fgeo = dupf(m.fgeo);
  A.nbn = dup(dgh::neighbour_nodes(re, m));
  A.torder = dup(dgh::tile_order(m, dgb::kTile, 8));
  std::vector<int32_t> fm(re.Fmask.begin(), re.Fmask.end());
  A.fmask = dup(fm);
  A.mat = dupf(dgh::mfma_material(N, K, a.data(), b.data(), d.data()));
  A.zp = dupf(zp); A.zs = dupf(zs);
  const bool f32 = grid == 2 || grid == 4;   // FP32 matrix-core kernel
  float* rraw = nullptr;
  if (grid == 4) {   // the FP32 kernel that also stores R q: output R q
    if (N > 4) return 3;
    rraw = alloc<float>(9 * K * Np);
    A.r_out = rraw;
    if (!lsrk) { A.res = alloc<float>(9 * K * Np); A.q_out = alloc<float>(9 * K * Np); }
    for (int64_t i = 0; i < 9 * K * Np; ++i) A.res[i] = 0.f;
    A.lsrk = 1;
  }
  if (f32) {
    const std::vector<float> ff = dgh::mfma_fragments_f32(re);
    A.frags = reinterpret_cast<const dgb::u32x4*>(dup(ff));
  } else {
    A.frags = reinterpret_cast<const dgb::u32x4*>(dup(fr));
  }
  A.K = K; A.a = 0.f; A.b = 1.f; A.dt = 1.f; A.upwind = upwind;
  if (!rraw) A.lsrk = lsrk;
  const bool rst = rraw != nullptr;
  grid = int((K + dgb::kTile - 1) / dgb::kTile);   // one workgroup per element tile
  if (rst) {
    switch (N) {
      case 1: run_grid(grid, [=]() { dgb::stage_bx_r<1>(A); }); break;
      case 2: run_grid(grid, [=]() { dgb::stage_bx_r<2>(A); }); break;
      case 3: run_grid(grid, [=]() { dgb::stage_bx_r<3>(A); }); break;
      default: run_grid(grid, [=]() { dgb::stage_bx_r<4>(A); }); break;
    }
    for (int64_t i = 0; i < 9 * K * Np; ++i) out[i] = double(rraw[i]);
    return 0;
  }
  switch (N) {
    case 1: f32 ? run<1, true>(A, grid) : run<1, false>(A, grid); break;
    case 2: f32 ? run<2, true>(A, grid) : run<2, false>(A, grid); break;
    case 3: f32 ? run<3, true>(A, grid) : run<3, false>(A, grid); break;
    case 4: f32 ? run<4, true>(A, grid) : run<4, false>(A, grid); break;
    default: return 3;
  }
  for (int64_t i = 0; i < 9 * K * Np; ++i)
    out[i] = lsrk ? double(A.q_out[i]) - double(A.q_in[i]) : double(A.rhs_out[i]);
  return 0;
}

// input file: int32 N, flux_upwind, kernel (1: BF16x3 matrix-core kernel, 2:
// FP32 matrix-core kernel, 3: FP64 matrix-core kernel, every order, 4: the
// FP32 kernel that also stores R q, whose R q is the output), lsrk; int64 K; then float64
// vxyz[K*12], period[3], rho_q, cp_q, cs_q [K*Nq each], rho_n, cp_n, cs_n
// [K*Np each]; then float32 q[9*K*Np]
int main(int argc, char** argv) {
  if (argc != 3) { fprintf(stderr, "usage: emu in.bin out.bin\n"); return 2; }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t hdr[4]; int64_t K;
  if (fread(hdr, 4, 4, f) != 4 || fread(&K, 8, 1, f) != 1) return 2;
  const int N = hdr[0];
  const int Np = dgh::num_nodes(N), Nq = dgh::num_quad(N);
  auto rd = [&](size_t n) { std::vector<double> v(n); if (fread(v.data(), 8, n, f) != n) exit(2); return v; };
  auto vx = rd(K * 12), per = rd(3);
  auto rq = rd(K * Nq), pq = rd(K * Nq), sq = rd(K * Nq);
  auto rn = rd(K * Np), pn = rd(K * Np), sn = rd(K * Np);
  std::vector<float> q(9 * K * Np);
  std::vector<double> out(9 * K * Np);
  if (fread(q.data(), 4, q.size(), f) != q.size()) return 2;
  fclose(f);
  const int rc = emu_rhs(N, K, vx.data(), per.data(), rq.data(), pq.data(), sq.data(), rn.data(),
                         pn.data(), sn.data(), q.data(), out.data(), hdr[1], hdr[2], hdr[3]);
  if (rc) return rc;
  FILE* g = fopen(argv[2], "wb");
  fwrite(out.data(), 8, out.size(), g);
  fclose(g);
  return 0;
}
