// Runs one reverse stage of the tiled FP32 adjoint (dgt::adj_tile<N, rin> and
// dgt::adj_nodes, orders 1-4) on the CPU, for tests: each workgroup is 256
// host threads with real barriers and emulated matrix-core products (see
// emu_runtime.hpp).  Built with AddressSanitizer by the test, so any
// out-of-bounds access of the kernel source shows up on the CPU.
//
// rin = 0: adj_tile<N, false> computes R y; 1: R y is read from the input
// file and the tile computes the face-node jumps; 2: as the library's replay
// and reverse stage, dgb::stage_bx_r<N> first runs a stage on y and stores R y
// and (upwind) the jumps, which adj_tile<N, true> and adj_nodes then read.
//
// input file: int32 N, flux_upwind, rin; int64 K; float64 vxyz[K*12], period[3],
// rho_q, cp_q, cs_q [K*Nq each], rho_n, cp_n, cs_n [K*Np each]; float32
// y, lres, ly [9*K*Np each]; with rin = 1, float32 R y [9*K*Np]; float64 a, b, dt, ts;
// int32 nsrc; per source
// int64 element, float32 raw response [3*Np], float64 (f0, t0, amplitude).
// output file: float64 lres (= a lres + b ly), ly, grad [3*K*Nq], gradz
// [2*K*Np] after the stage (grad and gradz accumulated from zero).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "dg_adjt.hpp"
#include "dg_bx.hpp"
#include "dg_host.hpp"
#include "dg_mfma_host.hpp"

#include "emu_runtime.hpp"

int main(int argc, char** argv) {
  if (argc != 3) { fprintf(stderr, "usage: emu_adjoint in.bin out.bin\n"); return 2; }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t hdr[3]; int64_t K;
  if (fread(hdr, 4, 3, f) != 3 || fread(&K, 8, 1, f) != 1) return 2;
  const int N = hdr[0], upwind = hdr[1], rin = hdr[2];
  if (N < 1 || N > 4 || rin < 0 || rin > 2) return 3;
  const int Np = dgh::num_nodes(N), Nq = dgh::num_quad(N);
  auto rd = [&](size_t n) { std::vector<double> v(n); if (fread(v.data(), 8, n, f) != n) exit(2); return v; };
  auto rdf = [&](size_t n) { std::vector<float> v(n); if (fread(v.data(), 4, n, f) != n) exit(2); return v; };
  auto vx = rd(K * 12), per = rd(3);
  auto rq = rd(K * Nq), pq = rd(K * Nq), sq = rd(K * Nq);
  auto rn = rd(K * Np), pn = rd(K * Np), sn = rd(K * Np);
  const size_t n9 = size_t(9) * K * Np;
  auto y = rdf(n9), lres = rdf(n9), ly = rdf(n9);
  std::vector<float> rraw = rin == 1 ? rdf(n9) : std::vector<float>();
  auto sc = rd(4);
  int32_t nsrc = 0;
  if (fread(&nsrc, 4, 1, f) != 1) return 2;
  std::vector<int64_t> selem(nsrc);
  std::vector<float> sw(size_t(nsrc) * 3 * Np);
  std::vector<double> spar(size_t(nsrc) * 3);
  for (int i = 0; i < nsrc; ++i) {
    if (fread(&selem[i], 8, 1, f) != 1) return 2;
    if (fread(&sw[size_t(i) * 3 * Np], 4, 3 * Np, f) != size_t(3 * Np)) return 2;
    if (fread(&spar[3 * i], 8, 3, f) != 3) return 2;
  }
  fclose(f);

  dgh::RefElement re; std::string err;
  if (!dgh::build_ref_element(N, re, err)) { fprintf(stderr, "%s\n", err.c_str()); return 1; }
  dgh::MeshData m;
  if (!dgh::build_mesh(re, K, vx.data(), per.data(), m, err)) { fprintf(stderr, "%s\n", err.c_str()); return 1; }
  std::vector<double> a(K * Nq), b(K * Nq), d(K * Nq), zp(K * Np), zs(K * Np);
  for (int64_t i = 0; i < K * Nq; ++i) {
    a[i] = 1.0 / rq[i]; b[i] = rq[i] * (pq[i] * pq[i] - 2 * sq[i] * sq[i]);
    d[i] = rq[i] * sq[i] * sq[i];
  }
  for (int64_t i = 0; i < K * Np; ++i) { zp[i] = rn[i] * pn[i]; zs[i] = rn[i] * sn[i]; }
  std::vector<int32_t> nbface, invf;
  if (!dgh::adjoint_face_tables(re, m, nbface, invf, err)) { fprintf(stderr, "%s\n", err.c_str()); return 1; }

  const int NF4 = 4 * re.Nfp;
  float* yd = dup(y);
  float* lr = dup(lres);
  float* lyd = dup(ly);
  float* nu = alloc<float>(n9);
  float* gf = alloc<float>(size_t(9) * K * NF4);
  float* jmp = alloc<float>(size_t(8) * K * NF4);
  double* grad = alloc<double>(size_t(3) * K * Nq);
  double* gradz = alloc<double>(size_t(2) * K * Np);
  for (int64_t i = 0; i < 3 * K * Nq; ++i) grad[i] = 0.0;
  for (int64_t i = 0; i < 2 * K * Np; ++i) gradz[i] = 0.0;
  std::vector<int32_t> fm(re.Fmask.begin(), re.Fmask.end());

  dgt::TileArgs A{};
  A.y = yd; A.r = rin == 1 ? dup(rraw) : nullptr; A.lres = lr; A.ly = lyd; A.nu = nu; A.gf = gf; A.jmp = jmp; A.grad = grad;
  A.geo = dupf(m.geo); A.fgeo = dupf(m.fgeo);
  A.nbn = dup(dgh::neighbour_nodes(re, m));
  A.fmask = dup(fm);
  A.mat = dupf(dgh::mfma_material(N, K, a.data(), b.data(), d.data()));
  A.zp = dupf(zp); A.zs = dupf(zs);
  A.frags = dup(dgh::adj_fragments_f32(re));
  A.src_elem = nsrc ? dup(selem) : nullptr;
  A.src_w = nsrc ? dup(sw) : nullptr;
  A.src_par = nsrc ? dup(spar) : nullptr;
  A.nsrc = nsrc; A.ts = sc[3];
  A.K = K; A.a = float(sc[0]); A.b = float(sc[1]); A.s = sc[2]; A.upwind = upwind;
  A.jumps = 1;
  const int tiles = int((K + 15) / 16);
  float* jst = nullptr;   // the jumps the replay's stage stores (rin = 2)
  if (rin == 2) {
    dgb::BxArgs S{};
    S.q_in = yd;
    S.q_out = alloc<float>(n9);
    S.res = alloc<float>(n9);
    for (size_t i = 0; i < n9; ++i) S.res[i] = 0.f;
    S.geo = A.geo; S.fgeo = A.fgeo; S.nbn = A.nbn; S.fmask = A.fmask;
    S.torder = dup(dgh::tile_order(m, dgb::kTile, 8));
    S.mat = A.mat; S.zp = A.zp; S.zs = A.zs;
    S.frags = reinterpret_cast<const dgb::u32x4*>(dup(dgh::mfma_fragments_f32(re)));
    S.K = K; S.a = 0.f; S.b = 1.f; S.dt = 1.f; S.lsrk = 1; S.upwind = upwind;
    S.r_out = alloc<float>(n9);
    if (upwind) jst = S.j_out = alloc<float>(size_t(8) * K * NF4);
    const int sg = int((K + dgb::kTile - 1) / dgb::kTile);
    switch (N) {
      case 1: run_grid(sg, [=]() { dgb::stage_bx_r<1>(S); }); break;
      case 2: run_grid(sg, [=]() { dgb::stage_bx_r<2>(S); }); break;
      case 3: run_grid(sg, [=]() { dgb::stage_bx_r<3>(S); }); break;
      default: run_grid(sg, [=]() { dgb::stage_bx_r<4>(S); }); break;
    }
    A.r = S.r_out;
    A.jumps = 0;
  }
  if (rin) {
    switch (N) {
      case 1: run_grid(tiles, [=]() { dgt::adj_tile<1, true>(A); }); break;
      case 2: run_grid(tiles, [=]() { dgt::adj_tile<2, true>(A); }); break;
      case 3: run_grid(tiles, [=]() { dgt::adj_tile<3, true>(A); }); break;
      default: run_grid(tiles, [=]() { dgt::adj_tile<4, true>(A); }); break;
    }
  } else {
    switch (N) {
      case 1: run_grid(tiles, [=]() { dgt::adj_tile<1, false>(A); }); break;
      case 2: run_grid(tiles, [=]() { dgt::adj_tile<2, false>(A); }); break;
      case 3: run_grid(tiles, [=]() { dgt::adj_tile<3, false>(A); }); break;
      default: run_grid(tiles, [=]() { dgt::adj_tile<4, false>(A); }); break;
    }
  }
  dgt::NodeArgs B{};
  B.nu = nu; B.gf = gf; B.jmp = jst ? jst : jmp; B.ly = lyd; B.gradz = gradz;
  B.fgeo = A.fgeo; B.zp = A.zp; B.zs = A.zs; B.nbn = A.nbn;
  B.nbface = dup(nbface); B.invf = dup(invf);
  B.K = K; B.Np = Np; B.Nfp = re.Nfp; B.s = sc[2]; B.upwind = upwind;
  run_grid(int((K * Np + 255) / 256), [=]() { dgt::adj_nodes(B); });

  FILE* g = fopen(argv[2], "wb");
  std::vector<double> o(n9);
  for (size_t i = 0; i < n9; ++i) o[i] = lr[i];
  fwrite(o.data(), 8, n9, g);
  for (size_t i = 0; i < n9; ++i) o[i] = lyd[i];
  fwrite(o.data(), 8, n9, g);
  fwrite(grad, 8, size_t(3) * K * Nq, g);
  fwrite(gradz, 8, size_t(2) * K * Np, g);
  fclose(g);
  return 0;
}
