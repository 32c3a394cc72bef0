// Host-side layout of the BF16x3 matrix-core stage (see dg_mfma_host.hpp).
#include "dg_mfma_host.hpp"

#include <cstring>

#include "dg_mfma_layout.hpp"

namespace dgh {
namespace {

uint16_t bf16_rne(float f) {
  uint32_t b;
  std::memcpy(&b, &f, 4);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return uint16_t(b >> 16);
}
float bf16_val(uint16_t h) {
  const uint32_t b = uint32_t(h) << 16;
  float f;
  std::memcpy(&f, &b, 4);
  return f;
}

// Operator fragments in MFMA A-operand lane order: fragment (t, kb, hl) holds
// A[16 t + l % 16][32 kb + 8 (l / 16) + j] for lane l, j = 0..7, split into
// hi = bf16(a), lo = bf16(a - hi).  The K indices of V_q and P_q are permuted
// so that they consume the previous contraction's accumulator layout.
template <int N>
std::vector<uint16_t> build_frags(const RefElement& re) {
  using O = dgm::MOrd<N>;
  std::vector<uint16_t> out(size_t(O::NFRAG) * 64 * 8, 0);
  auto put = [&](int off, int KB, int t, int kb, auto&& aval) {
    for (int l = 0; l < 64; ++l)
      for (int j = 0; j < 8; ++j) {
        const int i = 16 * t + (l % 16);
        const int p = 32 * kb + 8 * (l / 16) + j;
        const double v = aval(i, p);
        const uint16_t hi = bf16_rne(float(v));
        const uint16_t lo = bf16_rne(float(v - double(bf16_val(hi))));
        out[((size_t(off + (t * KB + kb) * 2 + 0) * 64) + l) * 8 + j] = hi;
        out[((size_t(off + (t * KB + kb) * 2 + 1) * 64) + l) * 8 + j] = lo;
      }
  };
  const int Np = O::Np, NF4 = O::NF4, Nq = O::Nq;
  // [Dr | Ds | Dt | LIFT] with 8-row chunks: chunk h < 3 CV -> derivative
  // d = h / CV, node 8 (h % CV) + j; next CF chunks -> face node; rest zero
  auto avol = [&](int i, int p) -> double {
    if (i >= Np) return 0.0;
    const int h = p / 8, jj = p % 8;
    if (h < 3 * O::CV) {
      const int d = h / O::CV, m = 8 * (h % O::CV) + jj;
      if (m >= Np) return 0.0;
      const std::vector<double>& D = d == 0 ? re.Dr : d == 1 ? re.Ds : re.Dt;
      return D[size_t(i) * Np + m];
    }
    if (h < 3 * O::CV + O::CF) {
      const int jf = 8 * (h - 3 * O::CV) + jj;
      return jf < NF4 ? re.LIFT[size_t(i) * NF4 + jf] : 0.0;
    }
    return 0.0;
  };
  // accumulator row of K position p: tile 2 (p / 32) + (p % 8) / 4, row
  // 4 ((p % 32) / 8) + p % 4
  auto acc_row = [](int p) {
    const int kb = p / 32, g = (p % 32) / 8, jj = p % 8;
    return 16 * (2 * kb + jj / 4) + 4 * g + (jj % 4);
  };
  auto avq = [&](int i, int p) -> double {
    const int n = acc_row(p);
    return (i < Nq && n < Np) ? re.Vq[size_t(i) * Np + n] : 0.0;
  };
  auto apq = [&](int i, int p) -> double {
    const int qr = acc_row(p);
    return (i < Np && qr < Nq) ? re.Pq[size_t(i) * Nq + qr] : 0.0;
  };
  for (int t = 0; t < O::MT; ++t)
    for (int kb = 0; kb < O::KVB; ++kb) put(O::OFF_V, O::KVB, t, kb, avol);
  for (int t = 0; t < O::QT; ++t)
    for (int kb = 0; kb < O::KQB; ++kb) put(O::OFF_Q, O::KQB, t, kb, avq);
  for (int t = 0; t < O::MT; ++t)
    for (int kb = 0; kb < O::PKB; ++kb) put(O::OFF_P, O::PKB, t, kb, apq);
  return out;
}


int mfma_qp(int N) {
  switch (N) {
    case 1: return dgm::MOrd<1>::QP;
    case 2: return dgm::MOrd<2>::QP;
    case 3: return dgm::MOrd<3>::QP;
    default: return dgm::MOrd<4>::QP;
  }
}

}  // namespace

// N = 4 is switched off: its stage kernel (76 KB of LDS per workgroup, two
// workgroups per CU) faulted the GPU once although every index it forms is in
// bounds on the CPU; it stays disabled until the cause is known.
bool mfma_supported(int N) { return N >= 1 && N <= 3; }

std::vector<uint16_t> mfma_fragments(const RefElement& re) {
  switch (re.N) {
    case 1: return build_frags<1>(re);
    case 2: return build_frags<2>(re);
    case 3: return build_frags<3>(re);
    default: return build_frags<4>(re);
  }
}

std::vector<double> col_operators(const RefElement& re) {
  const int Np = re.Np, Nq = re.Nq, NF4 = 4 * re.Nfp;
  const int NpP = 4 * ((Np + 3) / 4), QP = 32 * ((Nq + 31) / 32);
  std::vector<double> out;
  // T[i][j] = M[j][i] for i < cols_in, j < rows_out (zero elsewhere)
  auto put = [&](const std::vector<double>& M, int mrows, int mcols, int trows, int tcols) {
    for (int i = 0; i < trows; ++i)
      for (int j = 0; j < tcols; ++j)
        out.push_back((i < mcols && j < mrows) ? M[size_t(j) * mcols + i] : 0.0);
  };
  put(re.Dr, Np, Np, Np, NpP);
  put(re.Ds, Np, Np, Np, NpP);
  put(re.Dt, Np, Np, Np, NpP);
  put(re.LIFT, Np, NF4, NF4, NpP);
  put(re.Vq, Nq, Np, Np, QP);
  put(re.Pq, Np, Nq, QP, NpP);
  return out;
}

std::vector<double> mfma_material(int N, int64_t K, const double* irho, const double* lam,
                                  const double* mu) {
  // [tile][field][QP][16]: the accumulator layout reads 16 elements of one
  // quadrature point contiguously
  const int QP = mfma_qp(N), Nq = num_quad(N);
  const int64_t ntiles = (K + 15) / 16;
  std::vector<double> blk(size_t(ntiles) * 3 * QP * 16, 0.0);
  const double* src[3] = {irho, lam, mu};
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 3; ++f)
      for (int qp = 0; qp < Nq; ++qp)
        blk[((size_t(k / 16) * 3 + f) * QP + qp) * 16 + (k % 16)] = src[f][size_t(k) * Nq + qp];
  return blk;
}

}  // namespace dgh
