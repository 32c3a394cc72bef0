// Host-side layout of the BF16x3 matrix-core stage (see dg_mfma_host.hpp).
#include "dg_mfma_host.hpp"

#include <cstring>

#include "dg_bx_layout.hpp"

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

// Operator fragments in MFMA A-operand lane order: fragment (t, s, h) holds,
// for lane l, the operator entries of row 16 t + l % 16 at the K slots
// 8 (l / 16) + j, j = 0..7, of K step s, as h = 0: hi = bf16(a), h = 1:
// lo = bf16(a - hi).  The meaning of each K slot (which node, direction,
// face node or quadrature point it carries) is the permutation described with
// the kernel's sizes; rows and slots beyond the element's counts are zero.
template <int N>
std::vector<uint16_t> build_frags(const RefElement& re) {
  using O = dgb::BOrd<N>;
  std::vector<uint16_t> out(size_t(O::NFRAG) * 64 * 8, 0);
  auto put = [&](int frag, auto&& aval) {   // aval(row offset in tile, g, j)
    for (int l = 0; l < 64; ++l)
      for (int j = 0; j < 8; ++j) {
        const double v = aval(l % 16, l / 16, j);
        const uint16_t hi = bf16_rne(float(v));
        const uint16_t lo = bf16_rne(float(v - double(bf16_val(hi))));
        out[(size_t(frag) * 64 + l) * 8 + j] = hi;
        out[(size_t(frag + 1) * 64 + l) * 8 + j] = lo;
      }
  };
  const int Np = O::Np, NF4 = O::NF4, Nq = O::Nq;
  for (int t = 0; t < O::RT; ++t)
    for (int s = 0; s < O::SVL; ++s)
      put(O::OFF_V + (t * O::SVL + s) * 2, [&](int r, int g, int j) -> double {
        const int n = 16 * t + r;
        if (n >= Np) return 0.0;
        if (s < O::SN && j < 6) {
          const int m = g + 4 * (2 * s + j / 3);
          if (m >= Np) return 0.0;
          const std::vector<double>& D = j % 3 == 0 ? re.Dr : j % 3 == 1 ? re.Ds : re.Dt;
          return D[size_t(n) * Np + m];
        }
        const int i = s < O::SN ? 2 * s + (j - 6) : 2 * O::SN + 8 * (s - O::SN) + j;
        const int jf = g + 4 * i;
        return jf < NF4 ? re.LIFT[size_t(n) * NF4 + jf] : 0.0;
      });
  for (int t = 0; t < O::QT; ++t)
    for (int s = 0; s < O::SVQ; ++s)
      put(O::OFF_Q + (t * O::SVQ + s) * 2, [&](int r, int g, int j) -> double {
        const int p = 16 * t + r;
        const int n = 16 * (2 * s + j / 4) + 4 * g + j % 4;
        return (p < Nq && n < Np) ? re.Vq[size_t(p) * Np + n] : 0.0;
      });
  for (int t = 0; t < O::RT; ++t)
    for (int c = 0; c < O::QC; ++c)
      put(O::OFF_P + (t * O::QC + c) * 2, [&](int r, int g, int j) -> double {
        const int n = 16 * t + r;
        const int p = 32 * c + 16 * (j / 4) + 4 * g + j % 4;
        return (n < Np && p < Nq) ? re.Pq[size_t(n) * Nq + p] : 0.0;
      });
  return out;
}

// Fragments of the FP32 / FP64 matrix-core stage (FOrd) in the working
// precision V, four steps per lane
template <int N, typename V>
std::vector<V> build_frags_f(const RefElement& re) {
  using O = dgb::FOrd<N>;
  const int Np = O::Np, NF4 = O::NF4, Nq = O::Nq;
  constexpr bool f64 = sizeof(V) == 8;   // accumulator row order of the FP64 product
  std::vector<V> out(size_t(O::NF4S) * 4, V(0));
  const std::vector<double>* D[3] = {&re.Dr, &re.Ds, &re.Dt};
  for (int t = 0; t < O::RT; ++t)
    for (int q = 0; q < O::SV4; ++q)
      for (int l = 0; l < 64; ++l)
        for (int j = 0; j < 4; ++j) {
          const int s = 4 * q + j, r = 16 * t + l % 16, g = l / 16;
          double v = 0.0;
          if (r < Np && s < O::SV) {
            if (s < 3 * O::NB) {
              const int m = 4 * (s / 3) + g;
              if (m < Np) v = (*D[s % 3])[size_t(r) * Np + m];
            } else {
              const int jf = 4 * (s - 3 * O::NB) + g;
              if (jf < NF4) v = re.LIFT[size_t(r) * NF4 + jf];
            }
          }
          out[((size_t(O::OFF_V) + size_t(t * O::SV4 + q) * 64) + l) * 4 + j] = V(v);
        }
  for (int u = 0; u < O::QT; ++u)
    for (int t = 0; t < O::RT; ++t)
      for (int l = 0; l < 64; ++l)
        for (int j = 0; j < 4; ++j) {
          const int p = 16 * u + l % 16, n = 16 * t + dgb::acc_row(f64, l / 16, j);
          const double v = (p < Nq && n < Np) ? re.Vq[size_t(p) * Np + n] : 0.0;
          out[((size_t(O::OFF_Q) + size_t(u * O::RT + t) * 64) + l) * 4 + j] = V(v);
        }
  for (int t = 0; t < O::RT; ++t)
    for (int u = 0; u < O::QT; ++u)
      for (int l = 0; l < 64; ++l)
        for (int j = 0; j < 4; ++j) {
          const int r = 16 * t + l % 16, p = 16 * u + dgb::acc_row(f64, l / 16, j);
          const double v = (r < Np && p < Nq) ? re.Pq[size_t(r) * Nq + p] : 0.0;
          out[((size_t(O::OFF_P) + size_t(t * O::QT + u) * 64) + l) * 4 + j] = V(v);
        }
  return out;
}

// Fragments of the high-order stage (EOrd): D_r, D_s, D_t, LIFT, V_q, P_q in
// plain K order, zero beyond the operator's rows and columns
template <int N>
std::vector<uint16_t> build_frags_e(const RefElement& re) {
  using O = dgb::EOrd<N>;
  std::vector<uint16_t> out(size_t(O::NFRAG) * 64 * 8, 0);
  auto put = [&](int frag, const std::vector<double>& M, int rows, int cols, int t, int s) {
    for (int l = 0; l < 64; ++l)
      for (int j = 0; j < 8; ++j) {
        const int r = 16 * t + l % 16, k = 32 * s + 8 * (l / 16) + j;
        const double v = (r < rows && k < cols) ? M[size_t(r) * cols + k] : 0.0;
        const uint16_t hi = bf16_rne(float(v));
        const uint16_t lo = bf16_rne(float(v - double(bf16_val(hi))));
        out[(size_t(frag) * 64 + l) * 8 + j] = hi;
        out[(size_t(frag + 1) * 64 + l) * 8 + j] = lo;
      }
  };
  const int Np = O::Np, NF4 = O::NF4, Nq = O::Nq;
  const std::vector<double>* D[3] = {&re.Dr, &re.Ds, &re.Dt};
  for (int d = 0; d < 3; ++d)
    for (int t = 0; t < O::RT; ++t)
      for (int s = 0; s < O::KN; ++s)
        put(O::OFF_D + ((d * O::RT + t) * O::KN + s) * 2, *D[d], Np, Np, t, s);
  for (int t = 0; t < O::RT; ++t)
    for (int s = 0; s < O::KF; ++s) put(O::OFF_L + (t * O::KF + s) * 2, re.LIFT, Np, NF4, t, s);
  for (int t = 0; t < O::QT; ++t)
    for (int s = 0; s < O::KN; ++s) put(O::OFF_V + (t * O::KN + s) * 2, re.Vq, Nq, Np, t, s);
  for (int t = 0; t < O::RT; ++t)
    for (int s = 0; s < O::KQ; ++s) put(O::OFF_P + (t * O::KQ + s) * 2, re.Pq, Np, Nq, t, s);
  return out;
}

template <int N>
std::vector<double> build_material(int64_t K, const double* irho, const double* lam,
                                   const double* mu, bool f64) {
  // [tile][field][chunk c][half u][lane l][4]: element 16 tile + l % 16,
  // quadrature point 32 c + 16 u + acc_row(l / 16, j)
  using O = dgb::BOrd<N>;
  const int64_t ntiles = (K + 15) / 16;
  std::vector<double> blk(size_t(ntiles) * 3 * O::MATS, 0.0);
  const double* src[3] = {irho, lam, mu};
  for (int64_t tl = 0; tl < ntiles; ++tl)
    for (int f = 0; f < 3; ++f)
      for (int c = 0; c < O::QC; ++c)
        for (int u = 0; u < 2; ++u)
          for (int l = 0; l < 64; ++l)
            for (int j = 0; j < 4; ++j) {
              const int64_t k = 16 * tl + l % 16;
              const int p = 32 * c + 16 * u + dgb::acc_row(f64, l / 16, j);
              if (k >= K || p >= O::Nq) continue;
              blk[(size_t(tl) * 3 + f) * O::MATS + ((size_t(c) * 2 + u) * 64 + l) * 4 + j] =
                  src[f][size_t(k) * O::Nq + p];
            }
  return blk;
}

}  // namespace

bool mfma_supported(int N) { return N >= 1 && N <= 7; }


std::vector<uint16_t> mfma_fragments(const RefElement& re) {
  switch (re.N) {
    case 1: return build_frags<1>(re);
    case 2: return build_frags<2>(re);
    case 3: return build_frags<3>(re);
    case 4: return build_frags<4>(re);
    case 5: return build_frags_e<5>(re);
    case 6: return build_frags_e<6>(re);
    default: return build_frags_e<7>(re);
  }
}

// FP32 (V = float) or FP64 (V = double) fragments of the orders 5-7 stage in
// the layout of EFOrd
template <int N, typename V>
std::vector<V> build_frags_ef(const RefElement& re) {
  using O = dgb::EFOrd<N>;
  std::vector<V> out(size_t(O::NFRAG) * 64 * 4, V(0));
  auto put = [&](int frag, const std::vector<double>& M, int rows, int cols, int t, int s) {
    for (int l = 0; l < 64; ++l)
      for (int j = 0; j < 4; ++j) {
        const int r = 16 * t + l % 16, k = 16 * s + 4 * j + l / 16;
        out[(size_t(frag) * 64 + l) * 4 + j] =
            (r < rows && k < cols) ? V(M[size_t(r) * cols + k]) : V(0);
      }
  };
  const int Np = O::Np, NF4 = O::NF4, Nq = O::Nq;
  const std::vector<double>* D[3] = {&re.Dr, &re.Ds, &re.Dt};
  for (int d = 0; d < 3; ++d)
    for (int t = 0; t < O::RT; ++t)
      for (int s = 0; s < O::KN; ++s)
        put(O::OFF_D + (d * O::RT + t) * O::KN + s, *D[d], Np, Np, t, s);
  for (int t = 0; t < O::RT; ++t)
    for (int s = 0; s < O::KF; ++s) put(O::OFF_L + t * O::KF + s, re.LIFT, Np, NF4, t, s);
  for (int t = 0; t < O::QT; ++t)
    for (int s = 0; s < O::KN; ++s) put(O::OFF_V + t * O::KN + s, re.Vq, Nq, Np, t, s);
  for (int t = 0; t < O::RT; ++t)
    for (int s = 0; s < O::KQ; ++s) put(O::OFF_P + t * O::KQ + s, re.Pq, Np, Nq, t, s);
  return out;
}

std::vector<float> mfma_fragments_f32(const RefElement& re) {
  switch (re.N) {
    case 1: return build_frags_f<1, float>(re);
    case 2: return build_frags_f<2, float>(re);
    case 3: return build_frags_f<3, float>(re);
    case 4: return build_frags_f<4, float>(re);
    case 5: return build_frags_ef<5, float>(re);
    case 6: return build_frags_ef<6, float>(re);
    default: return build_frags_ef<7, float>(re);
  }
}

std::vector<double> mfma_fragments_f64(const RefElement& re) {
  switch (re.N) {
    case 1: return build_frags_f<1, double>(re);
    case 2: return build_frags_f<2, double>(re);
    case 3: return build_frags_f<3, double>(re);
    case 4: return build_frags_f<4, double>(re);
    case 5: return build_frags_ef<5, double>(re);
    case 6: return build_frags_ef<6, double>(re);
    default: return build_frags_ef<7, double>(re);
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
                                  const double* mu, bool f64) {
  switch (N) {
    case 1: return build_material<1>(K, irho, lam, mu, f64);
    case 2: return build_material<2>(K, irho, lam, mu, f64);
    case 3: return build_material<3>(K, irho, lam, mu, f64);
    default: return build_material<4>(K, irho, lam, mu, f64);
  }
}

int mfma_frag_count(int N) {
  switch (N) {
    case 1: return dgb::BOrd<1>::NFRAG;
    case 2: return dgb::BOrd<2>::NFRAG;
    case 3: return dgb::BOrd<3>::NFRAG;
    case 4: return dgb::BOrd<4>::NFRAG;
    case 5: return dgb::EOrd<5>::NFRAG;
    case 6: return dgb::EOrd<6>::NFRAG;
    default: return dgb::EOrd<7>::NFRAG;
  }
}

namespace {

// FP32 operator fragments of the tiled adjoint kernel (the layout of
// dgt::AOrd<N>): [NG][64 lanes][4]
template <int N>
std::vector<float> build_adj_frags(const RefElement& re) {
  using O = dgt::AOrd<N>;
  const int Np = O::Np, NF4 = O::NF4, Nq = O::Nq;
  std::vector<float> out(size_t(O::NG) * 64 * 4, 0.f);
  const double* Dd[3] = {re.Dr.data(), re.Ds.data(), re.Dt.data()};
  // operator entries, zero outside the matrix
  auto D = [&](int d, int i, int j) { return i < Np && j < Np ? Dd[d][size_t(i) * Np + j] : 0.0; };
  auto L = [&](int i, int j) { return i < Np && j < NF4 ? re.LIFT[size_t(i) * NF4 + j] : 0.0; };
  auto V = [&](int p, int n) { return p < Nq && n < Np ? re.Vq[size_t(p) * Np + n] : 0.0; };
  auto P = [&](int n, int p) { return n < Np && p < Nq ? re.Pq[size_t(n) * Nq + p] : 0.0; };
  auto put = [&](int grp, int l, int item, double v) {
    out[(size_t(grp) * 64 + l) * 4 + item] = float(v);
  };
  for (int l = 0; l < 64; ++l) {
    const int r = l % 16, k = l / 16;
    for (int t = 0; t < O::RT; ++t)
      for (int s = 0; s < O::KN; ++s)
        for (int d = 0; d < 3; ++d) {
          put(O::G_D + t * O::KN + s, l, d, D(d, 16 * t + r, 4 * s + k));
          put(O::G_DT + t * O::KN + s, l, d, D(d, 4 * s + k, 16 * t + r));
        }
    for (int t = 0; t < O::RT; ++t)
      for (int s4 = 0; s4 < O::KF4; ++s4)
        for (int i = 0; i < 4; ++i)
          if (4 * s4 + i < O::KF) put(O::G_L + t * O::KF4 + s4, l, i, L(16 * t + r, 4 * (4 * s4 + i) + k));
    for (int u = 0; u < O::QT; ++u)
      for (int t = 0; t < O::RT; ++t)
        for (int j = 0; j < 4; ++j) {
          put(O::G_V + u * O::RT + t, l, j, V(16 * u + r, 16 * t + 4 * k + j));
          put(O::G_P + u * O::RT + t, l, j, P(16 * t + 4 * k + j, 16 * u + r));
          put(O::G_VT + u * O::RT + t, l, j, V(16 * u + 4 * k + j, 16 * t + r));
        }
    for (int f = 0; f < O::FT; ++f)
      for (int t = 0; t < O::RT; ++t)
        for (int j = 0; j < 4; ++j) put(O::G_LT + f * O::RT + t, l, j, L(16 * t + 4 * k + j, 16 * f + r));
    if (O::PACK) {
      const int n = 16 * (O::RT - 1) + k;   // zero past Np (k >= VLAST)
      for (int u = 0; u < O::QT; ++u) {
        put(O::G_VX + u, l, 0, V(16 * u + r, n));
        put(O::G_VX + u, l, 1, P(n, 16 * u + r));
      }
    }
  }
  return out;
}

}  // namespace

std::vector<float> adj_fragments_f32(const RefElement& re) {
  switch (re.N) {
    case 1: return build_adj_frags<1>(re);
    case 2: return build_adj_frags<2>(re);
    case 3: return build_adj_frags<3>(re);
    case 4: return build_adj_frags<4>(re);
    default: return {};
  }
}

int mfma_f32_frag_count(int N) {
  switch (N) {
    case 1: return dgb::FOrd<1>::NF4S;
    case 2: return dgb::FOrd<2>::NF4S;
    case 3: return dgb::FOrd<3>::NF4S;
    case 4: return dgb::FOrd<4>::NF4S;
    case 5: return dgb::EFOrd<5>::NFRAG * 64;
    case 6: return dgb::EFOrd<6>::NFRAG * 64;
    default: return dgb::EFOrd<7>::NFRAG * 64;
  }
}

int mfma_mats(int N) {
  switch (N) {
    case 1: return dgb::BOrd<1>::MATS;
    case 2: return dgb::BOrd<2>::MATS;
    case 3: return dgb::BOrd<3>::MATS;
    default: return dgb::BOrd<4>::MATS;
  }
}

size_t mfma_material_index(int N, int64_t k, int p, int f) {
  const int mats = mfma_mats(N);
  // inverse of the layout of build_material: p = 32 c + 16 u + 4 g + j,
  // lane l = 16 g + k % 16
  const int c = p / 32, u = (p % 32) / 16, g = (p % 16) / 4, j = p % 4;
  const int l = 16 * g + int(k % 16);
  return (size_t(k / 16) * 3 + f) * mats + ((size_t(c) * 2 + u) * 64 + l) * 4 + j;
}

}  // namespace dgh
