// Host FP64 precompute: reference element, periodic connectivity, geometry.
//
// Reference element [HW08 = Hesthaven & Warburton, Nodal DG Methods, 2008,
// Ch. 6 and 10]: orthonormal Koornwinder-Dubiner basis built from Jacobi
// polynomials (three-term recurrence), Vandermonde matrices, D_i = V_i V^-1,
// M^-1 = V V^T, face mass matrices from the orthonormal triangle basis,
// LIFT = M^-1 E.  Quadrature: collapsed Gauss-Jacobi (Stroud conical
// product) rule with N+1 points per direction, exact to degree 2N+1; the
// 1D rules come from the Golub-Welsch eigenproblem of the Jacobi matrix.
#include "dg_host.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <tuple>

namespace dgh {
namespace {

// face f of the reference tetrahedron: its three vertices, in the order that
// defines face-local barycentric coordinates
constexpr int kFaceVerts[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {0, 2, 3}};

// ---------------------------------------------------------------- Jacobi --
// Orthonormal Jacobi polynomials p_k^{(a,b)} with respect to (1-x)^a (1+x)^b
// on [-1,1], from x p_k = A_{k+1} p_{k+1} + B_k p_k + A_k p_{k-1}.
double jac_A(int k, double a, double b) {  // k >= 1
  const double h = 2.0 * k + a + b;
  return 2.0 / h *
         std::sqrt(k * (k + a) * (k + b) * (k + a + b) / ((h - 1.0) * (h + 1.0)));
}
double jac_B(int k, double a, double b) {
  if (a == b) return 0.0;
  const double h = 2.0 * k + a + b;
  return (b * b - a * a) / (h * (h + 2.0));
}
double jac_mu0(double a, double b) {  // integral of the weight
  return std::pow(2.0, a + b + 1.0) * std::tgamma(a + 1.0) * std::tgamma(b + 1.0) /
         std::tgamma(a + b + 2.0);
}
// p_0..p_n at x
void jacobi_all(double x, double a, double b, int n, double* p) {
  p[0] = 1.0 / std::sqrt(jac_mu0(a, b));
  if (n == 0) return;
  p[1] = ((x - jac_B(0, a, b)) * p[0]) / jac_A(1, a, b);
  for (int k = 1; k < n; ++k)
    p[k + 1] = ((x - jac_B(k, a, b)) * p[k] - jac_A(k, a, b) * p[k - 1]) /
               jac_A(k + 1, a, b);
}
double jacobi(double x, double a, double b, int n) {
  double p[32];
  jacobi_all(x, a, b, n, p);
  return p[n];
}
// d/dx p_n^{(a,b)} = sqrt(n (n+a+b+1)) p_{n-1}^{(a+1,b+1)}
double djacobi(double x, double a, double b, int n) {
  if (n == 0) return 0.0;
  return std::sqrt(n * (n + a + b + 1.0)) * jacobi(x, a + 1.0, b + 1.0, n - 1);
}

// eigenvalues of a small dense symmetric matrix (cyclic Jacobi rotations)
void sym_eigenvalues(int n, std::vector<double> A, std::vector<double>& ev) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    if (off < 1e-32) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double tt = (theta >= 0 ? 1.0 : -1.0) /
                          (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(tt * tt + 1.0), s = tt * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
      }
  }
  ev.resize(n);
  for (int i = 0; i < n; ++i) ev[i] = A[i * n + i];
  std::sort(ev.begin(), ev.end());
}

// n-point Gauss-Jacobi rule for weight (1-x)^a (1+x)^b (Golub-Welsch nodes,
// Newton-polished; Christoffel weights 1 / sum_k p_k(x_i)^2)
void gauss_jacobi(int n, double a, double b, std::vector<double>& x,
                  std::vector<double>& w) {
  std::vector<double> T(n * n, 0.0);
  for (int k = 0; k < n; ++k) {
    T[k * n + k] = jac_B(k, a, b);
    if (k + 1 < n) T[k * n + k + 1] = T[(k + 1) * n + k] = jac_A(k + 1, a, b);
  }
  sym_eigenvalues(n, T, x);
  w.resize(n);
  double p[32];
  for (int i = 0; i < n; ++i) {
    for (int it = 0; it < 3; ++it) {
      const double d = djacobi(x[i], a, b, n);
      if (d != 0.0) x[i] -= jacobi(x[i], a, b, n) / d;
    }
    jacobi_all(x[i], a, b, n - 1, p);
    double sum = 0.0;
    for (int k = 0; k < n; ++k) sum += p[k] * p[k];
    w[i] = 1.0 / sum;
  }
}

// ---------------------------------------------------------- dense algebra --
bool invert(int n, const std::vector<double>& A, std::vector<double>& Ai) {
  std::vector<double> M(A);
  Ai.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) Ai[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(M[r * n + c]) > std::fabs(M[piv * n + c])) piv = r;
    if (std::fabs(M[piv * n + c]) < 1e-300) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(M[c * n + k], M[piv * n + k]);
        std::swap(Ai[c * n + k], Ai[piv * n + k]);
      }
    const double inv = 1.0 / M[c * n + c];
    for (int k = 0; k < n; ++k) {
      M[c * n + k] *= inv;
      Ai[c * n + k] *= inv;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = M[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        M[r * n + k] -= f * M[c * n + k];
        Ai[r * n + k] -= f * Ai[c * n + k];
      }
    }
  }
  return true;
}

// C[m][n] = A[m][k] * B[k][n]
std::vector<double> matmul(int m, int k, int n, const std::vector<double>& A,
                           const std::vector<double>& B) {
  std::vector<double> C(size_t(m) * n, 0.0);
  for (int i = 0; i < m; ++i)
    for (int l = 0; l < k; ++l) {
      const double a = A[size_t(i) * k + l];
      for (int j = 0; j < n; ++j) C[size_t(i) * n + j] += a * B[size_t(l) * n + j];
    }
  return C;
}

// ----------------------------------------------------------------- basis --
// collapsed coordinates; singular edge/apex values are irrelevant because
// the basis and gradient are evaluated in cancelled (polynomial) form
void collapse(double r, double s, double t, double& a, double& b, double& c) {
  const double da = -s - t, db = 1.0 - t;
  a = (std::fabs(da) > 1e-14) ? 2.0 * (1.0 + r) / da - 1.0 : -1.0;
  b = (std::fabs(db) > 1e-14) ? 2.0 * (1.0 + s) / db - 1.0 : -1.0;
  c = t;
}

// Orthonormal tetrahedral basis phi_{ijk} = 2 sqrt2 f(a) g(b) h(c),
// f = p_i^{(0,0)}, g = p_j^{(2i+1,0)} (1-b)^i, h = p_k^{(2i+2j+2,0)} (1-c)^{i+j};
// optional gradient by the chain rule through the collapse:
//   d/dr = 4 f' g h / ((1-b)(1-c))
//   d/ds = 2(1+a) f' g h / ((1-b)(1-c)) + 2 f g' h / (1-c)
//   d/dt = 2(1+a) f' g h / ((1-b)(1-c)) + (1+b) f g' h / (1-c) + f g h'
// with each quotient cancelled against the explicit powers.
void tet_basis(int N, double r, double s, double t, double* phi, double* pr,
               double* ps, double* pt) {
  double a, b, c;
  collapse(r, s, t, a, b, c);
  const double sc = 2.0 * std::sqrt(2.0);
  int m = 0;
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N - i; ++j)
      for (int k = 0; k <= N - i - j; ++k, ++m) {
        const double f = jacobi(a, 0, 0, i);
        const double pj = jacobi(b, 2.0 * i + 1, 0, j);
        const double pk = jacobi(c, 2.0 * i + 2.0 * j + 2, 0, k);
        const double g = pj * std::pow(1.0 - b, i);
        const double h = pk * std::pow(1.0 - c, i + j);
        phi[m] = sc * f * g * h;
        if (!pr) continue;
        const double fa = djacobi(a, 0, 0, i);
        const double dpj = djacobi(b, 2.0 * i + 1, 0, j);
        const double dpk = djacobi(c, 2.0 * i + 2.0 * j + 2, 0, k);
        const double g_b = (i >= 1) ? pj * std::pow(1.0 - b, i - 1) : 0.0;  // g/(1-b)
        const double h_c = (i + j >= 1) ? pk * std::pow(1.0 - c, i + j - 1) : 0.0;
        double gp = dpj * std::pow(1.0 - b, i);
        if (i >= 1) gp -= i * pj * std::pow(1.0 - b, i - 1);
        double hp = dpk * std::pow(1.0 - c, i + j);
        if (i + j >= 1) hp -= (i + j) * pk * std::pow(1.0 - c, i + j - 1);
        const double ta = fa * g_b * h_c;
        pr[m] = sc * 4.0 * ta;
        ps[m] = sc * (2.0 * (1.0 + a) * ta + 2.0 * f * gp * h_c);
        pt[m] = sc * (2.0 * (1.0 + a) * ta + (1.0 + b) * f * gp * h_c + f * g * hp);
      }
}

// orthonormal triangle basis psi_{ij} = sqrt2 p_i(a) p_j^{(2i+1,0)}(b) (1-b)^i
void tri_basis(int N, double u, double v, double* psi) {
  const double a = (std::fabs(1.0 - v) > 1e-14) ? 2.0 * (1.0 + u) / (1.0 - v) - 1.0 : -1.0;
  const double b = v;
  int m = 0;
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N - i; ++j, ++m)
      psi[m] = std::sqrt(2.0) * jacobi(a, 0, 0, i) * jacobi(b, 2.0 * i + 1, 0, j) *
               std::pow(1.0 - b, i);
}

}  // namespace

bool build_ref_element(int N, RefElement& re, std::string& err) {
  if (N < 1 || N > 8) {
    err = "order N must be in [1, 8]";
    return false;
  }
  re = RefElement();
  re.N = N;
  const int Np = re.Np = num_nodes(N);
  const int Nfp = re.Nfp = num_face_nodes(N);
  const int Nq = re.Nq = num_quad(N);
  // equispaced nodes, r fastest, then s, then t
  for (int l = 0; l <= N; ++l)
    for (int k = 0; k <= N - l; ++k)
      for (int j = 0; j <= N - l - k; ++j) {
        re.r.push_back(-1.0 + 2.0 * j / N);
        re.s.push_back(-1.0 + 2.0 * k / N);
        re.t.push_back(-1.0 + 2.0 * l / N);
      }
  std::vector<double> V(Np * Np), Vr(Np * Np), Vs(Np * Np), Vt(Np * Np);
  for (int i = 0; i < Np; ++i)
    tet_basis(N, re.r[i], re.s[i], re.t[i], &V[i * Np], &Vr[i * Np], &Vs[i * Np],
              &Vt[i * Np]);
  std::vector<double> Vi;
  if (!invert(Np, V, Vi)) {
    err = "singular Vandermonde matrix";
    return false;
  }
  re.V = V;
  re.Dr = matmul(Np, Np, Np, Vr, Vi);
  re.Ds = matmul(Np, Np, Np, Vs, Vi);
  re.Dt = matmul(Np, Np, Np, Vt, Vi);
  // M^-1 = V V^T
  re.Minv.assign(Np * Np, 0.0);
  for (int i = 0; i < Np; ++i)
    for (int j = 0; j < Np; ++j) {
      double acc = 0.0;
      for (int m = 0; m < Np; ++m) acc += V[i * Np + m] * V[j * Np + m];
      re.Minv[i * Np + j] = acc;
    }

  // faces: node masks and face-local barycentrics
  re.Fmask.assign(4 * Nfp, -1);
  re.fbary.assign(4 * Nfp * 3, 0.0);
  for (int f = 0; f < 4; ++f) {
    int cnt = 0;
    for (int i = 0; i < Np; ++i) {
      const double r = re.r[i], s = re.s[i], t = re.t[i];
      const double val = (f == 0) ? t : (f == 1) ? s : (f == 2) ? r + s + t : r;
      if (std::fabs(val + 1.0) > 1e-10) continue;
      if (cnt >= Nfp) {
        err = "face node count mismatch";
        return false;
      }
      re.Fmask[f * Nfp + cnt] = i;
      const double lam[4] = {-(1.0 + r + s + t) / 2.0, (1.0 + r) / 2.0,
                             (1.0 + s) / 2.0, (1.0 + t) / 2.0};
      for (int c = 0; c < 3; ++c) re.fbary[(f * Nfp + cnt) * 3 + c] = lam[kFaceVerts[f][c]];
      ++cnt;
    }
    if (cnt != Nfp) {
      err = "face node count mismatch";
      return false;
    }
  }
  // face mass matrices (M_f = (V2 V2^T)^-1 in the face parameters) -> E
  std::vector<double> E(size_t(Np) * 4 * Nfp, 0.0);
  for (int f = 0; f < 4; ++f) {
    std::vector<double> V2(Nfp * Nfp);
    for (int i = 0; i < Nfp; ++i) {
      const int v = re.Fmask[f * Nfp + i];
      double u0, u1;
      if (f == 0) { u0 = re.r[v]; u1 = re.s[v]; }
      else if (f == 1) { u0 = re.r[v]; u1 = re.t[v]; }
      else { u0 = re.s[v]; u1 = re.t[v]; }
      tri_basis(N, u0, u1, &V2[i * Nfp]);
    }
    std::vector<double> VVt(Nfp * Nfp, 0.0), Mf;
    for (int i = 0; i < Nfp; ++i)
      for (int j = 0; j < Nfp; ++j) {
        double acc = 0.0;
        for (int m = 0; m < Nfp; ++m) acc += V2[i * Nfp + m] * V2[j * Nfp + m];
        VVt[i * Nfp + j] = acc;
      }
    if (!invert(Nfp, VVt, Mf)) {
      err = "singular face Vandermonde";
      return false;
    }
    for (int i = 0; i < Nfp; ++i)
      for (int j = 0; j < Nfp; ++j)
        E[size_t(re.Fmask[f * Nfp + i]) * 4 * Nfp + f * Nfp + j] = Mf[i * Nfp + j];
  }
  re.LIFT = matmul(Np, Np, 4 * Nfp, re.Minv, E);

  // quadrature: q = ia + n*(ib + n*ic)
  const int n = N + 1;
  std::vector<double> xa, wa, xb, wb, xc, wc;
  gauss_jacobi(n, 0.0, 0.0, xa, wa);
  gauss_jacobi(n, 1.0, 0.0, xb, wb);
  gauss_jacobi(n, 2.0, 0.0, xc, wc);
  for (int ic = 0; ic < n; ++ic)
    for (int ib = 0; ib < n; ++ib)
      for (int ia = 0; ia < n; ++ia) {
        const double a = xa[ia], b = xb[ib], c = xc[ic];
        re.rq.push_back(0.25 * (1.0 + a) * (1.0 - b) * (1.0 - c) - 1.0);
        re.sq.push_back(0.5 * (1.0 + b) * (1.0 - c) - 1.0);
        re.tq.push_back(c);
        re.wq.push_back(wa[ia] * wb[ib] * wc[ic] / 8.0);
      }
  // Vq = B(quad) V^-1 ; Pq = M^-1 Vq^T W
  std::vector<double> Bq(size_t(Nq) * Np);
  for (int q = 0; q < Nq; ++q)
    tet_basis(N, re.rq[q], re.sq[q], re.tq[q], &Bq[size_t(q) * Np], nullptr, nullptr,
              nullptr);
  re.Vq = matmul(Nq, Np, Np, Bq, Vi);
  std::vector<double> VqTW(size_t(Np) * Nq);
  for (int i = 0; i < Np; ++i)
    for (int q = 0; q < Nq; ++q) VqTW[size_t(i) * Nq + q] = re.Vq[size_t(q) * Np + i] * re.wq[q];
  re.Pq = matmul(Np, Np, Nq, re.Minv, VqTW);
  return true;
}

// ----------------------------------------------------------------- mesh ---
bool build_mesh(const RefElement& re, int64_t K, const double* vxyz,
                const double* period, MeshData& m, std::string& err) {
  if (K <= 0 || !vxyz || !period) {
    err = "mesh: K must be positive and arrays non-null";
    return false;
  }
  if (K > (int64_t(1) << 31) / 8) {
    err = "mesh: too many elements for 32-bit connectivity";
    return false;
  }
  for (int d = 0; d < 3; ++d)
    if (!(period[d] > 0.0) || !std::isfinite(period[d])) {
      err = "mesh: period lengths must be positive and finite";
      return false;
    }
  m = MeshData();
  m.K = K;
  for (int d = 0; d < 3; ++d) m.period[d] = period[d];
  m.vx.assign(vxyz, vxyz + K * 12);
  m.geo.resize(K * 9);
  m.fgeo.resize(K * 16);
  m.J.resize(K);
  // reference outward normals scaled so that |G^T nhat| J is the area element
  // with respect to each face's parameters (face 2 is parametrised by (s,t),
  // whose area is 1/sqrt3 of its true reference area)
  const double nhat[4][3] = {{0, 0, -1}, {0, -1, 0}, {1, 1, 1}, {-1, 0, 0}};
  double vmin = 1e300;
  for (int64_t k = 0; k < K; ++k) {
    const double* X = vxyz + k * 12;
    double F[3][3];  // F[i][j] = d x_i / d rst_j
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) F[i][j] = 0.5 * (X[(j + 1) * 3 + i] - X[i]);
    const double J = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
                     F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                     F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
    if (!(J > 0.0) || !std::isfinite(J)) {
      err = "mesh: element " + std::to_string(k) + " has non-positive orientation";
      return false;
    }
    vmin = std::min(vmin, J);
    // G = F^-1 via the adjugate; G[i][j] = d rst_i / d x_j
    double G[3][3];
    G[0][0] = (F[1][1] * F[2][2] - F[1][2] * F[2][1]) / J;
    G[0][1] = (F[0][2] * F[2][1] - F[0][1] * F[2][2]) / J;
    G[0][2] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) / J;
    G[1][0] = (F[1][2] * F[2][0] - F[1][0] * F[2][2]) / J;
    G[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) / J;
    G[1][2] = (F[0][2] * F[1][0] - F[0][0] * F[1][2]) / J;
    G[2][0] = (F[1][0] * F[2][1] - F[1][1] * F[2][0]) / J;
    G[2][1] = (F[0][1] * F[2][0] - F[0][0] * F[2][1]) / J;
    G[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) / J;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) m.geo[k * 9 + i * 3 + j] = G[i][j];
    m.J[k] = J;
    for (int f = 0; f < 4; ++f) {
      double nv[3];
      for (int j = 0; j < 3; ++j)
        nv[j] = G[0][j] * nhat[f][0] + G[1][j] * nhat[f][1] + G[2][j] * nhat[f][2];
      const double len = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
      const double sJ = J * len;
      for (int j = 0; j < 3; ++j) m.fgeo[k * 16 + f * 4 + j] = nv[j] / len;
      m.fgeo[k * 16 + f * 4 + 3] = sJ / J;
    }
  }

  // face matching: key = centroid modulo the period on a fine lattice
  const double delta = 1e-7 * std::cbrt(vmin);
  long long wrap[3];
  for (int d = 0; d < 3; ++d) wrap[d] = std::llround(period[d] / delta);
  struct FaceKey {
    std::array<long long, 3> key;
    int64_t id;
  };
  std::vector<FaceKey> keys(K * 4);
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) {
      FaceKey fk;
      for (int d = 0; d < 3; ++d) {
        double c = 0.0;
        for (int v = 0; v < 3; ++v) c += vxyz[k * 12 + kFaceVerts[f][v] * 3 + d];
        c /= 3.0;
        c -= period[d] * std::floor(c / period[d]);
        long long q = std::llround(c / delta) % wrap[d];
        if (q < 0) q += wrap[d];
        fk.key[d] = q;
      }
      fk.id = k * 4 + f;
      keys[k * 4 + f] = fk;
    }
  std::sort(keys.begin(), keys.end(), [](const FaceKey& a, const FaceKey& b) {
    return a.key < b.key || (a.key == b.key && a.id < b.id);
  });
  m.EToE.assign(K * 4, -1);
  m.EToF.assign(K * 4, 0);
  m.EToP.assign(K * 4, 0);
  for (size_t i = 0; i < keys.size(); i += 2) {
    if (i + 1 >= keys.size() || keys[i].key != keys[i + 1].key ||
        (i + 2 < keys.size() && keys[i + 2].key == keys[i].key)) {
      err = "mesh: face matching failed (a face is not shared by exactly two "
            "elements of the periodic mesh)";
      return false;
    }
    const int64_t a = keys[i].id, b = keys[i + 1].id;
    m.EToE[a] = int32_t(b / 4);
    m.EToF[a] = uint8_t(b % 4);
    m.EToE[b] = int32_t(a / 4);
    m.EToF[b] = uint8_t(a % 4);
  }

  // trace patterns: vertex correspondence of the two faces (after the
  // periodic shift) -> permutation sigma; pattern (f, f', sigma) maps own
  // face node i to the neighbour volume node with permuted face barycentrics
  const int Nfp = re.Nfp;
  std::map<std::tuple<int, int, int, int, int>, int> pat_id;
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) {
      const int64_t nb = m.EToE[k * 4 + f];
      const int nf = m.EToF[k * 4 + f];
      double ca[3] = {0, 0, 0}, cb[3] = {0, 0, 0};
      for (int v = 0; v < 3; ++v)
        for (int d = 0; d < 3; ++d) {
          ca[d] += vxyz[k * 12 + kFaceVerts[f][v] * 3 + d] / 3.0;
          cb[d] += vxyz[nb * 12 + kFaceVerts[nf][v] * 3 + d] / 3.0;
        }
      double shift[3];
      for (int d = 0; d < 3; ++d)
        shift[d] = period[d] * std::round((ca[d] - cb[d]) / period[d]);
      int sigma[3];
      for (int c = 0; c < 3; ++c) {
        sigma[c] = -1;
        const double* A = vxyz + k * 12 + kFaceVerts[f][c] * 3;
        for (int e = 0; e < 3; ++e) {
          const double* B = vxyz + nb * 12 + kFaceVerts[nf][e] * 3;
          double dist = 0.0;
          for (int d = 0; d < 3; ++d) dist += std::fabs(A[d] - B[d] - shift[d]);
          if (dist < 1e3 * delta) sigma[c] = e;
        }
        if (sigma[c] < 0) {
          err = "mesh: matched faces do not share vertices";
          return false;
        }
      }
      const auto key = std::make_tuple(f, nf, sigma[0], sigma[1], sigma[2]);
      auto it = pat_id.find(key);
      int id;
      if (it == pat_id.end()) {
        id = int(pat_id.size());
        pat_id[key] = id;
        m.pat.resize(size_t(id + 1) * Nfp);
        for (int i = 0; i < Nfp; ++i) {
          const double* lam = &re.fbary[(f * Nfp + i) * 3];
          int found = -1;
          for (int j = 0; j < Nfp; ++j) {
            const double* mu = &re.fbary[(nf * Nfp + j) * 3];
            double dd = 0.0;
            for (int c = 0; c < 3; ++c) dd += std::fabs(mu[sigma[c]] - lam[c]);
            if (dd < 1e-10) found = j;
          }
          if (found < 0) {
            err = "mesh: face node permutation not found";
            return false;
          }
          m.pat[size_t(id) * Nfp + i] = re.Fmask[nf * Nfp + found];
        }
      } else {
        id = it->second;
      }
      m.EToP[k * 4 + f] = uint8_t(id);
    }
  m.npat = int(pat_id.size());
  return true;
}

std::vector<int32_t> neighbour_nodes(const RefElement& re, const MeshData& m) {
  const int Nfp = re.Nfp, NF4 = 4 * Nfp, Np = re.Np;
  std::vector<int32_t> out(size_t(m.K) * NF4);
  for (int64_t k = 0; k < m.K; ++k)
    for (int f = 0; f < 4; ++f) {
      const int64_t nb = m.EToE[k * 4 + f];
      const int32_t* pt = &m.pat[size_t(m.EToP[k * 4 + f]) * Nfp];
      for (int i = 0; i < Nfp; ++i) out[size_t(k) * NF4 + f * Nfp + i] = int32_t(nb * Np + pt[i]);
    }
  return out;
}

bool adjoint_face_tables(const RefElement& re, const MeshData& m, std::vector<int32_t>& nbface,
                         std::vector<int32_t>& invf, std::string& err) {
  const int Nfp = re.Nfp, NF4 = 4 * Nfp, Np = re.Np;
  nbface.assign(size_t(m.K) * NF4, 0);
  invf.assign(size_t(Np) * 3, -1);
  for (int64_t k = 0; k < m.K; ++k)
    for (int f = 0; f < 4; ++f) {
      const int64_t nb = m.EToE[k * 4 + f];
      const int fn = m.EToF[k * 4 + f];
      for (int i = 0; i < Nfp; ++i) {
        const int vP = m.pat[size_t(m.EToP[k * 4 + f]) * Nfp + i];
        int jn = -1;
        for (int i2 = 0; i2 < Nfp; ++i2)
          if (re.Fmask[fn * Nfp + i2] == vP) jn = fn * Nfp + i2;
        if (jn < 0) {
          err = "adjoint: face tables inconsistent";
          return false;
        }
        nbface[size_t(k) * NF4 + f * Nfp + i] = int32_t(nb * NF4 + jn);
      }
    }
  for (int j = 0; j < NF4; ++j) {
    const int n = re.Fmask[j];
    int s = 0;
    while (s < 3 && invf[n * 3 + s] >= 0) ++s;
    if (s == 3) {
      err = "adjoint: node on more than three faces";
      return false;
    }
    invf[n * 3 + s] = j;
  }
  return true;
}

std::vector<int32_t> tile_order(const MeshData& m, int tile, int parts) {
  const int64_t K = m.K, T = (K + tile - 1) / tile;
  std::vector<double> c(size_t(T) * 3, 0.0);
  double vol = 0.0;
  for (int64_t k = 0; k < K; ++k) {
    const int64_t t = k / tile;
    const int64_t nt = std::min<int64_t>(tile, K - t * tile);
    for (int d = 0; d < 3; ++d) {
      double x = 0.0;
      for (int v = 0; v < 4; ++v) x += m.vx[size_t(k) * 12 + v * 3 + d];
      c[size_t(t) * 3 + d] += x / (4.0 * double(nt));
    }
    vol += std::fabs(m.J[k]) * 4.0 / 3.0;   // reference tet volume 4/3
  }
  // typical element length: the edge of a cube of six elements' volume
  const double h = K > 0 ? std::cbrt(6.0 * vol / double(K)) : 1.0;
  std::vector<int32_t> ord(static_cast<size_t>(T));
  for (int64_t t = 0; t < T; ++t) ord[size_t(t)] = int32_t(t);
  // axis of largest centroid extent over ord[b, e); ties go to the higher axis
  auto longest = [&](int64_t b, int64_t e, int skip) {
    int best = -1;
    double ext = -1.0;
    for (int d = 2; d >= 0; --d) {
      if (d == skip) continue;
      double lo = 1e300, hi = -1e300;
      for (int64_t i = b; i < e; ++i) {
        const double x = c[size_t(ord[size_t(i)]) * 3 + d];
        lo = std::min(lo, x);
        hi = std::max(hi, x);
      }
      if (hi - lo > ext * (1.0 + 1e-9) + 1e-12) { ext = hi - lo; best = d; }
    }
    return best;
  };
  auto sweep = [&](int64_t b, int64_t e, int d) {
    double lo = 1e300;
    for (int64_t i = b; i < e; ++i) lo = std::min(lo, c[size_t(ord[size_t(i)]) * 3 + d]);
    std::stable_sort(ord.begin() + b, ord.begin() + e, [&](int32_t x, int32_t y) {
      // bucket boundaries half a length above the multiples of h: tiles of
      // one layer sit at or just above them, not straddling
      const int64_t bx = int64_t(std::floor((c[size_t(x) * 3 + d] - lo) / h + 0.5));
      const int64_t by = int64_t(std::floor((c[size_t(y) * 3 + d] - lo) / h + 0.5));
      return bx != by ? bx < by : x < y;
    });
  };
  // Within a slab, strips of kStrip typical lengths across the sweep axis:
  // the slab is swept strip by strip, so the tiles a sweep step covers (the
  // strip's cross-section) are few and face neighbours along every axis
  // inside a strip run a cross-section apart, within reach of the XCD's L2;
  // only the neighbours across a strip boundary are far apart.
  constexpr int kStrip = 8;
  auto strip_sweep = [&](int64_t b, int64_t e, int du, int dv) {
    double lu = 1e300, lv = 1e300;
    for (int64_t i = b; i < e; ++i) {
      lu = std::min(lu, c[size_t(ord[size_t(i)]) * 3 + du]);
      lv = std::min(lv, c[size_t(ord[size_t(i)]) * 3 + dv]);
    }
    auto bucket = [&](int32_t t, int d, double lo) {
      return int64_t(std::floor((c[size_t(t) * 3 + d] - lo) / h + 0.5));
    };
    std::stable_sort(ord.begin() + b, ord.begin() + e, [&](int32_t x, int32_t y) {
      const int64_t sx = bucket(x, dv, lv) / kStrip, sy = bucket(y, dv, lv) / kStrip;
      if (sx != sy) return sx < sy;
      const int64_t ux = bucket(x, du, lu), uy = bucket(y, du, lu);
      return ux != uy ? ux < uy : x < y;
    });
  };
  if (T == 0) return ord;
  const int a0 = longest(0, T, -1);
  sweep(0, T, a0);
  const int64_t per = T / parts, rem = T % parts;
  for (int x = 0; x < parts; ++x) {
    const int64_t b = x * per + std::min<int64_t>(x, rem);
    const int64_t e = b + per + (x < rem ? 1 : 0);
    if (e - b < 2) continue;
    std::sort(ord.begin() + b, ord.begin() + e);   // element order within the slab
    const int du = longest(b, e, a0);               // sweep axis
    const int dv = 3 - a0 - du;                     // strip axis
    strip_sweep(b, e, du, dv);
  }
  return ord;
}

void basis_at(const RefElement& re, double r, double s, double t, double* psi) {
  tet_basis(re.N, r, s, t, psi, nullptr, nullptr, nullptr);
}

bool locate_point(const RefElement& re, const MeshData& m, const double* x, int64_t& k,
                  double* rst) {
  (void)re;
  for (int64_t e = 0; e < m.K; ++e) {
    // r + 1 = (d r / d x) (x - x_0) for the affine map of element e, with
    // x - x_0 taken as the nearest periodic image (elements are smaller
    // than half the period)
    const double* v0 = &m.vx[size_t(e) * 12];
    const double* G = &m.geo[size_t(e) * 9];
    double dx[3];
    for (int d = 0; d < 3; ++d) {
      dx[d] = x[d] - v0[d];
      dx[d] -= m.period[d] * std::nearbyint(dx[d] / m.period[d]);
    }
    double lo[3], mn = 1.0;
    for (int i = 0; i < 3; ++i) {
      lo[i] = G[i * 3 + 0] * dx[0] + G[i * 3 + 1] * dx[1] + G[i * 3 + 2] * dx[2] - 1.0;
      mn = std::min(mn, (1.0 + lo[i]) / 2.0);
    }
    mn = std::min(mn, -(1.0 + lo[0] + lo[1] + lo[2]) / 2.0);
    if (mn >= -1e-12) {
      k = e;
      for (int i = 0; i < 3; ++i) rst[i] = lo[i];
      return true;
    }
  }
  return false;
}

static void map_points(const RefElement& re, const MeshData& m, const std::vector<double>& r,
                       const std::vector<double>& s, const std::vector<double>& t,
                       double* out) {
  const size_t np = r.size();
  for (int64_t k = 0; k < m.K; ++k) {
    const double* X = &m.vx[k * 12];
    for (size_t p = 0; p < np; ++p)
      for (int d = 0; d < 3; ++d) {
        const double x0 = X[d];
        out[(k * np + p) * 3 + d] =
            x0 + 0.5 * ((X[3 + d] - x0) * (r[p] + 1.0) + (X[6 + d] - x0) * (s[p] + 1.0) +
                        (X[9 + d] - x0) * (t[p] + 1.0));
      }
  }
  (void)re;
}

void node_coords(const RefElement& re, const MeshData& m, double* out) {
  map_points(re, m, re.r, re.s, re.t, out);
}
void quad_coords(const RefElement& re, const MeshData& m, double* out) {
  map_points(re, m, re.rq, re.sq, re.tq, out);
}

}  // namespace dgh
