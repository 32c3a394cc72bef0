"""Reference tetrahedron for the oracle: nodes, orthonormal basis, derivative
matrices, face mass matrices, LIFT, quadrature, interpolation to and
projection from quadrature points.  Plain FP64 NumPy/SciPy.

Reference tetrahedron: vertices (-1,-1,-1), (1,-1,-1), (-1,1,-1), (-1,-1,1).
Faces (numbering of [HW08] Ch. 10):
    face 0: t = -1          (parametrised by (r, s))
    face 1: s = -1          (parametrised by (r, t))
    face 2: r + s + t = -1  (parametrised by (s, t))
    face 3: r = -1          (parametrised by (s, t))

Nodes: the equispaced nodal set of degree N, enumerated with the t-index
outermost, then the s-index, then the r-index (r fastest).  The semi-discrete
operator on polynomials does not depend on this choice where the impedance is
constant on each face (tested in tests/test_oracle_pins.py).

Pins (tests/test_oracle_pins.py): derivative matrices exact on monomials;
quadrature exact on barycentric monomials (closed form); mass and face mass
against a monomial Gram matrix with the closed-form simplex integral;
summation-by-parts identity linking Dr, the mass matrix and face masses;
P_q V_q = I.
"""
from __future__ import annotations

from dataclasses import dataclass
from functools import lru_cache

import numpy as np
from scipy.special import eval_jacobi, gammaln, roots_jacobi

REF_VERTS = np.array([[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0],
                      [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]])
# vertex indices of each face, in the order used for its parametrisation
FACE_VERTS = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))


def n_nodes(N):
    return (N + 1) * (N + 2) * (N + 3) // 6


def n_face_nodes(N):
    return (N + 1) * (N + 2) // 2


# --------------------------------------------------------------------------
# orthonormal Jacobi polynomials (via scipy's classical Jacobi polynomials
# and their closed-form norm)
# --------------------------------------------------------------------------

def _jacobi_norm2(n, a, b):
    """Squared L2 norm of P_n^{(a,b)} with weight (1-x)^a (1+x)^b on [-1,1]."""
    return np.exp((a + b + 1) * np.log(2.0) - np.log(2 * n + a + b + 1)
                  + gammaln(n + a + 1) + gammaln(n + b + 1)
                  - gammaln(n + a + b + 1) - gammaln(n + 1))


def jacobi_p(n, a, b, x):
    """Orthonormal Jacobi polynomial of degree n."""
    return eval_jacobi(n, a, b, x) / np.sqrt(_jacobi_norm2(n, a, b))


def jacobi_dp(n, a, b, x):
    """Derivative of the orthonormal Jacobi polynomial of degree n, from
    d/dx P_n^{(a,b)} = (n + a + b + 1)/2 P_{n-1}^{(a+1,b+1)}."""
    if n == 0:
        return np.zeros_like(np.asarray(x, dtype=np.float64))
    d = 0.5 * (n + a + b + 1) * eval_jacobi(n - 1, a + 1, b + 1, x)
    return d / np.sqrt(_jacobi_norm2(n, a, b))


# --------------------------------------------------------------------------
# nodes and basis
# --------------------------------------------------------------------------

def equispaced_nodes(N):
    """Equispaced nodes of degree N on the reference tetrahedron, r fastest,
    then s, then t."""
    pts = []
    for l in range(N + 1):
        for k in range(N + 1 - l):
            for j in range(N + 1 - l - k):
                pts.append((-1.0 + 2.0 * j / N, -1.0 + 2.0 * k / N,
                            -1.0 + 2.0 * l / N))
    return np.array(pts)


def warped_nodes(N):
    """An alternative symmetric nodal set used only to show that the DG
    operator does not depend on the nodal basis: barycentric coordinates
    lam_m = g(i_m) / sum_n g(i_n), where g(i) = (1 + x_i)/2 and x_i are the
    Gauss-Lobatto-Legendre points; faces and edges map onto themselves and
    edges carry the Gauss-Lobatto-Legendre distribution."""
    if N == 1:
        u = np.array([0.0, 1.0])
    else:
        xi = np.sort(roots_jacobi(N - 1, 1, 1)[0])
        u = 0.5 * (1.0 + np.concatenate([[-1.0], xi, [1.0]]))
    pts = []
    for l in range(N + 1):
        for k in range(N + 1 - l):
            for j in range(N + 1 - l - k):
                i = N - j - k - l
                g = u[[i, j, k, l]]
                lam = g / g.sum()
                pts.append(lam @ REF_VERTS)
    return np.array(pts)


def _collapse(r, s, t):
    """Collapsed coordinates (a, b, c) of [HW08] Ch. 10; the singular edge
    s + t = 0 and apex t = 1 are given a = -1 / b = -1 (the basis and its
    gradient below are written so that these values do not matter)."""
    r, s, t = (np.asarray(v, dtype=np.float64) for v in (r, s, t))
    den_a = -s - t
    den_b = 1.0 - t
    ok_a = np.abs(den_a) > 1e-14
    ok_b = np.abs(den_b) > 1e-14
    a = np.where(ok_a, 2.0 * (1.0 + r) / np.where(ok_a, den_a, 1.0) - 1.0, -1.0)
    b = np.where(ok_b, 2.0 * (1.0 + s) / np.where(ok_b, den_b, 1.0) - 1.0, -1.0)
    return a, b, t


def mode_indices(N):
    """(i, j, k) of each orthonormal mode, i outermost."""
    return [(i, j, k) for i in range(N + 1) for j in range(N + 1 - i)
            for k in range(N + 1 - i - j)]


def basis(N, r, s, t):
    """Orthonormal tetrahedral basis [HW08, eq. 10.6 ff.] at points: returns
    V [npts, Np] with V[p, m] = phi_m(r_p, s_p, t_p)."""
    a, b, c = _collapse(r, s, t)
    cols = []
    for (i, j, k) in mode_indices(N):
        f = jacobi_p(i, 0, 0, a)
        g = jacobi_p(j, 2 * i + 1, 0, b) * (1.0 - b) ** i
        h = jacobi_p(k, 2 * i + 2 * j + 2, 0, c) * (1.0 - c) ** (i + j)
        cols.append(2.0 * np.sqrt(2.0) * f * g * h)
    return np.stack(cols, axis=-1)


def basis_grad(N, r, s, t):
    """Gradient of the orthonormal basis with respect to (r, s, t).

    With phi = f(a) g(b) h(c), g = P_j(b)(1-b)^i, h = P_k(c)(1-c)^(i+j), the
    chain rule through the collapse gives
      d/dr = 4/((1-b)(1-c)) f' g h
      d/ds = 2(1+a)/((1-b)(1-c)) f' g h + 2/(1-c) f g' h
      d/dt = 2(1+a)/((1-b)(1-c)) f' g h + (1+b)/(1-c) f g' h + f g h'
    and each division is cancelled against the explicit (1-b)^i, (1-c)^(i+j)
    factors (f' = 0 when i = 0, g' = 0 when i + j = 0), so the expressions
    are polynomial and valid on the singular edge and apex."""
    a, b, c = _collapse(r, s, t)
    dr, ds, dt = [], [], []
    for (i, j, k) in mode_indices(N):
        f = jacobi_p(i, 0, 0, a)
        fa = jacobi_dp(i, 0, 0, a)
        Pj = jacobi_p(j, 2 * i + 1, 0, b)
        dPj = jacobi_dp(j, 2 * i + 1, 0, b)
        Pk = jacobi_p(k, 2 * i + 2 * j + 2, 0, c)
        dPk = jacobi_dp(k, 2 * i + 2 * j + 2, 0, c)
        # g/(1-b), h/(1-c): only needed when the matching numerator is nonzero
        g_over = Pj * (1.0 - b) ** (i - 1) if i >= 1 else np.zeros_like(b)
        h_over = Pk * (1.0 - c) ** (i + j - 1) if i + j >= 1 else np.zeros_like(c)
        g = Pj * (1.0 - b) ** i
        h = Pk * (1.0 - c) ** (i + j)
        gb = dPj * (1.0 - b) ** i
        if i >= 1:
            gb = gb - i * Pj * (1.0 - b) ** (i - 1)
        hc = dPk * (1.0 - c) ** (i + j)
        if i + j >= 1:
            hc = hc - (i + j) * Pk * (1.0 - c) ** (i + j - 1)
        term_a = fa * g_over * h_over          # f' g h / ((1-b)(1-c))
        vr = 4.0 * term_a
        vs = 2.0 * (1.0 + a) * term_a + 2.0 * f * gb * h_over
        vt = (2.0 * (1.0 + a) * term_a + (1.0 + b) * f * gb * h_over
              + f * g * hc)
        sc = 2.0 * np.sqrt(2.0)
        dr.append(sc * vr)
        ds.append(sc * vs)
        dt.append(sc * vt)
    return (np.stack(dr, axis=-1), np.stack(ds, axis=-1),
            np.stack(dt, axis=-1))


# --------------------------------------------------------------------------
# quadrature
# --------------------------------------------------------------------------

def tet_quadrature(N):
    """Collapsed (Stroud conical-product) Gauss-Jacobi rule with N+1 points
    per direction: weights (1-a)^0, (1-b)^1, (1-c)^2 in the collapsed
    coordinates, exact for polynomials of total degree 2N+1 on the reference
    tetrahedron.  Point q = ia + (N+1)*(ib + (N+1)*ic) (a fastest).
    Returns (r, s, t, w)."""
    n = N + 1
    xa, wa = roots_jacobi(n, 0, 0)
    xb, wb = roots_jacobi(n, 1, 0)
    xc, wc = roots_jacobi(n, 2, 0)
    A, B, C = np.meshgrid(xa, xb, xc, indexing="ij")
    WA, WB, WC = np.meshgrid(wa, wb, wc, indexing="ij")
    # q = ia + n*(ib + n*ic): transpose so a varies fastest when raveled
    A, B, C = (M.transpose(2, 1, 0).ravel() for M in (A, B, C))
    W = (WA * WB * WC).transpose(2, 1, 0).ravel() / 8.0
    r = 0.25 * (1.0 + A) * (1.0 - B) * (1.0 - C) - 1.0
    s = 0.5 * (1.0 + B) * (1.0 - C) - 1.0
    t = C
    return r, s, t, W


def tri_quadrature(N):
    """Collapsed Gauss-Jacobi rule on the reference triangle
    {(x, y): x, y >= -1, x + y <= 0}, exact for degree 2N+1."""
    n = N + 1
    xa, wa = roots_jacobi(n, 0, 0)
    xb, wb = roots_jacobi(n, 1, 0)
    A, B = np.meshgrid(xa, xb, indexing="ij")
    WA, WB = np.meshgrid(wa, wb, indexing="ij")
    x = 0.5 * (1.0 + A) * (1.0 - B) - 1.0
    y = B
    return x.ravel(), y.ravel(), (WA * WB).ravel() / 2.0


def face_point(f, u, v):
    """Map face parameters (u, v) on the reference triangle to (r, s, t) on
    face f of the reference tetrahedron."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    m1 = -np.ones_like(u)
    if f == 0:
        return u, v, m1
    if f == 1:
        return u, m1, v
    if f == 2:
        return -1.0 - u - v, u, v
    if f == 3:
        return m1, u, v
    raise ValueError(f)


def face_params(f, r, s, t):
    """Inverse of face_point restricted to face f."""
    return {0: (r, s), 1: (r, t), 2: (s, t), 3: (s, t)}[f]


# --------------------------------------------------------------------------
# the reference element
# --------------------------------------------------------------------------

@dataclass
class RefElement:
    N: int
    Np: int
    Nfp: int
    Nq: int
    r: np.ndarray
    s: np.ndarray
    t: np.ndarray
    V: np.ndarray          # Vandermonde [Np, Np] (rows: nodes, cols: modes)
    Dr: np.ndarray
    Ds: np.ndarray
    Dt: np.ndarray
    M: np.ndarray          # reference mass matrix (nodal)
    Minv: np.ndarray
    Fmask: np.ndarray      # [4, Nfp] volume-node index of each face node
    Ef: np.ndarray         # [4, Np, Nfp] face mass (param coords) at face columns
    LIFT: np.ndarray       # [Np, 4*Nfp]
    rq: np.ndarray
    sq: np.ndarray
    tq: np.ndarray
    wq: np.ndarray
    Vq: np.ndarray         # [Nq, Np] nodal -> quadrature interpolation
    Pq: np.ndarray         # [Np, Nq] quadrature -> nodal L2 projection


@lru_cache(maxsize=None)
def ref_element(N: int, nodes: str = "equi") -> RefElement:
    if N < 1:
        raise ValueError("order N must be >= 1")
    pts = equispaced_nodes(N) if nodes == "equi" else warped_nodes(N)
    r, s, t = pts.T
    Np = n_nodes(N)
    Nfp = n_face_nodes(N)
    V = basis(N, r, s, t)
    Vr, Vs, Vt = basis_grad(N, r, s, t)
    Vinv = np.linalg.inv(V)
    Dr, Ds, Dt = Vr @ Vinv, Vs @ Vinv, Vt @ Vinv

    # quadrature and nodal interpolation to it
    rq, sq, tq, wq = tet_quadrature(N)
    Vq = basis(N, rq, sq, tq) @ Vinv
    # nodal mass matrix by quadrature (degree 2N integrand, rule exact to 2N+1)
    M = Vq.T @ (wq[:, None] * Vq)
    Minv = np.linalg.inv(M)
    Pq = Minv @ (Vq.T * wq[None, :])

    # face nodes: volume nodes with the face's defining coordinate at -1
    tol = 1e-10
    conds = (np.abs(1 + t) < tol, np.abs(1 + s) < tol,
             np.abs(1 + r + s + t) < tol, np.abs(1 + r) < tol)
    Fmask = np.array([np.nonzero(cnd)[0] for cnd in conds])
    assert Fmask.shape == (4, Nfp)

    # face mass by quadrature in the face parameters: the volume Lagrange
    # basis restricted to the face is the face Lagrange basis
    uq, vq, wfq = tri_quadrature(N)
    Ef = np.zeros((4, Np, Nfp))
    for f in range(4):
        rf, sf, tf = face_point(f, uq, vq)
        L = basis(N, rf, sf, tf) @ Vinv          # [nfq, Np]
        Mf = L.T @ (wfq[:, None] * L)            # [Np, Np]
        Ef[f] = Mf[:, Fmask[f]]
    E = np.concatenate([Ef[f] for f in range(4)], axis=1)   # [Np, 4 Nfp]
    LIFT = Minv @ E
    return RefElement(N=N, Np=Np, Nfp=Nfp, Nq=len(wq), r=r, s=s, t=t, V=V,
                      Dr=Dr, Ds=Ds, Dt=Dt, M=M, Minv=Minv, Fmask=Fmask,
                      Ef=Ef, LIFT=LIFT, rq=rq, sq=sq, tq=tq, wq=wq, Vq=Vq,
                      Pq=Pq)
