"""Pins of the oracle's reference element and mesh against closed forms and
brute force that do not use the oracle's own construction route
(orthonormal basis + Vandermonde inverse + Gauss-Jacobi quadrature)."""
from itertools import product
from math import factorial

import numpy as np
import pytest

from oracle.mesh import build_mesh
from oracle.refelem import (REF_VERTS, face_point, n_face_nodes, n_nodes,
                            ref_element, tet_quadrature, basis)


def _unit_tet_monomial_integral(a, b, c):
    """int over {x,y,z >= 0, x+y+z <= 1} of x^a y^b z^c = a! b! c! / (a+b+c+3)!"""
    return factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)


def _unit_tri_monomial_integral(a, b):
    return factorial(a) * factorial(b) / factorial(a + b + 2)


def _exponents3(deg):
    return [(a, b, c) for a in range(deg + 1) for b in range(deg + 1 - a)
            for c in range(deg + 1 - a - b)]


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7])
def test_quadrature_exact_degree_2N_plus_1(N):
    r, s, t, w = tet_quadrature(N)
    assert np.all(w > 0)
    x, y, z = (1 + r) / 2, (1 + s) / 2, (1 + t) / 2    # unit tet, dV_ref = 8 dV
    for (a, b, c) in _exponents3(2 * N + 1):
        got = np.sum(w * x**a * y**b * z**c)
        ref = 8.0 * _unit_tet_monomial_integral(a, b, c)
        assert abs(got - ref) <= 1e-14 * max(1.0, abs(ref)) + 1e-16, (a, b, c)
    # degree 2N+2 is generally not integrated exactly (the rule is not overkill)
    errs = [abs(np.sum(w * x**a * y**b * z**c) - 8.0 * _unit_tet_monomial_integral(a, b, c))
            for (a, b, c) in _exponents3(2 * N + 2) if a + b + c == 2 * N + 2]
    assert max(errs) > 1e-12


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7])
def test_derivative_matrices_exact_on_monomials(N):
    re = ref_element(N)
    r, s, t = re.r, re.s, re.t
    scale = max(1.0, np.abs(re.Dr).max())
    for (a, b, c) in _exponents3(N):
        u = r**a * s**b * t**c
        ur = a * r**max(a - 1, 0) * s**b * t**c
        us = b * r**a * s**max(b - 1, 0) * t**c
        ut = c * r**a * s**b * t**max(c - 1, 0)
        for D, du in ((re.Dr, ur), (re.Ds, us), (re.Dt, ut)):
            assert np.abs(D @ u - du).max() < 1e-13 * scale * re.Np


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_mass_matrices_against_monomial_gram(N):
    """Nodal mass and face mass from monomials in (x, y, z) = ((1+r)/2, ...)
    and the closed-form simplex integrals, with no orthonormal basis."""
    re = ref_element(N)
    ex = _exponents3(N)
    x, y, z = (1 + re.r) / 2, (1 + re.s) / 2, (1 + re.t) / 2
    Vm = np.stack([x**a * y**b * z**c for (a, b, c) in ex], axis=1)
    C = np.linalg.inv(Vm)                       # Lagrange coefficients
    G = np.array([[8.0 * _unit_tet_monomial_integral(a1 + a2, b1 + b2, c1 + c2)
                   for (a2, b2, c2) in ex] for (a1, b1, c1) in ex])
    M_bf = C.T @ G @ C
    assert np.abs(M_bf - re.M).max() < 1e-12 * np.abs(re.M).max()
    # face masses: face Lagrange basis from 2D monomials in the face params
    ex2 = [(a, b) for a in range(N + 1) for b in range(N + 1 - a)]
    for f in range(4):
        idx = re.Fmask[f]
        u, v = {0: (re.r, re.s), 1: (re.r, re.t), 2: (re.s, re.t),
                3: (re.s, re.t)}[f]
        X, Y = (1 + u[idx]) / 2, (1 + v[idx]) / 2
        V2 = np.stack([X**a * Y**b for (a, b) in ex2], axis=1)
        C2 = np.linalg.inv(V2)
        G2 = np.array([[4.0 * _unit_tri_monomial_integral(a1 + a2, b1 + b2)
                        for (a2, b2) in ex2] for (a1, b1) in ex2])
        Mf = C2.T @ G2 @ C2
        assert np.abs(re.Ef[f][idx] - Mf).max() < 1e-12 * np.abs(Mf).max()
        other = np.setdiff1d(np.arange(re.Np), idx)
        assert np.abs(re.Ef[f][other]).max() < 1e-13


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7])
def test_summation_by_parts(N):
    """int (l_i d_r l_j + d_r l_i l_j) = surface integral of l_i l_j n_r.
    Reference outward normals times face area scale (param-area element):
    d/dr: +1 on face 2, -1 on face 3; d/ds: -1 on face 1, +1 on face 2;
    d/dt: -1 on face 0, +1 on face 2."""
    re = ref_element(N)

    def Efull(f):
        E = np.zeros((re.Np, re.Np))
        E[:, re.Fmask[f]] = re.Ef[f]
        return E
    sgn = {"r": {2: 1, 3: -1}, "s": {1: -1, 2: 1}, "t": {0: -1, 2: 1}}
    for key, D in (("r", re.Dr), ("s", re.Ds), ("t", re.Dt)):
        lhs = re.M @ D + (re.M @ D).T
        rhs = sum(c * Efull(f) for f, c in sgn[key].items())
        assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7])
def test_projection_interpolation_identities(N):
    re = ref_element(N)
    assert np.abs(re.Pq @ re.Vq - np.eye(re.Np)).max() < 1e-12
    # orthonormality of the modal basis under the quadrature
    Bq = basis(N, re.rq, re.sq, re.tq)
    assert np.abs(Bq.T @ (re.wq[:, None] * Bq) - np.eye(re.Np)).max() < 1e-13
    # Vq reproduces polynomials of degree N at the quadrature points
    for (a, b, c) in _exponents3(N):
        u = re.r**a * re.s**b * re.t**c
        uq = re.rq**a * re.sq**b * re.tq**c
        assert np.abs(re.Vq @ u - uq).max() < 1e-12
    assert re.Np == n_nodes(N) and re.Nfp == n_face_nodes(N)
    assert re.Nq == (N + 1) ** 3


def test_face_nodes_lie_on_faces():
    for N in (1, 3, 5):
        re = ref_element(N)
        pts = np.stack([re.r, re.s, re.t], axis=1)
        for f in range(4):
            vals = {0: pts[:, 2], 1: pts[:, 1], 2: pts.sum(1), 3: pts[:, 0]}[f]
            target = {0: -1, 1: -1, 2: -1, 3: -1}[f]
            assert np.allclose(vals[re.Fmask[f]], target)


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("N", [1, 3])
def test_mesh_geometry_and_connectivity(n, N):
    re = ref_element(N)
    m = build_mesh(n, re)
    assert m.K == 6 * n**3
    vol = m.J * 4.0 / 3.0
    assert np.all(vol > 0)
    assert abs(vol.sum() - 1.0) < 1e-13
    # each element's volume from its vertices (independent of the ref map)
    VX = m.VX
    det = np.linalg.det(np.stack([VX[:, 1] - VX[:, 0], VX[:, 2] - VX[:, 0],
                                  VX[:, 3] - VX[:, 0]], axis=-1)) / 6.0
    assert np.allclose(det, vol)
    # neighbours are reciprocal; normals opposite; area elements equal
    k = np.arange(m.K)
    for f in range(4):
        nb, nf = m.EToE[:, f], m.EToF[:, f]
        assert np.all(m.EToE[nb, nf] == k)
        assert np.all(m.EToF[nb, nf] == f)
        assert np.allclose(m.nrm[nb, nf], -m.nrm[:, f], atol=1e-14)
        assert np.allclose(m.sJ[nb, nf], m.sJ[:, f], rtol=1e-14)
    # unit normals; each face normal is orthogonal to the face's edges
    assert np.allclose(np.linalg.norm(m.nrm, axis=-1), 1.0)
    # paired trace nodes coincide modulo the period
    xf = m.x.reshape(-1, 3)
    d = xf[m.vmapM] - xf[m.vmapP]
    d -= np.rint(d)
    assert np.abs(d).max() < 1e-12
    # the face area elements sum (times reference area 2) to the surface area
    # of n^3 cubes' worth of internal/periodic faces: each hex face of side H
    # is cut into two triangles; total area counted from both sides.
    area = (2.0 * m.sJ).sum()
    H = 1.0 / n
    # per hex: 6 boundary triangles-pairs (12 tris, area H^2/2 each, shared by
    # two hexes) plus 6 interior faces of the Kuhn split (2 per diagonal plane)
    interior = 6 * (np.sqrt(2.0) * H * H / 2.0)   # six triangles of area sqrt2 H^2/2
    boundary = 12 * (H * H / 2.0)
    # sum over elements of their 4 faces = 2 * (number of distinct faces area)
    assert abs(area - n**3 * (2 * interior + boundary)) < 1e-10


def test_mesh_outward_normals_point_away():
    re = ref_element(2)
    m = build_mesh(2, re)
    cen = m.VX.mean(axis=1)
    for f, fv in enumerate(((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))):
        fc = m.VX[:, list(fv)].mean(axis=1)
        assert np.all(np.einsum("ki,ki->k", fc - cen, m.nrm[:, f]) > 0)
