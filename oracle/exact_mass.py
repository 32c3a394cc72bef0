"""Exact-mass variant of the oracle's right-hand side, for comparison with
the weight-adjusted (WADG) mass inverse.  Plain FP64 NumPy.

With the raw right-hand side r = M^-1 (weak residual) (volume, flux, LIFT;
oracle.dg.ElasticDG.rhs_raw), the semi-discrete system with the exact
variable-coefficient mass matrices is, per element k,

    M_rho dv/dt = M r_v,          (M_rho)_ij = int rho phi_i phi_j,
    M_S dsigma/dt = M r_s,        (M_S)_(a i)(b j) = int S_ab phi_i phi_j,

with S = C^-1 the compliance in the tensor-component Voigt order of the
state (xx yy zz yz xz xy): on the normal block
S = (I - lam / (3 lam + 2 mu) 1 1^T) / (2 mu), on each shear component
1 / (2 mu).  Integrals use the element's quadrature rule (exact for
polynomial media of degree 1).  WADG replaces M_rho^-1 M by
M^-1 M_(1/rho) and M_S^-1 M by M^-1 M_C [CHW17, C18]; both are exact for
constant media.

Pins (tests/test_oracle_exact_mass.py): equality with WADG in homogeneous
media; skew-symmetry of the exact-mass operator with central fluxes in the
energy inner product v^T M_rho v + sigma^T D M_S sigma (D = 1 on the normal
and 2 on the shear components); the WADG difference decreases under mesh
refinement.
"""
from __future__ import annotations

import numpy as np

from .dg import ElasticDG


def compliance(lam, mu):
    """S = C^-1 at each point: [..., 6, 6] in the state's Voigt order."""
    shp = np.shape(lam)
    S = np.zeros(shp + (6, 6))
    a = 1.0 / (2.0 * mu)
    b = -lam / ((3.0 * lam + 2.0 * mu) * 2.0 * mu)
    for i in range(3):
        for j in range(3):
            S[..., i, j] = b + (a if i == j else 0.0)
    for i in range(3, 6):
        S[..., i, i] = a
    return S


def element_mass_matrices(op: ElasticDG, k):
    """(M_rho, M_S) of element k without the Jacobian (it cancels against M)."""
    ref, mat = op.ref, op.mat
    Vq, w = ref.Vq, ref.wq
    rho = 1.0 / mat.irho_q[k]
    Mr = Vq.T @ ((w * rho)[:, None] * Vq)
    S = compliance(mat.lam_q[k], mat.mu_q[k])            # [Nq, 6, 6]
    Np = op.Np
    MS = np.zeros((6 * Np, 6 * Np))
    for a in range(6):
        for b in range(6):
            MS[a * Np:(a + 1) * Np, b * Np:(b + 1) * Np] = Vq.T @ ((w * S[:, a, b])[:, None] * Vq)
    return Mr, MS


def rhs_exact(op: ElasticDG, q):
    """dq/dt with the exact mass matrices (all elements)."""
    r = op.rhs_raw(q)
    M = op.ref.M
    out = np.empty_like(r)
    Np = op.Np
    for k in range(op.K):
        Mr, MS = element_mass_matrices(op, k)
        out[0:3, k] = np.linalg.solve(Mr, (r[0:3, k] @ M.T).T).T
        rs = (r[3:9, k] @ M.T).reshape(6 * Np)
        out[3:9, k] = np.linalg.solve(MS, rs).reshape(6, Np)
    return out
