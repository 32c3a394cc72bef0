"""Pins of the exact-mass variant (oracle/exact_mass.py) and its comparison
with the weight-adjusted mass inverse."""
import numpy as np
import pytest

import synth
from oracle.dg import ElasticDG
from oracle.exact_mass import element_mass_matrices, rhs_exact


def test_equals_wadg_in_homogeneous_media():
    op = ElasticDG(2, 3, lambda x: synth.homogeneous_media(x, rho=1.7, cp=3.1, cs=1.4))
    q = synth.random_state(op.K, op.Np, seed=4)
    a, b = rhs_exact(op, q), op.rhs(q)
    assert np.abs(a - b).max() <= 1e-11 * np.abs(b).max()


@pytest.mark.parametrize("N", [1, 2])
def test_skew_in_the_exact_energy_with_central_flux(N):
    op = ElasticDG(1, N, synth.fourier_media, flux="central")
    n = 9 * op.K * op.Np
    A = np.zeros((n, n))
    e = np.zeros(n)
    for i in range(n):
        e[i] = 1.0
        A[:, i] = rhs_exact(op, e.reshape(9, op.K, op.Np)).ravel()
        e[i] = 0.0
    # energy matrix H: J_k blockdiag(M_rho, D M_S) per element, in state order
    Np, K = op.Np, op.K
    H = np.zeros((n, n))
    D = np.array([1, 1, 1, 2, 2, 2], dtype=float)
    for k in range(K):
        Mr, MS = element_mass_matrices(op, k)
        J = op.mesh.J[k]
        for a in range(3):
            ia = a * K * Np + k * Np
            for b in range(3):
                if a == b:
                    H[ia:ia + Np, ia:ia + Np] = J * Mr
        for a in range(6):
            ia = (3 + a) * K * Np + k * Np
            for b in range(6):
                ib = (3 + b) * K * Np + k * Np
                H[ia:ia + Np, ib:ib + Np] = J * D[a] * MS[a * Np:(a + 1) * Np, b * Np:(b + 1) * Np]
    S = H @ A
    assert np.abs(S + S.T).max() <= 1e-11 * np.abs(S).max()


def test_wadg_difference_shrinks_with_refinement():
    """On a smooth state in smooth media, |rhs_WADG - rhs_exact| / |rhs|
    decreases as the mesh is refined (the weight-adjusted inverse is
    consistent)."""
    diffs = []
    for n in (2, 4):
        op = ElasticDG(n, 2, synth.fourier_media)
        q = op.project_function(lambda x: synth.plane_p_wave(x, 0.0) + synth.plane_s_wave(x, 0.1))
        a, b = rhs_exact(op, q), op.rhs(q)
        diffs.append(np.sqrt(op.l2_sq(a - b).sum() / op.l2_sq(a).sum()))
    print("WADG vs exact mass:", diffs)
    assert diffs[1] < 0.5 * diffs[0]
