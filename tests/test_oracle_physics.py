"""Pins of the oracle's DG operator and time integrator against exact plane
waves, convergence order, the semi-discrete energy identity, homogeneous
reductions, conservation, basis independence and the LSRK(5,4) stability
polynomial.  Each pin fails for a plausible mistake (see
test_oracle_mutations.py, which plants such mistakes and checks that)."""
import os

import numpy as np
import pytest

import synth
from oracle.dg import ElasticDG, LSRK_A, LSRK_B, LSRK_C, lsrk_step

D9 = np.array([1, 1, 1, 1, 1, 1, 2, 2, 2], dtype=np.float64)


def assemble(op, raw=False):
    """Dense operator A with dq/dt = A q (column by column)."""
    n = 9 * op.K * op.Np
    A = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        q = e.reshape(9, op.K, op.Np)
        r = op.rhs_raw(q) if raw else op.rhs(q)
        A[:, j] = r.ravel()
        e[j] = 0.0
    return A


def energy_weight(op):
    """G = blockdiag over (field, element) of w_f J_k M_hat, w = (1,..,1,2,2,2):
    the Voigt inner product counts each shear stress twice."""
    G = np.zeros((9, op.K, op.Np, 9, op.K, op.Np))
    for f in range(9):
        for k in range(op.K):
            G[f, k, :, f, k, :] = D9[f] * op.mesh.J[k] * op.ref.M
    n = 9 * op.K * op.Np
    return G.reshape(n, n)


@pytest.mark.parametrize("N", [1, 2])
def test_central_flux_raw_operator_is_energy_skew(N):
    op = ElasticDG(1, N, synth.homogeneous_media, flux="central")
    S = energy_weight(op) @ assemble(op, raw=True)
    assert np.abs(S + S.T).max() < 1e-12 * np.abs(S).max()


@pytest.mark.parametrize("N", [1, 2])
def test_upwind_raw_operator_is_dissipative(N):
    """Constant impedance on every face: S + S^T is negative semidefinite,
    and strictly dissipative (some negative eigenvalues)."""
    op = ElasticDG(1, N, synth.homogeneous_media, flux="upwind")
    S = energy_weight(op) @ assemble(op, raw=True)
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert ev.max() < 1e-12 * np.abs(S).max()
    assert ev.min() < -1e-3


def test_wadg_central_variable_media_conserves_energy():
    """With heterogeneous media the weight-adjusted operator A = W K_raw has
    H A skew with H = G W^{-1} symmetric positive definite, so the spectrum
    of A is purely imaginary."""
    op = ElasticDG(1, 2, synth.fourier_media, flux="central")
    A = assemble(op)
    ev = np.linalg.eigvals(A)
    assert np.abs(ev.real).max() < 1e-9 * np.abs(ev).max()
    # and H = G W^-1 is symmetric positive definite
    Kraw = assemble(op, raw=True)
    G = energy_weight(op)
    # W is block diagonal per element: recover it from A = W Kraw on the
    # range of Kraw by applying rhs to unit raw vectors through wadg()
    n = A.shape[0]
    W = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        W[:, j] = op.wadg(e.reshape(9, op.K, op.Np), np.arange(op.K)).ravel()
        e[j] = 0.0
    assert np.allclose(W @ Kraw, A, atol=1e-10 * np.abs(A).max())
    H = G @ np.linalg.inv(W)
    assert np.abs(H - H.T).max() < 1e-10 * np.abs(H).max()
    assert np.linalg.eigvalsh(0.5 * (H + H.T)).min() > 0


def test_upwind_variable_media_dissipates():
    op = ElasticDG(1, 2, synth.fourier_media, flux="upwind")
    ev = np.linalg.eigvals(assemble(op))
    assert ev.real.max() < 1e-9 * np.abs(ev).max()


@pytest.mark.parametrize("flux", ["upwind", "central"])
def test_wadg_homogeneous_reduces_to_pointwise_coefficients(flux):
    rho, cp, cs = 2.0, 3.0, 1.5
    lam, mu = rho * (cp * cp - 2 * cs * cs), rho * cs * cs
    op = ElasticDG(2, 3, lambda x: synth.homogeneous_media(x, rho, cp, cs), flux=flux)
    q = synth.random_state(op.K, op.Np, seed=3)
    raw = op.rhs_raw(q)
    full = op.rhs(q)
    exp = np.empty_like(raw)
    exp[0:3] = raw[0:3] / rho
    tr = raw[3] + raw[4] + raw[5]
    for i in range(3):
        exp[3 + i] = lam * tr + 2 * mu * raw[3 + i]
        exp[6 + i] = 2 * mu * raw[6 + i]
    assert np.abs(full - exp).max() < 1e-12 * np.abs(exp).max()


@pytest.mark.parametrize("flux", ["upwind", "central"])
def test_momentum_conserved_homogeneous(flux):
    op = ElasticDG(2, 2, synth.homogeneous_media, flux=flux)
    q = synth.random_state(op.K, op.Np, seed=4)
    r = op.rhs(q)
    ones = np.ones(op.Np)
    mom = np.einsum("k,fkp,pq,q->f", op.mesh.J, r[0:3], op.ref.M, ones)
    scale = np.einsum("k,fkp,pq,q->f", op.mesh.J, np.abs(r[0:3]), op.ref.M, ones)
    assert np.abs(mom).max() < 1e-12 * scale.max()


@pytest.mark.parametrize("wave", ["p", "s"])
def test_semidiscrete_consistency_with_plane_waves(wave):
    """rhs(P q_exact) -> P d/dt q_exact as h -> 0, at rate >= N (order N=2)."""
    fun = synth.plane_p_wave if wave == "p" else synth.plane_s_wave
    errs = []
    for n in (2, 4):
        op = ElasticDG(n, 2, synth.homogeneous_media)
        q = op.project_function(lambda x: fun(x, 0.0))
        dt = 1e-6
        dq = op.project_function(lambda x: (fun(x, dt) - fun(x, -dt)) / (2 * dt))
        r = op.rhs(q)
        errs.append(np.sqrt(op.l2_sq(r - dq).sum() / op.l2_sq(dq).sum()))
    rate = np.log2(errs[0] / errs[1])
    assert rate > 1.8, errs


def test_plane_p_wave_order3_cube4_T05():
    """The order-3 plane-wave workload: n=4 (384 tets), rho=1 cp=2 cs=1,
    P wave along (1,1,0), upwind, LSRK(5,4) to T=0.5 at CFL 0.5.  Its L2
    error against the exact solution is bounded by the interpolation-error
    scale (h/pi)^(N+1)-ish; we pin it below 1e-2 (measured 6.8e-3), and the
    quantity is recorded for the GPU comparison."""
    op = ElasticDG(4, 3, synth.homogeneous_media)
    q0 = op.project_function(lambda x: synth.plane_p_wave(x, 0.0))
    dt, ns = op.cfl_dt(0.5)
    assert ns == 182
    q = op.run(q0, 0.0, dt, ns)
    qe = op.project_function(lambda x: synth.plane_p_wave(x, 0.5))
    err = np.sqrt(op.l2_sq(q - qe).sum() / op.l2_sq(qe).sum())
    assert err < 1e-2


def _plane_wave_errors(wave, N, ns, T=0.1):
    """Relative L2 error against the exact plane wave after LSRK(5,4) to T
    at CFL 0.5, on the n^3 x 6 cubes of `ns` (homogeneous, upwind)."""
    fun = synth.plane_p_wave if wave == "p" else synth.plane_s_wave
    errs = []
    for n in ns:
        op = ElasticDG(n, N, synth.homogeneous_media)
        q0 = op.project_function(lambda x: fun(x, 0.0))
        dt, nst = op.cfl_dt(T)
        q = op.run(q0, 0.0, dt, nst)
        qe = op.project_function(lambda x: fun(x, T))
        errs.append(np.sqrt(op.l2_sq(q - qe).sum() / op.l2_sq(qe).sum()))
    return np.array(errs)


@pytest.mark.parametrize("wave", ["p", "s"])
def test_convergence_order_N_plus_1(wave):
    """PA2 at N = 3: plane P and S waves on n = 2, 4, 8 to T = 0.1.  The
    observed order between n = 4 and n = 8 is close to N + 1 = 4 (measured
    3.79 for P, 3.77 for S); n = 2 is pre-asymptotic for the S wave."""
    errs = _plane_wave_errors(wave, 3, (2, 4, 8))
    rates = np.log2(errs[:-1] / errs[1:])
    assert rates[-1] >= 3.7, (errs, rates)
    assert np.all(rates > 2.5), (errs, rates)


@pytest.mark.slow
@pytest.mark.skipif(not os.environ.get("DG_SLOW_PINS"),
                    reason="about 13 minutes per wave on 8 cores; set DG_SLOW_PINS=1")
@pytest.mark.parametrize("wave", ["p", "s"])
def test_convergence_order_N_plus_1_to_n16(wave):
    """PA2 as stated, N = 3 and n = 2, 4, 8, 16 (24,576 tets at n = 16).
    Measured errors: P 9.26e-2, 6.62e-3, 4.79e-4, 3.09e-5 (least-squares
    slope 3.84, finest pair 3.95); S 7.34e-2, 1.10e-2, 8.03e-4, 5.93e-5
    (slope over n = 4-16: 3.77)."""
    errs = _plane_wave_errors(wave, 3, (2, 4, 8, 16))
    h = 1.0 / np.array([2.0, 4.0, 8.0, 16.0])
    fine = np.polyfit(np.log(h[1:]), np.log(errs[1:]), 1)[0]
    assert fine >= 3.7, errs
    if wave == "p":
        assert np.polyfit(np.log(h), np.log(errs), 1)[0] >= 3.8, errs


def test_basis_independence():
    """Homogeneous media (constant impedance per face): the RHS of the same
    polynomial state is the same polynomial for two different nodal sets,
    compared at the quadrature points."""
    fun = lambda x: synth.plane_p_wave(x, 0.1) + 0.3 * synth.gaussian_pulse(x, width=0.2)
    out = []
    for nodes in ("equi", "warped"):
        op = ElasticDG(2, 3, synth.homogeneous_media, nodes=nodes)
        q = op.project_function(fun)
        out.append(op.rhs(q) @ op.ref.Vq.T)
    assert np.abs(out[0] - out[1]).max() < 1e-11 * np.abs(out[0]).max()


def test_lsrk_stability_polynomial_and_order():
    # stability polynomial R(z) = sum c_k z^k from y' = z y, one step dt = 1
    zs = np.linspace(-1.0, 1.0, 11)
    R = []
    for z in zs:
        y, _ = lsrk_step(lambda y, t: z * y, 1.0, 0.0, 0.0, 1.0)
        R.append(y)
    coef = np.polynomial.polynomial.polyfit(zs, R, 5)
    assert np.allclose(coef, [1, 1, 1 / 2, 1 / 6, 1 / 24, 1 / 200], atol=1e-12)
    # fourth order on a non-autonomous ODE y' = -y + cos(t), y(0)=1
    exact = lambda t: 0.5 * (np.cos(t) + np.sin(t)) + 0.5 * np.exp(-t)
    errs = []
    for nst in (10, 20, 40):
        dt, y, res, t = 2.0 / nst, 1.0, 0.0, 0.0
        for _ in range(nst):
            y, res = lsrk_step(lambda y, tt: -y + np.cos(tt), y, res, t, dt)
            t += dt
        errs.append(abs(y - exact(2.0)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 3.8), rates
    # consistency of the abscissae: c_s = sum of b's in the effective tableau
    assert float(LSRK_C[0]) == 0.0 and abs(float(LSRK_C[1]) - float(LSRK_B[0])) < 1e-16
    assert float(LSRK_A[0]) == 0.0


def _split_mesh(n, N):
    from oracle.mesh import build_mesh
    from oracle.refelem import ref_element
    return build_mesh(n, ref_element(N), synth.split_tet_vertices(synth.kuhn_cube_vertices(n)))


def test_split_mesh_energy_momentum_and_plane_waves():
    """The Kuhn cube with element 0 split at its centroid (K = 6 n^3 + 3, an
    odd count): the new faces are matched and paired, so the central-flux raw
    operator stays energy-skew and the upwind one dissipative; momentum is
    conserved; and the plane-wave consistency error equals the unsplit
    mesh's to within 2%."""
    op = ElasticDG(1, 1, synth.homogeneous_media, flux="central", mesh=_split_mesh(1, 1))
    assert op.K == 9
    S = energy_weight(op) @ assemble(op, raw=True)
    assert np.abs(S + S.T).max() < 1e-12 * np.abs(S).max()
    op = ElasticDG(1, 1, synth.homogeneous_media, flux="upwind", mesh=_split_mesh(1, 1))
    S = energy_weight(op) @ assemble(op, raw=True)
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert ev.max() < 1e-12 * np.abs(S).max() and ev.min() < -1e-3
    op = ElasticDG(2, 2, synth.homogeneous_media, flux="upwind", mesh=_split_mesh(2, 2))
    q = synth.random_state(op.K, op.Np, seed=4)
    r = op.rhs(q)
    ones = np.ones(op.Np)
    mom = np.einsum("k,fkp,pq,q->f", op.mesh.J, r[0:3], op.ref.M, ones)
    scale = np.einsum("k,fkp,pq,q->f", op.mesh.J, np.abs(r[0:3]), op.ref.M, ones)
    assert np.abs(mom).max() < 1e-12 * scale.max()
    errs = []
    for mesh in (None, _split_mesh(2, 2)):
        op = ElasticDG(2, 2, synth.homogeneous_media, mesh=mesh)
        q = op.project_function(lambda x: synth.plane_p_wave(x, 0.0))
        dt = 1e-6
        dq = op.project_function(lambda x: (synth.plane_p_wave(x, dt) - synth.plane_p_wave(x, -dt)) / (2 * dt))
        errs.append(np.sqrt(op.l2_sq(op.rhs(q) - dq).sum() / op.l2_sq(dq).sum()))
    assert abs(errs[1] - errs[0]) < 0.02 * errs[0], errs
