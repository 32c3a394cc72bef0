"""Pins of the oracle's discrete adjoint (oracle/adjoint.py): the gradient of
a receiver misfit with respect to the weight-adjusted material weights
(1/rho, lam, mu at the quadrature points) against central finite differences
of the forward run, for both fluxes, and a planted mistake that the check
catches."""
import numpy as np
import pytest

import synth
from oracle import adjoint as adj
from oracle.dg import ElasticDG

SRC = [dict(x=np.array([0.3, 0.6, 0.2]), d=np.array([0.2, -0.4, 0.9]), f0=3.0,
            t0=1.2 / 3.0, amp=1.0)]
RECS = np.array([[0.7, 0.25, 0.55], [0.15, 0.8, 0.4]])


def _problem(flux, N=2, n=1):
    op = ElasticDG(n, N, synth.fourier_media, flux=flux)
    m = np.stack([op.mat.irho_q, op.mat.lam_q, op.mat.mu_q]).copy()
    q0 = synth.random_state(op.K, op.Np, seed=3) * 0.1
    return op, m, q0


def _J(op, m, q0, d, dt, nsteps):
    tr = adj.forward_trace(op, m, q0, 0.0, dt, nsteps, SRC, RECS)
    return 0.5 * np.sum((tr - d) ** 2), tr


@pytest.mark.parametrize("flux", ["central", "upwind"])
def test_gradient_matches_central_differences(flux):
    op, m, q0 = _problem(flux)
    dt, nsteps = 0.01, 8
    rng = np.random.default_rng(5)
    d = rng.standard_normal((nsteps, len(RECS), 3)) * 0.05
    _, tr = _J(op, m, q0, d, dt, nsteps)
    g = adj.gradient(op, m, q0, 0.0, dt, nsteps, SRC, RECS, tr - d)
    for _ in range(4):
        delta = rng.standard_normal(m.shape) * m      # relative perturbation
        eps = 1e-6
        jp, _ = _J(op, m + eps * delta, q0, d, dt, nsteps)
        jm, _ = _J(op, m - eps * delta, q0, d, dt, nsteps)
        fd = (jp - jm) / (2 * eps)
        an = float(np.sum(g * delta))
        assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-12), (fd, an)


def test_gradient_check_catches_a_dropped_trace_term(monkeypatch):
    op, m, q0 = _problem("central")
    dt, nsteps = 0.01, 6
    rng = np.random.default_rng(6)
    d = rng.standard_normal((nsteps, len(RECS), 3)) * 0.05
    _, tr = _J(op, m, q0, d, dt, nsteps)
    good = adj._dm

    def bad(op_, lam, r):
        g = good(op_, lam, r)
        g[1] = 0.0                                   # mistake: no lam sensitivity
        return g
    monkeypatch.setattr(adj, "_dm", bad)
    g = adj.gradient(op, m, q0, 0.0, dt, nsteps, SRC, RECS, tr - d)
    delta = np.zeros_like(m)
    delta[1] = rng.standard_normal(m.shape[1:]) * m[1]
    eps = 1e-6
    fd = (_J(op, m + eps * delta, q0, d, dt, nsteps)[0]
          - _J(op, m - eps * delta, q0, d, dt, nsteps)[0]) / (2 * eps)
    assert abs(fd - float(np.sum(g * delta))) > 1e-3 * abs(fd)


def _material_sets(op):
    """rho, lam, mu at the quadrature points and at the nodes of the
    oracle's media (six [K, *] arrays)."""
    mat = op.mat
    rho_q = 1.0 / mat.irho_q
    rho_n = synth.fourier_media(op.mesh.x)[0]
    mu_n = mat.Zs_n ** 2 / rho_n
    lam_n = mat.Zp_n ** 2 / rho_n - 2.0 * mu_n
    return [rho_q, mat.lam_q.copy(), mat.mu_q.copy(), rho_n, lam_n, mu_n]


def _m_z(P):
    """Weights m = (1/rho, lam, mu) at the quadrature points and impedances
    z = (sqrt(rho (lam + 2 mu)), sqrt(rho mu)) at the nodes."""
    rho_q, lam_q, mu_q, rho_n, lam_n, mu_n = P
    m = np.stack([1.0 / rho_q, lam_q, mu_q])
    z = np.stack([np.sqrt(rho_n * (lam_n + 2.0 * mu_n)), np.sqrt(rho_n * mu_n)])
    return m, z


def test_impedance_gradient_matches_central_differences():
    op, m, q0 = _problem("upwind")
    z = np.stack([op.mat.Zp_n, op.mat.Zs_n]).copy()
    dt, nsteps = 0.01, 8
    rng = np.random.default_rng(15)
    d = rng.standard_normal((nsteps, len(RECS), 3)) * 0.05
    tr = adj.forward_trace(op, m, q0, 0.0, dt, nsteps, SRC, RECS, z)
    gm, gz = adj.gradient(op, m, q0, 0.0, dt, nsteps, SRC, RECS, tr - d, z=z, with_z=True)
    assert np.abs(gz).max() > 0
    for _ in range(4):
        delta = rng.standard_normal(z.shape) * z
        eps = 1e-6
        J = [0.5 * np.sum((adj.forward_trace(op, m, q0, 0.0, dt, nsteps, SRC, RECS,
                                               z + sg * eps * delta) - d) ** 2)
             for sg in (1.0, -1.0)]
        fd = (J[0] - J[1]) / (2 * eps)
        an = float(np.sum(gz * delta))
        assert abs(fd - an) <= 1e-6 * abs(fd), (fd, an)


@pytest.mark.parametrize("flux", ["upwind", "central"])
def test_gradient_in_rho_lam_mu_matches_central_differences(flux):
    """The gradient with respect to the material fields: rho, lam, mu at the
    quadrature points and at the nodes perturbed together, with m and the
    impedances recomputed from them, against the chain rule through
    (dJ/dm, dJ/dz)."""
    op, _, q0 = _problem(flux)
    P = _material_sets(op)
    m, z = _m_z(P)
    assert np.allclose(z[0], op.mat.Zp_n) and np.allclose(m[0], op.mat.irho_q)
    dt, nsteps = 0.01, 8
    rng = np.random.default_rng(16)
    d = rng.standard_normal((nsteps, len(RECS), 3)) * 0.05
    tr = adj.forward_trace(op, m, q0, 0.0, dt, nsteps, SRC, RECS, z)
    gm, gz = adj.gradient(op, m, q0, 0.0, dt, nsteps, SRC, RECS, tr - d, z=z, with_z=True)
    for _ in range(3):
        dP = [rng.standard_normal(p.shape) * p * 0.1 for p in P]
        rho_q, lam_q, mu_q, rho_n, lam_n, mu_n = P
        drq, dlq, dmq, drn, dln, dmn = dP
        dm = np.stack([-drq / rho_q ** 2, dlq, dmq])
        dz = np.stack([(drn * (lam_n + 2 * mu_n) + rho_n * (dln + 2 * dmn)) / (2 * z[0]),
                       (drn * mu_n + rho_n * dmn) / (2 * z[1])])
        an = float(np.sum(gm * dm) + np.sum(gz * dz))
        eps = 1e-6
        J = []
        for sg in (1.0, -1.0):
            mm, zz = _m_z([p + sg * eps * dp for p, dp in zip(P, dP)])
            J.append(0.5 * np.sum((adj.forward_trace(op, mm, q0, 0.0, dt, nsteps, SRC, RECS,
                                                     zz) - d) ** 2))
        fd = (J[0] - J[1]) / (2 * eps)
        assert abs(fd - an) <= 1e-6 * abs(fd), (fd, an)


def test_impedance_gradient_check_catches_a_misplaced_neighbour_term(monkeypatch):
    """A planted mistake: the derivative with respect to the neighbour-side
    P impedance summed onto the own node instead of the neighbour's."""
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(adj._dz))
    old = "[(0, iM), (0, iP), (1, iM), (1, iP)]"
    assert old in src
    ns = dict(vars(adj))
    exec(compile(src.replace(old, "[(0, iM), (0, iM), (1, iM), (1, iP)]"), "<mutant>", "exec"), ns)
    monkeypatch.setattr(adj, "_dz", ns["_dz"])
    op, m, q0 = _problem("upwind")
    z = np.stack([op.mat.Zp_n, op.mat.Zs_n]).copy()
    dt, nsteps = 0.01, 6
    rng = np.random.default_rng(17)
    d = rng.standard_normal((nsteps, len(RECS), 3)) * 0.05
    tr = adj.forward_trace(op, m, q0, 0.0, dt, nsteps, SRC, RECS, z)
    _, gz = adj.gradient(op, m, q0, 0.0, dt, nsteps, SRC, RECS, tr - d, z=z, with_z=True)
    delta = np.zeros_like(z)
    delta[0] = rng.standard_normal(z.shape[1:]) * z[0]
    eps = 1e-6
    J = [0.5 * np.sum((adj.forward_trace(op, m, q0, 0.0, dt, nsteps, SRC, RECS,
                                           z + sg * eps * delta) - d) ** 2) for sg in (1.0, -1.0)]
    fd = (J[0] - J[1]) / (2 * eps)
    assert abs(fd - float(np.sum(gz * delta))) > 1e-3 * abs(fd)
