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
