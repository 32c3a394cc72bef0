"""Pins of the oracle's point sources and receivers (oracle/source.py):
closed forms of the Ricker wavelet, exact reproduction of polynomials by the
receivers, momentum injection and the delta action of a source in
homogeneous media, and discrete reciprocity for central fluxes."""
import numpy as np
import pytest

import synth
from oracle.dg import ElasticDG
from oracle.source import (locate, make_forcing, receiver, ricker, run_with_receivers,
                           sample, source_vector)


def test_ricker_closed_forms():
    f0, t0 = 7.0, 1.2 / 7.0
    assert ricker(t0, f0, t0, amp=2.5) == pytest.approx(2.5, abs=1e-15)
    h = 1e-6
    assert abs(ricker(t0 + h, f0, t0) - ricker(t0 - h, f0, t0)) < 1e-12
    tz = 1.0 / (np.sqrt(2.0) * np.pi * f0)
    assert abs(ricker(t0 + tz, f0, t0)) < 1e-14 and abs(ricker(t0 - tz, f0, t0)) < 1e-14
    t = np.linspace(t0 - 12.0 / f0, t0 + 12.0 / f0, 200001)
    w = ricker(t, f0, t0)
    assert abs(np.trapezoid(w, t)) < 1e-9       # zero mean
    assert np.trapezoid(w * w, t) > 0.05 / f0   # and not zero


@pytest.mark.parametrize("N", [1, 3])
def test_locate_maps_back(N):
    op = ElasticDG(2, N, synth.homogeneous_media)
    rng = np.random.default_rng(1)
    for x in rng.random((20, 3)):
        k, rst = locate(op, x)
        VX = op.mesh.VX[k]
        back = VX[0] + (VX[1:] - VX[0]).T @ ((rst + 1.0) / 2.0)
        assert np.allclose(back, x, atol=1e-13)
        lam = np.concatenate([[-(1 + rst.sum()) / 2], (1 + rst) / 2])
        assert lam.min() >= -1e-12


def _poly(rng, N):
    """A random polynomial of total degree N in (x, y, z) and its evaluator."""
    terms = [(a, b, c) for a in range(N + 1) for b in range(N + 1 - a)
             for c in range(N + 1 - a - b)]
    coef = rng.standard_normal(len(terms))

    def p(x):
        x = np.asarray(x)
        return sum(cf * x[..., 0] ** a * x[..., 1] ** b * x[..., 2] ** c
                   for cf, (a, b, c) in zip(coef, terms))
    return p


@pytest.mark.parametrize("N", [2, 4])
def test_receivers_reproduce_polynomials(N):
    op = ElasticDG(2, N, synth.homogeneous_media)
    rng = np.random.default_rng(2)
    q = np.zeros((9, op.K, op.Np))
    ps = [_poly(rng, N) for _ in range(3)]
    for c in range(3):
        q[c] = ps[c](op.mesh.x)
    pts = rng.random((10, 3)) * 0.999
    got = sample(op, q, [receiver(op, x) for x in pts])
    want = np.stack([[ps[c](x) for c in range(3)] for x in pts])
    assert np.allclose(got, want, rtol=0, atol=1e-11 * np.abs(want).max())


@pytest.mark.parametrize("N", [2, 3])
def test_source_momentum_and_delta_action_homogeneous(N):
    rho = 2.0
    op = ElasticDG(2, N, lambda x: synth.homogeneous_media(x, rho=rho, cp=3.0, cs=1.5))
    rng = np.random.default_rng(3)
    xs = rng.random(3)
    d = np.array([0.3, -0.5, 0.8])
    s = source_vector(op, xs, d)
    assert np.all(s[3:] == 0.0)
    M = op.ref.M
    J = op.mesh.J
    # momentum rate: sum_k 1^T M_k (rho s_c) = d_c
    mom = np.array([np.sum(J[:, None] * ((rho * s[c]) @ M)) for c in range(3)])
    assert np.allclose(mom, d, atol=1e-13)
    # delta action on a polynomial of degree N
    p = _poly(rng, N)
    pn = p(op.mesh.x)                              # [K, Np]
    act = np.array([np.sum(J[:, None] * ((rho * s[c]) @ M) * pn) for c in range(3)])
    assert np.allclose(act, p(xs) * d, rtol=1e-12, atol=1e-12 * abs(p(xs)))


def _reciprocity_defect(op, pairs=((0, 2), (1, 1), (2, 0))):
    xs, xr = np.array([0.31, 0.42, 0.27]), np.array([0.68, 0.55, 0.71])
    f0 = 4.0
    dt, nsteps = 2e-3, 60
    q0 = np.zeros((9, op.K, op.Np))
    worst = 0.0
    for i, j in pairs:
        ej, ei = np.eye(3)[j], np.eye(3)[i]
        src_a = [dict(x=xs, d=ej, f0=f0, t0=1.2 / f0)]
        src_b = [dict(x=xr, d=ei, f0=f0, t0=1.2 / f0)]
        _, ta = run_with_receivers(op, q0, 0.0, dt, nsteps, src_a, [xr])
        _, tb = run_with_receivers(op, q0, 0.0, dt, nsteps, src_b, [xs])
        a, b = ta[:, 0, i], tb[:, 0, j]
        assert np.abs(a).max() > 1e-6
        worst = max(worst, np.abs(a - b).max() / np.abs(a).max())
    return worst


def test_reciprocity_central_flux():
    """G_ij(x_r, x_s) = G_ji(x_s, x_r): v_i at x_r from a force along e_j at
    x_s equals v_j at x_s from a force along e_i at x_r (central fluxes,
    heterogeneous media, fully discrete LSRK)."""
    op = ElasticDG(2, 2, synth.fourier_media, flux="central")
    assert _reciprocity_defect(op) <= 1e-10


def test_reciprocity_detects_a_missing_mass_inverse(monkeypatch):
    """Planted mistake: sources that skip the weight-adjusted inverse break
    the reciprocity pin in heterogeneous media."""
    import oracle.source as src
    from oracle.refelem import basis

    def no_wadg(op, x, d):
        k, rst = src.locate(op, x)
        psi = basis(op.ref.N, *[np.array([c]) for c in rst])[0]
        s = np.zeros((9, op.K, op.Np))
        for c in range(3):
            s[c, k] = op.ref.V @ psi / op.mesh.J[k] * d[c]
        return s
    monkeypatch.setattr(src, "source_vector", no_wadg)
    op = ElasticDG(2, 2, synth.fourier_media, flux="central")
    assert _reciprocity_defect(op, pairs=((0, 2),)) > 1e-3
