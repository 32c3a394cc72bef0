"""Point sources and receivers for the oracle.  Plain FP64 NumPy.

Source model.  A point force f(t) d applied at x_s enters the momentum
equation as rho dv/dt = div(sigma) + delta(x - x_s) f(t) d.  In the
discrete equation of the element k that contains x_s, the delta function acts
on the test functions by point evaluation, so the raw (pre mass-inverse)
right-hand side of the velocity rows gains

    M_k^-1 l(x^_s) f(t) d = (1 / J_k) V psi(x^_s) f(t) d,

with l the nodal (Lagrange) basis, psi the orthonormal basis and
M_k = J_k V^-T V^-1 the element mass matrix [HW08, Ch. 10].  Like every
other raw term, it then passes through the weight-adjusted mass inverse
[CHW17, C18]:

    s = P_q[(1/rho)_q V_q ((1 / J_k) V psi(x^_s))] d.

The time signal is the Ricker wavelet
    f(t) = A (1 - 2 pi^2 f0^2 (t - t0)^2) exp(-pi^2 f0^2 (t - t0)^2).

Receiver model.  v(x_r) = l(x^_r) . v_k, the polynomial of the element that
contains x_r evaluated at x_r.

Points are located by their reference coordinates r = 2 G^-1 (x - x_0) - 1,
G = [x_1 - x_0, x_2 - x_0, x_3 - x_0], in each element (the first element
whose barycentric coordinates are all >= -1e-12 wins), after reducing x
modulo the unit period.

Pins (tests/test_oracle_sources.py): the Ricker closed forms (value 1 and
zero slope at t0, zeros at t0 +- 1/(sqrt(2) pi f0), zero mean); receivers
reproduce polynomials of degree N exactly; in homogeneous media the source
injects momentum at the rate f(t) d and acts on polynomials p as
p(x_s) f(t) d; with central fluxes the receiver traces obey discrete
reciprocity, G_ij(x_r, x_s) = G_ji(x_s, x_r), to rounding.
"""
from __future__ import annotations

import numpy as np

from .refelem import basis


def ricker(t, f0, t0, amp=1.0):
    """Ricker wavelet A (1 - 2 (pi f0 (t - t0))^2) exp(-(pi f0 (t - t0))^2)."""
    a = (np.pi * f0 * (np.asarray(t, dtype=np.float64) - t0)) ** 2
    return amp * (1.0 - 2.0 * a) * np.exp(-a)


def locate(op, x):
    """Element index k and reference coordinates (r, s, t) of the physical
    point x (reduced modulo the unit period)."""
    x = np.mod(np.asarray(x, dtype=np.float64), 1.0)
    VX = op.mesh.VX                                      # [K, 4, 3]
    G = (VX[:, 1:, :] - VX[:, :1, :]).transpose(0, 2, 1)  # columns x_i - x_0
    # x = x_0 + G (rst + 1) / 2
    rst = 2.0 * np.linalg.solve(G, (x[None, :] - VX[:, 0, :])[..., None])[..., 0] - 1.0
    lam = np.concatenate([-(1.0 + rst.sum(axis=1, keepdims=True)) / 2.0,
                          (1.0 + rst) / 2.0], axis=1)
    inside = np.nonzero(lam.min(axis=1) >= -1e-12)[0]
    if inside.size == 0:
        raise ValueError(f"point {x} lies in no element")
    k = int(inside[0])
    return k, rst[k]


def lagrange_at(op, rst):
    """Nodal basis values l(x^) at a reference point: l = V^-T psi(x^)."""
    ref = op.ref
    psi = basis(ref.N, *[np.array([c]) for c in rst])[0]
    return np.linalg.solve(ref.V.T, psi)


def source_vector(op, x, d):
    """Right-hand-side response s (shape [9, K, Np], velocity rows only) to a
    unit point force in direction d at x, after the mass inverse."""
    k, rst = locate(op, x)
    ref = op.ref
    psi = basis(ref.N, *[np.array([c]) for c in rst])[0]
    raw = np.zeros((9, 1, op.Np))
    for c in range(3):
        raw[c, 0] = ref.V @ psi / op.mesh.J[k] * d[c]
    s = np.zeros((9, op.K, op.Np))
    s[:, k] = op.wadg(raw, np.array([k]))[:, 0]
    return s


def receiver(op, x):
    """(element, weights) such that v(x) = weights . v[:, element]."""
    k, rst = locate(op, x)
    return k, lagrange_at(op, rst)


def sample(op, q, receivers):
    """Velocity at each receiver: [nrec, 3]."""
    return np.array([[w @ q[c, k] for c in range(3)] for (k, w) in receivers])


def make_forcing(op, sources):
    """sources: list of dicts with x, d, f0, t0, amp.  Returns f(t) giving the
    sum of the sources' right-hand-side contributions at time t."""
    vecs = [(source_vector(op, s["x"], np.asarray(s["d"], dtype=np.float64)), s)
            for s in sources]

    def forcing(t):
        out = np.zeros((9, op.K, op.Np))
        for v, s in vecs:
            out += ricker(t, s["f0"], s["t0"], s.get("amp", 1.0)) * v
        return out
    return forcing


def run_with_receivers(op, q0, t0, dt, nsteps, sources, receiver_points):
    """LSRK(5,4) run with point sources; velocity at the receivers after
    every step.  Returns (q, trace[nsteps, nrec, 3])."""
    forcing = make_forcing(op, sources) if sources else None
    recs = [receiver(op, x) for x in receiver_points]
    q, res = q0, np.zeros_like(q0)
    trace = np.zeros((nsteps, len(recs), 3))
    for i in range(nsteps):
        q, res = op.step(q, res, dt, t0 + i * dt, forcing)
        trace[i] = sample(op, q, recs)
    return q, trace
