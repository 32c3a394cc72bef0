"""Discrete adjoint of the oracle's LSRK(5,4) run with point sources and
receivers, for tiny meshes.  Plain FP64 NumPy.

Forward map.  The material enters the operator in two places: the
weights m = (1/rho, lam, mu) at the quadrature points (shape [3, K, Nq]) of
the weight-adjusted mass inverse W(m) [CHW17, C18], and the impedances
z = (Zp, Zs) = (rho cp, rho cs) at the nodes (shape [2, K, Np]) of the
upwind flux inside the raw operator R(z) (with central fluxes R does not
depend on z).  With s_raw the raw source vectors, one stage is
    res_s = a_s res_{s-1} + dt W(m) (R(z) y_{s-1} + s_raw g(t_s)),
    y_s = y_{s-1} + b_s res_s             [CK94],
and the receivers sample the velocity after every step, u_n = E q_n.

Adjoint.  For a scalar J(u) with dJ/du = resid, the reverse sweep runs the
stages backwards:
    lres += b_s ly;  grad_m += dt d/dm <lres, W(m) r_s>;  mu = W^T lres;
    ly += dt R^T mu;  grad_z += dt d/dz <mu, R(z) y_{s-1}>;  lres *= a_s,
with r_s = R y_{s-1} + s_raw g(t_s) and ly += E^T resid_n before step n is
reversed.  R^T is the transpose of the assembled raw operator (built column
by column from the oracle's own right-hand side), W^T and d/dm follow from
W(m) r = P_q[m-weighted V_q r]:
    (W^T l)_v = V_q^T (1/rho) P_q^T l_v,
    (W^T l)_s = V_q^T [lam tr(P_q^T l_s) I + 2 mu P_q^T l_s]  (diagonal trace),
    d/d(1/rho) = sum_c (P_q^T l_c)(V_q r_c),  c = v_x, v_y, v_z,
    d/d lam    = tr(P_q^T l_s) tr(V_q r_s),
    d/d mu     = 2 sum_c (P_q^T l_c)(V_q r_c),  c = stress components.
d/dz <mu, R(z) y> = d/dz sum over face nodes of (Fscale LIFT^T mu) . flux:
each face node's flux depends on the four impedances it reads (its own
node's and the neighbouring node's, P and S); the derivative with respect to
each is taken by the complex-step method (Squire and Trapp, SIAM Review
1998: for a function analytic in its argument, Im f(x + i h) / h with
h = 1e-30 is its derivative to rounding, with no cancellation) and summed
onto the node the face node reads it from.  A gradient with respect to
rho, lam, mu fields follows by the chain rule through m and z.

Pins (tests/test_oracle_adjoint.py): the gradients against central finite
differences of J along random directions, for both fluxes: in m, in z, and
in rho, lam, mu perturbed together with m and z recomputed from them; and
planted mistakes (a dropped trace term, a dropped neighbour-side impedance
term) that the checks catch.

This module is test infrastructure: only the tests use it.
"""
from __future__ import annotations

import numpy as np

from .dg import LSRK_A, LSRK_B, LSRK_C, ElasticDG, riemann_flux
from .refelem import basis
from .source import locate, receiver, ricker, source_vector


def with_weights(op: ElasticDG, m, z=None):
    """The operator with its weight-adjusted material replaced by m and, if
    given, its nodal impedances by z = (Zp, Zs)."""
    op.mat.irho_q = np.array(m[0], dtype=np.float64)
    op.mat.lam_q = np.array(m[1], dtype=np.float64)
    op.mat.mu_q = np.array(m[2], dtype=np.float64)
    if z is not None:
        op.mat.Zp_n = np.array(z[0], dtype=np.float64)
        op.mat.Zs_n = np.array(z[1], dtype=np.float64)
    return op


def raw_matrix(op: ElasticDG):
    """Dense raw operator R (volume + lifted flux), column by column."""
    n = 9 * op.K * op.Np
    R = np.zeros((n, n))
    e = np.zeros(n)
    for i in range(n):
        e[i] = 1.0
        R[:, i] = op.rhs_raw(e.reshape(9, op.K, op.Np)).ravel()
        e[i] = 0.0
    return R


def raw_sources(op: ElasticDG, sources):
    """Raw (pre mass-inverse) source vectors M_k^-1 l(x^_s) d, one
    [9, K, Np] array per source."""
    out = []
    for s in sources:
        k, rst = locate(op, s["x"])
        psi = basis(op.ref.N, *[np.array([c]) for c in rst])[0]
        v = np.zeros((9, op.K, op.Np))
        for c in range(3):
            v[c, k] = op.ref.V @ psi / op.mesh.J[k] * s["d"][c]
        out.append(v)
    return out


def _wT(op, lam, m):
    """W(m)^T applied to lam [9, K, Np]."""
    ref = op.ref
    p = lam @ ref.Pq                                       # P_q^T l: [9, K, Nq]
    o = np.empty_like(p)
    o[0:3] = m[0][None] * p[0:3]
    tr = p[3] + p[4] + p[5]
    for i in range(3):
        o[3 + i] = m[1] * tr + 2.0 * m[2] * p[3 + i]
    for i in range(3, 6):
        o[3 + i] = 2.0 * m[2] * p[3 + i]
    return o @ ref.Vq                                      # V_q^T: [9, K, Np]


def _dm(op, lam, r):
    """d/dm <lam, W(m) r>: [3, K, Nq]."""
    ref = op.ref
    p = lam @ ref.Pq
    w = r @ ref.Vq.T
    g = np.empty((3,) + p.shape[1:])
    g[0] = np.sum(p[0:3] * w[0:3], axis=0)
    g[1] = (p[3] + p[4] + p[5]) * (w[3] + w[4] + w[5])
    g[2] = 2.0 * np.sum(p[3:9] * w[3:9], axis=0)
    return g


def _dz(op, mu, y):
    """d/dz <mu, R(z) y> for the upwind flux: [2, K, Np] (Zp, Zs)."""
    m, mat, ref = op.mesh, op.mat, op.ref
    K, Np, Nfp = op.K, op.Np, ref.Nfp
    gf = (mu @ ref.LIFT).reshape(9, K, 4, Nfp) * m.Fscale[None, :, :, None]
    qf = y.reshape(9, -1)
    iM, iP = m.vmapM, m.vmapP
    qM, qP = qf[:, iM], qf[:, iP]
    n = m.nrm[:, :, None, :]
    Z = [mat.Zp_n.ravel()[iM], mat.Zp_n.ravel()[iP], mat.Zs_n.ravel()[iM], mat.Zs_n.ravel()[iP]]
    h = 1e-30
    out = np.zeros((2, K * Np))
    # slot order of riemann_flux: ZpM, ZpP, ZsM, ZsP
    for slot, (which, idx) in enumerate([(0, iM), (0, iP), (1, iM), (1, iP)]):
        Zc = [z.astype(np.complex128) for z in Z]
        Zc[slot] = Zc[slot] + 1j * h
        f = riemann_flux(qM, qP, n, "upwind", tuple(Zc))
        d = np.sum(gf * f.imag, axis=0) / h                 # [K, 4, Nfp]
        np.add.at(out[which], idx.ravel(), d.ravel())
    return out.reshape(2, K, Np)


def forward_trace(op, m, q0, t0, dt, nsteps, sources, receiver_points, z=None):
    """Receiver velocities [nsteps, nrec, 3] of the run with weights m (and
    impedances z, if given)."""
    with_weights(op, m, z)
    vecs = [source_vector(op, s["x"], np.asarray(s["d"], np.float64)) for s in sources]
    recs = [receiver(op, x) for x in receiver_points]

    def forcing(t):
        out = np.zeros((9, op.K, op.Np))
        for v, s in zip(vecs, sources):
            out += ricker(t, s["f0"], s["t0"], s.get("amp", 1.0)) * v
        return out
    q, res = q0.copy(), np.zeros_like(q0)
    tr = np.zeros((nsteps, len(recs), 3))
    for i in range(nsteps):
        q, res = op.step(q, res, dt, t0 + i * dt, forcing if sources else None)
        for r, (k, w) in enumerate(recs):
            tr[i, r] = [w @ q[c, k] for c in range(3)]
    return tr


def gradient(op, m, q0, t0, dt, nsteps, sources, receiver_points, resid, R=None,
             z=None, with_z=False):
    """dJ/dm for dJ/d(trace) = resid [nsteps, nrec, 3]; with with_z, the pair
    (dJ/dm, dJ/dz) with z = (Zp, Zs) at the nodes (zero for central fluxes)."""
    with_weights(op, m, z)
    if R is None:
        R = raw_matrix(op)
    shp = (9, op.K, op.Np)
    raws = raw_sources(op, sources)
    recs = [receiver(op, x) for x in receiver_points]
    a = [float(x) for x in LSRK_A]
    b = [float(x) for x in LSRK_B]
    c = [float(x) for x in LSRK_C]

    def raw_rhs(y, t):
        r = (R @ y.ravel()).reshape(shp)
        for v, s in zip(raws, sources):
            r = r + ricker(t, s["f0"], s["t0"], s.get("amp", 1.0)) * v
        return r

    def F(y, t):
        return op.wadg(raw_rhs(y, t), np.arange(op.K))

    # forward, keeping every step's start state
    qs = [q0.copy()]
    q = q0.copy()
    for i in range(nsteps):
        y, res = q, np.zeros(shp)
        for s in range(5):
            res = a[s] * res + dt * F(y, t0 + (i + c[s]) * dt)
            y = y + b[s] * res
        q = y
        qs.append(q)
    # reverse sweep
    grad = np.zeros((3, op.K, op.ref.Nq))
    gradz = np.zeros((2, op.K, op.Np))
    ly = np.zeros(shp)
    for i in reversed(range(nsteps)):
        for r, (k, w) in enumerate(recs):
            for cc in range(3):
                ly[cc, k] += w * resid[i, r, cc]
        ys = [qs[i]]
        res = np.zeros(shp)
        for s in range(5):                     # the step's stage inputs
            res = a[s] * res + dt * F(ys[-1], t0 + (i + c[s]) * dt)
            ys.append(ys[-1] + b[s] * res)
        lres = np.zeros(shp)
        for s in reversed(range(5)):
            lres = lres + b[s] * ly
            ts = t0 + (i + c[s]) * dt
            grad += dt * _dm(op, lres, raw_rhs(ys[s], ts))
            mu = _wT(op, lres, m)
            ly = ly + dt * (R.T @ mu.ravel()).reshape(shp)
            if with_z and op.flux == "upwind":
                gradz += dt * _dz(op, mu, ys[s])
            lres = a[s] * lres
    return (grad, gradz) if with_z else grad
