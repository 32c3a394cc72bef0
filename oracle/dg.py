"""The semi-discrete DG right-hand side for the velocity-stress elastic wave
equation and its LSRK(5,4) time integration, for the oracle.  Plain FP64.

PDE (first-order velocity-stress form, isotropic):
    rho dv/dt     = div(sigma)
    d sigma/dt    = C : eps(v),   C:e = lam tr(e) I + 2 mu e,
    eps(v)        = (grad v + grad v^T) / 2.
State layout: q[9, K, Np], fields (v_x, v_y, v_z, s_xx, s_yy, s_zz, s_yz,
s_xz, s_xy).

Semi-discrete operator, per element, in the order computed below:
 1. volume (strong form [HW08, Ch. 10]): r_v = div(sigma_h),
    r_s = eps(v_h) (tensor components, not engineering strain); derivatives
    by the chain rule d/dx_j = sum_i (dr_i/dx_j) D_i.
 2. face flux at each face node [WSG10]: with n the outward normal of the
    element, t = sigma n, jumps [[a]] = a+ - a-, normal/tangential splits
    a_n = a.n, a_t = a - a_n n:
      upwind:  dv_n = (Zp+ [[v_n]] + [[t_n]]) / (Zp- + Zp+),
               dv_t = (Zs+ [[v_t]] + [[t_t]]) / (Zs- + Zs+),
               dt_n = Zp- dv_n,  dt_t = Zs- dv_t;
      central: dv = [[v]]/2,  dt = [[t]]/2;
    flux for the velocity equations f_v = dt_n n + dt_t, for the stress
    equations f_s = sym(dv (x) n), dv = dv_n n + dv_t.  Zp = rho cp,
    Zs = rho cs, each side's value taken from its own nodal material.
 3. lift: r += LIFT (Fscale * f) [HW08, Ch. 10].
 4. weight-adjusted mass inverse [CHW17, C18]:
      dv/dt     = P_q[(1/rho)_q (V_q r_v)],
      dsigma/dt = P_q[lam_q tr(V_q r_s) I + 2 mu_q (V_q r_s)].

Time integration: LSRK(5,4) [CK94], five stages of
    res <- a_s res + dt F(q, t + c_s dt);   q <- q + b_s res.

Pins (tests/test_oracle_pins.py, tests/test_oracle_physics.py,
tests/test_oracle_riemann.py): exact plane P and S waves, convergence order
N+1, skew-symmetry (central) and negative-semidefiniteness (upwind) of the
energy-weighted assembled operator, also with the impedance jumping across
every face, WADG reducing to the constant-coefficient operator in
homogeneous media, momentum conservation, the LSRK stability polynomial and
order.  Where Z- != Z+ the upwind flux is pinned by the Riemann problem it
solves: the interface state is single-valued, each side's jump satisfies
that side's wave relation, and normal incidence transmits the closed-form
state.

This module is test infrastructure: only the tests, the smoke check and the
benchmark's CPU baseline use it.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction

import numpy as np

from .mesh import Mesh, build_mesh
from .refelem import RefElement, ref_element

NF = 9

# LSRK(5,4), 2N-storage, [CK94] (solution 3 of the five-stage family)
LSRK_A = [Fraction(0), Fraction(-567301805773, 1357537059087),
          Fraction(-2404267990393, 2016746695238),
          Fraction(-3550918686646, 2091501179385),
          Fraction(-1275806237668, 842570457699)]
LSRK_B = [Fraction(1432997174477, 9575080441755),
          Fraction(5161836677717, 13612068292357),
          Fraction(1720146321549, 2090206949498),
          Fraction(3134564353537, 4481467310338),
          Fraction(2277821191437, 14882151754819)]
LSRK_C = [Fraction(0), Fraction(1432997174477, 9575080441755),
          Fraction(2526269341429, 6820363962896),
          Fraction(2006345519317, 3224310063776),
          Fraction(2802321613138, 2924317926251)]


def lsrk_step(F, y, res, t, dt):
    """One step of LSRK(5,4) [CK94] for dy/dt = F(y, t):
    for s = 1..5: res <- a_s res + dt F(y, t + c_s dt); y <- y + b_s res."""
    for s in range(5):
        res = float(LSRK_A[s]) * res + dt * F(y, t + float(LSRK_C[s]) * dt)
        y = y + float(LSRK_B[s]) * res
    return y, res


@dataclass
class Material:
    """Material samples: 1/rho, lam, mu at quadrature points [K, Nq];
    Zp, Zs at volume nodes [K, Np] (faces read them through the traces)."""
    irho_q: np.ndarray
    lam_q: np.ndarray
    mu_q: np.ndarray
    Zp_n: np.ndarray
    Zs_n: np.ndarray


def material_from_samples(rho_q, cp_q, cs_q, rho_n, cp_n, cs_n) -> Material:
    rho_q, cp_q, cs_q, rho_n, cp_n, cs_n = (
        np.asarray(a, dtype=np.float64) for a in (rho_q, cp_q, cs_q, rho_n, cp_n, cs_n))
    return Material(irho_q=1.0 / rho_q,
                    lam_q=rho_q * (cp_q * cp_q - 2.0 * cs_q * cs_q),
                    mu_q=rho_q * cs_q * cs_q,
                    Zp_n=rho_n * cp_n, Zs_n=rho_n * cs_n)


def riemann_flux(qM, qP, n, flux, Z=None):
    """The face flux of step 2 from the traces qM (own side) and qP
    (neighbour) [9, ...], the outward normals n [..., 3] and, for the upwind
    flux, the impedances Z = (ZpM, ZpP, ZsM, ZsP) at the same face nodes."""
    nx, ny, nz = n[..., 0], n[..., 1], n[..., 2]

    def traction(Q):
        return np.stack([Q[3] * nx + Q[8] * ny + Q[7] * nz,
                         Q[8] * nx + Q[4] * ny + Q[6] * nz,
                         Q[7] * nx + Q[6] * ny + Q[5] * nz])
    vM, vP = qM[0:3], qP[0:3]
    tM, tP = traction(qM), traction(qP)
    nv = np.stack([nx, ny, nz])                              # [3, ...]
    jv = vP - vM
    jt = tP - tM
    if flux == "central":
        dv = 0.5 * jv
        dt = 0.5 * jt
    else:
        ZpM, ZpP, ZsM, ZsP = Z
        jvn = np.sum(jv * nv, axis=0)
        jtn = np.sum(jt * nv, axis=0)
        jvt = jv - jvn * nv
        jtt = jt - jtn * nv
        dvn = (ZpP * jvn + jtn) / (ZpM + ZpP)
        dvt = (ZsP * jvt + jtt) / (ZsM + ZsP)
        dv = dvn * nv + dvt
        dt = (ZpM * dvn) * nv + ZsM * dvt
    f = np.empty((9,) + dv.shape[1:], dtype=dv.dtype)
    f[0:3] = dt
    f[3] = dv[0] * nv[0]
    f[4] = dv[1] * nv[1]
    f[5] = dv[2] * nv[2]
    f[6] = 0.5 * (dv[1] * nv[2] + dv[2] * nv[1])
    f[7] = 0.5 * (dv[0] * nv[2] + dv[2] * nv[0])
    f[8] = 0.5 * (dv[0] * nv[1] + dv[1] * nv[0])
    return f


class ElasticDG:
    """Oracle DG operator on the periodic Kuhn cube of n^3 x 6 tetrahedra."""

    def __init__(self, n: int, N: int, media, flux: str = "upwind",
                 mesh: Mesh | None = None, nodes: str = "equi"):
        if flux not in ("upwind", "central"):
            raise ValueError(flux)
        self.ref: RefElement = ref_element(N, nodes)
        self.mesh: Mesh = mesh if mesh is not None else build_mesh(n, self.ref)
        self.flux = flux
        m = self.mesh
        rho_q, cp_q, cs_q = media(m.xq)
        rho_n, cp_n, cs_n = media(m.x)
        self.mat = material_from_samples(rho_q, cp_q, cs_q, rho_n, cp_n, cs_n)
        self.N, self.K, self.Np = N, m.K, self.ref.Np

    # ------------------------------------------------------------------
    def project(self, fq):
        """L2 projection of quadrature-point samples fq[..., K, Nq]."""
        return fq @ self.ref.Pq.T

    def project_function(self, fun):
        """L2 projection of fun(x[..., 3]) -> [9, ...] onto the nodal basis."""
        return self.project(fun(self.mesh.xq))

    # ------------------------------------------------------------------
    def volume(self, q, elems):
        """Step 1: r_v = div(sigma), r_s = eps(v) at the nodes."""
        ref = self.ref
        qe = q[:, elems]                                    # [9, k, Np]
        gr = np.stack([qe @ ref.Dr.T, qe @ ref.Ds.T, qe @ ref.Dt.T])  # [3rst, 9, k, Np]
        rx = self.mesh.rx[elems]                             # [k, rst, xyz]
        # grad[j][f] = d q_f / d x_j
        grad = np.einsum("kij,ifkp->jfkp", rx, gr)          # [3xyz, 9, k, Np]
        dx, dy, dz = grad[0], grad[1], grad[2]
        vx, vy, vz, sxx, syy, szz, syz, sxz, sxy = range(9)
        r = np.empty_like(qe)
        r[0] = dx[sxx] + dy[sxy] + dz[sxz]
        r[1] = dx[sxy] + dy[syy] + dz[syz]
        r[2] = dx[sxz] + dy[syz] + dz[szz]
        r[3] = dx[vx]
        r[4] = dy[vy]
        r[5] = dz[vz]
        r[6] = 0.5 * (dz[vy] + dy[vz])
        r[7] = 0.5 * (dz[vx] + dx[vz])
        r[8] = 0.5 * (dy[vx] + dx[vy])
        return r

    def face_flux(self, q, elems):
        """Step 2: the numerical flux f[9, k, 4, Nfp] at every face node of
        the elements `elems`, before the Fscale scaling: rows 0-2 are the
        traction correction dt, rows 3-8 the Voigt components of
        sym(dv (x) n).  (dv, dt) is the jump from this side's trace to the
        state the face's Riemann problem leaves at the interface [WSG10]."""
        m, mat = self.mesh, self.mat
        qf = q.reshape(NF, -1)
        iM = m.vmapM[elems]                                  # [k, 4, Nfp]
        iP = m.vmapP[elems]
        n = m.nrm[elems][:, :, None, :]                      # [k, 4, 1, 3]
        Z = None
        if self.flux == "upwind":
            Z = (mat.Zp_n.ravel()[iM], mat.Zp_n.ravel()[iP],
                 mat.Zs_n.ravel()[iM], mat.Zs_n.ravel()[iP])
        return riemann_flux(qf[:, iM], qf[:, iP], n, self.flux, Z)

    def surface(self, q, elems):
        """Step 3: the face flux scaled by Fscale and lifted to the nodes."""
        f = self.face_flux(q, elems) * self.mesh.Fscale[elems][None, :, :, None]
        k = f.shape[1]
        return f.reshape(NF, k, -1) @ self.ref.LIFT.T        # [9, k, Np]

    def wadg(self, r, elems):
        """Step 4: weight-adjusted mass inverse."""
        ref, mat = self.ref, self.mat
        rq = r @ ref.Vq.T                                    # [9, k, Nq]
        irho = mat.irho_q[elems]
        lam = mat.lam_q[elems]
        mu = mat.mu_q[elems]
        out = np.empty_like(rq)
        out[0:3] = irho[None] * rq[0:3]
        tr = rq[3] + rq[4] + rq[5]
        for i in range(3):
            out[3 + i] = lam * tr + 2.0 * mu * rq[3 + i]
        for i in range(3, 6):
            out[3 + i] = 2.0 * mu * rq[3 + i]
        return out @ ref.Pq.T

    def rhs_raw(self, q, elems=None):
        """Volume + lifted flux, before the mass-inverse weighting."""
        if elems is None:
            elems = np.arange(self.K)
        return self.volume(q, elems) + self.surface(q, elems)

    def rhs(self, q, elems=None):
        """dq/dt for the elements in `elems` (all if None): [9, k, Np]."""
        if elems is None:
            elems = np.arange(self.K)
        elems = np.asarray(elems)
        return self.wadg(self.rhs_raw(q, elems), elems)

    # ------------------------------------------------------------------
    def step(self, q, res, dt, t=0.0, forcing=None):
        """One LSRK(5,4) step; returns (q, res) (new arrays).  `forcing`,
        if given, is a callable f(t) -> array added to the right-hand side."""
        if forcing is None:
            return lsrk_step(lambda y, tt: self.rhs(y), q, res, t, dt)
        return lsrk_step(lambda y, tt: self.rhs(y) + forcing(tt), q, res, t, dt)

    def run(self, q, t0, dt, nsteps, forcing=None):
        res = np.zeros_like(q)
        t = t0
        for _ in range(nsteps):
            q, res = self.step(q, res, dt, t, forcing)
            t = t + dt
        return q

    # ------------------------------------------------------------------
    def l2_sq(self, e):
        """Per-field squared L2 norm by quadrature: sum_k J_k sum_q w_q (V_q e)^2."""
        eq = e @ self.ref.Vq.T
        return np.einsum("fkq,q,k->f", eq * eq, self.ref.wq, self.mesh.J)

    def rel_l2(self, a, b):
        """Per-field relative L2 difference ||a - b|| / ||b||."""
        return np.sqrt(self.l2_sq(a - b) / self.l2_sq(b))

    def cfl_dt(self, T, cfl=0.5, cpmax=None):
        """Time step from dt = cfl * h_min / (cp_max (N+1)^2), with
        h_min = min_k 3 Vol_k / max_f Area_{k,f}; rounded so that an integer
        number of steps reaches T.  Returns (dt, nsteps)."""
        m = self.mesh
        vol = m.J * (4.0 / 3.0)
        area = m.sJ * np.array([2.0, 2.0, 2.0, 2.0])[None, :]
        hmin = np.min(3.0 * vol / area.max(axis=1))
        if cpmax is None:
            cpmax = float(np.max(np.sqrt((self.mat.lam_q + 2 * self.mat.mu_q)
                                         * self.mat.irho_q)))
        dtc = cfl * hmin / (cpmax * (self.N + 1) ** 2)
        nsteps = int(np.ceil(T / dtc - 1e-12))
        return T / nsteps, nsteps
