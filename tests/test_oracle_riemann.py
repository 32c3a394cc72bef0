"""Pins of the oracle's upwind flux where the impedance jumps across a face
(Z- != Z+), on element-constant media: each element has its own rho, cp, cs.

The exact-Riemann (upwind) flux of [WSG10] is defined by the state the
face's Riemann problem leaves at the interface.  Three properties of that
state are checked here, none of which restates the solved flux formula:

* single-valued interface state: the velocity and the traction that the
  two sides of a face reach are the same (traction equal and opposite, since
  the normals are), as continuity of displacement and balance of forces
  require at a welded interface;
* the jump from each side's trace to the interface state is carried by the
  wave that travels into that side, so it satisfies that side's jump
  condition: normal traction jump = Z_p times normal velocity jump, and
  tangential traction jump = Z_s times tangential velocity jump, with the
  side's own impedances;
* normal incidence: a plane P or S wave arriving from one side at a quiet
  medium on the other leaves the textbook transmitted state at the
  interface, velocity 2 Z1 / (Z1 + Z2) and traction 2 Z2 / (Z1 + Z2) times
  the incident values (reflection R = (Z2 - Z1) / (Z1 + Z2) for the
  traction, the rest being the reflected wave).

The energy identity is checked on the same media: with the impedance
constant on each side of every face, S + S^T of the energy-weighted raw
operator is negative semidefinite for the upwind flux (PA3).

The first two properties determine the flux uniquely; the energy rate does
not, because it is symmetric in Z- and Z+ (a flux with the two sides'
impedances exchanged dissipates at exactly the same rate, and so converges
to the same interface reflection under refinement).  The swap mutants in
test_oracle_mutations.py fail the first property.
"""
import numpy as np
import pytest

import synth
from oracle.dg import ElasticDG, material_from_samples


def element_media_op(n, N, flux="upwind", seed=12):
    """Oracle operator whose media are constant per element."""
    op = ElasticDG(n, N, synth.homogeneous_media, flux=flux)
    op.mat = material_from_samples(
        *synth.element_constant_samples(op.K, op.ref.Nq, op.Np, seed))
    return op


def _traction(q, nrm):
    """sigma n for Voigt stresses q[3:9, ...] and normals nrm[..., 3]."""
    nx, ny, nz = nrm[..., 0], nrm[..., 1], nrm[..., 2]
    return np.stack([q[3] * nx + q[8] * ny + q[7] * nz,
                     q[8] * nx + q[4] * ny + q[6] * nz,
                     q[7] * nx + q[6] * ny + q[5] * nz])


def _dv_from_flux(f, nrm):
    """Recover the velocity jump dv from the Voigt rows of sym(dv (x) n):
    with S = sym(dv n^T), S n = (dv + n (dv.n)) / 2 and n.S n = dv.n."""
    Sn = _traction(f, nrm)
    dvn = np.sum(Sn * np.moveaxis(nrm, -1, 0), axis=0)
    return 2.0 * Sn - np.moveaxis(nrm, -1, 0) * dvn


def interface_states(op, q):
    """For every face node of every element: the interface velocity and
    traction reached from this side (v + dv, sigma n + dt) and from the
    paired node on the neighbour's face, expressed along this side's
    normal.  Returns (v_here, t_here, v_there, t_there), each [3, K, 4, Nfp]."""
    m = op.mesh
    K, Nfp = op.K, op.ref.Nfp
    f = op.face_flux(q, np.arange(K))                       # [9, K, 4, Nfp]
    nrm = np.broadcast_to(m.nrm[:, :, None, :], (K, 4, Nfp, 3))
    qf = q.reshape(9, -1)
    qM = qf[:, m.vmapM]                                     # [9, K, 4, Nfp]
    v_here = qM[0:3] + _dv_from_flux(f, nrm)
    t_here = _traction(qM, nrm) + f[0:3]
    # slot (k', f', j) on the neighbour that holds the paired node
    kk = m.EToE[:, :, None].repeat(Nfp, axis=2)
    ff = m.EToF[:, :, None].repeat(Nfp, axis=2)
    cand = m.vmapM[kk, ff]                                  # [K, 4, Nfp, Nfp]
    j = np.argmax(cand == m.vmapP[..., None], axis=-1)
    assert np.all(np.take_along_axis(cand, j[..., None], -1)[..., 0] == m.vmapP)
    v_there = v_here[:, kk, ff, j]
    t_there = -t_here[:, kk, ff, j]       # the neighbour's normal is -n
    return v_here, t_here, v_there, t_there


def riemann_defects(op, q):
    """(continuity defect, jump-condition defect), relative to the traces."""
    m = op.mesh
    K, Nfp = op.K, op.ref.Nfp
    v_h, t_h, v_t, t_t = interface_states(op, q)
    nrm = np.moveaxis(np.broadcast_to(m.nrm[:, :, None, :], (K, 4, Nfp, 3)), -1, 0)
    scale = np.abs(q).max() * max(1.0, op.mat.Zp_n.max())
    cont = max(np.abs(v_h - v_t).max() * op.mat.Zp_n.max(),
               np.abs(t_h - t_t).max()) / scale
    # the jump from this side's trace to the interface state
    qM = q.reshape(9, -1)[:, m.vmapM]
    dv = v_h - qM[0:3]
    dt = t_h - _traction(qM, np.moveaxis(nrm, 0, -1))
    dvn = np.sum(dv * nrm, axis=0)
    dtn = np.sum(dt * nrm, axis=0)
    ZpM = op.mat.Zp_n.ravel()[m.vmapM]
    ZsM = op.mat.Zs_n.ravel()[m.vmapM]
    jump = max(np.abs(dtn - ZpM * dvn).max(),
               np.abs((dt - dtn * nrm) - ZsM * (dv - dvn * nrm)).max()) / scale
    return cont, jump


@pytest.mark.parametrize("N", [1, 3])
def test_upwind_interface_state_is_single_valued(N):
    op = element_media_op(2, N)
    assert np.ptp(op.mat.Zp_n) > 0.5          # the impedance does jump
    q = synth.random_state(op.K, op.Np, seed=40 + N)
    cont, _ = riemann_defects(op, q)
    assert cont < 1e-13, cont


@pytest.mark.parametrize("N", [1, 3])
def test_upwind_jump_travels_into_each_side_with_its_own_impedance(N):
    op = element_media_op(2, N)
    q = synth.random_state(op.K, op.Np, seed=50 + N)
    _, jump = riemann_defects(op, q)
    assert jump < 1e-13, jump


def normal_incidence_defect(op, wave, elem=0, face=0, amp=0.7):
    """A plane P wave (v along n) or S wave (v along a tangent p) arriving
    at face `face` of element `elem` from inside it, with every other
    element at rest: relative difference between the interface state the
    oracle's flux implies on this side and the closed-form transmitted state
    v* = 2 Z1/(Z1 + Z2) v_inc, t* = 2 Z2/(Z1 + Z2) t_inc."""
    m = op.mesh
    n = m.nrm[elem, face]
    nb = m.EToE[elem, face]
    rho1, cp1, cs1 = (a[elem] for a in synth.element_constant_params(op.K))
    rho2, cp2, cs2 = (a[nb] for a in synth.element_constant_params(op.K))
    lam1, mu1 = rho1 * (cp1 ** 2 - 2 * cs1 ** 2), rho1 * cs1 ** 2
    if wave == "p":
        Z1, Z2 = rho1 * cp1, rho2 * cp2
        v = amp * n
        # a plane P wave moving along n: sigma = -(lam I + 2 mu n n^T) v.n / cp
        sig = -(lam1 * np.eye(3) + 2 * mu1 * np.outer(n, n)) * amp / cp1
    else:
        Z1, Z2 = rho1 * cs1, rho2 * cs2
        p = np.cross(n, [0.3, -0.5, 0.8])
        p /= np.linalg.norm(p)
        v = amp * p
        # a plane S wave moving along n: sigma = -(mu / cs)(p n^T + n p^T) amp
        sig = -(mu1 / cs1) * (np.outer(p, n) + np.outer(n, p)) * amp
    q = np.zeros((9, op.K, op.Np))
    q[0:3, elem] = v[:, None]
    voigt = [sig[0, 0], sig[1, 1], sig[2, 2], sig[1, 2], sig[0, 2], sig[0, 1]]
    q[3:9, elem] = np.array(voigt)[:, None]
    t_inc = sig @ n
    assert np.allclose(t_inc, -Z1 * v)        # the wave moves along +n
    v_h, t_h, _, _ = interface_states(op, q)
    v_star = v_h[:, elem, face]                # [3, Nfp]
    t_star = t_h[:, elem, face]
    v_exact = 2 * Z1 / (Z1 + Z2) * v
    t_exact = 2 * Z2 / (Z1 + Z2) * t_inc
    return max(np.abs(v_star - v_exact[:, None]).max() / np.abs(v).max(),
               np.abs(t_star - t_exact[:, None]).max() / np.abs(t_inc).max())


@pytest.mark.parametrize("wave", ["p", "s"])
@pytest.mark.parametrize("elem,face", [(0, 0), (5, 2), (17, 3), (30, 1)])
def test_normal_incidence_transmits_the_closed_form_state(wave, elem, face):
    op = element_media_op(2, 2)
    assert normal_incidence_defect(op, wave, elem, face) < 1e-13


def test_normal_incidence_reflection_coefficient():
    """The reflected traction, t* - t_inc, is R t_inc with R = (Z2 - Z1) /
    (Z1 + Z2): this follows from the transmitted state above and is spelled
    out once for a face where the impedance rises by more than 1.5x."""
    op = element_media_op(2, 2)
    m = op.mesh
    rho, cp, cs = synth.element_constant_params(op.K)
    Zp = rho * cp
    elem, face = next((k, f) for k in range(op.K) for f in range(4)
                      if Zp[m.EToE[k, f]] > 1.5 * Zp[k])
    Z1, Z2 = Zp[elem], Zp[m.EToE[elem, face]]
    n = m.nrm[elem, face]
    lam1, mu1 = rho[elem] * (cp[elem] ** 2 - 2 * cs[elem] ** 2), rho[elem] * cs[elem] ** 2
    sig = -(lam1 * np.eye(3) + 2 * mu1 * np.outer(n, n)) / cp[elem]
    q = np.zeros((9, op.K, op.Np))
    q[0:3, elem] = n[:, None]
    q[3:9, elem] = np.array([sig[0, 0], sig[1, 1], sig[2, 2], sig[1, 2],
                             sig[0, 2], sig[0, 1]])[:, None]
    _, t_h, _, _ = interface_states(op, q)
    t_inc = sig @ n
    refl = t_h[:, elem, face] - t_inc[:, None]
    R = (Z2 - Z1) / (Z1 + Z2)
    assert np.abs(refl - R * t_inc[:, None]).max() < 1e-13 * np.abs(t_inc).max()


@pytest.mark.parametrize("N", [1, 2])
def test_upwind_raw_operator_dissipative_on_element_constant_media(N):
    """PA3 with Z- != Z+ on every face but constant on each side of it: the
    energy-weighted raw operator S satisfies S + S^T <= 0 exactly."""
    from test_oracle_physics import assemble, energy_weight
    op = element_media_op(1, N)
    S = energy_weight(op) @ assemble(op, raw=True)
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert ev.max() < 1e-12 * np.abs(S).max()
    assert ev.min() < -1e-3
