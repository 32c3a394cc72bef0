"""Plant plausible mistakes in the oracle (on the CPU, by rewriting one line
of a method's source) and check that the cheap pins reject each of them.
This shows the pins are strong enough to trust the oracle."""
import inspect
import textwrap

import numpy as np
import pytest

import oracle.dg as odg
import synth
from oracle.dg import ElasticDG


def _mutant(method, old, new):
    src = textwrap.dedent(inspect.getsource(method))
    assert old in src, old
    ns = dict(vars(odg))
    exec(compile(src.replace(old, new, 1), "<mutant>", "exec"), ns)
    return ns[method.__name__]


def _skew_defect(flux):
    op = ElasticDG(1, 1, synth.homogeneous_media, flux=flux)
    n = 9 * op.K * op.Np
    A = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        A[:, j] = op.rhs_raw(e.reshape(9, op.K, op.Np)).ravel()
        e[j] = 0.0
    w = np.array([1, 1, 1, 1, 1, 1, 2, 2, 2], float)
    G = np.kron(np.diag(w), np.kron(np.diag(op.mesh.J), op.ref.M))
    S = G @ A
    if flux == "central":
        return np.abs(S + S.T).max() / np.abs(S).max()
    return np.linalg.eigvalsh(0.5 * (S + S.T)).max() / np.abs(S).max()


def _consistency_rate():
    errs = []
    for n in (2, 4):
        op = ElasticDG(n, 2, synth.homogeneous_media)
        f = lambda x, t: synth.plane_p_wave(x, t) + synth.plane_s_wave(x, t)
        q = op.project_function(lambda x: f(x, 0.0))
        dq = op.project_function(lambda x: (f(x, 1e-6) - f(x, -1e-6)) / 2e-6)
        errs.append(np.sqrt(op.l2_sq(op.rhs(q) - dq).sum() / op.l2_sq(dq).sum()))
    return np.log2(errs[0] / errs[1]), errs[1]


def _homogeneous_defect():
    rho, cp, cs = 2.0, 3.0, 1.5
    lam, mu = rho * (cp * cp - 2 * cs * cs), rho * cs * cs
    op = ElasticDG(1, 2, lambda x: synth.homogeneous_media(x, rho, cp, cs))
    q = synth.random_state(op.K, op.Np, seed=3)
    raw, full = op.rhs_raw(q), op.rhs(q)
    exp = np.empty_like(raw)
    exp[0:3] = raw[0:3] / rho
    tr = raw[3] + raw[4] + raw[5]
    for i in range(3):
        exp[3 + i] = lam * tr + 2 * mu * raw[3 + i]
        exp[6 + i] = 2 * mu * raw[6 + i]
    return np.abs(full - exp).max() / np.abs(exp).max()


def _interface_pins_pass():
    """The pins of test_oracle_riemann.py on element-constant media, where
    Z- != Z+ at every face: single-valued interface state, each side's jump
    condition with its own impedance, normal-incidence transmission."""
    from test_oracle_riemann import (element_media_op, normal_incidence_defect,
                                     riemann_defects)
    op = element_media_op(2, 2)
    q = synth.random_state(op.K, op.Np, seed=41)
    cont, jump = riemann_defects(op, q)
    inc = max(normal_incidence_defect(op, w, 5, 2) for w in ("p", "s"))
    return cont < 1e-13 and jump < 1e-13 and inc < 1e-13


def _all_pins_pass():
    ok_c = _skew_defect("central") < 1e-12
    ok_u = _skew_defect("upwind") < 1e-12
    rate, err = _consistency_rate()
    ok_rate = rate > 1.8 and err < 0.3
    ok_h = _homogeneous_defect() < 1e-12
    return ok_c and ok_u and ok_rate and ok_h and _interface_pins_pass()


MUTATIONS = [
    ("riemann_flux", "dt = 0.5 * jt", "dt = -0.5 * jt"),               # flux sign
    ("riemann_flux", "dv = 0.5 * jv", "dv = 1.0 * jv"),                # flux weight
    ("riemann_flux", "dt = (ZpM * dvn) * nv + ZsM * dvt", "dt = (ZpM * dvn) * nv - ZsM * dvt"),
    ("riemann_flux", "dvn = (ZpP * jvn + jtn) / (ZpM + ZpP)", "dvn = (ZpP * jvn - jtn) / (ZpM + ZpP)"),
    ("riemann_flux", "f[6] = 0.5 * (dv[1] * nv[2] + dv[2] * nv[1])", "f[6] = (dv[1] * nv[2] + dv[2] * nv[1])"),
    ("riemann_flux", "Q[8] * nx + Q[4] * ny + Q[6] * nz", "Q[8] * nx + Q[4] * ny + Q[7] * nz"),
    # the two sides' impedances exchanged: same energy rate, wrong flux
    ("face_flux", "Z = (mat.Zp_n.ravel()[iM], mat.Zp_n.ravel()[iP],",
     "Z = (mat.Zp_n.ravel()[iP], mat.Zp_n.ravel()[iM],"),
    ("face_flux", "mat.Zs_n.ravel()[iM], mat.Zs_n.ravel()[iP])",
     "mat.Zs_n.ravel()[iP], mat.Zs_n.ravel()[iM])"),
    # the traction jump taken with the neighbour's impedance
    ("riemann_flux", "dt = (ZpM * dvn) * nv + ZsM * dvt", "dt = (ZpP * dvn) * nv + ZsM * dvt"),
    ("riemann_flux", "dt = (ZpM * dvn) * nv + ZsM * dvt", "dt = (ZpM * dvn) * nv + ZsP * dvt"),
    # shear impedance in the normal part
    ("riemann_flux", "dvn = (ZpP * jvn + jtn) / (ZpM + ZpP)", "dvn = (ZsP * jvn + jtn) / (ZpM + ZpP)"),
    ("surface", "f = self.face_flux(q, elems) * self.mesh.Fscale[elems][None, :, :, None]",
     "f = self.face_flux(q, elems)"),
    ("volume", "r[6] = 0.5 * (dz[vy] + dy[vz])", "r[6] = (dz[vy] + dy[vz])"),
    ("volume", "r[1] = dx[sxy] + dy[syy] + dz[syz]", "r[1] = dx[sxy] + dy[syy] + dz[sxz]"),
    ("volume", "qe @ ref.Ds.T, qe @ ref.Dt.T", "qe @ ref.Dt.T, qe @ ref.Ds.T"),
    ("volume", 'np.einsum("kij,ifkp->jfkp", rx, gr)', 'np.einsum("kji,ifkp->jfkp", rx, gr)'),
    ("wadg", "out[3 + i] = 2.0 * mu * rq[3 + i]", "out[3 + i] = lam * tr + 2.0 * mu * rq[3 + i]"),
    ("wadg", "out[3 + i] = lam * tr + 2.0 * mu * rq[3 + i]", "out[3 + i] = lam * tr + mu * rq[3 + i]"),
    ("wadg", "return out @ ref.Pq.T", "return out @ ref.Vq"),
]


def test_unmutated_oracle_passes_the_pins():
    assert _all_pins_pass()


@pytest.mark.parametrize("meth,old,new", MUTATIONS)
def test_planted_mistake_is_caught(monkeypatch, meth, old, new):
    owner = ElasticDG if hasattr(ElasticDG, meth) else odg
    monkeypatch.setattr(owner, meth, _mutant(getattr(owner, meth), old, new))
    assert not _all_pins_pass()


def test_planted_lsrk_coefficient_mistake_is_caught(monkeypatch):
    from fractions import Fraction
    bad = list(odg.LSRK_B)
    bad[2] = bad[2] + Fraction(1, 1000)
    monkeypatch.setattr(odg, "LSRK_B", bad)
    zs = np.linspace(-1.0, 1.0, 11)
    R = [odg.lsrk_step(lambda y, t: z * y, 1.0, 0.0, 0.0, 1.0)[0] for z in zs]
    coef = np.polynomial.polynomial.polyfit(zs, R, 5)
    assert not np.allclose(coef, [1, 1, 1 / 2, 1 / 6, 1 / 24, 1 / 200], atol=1e-12)
