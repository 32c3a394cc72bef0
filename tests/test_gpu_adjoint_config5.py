"""Discrete adjoint at the adjoint workload's size (run on an MI355X): order 4
on the 24^3 x 6 cube (82,944 tets), smooth random media, 4 Ricker forces,
64 receivers, a checkpoint every 20 steps.  40 LSRK(5,4) steps of a smooth
initial state (the workload's 400 would make the 81 forward runs of this
test take minutes).

* FP64: the gradient of J = 1/2 |traces - d|^2 with respect to the
  material fields rho, lam, mu at the quadrature points and at the nodes
  (chained through the weights (1/rho, lam, mu) and the upwind flux's
  impedances Zp = sqrt(rho (lam + 2 mu)), Zs = sqrt(rho mu)) against central
  differences of the same GPU run, which perturb the fields and recompute
  the weights and impedances: along 32 random directions within 1e-6 of the
  sum of the six fields' contributions (step 1e-5: the quotient's truncation
  error ~1e-10, its rounding error ~1e-16 |J| / 1e-5), and along 8
  directions of the nodal fields alone (the impedance path) within 1e-4
  (step 1e-3);
* FP32: each field's gradient against the FP64 one within 1e-3 of the whole
  gradient's norm (the bound of the small-mesh FP32 test); the nodal
  fields' part is a difference of face jumps that FP32 rounding dominates
  for this smooth state, a few percent of its own size and 1e-5 of the
  whole."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


N_CELLS, ORDER, STEPS, EVERY = 24, 4, 40, 20


def _problem():
    rng = np.random.default_rng(55)
    f0 = rng.uniform(5.0, 15.0, 4)
    return dict(src_x=rng.random((4, 3)), src_d=rng.standard_normal((4, 3)), f0=f0,
                t0=1.2 / f0, recs=rng.random((64, 3)), rng=rng)


def _context(precision, pb):
    from paper_2008_09441_amd import B, Solver
    s = Solver(ORDER, precision=precision, flux="upwind", device=0)
    s.upload_mesh(synth.kuhn_cube_vertices(N_CELLS))
    xq, xn = s.quad_coords(), s.node_coords()
    rq, pq, sq = synth.fourier_media(xq, seed=77)
    rn, pn, sn = synth.fourier_media(xn, seed=77)
    # the material fields rho, lam, mu at the quadrature points and nodes
    P = [rq, rq * (pq ** 2 - 2 * sq ** 2), rq * sq ** 2, rn, rn * (pn ** 2 - 2 * sn ** 2),
         rn * sn ** 2]
    m, (zp, zs) = _weights(P)
    B.dg_material_set_weights(s.ctx, m[0], m[1], m[2], zp, zs)
    s.set_sources(pb["src_x"], pb["src_d"], pb["f0"], pb["t0"], 1.0)
    s.set_receivers(pb["recs"])
    q0 = s.project_function(lambda x: synth.plane_p_wave(x, 0.1) + synth.plane_s_wave(x, 0.2)
                            + synth.gaussian_pulse(x, width=0.1))
    return s, P, q0


def _weights(P):
    """m = (1/rho, lam, mu) at the quadrature points, (Zp, Zs) at the nodes."""
    rq, lq, mq, rn, ln, mn = P
    return (np.stack([1.0 / rq, lq, mq]),
            (np.sqrt(rn * (ln + 2.0 * mn)), np.sqrt(rn * mn)))


def _dt():
    return 0.5 * (1.0 / N_CELLS) / math.sqrt(2.0) / (4.0 * (ORDER + 1) ** 2)


def _forward(s, m, zp, zs, q0):
    from paper_2008_09441_amd import B
    B.dg_material_set_weights(s.ctx, m[0], m[1], m[2], zp, zs)
    s.set_state(q0)
    tr = np.empty((STEPS, 64, 3), dtype=s.dtype)
    B.dg_adjoint_forward(s.ctx, 0.0, _dt(), STEPS, EVERY, tr)
    return tr.astype(np.float64)


def _gradient(s, P, q0, d):
    """dJ/dP for the six material fields, by the chain rule from libdg's
    dJ/dm and dJ/d(Zp, Zs)."""
    from paper_2008_09441_amd import B
    m, (zp, zs) = _weights(P)
    tr = _forward(s, m, zp, zs, q0)
    g = np.empty(m.shape)
    gz = np.empty((2,) + zp.shape)
    B.dg_adjoint_backward(s.ctx, (tr - d).astype(s.dtype), g, gz)
    rq, lq, mq, rn, ln, mn = P
    return [-g[0] / rq ** 2, g[1], g[2],
            gz[0] * (ln + 2 * mn) / (2 * zp) + gz[1] * mn / (2 * zs),
            gz[0] * rn / (2 * zp),
            gz[0] * rn / zp + gz[1] * rn / (2 * zs)]


def test_config5_gradient_fp64_matches_central_differences_and_fp32():
    pb = _problem()
    s, P, q0 = _context("fp64", pb)
    m, (zp, zs) = _weights(P)
    d = 0.5 * _forward(s, m, zp, zs, q0)          # synthetic data: half the signal
    g = _gradient(s, P, q0, d)

    def J(PP):
        mm, (zzp, zzs) = _weights(PP)
        return 0.5 * float(np.sum((_forward(s, mm, zzp, zzs, q0) - d) ** 2))
    rng = pb["rng"]
    worst = 0.0
    for _ in range(32):
        dP = [rng.standard_normal(p.shape) * p for p in P]
        eps = 1e-5   # truncation ~eps^2, rounding of J ~1e-16 |J| / eps
        fd = (J([p + eps * dp for p, dp in zip(P, dP)])
              - J([p - eps * dp for p, dp in zip(P, dP)])) / (2 * eps)
        parts = [float(np.sum(gi * dp)) for gi, dp in zip(g, dP)]
        an = float(sum(parts))
        # relative to the sum of the six fields' contributions, which the
        # directional derivative can cancel down to a small |fd|
        worst = max(worst, abs(fd - an) / sum(abs(x) for x in parts))
    print(f"32 directions: max |fd - adjoint| / sum |parts| = {worst:.2e}", flush=True)
    assert worst <= 1e-6
    # the nodal fields alone, which enter only through the flux impedances:
    # for a smooth state the face jumps, and with them dJ/dZ, are small, so
    # these directions get their own check (a larger step: the derivative is
    # ~1e-5 of the weights' part, the rounding of J stays the same)
    worst_z = 0.0
    for _ in range(8):
        dP = [np.zeros_like(p) for p in P[:3]] + [rng.standard_normal(p.shape) * p
                                                   for p in P[3:]]
        eps = 1e-3
        fd = (J([p + eps * dp for p, dp in zip(P, dP)])
              - J([p - eps * dp for p, dp in zip(P, dP)])) / (2 * eps)
        an = float(sum(np.sum(gi * dp) for gi, dp in zip(g, dP)))
        print(f"nodal fields: fd {fd:.6e} adjoint {an:.6e}", flush=True)
        worst_z = max(worst_z, abs(fd - an) / abs(fd))
    print(f"8 nodal directions: max |fd - adjoint| / |fd| = {worst_z:.2e}", flush=True)
    assert worst_z <= 1e-4
    s.close()
    s32, P32, q032 = _context("fp32", pb)
    g32 = _gradient(s32, P32, q032, d)
    s32.close()
    # each field's FP32 gradient against the FP64 one, relative to the norm
    # of the whole gradient: the nodal fields' part (the impedance path) is
    # a difference of face jumps that FP32 rounding dominates for this
    # smooth state (a few percent of its own size), but 1e-5 of the whole
    total = float(np.sqrt(sum(np.sum(b * b) for b in g)))
    for i, (a, b) in enumerate(zip(g32, g)):
        rel = float(np.linalg.norm(a - b) / total)
        own = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        print(f"fp32 gradient {i} vs fp64: {rel:.2e} of the whole, {own:.2e} of its own",
              flush=True)
        assert rel <= 1e-3
