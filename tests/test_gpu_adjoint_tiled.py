"""The tiled FP32 adjoint on the matrix cores (orders 1-4: dgt::adj_tile<N>
and dgt::adj_nodes, reading R y and, for the upwind flux, the face-node
jumps that the replay's stage kernel stores) against the FP64 generic
adjoint kernels on the same run (run on an MI355X): gradients in the
weights m = (1/rho, lam, mu) and,
for the upwind flux, in the impedances (Zp, Zs), with point sources and
receivers and a ragged last checkpoint interval, on the Kuhn mesh and on
an odd element count (a ragged last element tile).  The FP64 path matches
the oracle's discrete adjoint to 1e-10 (test_gpu_adjoint.py); the FP32 one
must agree with it to 1e-5 (per-field relative L2; measured 1e-7 to 7e-7
over these cases), and two reverse sweeps of one forward run must give
bit-identical gradients (no atomics)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


SRC = [dict(x=np.array([0.3, 0.6, 0.2]), d=np.array([0.2, -0.4, 0.9]), f0=3.0, t0=1.2 / 3.0),
       dict(x=np.array([0.8, 0.1, 0.7]), d=np.array([-0.5, 0.3, 0.1]), f0=4.0, t0=0.3)]
RECS = np.array([[0.7, 0.25, 0.55], [0.15, 0.8, 0.4], [0.5, 0.5, 0.9]])


def _solver(n, N, flux, precision, vx):
    from paper_2008_09441_amd import B, Solver
    s = Solver(N, precision=precision, flux=flux, device=0)
    s.upload_mesh(vx)
    xq, xn = s.quad_coords(), s.node_coords()
    rq, pq, sq = synth.fourier_media(xq, seed=11)
    rn, pn, sn = synth.fourier_media(xn, seed=11)
    m = np.stack([1.0 / rq, rq * (pq ** 2 - 2 * sq ** 2), rq * sq ** 2])
    zp, zs = rn * pn, rn * sn
    B.dg_material_set_weights(s.ctx, m[0], m[1], m[2], zp, zs)
    s.set_sources(np.stack([x["x"] for x in SRC]), np.stack([x["d"] for x in SRC]),
                  [x["f0"] for x in SRC], [x["t0"] for x in SRC], 1.0)
    s.set_receivers(RECS)
    return s, m, zp


def _grads(s, m, zp, q0, dt, nsteps, every, d, sweeps=1):
    from paper_2008_09441_amd import B
    s.set_state(q0.astype(s.dtype))
    tr = np.empty((nsteps, len(RECS), 3), dtype=s.dtype)
    B.dg_adjoint_forward(s.ctx, 0.0, dt, nsteps, every, tr)
    out = []
    for _ in range(sweeps):
        g = np.empty(m.shape)
        gz = np.empty((2,) + zp.shape)
        B.dg_adjoint_backward(s.ctx, (tr - d).astype(s.dtype), g, gz)
        out.append((g, gz))
    return tr, out


def _rel(a, b):
    a, b = a.reshape(len(b), -1), b.reshape(len(b), -1)
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


@pytest.mark.parametrize("n,N,flux,split", [(2, 1, "upwind", False), (2, 2, "central", True),
                                            (2, 3, "upwind", True), (3, 4, "upwind", False),
                                            (2, 4, "central", True)])
def test_tiled_fp32_adjoint_matches_the_fp64_adjoint(n, N, flux, split):
    print(f"case tiled adjoint n={n} N={N} {flux} split={split}", flush=True)
    vx = synth.kuhn_cube_vertices(n)
    if split:
        vx = synth.split_tet_vertices(vx)
    s64, m, zp = _solver(n, N, flux, "fp64", vx)
    s32, _, _ = _solver(n, N, flux, "fp32", vx)
    K, Np, _, _ = s64.sizes()
    q0 = synth.random_state(K, Np, seed=9) * 0.1
    dt, nsteps, every = 0.004, 11, 4
    d = np.random.default_rng(7).standard_normal((nsteps, len(RECS), 3)) * 0.05
    tr64, [(g64, z64)] = _grads(s64, m, zp, q0, dt, nsteps, every, d)
    tr32, [(g32, z32), (g32b, z32b)] = _grads(s32, m, zp, q0, dt, nsteps, every, d, sweeps=2)
    s64.close()
    s32.close()
    assert np.isfinite(g32).all() and np.isfinite(z32).all()
    assert np.array_equal(g32, g32b) and np.array_equal(z32, z32b)
    eg = _rel(g32, g64)
    print("gradient m, FP32 tiled vs FP64, per field:", np.array2string(eg, precision=2))
    assert eg.max() <= 1e-5
    if flux == "upwind":
        ez = _rel(z32, z64)
        print("gradient z, FP32 tiled vs FP64, per field:", np.array2string(ez, precision=2))
        assert np.linalg.norm(z64) > 0 and ez.max() <= 1e-5
    else:
        assert not z32.any()


@pytest.mark.parametrize("flux", ["upwind", "central"])
def test_generic_fp32_adjoint_order5_matches_the_fp64_adjoint(flux):
    """FP32 contexts above order 4 keep the generic adjoint kernels: their
    gradients against the FP64 adjoint of the same run, as above."""
    print(f"case generic FP32 adjoint N=5 {flux}", flush=True)
    n, N = 2, 5
    vx = synth.kuhn_cube_vertices(n)
    s64, m, zp = _solver(n, N, flux, "fp64", vx)
    s32, _, _ = _solver(n, N, flux, "fp32", vx)
    K, Np, _, _ = s64.sizes()
    q0 = synth.random_state(K, Np, seed=19) * 0.1
    dt, nsteps, every = 0.002, 7, 3
    d = np.random.default_rng(17).standard_normal((nsteps, len(RECS), 3)) * 0.05
    _, [(g64, z64)] = _grads(s64, m, zp, q0, dt, nsteps, every, d)
    _, [(g32, z32)] = _grads(s32, m, zp, q0, dt, nsteps, every, d)
    s64.close()
    s32.close()
    eg = _rel(g32, g64)
    print("gradient m, FP32 generic vs FP64, per field:", np.array2string(eg, precision=2))
    assert np.isfinite(g32).all() and eg.max() <= 1e-5
    if flux == "upwind":
        ez = _rel(z32, z64)
        print("gradient z, FP32 generic vs FP64, per field:", np.array2string(ez, precision=2))
        assert ez.max() <= 1e-5
    else:
        assert not z32.any()
