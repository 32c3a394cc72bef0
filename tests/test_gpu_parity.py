"""GPU parity of libdg against the FP64 oracle (run on an MI355X).

FP64: per-field relative L2 difference <= 1e-12 for the right-hand side and
for one LSRK(5,4) step.  FP32: per-field relative L2 <= 2e-5 for the
right-hand side (single-precision rounding of O(Np) length contractions,
amplified by the operator norms), measured values printed."""
import numpy as np
import pytest

import synth
from gpu_common import assert_parity, make_pair, rel_l2_per_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", dtype)


CASES = [  # (n, N): several element blocks and a ragged last block
    (3, 1), (3, 2), (3, 3), (4, 3), (3, 4), (2, 5), (2, 6), (2, 7)]


@pytest.mark.parametrize("n,N", CASES)
@pytest.mark.parametrize("flux", ["upwind", "central"])
def test_rhs_fp64_matches_oracle(n, N, flux):
    print(f"case rhs fp64 n={n} N={N} flux={flux}", flush=True)
    op, s = make_pair(n, N, synth.fourier_media, flux, "fp64")
    q = synth.random_state(op.K, op.Np, seed=10 + N)
    ref = op.rhs(q)
    got = s.rhs(_dev(q, torch.float64)).cpu().numpy()
    assert_parity(got, ref, 1e-12, "per-field rel L2")


@pytest.mark.parametrize("n,N", [(3, 3), (3, 4), (2, 7)])
def test_rhs_fp32_matches_oracle(n, N):
    print(f"case rhs fp32 n={n} N={N}", flush=True)
    op, s = make_pair(n, N, synth.fourier_media, "upwind", "fp32")
    q = synth.random_state(op.K, op.Np, seed=20 + N).astype(np.float32).astype(np.float64)
    ref = op.rhs(q)
    got = s.rhs(_dev(q, torch.float32)).cpu().numpy()
    assert_parity(got, ref, 2e-5, "per-field rel L2")


@pytest.mark.parametrize("N", [2, 4, 6])
@pytest.mark.parametrize("precision,bound", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_odd_element_count_fp64_fp32(N, precision, bound):
    """The centroid-split Kuhn cube (K = 51, non-Kuhn element shapes) on the
    FP64 and FP32 matrix-core kernels (the tiled kernels at orders 1-4, one
    element per workgroup at 5-7): right-hand side and one LSRK step
    against the oracle on the same mesh."""
    print(f"case odd K {precision} N={N}", flush=True)
    vx = synth.split_tet_vertices(synth.kuhn_cube_vertices(2))
    op, s = make_pair(2, N, synth.fourier_media, "upwind", precision, vertices=vx)
    dtype = torch.float64 if precision == "fp64" else torch.float32
    q = synth.random_state(op.K, op.Np, seed=70 + N)
    if precision == "fp32":
        q = q.astype(np.float32).astype(np.float64)
    assert_parity(s.rhs(_dev(q, dtype)).cpu().numpy(), op.rhs(q), bound, "rhs")
    dt = 1e-3
    ref, _ = op.step(q, np.zeros_like(q), dt)
    s.set_state(q)
    s.step(0.0, dt)
    assert_parity(s.get_state(), ref, bound, "one step")


@pytest.mark.parametrize("n,N", [(3, 3), (3, 4)])
def test_one_lsrk_step_fp64_matches_oracle(n, N):
    print(f"case step fp64 n={n} N={N}", flush=True)
    op, s = make_pair(n, N, synth.fourier_media, "upwind", "fp64")
    q0 = synth.random_state(op.K, op.Np, seed=30 + N)
    dt = 1e-3
    ref, _ = op.step(q0, np.zeros_like(q0), dt)
    s.set_state(q0)
    s.step(0.0, dt)
    got = s.get_state()
    assert_parity(got, ref, 1e-12, "per-field rel L2")


def test_rhs_is_deterministic():
    op, s = make_pair(3, 4, synth.fourier_media, "upwind", "fp32", oracle=False)
    K, Np, _, _ = s.sizes()
    q = _dev(synth.random_state(K, Np, seed=5), torch.float32)
    a = s.rhs(q)
    b = s.rhs(q)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_plane_wave_order3_workload_fp64():
    """n=4 (384 tets), N=3, rho=1 cp=2 cs=1, plane P wave along (1,1,0),
    upwind, LSRK(5,4) to T=0.5 at CFL 0.5 (182 steps): the GPU run matches
    the oracle run and both are within the discretisation error of the
    exact solution."""
    op, s = make_pair(4, 3, synth.homogeneous_media, "upwind", "fp64")
    q0 = op.project_function(lambda x: synth.plane_p_wave(x, 0.0))
    dt, ns = op.cfl_dt(0.5)
    s.set_state(q0)
    s.run(0.0, dt, ns)
    got = s.get_state()
    ref = op.run(q0, 0.0, dt, ns)
    err = rel_l2_per_field(got, ref)
    print("GPU vs oracle after", ns, "steps:", np.array2string(err, precision=2))
    nz = np.linalg.norm(ref.reshape(9, -1), axis=1) > 1e-8
    assert err[nz].max() <= 1e-11
    qe = op.project_function(lambda x: synth.plane_p_wave(x, 0.5))
    e_exact = np.sqrt(op.l2_sq(got - qe).sum() / op.l2_sq(qe).sum())
    print("error vs exact solution:", e_exact)
    assert e_exact < 1e-2


# --------------------------------------------------------------------------
# BF16x3 matrix-core path: per-field relative L2 against the FP64 oracle.
# Each split product carries ~2^-17 relative error; sums of O(Np) terms with
# operator entries up to ~10 give ~1e-5 on random states.  Bound: 1e-4
# for random and smooth projected states alike (smooth data cancels more in
# the derivative sums, so its relative error is the larger); measured values
# are printed.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,N", [(3, 1), (3, 2), (3, 3), (4, 3), (3, 4), (5, 4), (2, 5),
                                 (2, 6), (2, 7)])
@pytest.mark.parametrize("flux", ["upwind", "central"])
def test_rhs_bf16x3_matches_oracle(n, N, flux):
    print(f"case rhs bf16x3 n={n} N={N} flux={flux}", flush=True)
    op, s = make_pair(n, N, synth.fourier_media, flux, "bf16x3")
    q = synth.random_state(op.K, op.Np, seed=40 + N).astype(np.float32).astype(np.float64)
    ref = op.rhs(q)
    got = s.rhs(_dev(q, torch.float32)).cpu().numpy()
    assert_parity(got, ref, 1e-4, "per-field rel L2")


def test_rhs_bf16x3_smooth_state():
    op, s = make_pair(4, 3, synth.fourier_media, "upwind", "bf16x3")
    q = op.project_function(lambda x: synth.plane_p_wave(x, 0.1) + synth.plane_s_wave(x, 0.2)
                            + synth.gaussian_pulse(x, width=0.15))
    q = q.astype(np.float32).astype(np.float64)
    ref = op.rhs(q)
    got = s.rhs(_dev(q, torch.float32)).cpu().numpy()
    assert_parity(got, ref, 1e-4, "bf16x3")
    _, s32 = make_pair(4, 3, synth.fourier_media, "upwind", "fp32", oracle=False)
    err32 = rel_l2_per_field(s32.rhs(_dev(q, torch.float32)).cpu().numpy(), ref)
    print("fp32   per-field rel L2:", np.array2string(err32, precision=2))


@pytest.mark.parametrize("n,N", [(3, 4), (4, 3), (3, 2), (2, 7)])
def test_one_lsrk_step_bf16x3_matches_oracle(n, N):
    op, s = make_pair(n, N, synth.fourier_media, "upwind", "bf16x3")
    q0 = synth.random_state(op.K, op.Np, seed=50 + N).astype(np.float32).astype(np.float64)
    dt = 1e-3
    ref, _ = op.step(q0, np.zeros_like(q0), dt)
    s.set_state(q0)
    s.step(0.0, dt)
    got = s.get_state()
    assert_parity(got, ref, 1e-5, "per-field rel L2")


@pytest.mark.parametrize("N", [2, 4, 5, 6, 7])
def test_bf16x3_odd_element_count(N):
    """Kuhn cube n = 2 with element 0 split at its centroid (K = 51, odd):
    four elements of a non-Kuhn shape, with face pairings the Kuhn cube does
    not have, and a last 16-element tile of three elements at orders 1-4.
    Right-hand side (bound 1e-4) and one LSRK step (1e-5) against the oracle
    on the same mesh."""
    print(f"case odd K bf16x3 N={N}", flush=True)
    vx = synth.split_tet_vertices(synth.kuhn_cube_vertices(2))
    op, s = make_pair(2, N, synth.fourier_media, "upwind", "bf16x3", vertices=vx)
    assert op.K == 51
    q = synth.random_state(op.K, op.Np, seed=60 + N).astype(np.float32).astype(np.float64)
    assert_parity(s.rhs(_dev(q, torch.float32)).cpu().numpy(), op.rhs(q), 1e-4, "rhs per-field rel L2")
    dt = 1e-3
    ref, _ = op.step(q, np.zeros_like(q), dt)
    s.set_state(q)
    s.step(0.0, dt)
    assert_parity(s.get_state(), ref, 1e-5, "one step per-field rel L2")


def test_bf16x3_rejects_unsupported_order():
    from paper_2008_09441_amd import B
    for N in (0, 8):
        with pytest.raises(B.DGError):
            B.dg_create(N, B.DG_FP32_BF16X3, B.DG_FLUX_UPWIND, 0)
