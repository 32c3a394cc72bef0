"""Element-constant media (each element its own rho, cp, cs): the material
jumps across every face, so Z- != Z+ and the general exact-Riemann flux is
exercised on both sides.  GPU right-hand side and one step against the
oracle in every precision."""
import numpy as np
import pytest

import synth
from gpu_common import assert_parity
from oracle.dg import ElasticDG, material_from_samples

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _pair(n, N, precision):
    from paper_2008_09441_amd import B, Solver
    op = ElasticDG(n, N, synth.homogeneous_media, flux="upwind")
    samples = synth.element_constant_samples(op.K, op.ref.Nq, op.Np, seed=12)
    arrs_q, arrs_n = samples[:3], samples[3:]
    op.mat = material_from_samples(*arrs_q, *arrs_n)
    s = Solver(N, precision=precision, flux="upwind", device=0)
    s.upload_mesh(synth.kuhn_cube_vertices(n))
    B.dg_material_upload(s.ctx, *arrs_q, *arrs_n)
    return op, s


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5), ("bf16x3", 1e-4)])
def test_rhs_element_constant_media(precision, tol):
    print(f"case element media rhs {precision}", flush=True)
    op, s = _pair(3, 3, precision)
    q = synth.random_state(op.K, op.Np, seed=71)
    if precision != "fp64":
        q = q.astype(np.float32).astype(np.float64)
    ref = op.rhs(q)
    dt = torch.float64 if precision == "fp64" else torch.float32
    got = s.rhs(torch.from_numpy(q).to("cuda:0", dt)).cpu().numpy()
    assert_parity(got, ref, tol, f"element media rhs {precision}")


def test_step_element_constant_media_fp64():
    op, s = _pair(3, 4, "fp64")
    q0 = synth.random_state(op.K, op.Np, seed=72)
    ref, _ = op.step(q0, np.zeros_like(q0), 1e-3)
    s.set_state(q0)
    s.step(0.0, 1e-3)
    assert_parity(s.get_state(), ref, 1e-12, "element media step fp64")
