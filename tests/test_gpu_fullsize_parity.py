"""Parity at the full size of the order-4 heterogeneous workload: the
periodic 48^3 x 6 Kuhn cube (663,552 tets), N = 4, Fourier media, in the
launch configuration the benchmark times (the tiled matrix-core kernel with
its XCD slab tile order, in every precision).

The oracle evaluates the right-hand side on a subset of elements, so the
GPU result is compared element by element on about 2,000 sampled elements:
random ones, every element of the tiles on each side of each XCD slab
boundary in the launch order, the first and last tiles, and elements on the
periodic faces of the cube.  One LSRK step is compared on a smaller sample
through the oracle's own LSRK step, restricted to the elements each stage
must be valid on (the sample, grown by one ring of face neighbours per
remaining stage).

Bounds: FP64 1e-12 per-field relative L2 and max norm (one right-hand side
and one step); FP32 2e-5 and BF16x3 1e-4 for the right-hand side, BF16x3
1e-5 for one step (the state changes by dt times the right-hand side), each
with its max-norm bound (gpu_common.MAX_OVER_L2)."""
import numpy as np
import pytest

import synth
from gpu_common import assert_parity
from oracle.dg import ElasticDG

# the oracle on 663,552 elements takes about a minute to build
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
torch = pytest.importorskip("torch")

n, N = 48, 4


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def oracle_op():
    print(f"building the oracle on {n}^3 x 6 at N = {N}", flush=True)
    op = ElasticDG(n, N, synth.fourier_media)
    # the media samples the library gets, at the oracle's coordinates
    op.media_q = synth.fourier_media(op.mesh.xq)
    op.media_n = synth.fourier_media(op.mesh.x)
    print("oracle built", flush=True)
    return op


@pytest.fixture(scope="module")
def samples(oracle_op):
    op = oracle_op
    from paper_2008_09441_amd import B, Solver
    s = Solver(N, precision="bf16x3", device=0)
    s.upload_mesh(synth.kuhn_cube_vertices(n))
    order = B.dg_tile_order(s.ctx)
    s.close()
    T = order.size
    # XCD slab boundaries: slab x holds launch positions [b_x, b_{x+1})
    per, rem = divmod(T, 8)
    bounds = [x * per + min(x, rem) for x in range(9)]
    pos = {0, T - 1}
    for b in bounds[1:-1]:
        pos.update((b - 1, b))
    tiles = order[sorted(pos)]
    el = set((tiles[:, None] * 16 + np.arange(16)[None, :]).ravel().tolist())
    # elements on the periodic faces (hexahedra with i, j or k at 0 or n-1)
    hexes = np.arange(op.K) // 6
    i, j, k = hexes % n, (hexes // n) % n, hexes // (n * n)
    on_face = np.nonzero((i == 0) | (i == n - 1) | (j == 0) | (j == n - 1)
                         | (k == 0) | (k == n - 1))[0]
    rng = np.random.default_rng(2024)
    el.update(rng.choice(on_face, 300, replace=False).tolist())
    el.update(rng.choice(op.K, 2000 - len(el), replace=False).tolist())
    el = np.array(sorted(x for x in el if x < op.K))
    # a small sample for the LSRK step: slab-boundary tiles and random ones
    step_el = np.unique(np.concatenate([
        tiles[:4] * 16 + 3, (tiles[-4:] * 16 + 11), rng.choice(op.K, 24, replace=False)]))
    print(f"{el.size} sampled elements, {step_el.size} for the step", flush=True)
    return el, step_el


def _solver(op, precision):
    from paper_2008_09441_amd import B, Solver
    s = Solver(N, precision=precision, device=0)
    s.upload_mesh(synth.kuhn_cube_vertices(n))
    B.dg_material_upload(s.ctx, *op.media_q, *op.media_n)
    return s


def _rings(op, el, depth):
    """el grown by `depth` rings of face neighbours: [E_0, ..., E_depth]."""
    out = [np.asarray(el)]
    for _ in range(depth):
        cur = out[-1]
        out.append(np.unique(np.concatenate([cur, op.mesh.EToE[cur].ravel()])))
    return out


def _oracle_step_on(op, q0, el, dt):
    """The oracle's LSRK step, with stage s evaluating the right-hand side
    only on the elements whose stage value the later stages still read."""
    from oracle.dg import lsrk_step
    rings = _rings(op, el, 5)
    stage = [0]

    def F(y, t):
        e = rings[4 - stage[0]]
        stage[0] += 1
        r = np.zeros_like(y)
        r[:, e] = op.rhs(y, e)
        return r
    y, _ = lsrk_step(F, q0, np.zeros_like(q0), 0.0, dt)
    return y[:, el]


@pytest.mark.parametrize("precision,bound", [("fp64", 1e-12), ("fp32", 2e-5), ("bf16x3", 1e-4)])
def test_fullsize_rhs_matches_oracle(oracle_op, samples, precision, bound):
    op = oracle_op
    el, _ = samples
    print(f"case full-size rhs {precision} K={op.K}", flush=True)
    s = _solver(op, precision)
    q = synth.random_state(op.K, op.Np, seed=481)
    if precision != "fp64":
        q = q.astype(np.float32).astype(np.float64)
    got = s.rhs(torch.from_numpy(q).to("cuda:0", s.torch_dtype))
    got = got[:, torch.from_numpy(el).to("cuda:0")].cpu().numpy()
    s.close()
    ref = op.rhs(q, el)
    assert_parity(got, ref, bound, f"full-size rhs {precision}")


@pytest.mark.parametrize("precision,bound", [("fp64", 1e-12), ("bf16x3", 1e-5)])
def test_fullsize_step_matches_oracle(oracle_op, samples, precision, bound):
    op = oracle_op
    _, el = samples
    print(f"case full-size step {precision} K={op.K}", flush=True)
    s = _solver(op, precision)
    q0 = 0.1 * synth.random_state(op.K, op.Np, seed=482)
    q0[0] += op.project(synth.gaussian_pulse_vx(op.mesh.xq))
    if precision != "fp64":
        q0 = q0.astype(np.float32).astype(np.float64)
    dt = 2e-4
    s.set_state(q0)
    s.step(0.0, dt)
    got = s.get_state()[:, el]
    s.close()
    ref = _oracle_step_on(op, q0, el, dt)
    assert_parity(got, ref, bound, f"full-size step {precision}")
