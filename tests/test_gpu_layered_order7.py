"""Order-7 workload with layered media: five piecewise-constant layers whose
interfaces cut through elements (so Z- != Z+ on faces across an interface
and the weights jump inside elements), on the BF16x3 matrix-core path of
orders 5-7 (run on an MI355X).

* small cube (n = 3, 162 tets) against the FP64 oracle: the right-hand side
  of a random and of a smooth state, and ten LSRK(5,4) steps of the smooth
  state (plane P and S waves plus a Gaussian velocity pulse);
* the 24^3 x 6 cube (82,944 tets) against the FP64 GPU path (itself pinned
  to the oracle at 1e-12 in test_gpu_parity.py): ten steps.

Bound: per-field relative L2 <= 1e-4, the stated bound of the BF16x3 path
(1e-3 for the right-hand side of the smooth state, see the test); measured
values are printed."""
import math
import time

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


def _dt(n, N, cp_max=4.5, cfl=0.5):
    # CFL rule with h_min of the Kuhn cube and the layered media's cp_max
    return cfl * (1.0 / n) / math.sqrt(2.0) / (cp_max * (N + 1) ** 2)


def _smooth(x, width):
    # every field nonzero: plane P and S waves plus a Gaussian velocity pulse
    return (synth.plane_p_wave(x, 0.1) + synth.plane_s_wave(x, 0.2)
            + synth.gaussian_pulse(x, width=width))


def test_layered_order7_bf16x3_matches_oracle():
    n, N = 3, 7
    print(f"case layered bf16x3 n={n} N={N}", flush=True)
    op, s = make_pair(n, N, synth.layered_media, "upwind", "bf16x3")
    # right-hand side of a random state: the stated bound
    q = synth.random_state(op.K, op.Np, seed=77).astype(np.float32).astype(np.float64)
    got = s.rhs(torch.from_numpy(q).to("cuda:0", torch.float32)).cpu().numpy()
    assert_parity(got, op.rhs(q), 1e-4, "rhs (random state) per-field rel L2")
    # right-hand side of a smooth state: the derivative sums cancel, so the
    # 2^-16 error of each split product is relative to sum |D_ij q_j| rather
    # than to |sum D_ij q_j|; at order 7 that ratio is ~10, hence 1e-3
    q0 = op.project_function(lambda x: _smooth(x, 0.15)).astype(np.float32).astype(np.float64)
    got = s.rhs(torch.from_numpy(q0).to("cuda:0", torch.float32)).cpu().numpy()
    assert_parity(got, op.rhs(q0), 1e-3, "rhs (smooth state) per-field rel L2")
    # ten LSRK(5,4) steps of the smooth state: the stated bound on the state
    dt, steps = _dt(n, N), 10
    ref = op.run(q0, 0.0, dt, steps)
    s.set_state(q0)
    s.run(0.0, dt, steps)
    assert_parity(s.get_state(), ref, 1e-4, f"{steps} steps per-field rel L2")


def test_layered_order7_full_size_bf16x3_matches_fp64_gpu():
    from paper_2008_09441_amd import B, Solver
    n, N, steps = 24, 7, 10
    print(f"case layered bf16x3 vs fp64 n={n} N={N}", flush=True)
    solvers = {}
    for prec in ("bf16x3", "fp64"):
        s = Solver(N, precision=prec, flux="upwind", device=0)
        s.upload_mesh(synth.kuhn_cube_vertices(n))
        rq, pq, sq = synth.layered_media(s.quad_coords())
        rn, pn, sn = synth.layered_media(s.node_coords())
        B.dg_material_upload(s.ctx, rq, pq, sq, rn, pn, sn)
        solvers[prec] = s
    q0 = solvers["fp64"].project_function(lambda x: _smooth(x, 0.1))
    q0 = q0.astype(np.float32).astype(np.float64)
    dt = _dt(n, N)
    out = {}
    for prec, s in solvers.items():
        s.set_state(q0)
        s.run(0.0, dt, 1)           # warm-up step
        s.set_state(q0)
        s.synchronize()
        t0 = time.perf_counter()
        s.run(0.0, dt, steps)
        s.synchronize()
        print(f"{prec}: {(time.perf_counter() - t0) / (5 * steps) * 1e3:.3f} ms per stage", flush=True)
        out[prec] = s.get_state()
    assert_parity(out["bf16x3"], out["fp64"], 1e-4, f"{steps} steps per-field rel L2 (bf16x3 vs fp64 GPU)")
