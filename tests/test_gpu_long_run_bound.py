"""The stated reduced-precision bounds over the order-4 workload's full run:
48^3 x 6 = 663,552 tets, N = 4, Fourier media, Gaussian velocity pulse,
upwind, 200 LSRK(5,4) steps at CFL 0.5, the FP32 and BF16x3 paths against
the FP64 GPU path (itself pinned to the oracle at 1e-12 per right-hand side
and step, also at this size in test_gpu_fullsize_parity.py).

The error of each field is measured in the energy norm and divided by the
energy norm of the FP64 state (bench.EnergyNorm), which the upwind scheme
does not increase, so one bound holds at every step count: FP32 <= 1e-6 and
BF16x3 <= 1e-5 (bench.ENERGY_BOUND).  Checked after 25 steps (the length of
the short benchmark run), 100 and 200."""
import math

import numpy as np
import pytest

import synth

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_reduced_precision_within_bound_over_200_steps():
    import bench
    from paper_2008_09441_amd import B, Solver
    n, N = 48, 4
    print(f"case long run {n}^3x6 N={N}: sampling media", flush=True)
    solvers = {p: Solver(N, precision=p, flux="upwind", device=0)
               for p in ("fp64", "fp32", "bf16x3")}
    for s in solvers.values():
        s.upload_mesh(synth.kuhn_cube_vertices(n))
    s64 = solvers["fp64"]
    xq = s64.quad_coords()
    media_q = synth.fourier_media(xq)
    media_n = synth.fourier_media(s64.node_coords())
    K, Np = s64.sizes()[:2]
    q0 = np.zeros((9, K, Np))
    q0[0] = s64.project(synth.gaussian_pulse_vx(xq)[None])[0]
    del xq
    for s in solvers.values():
        B.dg_material_upload(s.ctx, *media_q, *media_n)
        s.set_state(q0)
    norm = bench.EnergyNorm(s64, *media_q)
    dt = 0.5 * (1.0 / n) / math.sqrt(2.0) / (4.0 * (N + 1) ** 2)
    done = 0
    worst = {"fp32": 0.0, "bf16x3": 0.0}
    for upto in (25, 100, 200):
        for s in solvers.values():
            s.run(done * dt, dt, upto - done)
        done = upto
        ref = s64.get_state()
        for p in ("fp32", "bf16x3"):
            e = norm.errors(solvers[p].get_state().astype(np.float64), ref, p)
            worst[p] = max(worst[p], e["max"])
            print(f"{p} after {upto} steps, per-field error / energy norm: "
                  f"{np.array2string(np.array(e['rel_per_field_of_energy']), precision=2)}",
                  flush=True)
    for s in solvers.values():
        s.close()
    for p, v in worst.items():
        assert v <= bench.ENERGY_BOUND[p], (p, v)
