"""GPU parity of point sources (Ricker forces through the weight-adjusted mass
inverse) and receivers against the oracle (oracle/source.py).

FP64: state and receiver traces within 1e-12 / 1e-11 relative to the oracle
run with the same sources.  FP32 and BF16x3: traces within 1e-4 of the
largest trace value (the per-product errors of BF16x3, ~2^-16, accumulated
over the run)."""
import numpy as np
import pytest

import synth
from gpu_common import assert_parity, make_pair, rel_l2_per_field
from oracle.source import make_forcing, run_with_receivers

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


SOURCES = [dict(x=np.array([0.31, 0.42, 0.27]), d=np.array([0.0, 0.0, 1.0]), f0=6.0,
                t0=1.2 / 6.0, amp=1.5),
           dict(x=np.array([0.77, 0.18, 0.64]), d=np.array([0.6, -0.8, 0.0]), f0=9.0,
                t0=1.2 / 9.0, amp=0.7)]
RECEIVERS = np.array([[0.5, 0.5, 0.5], [0.12, 0.88, 0.33], [0.31, 0.42, 0.27]])


def _set(s, sources=SOURCES, shift=(0.0, 0.0, 0.0)):
    s.set_sources(np.stack([src["x"] + np.asarray(shift) for src in sources]),
                  np.stack([src["d"] for src in sources]),
                  [src["f0"] for src in sources], [src["t0"] for src in sources],
                  [src["amp"] for src in sources])
    s.set_receivers(RECEIVERS)


def _oracle_run(op, nsteps, dt):
    q0 = np.zeros((9, op.K, op.Np))
    return run_with_receivers(op, q0, 0.0, dt, nsteps, SOURCES, RECEIVERS)


def test_rhs_with_sources_fp64():
    print("case rhs+sources fp64 n=3 N=3", flush=True)
    op, s = make_pair(3, 3, synth.fourier_media, "upwind", "fp64")
    _set(s)
    q = synth.random_state(op.K, op.Np, seed=61)
    t = 0.17
    ref = op.rhs(q) + make_forcing(op, SOURCES)(t)
    got = s.rhs(torch.from_numpy(q).to("cuda:0"), t=t).cpu().numpy()
    assert_parity(got, ref, 1e-12, "per-field rel L2")


@pytest.mark.parametrize("flux", ["upwind", "central"])
def test_run_record_fp64(flux):
    print(f"case run_record fp64 n=3 N=3 flux={flux}", flush=True)
    op, s = make_pair(3, 3, synth.fourier_media, flux, "fp64")
    dt, nsteps = 2e-3, 60
    q_ref, tr_ref = _oracle_run(op, nsteps, dt)
    _set(s)
    s.set_state(np.zeros((9, op.K, op.Np)))
    tr = s.run_record(0.0, dt, nsteps)
    q = s.get_state()
    terr = np.abs(tr - tr_ref).max() / np.abs(tr_ref).max()
    print("trace max rel", terr)
    assert np.abs(tr_ref).max() > 1e-4
    assert_parity(q, q_ref, 1e-12, "state")
    assert terr <= 1e-11


def test_sources_at_periodic_image_and_device_trace():
    op, s = make_pair(3, 2, synth.fourier_media, "upwind", "fp64", oracle=False)
    K, Np, _, _ = s.sizes()
    dt, nsteps = 2e-3, 20
    _set(s)
    s.set_state(np.zeros((9, K, Np)))
    a = s.run_record(0.0, dt, nsteps)
    _set(s, shift=(1.0, -2.0, 0.0))
    s.set_state(np.zeros((9, K, Np)))
    dev = torch.empty((nsteps, len(RECEIVERS), 3), dtype=torch.float64, device="cuda:0")
    s.run_record(0.0, dt, nsteps, out=dev)
    torch.cuda.synchronize()
    b = dev.cpu().numpy()
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
    assert np.allclose(s.sample_receivers(), b[-1], rtol=0, atol=1e-15 * np.abs(b).max())


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_run_record_reduced_precision(precision):
    print(f"case run_record {precision} n=3 N=3", flush=True)
    op, s = make_pair(3, 3, synth.fourier_media, "upwind", precision)
    dt, nsteps = 2e-3, 60
    _, tr_ref = _oracle_run(op, nsteps, dt)
    _set(s)
    s.set_state(np.zeros((9, op.K, op.Np)))
    tr = s.run_record(0.0, dt, nsteps).astype(np.float64)
    terr = np.abs(tr - tr_ref).max() / np.abs(tr_ref).max()
    print(precision, "trace error / max:", terr)
    assert terr <= 1e-4


def test_source_argument_errors():
    from paper_2008_09441_amd import B, Solver
    s = Solver(2, precision="fp64", device=0)
    s.upload_mesh(synth.kuhn_cube_vertices(2))
    with pytest.raises(B.DGError) as e:      # material first
        s.set_sources([[0.5, 0.5, 0.5]], [[0, 0, 1]], 5.0, 0.2)
    assert e.value.status == B.DG_ESTATE
    op, s = make_pair(2, 2, synth.homogeneous_media, "upwind", "fp64", oracle=False)
    with pytest.raises(B.DGError) as e:
        s.set_sources([[0.5, 0.5, 0.5]], [[0, 0, 1]], 0.0, 0.2)
    assert e.value.status == B.DG_EINVAL
    with pytest.raises(B.DGError) as e:
        s.set_sources([[0.5, np.nan, 0.5]], [[0, 0, 1]], 5.0, 0.2)
    assert e.value.status == B.DG_ENONFINITE
    K, Np, _, _ = s.sizes()
    s.set_state(np.zeros((9, K, Np)))
    with pytest.raises(B.DGError) as e:      # no receivers yet
        B.dg_receivers_sample(s.ctx, np.empty((1, 3)), False)
    assert e.value.status == B.DG_ESTATE
