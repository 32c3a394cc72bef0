"""The allocation-free batched step (dg_batch_advance_noalloc): its slot
table is the library's static device array instead of a batch object's
buffer.  Against dg_batch_advance on the same inputs, bit for bit, on two
calls in a row, the second with fewer and smaller contexts (the static
table keeps the first call's contents, which must not leak into the
second); more than 64 contexts are refused."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _ctx(n, N, stream, seed, nsteps):
    from paper_2008_09441_amd import B, Solver
    rng = np.random.default_rng(seed)
    s = Solver(N, precision="fp32", device=0, stream=stream.cuda_stream)
    s.upload_mesh(synth.kuhn_cube_vertices(n))
    s.upload_media(lambda x: synth.fourier_media(x, seed=seed, n_modes=4))
    f0 = float(rng.uniform(5.0, 15.0))
    s.set_sources(rng.random((1, 3)), rng.standard_normal((1, 3)), f0, 1.2 / f0, 1.0)
    s.set_receivers(rng.random((4, 3)))
    B.dg_trace_reserve(s.ctx, nsteps)
    B.dg_state_zero(s.ctx)
    B.dg_time_set(s.ctx, 0.0)
    return s


def _dt(n, N):
    return 0.5 * (1.0 / n) / np.sqrt(2.0) / (4.0 * (N + 1) ** 2)


@pytest.mark.parametrize("N", [3, 5])
def test_noalloc_batch_matches_the_allocating_batch(N):
    from paper_2008_09441_amd import B
    print(f"case no-allocation batch N={N}", flush=True)
    calls = [((2, 3, 4), 6), ((2, 3), 3)]        # the second call: fewer, smaller contexts
    st = torch.cuda.Stream()
    b = B.dg_batch_create(0, 8)
    try:
        for sizes, steps in calls:
            ref = [_ctx(n, N, st, 200 + i, steps) for i, n in enumerate(sizes)]
            got = [_ctx(n, N, st, 200 + i, steps) for i, n in enumerate(sizes)]
            dts = [_dt(n, N) for n in sizes]
            B.dg_batch_advance(b, st.cuda_stream, [s.ctx for s in ref], dts, steps)
            B.dg_batch_advance_noalloc(st.cuda_stream, [s.ctx for s in got], dts, steps)
            for x, y in zip(ref, got):
                tx = np.empty((steps, 4, 3), np.float32)
                ty = np.empty((steps, 4, 3), np.float32)
                B.dg_trace_copy(x.ctx, tx, steps)
                B.dg_trace_copy(y.ctx, ty, steps)
                assert np.abs(tx).max() > 0
                assert np.array_equal(tx, ty)
                assert np.array_equal(x.get_state(), y.get_state())
                assert B.dg_time_get(x.ctx) == B.dg_time_get(y.ctx)
            for s in ref + got:
                s.close()
    finally:
        B.dg_batch_destroy(b)


def test_noalloc_batch_refuses_more_than_its_slots():
    from paper_2008_09441_amd import B
    st = torch.cuda.Stream()
    s = _ctx(2, 3, st, 1, 2)
    with pytest.raises(B.DGError) as e:
        B.dg_batch_advance_noalloc(st.cuda_stream, [s.ctx] * 65, [1e-3] * 65, 1)
    assert e.value.status == B.DG_EINVAL
    assert "at most 64" in str(e.value)
    s.close()
