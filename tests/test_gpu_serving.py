"""Serving: continuous batching of independent solves (paper_2008_09441_amd.
serving).  Each result is the same alone and in the mix (bit for bit: the
kernels are deterministic and contexts share nothing), graph replay equals
plain launches, the device-clock run equals the host-time run, a served
trace matches the oracle within the FP32 bound, and admission keeps the
running requests inside the HBM budget."""
import numpy as np
import pytest

import synth
from oracle.dg import ElasticDG
from oracle.source import run_with_receivers

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _small_requests(k=6, precision="fp32"):
    from paper_2008_09441_amd.serving import poisson_workload
    reqs = poisson_workload(k, rate=1e9, n_range=(3, 5), orders=(2, 3, 4), steps=(20, 45),
                            nrec=4, precision=precision, seed=7)
    for r in reqs:
        r.arrival = 0.0
    return reqs


def test_result_same_alone_and_in_the_mix():
    from paper_2008_09441_amd.serving import Server
    reqs = _small_requests()
    print("case serving mix of", len(reqs), "requests", flush=True)
    mix = Server(max_active=len(reqs), chunk=8).run(reqs)
    for r, m in zip(reqs, mix):
        alone = Server(max_active=1, chunk=8).run([r])[0]
        assert np.array_equal(alone.trace, m.trace), r.rid
        assert np.abs(m.trace).max() > 0


def test_graph_replay_equals_plain_launches():
    from paper_2008_09441_amd.serving import Server
    reqs = _small_requests(3)
    a = Server(max_active=3, chunk=7, graphs=True).run(reqs)
    b = Server(max_active=3, chunk=7, graphs=False).run(reqs)
    for x, y in zip(a, b):
        assert np.array_equal(x.trace, y.trace)


def test_device_clock_run_equals_host_time_run_fp64():
    from paper_2008_09441_amd import B, Solver
    n, N, steps, dt, f0 = 3, 3, 30, 2e-3, 6.0
    recs = np.array([[0.5, 0.5, 0.5], [0.2, 0.7, 0.1]])
    out = []
    for mode in ("host", "clock"):
        s = Solver(N, precision="fp64", device=0, stream=torch.cuda.Stream().cuda_stream)
        s.upload_mesh(synth.kuhn_cube_vertices(n))
        s.upload_media(synth.fourier_media)
        s.set_sources([[0.3, 0.4, 0.6]], [[0.0, 1.0, 0.0]], f0, 1.2 / f0, 1.0)
        s.set_receivers(recs)
        B.dg_state_zero(s.ctx)
        if mode == "host":
            out.append(s.run_record(0.0, dt, steps))
        else:
            B.dg_trace_reserve(s.ctx, steps)
            B.dg_time_set(s.ctx, 0.0)
            for _ in range(3):
                B.dg_graph_advance(s.ctx, dt, 10)
            tr = np.empty((steps, 2, 3))
            B.dg_trace_copy(s.ctx, tr, steps)
            t, k = B.dg_time_get(s.ctx)
            assert k == steps and abs(t - steps * dt) < 1e-15
            out.append(tr)
        s.close()
    assert np.abs(out[0] - out[1]).max() <= 1e-13 * np.abs(out[0]).max()


def test_served_trace_matches_oracle_fp32():
    from paper_2008_09441_amd.serving import Request, Server
    rng = np.random.default_rng(3)
    r = Request(rid=0, n=3, N=3, nsteps=40, media_seed=11, src_x=np.array([0.3, 0.6, 0.45]),
                src_d=np.array([0.0, 0.6, 0.8]), f0=8.0, receivers=rng.random((5, 3)))
    res = Server(max_active=1, chunk=10).run([r])[0]
    media = lambda x: synth.fourier_media(x, seed=r.media_seed, n_modes=r.media_modes)  # noqa: E731
    op = ElasticDG(r.n, r.N, media)
    src = [dict(x=r.src_x, d=r.src_d, f0=r.f0, t0=r.t0, amp=1.0)]
    _, ref = run_with_receivers(op, np.zeros((9, op.K, op.Np)), 0.0, r.dt, r.nsteps, src,
                                r.receivers)
    err = np.abs(res.trace - ref).max() / np.abs(ref).max()
    print("served trace vs oracle:", err)
    assert err <= 1e-4


def test_admission_stays_within_budget():
    from paper_2008_09441_amd.serving import Server
    reqs = _small_requests(6)
    big = max(r.footprint() for r in reqs)
    srv = Server(hbm_budget=int(2.5 * big), max_active=6, chunk=8)
    res = srv.run(reqs)
    assert len(res) == 6
    assert srv.stats["peak_footprint_bytes"] <= srv.hbm_budget
    assert srv.stats["peak_active"] >= 1
    print(srv.stats)


def test_footprint_bounds_the_allocations():
    from paper_2008_09441_amd import B
    from paper_2008_09441_amd.serving import prepare
    reqs = _small_requests(2, precision="bf16x3")
    for r in reqs:
        s = prepare(r, torch.cuda.Stream())
        used = B.dg_memory(s.ctx)
        assert 0 < used <= r.footprint()
        s.close()
    r = reqs[0]
    fp = r.footprint()
    r.footprint = lambda: fp // 2          # a budget too small for the request
    with pytest.raises(B.DGError) as e:
        prepare(r, torch.cuda.Stream())
    assert e.value.status == B.DG_ENOMEM


# --------------------------------------------------------------------------
# batched stepping: one launch per stage over a slot table of contexts
# --------------------------------------------------------------------------

def _ctx(n, N, precision, stream, seed, nsteps):
    from paper_2008_09441_amd import B, Solver
    rng = np.random.default_rng(seed)
    s = Solver(N, precision=precision, device=0, stream=stream.cuda_stream)
    s.upload_mesh(synth.kuhn_cube_vertices(n))
    s.upload_media(lambda x: synth.fourier_media(x, seed=seed, n_modes=4))
    f0 = float(rng.uniform(5.0, 15.0))
    s.set_sources(rng.random((1, 3)), rng.standard_normal((1, 3)), f0, 1.2 / f0, 1.0)
    s.set_receivers(rng.random((4, 3)))
    B.dg_trace_reserve(s.ctx, nsteps)
    B.dg_state_zero(s.ctx)
    B.dg_time_set(s.ctx, 0.0)
    return s


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("N", [3, 5])
def test_batched_advance_is_bit_identical_to_each_context_alone(precision, N):
    """Three contexts of different sizes (and time steps) advanced alone with
    dg_advance, and together with dg_batch_advance, in runs of 7 and 5 steps
    (an odd run flips the state buffers): traces, states and clocks agree bit
    for bit.  Order 3 runs the tiled kernel, order 5 the one-element one."""
    from paper_2008_09441_amd import B
    print(f"case batched advance {precision} N={N}", flush=True)
    sizes, steps = (2, 3, 4), (7, 5)
    dts = [0.5 * (1.0 / n) / np.sqrt(2.0) / (4.0 * (N + 1) ** 2) for n in sizes]
    total = sum(steps)
    alone = []
    for i, n in enumerate(sizes):
        st = torch.cuda.Stream()
        s = _ctx(n, N, precision, st, 100 + i, total)
        for k in steps:
            B.dg_advance(s.ctx, dts[i], k)
        tr = np.empty((total, 4, 3), dtype=s.dtype)
        B.dg_trace_copy(s.ctx, tr, total)
        alone.append((tr, s.get_state(), B.dg_time_get(s.ctx)))
        s.close()
    st = torch.cuda.Stream()
    ctxs = [_ctx(n, N, precision, st, 100 + i, total) for i, n in enumerate(sizes)]
    b = B.dg_batch_create(0, 8)
    try:
        for k in steps:
            B.dg_batch_advance(b, st.cuda_stream, [s.ctx for s in ctxs], dts, k)
        for i, s in enumerate(ctxs):
            tr = np.empty((total, 4, 3), dtype=s.dtype)
            B.dg_trace_copy(s.ctx, tr, total)
            assert np.abs(tr).max() > 0
            assert np.array_equal(tr, alone[i][0]), i
            assert np.array_equal(s.get_state(), alone[i][1]), i
            assert B.dg_time_get(s.ctx) == alone[i][2]
    finally:
        B.dg_batch_destroy(b)
        for s in ctxs:
            s.close()


def test_batched_advance_rejects_bad_batches():
    from paper_2008_09441_amd import B
    st = torch.cuda.Stream()
    a = _ctx(2, 3, "fp32", st, 1, 4)
    c = _ctx(2, 4, "fp32", st, 2, 4)
    b = B.dg_batch_create(0, 2)
    try:
        for ctxs in ([a, c], [a, a], [a, a, a]):
            with pytest.raises(B.DGError) as e:
                B.dg_batch_advance(b, st.cuda_stream, [x.ctx for x in ctxs],
                                   [1e-3] * len(ctxs), 1)
            assert e.value.status == B.DG_EINVAL
        from paper_2008_09441_amd import Solver
        d = Solver(3, precision="fp64", device=0, stream=st.cuda_stream)
        d.upload_mesh(synth.kuhn_cube_vertices(2))
        d.upload_media(synth.fourier_media)
        B.dg_state_zero(d.ctx)
        with pytest.raises(B.DGError) as e:
            B.dg_batch_advance(b, st.cuda_stream, [d.ctx], [1e-3], 1)
        assert e.value.status == B.DG_EINVAL
        d.close()
    finally:
        B.dg_batch_destroy(b)
        a.close()
        c.close()


def test_batched_server_results_same_alone_and_in_the_mix():
    """Batched serving: each request's trace is bit-identical served alone,
    in a batched mix and by the per-request graph server."""
    from paper_2008_09441_amd.serving import Server
    reqs = _small_requests(6)
    print("case batched serving mix of", len(reqs), "requests", flush=True)
    srv = Server(max_active=len(reqs), chunk=8, batched=True)
    mix = srv.run(reqs)
    print(srv.stats, "batch launches", srv.batch_launches)
    graphs = Server(max_active=len(reqs), chunk=8).run(reqs)
    for r, m, g in zip(reqs, mix, graphs):
        alone = Server(max_active=1, chunk=8, batched=True).run([r])[0]
        assert np.array_equal(alone.trace, m.trace), r.rid
        assert np.array_equal(g.trace, m.trace), r.rid
        assert np.abs(m.trace).max() > 0
