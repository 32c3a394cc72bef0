"""Continuous-batching server for many independent DG elastic-wave solves on
one GPU.

Each request is one periodic Kuhn cube of n^3 x 6 tetrahedra at order N,
with its own seeded smooth media, one Ricker point force and a set of
receivers, run for a given number of LSRK(5,4) steps.  The server:

* admits requests in arrival order as soon as a slot is free and their
  device footprint (``dg_footprint``: state, media, mesh, sources,
  receivers and the whole receiver trace) fits in the HBM budget that the
  running requests leave; each context is created with that footprint as
  its own budget, so the library refuses to allocate beyond it;
* prepares admitted requests on worker threads (host mesh precompute,
  uploads), while the GPU keeps running the others;
* keeps every request's state resident on the device in its own context,
  on its own stream (default priority), and advances it in chunks of
  ``chunk`` steps: ``dg_graph_advance`` replays a captured hipGraph of the
  chunk's stage, source and receiver kernels, which read the time from the
  context's device clock;
* launches the next chunk of a request as soon as its previous one is
  done, so chunks of different requests overlap on the device, and new
  requests join between chunks (continuous batching);
* or, in batched mode (``batched=True``), keeps one slot table per order
  and precision (``dg_batch_advance``): all running requests of that order
  advance together, each stage of the whole group being one launch over
  the slots, with every request on its own dt and device clock; a chunk
  runs the steps every member still needs at least, requests that finish
  leave and newly prepared ones join at chunk boundaries;
* on completion copies the receiver trace, frees the context and reports
  the request's latency (finish - arrival) and queueing delay.

A request's result does not depend on what else runs: every kernel of the
path is deterministic and contexts share no device memory.
"""
from __future__ import annotations

import concurrent.futures as cf
import math
import time
from dataclasses import dataclass

import numpy as np

from . import _binding as B
from . import PRECISIONS, Solver


@dataclass
class Request:
    rid: int
    n: int                       # hexahedra per cube side: K = 6 n^3
    N: int                       # order
    nsteps: int
    media_seed: int
    src_x: np.ndarray            # [3]
    src_d: np.ndarray            # [3]
    f0: float
    receivers: np.ndarray        # [nrec, 3]
    arrival: float = 0.0         # seconds after the start of the run
    precision: str = "fp32"
    cfl: float = 0.5
    media_modes: int = 4

    @property
    def K(self):
        return 6 * self.n ** 3

    @property
    def Np(self):
        return (self.N + 1) * (self.N + 2) * (self.N + 3) // 6

    @property
    def dt(self):
        # CFL rule with h_min of the Kuhn cube and cp_max = 4
        return self.cfl * (1.0 / self.n) / math.sqrt(2.0) / (4.0 * (self.N + 1) ** 2)

    @property
    def t0(self):
        return 1.2 / self.f0

    def footprint(self):
        return B.dg_footprint(self.N, PRECISIONS[self.precision], self.K, 1,
                              len(self.receivers), self.nsteps)

    def dofs(self):
        return 9 * self.K * self.Np * self.nsteps


@dataclass
class Result:
    rid: int
    trace: np.ndarray            # [nsteps, nrec, 3]
    arrival: float
    admitted: float
    started: float
    finished: float
    footprint: int
    dofs: int

    @property
    def latency(self):
        return self.finished - self.arrival

    @property
    def queued(self):
        return self.admitted - self.arrival


@dataclass
class _Active:
    req: Request
    solver: Solver
    stream: object
    admitted: float
    started: float = 0.0
    done_steps: int = 0
    event: object = None


def _collect(a: _Active):
    """Receiver trace of a finished request, then its context is released
    (worker thread: both wait for the request's stream)."""
    tr = np.empty((a.req.nsteps, len(a.req.receivers), 3), dtype=a.solver.dtype)
    B.dg_trace_copy(a.solver.ctx, tr, a.req.nsteps)
    a.solver.close()
    return tr


def prepare(req: Request, stream, device=0):
    """Context of one request on its stream: mesh, media, source, receivers,
    trace, zero state, clock at 0.  Host-side work; safe on a worker thread."""
    import synth
    s = Solver(req.N, precision=req.precision, flux="upwind", device=device,
               stream=stream.cuda_stream, hbm_budget_bytes=req.footprint())
    s.upload_mesh(synth.kuhn_cube_vertices(req.n))
    s.upload_media(lambda x: synth.fourier_media(x, seed=req.media_seed,
                                                  n_modes=req.media_modes))
    s.set_sources(req.src_x[None], req.src_d[None], req.f0, req.t0, 1.0)
    s.set_receivers(req.receivers)
    B.dg_trace_reserve(s.ctx, req.nsteps)
    B.dg_state_zero(s.ctx)
    B.dg_time_set(s.ctx, 0.0)
    return s


@dataclass
class _Group:
    """Running requests of one order and precision in batched mode: their
    contexts live on one stream and advance through one slot table; up to
    `depth` chunks are queued on the stream at a time, so the device never
    waits for the host between chunks."""
    stream: object
    batch: object
    members: list
    inflight: list


class Server:
    """See the module docstring.  hbm_budget: device bytes the running
    requests may hold together; max_active: running requests at most;
    chunk: steps per launch; graphs: replay captured hipGraphs (else plain
    launches); batched: advance the running requests of each order together
    through dg_batch_advance (then `graphs` is not used)."""

    def __init__(self, hbm_budget=64 << 30, max_active=16, chunk=10, graphs=True,
                 workers=4, device=0, batched=False, depth=2):
        self.hbm_budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.chunk = int(chunk)
        self.graphs = graphs
        self.batched = bool(batched)
        self.depth = int(depth)
        self.workers = int(workers)
        self.device = device
        self.stats = {}
        self._groups = {}
        self.batch_launches = 0

    def _group(self, req: Request):
        import torch
        key = (req.N, req.precision)
        if key not in self._groups:
            self._groups[key] = _Group(torch.cuda.Stream(device=self.device),
                                       B.dg_batch_create(self.device, self.max_active), [], [])
        return self._groups[key]

    def _launch_group(self, g: _Group):
        """Queue one chunk for the members that still have steps to queue:
        the steps every one of them needs at least (at most `chunk`)."""
        import torch
        run = [a for a in g.members if a.done_steps < a.req.nsteps]
        if not run:
            return False
        steps = min([self.chunk] + [a.req.nsteps - a.done_steps for a in run])
        B.dg_batch_advance(g.batch, g.stream.cuda_stream, [a.solver.ctx for a in run],
                           [a.req.dt for a in run], steps)
        self.batch_launches += 1
        ev = torch.cuda.Event()
        ev.record(g.stream)
        for a in run:
            a.done_steps += steps
            a.event = ev            # the chunk that holds the member's latest steps
        g.inflight.append(ev)
        return True

    def _launch_chunk(self, a: _Active):
        import torch
        steps = min(self.chunk, a.req.nsteps - a.done_steps)
        if self.graphs:
            B.dg_graph_advance(a.solver.ctx, a.req.dt, steps)
        else:
            B.dg_advance(a.solver.ctx, a.req.dt, steps)
        a.done_steps += steps
        ev = torch.cuda.Event()
        ev.record(a.stream)
        a.event = ev

    def run(self, requests, clock=time.perf_counter, on_result=None):
        """Serve the requests (arrival times relative to the start); returns
        the results in request order.  on_result(result), if given, is
        called as each request completes."""
        import torch
        for r in requests:
            if r.footprint() > self.hbm_budget:
                raise ValueError(f"request {r.rid} needs {r.footprint()} bytes, more than "
                                 f"the whole budget {self.hbm_budget}")
        order = sorted(requests, key=lambda r: (r.arrival, r.rid))
        results = {}
        finishing = {}                # future -> finished member (batched mode)
        waiting = []                  # arrived, not admitted
        preparing = {}                # future -> (req, stream, admitted)
        active = []
        used = 0
        peak_used, peak_active = 0, 0
        nxt = 0
        pool = cf.ThreadPoolExecutor(max_workers=self.workers)
        start = clock()
        try:
            while len(results) < len(order):
                now = clock() - start
                progressed = False
                while nxt < len(order) and order[nxt].arrival <= now:
                    waiting.append(order[nxt])
                    nxt += 1
                # admission in arrival order while a slot and the budget allow
                while waiting and len(active) + len(preparing) < self.max_active:
                    r = waiting[0]
                    fp = r.footprint()
                    if used + fp > self.hbm_budget:
                        break
                    waiting.pop(0)
                    used += fp
                    peak_used = max(peak_used, used)
                    stream = (self._group(r).stream if self.batched
                              else torch.cuda.Stream(device=self.device))
                    fut = pool.submit(prepare, r, stream, self.device)
                    preparing[fut] = (r, stream, now)
                    progressed = True
                # prepared contexts start running
                for fut in [f for f in preparing if f.done()]:
                    r, stream, adm = preparing.pop(fut)
                    a = _Active(r, fut.result(), stream, adm, started=clock() - start)
                    active.append(a)
                    peak_active = max(peak_active, len(active))
                    if self.batched:
                        self._group(r).members.append(a)   # joins at the next chunk
                    else:
                        self._launch_chunk(a)
                    progressed = True

                def finish(a):
                    nonlocal used
                    tr = np.empty((a.req.nsteps, len(a.req.receivers), 3),
                                  dtype=a.solver.dtype)
                    B.dg_trace_copy(a.solver.ctx, tr, a.req.nsteps)
                    a.solver.close()
                    fin = clock() - start
                    results[a.req.rid] = Result(a.req.rid, tr, a.req.arrival, a.admitted,
                                                a.started, fin, a.req.footprint(),
                                                a.req.dofs())
                    if on_result is not None:
                        on_result(results[a.req.rid])
                    active.remove(a)
                    used -= a.req.footprint()
                if self.batched:
                    # retired chunks, finished members (their trace copy and
                    # context release run on a worker, so that the group's
                    # queued chunks keep the device busy), new chunks
                    for g in self._groups.values():
                        g.inflight = [e for e in g.inflight if not e.query()]
                        for a in [a for a in g.members
                                  if a.done_steps >= a.req.nsteps and a.event.query()]:
                            g.members.remove(a)
                            finishing[pool.submit(_collect, a)] = a
                            progressed = True
                        while len(g.inflight) < self.depth and self._launch_group(g):
                            progressed = True
                    for fut in [f for f in finishing if f.done()]:
                        a = finishing.pop(fut)
                        tr = fut.result()
                        fin = clock() - start
                        results[a.req.rid] = Result(a.req.rid, tr, a.req.arrival, a.admitted,
                                                    a.started, fin, a.req.footprint(),
                                                    a.req.dofs())
                        if on_result is not None:
                            on_result(results[a.req.rid])
                        active.remove(a)
                        used -= a.req.footprint()
                        progressed = True
                else:
                    # next chunk for every request whose chunk is done
                    for a in list(active):
                        if not a.event.query():
                            continue
                        progressed = True
                        if a.done_steps < a.req.nsteps:
                            self._launch_chunk(a)
                            continue
                        finish(a)
                if not progressed:
                    time.sleep(2e-4)
        finally:
            pool.shutdown(wait=True)
            for a in active:
                a.solver.close()
            for g in self._groups.values():
                B.dg_batch_destroy(g.batch)
            self._groups = {}
        end = clock() - start
        res = [results[r.rid] for r in requests]
        lat = np.array([x.latency for x in res])
        first = min(r.arrival for r in requests)
        self.stats = {
            "requests": len(res),
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_queue_s": float(np.mean([x.queued for x in res])),
            "makespan_s": end - first,
            "dof_updates_per_s": float(sum(x.dofs for x in res) / (end - first)),
            "peak_active": peak_active,
            "mode": "batched" if self.batched else ("graphs" if self.graphs else "plain"),
            "peak_footprint_bytes": peak_used,
            "hbm_budget_bytes": self.hbm_budget,
        }
        return res


def poisson_workload(nreq, rate, n_range=(8, 32), orders=(3, 4, 5), steps=(100, 800),
                     f0_range=(5.0, 15.0), nrec=16, precision="fp32", seed=0):
    """Seeded synthetic request stream: Poisson arrivals at `rate` per
    second, n uniform in n_range, N from `orders`, steps uniform in `steps`,
    one Ricker force (f0 uniform in f0_range, random position and direction)
    and nrec random receivers per request."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(nreq):
        t += rng.exponential(1.0 / rate)
        d = rng.standard_normal(3)
        out.append(Request(
            rid=i, n=int(rng.integers(n_range[0], n_range[1] + 1)),
            N=int(rng.choice(orders)), nsteps=int(rng.integers(steps[0], steps[1] + 1)),
            media_seed=int(10_000 + i), src_x=rng.random(3), src_d=d / np.linalg.norm(d),
            f0=float(rng.uniform(*f0_range)), receivers=rng.random((nrec, 3)), arrival=t,
            precision=precision))
    return out
