"""Host-side pieces of the serving layer: the seeded workload generator and
the footprint estimate (no GPU)."""
import numpy as np

from paper_2008_09441_amd import B
from paper_2008_09441_amd.serving import Request, poisson_workload


def test_workload_is_seeded_and_in_range():
    a = poisson_workload(50, rate=10.0, seed=3)
    b = poisson_workload(50, rate=10.0, seed=3)
    assert [(r.n, r.N, r.nsteps, r.arrival) for r in a] == [(r.n, r.N, r.nsteps, r.arrival)
                                                            for r in b]
    assert all(8 <= r.n <= 32 and r.N in (3, 4, 5) and 100 <= r.nsteps <= 800 for r in a)
    arr = np.array([r.arrival for r in a])
    assert np.all(np.diff(arr) > 0)
    assert all(abs(np.linalg.norm(r.src_d) - 1.0) < 1e-12 for r in a)


def test_footprint_grows_with_the_request():
    base = dict(rid=0, media_seed=1, src_x=np.zeros(3), src_d=np.array([0, 0, 1.0]), f0=5.0,
                receivers=np.zeros((16, 3)))
    f = [Request(n=n, N=4, nsteps=100, **base).footprint() for n in (8, 16, 32)]
    assert f[0] < f[1] < f[2]
    # the state and residual alone: 3 x 9 K Np floats
    r = Request(n=16, N=4, nsteps=100, **base)
    assert r.footprint() > 3 * 9 * r.K * r.Np * 4
    assert B.dg_footprint(4, B.DG_FP32, r.K, 1, 16, 200) > r.footprint()
