"""Helpers for the GPU parity tests: build the same problem on the oracle and
on libdg from the same seeded inputs, and compare results field by field."""
import numpy as np

import synth
from oracle.dg import ElasticDG

# Element-wise bound relative to the L2 bound.  For an error spread over
# the entries, max|d| / max|ref| stays within about 2x of the per-field
# relative L2 difference (the error's max/rms is 4-5 over 1e4-1e6 entries,
# the reference's rms/max 0.3-0.5); 5x leaves room for that spread, while an
# error confined to a fraction f of the entries is f^(-1/2) times larger in
# the max norm than in L2 and fails it.
MAX_OVER_L2 = 5.0


def rel_l2_per_field(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(9, -1)
    b = np.asarray(b, dtype=np.float64).reshape(9, -1)
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def max_rel_per_field(a, b):
    """Per-field max |a - b| / max |b|."""
    a = np.asarray(a, dtype=np.float64).reshape(9, -1)
    b = np.asarray(b, dtype=np.float64).reshape(9, -1)
    return np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)


def assert_parity(got, ref, l2_bound, what="", max_bound=None):
    """Per-field relative L2 <= l2_bound and per-field max |d| / max |ref| <=
    max_bound (l2_bound for FP64-level bounds, MAX_OVER_L2 x l2_bound for
    reduced precision when not given); prints both."""
    if max_bound is None:
        max_bound = l2_bound if l2_bound <= 1e-10 else MAX_OVER_L2 * l2_bound
    l2 = rel_l2_per_field(got, ref)
    mx = max_rel_per_field(got, ref)
    print(f"{what} per-field rel L2: {np.array2string(l2, precision=2)}", flush=True)
    print(f"{what} per-field max rel:  {np.array2string(mx, precision=2)}", flush=True)
    assert l2.max() <= l2_bound, (what, l2)
    assert mx.max() <= max_bound, (what, mx)
    return l2, mx


def make_pair(n, N, media, flux="upwind", precision="fp64", oracle=True, vertices=None):
    """Oracle operator and libdg solver on the periodic Kuhn cube n^3 x 6 (or
    on the mesh `vertices` derived from it, e.g. with a split element) with
    identical media samples (taken at the oracle's coordinates)."""
    from paper_2008_09441_amd import Solver
    vx = synth.kuhn_cube_vertices(n) if vertices is None else vertices
    mesh = None
    if vertices is not None and oracle:
        from oracle.mesh import build_mesh
        from oracle.refelem import ref_element
        mesh = build_mesh(n, ref_element(N), vertices)
    op = ElasticDG(n, N, media, flux=flux, mesh=mesh) if oracle else None
    s = Solver(N, precision=precision, flux=flux, device=0)
    s.upload_mesh(vx)
    if op is not None:
        xq, xn = op.mesh.xq, op.mesh.x
    else:
        xq, xn = s.quad_coords(), s.node_coords()
    rq, pq, sq = media(xq)
    rn, pn, sn = media(xn)
    from paper_2008_09441_amd import B
    B.dg_material_upload(s.ctx, rq, pq, sq, rn, pn, sn)
    return op, s
