"""Helpers for the GPU parity tests: build the same problem on the oracle and
on libdg from the same seeded inputs."""
import numpy as np

import synth
from oracle.dg import ElasticDG


def rel_l2_per_field(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(9, -1)
    b = np.asarray(b, dtype=np.float64).reshape(9, -1)
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


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
