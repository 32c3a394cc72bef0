"""CPU tests of libdg's host side (host-only context, no GPU): the C-ABI
exports, the FP64 reference element, connectivity and geometry against the
independently written oracle, and the argument/state validation."""
import re
import os

import numpy as np
import pytest

import synth
from oracle.mesh import build_mesh, kuhn_vertices
from oracle.refelem import ref_element

B = pytest.importorskip("paper_2008_09441_amd._binding")
from paper_2008_09441_amd import Solver  # noqa: E402

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "dg.h")


def test_library_exports_every_declared_symbol():
    src = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:dg_status|void|const char\*)\s+(dg_\w+)\s*\(",
                              src, re.M))
    assert len(declared) >= 18
    for name in declared:
        assert hasattr(B.lib, name), name
    assert declared == set(B.EXPORTS)


def _host(N, n=None, media=None):
    s = Solver(N, precision="fp64", device=-1)
    if n is not None:
        s.upload_mesh(synth.kuhn_cube_vertices(n))
    return s


def test_kuhn_vertices_match_between_input_generator_and_oracle():
    for n in (1, 2, 3):
        assert np.array_equal(synth.kuhn_cube_vertices(n), kuhn_vertices(n))


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7])
def test_reference_operators_match_oracle(N):
    s = _host(N)
    ro = ref_element(N)
    tol = 1e-12 * max(1.0, np.abs(ro.Dr).max())
    assert np.abs(s_op(s, 6) - np.stack([ro.r, ro.s, ro.t], 1)).max() < 1e-15
    for w, ref in ((0, ro.Dr), (1, ro.Ds), (2, ro.Dt)):
        assert np.abs(s_op(s, w) - ref).max() < tol
    assert np.array_equal(B.dg_face_nodes(s.ctx), ro.Fmask)
    L = s_op(s, 3)
    assert np.abs(L - ro.LIFT).max() < 1e-11 * np.abs(ro.LIFT).max()
    assert np.abs(s_op(s, 4) - ro.Vq).max() < 1e-12
    assert np.abs(s_op(s, 5) - ro.Pq).max() < 1e-11 * np.abs(ro.Pq).max()
    qw = s_op(s, 7)
    assert np.abs(qw - np.stack([ro.rq, ro.sq, ro.tq, ro.wq], 1)).max() < 1e-14


def s_op(s, w):
    return B.dg_ref_operator(s.ctx, w)


@pytest.mark.parametrize("n,N", [(1, 1), (2, 3), (3, 2), (4, 4)])
def test_connectivity_and_geometry_match_oracle(n, N):
    s = _host(N, n)
    ro = ref_element(N)
    m = build_mesh(n, ro)
    etoe, etof, nbn = B.dg_connectivity(s.ctx)
    assert np.array_equal(etoe, m.EToE)
    assert np.array_equal(etof, m.EToF)
    # the oracle's flat neighbour index = k' * Np + node
    assert np.array_equal(etoe[:, :, None] * ro.Np + nbn, m.vmapP)
    geo, fgeo, J = B.dg_geometry(s.ctx)
    assert np.abs(geo.reshape(-1, 3, 3) - m.rx).max() < 1e-12 * n
    assert np.abs(J - m.J).max() < 1e-15
    assert np.abs(fgeo[..., :3] - m.nrm).max() < 1e-13
    assert np.abs(fgeo[..., 3] - m.Fscale).max() < 1e-10 * m.Fscale.max()
    assert np.abs(s.node_coords() - m.x).max() < 1e-14
    assert np.abs(s.quad_coords() - m.xq).max() < 1e-14


def test_projection_matches_oracle():
    from oracle.dg import ElasticDG
    op = ElasticDG(2, 3, synth.homogeneous_media)
    s = _host(3, 2)
    fq = synth.gaussian_pulse(op.mesh.xq, width=0.2)
    assert np.abs(s.project(fq) - op.project(fq)).max() < 1e-13


def test_validation_and_state_errors():
    with pytest.raises(B.DGError) as e:
        B.dg_create(0, B.DG_FP64, B.DG_FLUX_UPWIND, -1)
    assert e.value.status == B.DG_EINVAL
    with pytest.raises(B.DGError):
        B.dg_create(3, 7, B.DG_FLUX_UPWIND, -1)
    s = _host(2)
    # material before mesh -> state error
    a = np.ones(64)
    assert B.lib.dg_material_upload(s.ctx, *[a.ctypes.data] * 6) == B.DG_ESTATE
    assert "mesh" in B.lib.dg_last_error(s.ctx).decode()
    # inverted element
    v = synth.kuhn_cube_vertices(2)
    bad = v.copy()
    bad[5, [2, 3]] = bad[5, [3, 2]]
    with pytest.raises(B.DGError) as e:
        s.upload_mesh(bad)
    assert e.value.status == B.DG_EINVAL and "orientation" in str(e.value)
    # a box that is not periodic at this size: faces do not match
    with pytest.raises(B.DGError) as e:
        s.upload_mesh(v, period=(2.0, 1.0, 1.0))
    assert e.value.status == B.DG_EINVAL and "match" in str(e.value)
    # non-finite vertex
    nanv = v.copy()
    nanv[0, 0, 0] = np.nan
    with pytest.raises(B.DGError) as e:
        s.upload_mesh(nanv)
    assert e.value.status == B.DG_ENONFINITE
    s.upload_mesh(v)
    K, Np, _, Nq = s.sizes()
    assert K == 48
    ones_q, ones_n = np.ones((K, Nq)), np.ones((K, Np))
    with pytest.raises(B.DGError) as e:
        B.dg_material_upload(s.ctx, -ones_q, 2 * ones_q, ones_q, ones_n, 2 * ones_n, ones_n)
    assert e.value.status == B.DG_EINVAL
    with pytest.raises(B.DGError) as e:
        B.dg_material_upload(s.ctx, ones_q, ones_q, ones_q, ones_n, 2 * ones_n, ones_n)
    assert e.value.status == B.DG_EINVAL      # cp < sqrt(2) cs
    nanq = ones_q.copy()
    nanq[3, 4] = np.inf
    with pytest.raises(B.DGError) as e:
        B.dg_material_upload(s.ctx, nanq, 2 * ones_q, ones_q, ones_n, 2 * ones_n, ones_n)
    assert e.value.status == B.DG_ENONFINITE
    B.dg_material_upload(s.ctx, ones_q, 2 * ones_q, ones_q, ones_n, 2 * ones_n, ones_n)
    # compute calls on a host-only context report a device error
    with pytest.raises(B.DGError) as e:
        B.dg_step(s.ctx, 0.0, 1e-3)
    assert e.value.status == B.DG_EDEVICE
    z = np.zeros(9 * K * Np)
    assert B.lib.dg_rhs(s.ctx, z.ctypes.data, z[1:].ctypes.data, 0.0) == B.DG_EDEVICE
    with pytest.raises(ValueError):
        B.dg_rhs(s.ctx, z, z)        # host arrays are rejected by the binding
    s.close()


def test_wrong_shapes_rejected_before_the_library():
    s = _host(2, 1)
    with pytest.raises(ValueError):
        B.dg_material_upload(s.ctx, *[np.ones((6, 26))] * 3, *[np.ones((6, 10))] * 3)
    with pytest.raises(ValueError):
        B.dg_mesh_upload(s.ctx, np.zeros((6, 3, 3)), np.ones(3))


def test_sources_and_receivers_need_a_device_context():
    """A host-only context refuses sources and receivers (they set up device
    arrays) with DG_EDEVICE, after argument checks."""
    from paper_2008_09441_amd import B
    ctx = B.dg_create(2, B.DG_FP64, B.DG_FLUX_UPWIND, -1)
    try:
        B.dg_mesh_upload(ctx, synth.kuhn_cube_vertices(2), np.ones(3))
        with pytest.raises(B.DGError) as e:
            B.dg_sources_set(ctx, [[0.5, 0.5, 0.5]], [[0, 0, 1]], 5.0, 0.2, 1.0)
        assert e.value.status == B.DG_EDEVICE
        with pytest.raises(B.DGError) as e:
            B.dg_receivers_set(ctx, [[0.5, 0.5, 0.5]])
        assert e.value.status == B.DG_EDEVICE
    finally:
        B.dg_destroy(ctx)


@pytest.mark.parametrize("n", [4, 8, 16])
def test_tile_order_sweeps_slabs(n):
    # tile processing order of the matrix-core stage on the Kuhn cube: a
    # permutation; each of the eight launch ranges is one slab of hexahedron
    # layers, swept strip by strip (strips 8 hexahedra wide), so that
    # face-neighbour tiles in the same range run at most two strip
    # cross-sections apart, except across a strip boundary or the periodic
    # seam (at most one pair in 8 of the range's face pairs)
    s = _host(4, n)
    order = B.dg_tile_order(s.ctx)
    K = 6 * n ** 3
    T = (K + 15) // 16
    assert np.array_equal(np.sort(order), np.arange(T))
    pos = np.empty(T, dtype=np.int64)
    pos[order] = np.arange(T)
    per, rem = divmod(T, 8)
    part = np.empty(T, dtype=np.int64)
    for x in range(8):
        b = x * per + min(x, rem)
        part[order[b:b + per + (1 if x < rem else 0)]] = x
    hexes = np.arange(K) // 6
    ijk = np.stack([hexes % n, (hexes // n) % n, hexes // (n * n)], 1)
    tile_of = np.arange(K) // 16
    # one slab axis: every range covers n / 8 layers along it (or one layer)
    layers = [max(len(np.unique(ijk[part[tile_of] == x, a])) for x in range(8))
              for a in range(3)]
    assert min(layers) == max(1, n // 8)
    etoe, _, _ = B.dg_connectivity(s.ctx)
    ea = np.repeat(np.arange(K), 4)
    eb = etoe.reshape(-1)
    ta, tb = tile_of[ea], tile_of[eb]
    same = (part[ta] == part[tb]) & (ta != tb)
    assert same.sum() > 0
    # a strip's cross-section: 8 hexahedra by the slab's layers, in tiles
    cross = -(-6 * min(8, n) * max(1, n // 8) // 16)
    near = np.abs(pos[ta[same]] - pos[tb[same]]) <= 2 * cross
    assert near.mean() >= 7 / 8, near.mean()
