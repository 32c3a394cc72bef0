"""Periodic Kuhn tetrahedral mesh of the unit cube, face connectivity, node
traces and affine geometric factors, for the oracle.  Plain FP64 NumPy.

Mesh: the cube [0,1]^3 is cut into n^3 hexahedra of side H = 1/n, hexahedron
(i, j, k) with index i + n*(j + n*k); each is split into six Kuhn tetrahedra
along its main diagonal, one per permutation (a, b, c) of the axes in
lexicographic order: corner x0, then x0 + H e_a, x0 + H (e_a + e_b),
x0 + H (1,1,1).  For odd permutations the last two vertices are swapped so
that every element has positive orientation.  Element index = 6*hex + perm.
build_mesh also takes other meshes of the same cube whose face centroids lie
on the lattice of H/12: the Kuhn cube with elements split at their centroids
into four, which gives odd element counts and non-Kuhn element shapes.
Vertex coordinates are kept unwrapped per element; periodicity enters only
through face matching (face centroids compared modulo 1) and trace pairing
(node coordinates compared after shifting the neighbour face by the integer
period vector that maps its centroid onto this face's centroid).

Geometry (affine map x = x0 + F (r+1, s+1, t+1)/2 with F = [x1-x0, x2-x0,
x3-x0]/2): metric terms are the rows of F^-1, J = det F, outward unit
normals from the physical face vertices, and sJ_f the area element of face f
with respect to the parameters used for its face mass matrix, so that the
lifting scale is Fscale_f = sJ_f / J [HW08, Ch. 10].

Pins (tests/test_oracle_pins.py): element volumes sum to 1 and are positive;
matched faces have opposite normals and equal area elements; paired trace
nodes coincide modulo the period; each face appears exactly twice.
"""
from __future__ import annotations

from dataclasses import dataclass
from itertools import permutations

import numpy as np

from .refelem import FACE_VERTS, RefElement, face_params

PERMS = list(permutations(range(3)))


def _perm_parity(p):
    inv = sum(1 for i in range(3) for j in range(i + 1, 3) if p[i] > p[j])
    return inv % 2


def kuhn_vertices(n):
    """Per-element vertex coordinates [K, 4, 3] of the periodic Kuhn mesh."""
    H = 1.0 / n
    ii, jj, kk = np.meshgrid(np.arange(n), np.arange(n), np.arange(n),
                             indexing="ij")
    # hex index i + n*(j + n*k): i fastest
    corner = np.stack([ii.transpose(2, 1, 0).ravel(),
                       jj.transpose(2, 1, 0).ravel(),
                       kk.transpose(2, 1, 0).ravel()], axis=-1).astype(np.float64)
    eye = np.eye(3)
    tets = []
    for p in PERMS:
        a, b, _ = p
        v0 = np.zeros(3)
        v1 = eye[a]
        v2 = eye[a] + eye[b]
        v3 = np.ones(3)
        if _perm_parity(p) == 1:
            v2, v3 = v3, v2
        tets.append(np.stack([v0, v1, v2, v3]))
    tets = np.stack(tets)                              # [6, 4, 3]
    X = (corner[:, None, None, :] + tets[None, :, :, :]) * H   # [n^3, 6, 4, 3]
    return X.reshape(-1, 4, 3)


@dataclass
class Mesh:
    n: int
    K: int
    VX: np.ndarray       # [K, 4, 3] vertex coordinates
    x: np.ndarray        # [K, Np, 3] node coordinates
    xq: np.ndarray       # [K, Nq, 3] quadrature point coordinates
    EToE: np.ndarray     # [K, 4] neighbour element across each face
    EToF: np.ndarray     # [K, 4] neighbour's face index
    rx: np.ndarray       # [K, 3, 3]: rx[k, i, j] = d(r_i)/d(x_j)
    J: np.ndarray        # [K]
    nrm: np.ndarray      # [K, 4, 3] outward unit normals
    sJ: np.ndarray       # [K, 4]
    Fscale: np.ndarray   # [K, 4]
    vmapM: np.ndarray    # [K, 4, Nfp] flat own node index  k*Np + node
    vmapP: np.ndarray    # [K, 4, Nfp] flat neighbour node index


def _face_keys(VX, n):
    """Integer key of each face centroid modulo the period.  Centroids of
    Kuhn faces are multiples of H/3, and those of the faces made by splitting
    a Kuhn element at its centroid multiples of H/12, so 12n * centroid is
    integral."""
    K = VX.shape[0]
    keys = np.empty((K, 4), dtype=np.int64)
    m = 12 * n
    for f, fv in enumerate(FACE_VERTS):
        c = VX[:, list(fv), :].sum(axis=1) / 3.0            # [K, 3]
        ci = np.mod(np.rint(c * m).astype(np.int64), m)
        keys[:, f] = ci[:, 0] + m * (ci[:, 1] + m * ci[:, 2])
    return keys


def build_mesh(n: int, ref: RefElement, VX: np.ndarray | None = None) -> Mesh:
    """Geometry and connectivity of the periodic unit cube meshed by VX
    [K, 4, 3] (positively oriented tetrahedra; default the Kuhn cube of n^3 x
    6 elements).  Face centroids must lie on the lattice of H/12, H = 1/n:
    the Kuhn cube, possibly with elements split at their centroids."""
    VX = kuhn_vertices(n) if VX is None else np.asarray(VX, dtype=np.float64)
    K = VX.shape[0]
    Np, Nfp = ref.Np, ref.Nfp

    # affine map
    F = np.stack([VX[:, 1] - VX[:, 0], VX[:, 2] - VX[:, 0],
                  VX[:, 3] - VX[:, 0]], axis=-1) / 2.0          # [K, 3(x), 3(rst)]
    J = np.linalg.det(F)
    rx = np.linalg.inv(F)                                        # [K, rst, x]
    ref_nodes = np.stack([ref.r, ref.s, ref.t], axis=-1) + 1.0
    x = VX[:, None, 0, :] + np.einsum("kij,pj->kpi", F, ref_nodes)
    ref_q = np.stack([ref.rq, ref.sq, ref.tq], axis=-1) + 1.0
    xq = VX[:, None, 0, :] + np.einsum("kij,pj->kpi", F, ref_q)

    # normals and face area elements
    nrm = np.zeros((K, 4, 3))
    sJ = np.zeros((K, 4))
    # reference-parameter tangents of each face: d(r,s,t)/du, d(r,s,t)/dv
    tang = {0: ((1, 0, 0), (0, 1, 0)), 1: ((1, 0, 0), (0, 0, 1)),
            2: ((-1, 1, 0), (-1, 0, 1)), 3: ((0, 1, 0), (0, 0, 1))}
    for f, fv in enumerate(FACE_VERTS):
        tu = F @ np.array(tang[f][0], dtype=np.float64)
        tv = F @ np.array(tang[f][1], dtype=np.float64)
        cr = np.cross(tu, tv)
        area = np.linalg.norm(cr, axis=-1)
        nf = cr / area[:, None]
        opp = [v for v in range(4) if v not in fv][0]
        # orient away from the opposite vertex
        sgn = np.sign(np.einsum("ki,ki->k", nf, VX[:, fv[0]] - VX[:, opp]))
        nrm[:, f] = nf * sgn[:, None]
        sJ[:, f] = area
    Fscale = sJ / J[:, None]

    # face matching by centroid modulo the period
    keys = _face_keys(VX, n).ravel()
    order = np.argsort(keys, kind="stable")
    sk = keys[order]
    if not (np.all(sk[0::2] == sk[1::2]) and
            (len(sk) < 3 or np.all(sk[2::2] != sk[1:-1:2]))):
        raise RuntimeError("face matching failed: a face key is not shared "
                           "by exactly two faces")
    partner = np.empty_like(order)
    partner[order[0::2]] = order[1::2]
    partner[order[1::2]] = order[0::2]
    EToE = (partner // 4).reshape(K, 4)
    EToF = (partner % 4).reshape(K, 4)

    # trace pairing by node coordinates modulo the period
    vmapM = np.zeros((K, 4, Nfp), dtype=np.int64)
    vmapP = np.zeros((K, 4, Nfp), dtype=np.int64)
    kk = np.arange(K)
    tol = 1e-8 / n
    chunk = 32768
    for f in range(4):
        vmapM[:, f, :] = kk[:, None] * Np + ref.Fmask[f][None, :]
        for k0 in range(0, K, chunk):
            sl = slice(k0, min(K, k0 + chunk))
            xm = x[sl][:, ref.Fmask[f], :]                      # [k, Nfp, 3]
            nb = EToE[sl, f]
            nbmask = ref.Fmask[EToF[sl, f]]                     # [k, Nfp]
            xp = x[nb[:, None], nbmask, :]                      # [k, Nfp, 3]
            # the periodic image of the neighbour face that coincides with
            # this face: an integer shift fixed by the two face centroids
            # (comparing single nodes modulo 1 is ambiguous when n = 1)
            shift = np.rint(xm.mean(axis=1) - xp.mean(axis=1))  # [k, 3]
            d = xm[:, :, None, :] - (xp + shift[:, None, :])[:, None, :, :]
            dist = np.sqrt(np.sum(d * d, axis=-1))              # [k, Nfp, Nfp]
            jmin = np.argmin(dist, axis=-1)
            if np.any(np.take_along_axis(dist, jmin[..., None], -1) > tol):
                raise RuntimeError("trace pairing failed")
            vmapP[sl, f, :] = (nb[:, None] * Np
                               + np.take_along_axis(nbmask, jmin, -1))
    return Mesh(n=n, K=K, VX=VX, x=x, xq=xq, EToE=EToE, EToF=EToF, rx=rx,
                J=J, nrm=nrm, sJ=sJ, Fscale=Fscale, vmapM=vmapM, vmapP=vmapP)


def face_param_check(ref: RefElement):
    """Face parameters of each face's nodes (used by tests)."""
    return [face_params(f, ref.r[ref.Fmask[f]], ref.s[ref.Fmask[f]],
                        ref.t[ref.Fmask[f]]) for f in range(4)]
