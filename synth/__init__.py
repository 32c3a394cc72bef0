"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds input generators only: material fields sampled at given
points, initial conditions and exact plane-wave fields as functions of
position and time, random states.  It contains none of the discontinuous
Galerkin arithmetic (no basis, no operators, no fluxes), so both the oracle
and the GPU path may take their inputs from here without sharing code.

Field order everywhere is (v_x, v_y, v_z, s_xx, s_yy, s_zz, s_yz, s_xz, s_xy):
three particle velocities followed by the six independent stress components
in Voigt order.
"""
from __future__ import annotations

import numpy as np

NFIELDS = 9


# --------------------------------------------------------------------------
# material fields: each returns (rho, cp, cs) sampled at points x[..., 3]
# --------------------------------------------------------------------------

def homogeneous_media(x, rho=1.0, cp=2.0, cs=1.0):
    """Constant density and wave speeds (the order-3 plane-wave workload)."""
    shp = np.asarray(x).shape[:-1]
    return (np.full(shp, float(rho)), np.full(shp, float(cp)),
            np.full(shp, float(cs)))


def _fourier_unit(x, seed, n_modes=16, kmax=3):
    """A smooth periodic field in [0, 1]: 0.5 * (1 + g / sum|a_m|) with
    g = sum_m a_m cos(2 pi k_m . x + phi_m), k_m integer in [-kmax, kmax]^3
    without the zero vector, a_m ~ U(0.5, 1), phi_m ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    ks = []
    while len(ks) < n_modes:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if np.any(k != 0):
            ks.append(k)
    ks = np.array(ks, dtype=np.float64)
    a = rng.uniform(0.5, 1.0, size=n_modes)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    x = np.asarray(x, dtype=np.float64)
    shp = x.shape[:-1]
    # evaluated with torch's multi-threaded CPU kernels (FP64): the largest
    # workload samples ~1e8 points
    import torch
    xt = torch.from_numpy(np.ascontiguousarray(x.reshape(-1, 3)))
    g = torch.zeros(xt.shape[0], dtype=torch.float64)
    for m in range(n_modes):
        arg = xt @ torch.from_numpy(2.0 * np.pi * ks[m])
        arg += phi[m]
        g.add_(torch.cos_(arg), alpha=float(a[m]))
    g = g.numpy().reshape(shp)
    return 0.5 * (1.0 + g / np.sum(np.abs(a)))


def fourier_media(x, seed=9441, n_modes=16):
    """Smooth heterogeneous media from three independent seeded sums of
    n_modes (16) random Fourier modes: rho in [1, 3], cp in [2, 4],
    cs = cp / [1.6, 2.0]."""
    s_rho = _fourier_unit(x, seed + 0, n_modes)
    s_p = _fourier_unit(x, seed + 1, n_modes)
    s_r = _fourier_unit(x, seed + 2, n_modes)
    rho = 1.0 + 2.0 * s_rho
    cp = 2.0 + 2.0 * s_p
    cs = cp / (1.6 + 0.4 * s_r)
    return rho, cp, cs


def layered_params(seed=9443, n_layers=5, n_cells=24):
    """Interface depths and per-layer (rho, cp, cs) of the layered workload.

    Four interface depths z_1 < ... < z_4 drawn in (0, 1), redrawn while any
    lies within 1e-3 of an element-layer boundary j / n_cells, so that the
    interfaces cut through elements.  cp is drawn per layer and rescaled
    affinely onto [1.5, 4.5] (a contrast of exactly 3x); cs = cp / 1.8;
    rho ~ U[1, 3].
    """
    rng = np.random.default_rng(seed)
    while True:
        z = np.sort(rng.uniform(0.0, 1.0, size=n_layers - 1))
        dist = np.abs(z * n_cells - np.round(z * n_cells)) / n_cells
        if np.all(dist > 1e-3) and np.all(np.diff(z) > 1e-3):
            break
    cp = rng.uniform(1.5, 4.5, size=n_layers)
    cp = 1.5 + 3.0 * (cp - cp.min()) / (cp.max() - cp.min())
    cs = cp / 1.8
    rho = rng.uniform(1.0, 3.0, size=n_layers)
    return z, rho, cp, cs


def layered_media(x, seed=9443, n_cells=24):
    """Five piecewise-constant layers in z (periodic: z mod 1); a point with
    z >= z_i belongs to the layer above interface i."""
    z_if, rho_l, cp_l, cs_l = layered_params(seed, n_cells=n_cells)
    z = np.mod(np.asarray(x, dtype=np.float64)[..., 2], 1.0)
    layer = np.searchsorted(z_if, z, side="right")
    return rho_l[layer], cp_l[layer], cs_l[layer]


# --------------------------------------------------------------------------
# initial conditions and exact solutions: each returns fields[9, ...]
# --------------------------------------------------------------------------

def gaussian_pulse_vx(x, x0=(0.5, 0.5, 0.5), width=0.05):
    """The only nonzero field of the Gaussian velocity pulse:
    v_x = exp(-|x - x0|^2 / (2 w^2))."""
    x = np.asarray(x, dtype=np.float64)
    d = x - np.asarray(x0, dtype=np.float64)
    return np.exp(-np.sum(d * d, axis=-1) / (2.0 * width * width))


def gaussian_pulse(x, x0=(0.5, 0.5, 0.5), width=0.05):
    """v_x = exp(-|x - x0|^2 / (2 w^2)), every other field zero."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((NFIELDS,) + x.shape[:-1])
    out[0] = gaussian_pulse_vx(x, x0, width)
    return out


def _voigt(m):
    """3x3 symmetric tensor -> six Voigt components (xx, yy, zz, yz, xz, xy)."""
    return np.array([m[0, 0], m[1, 1], m[2, 2], m[1, 2], m[0, 2], m[0, 1]])


def plane_p_wave(x, t, rho=1.0, cp=2.0, cs=1.0, kvec=(2 * np.pi, 2 * np.pi, 0.0)):
    """Exact periodic plane P wave travelling along k:
    v = d sin(k.x - cp|k| t), sigma = -(1/cp)(lam I + 2 mu d d^T) sin(...),
    with d = k/|k|, lam = rho (cp^2 - 2 cs^2), mu = rho cs^2."""
    k = np.asarray(kvec, dtype=np.float64)
    kn = np.linalg.norm(k)
    d = k / kn
    lam = rho * (cp * cp - 2.0 * cs * cs)
    mu = rho * cs * cs
    x = np.asarray(x, dtype=np.float64)
    ph = np.sin(x @ k - cp * kn * t)
    S = -(lam * np.eye(3) + 2.0 * mu * np.outer(d, d)) / cp
    out = np.empty((NFIELDS,) + x.shape[:-1])
    for i in range(3):
        out[i] = d[i] * ph
    sv = _voigt(S)
    for i in range(6):
        out[3 + i] = sv[i] * ph
    return out


def plane_s_wave(x, t, rho=1.0, cp=2.0, cs=1.0, kvec=(2 * np.pi, 2 * np.pi, 0.0),
                 pol=(0.0, 0.0, 1.0)):
    """Exact periodic plane S wave: v = p sin(k.x - cs|k| t),
    sigma = -(mu/cs)(p d^T + d p^T) sin(...), polarisation p orthogonal to k."""
    k = np.asarray(kvec, dtype=np.float64)
    kn = np.linalg.norm(k)
    d = k / kn
    p = np.asarray(pol, dtype=np.float64)
    p = p - (p @ d) * d
    p = p / np.linalg.norm(p)
    mu = rho * cs * cs
    x = np.asarray(x, dtype=np.float64)
    ph = np.sin(x @ k - cs * kn * t)
    S = -(mu / cs) * (np.outer(p, d) + np.outer(d, p))
    out = np.empty((NFIELDS,) + x.shape[:-1])
    for i in range(3):
        out[i] = p[i] * ph
    sv = _voigt(S)
    for i in range(6):
        out[3 + i] = sv[i] * ph
    return out


def random_state(K, Np, seed=0, dtype=np.float64):
    """A seeded random nodal state of shape [9, K, Np] (values in [-1, 1])."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(NFIELDS, K, Np)).astype(dtype)


# --------------------------------------------------------------------------
# meshes: per-element vertex coordinates [K, 4, 3] of a periodic box
# --------------------------------------------------------------------------

def kuhn_cube_vertices(n, length=1.0):
    """The periodic cube [0, L]^3 cut into n^3 hexahedra (hexahedron
    i + n*(j + n*k) with corner (i, j, k) L/n), each split into the six Kuhn
    tetrahedra that share its main diagonal: for each permutation (a, b, c)
    of the axes in lexicographic order, the path corner -> +e_a -> +e_b ->
    +e_c.  Odd permutations list their last two vertices swapped, so that
    every element is positively oriented.  Element index 6*hex + perm."""
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    odd = [False, True, True, False, False, True]
    local = np.zeros((6, 4, 3))
    for p, (a, b, c) in enumerate(perms):
        path = [np.zeros(3)]
        for ax in (a, b, c):
            nxt = path[-1].copy()
            nxt[ax] += 1.0
            path.append(nxt)
        if odd[p]:
            path[2], path[3] = path[3], path[2]
        local[p] = np.array(path)
    out = np.empty((n, n, n, 6, 4, 3))
    for k in range(n):
        for j in range(n):
            for i in range(n):
                out[k, j, i] = local + np.array([i, j, k], dtype=np.float64)
    return (out * (length / n)).reshape(-1, 4, 3)

def split_tet_vertices(vx, k=0):
    """Element k of a tetrahedral mesh [K, 4, 3] replaced by the four
    tetrahedra that join its centroid to its faces (sub-tetrahedron i takes
    the centroid in place of vertex i, so each keeps the orientation of k):
    the first takes k's place, the other three are appended.  From the Kuhn
    cube this gives K = 6 n^3 + 3 elements, an odd count."""
    v = np.asarray(vx, dtype=np.float64)
    c = v[k].mean(axis=0)
    subs = []
    for i in range(4):
        t = v[k].copy()
        t[i] = c
        subs.append(t)
    out = np.concatenate([v, np.stack(subs[1:])])
    out[k] = subs[0]
    return out



def element_constant_params(K, seed=12):
    """Per-element (rho, cp, cs) of element-constant media: rho ~ U[1, 3],
    cp ~ U[2, 4], cs = cp / U[1.6, 2.0], one draw per element, so that the
    material jumps across every face."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(1.0, 3.0, K)
    cp = rng.uniform(2.0, 4.0, K)
    cs = cp / rng.uniform(1.6, 2.0, K)
    return rho, cp, cs


def element_constant_samples(K, Nq, Np, seed=12):
    """Element-constant media repeated at every quadrature point [K, Nq] and
    every node [K, Np]: (rho_q, cp_q, cs_q, rho_n, cp_n, cs_n)."""
    rho, cp, cs = element_constant_params(K, seed)
    at_q = [np.repeat(a[:, None], Nq, axis=1) for a in (rho, cp, cs)]
    at_n = [np.repeat(a[:, None], Np, axis=1) for a in (rho, cp, cs)]
    return (*at_q, *at_n)
