"""CPU check of the tiled FP32 adjoint kernels (dgt::adj_tile<N> and
dgt::adj_nodes, orders 1-4): one reverse stage runs on host threads
(tests/emu/emu_adjoint.cpp, with the replay stage kernel that stores R y
and the face-node jumps) built with AddressSanitizer, so any
out-of-bounds index fails the test, and its results are compared with the
oracle's discrete adjoint of the same stage (oracle/adjoint.py):

    l = a lres + b ly,   r = R y + f(ts) s_raw,
    grad  = dt d/dm <l, W(m) r>,     mu = W(m)^T l,
    ly'   = ly + dt R^T mu,          gradz = dt d/dz <mu, R(z) y>,

with R^T from the oracle's dense raw operator.  FP32 products against FP64:
per-field relative L2 within 2e-5 (l, ly', grad) and 1e-4 (gradz, whose
face terms cancel)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from oracle import adjoint as oadj
from oracle.dg import ElasticDG
from oracle.mesh import build_mesh
from oracle.refelem import ref_element
from oracle.source import ricker

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2008_09441_amd", "csrc")
CXX = shutil.which("clang++") or "/opt/rocm/llvm/bin/clang++"


@pytest.fixture(scope="module")
def emu_adj(tmp_path_factory):
    if not os.path.exists(CXX):
        pytest.skip("clang++ not available")
    exe = str(tmp_path_factory.mktemp("emu") / "emu_adjoint")
    cmd = [CXX, "-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
           "-I", os.path.join(HERE, "emu", "include"), "-I", CSRC,
           os.path.join(HERE, "emu", "emu_adjoint.cpp"), os.path.join(CSRC, "dg_host.cpp"),
           os.path.join(CSRC, "dg_mfma_host.cpp"), "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("emulator does not build here: " + r.stderr[-500:])
    return exe


def rel_l2_per_field(a, b):
    """Relative L2 error of each leading-index slice (field) of a against b."""
    a = np.asarray(a, np.float64).reshape(len(b), -1)
    b = np.asarray(b, np.float64).reshape(len(b), -1)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


def _case(exe, tmp_path, n, N, flux, split=False, nsrc=0, rin=False):
    vx = synth.kuhn_cube_vertices(n)
    mesh = None
    if split:   # one element split at its centroid: an odd element count
        vx = synth.split_tet_vertices(vx)
        mesh = build_mesh(n, ref_element(N), vx)
    op = ElasticDG(n, N, synth.fourier_media, flux=flux, mesh=mesh)
    K, Np = op.K, op.Np
    rng = np.random.default_rng(100 + 10 * N + n)
    y = synth.random_state(K, Np, seed=60 + N).astype(np.float32)
    lres = (rng.standard_normal((9, K, Np)) * 0.3).astype(np.float32)
    ly = rng.standard_normal((9, K, Np)).astype(np.float32)
    a, b, dt, ts = -0.4801594636, 0.3465, 0.0125, 0.21
    srcs = []
    for i in range(nsrc):
        srcs.append(dict(k=int(rng.integers(K)), w=rng.standard_normal((3, Np)).astype(np.float32),
                         f0=float(rng.uniform(2, 6)), t0=0.15, amp=float(rng.uniform(0.5, 2))))
    parts = [np.array([N, 1 if flux == "upwind" else 0, int(rin)], np.int32).tobytes(),
             np.array([K], np.int64).tobytes(), vx.astype(np.float64).tobytes(),
             np.ones(3).tobytes()]
    for arr in synth.fourier_media(op.mesh.xq) + synth.fourier_media(op.mesh.x):
        parts.append(np.ascontiguousarray(arr, np.float64).tobytes())
    parts += [y.tobytes(), lres.tobytes(), ly.tobytes()]
    if rin == 1:   # R y as the replay's FP32 stage would store it
        parts.append(op.rhs_raw(y.astype(np.float64)).astype(np.float32).tobytes())
    parts += [np.array([a, b, dt, ts]).tobytes(), np.array([nsrc], np.int32).tobytes()]
    for s in srcs:
        parts += [np.array([s["k"]], np.int64).tobytes(), s["w"].tobytes(),
                  np.array([s["f0"], s["t0"], s["amp"]]).tobytes()]
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    fin.write_bytes(b"".join(parts))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([exe, str(fin), str(fout)], capture_output=True, text=True, env=env,
                       timeout=900)
    assert r.returncode == 0, r.stderr[-2000:]
    out = np.fromfile(fout, np.float64)
    n9, Nq = 9 * K * Np, op.ref.Nq
    got_l = out[:n9].reshape(9, K, Np)
    got_ly = out[n9:2 * n9].reshape(9, K, Np)
    got_g = out[2 * n9:2 * n9 + 3 * K * Nq].reshape(3, K, Nq)
    got_z = out[2 * n9 + 3 * K * Nq:].reshape(2, K, Np)

    # the oracle's reverse stage (FP64 from the same FP32 inputs)
    m = np.stack([op.mat.irho_q, op.mat.lam_q, op.mat.mu_q])
    l = np.float32(a) * lres.astype(np.float64) + np.float32(b) * ly.astype(np.float64)
    yy = y.astype(np.float64)
    r_ = op.rhs_raw(yy)
    for s in srcs:
        r_[0:3, s["k"]] += ricker(ts, s["f0"], s["t0"], s["amp"]) * s["w"].astype(np.float64)
    ref_g = dt * oadj._dm(op, l, r_)
    mu = oadj._wT(op, l, m)
    R = oadj.raw_matrix(op)
    ref_ly = ly.astype(np.float64) + dt * (R.T @ mu.ravel()).reshape(9, K, Np)
    errs = {"l": rel_l2_per_field(got_l, l).max(), "ly": rel_l2_per_field(got_ly, ref_ly).max(),
            "grad": rel_l2_per_field(got_g, ref_g).max()}
    if flux == "upwind":
        ref_z = dt * oadj._dz(op, mu, yy)
        errs["gradz"] = rel_l2_per_field(got_z, ref_z).max()
    else:
        assert not got_z.any()
    return errs


def _check(errs):
    print({k: f"{v:.2e}" for k, v in errs.items()})
    assert errs["l"] <= 2e-5 and errs["ly"] <= 2e-5 and errs["grad"] <= 2e-5
    assert errs.get("gradz", 0.0) <= 1e-4


@pytest.mark.parametrize("rin", [0, 1, 2])
@pytest.mark.parametrize("n,N,flux", [(1, 1, "upwind"), (2, 1, "central"), (2, 2, "upwind"),
                                      (1, 3, "central"), (1, 4, "upwind")])
def test_adjoint_tile_kernels_in_bounds_and_match_the_oracle(emu_adj, tmp_path, n, N, flux, rin):
    """Three variants: R y computed in the kernel (rin 0); R y given, the
    face-node jumps computed in the kernel (1); and as in the library, R y
    and the jumps stored by the replay's stage kernel stage_bx_r<N> run on
    the same stage input first (2)."""
    _check(_case(emu_adj, tmp_path, n, N, flux, rin=rin))


@pytest.mark.parametrize("rin", [0, 1, 2])
@pytest.mark.parametrize("n,N,flux,nsrc", [(2, 3, "upwind", 2), (1, 4, "central", 1)])
def test_adjoint_tile_kernels_odd_count_and_sources(emu_adj, tmp_path, n, N, flux, nsrc, rin):
    """An odd element count (one element split at its centroid, non-Kuhn
    shapes, a ragged last tile) with point sources inside the tiles."""
    _check(_case(emu_adj, tmp_path, n, N, flux, split=True, nsrc=nsrc, rin=rin))
