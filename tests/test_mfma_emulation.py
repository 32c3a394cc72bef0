"""CPU check of the stage kernel sources: the unchanged kernels (the BF16x3
and FP32 matrix-core kernels of orders 1-4 and 5-7, the FP64 matrix-core
kernels of orders 1-4 and 5-7) run on host threads
(tests/emu) built with AddressSanitizer, so any out-of-bounds index fails the
test, and their results are compared with the FP64 oracle (BF16x3: 1e-4,
FP32: 2e-5, FP64: 1e-12 per-field relative L2)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from gpu_common import rel_l2_per_field
from oracle.dg import ElasticDG
from oracle.mesh import build_mesh
from oracle.refelem import ref_element

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2008_09441_amd", "csrc")
CXX = shutil.which("clang++") or "/opt/rocm/llvm/bin/clang++"


@pytest.fixture(scope="module")
def emu_exe(tmp_path_factory):
    if not os.path.exists(CXX):
        pytest.skip("clang++ not available")
    exe = str(tmp_path_factory.mktemp("emu") / "emu_stage")
    cmd = [CXX, "-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
           "-I", os.path.join(HERE, "emu", "include"), "-I", CSRC,
           os.path.join(HERE, "emu", "emu_stage.cpp"), os.path.join(CSRC, "dg_host.cpp"),
           os.path.join(CSRC, "dg_mfma_host.cpp"), "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("emulator does not build here: " + r.stderr[-500:])
    return exe


def _run(exe, tmp_path, n, N, flux="upwind", grid=1, lsrk=0, split=False, raw=False):
    vx = synth.kuhn_cube_vertices(n)
    mesh = None
    if split:   # one element split at its centroid: K = 6 n^3 + 3 (odd)
        vx = synth.split_tet_vertices(vx)
        mesh = build_mesh(n, ref_element(N), vx)
    op = ElasticDG(n, N, synth.fourier_media, flux=flux, mesh=mesh)
    q = synth.random_state(op.K, op.Np, seed=40 + N).astype(np.float32)
    parts = [np.array([N, 1 if flux == "upwind" else 0, grid, lsrk], np.int32).tobytes(),
             np.array([op.K], np.int64).tobytes(),
             vx.astype(np.float64).tobytes(),
             np.ones(3).tobytes()]
    for a in synth.fourier_media(op.mesh.xq) + synth.fourier_media(op.mesh.x):
        parts.append(np.ascontiguousarray(a, np.float64).tobytes())
    parts.append(q.tobytes())
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    fin.write_bytes(b"".join(parts))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([exe, str(fin), str(fout)], capture_output=True, text=True, env=env,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    got = np.fromfile(fout, np.float64).reshape(9, op.K, op.Np)
    ref = op.rhs_raw(q.astype(np.float64)) if raw else op.rhs(q.astype(np.float64))
    return rel_l2_per_field(got, ref)


@pytest.mark.parametrize("n,N,flux", [(2, 1, "central"), (3, 2, "upwind"), (3, 3, "central"),
                                      (3, 4, "upwind"), (2, 4, "central"), (1, 5, "upwind"),
                                      (1, 6, "central"), (2, 7, "upwind")])
def test_stage_kernel_source_in_bounds_and_accurate(emu_exe, tmp_path, n, N, flux):
    err = _run(emu_exe, tmp_path, n, N, flux)
    print("per-field rel L2:", np.array2string(err, precision=2))
    assert err.max() <= 1e-4


@pytest.mark.parametrize("n,N,flux,lsrk", [(1, 5, "upwind", 0), (1, 6, "central", 1),
                                           (1, 7, "upwind", 0), (2, 4, "upwind", 0)])
def test_stage_kernel_odd_element_count(emu_exe, tmp_path, n, N, flux, lsrk):
    """A mesh with an odd element count (one Kuhn element split at its
    centroid): elements of a non-Kuhn shape, and a ragged last 16-element
    tile at order 4."""
    err = _run(emu_exe, tmp_path, n, N, flux, lsrk=lsrk, split=True)
    print("per-field rel L2:", np.array2string(err, precision=2))
    assert err.max() <= 1e-4


@pytest.mark.parametrize("n,N,flux", [(2, 1, "upwind"), (3, 2, "central"), (3, 3, "upwind"),
                                      (3, 4, "upwind"), (2, 4, "central")])
def test_fp32_matrix_kernel_source_in_bounds_and_accurate(emu_exe, tmp_path, n, N, flux):
    err = _run(emu_exe, tmp_path, n, N, flux, grid=2)
    print("per-field rel L2:", np.array2string(err, precision=2))
    assert err.max() <= 2e-5


@pytest.mark.parametrize("n,N,flux,lsrk", [(1, 5, "upwind", 0), (1, 6, "central", 0),
                                           (1, 7, "upwind", 1), (1, 6, "upwind", 0)])
def test_fp32_matrix_kernel_orders_5_to_7(emu_exe, tmp_path, n, N, flux, lsrk):
    """The FP32 matrix-core kernel of orders 5-7 (one element per workgroup,
    v_mfma_f32_16x16x4_f32), the last case on the odd-count mesh."""
    err = _run(emu_exe, tmp_path, n, N, flux, grid=2, lsrk=lsrk, split=(flux == "upwind" and N == 6))
    print("per-field rel L2:", np.array2string(err, precision=2))
    assert err.max() <= 2e-5


def test_fp32_matrix_kernel_odd_element_count(emu_exe, tmp_path):
    err = _run(emu_exe, tmp_path, 2, 4, "upwind", grid=2, split=True)
    assert err.max() <= 2e-5


def test_fp32_matrix_kernel_lsrk_mode(emu_exe, tmp_path):
    err = _run(emu_exe, tmp_path, 2, 4, "upwind", grid=2, lsrk=1)
    assert err.max() <= 2e-5


@pytest.mark.parametrize("n,N", [(2, 4), (1, 7)])
def test_stage_kernel_lsrk_mode(emu_exe, tmp_path, n, N):
    # with a = 0, b = dt = 1 the LSRK increment q_out - q_in equals the rhs
    err = _run(emu_exe, tmp_path, n, N, "upwind", lsrk=1)
    assert err.max() <= 1e-4


@pytest.mark.parametrize("n,N,flux", [(3, 1, "upwind"), (3, 2, "central"), (3, 3, "upwind"),
                                      (3, 4, "upwind"), (2, 4, "central")])
def test_fp64_matrix_kernel_source_in_bounds_and_accurate(emu_exe, tmp_path, n, N, flux):
    """The FP64 matrix-core tiled kernel (orders 1-4, v_mfma_f64_16x16x4f64):
    the tiling of the FP32 kernel in double precision, at the FP64 bound."""
    err = _run(emu_exe, tmp_path, n, N, flux, grid=3)
    print("per-field rel L2:", np.array2string(err, precision=2))
    assert err.max() <= 1e-12


@pytest.mark.parametrize("lsrk,split", [(1, False), (0, True), (1, True)])
def test_fp64_matrix_kernel_lsrk_and_odd_count(emu_exe, tmp_path, lsrk, split):
    err = _run(emu_exe, tmp_path, 2, 4, "upwind", grid=3, lsrk=lsrk, split=split)
    print("per-field rel L2:", np.array2string(err, precision=2))
    assert err.max() <= 1e-12


@pytest.mark.parametrize("n,N,flux,lsrk,split", [(1, 5, "upwind", 0, False),
                                                 (1, 6, "central", 1, False),
                                                 (1, 7, "upwind", 0, False),
                                                 (1, 6, "upwind", 0, True)])
def test_fp64_matrix_kernel_orders_5_to_7(emu_exe, tmp_path, n, N, flux, lsrk, split):
    """The FP64 matrix-core kernel of orders 5-7 (one element per workgroup,
    v_mfma_f64_16x16x4f64 with its measured accumulator row order), at the
    FP64 bound; the last case on the odd-count mesh."""
    err = _run(emu_exe, tmp_path, n, N, flux, grid=3, lsrk=lsrk, split=split)
    print("per-field rel L2:", np.array2string(err, precision=2))
    assert err.max() <= 1e-12


@pytest.mark.parametrize("n,N,flux,split", [(2, 1, "upwind", False), (3, 2, "central", False),
                                            (3, 3, "upwind", False), (2, 4, "upwind", True)])
def test_fp32_matrix_kernel_stores_the_raw_rhs(emu_exe, tmp_path, n, N, flux, split):
    """stage_bx_r<N>, the FP32 kernel of the adjoint's replay: besides its
    stage it stores R q (volume terms and LIFT before the mass inverse),
    checked against the oracle's raw right-hand side."""
    err = _run(emu_exe, tmp_path, n, N, flux, grid=4, split=split, raw=True)
    print("per-field rel L2:", np.array2string(err, precision=2))
    assert err.max() <= 2e-5
