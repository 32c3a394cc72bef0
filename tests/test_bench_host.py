"""Host-side parts of bench.py (no GPU): more than one GPU is refused with a
message, the kernel names the JSON line reports, and the algorithmic bytes
its HBM roofline is computed from."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_kernel_names():
    assert bench.stage_kernel_name("bf16x3", 4) == "stage_bx<4>"
    assert bench.stage_kernel_name("bf16x3", 7) == "stage_be<7>"
    assert bench.stage_kernel_name("fp32", 3) == "stage_bx<3,f32>"
    assert bench.stage_kernel_name("fp32", 6) == "stage_be<6,f32>"
    assert bench.stage_kernel_name("fp64", 4) == "stage_bx_d<4>"
    assert bench.stage_kernel_name("fp64", 5) == "stage_be_d<5>"


def test_algorithmic_bytes_per_element_stage():
    # order 4: q and res read and written (4 x 9 x 35), 1/rho, lam, mu at
    # 125 points, Zp and Zs at 35 nodes, 9 metric terms and 16 face values
    # (all 4 bytes in FP32), plus 20 bytes of neighbour ids and patterns
    assert bench.alg_bytes_per_elem_stage(4, 4) == 4 * (4 * 9 * 35 + 3 * 125 + 2 * 35 + 9 + 16) + 20
    assert bench.alg_bytes_per_elem_stage(4, 4) == 6940
    assert bench.alg_bytes_per_elem_stage(4, 8) == 13860
