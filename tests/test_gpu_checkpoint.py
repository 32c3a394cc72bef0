"""Checkpoint and resume (run on an MI355X): a run stopped after n1 steps,
its state saved to a file with dg_state_get and its context destroyed, then
restored into a fresh context with dg_state_set and run n2 more steps, ends
bit for bit where an uninterrupted run of n1 + n2 steps ends.  Between steps
the state q is the whole LSRK(5,4) state: the first stage's coefficient
a_1 = 0 discards the low-storage residual of the previous step [CK94]."""
import numpy as np
import pytest

import synth
from gpu_common import make_pair

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(n, N, precision):
    _, s = make_pair(n, N, synth.fourier_media, "upwind", precision, oracle=False)
    return s


@pytest.mark.parametrize("N,precision", [(3, "fp64"), (4, "bf16x3"), (4, "fp32"),
                                         (6, "bf16x3"), (6, "fp64")])
def test_resume_from_checkpoint_is_bit_identical(tmp_path, N, precision):
    n, n1, n2 = 3, 7, 6
    dt = 1e-3
    print(f"case checkpoint N={N} {precision} n={n} steps {n1}+{n2}", flush=True)
    q0 = synth.random_state(6 * n ** 3, (N + 1) * (N + 2) * (N + 3) // 6, seed=70 + N)

    whole = _solver(n, N, precision)
    whole.set_state(q0)
    whole.run(0.0, dt, n1 + n2)
    q_whole = whole.get_state()
    whole.close()

    first = _solver(n, N, precision)
    first.set_state(q0)
    first.run(0.0, dt, n1)
    ck = tmp_path / "state.npy"
    np.save(ck, first.get_state())
    first.close()                      # the interrupted run is gone

    resumed = _solver(n, N, precision)
    resumed.set_state(np.load(ck))
    resumed.run(n1 * dt, dt, n2)
    q_resumed = resumed.get_state()
    resumed.close()

    assert q_whole.dtype == q_resumed.dtype
    assert np.isfinite(q_whole).all()
    assert not np.array_equal(q_whole, q0.astype(q_whole.dtype))   # it moved
    assert np.array_equal(q_whole, q_resumed), "resumed run differs from the uninterrupted one"
