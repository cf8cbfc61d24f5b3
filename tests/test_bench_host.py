"""Host-side logic of the benchmark (no GPU): the checkpoint count that the
roofline's algorithmic flop count uses follows the stack kernel's rule (the
first exposure in epoch order, then every exposure more than 12 days after
the last checkpoint), and the one-GPU guard."""
import subprocess
import sys

import bench


def test_checkpoint_count_follows_the_kernel_rule():
    # epoch order 0, 1, 5, 12, 13, 25.1, 30: checkpoints at 0, 13 (> 12 after 0) and 25.1 (> 12 after 13);
    # 12 is exactly 12 days after 0 and is not one
    exps = [dict(t=t) for t in (5.0, 0.0, 1.0, 12.0, 13.0, 25.1, 30.0)]
    assert bench.checkpoints(exps) == 3
    assert bench.checkpoints([dict(t=3.0)]) == 1
    assert bench.checkpoints([dict(t=float(d)) for d in range(0, 200, 10)]) == 10


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 or "one GPU" in (r.stdout + r.stderr)
    assert "one GPU" in (r.stdout + r.stderr)
