"""Host-side logic of the benchmark (no GPU): the checkpoint count that the
roofline's algorithmic flop count uses follows the stack kernel's rule (the
first exposure in epoch order, then every exposure more than 16 days after
the last checkpoint), and the one-GPU guard."""
import subprocess
import sys

import bench


def test_checkpoint_count_follows_the_kernel_rule():
    # epoch order 0, 1, 5, 16, 17, 33.1, 40: checkpoints at 0, 17 (> 16 after 0) and 33.1 (> 16 after 17);
    # 16 is exactly 16 days after 0 and is not one
    exps = [dict(t=t) for t in (5.0, 0.0, 1.0, 16.0, 17.0, 33.1, 40.0)]
    assert bench.checkpoints(exps) == 3
    assert bench.checkpoints([dict(t=3.0)]) == 1
    assert bench.checkpoints([dict(t=float(d)) for d in range(0, 200, 10)]) == 10


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 or "one GPU" in (r.stdout + r.stderr)
    assert "one GPU" in (r.stdout + r.stderr)
