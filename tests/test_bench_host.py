"""Host-only checks of the benchmark script's contract (no GPU needed)."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    # one GPU per run: N > 1 exits with a message and a non-zero status before touching a device
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == "" or not r.stdout.strip().startswith("{")


def test_lowrank_work_matches_the_per_matrix_counts():
    sys.path.insert(0, ROOT)
    import bench
    p, q, c = 232, 200, 3
    w = bench.lowrank_work([(p, q, c)])
    s, l = 200, 232
    assert w["gram"] == c * 4.0 * l * s * s
    assert w["reproj"] == 2 * w["gram"]
    assert abs(w["tridiag"] - c * 16.0 / 3.0 * s ** 3) < 1e-6 * w["tridiag"]
    # orientation does not matter: the smaller side is s
    assert bench.lowrank_work([(q, p, c)]) == w
