"""bench.py's command line without a GPU: more than one GPU is refused with a
message (one JSON line, exit status 2) before anything touches a device, and
the algorithmic flop count of a sweep matches its closed form."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 2
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("{")][-1]
    assert "one GPU" in json.loads(line)["error"]


def test_sweep_flops_closed_form():
    import bench
    # 2 [4 N (chi^3 D^2 + chi^3 D^4 + 2 chi^2 D^6 d) + N (10 + 8 q) n^2 k + N (2 chi^3 D^4 + 2 chi^2 D^6 d)],
    # N = 16 cuts, n = chi D^2, k = chi + p (capped at n)
    D, chi, d, p, q = 6, 144, 2, 48, 1
    n, k, N = chi * D * D, chi + p, 16
    F = 2 * (4 * N * (chi ** 3 * D ** 2 + chi ** 3 * D ** 4 + 2 * chi ** 2 * D ** 6 * d)
             + N * (10 + 8 * q) * n * n * k + N * (2 * chi ** 3 * D ** 4 + 2 * chi ** 2 * D ** 6 * d))
    assert abs(bench.flops_per_sweep(D, chi, d, p, q) - F) <= 1e-9 * F
