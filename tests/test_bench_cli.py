"""The benchmark's command-line contract, on the host: one GPU only (a
request for more exits with status 2 and says why), and every workload is
offered."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


def test_help_lists_the_workloads():
    r = _bench("--help")
    assert r.returncode == 0
    for w in ("tg", "cavity", "precision", "batch", "warmstart", "small"):
        assert w in r.stdout
