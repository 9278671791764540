"""bench.py's command line without a GPU: it refuses more than one GPU and
unknown workload sections before it touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in r.stderr or "--gpus 1" in r.stderr


def test_unknown_section_is_refused():
    r = _run("--sections", "lowdin,nonesuch")
    assert r.returncode == 2
    assert "nonesuch" in r.stderr and "batched" in r.stderr
