"""bench.py's command line on the CPU: more than one GPU is refused with a message, and
a malformed launch shape is refused before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_launch_shape_option_is_checked_before_any_device_work():
    """--launch takes three integers U,X,T and cannot be combined with --tune;
    a malformed value ends the run with a usage error before the GPU is touched."""
    for extra in (["--launch", "8,2"], ["--launch", "8,2,384", "--tune", "100"]):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *extra],
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 2, extra
        assert "--launch" in r.stderr and r.stdout == ""
