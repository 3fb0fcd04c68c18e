"""bench.py's command line on the CPU: a request for more than one GPU is refused
with a message before anything touches a device (this build runs on one GPU; the
slab decomposition across GPUs is a design only), and the help text lists the
switches the profiling commands use."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_help_lists_the_profiling_switches():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--no-variants", "--no-cpu", "--no-ensemble", "--no-surrogate", "--no-shapes",
                 "--copy-calibrate"):
        assert flag in r.stdout, flag
