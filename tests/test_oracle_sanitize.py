"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a C
driver (oracle/sanitize_main.c) runs every boundary, coupling and property mode
on ragged grids (down to a single node) through the oracle built with
-fsanitize=address,undefined; any invalid access or undefined arithmetic ends
the run with a report and a nonzero status."""
import os
import shutil
import subprocess

import pytest

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is needed for the sanitizer build")
def test_oracle_runs_clean_under_sanitizers():
    subprocess.run(["make", "-s", "-B", "-C", ORACLE, "sanitize"], check=True, capture_output=True)
    # verify_asan_link_order=0: the run may start with other libraries preloaded
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([os.path.join(ORACLE, "oracle_sanitize")], capture_output=True, text=True, env=env,
                       timeout=300)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitize: all cases ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
