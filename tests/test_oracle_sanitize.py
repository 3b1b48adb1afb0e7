"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU): a
small driver (tests/sanitize/oracle_main.c) that runs its step, observables,
inversion and the reduced state's step and recovery on a ragged grid, built
with -fsanitize=address,undefined and no recovery from a report."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_runs_clean_under_sanitizers():
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_san")
        cmd = [gcc, "-O1", "-g", "-std=gnu11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer", os.path.join(ROOT, "tests", "sanitize", "oracle_main.c"), "-lm",
               "-o", exe]
        b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
        if b.returncode != 0 and ("asan" in b.stderr or "ubsan" in b.stderr):
            pytest.skip("sanitizer runtimes not available: " + b.stderr[-300:])
        assert b.returncode == 0, b.stderr[-2000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        env.pop("LD_PRELOAD", None)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert r.returncode == 0 and r.stdout.startswith("ok"), (r.returncode, r.stdout, r.stderr[-3000:])
