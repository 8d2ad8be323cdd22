"""The C cascade oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host code
only) and run on small seeded inputs and edge cases: flat stretches and a flat query, a band wider
than the query, band 0, m = 1 and 2, a series as long as the query.  No sanitizer report, and the
single-query, many-query and full-DTW entry points agree."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_driver")
        build = subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined",
                                "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-o", exe,
                                os.path.join(HERE, "sanitize", "oracle_driver.c"),
                                os.path.join(ROOT, "oracle", "cascade.c"), "-lm"],
                               capture_output=True, text=True)
        if build.returncode != 0 and "sanitize" in build.stderr:
            pytest.skip("the sanitizer runtimes are not installed: " + build.stderr[-300:])
        assert build.returncode == 0, build.stderr[-2000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
                   OMP_NUM_THREADS="2")
        run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        print(run.stdout)
        assert "runtime error" not in run.stderr, run.stderr[-3000:]
        assert "ERROR: AddressSanitizer" not in run.stderr, run.stderr[-3000:]
        assert "ERROR: LeakSanitizer" not in run.stderr, run.stderr[-3000:]
        assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-2000:]
