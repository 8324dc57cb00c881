"""The serving scheduler under ThreadSanitizer: the host code of the library
is built with -fsanitize=thread and the scheduler tests (simulated executor,
no GPU) run against it in a child process; any data race between the
caller's threads and the scheduler thread fails the test."""
import os
import subprocess
import sys

import pytest

from conftest import ROOT


@pytest.mark.slow
def test_scheduler_is_race_free_under_tsan(tmp_path):
    from paper_1908_11807_amd import build
    lib = build.build_tsan_library()
    env = dict(os.environ)
    env["ABX_LIBRARY"] = lib
    env["LD_PRELOAD"] = build.tsan_runtime()
    # halt at the first report; the interpreter itself is not instrumented
    env["TSAN_OPTIONS"] = "halt_on_error=1 exitcode=66 report_signal_unsafe=0"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        "--timeout", "120", "--timeout-method", "thread",
                        os.path.join(ROOT, "tests", "test_serve_cpu.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "ThreadSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
