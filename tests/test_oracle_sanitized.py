"""The CPU oracle (test infrastructure) under AddressSanitizer, LeakSanitizer and
UndefinedBehaviorSanitizer: tests/sanitize_driver.c calls every entry point of the oracle's C
library, built serially with the sanitizers, on a 20-triangle sphere for temporal orders 0 and 1
and both cutoffs, and checks block symmetry, the split quadrature-point count and finite values."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_sanitized")
    flags = ["-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined"]
    build = subprocess.run([gcc] + flags + [os.path.join(ROOT, "tests", "sanitize_driver.c"),
                                            os.path.join(ROOT, "oracle", "tdbem_oracle.c"), "-lm", "-o", exe],
                           capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr:
        pytest.skip("the sanitizer runtimes are not installed: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, run.stderr[-4000:]
    assert "oracle sanitized run ok" in run.stdout
    assert "runtime error" not in run.stderr and "ERROR: AddressSanitizer" not in run.stderr
