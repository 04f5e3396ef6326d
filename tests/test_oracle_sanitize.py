"""Host-sanitizer run of the CPU oracle (test infrastructure): the oracle's C
source built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc, no
GPU code involved) and driven through every entry point on ragged, odd,
tiny and island-rich masks (tests/oracle_sanitize_main.c).  A memory error,
a leak or undefined behaviour makes the run fail with the sanitizer's
report."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "orc_san")
        cmd = [gcc, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all", os.path.join(HERE, "oracle_sanitize_main.c"), "-o", exe, "-lm"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0 and "sanitize" in r.stderr and "unrecognized" in r.stderr:
            pytest.skip("this gcc has no sanitizers")
        assert r.returncode == 0, r.stderr
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert run.returncode == 0, run.stderr[-4000:]
        assert "runtime error" not in run.stderr, run.stderr[-4000:]
        assert "oracle sanitizer run: ok" in run.stdout
