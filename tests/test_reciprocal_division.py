"""Host pin of the division the relaxation kernels use where a cell's
diagonal stays in registers over many passes (the finest level's table of
reciprocals of 1..12, the small-level call's per-cell reciprocals): one
correction step from the correctly rounded reciprocal gives the correctly
rounded quotient (Markstein's theorem), checked bit for bit against the
division on random FP64 and FP32 pairs (tests/reciprocal_division_main.c)."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_reciprocal_correction_equals_division():
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "rcpdiv")
        # no contraction: every product and sum rounds on its own, the two
        # fused multiply-adds are the explicit fma calls
        cmd = [gcc, "-std=c11", "-O2", "-ffp-contract=off", os.path.join(HERE, "reciprocal_division_main.c"),
               "-o", exe, "-lm"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        run = subprocess.run([exe, "2000000"], capture_output=True, text=True, timeout=300)
        assert run.returncode == 0, run.stdout + run.stderr
        assert "fp64 mismatches 0 fp32 mismatches 0" in run.stdout, run.stdout
