"""CPU check of the activation rule's sin and cos (csrc/act_math.h, shared by
the train and evaluation kernels) against FP64 sin and cos: a dense sweep over
several periods (all four quadrants), the quadrant boundaries and their float
neighbours, and log-uniform magnitudes of both signs up to the stated bound."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_sin_cos_against_fp64(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("needs g++")
    exe = str(tmp_path / "sincos")
    r = subprocess.run(["g++", "-std=c++17", "-O2", "-o", exe, os.path.join(ROOT, "tests", "host", "sincos_check.cpp")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    m = dict(re.findall(r"(\w+) ([0-9.e+-]+)", r.stdout))
    assert int(m["n"]) > 8_000_000
    # the polynomials' error (about 1e-7) plus one rounding of the reduced argument
    for k in ("worst_sin", "worst_cos", "worst_sin_small", "worst_cos_small"):
        assert float(m[k]) < 2e-7, r.stdout
