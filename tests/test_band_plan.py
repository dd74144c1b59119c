"""Host logic of the banded preconditioner's plan (CPU): the elimination order from both
ends of the band and the super-row grouping of the substitutions, checked by
band_plan_check.cpp over several thousand (M, q, b) plans against brute force (coupling
sets, fill-free elimination) and a numerical substitution with random scalar blocks."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1403_5044_amd", "csrc")


def test_band_plan_invariants(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "band_plan_check")
    subprocess.run([cxx, "-O2", "-std=c++17", "-Wall", "-Werror", "-I", CSRC,
                    os.path.join(HERE, "band_plan_check.cpp"), "-o", exe],
                   check=True, capture_output=True, text=True, timeout=120)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok:"), r.stdout
