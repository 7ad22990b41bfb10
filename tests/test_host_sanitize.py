"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The tree plan (`csrc/plan.cpp`, the index sets and maps every kernel reads)
and the oracle's C routines are compiled with g++/gcc and
-fsanitize=address,undefined, then driven by small checkers under
tests/sanitize/: any out-of-bounds access, leak, overflow or undefined
operation aborts the checker.  The checkers also verify the plan's
structure (Section 2.1: halving rectangles, gamma on the cut, Gamma on the
perimeter, maps into the sons' frames).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host compiler")
def test_plan_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_check")
    _run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "paper_1708_02207_amd", "csrc"),
          os.path.join(ROOT, "tests", "sanitize", "plan_check.cpp"),
          os.path.join(ROOT, "paper_1708_02207_amd", "csrc", "plan.cpp"), "-o", exe], ROOT)
    out = _run([exe], ROOT)
    assert "0 failures" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host compiler")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-std=gnu11", *SAN, os.path.join(ROOT, "tests", "sanitize", "oracle_check.c"),
          os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe], ROOT)
    out = _run([exe], ROOT)
    assert "0 failures" in out
