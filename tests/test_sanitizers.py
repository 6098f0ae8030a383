"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The library's host-side parameter logic (csrc/params.cpp: validation of a
parameter set and the tile-edge rules) is fuzzed with valid and invalid
parameter sets, and the C oracle runs small systems covering every order,
meshes down to the order and positions on the faces and far outside the box.
Both are compiled here with the host compilers; any sanitizer report, or a
broken invariant, fails the test."""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc and g++")


def _build_and_run(cmd, exe):
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=ENV, timeout=600)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr, run.stderr
    return run.stdout


def test_parameter_logic_under_sanitizers(tmp_path):
    exe = tmp_path / "params_fuzz"
    csrc = ROOT / "paper_1702_04250_amd" / "csrc"
    out = _build_and_run(["g++", "-std=c++17", *SAN, f"-I{ROOT / 'include'}", f"-I{csrc}",
                          str(ROOT / "tests" / "sanitize" / "params_fuzz.cpp"), str(csrc / "params.cpp"),
                          "-o", str(exe)], exe)
    assert "params fuzz ok" in out


def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_run"
    out = _build_and_run(["gcc", "-std=gnu99", *SAN, str(ROOT / "tests" / "sanitize" / "oracle_run.c"),
                          str(ROOT / "oracle" / "oracle.c"), "-lm", "-o", str(exe)], exe)
    assert "oracle run ok" in out
