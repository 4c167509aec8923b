"""The host-side structure builder (csrc/structure.cpp) under AddressSanitizer
and UndefinedBehaviorSanitizer: tests/host/structure_check.cpp builds the
cluster and block trees for a grid of descriptors (1D and 2D, ragged sizes,
leaf 16..64, eta 0.5..2, N_block 1..64), checks their invariants, subdivides
admissible blocks as the rank-cap path does, and feeds invalid descriptors.
Host code only (g++, no device code), so it runs on the CPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_structure_builder_under_sanitizers(tmp_path):
    exe = str(tmp_path / "structure_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1812_08324_amd", "csrc"),
           os.path.join(ROOT, "tests", "host", "structure_check.cpp"),
           os.path.join(ROOT, "paper_1812_08324_amd", "csrc", "structure.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "failures 0" in r.stdout
