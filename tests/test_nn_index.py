"""The tiled convolution's index arithmetic (32-bit offsets, 24-bit multiplies,
multiply-shift division, float-reciprocal chunk split, tap cursor) against the
plain formulas, on the host: tests/nn_index_check.cpp is compiled against
paper_1806_10247_amd/csrc/nn_index.hpp and run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="needs hipcc")
def test_tiled_convolution_index_helpers_match_the_plain_formulas(tmp_path):
    exe = str(tmp_path / "nn_index_check")
    cc = HIPCC if os.path.exists(HIPCC) else shutil.which("hipcc")
    subprocess.run([cc, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "paper_1806_10247_amd", "csrc"),
                    "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "nn_index_check.cpp"),
                    "-o", exe], check=True, capture_output=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout, r.stdout
