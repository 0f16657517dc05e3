"""The state layout arithmetic of libwrls on the host (no GPU): the
library's own internal header (wrls_internal.h) is compiled into
tests/c/layout_check.cpp, which checks that entry_offsets maps every
(pixel, entry) of every predictor length, with and without the paper-mode
history, one-to-one onto the words of one state copy, keeps each group of
four entries in one aligned 16-byte vector and each 64-pixel chunk in its
own block, and that the export order (P, beta, history) maps onto the state
order (beta, P, history)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2106_08034_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "c", "layout_check.cpp")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_state_layout_is_a_bijection_with_aligned_vectors(tmp_path):
    exe = str(tmp_path / "layout_check")
    subprocess.run([os.path.join(ROCM, "bin", "hipcc"), "-std=c++17", "-O1", "-I", CSRC, SRC, "-o", exe],
                   check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "layout check: ok" in r.stdout
