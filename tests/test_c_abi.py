"""The C ABI from plain C: tests/c/abi_demo.c is compiled as strict C99
against include/wrls.h and linked with libwrls.so.  The header also
compiles as C++.  On the CPU the host-side calls run; on the GPU the
program steps frames through the C ABI alone, and its output is checked
against the FP64 oracle on the inputs it wrote."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "include")
PKG = os.path.join(ROOT, "paper_2106_08034_amd")
SRC = os.path.join(ROOT, "tests", "c", "abi_demo.c")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _build(tmp_path):
    from paper_2106_08034_amd import wrls
    wrls.lib()  # raises if libwrls.so is not built
    exe = str(tmp_path / "abi_demo")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", INC, SRC,
           "-o", exe, "-L", PKG, "-lwrls", "-Wl,-rpath," + PKG,
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    subprocess.run(cmd, check=True)
    return exe


def test_header_compiles_as_c99_and_cpp(tmp_path):
    src = tmp_path / "h.c"
    src.write_text('#include "wrls.h"\nint main(void) { return (int)sizeof(wrls_params); }\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-fsyntax-only",
                    "-I", INC, str(src)], check=True)
    subprocess.run(["g++", "-x", "c++", "-std=c++11", "-Wall", "-Wextra", "-Werror", "-fsyntax-only",
                    "-I", INC, str(src)], check=True)


def test_host_calls_from_c(tmp_path):
    exe = _build(tmp_path)
    r = subprocess.run([exe, "host"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    kv = dict(line.split(" ", 1) for line in r.stdout.strip().splitlines())
    assert kv["state_floats"] == "60"
    assert kv["state_bytes"] == str(240 * 1920 * 1080)
    assert kv["validate_ok"] == "0" and kv["validate_d11"] == "-4"
    assert "d = 11" in kv["error_d11"]
    assert kv["step_null"] == "-1"


@pytest.mark.gpu
def test_step_from_c_matches_oracle(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import oracle
    from parity import G1_TOL, g1, predictor, term_scale
    exe = _build(tmp_path)
    W, H, T = 150, 37, 5
    out_path = str(tmp_path / "out.f32")
    r = subprocess.run([exe, "gpu", str(W), str(H), str(T), out_path], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "frames %d" % T in r.stdout
    inputs = np.fromfile(out_path + ".inputs", dtype=np.float32).reshape(T, 13, H, W)
    got = np.fromfile(out_path, dtype=np.float32).reshape(3, H, W)
    o = oracle.Oracle(W, H, 8)
    for t in range(T):
        f = inputs[t]
        ref = o.step(f[0:3], f[3:10], f[10], f[11:13])
    e = g1(got, ref, term_scale(o.get_beta(), predictor(inputs[T - 1][3:10])))
    assert e <= G1_TOL, e
