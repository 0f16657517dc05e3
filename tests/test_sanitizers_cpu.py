"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code,
run on the CPU (no GPU):

* the FP64 oracle, driven through every entry point with non-finite inputs,
  border and huge motion, regions of interest, every weight mode, both
  interpolations and the automatic forgetting factor (tests/c/oracle_driver.c);
* the state layout arithmetic of the library's internal header
  (tests/c/layout_check.cpp);
* the host side of the C ABI (libwrls built with the sanitizers on its host
  code only; its device code is built as usual): parameter validation, size
  queries, NULL handles and arguments, the limit of the allocation-free
  batched step (tests/c/abi_validate.c).

Leak detection is on; a report from either sanitizer fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2106_08034_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _run(exe, marker):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert marker in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.run(["gcc", "-std=c99", "-O1", "-ffp-contract=off", "-fopenmp", "-Wall"] + SAN +
                   [os.path.join(ROOT, "oracle", "wrls_oracle.c"),
                    os.path.join(ROOT, "tests", "c", "oracle_driver.c"), "-lm", "-o", exe],
                   check=True, capture_output=True)
    _run(exe, "oracle driver: ok")


def test_layout_arithmetic_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "layout_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
                    "-I", CSRC] + SAN + [os.path.join(ROOT, "tests", "c", "layout_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    _run(exe, "layout check: ok")


def _clang_rt_dir():
    """clang, and the directory of its shared AddressSanitizer runtime."""
    clang = os.path.join(ROCM, "llvm", "bin", "clang")
    for name in ("libclang_rt.asan.so", "libclang_rt.asan-x86_64.so"):
        r = subprocess.run([clang, "-print-file-name=" + name], capture_output=True, text=True)
        path = r.stdout.strip()
        if os.path.isabs(path) and os.path.exists(path):
            return clang, os.path.dirname(path)
    pytest.skip("clang's shared AddressSanitizer runtime not found")


@pytest.mark.skipif(not shutil.which(os.path.join(ROCM, "bin", "hipcc")), reason="hipcc not found")
def test_c_abi_host_paths_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "libwrls_san.so")
    host_san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-omit-frame-pointer"):
        host_san += ["-Xarch_host", f]   # host code only: the device code is built as usual
    subprocess.run([os.path.join(ROCM, "bin", "hipcc"), "-O1", "-std=c++17", "-fPIC", "-shared",
                    "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
                   + host_san + ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", lib,
                                 os.path.join(CSRC, "wrls_kernels.hip"), os.path.join(CSRC, "wrls_api.hip")],
                   check=True, capture_output=True)
    clang, rtdir = _clang_rt_dir()
    exe = str(tmp_path / "abi_validate")
    subprocess.run([clang, "-std=c99", "-Wall", "-shared-libasan"] + SAN +
                   ["-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c", "abi_validate.c"),
                    "-L", str(tmp_path), "-lwrls_san", "-Wl,-rpath," + str(tmp_path), "-Wl,-rpath," + rtdir,
                    "-o", exe], check=True, capture_output=True)
    _run(exe, "abi validate: ok")
