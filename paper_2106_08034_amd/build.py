"""Builds libwrls.so (the HIP kernels and the C ABI) for gfx950 with hipcc,
in-tree, next to this file."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libwrls.so")
# the same sources with every kernel access tested (WRLS_CHECKED)
LIB_CHECKED = os.path.join(HERE, "libwrls_checked.so")
SOURCES = ["wrls_kernels.hip", "wrls_api.hip"]
ARCH = os.environ.get("WRLS_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=" + ARCH,
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False, checked: bool = False) -> str:
    """Compiles every source into libwrls.so (checked: libwrls_checked.so,
    with the kernels' access checks); raises on failure."""
    out = LIB_CHECKED if checked else LIB
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + (["-DWRLS_CHECKED"] if checked else []) + \
        ["-I", INCLUDE, "-I", CSRC, "-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building " + os.path.basename(out))
    os.replace(tmp, out)
    return out


def needs_build() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + [os.path.join(INCLUDE, "wrls.h")]
    return any(os.path.getmtime(p) > t for p in deps)


FIELDS = (("VGPRs", "VGPRs"), ("AGPRs", "AGPRs"), ("TotalSGPRs", "SGPRs"),
          ("VGPRs Spill", "VGPR spill"), ("SGPRs Spill", "SGPR spill"),
          ("ScratchSize [bytes/lane]", "scratch B/lane"), ("Occupancy [waves/SIMD]", "waves/SIMD"),
          ("LDS Size [bytes/block]", "static LDS B"))


def resource_usage(src: str = "") -> str:
    """The compiler's resource use of every kernel (registers, spills,
    scratch, occupancy, static LDS), from a device-only compile of the
    kernels (or of another source file `src` that includes the same headers)
    with the library's flags and -Rpass-analysis=kernel-resource-usage;
    a Markdown table, kernels demangled."""
    import re
    src = src or os.path.join(CSRC, "wrls_kernels.hip")
    out = os.path.join("/tmp", "wrls_resource_usage_%d.o" % os.getpid())
    cmd = [hipcc()] + [f for f in HIPCC_FLAGS if f != "-shared"] + [
        "--offload-device-only", "-c", "-Rpass-analysis=kernel-resource-usage",
        "-I", INCLUDE, "-I", CSRC, "-o", out, src]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise RuntimeError("hipcc failed")
    if os.path.exists(out):
        os.remove(out)
    rows, cur = [], None
    for line in r.stderr.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = {"name": m.group(1)}
            rows.append(cur)
            continue
        m = re.search(r"remark: +([^:]+): (\S+) \[-Rpass", line)
        if m and cur is not None:
            cur[m.group(1).strip()] = m.group(2)
    # _Float16 mangles as DF16_, which c++filt does not know: print it as half
    names = "\n".join(row["name"].replace("DF16_", "Dh") for row in rows)
    dem = subprocess.run(["c++filt"], input=names, capture_output=True, text=True).stdout.splitlines()
    lines = ["| kernel | " + " | ".join(h for _, h in FIELDS) + " |",
             "|---|" + "---|" * len(FIELDS)]
    for row, name in zip(rows, dem):
        name = name.replace("wrls::(anonymous namespace)::", "").split("(")[0]
        lines.append("| `%s` | " % name + " | ".join(row.get(k, "") for k, _ in FIELDS) + " |")
    return "\n".join(lines)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--resource-usage":
        print(resource_usage())
    else:
        print(build(verbose=True))
        print(build(verbose=True, checked=True))
