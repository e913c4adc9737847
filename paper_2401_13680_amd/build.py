"""Compile the HIP library libpst.so in-tree for gfx950 with hipcc.

    python -m paper_2401_13680_amd.build        # or build_library() from Python
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpst.so")
PROBE_LIB = os.path.join(HERE, "libpst_probe.so")
# sha256 of the profile kernel's gfx950 instructions in the last build
KERNEL_HASH = os.path.join(HERE, "libpst.k_profile.sha256")
SOURCES = ["pst_stats.hip", "pst_profile.hip", "pst_greedy.hip", "pst_label.hip", "pst_noalloc.hip", "pst_api.cpp",
           "pst_sched.cpp"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # keep FP32 math on the plain (non-packed) VALU instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build_library(verbose: bool = False, probe: bool = False) -> str:
    """Build libpst.so; probe=True builds libpst_probe.so instead, whose
    profile kernel counts how often each selection phase runs (pst_probe_read)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    lib = PROBE_LIB if probe else LIB
    tag = "_probe" if probe else ""
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, "_obj_" + os.path.splitext(src)[0] + tag + ".o")
        cmd = [hipcc, *HIPCC_FLAGS, *(["-DPST_PROBE"] if probe else []), "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc, "-O3", "-std=c++17", "-fPIC", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = lib + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    if not probe:
        with open(KERNEL_HASH, "w") as f:
            f.write(kernel_code_hash(hipcc) + "\n")
    return lib


def kernel_code_hash(hipcc: str) -> str:
    """sha256 over the gfx950 instructions of every k_profile instantiation
    (the device assembly between each kernel's label and its end, comments
    dropped): it changes when the kernel's machine code does, not when a
    comment or another kernel does."""
    import hashlib
    import re
    asm = subprocess.run([hipcc, *HIPCC_FLAGS, "--cuda-device-only", "-S", "-o", "-",
                          os.path.join(CSRC, "pst_profile.hip")], check=True, capture_output=True,
                         text=True).stdout
    h = hashlib.sha256()
    inside = False
    for line in asm.splitlines():
        if re.match(r"^_Z\w*k_profile\w*:", line):
            inside = True
        if inside:
            code = line.split(";")[0].rstrip()
            if code and not code.lstrip().startswith("//"):
                h.update(code.encode() + b"\n")
            if line.startswith(".Lfunc_end"):
                inside = False
    return h.hexdigest()


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv, probe="--probe" in sys.argv))
