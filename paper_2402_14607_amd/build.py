"""Build the HIP library in-tree: paper_2402_14607_amd/libqrngext.so (gfx950).

``python -m paper_2402_14607_amd.build`` or ``build()`` from Python.
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libqrngext.so")
SOURCES = ["ext_kernels.hip", "ext_api.cpp", "ext_batch.cpp", "ext_server.cpp", "serve_sim.cpp",
           "gf2_modulus.cpp", "ext_params.cpp", "ext_growing.cpp",
           "ext_bitslice.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # no packed-FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    """Compile every source into libqrngext.so (always recompiles)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + srcs
    t0 = time.time()
    res = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    # hipcc's host pass warns about the device-only target feature; drop that line
    noise = "is not a recognized feature for this target"
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines() if noise not in ln]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed (%d):\n%s" % (res.returncode, "\n".join(msgs)))
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built %s in %.1fs" % (LIB, time.time() - t0), file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
