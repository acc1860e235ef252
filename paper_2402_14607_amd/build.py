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
           "ext_bitslice.hip", "ext_noalloc.hip", "ext_copy.hip"]
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


def _run(cmd):
    res = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    # hipcc's host pass warns about the device-only target feature; drop that line
    noise = "is not a recognized feature for this target"
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines() if noise not in ln]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed (%d): %s\n%s" % (res.returncode, " ".join(cmd),
                                                          "\n".join(msgs)))
    return msgs


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source (in parallel, one object each) and link
    libqrngext.so (always recompiles)."""
    import concurrent.futures as cf
    import tempfile

    t0 = time.time()
    jobs = jobs or max(1, min(len(SOURCES), len(os.sched_getaffinity(0)), 16))
    with tempfile.TemporaryDirectory(prefix="qrngext_build_") as tmpd:
        objs = [os.path.join(tmpd, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [[HIPCC] + [f for f in FLAGS if f != "-shared"] + ["-c", os.path.join(CSRC, s),
                                                                 "-o", o]
                for s, o in zip(SOURCES, objs)]
        with cf.ThreadPoolExecutor(jobs) as pool:
            msgs = [m for ms in pool.map(_run, cmds) for m in ms]
        tmp = LIB + ".tmp%d" % os.getpid()
        msgs += _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built %s in %.1fs" % (LIB, time.time() - t0), file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
