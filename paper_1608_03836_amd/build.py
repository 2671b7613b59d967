"""Build the HIP library ``libwadg.so`` in-tree for gfx950.

Usage: ``python paper_1608_03836_amd/build.py`` (or ``__graft_entry__.build()``); run as a
script, since importing the package loads the library this builds.
"""

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libwadg.so")

SOURCES = ["reference.cpp", "stage_kernel.hip", "resident_kernel.hip", "adjoint_kernel.hip",
           "norms_kernel.hip", "convert_kernel.hip", "parareal_kernel.hip", "api.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of every code object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose=False, extra_flags=()):
    """Compile every source into ``libwadg.so`` next to this file.  Always
    recompiles; raises CalledProcessError on failure."""
    srcs = []
    for s in SOURCES:
        path = os.path.join(CSRC, s)
        # .cpp host sources are compiled as HIP too (one toolchain, one link)
        srcs += ["-x", "hip", path] if s.endswith(".cpp") else [path]
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + list(extra_flags) + ["-I", INCLUDE, "-I", CSRC] + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra_flags=sys.argv[1:])
