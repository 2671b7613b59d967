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
DEMO = os.path.join(PKG, "abi_demo")

SOURCES = ["reference.cpp", "stage_kernel.hip", "resident_kernel.hip", "split_kernel.hip",
           "adjoint_kernel.hip",
           "norms_kernel.hip", "l2_kernel.hip", "convert_kernel.hip", "parareal_kernel.hip", "launch.hip",
           "api.hip", "api_adjoint.hip", "api_batch.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of every code object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose=False, extra_flags=(), jobs=None):
    """Compile every source into ``libwadg.so`` next to this file: one
    relocatable device-and-host object per source, compiled in parallel, then
    one link.  Always recompiles; raises CalledProcessError on failure."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = [f for f in FLAGS if f != "-shared"] + list(extra_flags) + ["-I", INCLUDE, "-I", CSRC]

    def compile_one(src):
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = [HIPCC] + common + ["-c"] + lang + [path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    n = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=n) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    # the plain-C consumer of the library (csrc/abi_demo.c), linked against
    # it with the library's directory as run path
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", INCLUDE,
           "-I", "/opt/rocm/include", os.path.join(CSRC, "abi_demo.c"), "-o", DEMO,
           "-L", PKG, "-lwadg", "-L", "/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath,$ORIGIN", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra_flags=sys.argv[1:])
