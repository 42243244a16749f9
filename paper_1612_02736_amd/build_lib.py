"""Compile libhps.so in-tree for gfx950 (host C++ with g++, kernels with hipcc).

Usage: python -m paper_1612_02736_amd.build_lib   (or build() from Python)
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhps.so")
BUILD = os.path.join(HERE, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HOST_SRC = ["hps_api.cpp", "solve_ext.cpp", "plan.cpp", "spectral.cpp"]
DEV_SRC = ["kernels_gj_leaf.hip", "kernels_gjb_leaf.hip", "kernels_gj_merge.hip", "kernels_gj_blocked.hip",
           "kernels_gemm.hip", "kernels_mfma.hip", "kernels_apply.hip",
           "kernels_ext.hip", "noalloc.hip"]
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__",
             "-I" + os.path.join(ROCM, "include")]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))


def build(verbose=False, jobs=None):
    """Compile every source (in parallel, at most `jobs` at a time) and link."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD, exist_ok=True)
    cmds, objs = [], []
    for s in HOST_SRC:
        o = os.path.join(BUILD, s.replace(".cpp", ".o"))
        cmds.append(["g++"] + CXX_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in DEV_SRC:
        src = os.path.join(CSRC, s)
        if not os.path.exists(src):
            continue
        o = os.path.join(BUILD, s.replace(".hip", ".o"))
        cmds.append(["hipcc"] + HIP_FLAGS + ["-c", src, "-o", o])
        objs.append(o)
    jobs = jobs or min(len(cmds), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(_run, cmds))
    tmp = OUT + ".tmp"
    _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs +
         ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64"])
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
