"""Compile libbsw.so (HIP kernels for gfx950 + host runtime + C ABI).

Run as ``python -m paper_1907_12931_amd.build``; ``__graft_entry__.build()``
calls ``build()``.  The library is built in-tree next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbsw.so")
SOURCES = ["bsw_kernels.hip", "bsw_seed_kernels.hip", "bsw_sal_kernels.hip", "bsw_host.cpp",
           "bsw_fm_kernels.hip", "bsw_server.cpp", "bsw_seeds.cpp", "bsw_sal.cpp",
           "bsw_fm.cpp", "bsw_peak.hip", "bsw_lanev_s.hip", "bsw_lanev_m.hip",
           "bsw_lanev_l.hip", "bsw_lanev_x.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Werror=return-type",
    "-Werror=uninitialized",
]


def build(verbose: bool = False, jobs: int = 8) -> str:
    from concurrent.futures import ThreadPoolExecutor
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.rsplit(".", 1)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmds.append(["hipcc", *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), *lang,
                     "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)

    def compile_one(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    # the sources compile independently; the largest one sets the time
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        list(ex.map(compile_one, cmds))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
