"""Build libcubics.so (HIP, gfx950) in-tree with hipcc.

Each source is compiled to an object in parallel, then linked; objects go to
paper_1909_09213_amd/_build/ (not committed)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
SO = os.path.join(HERE, "libcubics.so")
# (source, extra flags, object name): the search kernels are compiled once per
# domain width so that their variants build in parallel
UNITS = [("cubics_search.hip", ["-DCUBICS_ONLY_WM=%d" % w], "cubics_search_w%d.o" % w) for w in (1, 2, 4, 8)]
UNITS += [(s, [], os.path.splitext(s)[0] + ".o")
          for s in ("cubics_mlp.hip", "cubics_host.cpp", "cubics_policy.cpp")]
FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(SO):
        return SO
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)

    def compile_one(unit):
        src, extra, name = unit
        obj = os.path.join(OBJ, name)
        cmd = [hipcc] + FLAGS + extra + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.check_call(cmd, cwd=CSRC)
        return obj

    jobs = min(len(UNITS), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, UNITS))
    tmp = SO + ".tmp%d" % os.getpid()
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd, cwd=CSRC)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
