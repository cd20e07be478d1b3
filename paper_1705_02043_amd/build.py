"""Build libpkifmm.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpkifmm.so")
SOURCES = ["kernels_points.hip", "kernels_p2p.hip", "kernels_gemm.hip", "kernels_oz.hip", "kernels_ops.hip", "plan.hip",
           "tree_host.cpp", "opcache.cpp"]
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         # packed FP32 instructions stay off: the compiler would otherwise form v_pk_* from scalar code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-Wno-unused-result"]


def build(verbose: bool = False, jobs: int = 8) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else ["-fopenmp"]
        cmd = [hipcc] + FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs)
            procs = []
    _wait(procs)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "-shared", "--offload-arch=gfx950", "-o", tmp] + objs + \
          ["-fopenmp", "-L/opt/rocm/lib", "-L/opt/rocm/llvm/lib", "-lrocsolver", "-lrocblas",
           "-Wl,-rpath,/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/llvm/lib"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def _wait(procs):
    bad = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 feature flag; that warning is harmless
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if p.returncode != 0:
            bad.append((src, "\n".join(lines)))
        elif lines and os.environ.get("PKIFMM_BUILD_VERBOSE"):
            print("\n".join(lines))
    if bad:
        for src, text in bad:
            sys.stderr.write(f"--- {src}\n{text}\n")
        raise RuntimeError("HIP build failed: " + ", ".join(s for s, _ in bad))


if __name__ == "__main__":
    print(build(verbose=True))
