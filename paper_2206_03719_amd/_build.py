"""Build libhs.so (gfx950 HIP kernels + the C-ABI host runtime) in-tree.

Every source is compiled with hipcc for gfx950 only; the host planner is
built with -ffp-contract=off so its FP64 arithmetic (Cholesky factors,
discount factors, bumped parameters) is plain IEEE.  Usage:
``python -m paper_2206_03719_amd._build`` (``__graft_entry__.build()`` calls it).
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libhs.so")
ARCH = "gfx950"

HIP_FLAGS = ["-std=c++17", "-O3", "--offload-arch=" + ARCH, "-fPIC", "-ffp-contract=on",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]
HOST_FLAGS = ["-std=c++17", "-O2", "-fPIC", "-ffp-contract=off", "-Wall"]

# the path-kernel variants are split over several sources so that they
# compile in parallel
SOURCES = [
    ("hs_paths_f32e.hip", HIP_FLAGS),
    ("hs_paths_f64e.hip", HIP_FLAGS),
    ("hs_paths_f32q.hip", HIP_FLAGS),
    ("hs_paths_f64q.hip", HIP_FLAGS),
    ("hs_paths_f32h.hip", HIP_FLAGS),
    ("hs_lsmc.hip", HIP_FLAGS),
    ("hs_paths_base.hip", HIP_FLAGS),
    ("hs_kernels.hip", HIP_FLAGS),
    ("hs_noalloc.hip", HIP_FLAGS),
    ("hs_plan.cpp", HOST_FLAGS),
    ("hs_api.cpp", HOST_FLAGS),
    ("hs_server.cpp", HOST_FLAGS),
]


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _compile(src, flags, verbose):
    obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), r.stderr[-6000:]))
    return obj


def build(verbose=False):
    os.makedirs(OUT_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 8)) as ex:
        futs = [ex.submit(_compile, s, f, verbose) for s, f in SOURCES]
        objs = [f.result() for f in futs]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-4000:])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
