"""Build the HIP library libhipster.so for gfx950 (in-tree).

    python -m paper_2005_01739_amd.build      (or python paper_2005_01739_amd/build.py)

Every source is compiled by hipcc for gfx950 only; packed FP32 instructions are
disabled.  Objects are compiled in parallel, then linked into one shared
library next to this file.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.environ.get("HIPSTER_BUILD_OUT") or os.path.join(HERE, "libhipster.so")
BUILD = os.environ.get("HIPSTER_BUILD_DIR") or os.path.join(HERE, "_build")
EXTRA = os.environ.get("HIPSTER_BUILD_DEFINES", "").split()  # e.g. -DHIPSTER_BK_WAVES_PER_EU=2
SOURCES = ["celllist.hip", "pairs.hip", "pk.hip", "bk.hip", "eii.hip", "api.hip", "analytic.cpp"]
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
         "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-function", "-Wno-unused-result",
         "-I" + CSRC, "-I" + os.path.join(os.path.dirname(HERE), "include"), *EXTRA]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    return "hipcc"


def _compile(src, verbose):
    obj = os.path.join(BUILD, src + ".o")
    cmd = [hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [hipcc(), *[f for f in FLAGS if f != "--offload-arch=gfx950"], "-x", "hip", "--offload-arch=gfx950",
               "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", OUT + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
