"""Build libhgrape.so (HIP for gfx950) in-tree.

    python paper_2304_06200_amd/build.py            # all sources, parallel
    python paper_2304_06200_amd/build.py --jobs 4

(run it by path: importing the package loads the library being rebuilt)

Every .hip/.cpp translation unit under csrc/ is compiled with hipcc for
--offload-arch=gfx950 (packed FP32 instructions disabled), except plan.cpp,
the FP64 planner, which is compiled with g++ and -ffp-contract=off so that
every operation is rounded as written.  Objects go to csrc/_build/.
"""
import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(CSRC, "_build")
LIB = os.path.join(HERE, "libhgrape.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
ARCH = "gfx950"

HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-variable", "-Wno-unused-but-set-variable"]
PLAN_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math"]


def _sources():
    out = []
    for f in sorted(os.listdir(CSRC)):
        if f.endswith(".hip") or f.endswith(".cpp"):
            out.append(os.path.join(CSRC, f))
    return out


def _cost_rank(src):
    # the widest sweep instantiations take minutes each: start them first so
    # the parallel build does not end on one of them
    f = os.path.basename(src)
    for rank, prefix in enumerate(("sweep_w13", "sweep_w9", "sweep_ell13", "sweep_ell9",
                                   "sweep_split", "sweep_w5")):
        if f.startswith(prefix):
            return rank
    return 99


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if os.path.basename(src) == "plan.cpp":
        cmd = ["g++"] + PLAN_FLAGS + ["-c", src, "-o", obj]
    else:
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = [HIPCC] + HIP_FLAGS + lang + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int = 0, verbose: bool = False) -> str:
    """Compile every translation unit and link libhgrape.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = _sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, sorted(srcs, key=_cost_rank)))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + \
        ["-L" + os.path.join(ROCM, "lib"), "-lrocblas", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", flush=True)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=0)
    a = ap.parse_args()
    build(a.jobs, verbose=True)
    sys.exit(0)
