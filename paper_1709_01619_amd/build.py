"""Build libcpr.so (HIP, gfx950) in-tree.

    python -m paper_1709_01619_amd.build [--jobs N] [--debug]

Every source under csrc/ is compiled by hipcc for gfx950 with packed FP32
instructions disabled, and linked into paper_1709_01619_amd/libcpr.so.
"""

from __future__ import annotations

import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libcpr.so")
BUILD_DIR = os.path.join(HERE, "_build")

ARCH = "gfx950"
COMMON = [
    "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


# Files whose arithmetic must round exactly as written (the forward stage
# and the limiter, which keep the scheme's x <-> y symmetry bit for bit):
# floating-point contraction is off there and fused multiply-adds are
# spelled out in the source.
NO_CONTRACT = {"cpr_stage.hip", "cpr_aux.hip"}


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def build(jobs: int | None = None, debug: bool = False, verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    opt = ["-O1", "-g"] if debug else ["-O3"]
    cc = hipcc()
    srcs = sources()

    def compile_one(src):
        obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        fp = ["-ffp-contract=off"] if os.path.basename(src) in NO_CONTRACT else []
        cmd = [cc, *COMMON, *opt, *fp, *lang, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        return obj

    n = jobs or min(8, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=n) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--debug", action="store_true")
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.debug, a.verbose))


if __name__ == "__main__":
    sys.exit(main())
