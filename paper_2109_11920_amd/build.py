"""Build libboac.so (gfx950) in-tree with hipcc.

    python -m paper_2109_11920_amd.build [--jobs N] [--verbose]

Every HIP translation unit is compiled with -ffp-contract=off (the compensated sums rely on it;
wanted FMAs are written as fmaf) and with packed FP32 instructions disabled.
"""
from __future__ import annotations

import argparse
import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libboac.so")
# kernels_persist.hip includes kernels_ray.hip, kernels_back.hip and kernels_misc.hip for their kernel bodies
# (the persistent executor inlines them); the kernels themselves are compiled from their own files
SOURCES = ["kernels_persist.hip", "kernels_ray.hip", "kernels_back.hip", "kernels_misc.hip", "kernels_gp.hip",
           "gp_host.cpp", "runtime.cpp"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libboac)")


def common_flags():
    return ["-std=c++17", "-O3", "-fPIC", "-pthread", f"--offload-arch={ARCH}", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
            "-I", os.path.join(HERE, "..", "include"), "-I", CSRC]


# Translation units whose kernels may use scratch memory: the persistent executor inlines every kernel
# body into one kernel under a 128-register budget, so it spills; every other kernel must not (a spill
# there means an accumulator array left unrolled, which multiplies its memory traffic).
SCRATCH_ALLOWED = {"kernels_persist.hip"}


def scratch_kernels(remarks: str):
    """(kernel, bytes per lane) of the kernels whose resource-usage remarks report scratch memory."""
    out, name = [], None
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name and int(m.group(1)) > 0:
            out.append((name, int(m.group(1))))
    return out


def compile_one(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + common_flags() + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".hip"):
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile {src} failed:\n{r.stdout}\n{r.stderr}")
    if src.endswith(".hip") and src not in SCRATCH_ALLOWED:
        bad = scratch_kernels(r.stderr)
        if bad:
            raise RuntimeError(f"compile {src}: kernels use scratch memory (spilled or unrolled-array registers): "
                               + ", ".join(f"{k} {b} B/lane" for k, b in bad))
    err = "\n".join(l for l in r.stderr.splitlines()
                    if "packed-fp32-ops" not in l and "kernel-resource-usage" not in l and l.strip())
    if err and verbose:
        print(err, file=sys.stderr)
    return obj


def build(jobs: int = 4, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: compile_one(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "-pthread", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 4))
    ap.add_argument("--verbose", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.verbose))


if __name__ == "__main__":
    main()
