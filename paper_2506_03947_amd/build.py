"""Builds libalphacirc.so (HIP, gfx950) in-tree.

    python -m paper_2506_03947_amd.build [--jobs N] [--debug]

Every .hip file under csrc/ is compiled to an object with hipcc for gfx950 and
the objects are linked into paper_2506_03947_amd/libalphacirc.so.  Packed FP32
instructions are disabled (-packed-fp32-ops) for all device code.
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libalphacirc.so")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags(debug: bool) -> list[str]:
    return [
        "--offload-arch=gfx950",
        "-std=c++17",
        "-fPIC",
        "-O1" if debug else "-O3",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", INCLUDE,
        "-I", CSRC,
        "-Wno-unused-result",
    ]


PER_ELL = ("stencil_ell.hip", "stencil_batch_ell.hip")   # compiled once per number of time blocks
ELLS = range(2, 17)


def _newest_dep(src: str) -> float:
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    deps.append(os.path.join(INCLUDE, "alphacirc.h"))
    return max(os.path.getmtime(d) for d in deps)


def compile_one(job, debug: bool, incremental: bool = False) -> str:
    src, ell = job
    tag = os.path.basename(src) + ("" if ell is None else f".l{ell}")
    obj = os.path.join(BUILD, tag + ".o")
    if incremental and os.path.exists(obj) and os.path.getmtime(obj) > _newest_dep(src):
        return obj
    cmd = [hipcc(), "-c", src, "-o", obj] + common_flags(debug)
    if ell is not None:
        cmd.append(f"-DAC_ELL={ell}")
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{res.stdout}\n{res.stderr}")
    return obj


def build(jobs: int | None = None, debug: bool = False, verbose: bool = True, incremental: bool = False) -> str:
    """Compile and link.  incremental=True reuses objects newer than their sources
    and every header (a development shortcut); the default recompiles everything."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    work = []
    for s in srcs:
        if os.path.basename(s) in PER_ELL:
            work += [(s, ell) for ell in ELLS]
        else:
            work.append((s, None))
    # largest units first
    work.sort(key=lambda j: 0 if j[1] is not None else 1)
    jobs = jobs or max(1, min(len(work), os.cpu_count() or 2))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda j: compile_one(j, debug, incremental), work))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-o", tmp] + objs + ["--offload-arch=gfx950", "-fPIC"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--debug", action="store_true")
    ap.add_argument("--incremental", action="store_true")
    a = ap.parse_args()
    try:
        build(a.jobs, a.debug, incremental=a.incremental)
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
