"""Build the HIP library ``libselscan_hip.so`` for gfx950 with hipcc.

Flags that matter for the results:
  * ``-ffp-contract=off``: HIP clang contracts a*b+c into FMA by default, which
    would round the trapezoid sums differently from their definition;
  * no fast-math: IEEE division and square root are required so that the
    cutoff decisions (EHH < cutoff) come out exactly as defined;
  * ``-Xclang -target-feature -Xclang -packed-fp32-ops``: no packed FP32
    instructions are generated.
"""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libselscan_hip.so")
SOURCES = ["ss_walk.hip", "ss_walk_mask.hip", "ss_walk_wide.hip", "ss_walk_batch.hip", "ss_sites.hip",
           "ss_genome.hip", "ss_micro.hip", "ss_capi.hip"]
ARCH = os.environ.get("SS_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags():
    return ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INCLUDE, "-I", CSRC]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into the shared library (always recompiles).

    Each source launches only its own kernels, so the sources are compiled to
    objects in parallel and then linked."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    tag = "%d" % os.getpid()

    def compile_one(src):
        obj = os.path.join(objdir, os.path.splitext(src)[0] + "." + tag + ".o")
        cmd = [hipcc()] + flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (src, res.stderr[-8000:]))
        if verbose:
            print(" ".join(cmd))
        return obj

    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", "0") or 0) or (os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp" + tag
    cmd = [hipcc()] + flags() + ["-shared"] + objs + ["-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    for o in objs:
        os.remove(o)
    if res.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + res.stderr[-8000:])
    if verbose:
        print(" ".join(cmd))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
