"""Build libwe.so (HIP, gfx950) in-tree.

Flags:
  --offload-arch=gfx950        MI355X only
  -ffp-contract=off            no a*b+c -> fma contraction: every FP64 step is
                               one rounded operation, in source order, which the
                               lane-per-walker path relies on for bit-identical
                               trajectories
  -target-feature -packed-fp32-ops   keep the compiler from emitting packed
                               FP32 instructions
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libwe.so")

SOURCES = ["we_runtime.hip", "work_queue.hip", "ssa_lane.hip", "ssa_wave.hip", "we_resample.hip", "reweight.hip",
           "committor.hip", "batch.hip", "checkpoint.hip", "ssa_group.hip", "peaks.hip"]


def hipcc() -> str:
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags():
    return ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
            "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-fvisibility=hidden", "-Wall", "-Wno-unused-result",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def build(verbose: bool = False, save_temps: str = "") -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [hipcc(), *flags(), "-c", os.path.join(CSRC, src), "-o", obj]
        if save_temps:
            cmd += ["-save-temps=obj"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, save_temps=("--asm" in sys.argv) and "1" or ""))
