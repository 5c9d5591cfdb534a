"""Build the HIP library ``libggfv.so`` in-tree for gfx950.

    python -m paper_2006_01748_amd.build

Every HIP source under ``csrc/`` is compiled with hipcc for gfx950 into one shared
library next to this file.  Floating-point contraction is off (the step's
arithmetic order is part of its contract) and packed FP32 instructions are
disabled.  The optimizer's sinking of common code out of the branches of a
condition is off: in the register-ring kernels it merges stores to different
ring slots into one store through a selected address, which moves the rings to
scratch memory.  The build fails if any kernel uses scratch memory or spills
(from the compiler's per-kernel resource report).
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_NAME = "libggfv.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-mcode-object-version=5",
    "-fPIC",
    "-ffp-contract=off",
    "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-result",
    "-mllvm", "-simplifycfg-sink-common=false",
    "-Rpass-analysis=kernel-resource-usage",
]

# Extra flags per source.  The lane-shift kernels carry several steps of a row
# sweep in registers at two or three waves per SIMD, so the order of
# independent instructions inside one wave decides how busy the vector unit
# is.  The scheduler's instruction-level-parallelism strategy measured faster
# for the FP32 instances on MI355X (compensated FP32 +5.5%, FP32 +2%) and only
# reorders instructions.  The FP64 instances (ggfv_fused_dpp_f64.hip) keep the
# default schedule: with their late stores the ILP schedule spills.
SOURCE_FLAGS = {
    "ggfv_fused_dpp.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
}


def scratch_users(text: str):
    """Kernels whose resource report shows scratch memory or spills."""
    bad, name = [], None
    for line in text.splitlines():
        if "remark: Function Name:" in line:
            name = line.split("Function Name:")[1].split("[")[0].strip()
        elif name and ("ScratchSize [bytes/lane]:" in line or "VGPRs Spill:" in line or "SGPRs Spill:" in line):
            value = line.split(":")[-1].split("[")[0].strip()
            if value not in ("0", ""):
                bad.append((name, line.split("remark:")[1].split("[")[0].strip()))
    return bad


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return path


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False, extra_flags=()) -> str:
    """Compile all sources (one object per source, in parallel) and link."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [hipcc(), *HIPCC_FLAGS, *SOURCE_FLAGS.get(os.path.basename(src), ()), *extra_flags,
               "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 target feature; harmless
        lines = [l for l in text.splitlines()
                 if "packed-fp32-ops" not in l and "kernel-resource-usage" not in l and l.strip()]
        if p.returncode != 0:
            failed.append((src, "\n".join(lines)))
            continue
        bad = scratch_users(text)
        if bad:
            failed.append((src, "kernels using scratch memory:\n" + "\n".join(f"  {n}: {w}" for n, w in bad)))
        elif lines and verbose:
            print("\n".join(lines))
    if failed:
        msg = "\n\n".join(f"{s}:\n{t}" for s, t in failed)
        raise RuntimeError(f"hipcc failed:\n{msg}")
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB_PATH)
