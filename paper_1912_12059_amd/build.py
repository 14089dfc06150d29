"""Build step for the HIP library ``libnsk.so`` (gfx950)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libnsk.so")
SOURCES = [os.path.join(HERE, "csrc", n) for n in ("nsk.hip", "batch.hip", "closure.hip", "implicit.hip")]
DEPENDS = SOURCES + [
    os.path.join(HERE, "csrc", "dg_kernels.hpp"),
    os.path.join(HERE, "csrc", "closure.hpp"),
    os.path.join(HERE, "csrc", "host_common.hpp"),
    os.path.join(HERE, "csrc", "subcell.hpp"),
    os.path.join(REPO, "include", "nsk.h"),
]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in VGPRs (the closure network applies its activation
    # to them with VALU instructions; in AGPRs each would first be copied out)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
]


def build_lib() -> str:
    """Compile every source to an object in parallel, then link libnsk.so."""
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(HERE, "csrc", os.path.basename(src) + ".o")
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC] + [f for f in FLAGS if f != "-shared"] + ["-c", "-o", obj, src]))
    if any(p.wait() != 0 for p in procs):
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    for obj in objs:
        os.remove(obj)
    return LIB


if __name__ == "__main__":
    print(build_lib())
