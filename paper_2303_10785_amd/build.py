"""Build libgbr.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["gbr_api.hip", "gbr_metrics.hip", "gbr_rhs.hip", "gbr_batch.hip", "gbr_stencil.hip", "gbr_bounds.hip",
           "gbr_probe.hip", "gbr_noalloc.hip"]
ARCH = os.environ.get("GBR_OFFLOAD_ARCH", "gfx950")


def library_path():
    return os.path.join(HERE, "libgbr.so")


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False, resource_usage=False):
    """Compile every HIP source for gfx950 and link libgbr.so (always rebuilds)."""
    out = library_path()
    tmp = out + ".tmp"
    flags = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
             # no packed FP32 instructions anywhere in the device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC,
             "-Wall", "-Wno-unused-result"]
    if resource_usage:
        flags += ["-Rpass-analysis=kernel-resource-usage"]
    cmd = [hipcc()] + flags + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    import sys
    print(build(verbose=True, resource_usage="--usage" in sys.argv))
