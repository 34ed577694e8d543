"""Builds libbri.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libbri.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["bri_kernels.hip", "bri_refine.hip", "bri_noalloc.hip", "bri_api.cpp", "bri_plan.cpp", "bri_tune.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for every device compilation.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                # MFMA accumulators in VGPRs: no per-iteration AGPR<->VGPR copies
                "-mllvm", "-amdgpu-mfma-vgpr-form"]
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result",
          "-I" + os.path.join(HERE, "..", "include"), "-I" + CSRC]


RESOURCE_REPORT = os.path.join(BUILD, "kernel_resources.txt")


def _resources(text: str) -> list:
    """(kernel, VGPRs, AGPRs, scratch bytes per lane) from hipcc's resource remarks."""
    rows, cur = [], None
    for line in text.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = {"name": m.group(1)}
            rows.append(cur)
            continue
        m = re.search(r"remark:\s+(VGPRs|AGPRs|ScratchSize) ?(?:\[bytes/lane\])?: (\d+)", line)
        if m and cur is not None:
            cur[m.group(1)] = int(m.group(2))
    return rows


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip", *DEVICE_FLAGS, "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    if src.endswith(".hip"):
        # Per-kernel register and scratch use, kept for inspection and tests.
        rows = _resources(r.stderr)
        with open(os.path.join(BUILD, os.path.splitext(src)[0] + ".resources.txt"), "w") as f:
            for row in rows:
                f.write(f"{row['name']} vgprs={row.get('VGPRs', 0)} agprs={row.get('AGPRs', 0)} "
                        f"scratch={row.get('ScratchSize', 0)}\n")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, *DEVICE_FLAGS, "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
