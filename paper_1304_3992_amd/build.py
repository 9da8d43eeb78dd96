"""Builds liblogfx.so (HIP kernels + host runtime + C ABI) for gfx950, in-tree.

    python -m paper_1304_3992_amd.build

Needs hipcc (ROCm); no GPU is needed to build.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblogfx.so")
# Mask radius pairs (ra <= rb) instantiated by logfx_kernels_inst.hip.
RADII = [(1, 1), (1, 2), (2, 2), (1, 3), (2, 3), (3, 3), (1, 4), (2, 4), (3, 4), (4, 4)]
ARCH = os.environ.get("LOGFX_ARCH", "gfx950")

# Packed FP32 instructions are disabled for all device code.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]


def _units():
    """(source, object, extra flags) of every translation unit."""
    b = os.path.join(HERE, "_build")
    units = [("logfx_host.cpp", os.path.join(b, "logfx_host.o"), []),
             ("logfx_dispatch.hip", os.path.join(b, "logfx_dispatch.o"), ["-x", "hip"]),
             ("logfx_gate.hip", os.path.join(b, "logfx_gate.o"), ["-x", "hip"]),
             ("logfx_pass2z.hip", os.path.join(b, "logfx_pass2z.o"), ["-x", "hip"])]
    for ra, rb in RADII:
        units.append(("logfx_kernels_inst.hip", os.path.join(b, f"logfx_kernels_r{ra}{rb}.o"),
                      ["-x", "hip", f"-DLOGFX_RA={ra}", f"-DLOGFX_RB={rb}"]))
    return units


def _vgpr_spills(remarks: str) -> list[str]:
    """Kernels whose resource-usage remarks report spilled vector registers."""
    out, name = [], None
    for line in remarks.splitlines():
        if "Function Name:" in line:
            name = line.split("Function Name:")[1].split()[0]
        elif "VGPRs Spill:" in line and name:
            n = int(line.split("VGPRs Spill:")[1].split()[0])
            if n > 0:
                out.append(f"{name} ({n})")
    return out


def build(verbose: bool = False, jobs: int | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    jobs = jobs or max(1, min(16, os.cpu_count() or 1))
    pending = list(_units())
    running, objs = [], []
    while pending or running:
        while pending and len(running) < jobs:
            src, obj, extra = pending.pop(0)
            # device units report each kernel's register use (spills refused below)
            remarks = ["-Rpass-analysis=kernel-resource-usage"] if "hip" in extra else []
            cmd = [hipcc, *HIP_FLAGS, *remarks, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *extra,
                   "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True), cmd))
            objs.append(obj)
        p, cmd = running.pop(0)
        err = p.communicate()[1]
        spills = _vgpr_spills(err)
        if p.returncode == 0 and "-Rpass-analysis=kernel-resource-usage" in cmd and "Function Name:" not in err:
            raise RuntimeError("no kernel resource-usage remarks from " + " ".join(cmd))
        err = "\n".join(l for l in err.splitlines()
                        if "packed-fp32-ops" not in l and "kernel-resource-usage" not in l)
        if p.returncode != 0:
            raise RuntimeError("compile failed: " + " ".join(cmd) + "\n" + err)
        if spills:
            raise RuntimeError("kernels spill vector registers (their neighbour reads across lanes "
                               "need every lane's registers intact): " + ", ".join(spills))
        if err.strip() and verbose:
            print(err, flush=True)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
