"""Builds libssp.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1106_2899_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libssp.so")
PROBE_LIB = os.path.join(PKG, "libssp_probe.so")  # VALU issue-cost probe (measurement only)

SOURCES = ["ssp_step.hip", "ssp_aux.hip", "ssp_adjoint.hip", "ssp_moduli.hip", "ssp_api.cpp"]
HEADERS = ["ssp_device.h", "ssp_internal.h"]

# Packed FP32 instructions are disabled for all device code (the compiler
# would otherwise pair float operations into v_pk_* forms).
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", f"-I{os.path.join(ROOT, 'include')}"]


def hipcc() -> str:
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libssp")


def build(verbose: bool = False, jobs: int = 3) -> str:
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="ssp_build_") as tmp:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            cmd = [cc, *COMMON]
            if src.endswith(".hip"):
                cmd += ["-x", "hip", *DEVICE_FLAGS]
            else:
                cmd += ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
            cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append(subprocess.Popen(cmd, cwd=tmp))
            objs.append(obj)
            if len([p for p in procs if p.poll() is None]) >= jobs:
                procs[0].wait()
        for p in procs:
            if p.wait() != 0:
                raise RuntimeError("hipcc failed")
        out_tmp = LIB + ".tmp"
        cmd = [cc, *DEVICE_FLAGS, "-shared", "-fPIC", "-o", out_tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd, cwd=tmp)
        os.replace(out_tmp, LIB)
        cmd = [cc, *COMMON, "-x", "hip", *DEVICE_FLAGS, "-shared", "-o", PROBE_LIB + ".tmp",
               os.path.join(CSRC, "issue_probe.hip")]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd, cwd=tmp)
        os.replace(PROBE_LIB + ".tmp", PROBE_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
