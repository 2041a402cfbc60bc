"""Build libtx.so in-tree with hipcc for gfx950.

    python -m paper_2401_13834_amd.build

Compiles every source under csrc/ and links them into
paper_2401_13834_amd/libtx.so.  Always rebuilds.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtx.so")
ARCH = "gfx950"

HIP_SOURCES = ["tx_kernels.hip"]
HOST_SOURCES = ["tx_plan.cpp", "tx_api.cpp", "tx_profile.cpp"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-ffp-contract=off", "-Wall", "-Wno-unused-result"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("command failed: " + " ".join(cmd))
    return r


def build(verbose=False):
    cc = hipcc()
    objs = []
    with tempfile.TemporaryDirectory(prefix="txbuild_") as tmp:
        for src in HIP_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            cmd = [cc, "-c", "-x", "hip", os.path.join(CSRC, src), "-o", obj] + COMMON + DEVICE
            if verbose:
                print(" ".join(cmd))
            _run(cmd)
            objs.append(obj)
        for src in HOST_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            cmd = [cc, "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + DEVICE
            if verbose:
                print(" ".join(cmd))
            _run(cmd)
            objs.append(obj)
        tmp_lib = LIB + ".tmp"
        cmd = [cc, "-shared", "-o", tmp_lib] + objs + [f"--offload-arch={ARCH}", "-fPIC"]
        if verbose:
            print(" ".join(cmd))
        _run(cmd)
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
