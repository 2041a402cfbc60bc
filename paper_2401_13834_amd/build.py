"""Build libtx.so (and the tx_peaks microbenchmark) in-tree with hipcc for gfx950.

    python -m paper_2401_13834_amd.build [-v]

Compiles every source under csrc/ (in parallel) and links them into
paper_2401_13834_amd/libtx.so; builds paper_2401_13834_amd/tx_peaks from
csrc/tx_peaks.hip.  Always rebuilds.
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
PEAKS = os.path.join(HERE, "tx_peaks")
ARCH = "gfx950"

HIP_SOURCES = ["tx_kernels_dedisp.hip", "tx_kernels_boxcar.hip", "tx_kernels_transpose.hip",
               "tx_kernels_downsample.hip", "tx_kernels_cluster.hip", "tx_kernels_stats.hip", "tx_kernels_norm.hip"]
HOST_SOURCES = ["tx_plan.cpp", "tx_api.cpp", "tx_profile.cpp", "tx_stream.cpp", "tx_batch.cpp", "tx_autotune.cpp",
                "tx_ranges.cpp", "tx_cluster.cpp", "tx_mask.cpp", "tx_norm.cpp"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-ffp-contract=off", "-Wall", "-Wno-unused-result"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run_all(cmds, verbose):
    procs = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd))
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = None
    for cmd, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out)
            failed = failed or cmd
    if failed:
        raise RuntimeError("command failed: " + " ".join(failed))


def build(verbose=False):
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="txbuild_") as tmp:
        objs, cmds = [], []
        for src in HIP_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            cmds.append([cc, "-c", "-x", "hip", os.path.join(CSRC, src), "-o", obj] + COMMON + DEVICE)
            objs.append(obj)
        for src in HOST_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            cmds.append([cc, "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + DEVICE)
            objs.append(obj)
        tmp_peaks = PEAKS + ".tmp"
        cmds.append([cc, os.path.join(CSRC, "tx_peaks.hip"), "-o", tmp_peaks, "-O3", "-std=c++17"] + DEVICE)
        _run_all(cmds, verbose)
        tmp_lib = LIB + ".tmp"
        _run_all([[cc, "-shared", "-o", tmp_lib] + objs + [f"--offload-arch={ARCH}", "-fPIC"]], verbose)
        os.replace(tmp_lib, LIB)
        os.replace(tmp_peaks, PEAKS)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
