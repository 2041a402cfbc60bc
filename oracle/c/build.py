"""Build the C oracle (test infrastructure) into oracle/c/libtx_oracle.so.

gcc, -O3 with auto-vectorisation for a portable x86-64 level (the library may
run on another host than the one that built it), OpenMP, and no
floating-point contraction (the delays must round exactly as written)."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tx_oracle.c")
SO = os.path.join(HERE, "libtx_oracle.so")
FLAGS = ["-O3", "-march=x86-64-v3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
         "-std=c11", "-Wall", "-Wno-unknown-pragmas"]


def build(force=False):
    if not force and os.path.exists(SO) and os.path.getmtime(SO) >= os.path.getmtime(SRC):
        return SO
    tmp = SO + ".tmp"
    subprocess.run(["gcc"] + FLAGS + [SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
