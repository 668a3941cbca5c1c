"""Build libmbh.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmbh.so")
SOURCES = ["mbh_lib.hip", "mbh_serve.hip"]
ARCH = os.environ.get("MBH_OFFLOAD_ARCH", "gfx950")


def hipcc_cmd(out: str = LIB, extra=()):
    return (["hipcc", "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=on",
             "-Wno-unused-result",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", out]
            + [os.path.join(CSRC, s) for s in SOURCES] + ["-lpthread"] + list(extra))


def build(verbose: bool = False) -> str:
    cmd = hipcc_cmd()
    if verbose:
        print(" ".join(cmd), flush=True)
    tmp = LIB + ".tmp"
    cmd[cmd.index("-o") + 1] = tmp
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
