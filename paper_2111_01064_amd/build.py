"""Build libmbh.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmbh.so")
SOURCES = ["mbh_lib.hip", "mbh_serve.hip", "mbh_sampler.hip", "mbh_ingest.hip"]
LIBS = ["-lpthread", "-lhipfft"]
ARCH = os.environ.get("MBH_OFFLOAD_ARCH", "gfx950")


def _flags():
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=on",
            "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def hipcc_cmd(out: str = LIB, extra=()):
    """One hipcc line that compiles and links every source (for reference)."""
    return (["hipcc"] + _flags() + ["-shared", "-o", out]
            + [os.path.join(CSRC, s) for s in SOURCES] + LIBS + list(extra))


def build(verbose: bool = False) -> str:
    """Compile the sources in parallel (one hipcc per source), then link."""
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = ["hipcc"] + _flags() + ["-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for p, cmd in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, cmd)
    tmp = LIB + ".tmp"
    link = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-o", tmp] + objs + LIBS
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
