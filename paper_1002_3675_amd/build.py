"""Build the HIP library libcbct.so (gfx950) in-tree with hipcc.

    python -m paper_1002_3675_amd.build

Every call compiles (no staleness shortcut), so a changed source is always
picked up.  Packed-FP32 instruction selection is disabled for all device
code.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["api.hip", "project.hip", "backproject.hip", "tv.hip", "misc.hip"]
LIB = os.path.join(HERE, "libcbct.so")
ARCH = os.environ.get("CBCT_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def flags():
    return ["--offload-arch=%s" % ARCH, "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]


def build(verbose: bool = False) -> str:
    objs = []
    jobs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [hipcc()] + flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append(subprocess.Popen(cmd))
        objs.append(obj)
    bad = [j.args for j in jobs if j.wait() != 0]
    if bad:
        raise RuntimeError("hipcc failed: %s" % bad)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=%s" % ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        try:
            os.remove(o)
        except OSError:
            pass
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
