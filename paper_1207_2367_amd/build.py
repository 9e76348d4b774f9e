"""Build the gfx950 shared library ``libnbody.so`` in-tree with hipcc.

Packed FP32 instructions are switched off for every device compilation
(``-Xclang -target-feature -Xclang -packed-fp32-ops``): the kernels are
written in scalar FP32/FP64 and must not be turned into packed forms.
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnbody.so")
SOURCES = ["force.hip", "integrate.hip", "capi.hip"]
ARCH = os.environ.get("NBODY_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(verbose: bool = True) -> str:
    """Compile every source to an object, then link libnbody.so (always
    rebuilds).  Returns the library path."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    t0 = time.time()
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = ["hipcc", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    for cmd, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 feature and says so
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l]
        if p.returncode != 0:
            sys.stderr.write("\n".join(lines) + "\n")
            raise RuntimeError("hipcc failed: " + " ".join(cmd))
        if verbose and any(l.strip() for l in lines):
            sys.stderr.write("\n".join(lines) + "\n")
    tmp = LIB + ".tmp"
    subprocess.check_call(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    # stand-alone probes: VALU throughput / v_rsq_f32 rounding, and the cost
    # of a barrier across the workgroups of a cooperative launch
    for name in ("valu_probe", "barrier_probe"):
        probe = os.path.join(HERE, name)
        subprocess.check_call(["hipcc", *[f for f in FLAGS if f != "-fPIC"], "-o",
                               probe + ".tmp", os.path.join(CSRC, name + ".hip")],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        os.replace(probe + ".tmp", probe)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s")
    return LIB


if __name__ == "__main__":
    build()
