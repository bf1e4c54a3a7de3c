"""Build the HIP library libibpm.so in the package directory (gfx950).

Run as `python -m paper_1109_3524_amd.build` or through __graft_entry__.build().
The host set-up code is compiled by g++ with floating-point contraction off;
the kernels and the C ABI by hipcc for gfx950 only.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libibpm.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# packed-FP32 instructions are disabled: hipcc must not form them on its own
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def _run_all(cmds):
    """Run the compile commands side by side; raise if any fails."""
    procs = []
    for cmd in cmds:
        print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
    bad = [cmd for cmd, p in procs if p.wait() != 0]
    if bad:
        raise subprocess.CalledProcessError(1, bad[0])


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = [os.path.join(BUILD, "setup.o")]
    cmds = [["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, "setup.cpp"), "-o", objs[0]]]
    for name in ("kernels.hip", "nn.hip", "spgemm.hip", "moving.hip", "api.hip"):
        o = os.path.join(BUILD, name.replace(".hip", ".o"))
        cmds.append([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, name), "-o", o])
        objs.append(o)
    _run_all(cmds)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    shutil.move(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
