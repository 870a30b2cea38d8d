"""Build libvstitch.so in-tree with hipcc for gfx950.

  python -m paper_2308_09209_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = [os.path.join(HERE, "csrc", n) for n in
           ("vs_host.cpp", "vs_kernels.hip", "vs_flow.hip", "vs_surr.hip", "vs_nn.hip", "vs_nn_host.cpp", "vs_nn_net.cpp", "vs_calib.hip", "vs_var.hip", "vs_noalloc.hip")]
OUT = os.path.join(HERE, "libvstitch.so")

# -ffp-contract=off: every fused multiply-add in the kernels is explicit, so
# the FP32 results follow one operation order.  Packed FP32 instructions are
# disabled for all device code.
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall"]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc] + FLAGS + ["-o", OUT + ".tmp"] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise RuntimeError("hipcc failed")
    if verbose and noise:
        print("\n".join(noise))
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
