"""Build libsrwcr.so in-tree for gfx950 with hipcc (no JIT, no torch extension)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/srwcr_kernels.hip", "csrc/srwcr_host.cpp", "csrc/srwcr_lbfgs.cpp", "csrc/srwcr_noalloc.hip"]
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-munsafe-fp-atomics",                       # native FP64 atomics in LDS and L2
    # No packed FP32 (v_pk_*_f32) in the device code: some of its forms have
    # been seen to give wrong results on gfx950.  hipcc's host (x86) pass prints
    # "'-packed-fp32-ops' is not a recognized feature for this target" once per
    # source; the gfx950 pass honours the flag (its code objects hold no
    # v_pk_*_f32 with it, hundreds without).
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    out = os.path.join(HERE, "libsrwcr.so")
    tmp = out + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc"),
           "-o", tmp, *[os.path.join(HERE, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libsrwcr.so")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
