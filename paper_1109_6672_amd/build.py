"""Builds ``liblbddf.so`` in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", "lbddf.hip")]
OUT = os.path.join(HERE, "liblbddf.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


OUT_FP64 = os.path.join(HERE, "liblbddf_fp64.so")  # the step's arithmetic in FP64


def _compile(out: str, extra: list, verbose: bool) -> str:
    tmp = out + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, *extra, "-o", tmp, *SOURCES]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed for {os.path.basename(out)}")
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    """Both libraries from the one source: FP32 arithmetic (liblbddf.so) and
    FP64 arithmetic (liblbddf_fp64.so, -DLB_ARITH_FP64); the same ABI and
    storage formats.  Returns the path of the FP32 one."""
    _compile(OUT_FP64, ["-DLB_ARITH_FP64"], verbose)
    return _compile(OUT, [], verbose)


if __name__ == "__main__":
    print(build(verbose=True))
