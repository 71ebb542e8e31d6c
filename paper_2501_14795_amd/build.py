"""Build libpic.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
SO = os.path.join(HERE, "libpic.so")
SOURCES = ["pic_api.hip", "k_push.hip", "k_sort.hip", "k_field.hip", "k_filter.hip", "k_window.hip", "k_diag.hip",
           "k_poisson.hip", "k_tilesort.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions (v_pk_*_f32) anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # float atomics in global memory as native instructions
    "-munsafe-fp-atomics",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    """Compile every HIP source into paper_2501_14795_amd/libpic.so."""
    tmp = SO + ".tmp"
    cmd = [HIPCC, *FLAGS, *(extra or []), "-I", INCLUDE, "-I", CSRC,
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
