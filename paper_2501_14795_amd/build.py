"""Build libpic.so (HIP, gfx950) in-tree with hipcc.

Every source is compiled to its own object (in parallel: the push kernel's
template instantiations dominate the build), then the objects are linked."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
SO = os.path.join(HERE, "libpic.so")
OBJ = os.path.join(ROOT, "_build")
SOURCES = ["pic_api.hip", "k_push.hip", "k_sort.hip", "k_field.hip", "k_filter.hip", "k_window.hip", "k_diag.hip",
           "k_poisson.hip", "k_tilesort.hip", "k_probe.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions (v_pk_*_f32) anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # float atomics in global memory as native instructions
    "-munsafe-fp-atomics",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, extra: list[str] | None = None, jobs: int | None = None) -> str:
    """Compile every HIP source and link paper_2501_14795_amd/libpic.so."""
    os.makedirs(OBJ, exist_ok=True)
    extra = list(extra or [])

    def compile_one(src):
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *FLAGS, *extra, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        # hipcc's host pass warns that it does not know the packed-FP32 feature: harmless
        out = "\n".join(ln for ln in r.stdout.splitlines() if "packed-fp32-ops" not in ln)
        if out.strip():
            print(out, flush=True)
        if r.returncode != 0:
            raise subprocess.CalledProcessError(r.returncode, cmd)
        return obj

    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1, 8)
    # the largest translation units first, so they do not finish last
    order = sorted(SOURCES, key=lambda s: -os.path.getsize(os.path.join(CSRC, s)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = dict(zip(order, ex.map(compile_one, order)))
    tmp = SO + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *[objs[s] for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
