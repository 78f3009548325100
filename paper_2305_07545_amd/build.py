"""Build the gfx950 KmerCo library (``libkmerco_hip.so``) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libkmerco_hip.so")
SOURCES = ["kc_kernels.hip", "kc_binned.hip", "kc_batched.hip", "kc_scan.hip", "kc_api.hip", "kc_batch_api.hip", "kc_serve.hip", "kc_fastx.hip", "kc_noalloc.hip"]
MICROBENCH_LIB = os.path.join(HERE, "libkmerco_microbench.so")
MICROBENCH_SOURCES = ["kc_microbench.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _compile(sources, out, verbose):
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", INCLUDE, "-I", CSRC,
           *[os.path.join(CSRC, s) for s in sources], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {out}:\n{r.stdout}")
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    """Compile every HIP source for gfx950: the KmerCo library and the
    memory-system microbenchmarks."""
    _compile(MICROBENCH_SOURCES, MICROBENCH_LIB, verbose)
    return _compile(SOURCES, LIB, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
