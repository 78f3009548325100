"""Roofline denominators for the KmerCo kernels on the local GPU.

Runs the memory-system microbenchmarks of ``libkmerco_microbench.so``:
uniform-random 64-bit reads / atomics and 32-bit atomicMin over footprints
from L2-sized to HBM-sized, a streaming copy, and LDS atomics.  Prints one
JSON object: {kind: {footprint_bytes: operations per second}}.
"""
from __future__ import annotations

import ctypes
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libkmerco_microbench.so")

KINDS = {"read64": 0, "add64": 1, "cas64": 2, "min32": 3, "add64_ret": 4, "copy64": 5, "lds": 6,
         "alu_add32": 7, "alu_mul_lo32": 8, "alu_mul_hi32": 9, "alu_mad64": 10}


def load():
    if not os.path.exists(LIB):
        raise RuntimeError(f"{LIB} not built")
    lib = ctypes.CDLL(LIB)
    lib.kcmb_run.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                             ctypes.POINTER(ctypes.c_double)]
    lib.kcmb_run.restype = ctypes.c_int
    return lib


def rate(kind: str, footprint: int, ops: int) -> float:
    """Operations per second (copy: bytes moved per second)."""
    ms = ctypes.c_double(0)
    rc = load().kcmb_run(KINDS[kind], footprint, ops, ctypes.byref(ms))
    if rc != 0:
        raise RuntimeError(f"kcmb_run({kind}, {footprint}) failed: {rc}")
    if kind == "copy64":
        n = min(ops, footprint // 8)
        return n * 16 / (ms.value / 1e3)
    return ops / (ms.value / 1e3)


def main(argv):
    import torch  # noqa: F401 - initialises the HIP runtime the same way the library sees it
    if argv and argv[0] == "--alu":
        # integer VALU issue rates (lane operations per second)
        out = {k: rate(k, 8, 1 << 34) for k in ("alu_add32", "alu_mul_lo32", "alu_mul_hi32",
                                                  "alu_mad64")}
        for k, v in out.items():
            print(f"{k:14s} {v / 1e12:8.2f} T lane-ops/s", flush=True)
        print(json.dumps(out))
        return
    if argv and argv[0] == "--copy":
        # one streaming copy of a known size (calibrates traffic counters):
        # reads and writes argv[1] bytes
        n = int(argv[1]) if len(argv) > 1 else 1 << 30
        print(json.dumps({"copy_bytes_each_way": n, "bytes_per_s": rate("copy64", n, n // 8)}))
        return
    sizes = [int(x) for x in argv] if argv else [
        512 << 10, 4 << 20, 32 << 20, 128 << 20, 512 << 20, 2 << 30, 8 << 30]
    ops = 1 << 27
    out = {}
    for kind in ["read64", "add64", "add64_ret", "cas64", "min32"]:
        out[kind] = {}
        for s in sizes:
            out[kind][s] = rate(kind, s, ops)
            print(f"{kind:10s} {s / 2**20:10.2f} MiB  {out[kind][s] / 1e9:8.2f} G/s", flush=True)
    out["copy64"] = {2 << 30: rate("copy64", 2 << 30, 1 << 28)}
    print(f"copy64 2 GiB {out['copy64'][2 << 30] / 1e9:.1f} GB/s", flush=True)
    out["lds"] = {128 << 10: rate("lds", 0, 1 << 30)}
    print(f"lds add+min pairs {out['lds'][128 << 10] / 1e9:.1f} G/s", flush=True)
    print(json.dumps({k: {str(s): v for s, v in d.items()} for k, d in out.items()}))


if __name__ == "__main__":
    main(sys.argv[1:])
