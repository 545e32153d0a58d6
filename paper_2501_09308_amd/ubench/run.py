"""Runs the gfx950 instruction-rate and copy microbenchmarks; prints JSON.

    python -m paper_2501_09308_amd.ubench.run
"""
import ctypes as C
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libxrdvi_ubench.so")

BLOCKS, THREADS, ITERS, CHAINS = 2048, 256, 8192, 8


def main():
    lib = C.CDLL(LIB)
    lib.xrdvi_ubench_alu.restype = C.c_double
    lib.xrdvi_ubench_alu.argtypes = [C.c_int] * 5
    lib.xrdvi_ubench_copy.restype = C.c_double
    lib.xrdvi_ubench_copy.argtypes = [C.c_size_t, C.c_int]
    lanes = BLOCKS * THREADS
    out = {"lanes": lanes, "iters": ITERS, "chains": CHAINS}
    for name, kind in [("fma", 0), ("exp", 1), ("rcp", 2), ("mix_rcp_1fma", 11),
                       ("mix_rcp_2fma", 12), ("mix_rcp_4fma", 14)]:
        ms = lib.xrdvi_ubench_alu(kind, BLOCKS, THREADS, ITERS, 5)
        if ms <= 0:
            raise RuntimeError(f"{name} failed: {ms}")
        steps = lanes * ITERS * CHAINS          # chain steps
        out[name] = {"ms": ms, "chain_steps_per_s": steps / (ms * 1e-3)}
        print(f"[ubench] {name}: {ms:.3f} ms", file=sys.stderr, flush=True)
    out["fma"]["tflops"] = 2 * out["fma"]["chain_steps_per_s"] / 1e12
    nbytes = 1 << 30
    ms = lib.xrdvi_ubench_copy(nbytes, 5)
    out["copy"] = {"bytes": nbytes, "ms": ms,
                   "gbs_read_plus_write": 2 * nbytes / (ms * 1e-3) / 1e9}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
