"""Autotuner for the tile shape of the strided FFT passes (columns per tile, threads per
workgroup), per mesh size, on the current GPU.

    python -m paper_1805_02247_amd.tune --sizes 64 128 256 512 [--write]

Times a batched forward + inverse 3-D real FFT through the library for every supported
shape and keeps the fastest; --write stores the result in fft_tiles.json next to this file,
which the binding applies when it loads the library.
"""
import argparse
import ctypes
import json
import os
import time

from . import _lib as L

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fft_tiles.json")
SHAPES = [(8, 256), (16, 256), (32, 256), (8, 512), (16, 512), (32, 512)]


def valid(n, pc, nth):
    return n * pc >= nth and (n * pc + n) * 8 <= 160 * 1024 and n * pc // nth <= 16


def time_shape(n, pc, nth, batch, reps):
    import torch

    from . import api

    L.check(L.lib().pmr_fft_set_tile(n, pc, nth))
    x = torch.randn(batch, n, n, n, device="cuda")
    X = api.fft_r2c(x)
    for _ in range(2):
        api.fft_c2r(api.fft_r2c(x))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        X = api.fft_r2c(x)
        api.fft_c2r(X)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def tune(sizes, write=False):
    result = {}
    for n in sizes:
        batch = max(1, (256 // n) ** 3 // 8) if n < 256 else 1
        reps = 20 if n <= 256 else 5
        times = {}
        for pc, nth in SHAPES:
            if valid(n, pc, nth):
                times[f"{pc}x{nth}"] = time_shape(n, pc, nth, batch, reps)
                print(f"n={n} batch={batch} columns={pc} threads={nth}: "
                      f"{times[f'{pc}x{nth}'] * 1e3:.3f} ms", flush=True)
        best = min(times, key=times.get)
        pc, nth = (int(v) for v in best.split("x"))
        result[str(n)] = {"columns": pc, "threads": nth, "ms": times[best] * 1e3,
                          "all_ms": {k: v * 1e3 for k, v in times.items()}}
        L.check(L.lib().pmr_fft_set_tile(n, pc, nth))
    if write:
        old = {}
        if os.path.exists(CACHE):
            with open(CACHE) as f:
                old = json.load(f)
        old.update(result)
        with open(CACHE, "w") as f:
            json.dump(old, f, indent=1, sort_keys=True)
    return result


def apply_cache():
    """Apply fft_tiles.json if present (called when the library is loaded)."""
    if not os.path.exists(CACHE):
        return {}
    with open(CACHE) as f:
        tiles = json.load(f)
    for n, t in tiles.items():
        L.lib().pmr_fft_set_tile(int(n), int(t["columns"]), int(t["threads"]))
    return tiles


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="+", default=[32, 64, 128, 256, 512])
    ap.add_argument("--write", action="store_true")
    args = ap.parse_args()
    print(json.dumps(tune(args.sizes, args.write)))
