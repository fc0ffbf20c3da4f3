"""Autotuner for the tile shapes of the strided FFT passes (columns per tile, threads per
workgroup, and the staging and radix of the butterflies: register images with radix-8
stages, or the LDS-staged tile with radix-8 or radix-4 stages), separately for the y pass,
the x pass
with single-input k-space operators and the x pass with multi-input operators, per mesh size,
on the current GPU.

    python -m paper_1805_02247_amd.tune --sizes 64 128 256 512 [--write]
    python -m paper_1805_02247_amd.tune --workload 256 512 256 10 1 64 [--write]

The first form times a batched forward + inverse 3-D real FFT through the library for every
supported shape. The second times whole gradient evaluations (forward + adjoint) of a
workload given as n_part n_mesh n_out n_steps batch hidden [precision], tuning each pass of
each mesh size it uses in turn with the others held fixed, which also ranks the operator
passes (force, force adjoint, smoothing) by their real cost, and then the kz-slab width of
the force transforms on the force mesh and the rows per wavefront of the paints (one and
three channels on the force mesh, one on the output mesh). --write stores the result in
fft_tiles.json next to this file, which the binding applies when it loads the library.
"""
import argparse
import json
import os
import time

from . import _lib as L

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fft_tiles.json")
SHAPES = [(8, 256), (16, 256), (32, 256), (8, 512), (16, 512), (32, 512)]
PASSES = {"y": L.PMR_FFT_YPASS, "x": L.PMR_FFT_XPASS, "xm": L.PMR_FFT_XPASS_MULTI}


def valid(n, pc, nth):
    return n * pc >= nth and (n * pc + n) * 8 <= 160 * 1024 and n * pc // nth <= 16


STAGINGS = {0: "reg", 1: "lds", 2: "lds4"}  # registers (radix 8), LDS radix 8, LDS radix 4


def register_capable(n, pc, nth):
    """Shapes whose butterflies can run on register images (otherwise staging 0 falls back
    to the LDS-staged radix-8 pass)."""
    p = n * pc // nth
    return n >= 64 and p >= 8 and p % 8 == 0


def candidates(n):
    out = []
    for pc, nth in SHAPES:
        if valid(n, pc, nth):
            for st in ((0, 1, 2) if register_capable(n, pc, nth) else (1, 2)):
                out.append((pc, nth, st))
    return out


def _key(c):
    return f"{c[0]}x{c[1]}x{STAGINGS[c[2]]}"


def _set(n, pass_, c):
    L.check(L.lib().pmr_fft_set_tile(n, pass_, c[0], c[1], c[2]))


def _timer(fn, reps, warmup=1):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _fft_step(n, batch):
    import torch

    from . import api
    x = torch.randn(batch, n, n, n, device="cuda")

    def step():
        api.fft_c2r(api.fft_r2c(x))
    return step


def _gradient_step(n_part, n_mesh, n_out, n_steps, batch, hidden, precision):
    """A gradient evaluation of the given workload on random inputs (timing only)."""
    import numpy as np
    import torch

    from . import api, cosmo
    cfg = api.Config(batch=batch, n_part=n_part, n_mesh=n_mesh, n_out=n_out, n_steps=n_steps,
                     mlp_hidden=hidden, precision=precision, box=400.0,
                     ckpt_every=2 if n_steps > 5 else 0, loss_kind=L.PMR_LOSS_LOGNORMAL)
    power = cosmo.linear_power(0.8, 0.2)
    pm = api.PMContext(cfg, "cuda")
    pm.set_prior(torch.from_numpy(cosmo.prior_inv_variance(n_part, cfg.box, power)))
    g = torch.Generator().manual_seed(0)

    def w(shape, fan_in):
        return torch.randn(*shape, generator=g, dtype=torch.float64).mul(np.sqrt(2.0 / fan_in)).float()
    pm.set_mlp({"W1": w((hidden, 3), 3), "b1": torch.zeros(hidden), "W2": w((hidden, hidden), hidden),
                "b2": torch.zeros(hidden), "W3": w((1, hidden), hidden), "b3": torch.zeros(1)})
    pm.set_target(torch.ones(batch, n_out ** 3, device="cuda"))
    pm.set_loss(api.LossParams(M0=1.0))
    white = torch.randn(batch, n_part, n_part, n_part, generator=g, dtype=torch.float64).numpy()
    modes = torch.stack([torch.from_numpy(cosmo.modes_from_white_noise(white[b], cfg.box, power)
                                          .reshape(-1)) for b in range(batch)]).to("cuda")
    ones = torch.ones(batch, dtype=torch.float64, device="cuda")
    grad = torch.empty(batch, pm.n_modes, dtype=torch.complex64, device="cuda")

    def step():
        pm.forward(modes, want_mass=False)
        pm.adjoint(ones, out=grad)
    step.pm = pm
    return step


def _tune_passes(step, sizes, reps, log):
    """Coordinate search: each (size, pass) in turn over all candidates, the others fixed at
    their current best."""
    best = {n: {p: _get(n, pid) for p, pid in PASSES.items()} for n in sizes}
    all_ms = {}
    for n in sizes:
        for p, pid in PASSES.items():
            times = {}
            for c in candidates(n):
                _set(n, pid, c)
                times[c] = _timer(step, reps)
                log(f"n={n} pass={p} columns={c[0]} threads={c[1]} "
                    f"staging={STAGINGS[c[2]]}: {times[c] * 1e3:.3f} ms")
            c = min(times, key=times.get)
            _set(n, pid, c)
            best[n][p] = c
            all_ms[(n, p)] = {_key(k): v * 1e3 for k, v in times.items()}
    return {str(n): {p: {"columns": best[n][p][0], "threads": best[n][p][1],
                         "staging": best[n][p][2], "all_ms": all_ms[(n, p)]} for p in PASSES}
            for n in sizes}


def _get(n, pass_):
    import ctypes
    c, t, s = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    L.check(L.lib().pmr_fft_get_tile(n, pass_, ctypes.byref(c), ctypes.byref(t), ctypes.byref(s)))
    return (c.value, t.value, s.value)


def tune(sizes, write=False, log=print):
    result = {}
    for n in sizes:
        batch = max(1, (256 // n) ** 3 // 8) if n < 256 else 1
        result.update(_tune_passes(_fft_step(n, batch), [n], 20 if n <= 256 else 5, log))
    if write:
        _write(result)
    return result


SLABS = (0, 16, 32, 64)


def _tune_slab(step, n, reps, log):
    """kz-slab width of the force transforms on the n^3 mesh (0: whole passes)."""
    times = {}
    for cols in SLABS:
        L.check(L.lib().pmr_fft_set_slab(n, cols))
        times[cols] = _timer(step, reps)
        log(f"n={n} slab={cols}: {times[cols] * 1e3:.3f} ms")
    best = min(times, key=times.get)
    L.check(L.lib().pmr_fft_set_slab(n, best))
    return {"columns": best, "all_ms": {str(k): v * 1e3 for k, v in times.items()}}


PAINT_ROWS = (1, 2, 4, 8, 16)


def _tune_paint(step, n, channels, reps, log):
    """Rows per wavefront of the paint with `channels` channels on the n^3 mesh."""
    import ctypes
    times = {}
    for rows in PAINT_ROWS:
        L.check(L.lib().pmr_paint_set_rows(n, channels, rows))
        c = ctypes.c_int()
        L.check(L.lib().pmr_paint_get_rows(n, channels, ctypes.byref(c)))
        times[rows] = _timer(step, reps)
        log(f"n={n} paint channels={channels} rows={rows}: {times[rows] * 1e3:.3f} ms")
    best = min(times, key=times.get)
    L.check(L.lib().pmr_paint_set_rows(n, channels, best))
    return {"columns": best, "all_ms": {str(k): v * 1e3 for k, v in times.items()}}


def tune_workload(n_part, n_mesh, n_out, n_steps, batch, hidden, precision=0, write=False,
                  log=print):
    step = _gradient_step(n_part, n_mesh, n_out, n_steps, batch, hidden, precision)
    sizes = sorted({n_mesh, n_out, n_part}, reverse=True)
    reps = 2 if n_mesh >= 512 else 5
    result = _tune_passes(step, sizes, reps, log)
    result[str(n_mesh)]["slab"] = _tune_slab(step, n_mesh, reps, log)
    # the paint shapes: density (1 channel) and adjoint (3 channels) on the force mesh, and
    # the final paint on the output mesh
    result[str(n_mesh)]["paint3"] = _tune_paint(step, n_mesh, 3, reps, log)
    result[str(n_mesh)]["paint1"] = _tune_paint(step, n_mesh, 1, reps, log)
    if n_out != n_mesh:
        result[str(n_out)]["paint1"] = _tune_paint(step, n_out, 1, reps, log)
    if write:
        _write(result)
    return result


def _write(result):
    old = {}
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            old = json.load(f)
    old.update(result)
    with open(CACHE, "w") as f:
        json.dump(old, f, indent=1, sort_keys=True)


def apply_cache():
    """Apply fft_tiles.json if present (called when the library is loaded)."""
    if not os.path.exists(CACHE):
        return {}
    with open(CACHE) as f:
        tiles = json.load(f)
    for n, per_pass in tiles.items():
        for p, t in per_pass.items():
            if p in PASSES:
                L.lib().pmr_fft_set_tile(int(n), PASSES[p], int(t["columns"]), int(t["threads"]),
                                         int(t.get("staging", 0)))
            elif p == "slab":
                L.lib().pmr_fft_set_slab(int(n), int(t["columns"]))
            elif p in ("paint1", "paint3"):
                L.lib().pmr_paint_set_rows(int(n), int(p[-1]), int(t["columns"]))
    return tiles


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="+", default=None)
    ap.add_argument("--workload", type=int, nargs="+", default=None,
                    help="n_part n_mesh n_out n_steps batch hidden [precision]")
    ap.add_argument("--write", action="store_true")
    args = ap.parse_args()
    say = lambda s: print(s, flush=True)  # noqa: E731
    if args.workload:
        out = tune_workload(*args.workload, write=args.write, log=say)
    else:
        out = tune(args.sizes or [32, 64, 128, 256, 512], args.write, log=say)
    print(json.dumps(out))
