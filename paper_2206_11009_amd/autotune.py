"""Autotuner for the launch shapes and schedules of the otip library.

    python -m paper_2206_11009_amd.autotune [--out PATH]

Measures, on the GPU it runs on:
  * the pricing scan's tile width (targets per workgroup, params.price_tile)
    for each problem size in SIZES, timing otip_price with kmax = m on grid
    coordinates and duals of the scale of an optimum (three repetitions, the
    median kept);
  * the number of batch workers (params.batch_workers) on the 512-instance
    uneven batch family, timing whole otip_solve_batch calls.
and writes the winners to tuning.json beside the library.  tuned(m, n, ...)
returns the parameter overrides for a problem from that file (the entry of the
nearest size on a log scale), or {} when no tuning has been recorded.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING = os.path.join(HERE, "tuning.json")
SIZES = [16, 32, 64, 128, 256]            # grid sides: m = n = side^2
TILES = [16, 32, 64, 128, 256]
WORKERS = [2, 4, 8, 12, 16]


def tuned(m: int, n: int, batched: bool = False, path: str = TUNING) -> dict:
    """Parameter overrides recorded by the autotuner for an m x n problem."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        t = json.load(f)
    out = {}
    entries = t.get("price_tile", {})
    if entries:
        key = min(entries, key=lambda k: abs(math.log(int(k.split("x")[0]) * int(k.split("x")[1]))
                                             - math.log(m * n)))
        out["price_tile"] = int(entries[key]["best"])
    if batched and "batch_workers" in t:
        out["batch_workers"] = int(t["batch_workers"]["best"])
    return out


def _grid(side):
    i = np.arange(side * side)
    return np.stack([i // side, i % side], 1).astype(np.int32)


def tune_price_tile(ctx, side: int, log):
    import torch
    import paper_2206_11009_amd as otip
    m = side * side
    xy = torch.as_tensor(_grid(side), device="cuda:0")
    rng = np.random.default_rng(side)
    # duals of an optimum's scale: a few reduced costs negative, most positive
    y = torch.as_tensor(rng.uniform(0.0, 0.02 * side * side, m), device="cuda:0")
    z = torch.as_tensor(rng.uniform(0.0, 0.02 * side * side, m), device="cuda:0")
    res = {}
    for tile in [0] + TILES:
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            otip.otip_price(ctx, xy, xy, y, z, None, m, otip.OTIP_FP64, tile=tile)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        res[str(tile)] = float(np.median(ts))
        log(f"price {side}x{side} tile {tile}: {1e3 * res[str(tile)]:.3f} ms")
    best = min((t for t in res if t != "0"), key=lambda t: res[t])
    return {"seconds": res, "best": int(best), "default_seconds": res["0"]}


def tune_batch_workers(ctx, log):
    import torch
    import paper_2206_11009_amd as otip
    sys.path.insert(0, os.path.dirname(HERE))
    from synthetic import batch_instances
    insts = batch_instances(512)
    dev = [[torch.as_tensor(x, device="cuda:0") for x in (i.a, i.b, i.xs, i.xt)] for i in insts]
    res = {}
    otip.otip_solve_batch(ctx, dev[:64], otip.params(batch_workers=16))   # warm buffers
    for w in WORKERS:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        otip.otip_solve_batch(ctx, dev, otip.params(batch_workers=w))
        torch.cuda.synchronize()
        res[str(w)] = time.perf_counter() - t0
        log(f"batch of 512 with {w} workers: {res[str(w)]:.2f} s")
    best = min(res, key=lambda k: res[k])
    return {"seconds": res, "best": int(best)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TUNING)
    ap.add_argument("--sides", default=",".join(str(s) for s in SIZES))
    ap.add_argument("--no-batch", action="store_true")
    args = ap.parse_args()
    import paper_2206_11009_amd as otip

    def log(msg):
        print(msg, flush=True)

    ctx = otip.Context(0)
    out = {"device": "MI355X (gfx950)", "price_tile": {}}
    for side in [int(s) for s in args.sides.split(",")]:
        out["price_tile"][f"{side * side}x{side * side}"] = tune_price_tile(ctx, side, log)
    if not args.no_batch:
        out["batch_workers"] = tune_batch_workers(ctx, log)
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    log(f"wrote {args.out}")


if __name__ == "__main__":
    main()
