"""Throughput of the full pricing scan (reduced costs of every variable, cost
generated on the fly, selection of the m most negative).

    python -m paper_2206_11009_amd.price_bench [--side 256] [--reps 10] [--precision fp64]

Grid pair side x side (m = n = side^2 variables per side, side^4 in all),
duals of the scale of an optimum (uniform in [0, 0.02 side^2], so that a few
percent of the reduced costs are negative), empty support, kmax = m.  Between
calls the duals move by a random step of `--perturb` times their range (an
outer iteration's change), so that each call's cutoff, guessed from the
previous call's selection, is tested as in a solve.  Prints one JSON line:
seconds per scan and reduced costs per second.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--side", type=int, default=256)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--perturb", type=float, default=0.01)
    args = ap.parse_args()
    import torch
    import paper_2206_11009_amd as otip

    side = args.side
    m = side * side
    i = np.arange(m)
    xy = torch.as_tensor(np.stack([i // side, i % side], 1).astype(np.int32), device="cuda:0")
    rng = np.random.default_rng(side)
    span = 0.02 * m
    ys = [torch.as_tensor(rng.uniform(0.0, span, m), device="cuda:0")]
    zs = [torch.as_tensor(rng.uniform(0.0, span, m), device="cuda:0")]
    for _ in range(args.reps):   # the duals of the next calls, prepared before timing
        ys.append(ys[-1] + torch.as_tensor(rng.uniform(-1, 1, m) * args.perturb * span,
                                           device="cuda:0"))
        zs.append(zs[-1] + torch.as_tensor(rng.uniform(-1, 1, m) * args.perturb * span,
                                           device="cuda:0"))
    prec = otip.OTIP_MIXED if args.precision == "mixed" else otip.OTIP_FP64
    ctx = otip.Context(0)
    otip.otip_price(ctx, xy, xy, ys[0], zs[0], None, m, prec, tile=args.tile)     # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(args.reps):
        _, _, _, nneg = otip.otip_price(ctx, xy, xy, ys[r + 1], zs[r + 1], None, m, prec,
                                        tile=args.tile)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.reps
    print(json.dumps({"side": side, "variables": m * m, "precision": args.precision,
                      "s_per_scan": sec, "gcosts_per_s": m * m / sec / 1e9,
                      "negative": nneg, "reps": args.reps, "perturb": args.perturb}),
          flush=True)


if __name__ == "__main__":
    main()
