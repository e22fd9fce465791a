"""Train the warm-start network on optimal duals of 32 x 32 grid problems.

    python -m paper_2206_11009_amd.ws_train --count 20000 --out DIR

Data: `count` pairs of Gaussian-mixture histograms on a 32 x 32 grid (1 to 5
bumps, the seeded generator of ``synthetic.batch_instances`` at indices
1,000,000 and up, disjoint from every evaluation family), each solved to a
certified relative gap of 1e-6 by the plain GPU method (otip_solve_batch).
Input: the two marginals times 32^2 (densities).  Target: the optimal duals in
the gauge mean(y) = mean(z), divided by 32^2 (normalised coordinates).
Training: Adam on the mean-squared error, with the library's own forward and
backward kernels (otip_ws_grad, otip_ws_adam); 5% of the data is held out.
Writes DIR/ws_weights.bin (FP32 parameters, the layout of otip_ws_param_count)
and DIR/ws_weights.json (recipe and losses).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SIDE = 32
FIRST = 1_000_000
LAYERS = [(2, 32), (32, 32), (32, 32), (32, 2)]


def he_uniform(seed: int) -> np.ndarray:
    """He-uniform weights (fan-in 9 * in channels), zero biases, in the flat
    layout W[out][in][3][3], b[out] per layer."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in LAYERS:
        lim = math.sqrt(6.0 / (9 * ci))
        parts.append(rng.uniform(-lim, lim, co * ci * 9))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def solve_duals(ctx, first: int, count: int, chunk: int, workers: int, log, budget=None):
    """Inputs (count, 2, 32, 32) and targets of the training instances; stops
    after the chunk that exceeds `budget` seconds and returns what it has."""
    import torch
    import paper_2206_11009_amd as otip
    from synthetic import batch_instances
    X = np.empty((count, 2, SIDE, SIDE), np.float32)
    T = np.empty((count, 2, SIDE, SIDE), np.float32)
    prm = otip.params(batch_workers=workers)
    keep = np.zeros(count, bool)
    t0 = time.perf_counter()
    for c0 in range(0, count, chunk):
        cn = min(chunk, count - c0)
        insts = batch_instances(cn, side_range=(SIDE, SIDE), first=first + c0)
        probs = [[torch.as_tensor(v, device=f"cuda:{ctx.device}") for v in (i.a, i.b, i.xs, i.xt)]
                 for i in insts]
        res = otip.otip_solve_batch(ctx, probs, prm)
        for q, (inst, r) in enumerate(zip(insts, res)):
            if not (r.status == otip.OTIP_OK and r.rel_gap <= 1e-6 and
                    r.marginal_residual <= 1e-8):
                log(f"training instance {first + c0 + q} not certified, left out: {r.info}")
                continue
            keep[c0 + q] = True
            shift = 0.5 * (r.z.mean() - r.y.mean())
            X[c0 + q, 0] = (inst.a * SIDE * SIDE).reshape(SIDE, SIDE)
            X[c0 + q, 1] = (inst.b * SIDE * SIDE).reshape(SIDE, SIDE)
            T[c0 + q, 0] = ((r.y + shift) / (SIDE * SIDE)).reshape(SIDE, SIDE)
            T[c0 + q, 1] = ((r.z - shift) / (SIDE * SIDE)).reshape(SIDE, SIDE)
        el = time.perf_counter() - t0
        log(f"solved {c0 + cn}/{count} training problems, {el:.0f} s "
            f"({(c0 + cn) / el:.1f}/s)")
        if budget is not None and el > budget and c0 + cn < count:
            log(f"time budget reached after the first {c0 + cn} problems")
            break
    return X[keep], T[keep]


def train(ctx, X, T, epochs: int, batch: int, lr: float, seed: int, log):
    import torch
    import paper_2206_11009_amd as otip
    dev = f"cuda:{ctx.device}"
    n = X.shape[0]
    nval = max(1, n // 20)
    Xd = torch.as_tensor(X, device=dev)
    Td = torch.as_tensor(T, device=dev)
    Xtr, Ttr, Xva, Tva = Xd[nval:], Td[nval:], Xd[:nval], Td[:nval]
    w = torch.as_tensor(he_uniform(seed), device=dev)
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    g = torch.empty_like(w)
    rng = np.random.default_rng(seed)
    steps_per_epoch = max(1, (n - nval) // batch)
    total = epochs * steps_per_epoch
    step = 0
    hist = []

    def val_loss():
        tot = 0.0
        for s in range(0, nval, 512):
            out = otip.otip_ws_forward(ctx, w, Xva[s:s + 512])
            tot += float(((out - Tva[s:s + 512]) ** 2).sum())
        return tot / (nval * 2 * SIDE * SIDE)

    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(n - nval), device=dev)
        run = 0.0
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            step += 1
            lr_t = 1e-2 * lr + (lr - 1e-2 * lr) * 0.5 * (1 + math.cos(math.pi * step / total))
            loss, _ = otip.otip_ws_grad(ctx, w, Xtr[idx], Ttr[idx], g)
            otip.otip_ws_adam(ctx, w, m, v, g, step, lr_t)
            run += loss
        vl = val_loss()
        hist.append({"epoch": ep + 1, "train_mse": run / steps_per_epoch, "val_mse": vl})
        log(f"epoch {ep + 1}/{epochs}: train mse {run / steps_per_epoch:.3e}, val mse {vl:.3e}")
    return w.cpu().numpy(), hist, nval


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--chunk", type=int, default=1024)
    ap.add_argument("--out", default=os.path.dirname(os.path.abspath(__file__)))
    ap.add_argument("--budget", type=float, default=None,
                    help="seconds of solving after which the data set is cut")
    args = ap.parse_args()
    import paper_2206_11009_amd as otip

    def log(msg):
        print(msg, flush=True)

    ctx = otip.Context(0)
    t0 = time.perf_counter()
    X, T = solve_duals(ctx, FIRST, args.count, args.chunk, args.workers, log, args.budget)
    t1 = time.perf_counter()
    w, hist, nval = train(ctx, X, T, args.epochs, args.batch, args.lr, args.seed, log)
    t2 = time.perf_counter()
    os.makedirs(args.out, exist_ok=True)
    w.astype("<f4").tofile(os.path.join(args.out, "ws_weights.bin"))
    meta = {"grid": SIDE, "training_problems": int(X.shape[0]), "first_index": FIRST,
            "held_out": nval, "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
            "seed": args.seed, "params": int(w.size), "solve_seconds": t1 - t0,
            "train_seconds": t2 - t1, "history": hist,
            "recipe": "synthetic.batch_instances(count, side_range=(32, 32), first=1000000); "
                      "plain otip_solve_batch to rel gap 1e-6; target (y + s, z - s) / 32^2 "
                      "with s = (mean z - mean y) / 2; input (a, b) * 32^2"}
    with open(os.path.join(args.out, "ws_weights.json"), "w") as f:
        json.dump(meta, f, indent=1)
    log(f"wrote {args.out}/ws_weights.bin ({w.size} parameters)")


if __name__ == "__main__":
    main()
