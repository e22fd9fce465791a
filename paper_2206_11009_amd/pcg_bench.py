"""Bandwidth of the Newton step's CG iteration (one launch: Schur SpMV with the
vector updates) at large n.

    python -m paper_2206_11009_amd.pcg_bench [--side 256] [--kappa 10]
        [--pattern random|local] [--maxit 200] [--precision 0|1]

Builds the Schur complement S_M = N - V^T M^-1 V (Section 4) of a synthetic
support on a side x side grid pair (m = n = side^2) with the library's own
assembly, then runs the library's Jacobi-PCG on S_M for at most maxit
iterations.  The support has about 2 kappa entries per source row (kappa (m +
n - 1) in all, the size of the initial support of Section 3.2 at factor
kappa): "random" draws each row's targets uniformly (nnz(S_M) close to the sum
of squared row degrees, the largest pattern for that support size), "local"
takes the targets nearest to the source pixel (a banded pattern like the
cost-driven supports of the method).  theta is log-uniform over 10^[-3, 3].
Prints one JSON line: sizes, the iteration launches that did work, their mean
duration from events recorded at the dispatches themselves, and the
algorithmic GB/s ((w + 4) nnz + (4 + 12 w) n bytes per launch) against the 8
TB/s HBM peak.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def support(side: int, kappa: float, pattern: str, seed: int) -> np.ndarray:
    m = n = side * side
    per_row = max(1, int(round(kappa * (m + n - 1) / m)))
    rng = np.random.default_rng(seed)
    if pattern == "random":
        cols = rng.integers(0, n, (m, per_row))
    else:
        # the per_row offsets of smallest length (ties by angle order of the
        # scan below), clipped to the grid
        rad = int(np.ceil(np.sqrt(per_row))) + 1
        offs = [(dx, dy) for dx in range(-rad, rad + 1) for dy in range(-rad, rad + 1)]
        offs.sort(key=lambda o: (o[0] * o[0] + o[1] * o[1], o))
        offs = np.array(offs[:per_row])
        i = np.arange(m)
        r, c = i // side, i % side
        rr = np.clip(r[:, None] + offs[None, :, 0], 0, side - 1)
        cc = np.clip(c[:, None] + offs[None, :, 1], 0, side - 1)
        cols = rr * side + cc
    rows = np.repeat(np.arange(m), cols.shape[1])
    rows = np.concatenate([rows, np.arange(n) % m])       # every column covered
    cols = np.concatenate([cols.reshape(-1), np.arange(n)])
    return np.unique(rows.astype(np.int64) + cols.astype(np.int64) * m)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--side", type=int, default=256)
    ap.add_argument("--kappa", type=float, default=10.0)
    ap.add_argument("--pattern", choices=["random", "local"], default="random")
    ap.add_argument("--maxit", type=int, default=200)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    import torch
    import paper_2206_11009_amd as otip

    m = n = args.side * args.side
    t0 = time.perf_counter()
    idx = support(args.side, args.kappa, args.pattern, args.seed)
    rng = np.random.default_rng(args.seed + 1)
    theta = 10.0 ** rng.uniform(-3.0, 3.0, idx.size)
    ctx = otip.Context(0)
    rp, ci, va, _, _ = otip.otip_schur(ctx, m, n, idx, theta)
    b = torch.as_tensor(rng.standard_normal(n), device="cuda:0")
    b -= b.mean()                        # the range of S_M (connected support)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    print(f"setup {t_setup:.1f} s: psi {idx.size} nnz(S) {int(va.shape[0])}", flush=True)
    otip.otip_pcg(ctx, rp, ci, va, b, rtol=1e-6, maxit=4, precision=args.precision)  # warm-up
    t0 = time.perf_counter()
    x, res = otip.otip_pcg(ctx, rp, ci, va, b, rtol=1e-12, maxit=args.maxit,
                           precision=args.precision)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gbs = res.spmv_bytes / res.spmv_seconds / 1e9 if res.spmv_seconds > 0 else 0.0
    print(json.dumps({"side": args.side, "m": m, "n": n, "kappa": args.kappa,
                      "pattern": args.pattern, "precision": args.precision, "psi": int(idx.size),
                      "nnz": int(va.shape[0]), "iterations": res.iterations,
                      "spmv_launches": res.spmv_launches, "spmv_us": res.spmv_seconds * 1e6,
                      "bytes_per_launch": res.spmv_bytes, "gb_per_s": gbs,
                      "frac_of_8000": gbs / 8000.0, "pcg_wall_s": wall}), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
