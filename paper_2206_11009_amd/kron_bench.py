"""Bandwidth of the dense Kronecker products on an m x n FP64 array.

    python -m paper_2206_11009_amd.kron_bench [--m 16384] [--n 16384] [--reps 20]

A x (row and column sums of X: one read of 8 m n bytes) and A^T [y; z]
(X_ij = y_i + z_j: one write of 8 m n bytes), each call synchronised.  Prints
one JSON line with seconds per call and algorithmic GB/s for both.
"""
from __future__ import annotations

import argparse
import json
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--m", type=int, default=16384)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args()
    import torch
    import paper_2206_11009_amd as otip

    m, n = args.m, args.n
    ctx = otip.Context(0)
    g = torch.Generator(device="cuda:0").manual_seed(0)
    X = torch.rand((n, m), dtype=torch.float64, device="cuda:0", generator=g)  # vec(X) contiguous
    rs = torch.empty(m, dtype=torch.float64, device="cuda:0")
    cs = torch.empty(n, dtype=torch.float64, device="cuda:0")
    y = torch.rand(m, dtype=torch.float64, device="cuda:0", generator=g)
    z = torch.rand(n, dtype=torch.float64, device="cuda:0", generator=g)
    out = {"m": m, "n": n, "bytes": 8.0 * m * n}
    for name, fn in [("A_x", lambda: otip.otip_kron_apply(ctx, X, rs, cs)),
                     ("AT_yz", lambda: otip.otip_kron_apply_t(ctx, y, z, X))]:
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.reps):
            fn()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / args.reps
        out[name] = {"s_per_call": sec, "gb_per_s": 8.0 * m * n / sec / 1e9,
                     "frac_of_8000": 8.0 * m * n / sec / 1e9 / 8000.0}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
