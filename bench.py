#!/usr/bin/env python
"""Benchmark of the interior-point-inspired column-generation OT solver on one
MI355X.

A step is one complete solve of one Kantorovich LP to a certified relative
duality gap <= 1e-6 (initial support, every Newton step and pricing scan, the
CG -> LDL^T switch, purification and the final full-scan certificate).  The
default workload is the 128 x 128 white-noise grid pair family (m = n = 16384,
268M variables, squared-Euclidean cost generated on the fly), the largest
configuration whose solves fit many timed steps in a few minutes; step k
solves seed k mod 3, in FP64 (the headline) and in the mixed-precision form
with the learned start.  The 256 x 256 pair (4.29e9 variables) takes minutes
per solve: run it with --config c5 --steps 1 --warmup 0.  Inputs are uploaded
to HBM before the timed region.

Prints one JSON line: seconds per LP (lower is better) of the plain FP64
method, the live roofline of the dominant kernel (HIP events recorded by each of
its dispatches; the timed kernels are the Schur SpMV, the pricing pass and the
dense factor's diagonal-block and trailing-update kernels, and the one with the
largest total time is reported, the others beside it), pricing throughput, the same instances solved by the
mixed-precision and learned-warm-start forms ("forms"; the network's prediction
is inside the timed region), the same instances under the 1-, 2- and inf-norm
costs of the paper's experiments ("norm_costs"), and the CPU oracle timed on a
bounded sample of the same workload.  --config c4 times whole batches of 512 uneven instances
(otip_solve_batch) and reports seconds per LP of the batch.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# HBM traffic per launch of a kernel on a workload, measured by rocprofv3
# --pmc FETCH_SIZE and WRITE_SIZE (separate runs) on `bench.py --config <cfg>
# --steps 1 --warmup 0 --no-cpu-baseline --no-forms`, scaled by what the
# counters read for a 1 GiB device copy, mean over the launches that did work;
# valid only for the kernel source it was measured on (the SHA-256 of the text
# of the listed functions).
KERNEL_TRAFFIC = {
    ("cg_step", "c3"): {"source": "paper_2206_11009_amd/csrc/schur.hip",
                        "functions": ["load_chunk", "cg_step"],
                        "sha256": "aa72e5b796946081a1d66dd41743c0e67e6194fce9b3ef43a634c6e26ff597de",
                        "bytes_per_launch": 10995319.7},
    ("ldl_update", "c3"): {"source": "paper_2206_11009_amd/csrc/dense.hip",
                           "functions": ["ldl_update"],
                           "sha256": "1bcb344e821bde84dfe7c46499b80875ff4f1e928d8e6c6f328d7bc88c1d6eac",
                           "bytes_per_launch": 4408930.8},
    ("ldl_diag", "c3"): {"source": "paper_2206_11009_amd/csrc/dense.hip",
                         "functions": ["ldl_diag"],
                         "sha256": "96f87f3041ccc01070127ff805ed6ea8d5ef17cb834cb68c4b02db230b83934c",
                         "bytes_per_launch": 102391.1},
}
FP64_VECTOR_PEAK_TF = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
FP64_MATRIX_PEAK_TF = 78.6     # dense FP64 matrix-core peak
PRICE_FLOPS_PER_COST = 7.0     # C_ij: one add + two FMAs (5 flops); r: two subtractions
WORKLOADS = {
    "c1": "16x16 Gaussian-mixture grid pair (m=n=256, 65,536 variables), 3 bumps, FP64",
    "c2": "64x64 Gaussian-mixture grid pair (m=n=4096, 16.8M variables), 5 bumps, FP64",
    "c3": "128x128 white-noise grid pair (m=n=16384, 268M variables)",
    "c4": "512 Gaussian-mixture grid pairs of side U{8..32} (1-5 bumps), batched",
    "c5": "256x256 Cauchy-bump grid pair (m=n=65536, 4.29e9 variables)",
}


def baseline_metric():
    with open(os.path.join(ROOT, "BASELINE.json")) as f:
        return json.load(f)["metric"]


def cpu_baseline(cfg, budget_s=20.0, fallback_its=None):
    """Time the CPU oracle on seed 0 of the workload for about budget_s seconds
    of outer iterations, then scale the mean time per outer iteration by the
    number of outer iterations the oracle needs for the whole solve (stored by
    tests/golden/make_golden.py)."""
    import oracle
    from synthetic import config_instance

    class Stop(Exception):
        pass

    inst = config_instance(cfg, 0)
    t0 = time.perf_counter()
    c0 = time.process_time()   # CPU time of all the process's threads
    marks = []

    def log(rec):
        marks.append(time.perf_counter())
        if time.perf_counter() - t0 > budget_s:
            raise Stop

    try:
        oracle.solve(inst.a, inst.b, inst.xs, inst.xt, log=log)
        done = True
    except Stop:
        done = False
    wall = time.perf_counter() - t0
    # the cores the oracle kept busy (its C scan and scipy's sparse kernels are
    # single-threaded; numpy's BLAS calls may use more)
    cores = max(1, int(round((time.process_time() - c0) / max(wall, 1e-9))))
    elapsed = (marks[-1] if marks else time.perf_counter()) - t0
    its = len(marks)
    golden = os.path.join(ROOT, "tests", "golden", f"oracle_{cfg}.json")
    full_its = None
    if os.path.exists(golden):
        with open(golden) as f:
            full_its = json.load(f)["results"][0]["iterations"]
    if full_its is None and not done:
        full_its = int(round(fallback_its or its))
    if done:
        value = elapsed
        how = f"complete oracle solve of seed 0 ({its} outer iterations)"
    else:
        value = elapsed / its * full_its
        how = (f"first {its} outer iterations of the seed-0 oracle solve ({elapsed:.1f} s), "
               f"mean time per iteration x {full_its} iterations of the oracle's full solve")
    return {"value": value, "unit": "s per LP (estimated)" if not done else "s per LP",
            "cores": cores, "kind": "oracle", "sample": how}


def upload(insts):
    import torch
    return [[torch.as_tensor(x, device="cuda:0") for x in (i.a, i.b, i.xs, i.xt)] for i in insts]


def side_of(inst):
    side = int(round(inst.m ** 0.5))
    return side if side * side == inst.m == inst.n else None


def progress(msg):
    """One line on stderr per finished solve (a long run keeps reporting)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def run_single(ctx, dev, insts, prm, weights, steps, warmup, cost_kind=0, label=""):
    """Seconds per LP over `steps` solves (after `warmup`), with the learned
    prediction (inside the timed region) when weights are given."""
    import torch
    import paper_2206_11009_amd as otip

    def one(k):
        a, b, xs, xt = dev[k]
        if weights is None:
            r = otip.otip_solve(ctx, a, b, xs, xt, prm, cost_kind=cost_kind)
        else:
            y0, z0 = otip.otip_ws_predict(ctx, weights, side_of(insts[k]), a, b)
            r = otip.otip_solve(ctx, a, b, xs, xt, prm, y0=y0, z0=z0, cost_kind=cost_kind)
        progress(f"{label} solve {k + 1}/{warmup + steps}: {r.seconds_total:.3f} s, "
                 f"{r.iterations} iterations, gap {r.rel_gap:.1e}")
        return r

    for k in range(warmup):
        one(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [one(warmup + k).info for k in range(steps)]
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, infos


def run_batch(ctx, dev, insts, prm, weights, steps, warmup):
    """Seconds per LP of whole-batch solves (otip_solve_batch)."""
    import torch
    import paper_2206_11009_amd as otip

    def one():
        if weights is None:
            return otip.otip_solve_batch(ctx, dev, prm)
        probs = []
        for (a, b, xs, xt), inst in zip(dev, insts):
            y0, z0 = otip.otip_ws_predict(ctx, weights, side_of(inst), a, b)
            probs.append((a, b, xs, xt, y0, z0))
        return otip.otip_solve_batch(ctx, probs, prm)

    for q in range(warmup):
        one()
        progress(f"batch {q + 1}/{warmup + steps}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for q in range(steps):
        infos += [r.info for r in one()]
        progress(f"batch {warmup + q + 1}/{warmup + steps}")
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / (steps * len(dev)), infos


def summary(sec, infos):
    n = len(infos)
    return {"s_per_lp": sec,
            "iterations_mean": sum(i["iterations"] for i in infos) / n,
            "cg_iterations_mean": sum(i["cg_iterations"] for i in infos) / n,
            "direct_iterations_mean": sum(i["direct_iterations"] for i in infos) / n,
            "rel_gap_max": max(i["rel_gap"] for i in infos),
            "certified": all(i["rel_gap"] <= 1e-6 and i["marginal_residual"] <= 1e-8
                             for i in infos)}


def kernel_source_sha256(path, names):
    """SHA-256 of the source text of the named functions (each from its
    signature to the first line that closes a top-level block), in order."""
    import hashlib
    with open(os.path.join(ROOT, path)) as f:
        src = f.read()
    h = hashlib.sha256()
    for name in names:
        start = src.find(f"void {name}(")
        if start < 0:
            return None
        end = src.find("\n}\n", start)
        h.update(src[start:end + 3].encode())
    return h.hexdigest()


def measured_traffic(kernel, cfg):
    """Counter-measured bytes per launch of a kernel on a workload, or None
    when none were taken or once its source differs from the one the counters
    were taken on."""
    t = KERNEL_TRAFFIC.get((kernel, cfg))
    if t is None or t["sha256"] is None:
        return None
    if kernel_source_sha256(t["source"], t["functions"]) != t["sha256"]:
        return None
    return t["bytes_per_launch"]


def rooflines(infos, cfg):
    spmv_ms = sum(i["spmv_ms"] for i in infos)
    spmv_n = sum(i["spmv_launches"] for i in infos)
    spmv_b = sum(i["spmv_bytes"] for i in infos)
    pr_ms = sum(i["price_ms"] for i in infos)
    pr_n = sum(i["price_launches"] for i in infos)
    pr_e = sum(i["price_elems"] for i in infos)
    spmv = {"bound": "hbm", "kernel": "CG iteration (cg_step: Schur SpMV with the vector updates "
            "and a single reduction; spmv_dir + cg_update for a Schur matrix beyond 96 MB)",
            "achieved": spmv_b / max(spmv_ms, 1e-12) / 1e6, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "avg_launch_us": 1e3 * spmv_ms / max(spmv_n, 1), "launches": spmv_n,
            "total_ms": spmv_ms, "traffic": measured_traffic("cg_step", cfg),
            "algorithmic_bytes_per_launch": spmv_b / max(spmv_n, 1)}
    price = {"bound": "alu", "kernel": "price_pass (pricing scan)",
             "achieved": PRICE_FLOPS_PER_COST * pr_e / max(pr_ms, 1e-12) / 1e9,
             "peak": FP64_VECTOR_PEAK_TF, "unit": "TFLOP/s",
             "avg_launch_us": 1e3 * pr_ms / max(pr_n, 1), "launches": pr_n, "total_ms": pr_ms,
             "traffic": None}
    dg_ms = sum(i["diag_ms"] for i in infos)
    dg_n = sum(i["diag_launches"] for i in infos)
    dg_f = sum(i["diag_flops"] for i in infos)
    up_ms = sum(i["update_ms"] for i in infos)
    up_n = sum(i["update_launches"] for i in infos)
    up_f = sum(i["update_flops"] for i in infos)
    diag = {"bound": "alu", "kernel": "ldl_diag (64x64 diagonal-block LDL^T and inverse of its "
            "unit lower factor, four wavefronts)",
            "achieved": dg_f / max(dg_ms, 1e-12) / 1e9, "peak": FP64_VECTOR_PEAK_TF,
            "unit": "TFLOP/s", "avg_launch_us": 1e3 * dg_ms / max(dg_n, 1), "launches": dg_n,
            "total_ms": dg_ms, "traffic": measured_traffic("ldl_diag", cfg),
            "algorithmic_flops_per_launch": dg_f / max(dg_n, 1)}
    update = {"bound": "mfma", "kernel": "ldl_update (trailing update of the dense LDL^T)",
              "achieved": up_f / max(up_ms, 1e-12) / 1e9, "peak": FP64_MATRIX_PEAK_TF,
              "unit": "TFLOP/s", "avg_launch_us": 1e3 * up_ms / max(up_n, 1), "launches": up_n,
              "total_ms": up_ms, "traffic": measured_traffic("ldl_update", cfg),
              "algorithmic_flops_per_launch": up_f / max(up_n, 1)}
    named = {"cg_step": spmv, "price_pass": price, "ldl_diag": diag, "ldl_update": update}
    for r in named.values():
        r["frac"] = r["achieved"] / r["peak"]
    top = max(named, key=lambda k: named[k]["total_ms"])
    other = {k: v for k, v in named.items() if k != top and v["launches"] > 0}
    return named[top], other, pr_e / max(pr_ms, 1e-12) / 1e6


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="precision of the headline (plain) measurement")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the mixed-precision and learned-warm-start forms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", action="store_true",
                    help="the library's per-iteration log on stderr (long solves)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures a single GPU; this build has no multi-GPU path "
              "(each LP solve runs on one MI355X).", file=sys.stderr)
        sys.exit(2)

    import paper_2206_11009_amd as otip
    from paper_2206_11009_amd.autotune import tuned
    from synthetic import CONFIGS, batch_instances, config_instance

    ctx = otip.Context(0)
    batched = args.config == "c4"
    if batched:
        insts = batch_instances(512)
        run = run_batch
    else:
        seeds = CONFIGS[args.config]["seeds"]
        insts = [config_instance(args.config, k % seeds) for k in range(args.warmup + args.steps)]
        run = run_single
    dev = upload(insts)
    prec = otip.OTIP_MIXED if args.precision == "mixed" else otip.OTIP_FP64
    tune = tuned(max(i.m for i in insts), max(i.n for i in insts), batched)
    if args.config == "c5":
        tune = dict(tune, max_iter=500)   # the iteration limit for this workload
    if args.verbose:
        tune = dict(tune, verbose=1)
    kw = {} if batched else {"label": f"{args.precision}_plain"}
    sec, infos = run(ctx, dev, insts, otip.params(profile=1, precision=prec, **tune), None,
                     args.steps, args.warmup, **kw)
    if not summary(sec, infos)["certified"]:
        raise SystemExit(f"solve not certified: {infos}")
    dominant, other, gcosts = rooflines(infos, args.config)

    forms = {f"{args.precision}_plain": summary(sec, infos)}
    weights = None
    if not args.no_forms and all(side_of(i) for i in insts) and os.path.exists(otip.WS_WEIGHTS):
        weights = otip.load_ws_weights(ctx)
        todo = [("mixed_plain", otip.OTIP_MIXED, None),
                (f"{args.precision}_learned", prec, weights),
                ("mixed_learned", otip.OTIP_MIXED, weights)]
        if args.config in ("c3", "c5"):
            # the metric's comparison (and, at 128 x 128, the mixed-precision
            # form alone): the whole run stays within a few minutes
            todo = [t for t in todo if t[0] == "mixed_learned" or
                    (args.config == "c3" and t[0] == "mixed_plain")]
        for name, p, w in todo:
            if name in forms:
                continue
            kw = {} if batched else {"label": name}
            s2, inf2 = run(ctx, dev, insts, otip.params(precision=p, **tune), w, args.steps,
                           args.warmup, **kw)
            forms[name] = summary(s2, inf2)
            forms[name]["speedup_vs_plain"] = sec / s2
    # the same problems under the costs of Section 5.1 (1-, 2- and inf-norm of
    # the pixel offset), plain FP64 method
    norm_costs = {}
    if not args.no_forms and not batched and args.config in ("c1", "c2"):
        for name, kind in (("l1", 1), ("l2", 2), ("linf", 3)):
            s3, inf3 = run_single(ctx, dev, insts,
                                  otip.params(precision=prec, max_iter=500, **tune), None,
                                  args.steps, args.warmup, cost_kind=kind, label=name)
            norm_costs[name] = summary(s3, inf3)

    out = {
        "metric": baseline_metric(),
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sec * (len(dev) if batched else 1),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config],
                   "instances": (f"512 per step" if batched else
                                 f"step k solves seed k mod {CONFIGS[args.config]['seeds']}"),
                   "certified_rel_gap": 1e-6, "precision": args.precision,
                   "form": "plain initial support",
                   "tuned": {k: v for k, v in tune.items() if k != "verbose"}},
        "roofline": dominant,
        "roofline_other": other,
        "pricing_gcosts_per_s": gcosts,
        "iterations_mean": forms[f"{args.precision}_plain"]["iterations_mean"],
        "cg_iterations_mean": forms[f"{args.precision}_plain"]["cg_iterations_mean"],
        "rel_gap_max": forms[f"{args.precision}_plain"]["rel_gap_max"],
        "forms": forms,
        "norm_costs": norm_costs,
    }
    if not args.no_cpu_baseline and not batched:
        progress("CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(args.config, fallback_its=out["iterations_mean"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
