"""Write the oracle's results on the synthetic workloads to tests/golden/.

Calls only the CPU oracle (``oracle.solve``) on the seeded instances of
``synthetic``; the GPU tests compare the HIP library with these stored values
at sizes where running the oracle inside a test would take minutes.

    python tests/golden/make_golden.py c1 c2
    python tests/golden/make_golden.py c2:costs

A name ``cfg:costs`` writes ``oracle_cfg_costs.json``: every seed of the workload
under each norm cost of Section 5.1 (1-, 2- and inf-norm, cost kinds 1-3).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synthetic import CONFIGS, config_instance  # noqa: E402


def costs(cfg):
    out = os.path.join(HERE, f"oracle_{cfg}_costs.json")
    rows = []
    for k in range(CONFIGS[cfg]["seeds"]):
        inst = config_instance(cfg, k)
        for kind in (1, 2, 3):
            t = time.perf_counter()
            r = oracle.solve(inst.a, inst.b, inst.xs, inst.xt,
                             oracle.OracleParams(cost_kind=kind))
            rows.append(dict(seed=k, cost_kind=kind, m=inst.m, n=inst.n, status=r.status,
                             objective=r.objective, dual_bound=r.dual_bound, rel_gap=r.rel_gap,
                             marginal_residual=r.marginal_residual, nnz=int(len(r.flows)),
                             iterations=r.iterations, seconds=time.perf_counter() - t))
            print(cfg, rows[-1], flush=True)
    with open(out, "w") as f:
        json.dump({"config": cfg, "generator": "synthetic.config_instance",
                   "solver": "oracle.solve (OracleParams(cost_kind=k))", "results": rows}, f,
                  indent=1)


def main(cfgs):
    for cfg in cfgs:
        if cfg.endswith(":costs"):
            costs(cfg.split(":")[0])
            continue
        out = os.path.join(HERE, f"oracle_{cfg}.json")
        rows = []
        for k in range(CONFIGS[cfg]["seeds"]):
            inst = config_instance(cfg, k)
            t = time.perf_counter()
            r = oracle.solve(inst.a, inst.b, inst.xs, inst.xt)
            rows.append(dict(seed=k, m=inst.m, n=inst.n, status=r.status, objective=r.objective,
                             dual_bound=r.dual_bound, rel_gap=r.rel_gap,
                             marginal_residual=r.marginal_residual, nnz=int(len(r.flows)),
                             iterations=r.iterations, cg_iterations=r.cg_iterations,
                             direct_iterations=r.direct_iterations,
                             seconds=time.perf_counter() - t))
            print(cfg, rows[-1], flush=True)
        with open(out, "w") as f:
            json.dump({"config": cfg, "generator": "synthetic.config_instance",
                       "solver": "oracle.solve (default OracleParams)", "results": rows}, f,
                      indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2"])
