"""Whole solves through the C-ABI against the CPU oracle and exact optima."""
import numpy as np
import pytest

import oracle
from synthetic import config_instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2206_11009_amd as otip
    c = otip.Context(0)
    yield c
    c.close()


def check_result(res, a, b, xs, xt):
    m, n = len(a), len(b)
    assert res.status == 0, res.info
    assert res.marginal_residual <= 1e-8
    assert res.rel_gap <= 1e-6
    assert len(res.flows) <= m + n - 1
    assert oracle.is_forest(res.rows, res.cols, m, n)
    # the reported numbers are those of the returned plan and duals
    c = oracle.sq_costs(xs, xt, res.rows, res.cols)
    assert abs(float((c * res.flows).sum()) - res.objective) <= 1e-12 * max(1, abs(res.objective))
    rmin, _ = oracle._cscan.rmin(xs, xt, res.y, res.z)
    assert rmin == pytest.approx(res.r_min, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("k", range(10))
def test_gaussian_16x16_matches_oracle(ctx, k):
    import paper_2206_11009_amd as otip
    inst = config_instance("c1", k)
    res = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt)
    ref = oracle.solve(inst.a, inst.b, inst.xs, inst.xt)
    check_result(res, inst.a, inst.b, inst.xs, inst.xt)
    assert abs(res.objective - ref.objective) <= 1e-6 * abs(ref.objective)


def test_uniform_vs_enumeration(ctx):
    import itertools
    import paper_2206_11009_amd as otip
    rng = np.random.default_rng(107)
    n = 7
    xs = rng.integers(0, 10, (n, 2)).astype(np.int32)
    xt = rng.integers(0, 10, (n, 2)).astype(np.int32)
    C = ((xs[:, None, :].astype(int) - xt[None, :, :]) ** 2).sum(-1)
    best = min(sum(C[i, s[i]] for i in range(n)) for s in itertools.permutations(range(n)))
    a = np.full(n, 1.0 / n)
    res = otip.otip_solve(ctx, a, a.copy(), xs, xt)
    assert abs(res.objective - best / n) <= 1e-9 * max(1.0, best / n)
    check_result(res, a, a, xs, xt)


@pytest.mark.parametrize("mode", ["paper_switch", "direct_only"])
@pytest.mark.parametrize("k", [0, 3, 6])
def test_solver_modes_16x16(ctx, k, mode):
    """The CG -> LDL^T switch by the support-drop rule alone (Section 4.3), and
    the direct solver throughout, reach the same certified optimum."""
    import paper_2206_11009_amd as otip
    inst = config_instance("c1", k)
    if mode == "paper_switch":
        prm = otip.params(switch_cost=0)
    else:
        prm = otip.params(linear_solver=otip.OTIP_LS_DIRECT)
    res = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt, prm)
    check_result(res, inst.a, inst.b, inst.xs, inst.xt)
    if mode == "paper_switch":
        assert res.cg_iterations > 0
    golden = {r["seed"]: r for r in load_golden("c1")}
    ref = golden[k]["objective"]
    assert abs(res.objective - ref) <= 1e-6 * abs(ref)


def load_golden(cfg):
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"oracle_{cfg}.json")
    with open(path) as f:
        return json.load(f)["results"]


@pytest.mark.parametrize("k", range(5))
def test_gaussian_64x64_matches_stored_oracle(ctx, k):
    """64x64 grids (16.8M variables): objective within 1e-6 of the oracle's
    stored optimum, certified gap and marginals, basic plan."""
    import paper_2206_11009_amd as otip
    inst = config_instance("c2", k)
    res = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt)
    check_result(res, inst.a, inst.b, inst.xs, inst.xt)
    ref = {r["seed"]: r for r in load_golden("c2")}[k]["objective"]
    assert abs(res.objective - ref) <= 1e-6 * abs(ref)


@pytest.mark.parametrize("k,precision", [(0, "mixed"), (1, "mixed"), (2, "mixed"), (0, "fp64")])
def test_white_noise_128x128_matches_stored_oracle(ctx, k, precision):
    """128x128 white-noise grids (268M variables), the mixed-precision form of
    the workload (FP32 pricing with the FP64 re-check, FP32 CG inside FP64
    refinement) and FP64: objective within 1e-6 of the FP64 oracle's stored
    optimum (its relative error printed), certified gap and marginals."""
    import paper_2206_11009_amd as otip
    inst = config_instance("c3", k)
    prec = otip.OTIP_MIXED if precision == "mixed" else otip.OTIP_FP64
    res = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt, otip.params(precision=prec))
    check_result(res, inst.a, inst.b, inst.xs, inst.xt)
    ref = {r["seed"]: r for r in load_golden("c3")}[k]["objective"]
    err = abs(res.objective - ref) / abs(ref)
    print(f"c3 seed {k} {precision}: objective {res.objective!r}, oracle {ref!r}, "
          f"relative error {err:.2e}, {res.iterations} iterations, {res.seconds_total:.2f} s")
    assert err <= 1e-6


@pytest.mark.parametrize("cfg,k", [("c1", 0), ("c1", 5), ("c2", 2)])
def test_mixed_precision_solve(ctx, cfg, k):
    """FP32 pricing with FP64 re-check and FP32 CG inside FP64 refinement reach
    the oracle's optimum with an FP64 certificate."""
    import paper_2206_11009_amd as otip
    inst = config_instance(cfg, k)
    res = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt,
                          otip.params(precision=otip.OTIP_MIXED, switch_cost=0))
    check_result(res, inst.a, inst.b, inst.xs, inst.xt)
    ref = {r["seed"]: r for r in load_golden(cfg)}[k]["objective"]
    assert abs(res.objective - ref) <= 1e-6 * abs(ref)


def test_profile_counts_dense_factor_launches(ctx):
    """With profiling on, every dense factorisation of the 256 x 256 Schur
    complement times its 4 diagonal-block launches and 3 trailing updates (one
    group of three panels: the second block's column after the first panel,
    the third block's column after the first two, the last block after all
    three).  The diagonal blocks' flops are the stated formula; the updates'
    are those of the rows the panels reach, so at most the full triangles'."""
    import paper_2206_11009_amd as otip
    inst = config_instance("c1", 1)
    res = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt, otip.params(profile=1))
    check_result(res, inst.a, inst.b, inst.xs, inst.xt)
    nd, nu = res.diag_launches, res.update_launches
    assert nd > 0 and nd % 4 == 0 and nu == 3 * nd // 4
    factorisations = nd // 4

    def first_col(panels, rows):   # a 64-wide block column of `rows` rows
        return 2.0 * panels * 64 * (64 * (rows - 64) + 64 * 65 / 2.0)

    assert res.diag_flops == pytest.approx(nd * 2.0 * 64 ** 3 / 3.0, rel=1e-12)
    per_factorisation = first_col(1, 192) + first_col(2, 128) + 64 ** 2 * 3 * 64
    assert 0.0 < res.update_flops <= factorisations * per_factorisation * (1 + 1e-12)
    assert res.diag_ms > 0.0 and res.update_ms > 0.0
    plain = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt)
    assert plain.diag_launches == 0
    assert plain.objective == pytest.approx(res.objective, rel=1e-9)
