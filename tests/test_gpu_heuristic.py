"""Heuristic pricing (Section 3.4), the return from the direct solver to CG
(remark of Section 4.3) and the Schur pattern kept across support updates
(remark of Section 4.2), through the C-ABI against the CPU oracle."""
import json
import os

import numpy as np
import pytest

import oracle
import oracle.ipm as I
from oracle import _cscan
from synthetic import config_instance, grid_coords

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def ctx():
    import paper_2206_11009_amd as otip
    c = otip.Context(0)
    yield c
    c.close()


def golden(cfg, k):
    with open(os.path.join(GOLDEN, f"oracle_{cfg}.json")) as f:
        return json.load(f)["results"][k]


def certified(res, inst):
    assert res.status == 0, res.info
    assert res.rel_gap <= 1e-6 and res.marginal_residual <= 1e-8
    assert len(res.flows) <= inst.m + inst.n - 1
    assert oracle.is_forest(res.rows, res.cols, inst.m, inst.n)


def bitmap_of(idx, mn):
    bm = np.zeros((mn + 31) // 32, np.uint32)
    np.bitwise_or.at(bm, (idx >> 5).astype(np.int64), (1 << (idx & 31)).astype(np.uint32))
    return bm.view(np.int32)


def grid_subset_size(side, L, kind):
    """|J| on a side x side grid pair, from the offsets: (side-|dx|)(side-|dy|)
    pairs per offset whose cost key is below L."""
    d = np.arange(-(side - 1), side)
    dx, dy = np.meshgrid(d, d, indexing="ij")
    if kind == 1:
        key = np.abs(dx) + np.abs(dy)
    elif kind == 3:
        key = np.maximum(np.abs(dx), np.abs(dy))
    else:
        key = dx * dx + dy * dy
    w = (side - np.abs(dx)) * (side - np.abs(dy))
    return int(w[key < L].sum())


@pytest.mark.parametrize("side,kind,radius", [(16, 0, 0.3), (64, 0, 0.1), (64, 1, 0.1),
                                              (64, 2, 0.15), (64, 3, 0.1), (128, 0, 0.05)])
def test_subset_pricing_is_bit_exact(ctx, side, kind, radius):
    """Pricing over J: the same selected columns, in the same (r, idx) order,
    the same reduced costs bit for bit and the same negative count as the
    oracle's scan restricted to J, on duals that make many reduced costs of J
    negative; |J| as counted from the grid's offsets."""
    import paper_2206_11009_amd as otip
    rng = np.random.default_rng(side * 10 + kind)
    xs = grid_coords(side)
    xt = grid_coords(side)
    m = n = side * side
    L = I.heuristic_key_limit(xs, xt, radius, kind)
    cJ = float(np.sqrt(L)) if kind == 2 else float(L)
    y = rng.uniform(0.0, 0.4 * cJ, m)
    z = rng.uniform(0.0, 0.4 * cJ, n)
    support = np.unique(rng.choice(m * n, 5 * (m + n), replace=False)).astype(np.int64)
    oi, oj, orr, nneg, size = otip.otip_price_subset(ctx, xs, xt, y, z,
                                                     bitmap_of(support, m * n), m, L, kind)
    idx, r, bneg = _cscan.price(xs, xt, y, z, support, m, kind, key_limit=L)
    assert size == grid_subset_size(side, L, kind)
    assert nneg == bneg and nneg > m     # the selection is a real top-m
    got = oi.cpu().numpy().astype(np.int64) + oj.cpu().numpy().astype(np.int64) * m
    np.testing.assert_array_equal(got, idx)
    np.testing.assert_array_equal(orr.cpu().numpy(), r)


def test_subset_pricing_with_few_negatives(ctx):
    """Fewer negative reduced costs in J than kmax: all of them, in order."""
    import paper_2206_11009_amd as otip
    side, kind = 32, 0
    xs = grid_coords(side)
    m = side * side
    L = I.heuristic_key_limit(xs, xs, 0.2, kind)
    rng = np.random.default_rng(77)
    y = rng.uniform(0.0, 0.3, m)
    z = rng.uniform(0.0, 0.3, m)
    _, _, count = _cscan.price(xs, xs, y, z, np.zeros(0, np.int64), 0, kind, key_limit=L)
    kmax = count + 7
    oi, oj, orr, nneg, size = otip.otip_price_subset(ctx, xs, xs, y, z, None, kmax, L, kind)
    idx, r, bneg = _cscan.price(xs, xs, y, z, np.zeros(0, np.int64), kmax, kind, key_limit=L)
    assert 0 < nneg == bneg == count < kmax and len(idx) == count
    got = oi.cpu().numpy().astype(np.int64) + oj.cpu().numpy().astype(np.int64) * m
    np.testing.assert_array_equal(got, idx)
    np.testing.assert_array_equal(orr.cpu().numpy(), r)


@pytest.mark.parametrize("cfg,k,radius", [("c1", 0, 0.15), ("c1", 3, 0.3), ("c2", 0, 0.1)])
def test_solve_with_heuristic_pricing_matches_oracle(ctx, cfg, k, radius):
    """heur_run = 3 iterations on J, then a full scan: the certified optimum is
    the oracle's (the stop test and the certificate scan all m n)."""
    import paper_2206_11009_amd as otip
    inst = config_instance(cfg, k)
    res = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt,
                          otip.params(heur_radius=radius, heur_run=3))
    certified(res, inst)
    assert res.heuristic_scans > 0
    ref = golden(cfg, k)["objective"]
    assert abs(res.objective - ref) <= 1e-6 * abs(ref)


def test_oracle_and_library_heuristic_solves_agree(ctx):
    """The same heuristic schedule on both sides (16 x 16, radius 0.2)."""
    import paper_2206_11009_amd as otip
    inst = config_instance("c1", 5)
    res = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt,
                          otip.params(heur_radius=0.2, heur_run=3))
    ref = oracle.solve(inst.a, inst.b, inst.xs, inst.xt,
                       oracle.OracleParams(heur_radius=0.2, heur_run=3))
    certified(res, inst)
    assert abs(res.objective - ref.objective) <= 1e-6 * abs(ref.objective)


def test_forced_switch_back_to_cg(ctx):
    """Direct solver from iteration 4, forced back to CG at iteration 8: one
    return, and the certified optimum of the oracle."""
    import paper_2206_11009_amd as otip
    inst = config_instance("c1", 1)
    res = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt,
                          otip.params(force_switch_at=4, force_switch_back_at=8, switch_cost=0))
    certified(res, inst)
    assert res.switches_back == 1 and res.direct_iterations >= 4
    ref = golden("c1", 1)["objective"]
    assert abs(res.objective - ref) <= 1e-6 * abs(ref)


def test_switch_back_rule_alternating_solvers(ctx):
    """Thresholds under which the support-drop rule fires at every chance and
    the growth rule at any growth: the solvers alternate while columns enter,
    and the solve still ends certified at the optimum."""
    import paper_2206_11009_amd as otip
    inst = config_instance("c1", 2)
    res = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt,
                          otip.params(switch_drop=-10.0, switch_back_grow=1e-9, switch_cost=0,
                                      max_iter=300))
    certified(res, inst)
    assert res.switches_back >= 3
    ref = golden("c1", 2)["objective"]
    assert abs(res.objective - ref) <= 1e-6 * abs(ref)


@pytest.mark.parametrize("cfg,k", [("c1", 4), ("c1", 9), ("c2", 1)])
def test_kept_schur_pattern_gives_the_same_optimum(ctx, cfg, k):
    """Support updates that only remove entries keep the Schur pattern (its
    extra entries are 0): the solve with and without the reuse reaches the
    same certified optimum.  (Such updates come late, once pricing finds no
    entering column; on the 64 x 64 family columns enter until the end.)"""
    import paper_2206_11009_amd as otip
    inst = config_instance(cfg, k)
    on = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt, otip.params(schur_reuse=1))
    off = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt, otip.params(schur_reuse=0))
    certified(on, inst)
    certified(off, inst)
    assert off.patterns_kept == 0
    if cfg == "c1":
        assert on.patterns_kept > 0
    assert abs(on.objective - off.objective) <= 1e-9 * abs(off.objective)
