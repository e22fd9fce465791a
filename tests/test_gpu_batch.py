"""Batched solves and warm-started initial supports through the C-ABI."""
import numpy as np
import pytest

import oracle
from synthetic import batch_instances, config_instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2206_11009_amd as otip
    c = otip.Context(0)
    yield c
    c.close()


def certified(res, inst):
    m, n = inst.m, inst.n
    assert res.status == 0, res.info
    assert res.rel_gap <= 1e-6 and res.marginal_residual <= 1e-8
    assert len(res.flows) <= m + n - 1
    assert oracle.is_forest(res.rows, res.cols, m, n)
    c = oracle.sq_costs(inst.xs, inst.xt, res.rows, res.cols)
    assert abs(float((c * res.flows).sum()) - res.objective) <= 1e-12 * max(1, abs(res.objective))


def test_batch_equals_single_solves(ctx):
    """Every instance of an uneven batch gives exactly what a lone solve gives
    (the batch only overlaps independent solves on several streams)."""
    import paper_2206_11009_amd as otip
    insts = batch_instances(24)
    res = otip.otip_solve_batch(ctx, [(i.a, i.b, i.xs, i.xt) for i in insts],
                                otip.params(batch_workers=6))
    assert len(res) == len(insts)
    for inst, r in zip(insts, res):
        certified(r, inst)
        one = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt)
        assert r.objective == one.objective and r.iterations == one.iterations
        np.testing.assert_array_equal(r.flows, one.flows)
        np.testing.assert_array_equal(r.y, one.y)


def test_batch_small_instances_vs_oracle(ctx):
    import paper_2206_11009_amd as otip
    insts = [i for i in batch_instances(60) if i.m <= 144][:6]
    assert len(insts) >= 3
    res = otip.otip_solve_batch(ctx, [(i.a, i.b, i.xs, i.xt) for i in insts])
    for inst, r in zip(insts, res):
        certified(r, inst)
        ref = oracle.solve(inst.a, inst.b, inst.xs, inst.xt)
        assert abs(r.objective - ref.objective) <= 1e-6 * abs(ref.objective)


def test_batch_reports_the_bad_instance(ctx):
    import paper_2206_11009_amd as otip
    insts = batch_instances(5)
    probs = [(i.a, i.b, i.xs, i.xt) for i in insts]
    bad = probs[3]
    probs[3] = (bad[0] * 2.0, bad[1], bad[2], bad[3])      # sum(a) != sum(b)
    with pytest.raises(otip.OtipError) as e:
        otip.otip_solve_batch(ctx, probs, otip.params(batch_workers=2))
    assert e.value.code == otip.OTIP_EINVAL and "instance 3" in str(e.value)
    # the context stays usable
    r = otip.otip_solve_batch(ctx, probs[:3])
    assert all(x.status == 0 for x in r)


def test_empty_batch(ctx):
    import paper_2206_11009_amd as otip
    assert otip.otip_solve_batch(ctx, []) == []


@pytest.mark.parametrize("cfg,k", [("c1", 1), ("c1", 4), ("c2", 0)])
def test_warm_start_from_optimal_duals(ctx, cfg, k):
    """Duals of an optimum as the prediction: the warm support holds an optimal
    basis, the optimum is unchanged and no more iterations are needed."""
    import paper_2206_11009_amd as otip
    inst = config_instance(cfg, k)
    plain = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt)
    warm = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt, y0=plain.y, z0=plain.z)
    certified(warm, inst)
    assert abs(warm.objective - plain.objective) <= 1e-9 * abs(plain.objective)
    assert warm.iterations <= plain.iterations


def test_warm_start_rubbish_duals_still_certified(ctx):
    import paper_2206_11009_amd as otip
    inst = config_instance("c1", 2)
    rng = np.random.default_rng(0)
    plain = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt)
    for y0, z0 in [(rng.uniform(-500, 500, inst.m), rng.uniform(-500, 500, inst.n)),
                   (np.zeros(inst.m), np.zeros(inst.n))]:
        warm = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt, y0=y0, z0=z0)
        certified(warm, inst)
        assert abs(warm.objective - plain.objective) <= 1e-6 * abs(plain.objective)


def test_warm_start_nonfinite_falls_back_to_plain(ctx):
    import paper_2206_11009_amd as otip
    inst = config_instance("c1", 3)
    plain = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt)
    y0 = np.zeros(inst.m)
    y0[5] = np.nan
    warm = otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt, y0=y0, z0=np.zeros(inst.n))
    assert warm.objective == plain.objective and warm.iterations == plain.iterations
