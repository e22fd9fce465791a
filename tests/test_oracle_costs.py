"""Pins of the oracle's other costs (Section 5.1: the 1-, 2- and inf-norm of
the pixel offset, besides the squared 2-norm of the default workload) to things
other than itself: scipy's pairwise distances fed to an LP solver (HiGHS), the
norm inequalities and their equalities on an axis, the 1-D monotone coupling,
brute-force pricing and certificates on scipy's distances, the initial support
rule on the sorted distances, and purification with non-integer costs."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog
from scipy.spatial.distance import cdist

import oracle
from oracle import _cscan
from synthetic import config_instance

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

METRIC = {1: "cityblock", 2: "euclidean", 3: "chebyshev"}


def dist(xs, xt, kind):
    """m x n costs from scipy's pairwise distances (independent of the oracle)."""
    if kind == 0:
        return cdist(xs.astype(float), xt.astype(float), "sqeuclidean")
    return cdist(xs.astype(float), xt.astype(float), METRIC[kind])


def lp_optimum(a, b, C):
    m, n = C.shape
    A = sp.vstack([sp.kron(np.ones((1, n)), sp.eye(m)), sp.kron(sp.eye(n), np.ones((1, m)))])
    r = linprog(C.reshape(-1, order="F"), A_eq=A, b_eq=np.concatenate([a, b]), bounds=(0, None),
                method="highs",
                options=dict(primal_feasibility_tolerance=1e-10, dual_feasibility_tolerance=1e-10))
    assert r.status == 0
    return r.fun


def certified(res, a, b, C):
    m, n = C.shape
    assert res.status == "optimal"
    assert len(res.flows) <= m + n - 1 and oracle.is_forest(res.rows, res.cols, m, n)
    ra = np.bincount(res.rows, weights=res.flows, minlength=m)
    rb = np.bincount(res.cols, weights=res.flows, minlength=n)
    assert np.abs(ra - a).sum() + np.abs(rb - b).sum() <= 1e-9
    # the objective and every reduced cost on scipy's distances
    assert abs(float(C[res.rows, res.cols] @ res.flows) - res.objective) <= 1e-12 * max(
        1.0, res.objective)
    r = C - res.y[:, None] - res.z[None, :]
    bound = a @ res.y + b @ res.z + a.sum() * min(0.0, r.min())
    assert (res.objective - bound) / max(1.0, res.objective) <= 1e-6


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_cost_function_matches_scipy_and_norm_relations(kind):
    rng = np.random.default_rng(40 + kind)
    xs = rng.integers(-3000, 3000, (50, 2)).astype(np.int32)
    xt = rng.integers(-3000, 3000, (60, 2)).astype(np.int32)
    ii, jj = np.meshgrid(np.arange(50), np.arange(60), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    c = oracle.costs(xs, xt, ii, jj, kind)
    ref = dist(xs, xt, kind).ravel()
    if kind == 2:
        # scipy's value and the correctly rounded root of the exact square
        # agree to an ulp; the oracle's is the latter exactly
        np.testing.assert_allclose(c, ref, rtol=4e-16)
        q = oracle.costs(xs, xt, ii, jj, 0)
        assert np.array_equal(c, np.sqrt(q))
    else:
        assert np.array_equal(c, ref)
    l1, l2, li = (oracle.costs(xs, xt, ii, jj, k) for k in (1, 2, 3))
    assert np.all(li <= l2 * (1 + 1e-15)) and np.all(l2 <= l1 * (1 + 1e-15))
    assert np.all(l1 <= 2 * li) and np.all(l2 <= math.sqrt(2) * li * (1 + 1e-15))
    # on an axis the three norms coincide
    ax = np.stack([xs[:, 0], np.zeros(50, np.int32)], 1)
    at = np.stack([xt[:, 0], np.zeros(60, np.int32)], 1)
    v = [oracle.costs(ax, at, ii, jj, k) for k in (1, 2, 3)]
    assert np.array_equal(v[0], v[1]) and np.array_equal(v[1], v[2])


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_pricing_and_rmin_on_scipy_distances(kind):
    rng = np.random.default_rng(50 + kind)
    m, n = 37, 29
    xs = rng.integers(0, 25, (m, 2)).astype(np.int32)
    xt = rng.integers(0, 25, (n, 2)).astype(np.int32)
    C = dist(xs, xt, kind)
    if kind == 2:  # the oracle's exact rounding of the root
        C = np.sqrt(cdist(xs.astype(float), xt.astype(float), "sqeuclidean"))
    y = rng.uniform(0, 20, m)
    z = rng.uniform(0, 20, n)
    sup = np.sort(rng.choice(m * n, 50, replace=False))
    R = (C - y[:, None]) - z[None, :]
    allr = R.reshape(-1, order="F")
    mask = np.ones(m * n, bool)
    mask[sup] = False
    cand = np.flatnonzero(mask & (allr < 0))
    order = cand[np.lexsort((cand, allr[cand]))]
    idx, r, nneg = _cscan.price(xs, xt, y, z, sup, 40, kind)
    assert nneg == len(cand)
    assert np.array_equal(idx, order[:40]) and np.array_equal(r, allr[order[:40]])
    rm, arg = _cscan.rmin(xs, xt, y, z, kind)
    assert rm == allr.min() and arg == int(np.argmin(allr))


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_initial_support_on_sorted_distances(kind):
    rng = np.random.default_rng(60 + kind)
    m, n = 30, 26
    xs = rng.integers(0, 12, (m, 2)).astype(np.int32)
    xt = rng.integers(0, 12, (n, 2)).astype(np.int32)
    idx, T = oracle.initial_support(xs, xt, 5.0, kind)
    C = dist(xs, xt, kind).reshape(-1, order="F")
    key = C ** 2 if kind == 2 else C
    key = np.rint(key).astype(np.int64)
    target = math.ceil(5.0 * (m + n - 1))
    # T is the smallest integer with at least `target` keys <= T
    assert (key <= T).sum() >= target and (key <= T - 1).sum() < target
    base = set(np.flatnonzero(key <= T).tolist())
    Cm = C.reshape(m, n, order="F")
    rows = {int(i) + int(np.argmin(Cm[i])) * m for i in range(m)}
    cols = {int(np.argmin(Cm[:, j])) + j * m for j in range(n)}
    assert set(idx.tolist()) == base | rows | cols


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_whole_solves_vs_lp_solver(kind):
    inst = config_instance("c1", kind)
    res = oracle.solve(inst.a, inst.b, inst.xs, inst.xt, oracle.OracleParams(cost_kind=kind))
    C = dist(inst.xs, inst.xt, kind)
    ref = lp_optimum(inst.a, inst.b, C)
    assert abs(res.objective - ref) <= 1e-7 * ref
    certified(res, inst.a, inst.b, C)
    rng = np.random.default_rng(70 + kind)
    m, n = 23, 31
    xs = rng.integers(-20, 20, (m, 2)).astype(np.int32)
    xt = rng.integers(-20, 20, (n, 2)).astype(np.int32)
    a = rng.uniform(0.2, 1.0, m); a /= a.sum()
    b = rng.uniform(0.2, 1.0, n); b /= b.sum()
    res = oracle.solve(a, b, xs, xt, oracle.OracleParams(cost_kind=kind))
    C = dist(xs, xt, kind)
    assert abs(res.objective - lp_optimum(a, b, C)) <= 1e-7 * max(1.0, res.objective)
    certified(res, a, b, C)


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_one_dimensional_monotone_coupling(kind):
    """Points on a line: every kind's cost is |x - x'|, convex, so the sorted
    (north-west corner) coupling is optimal."""
    rng = np.random.default_rng(80 + kind)
    m, n = 25, 34
    xa, xb = rng.integers(0, 100, m), rng.integers(0, 100, n)
    a = rng.uniform(0.1, 1, m); a /= a.sum()
    b = rng.uniform(0.1, 1, n); b /= b.sum()
    ia, ib = np.argsort(xa, kind="stable"), np.argsort(xb, kind="stable")
    aa, bb = a[ia].copy(), b[ib].copy()
    i = j = 0
    opt = 0.0
    while i < m and j < n:
        t = min(aa[i], bb[j])
        opt += t * abs(float(xa[ia[i]] - xb[ib[j]]))
        aa[i] -= t
        bb[j] -= t
        if aa[i] <= 1e-300:
            i += 1
        else:
            j += 1
    xs = np.stack([xa, np.zeros(m, int)], 1).astype(np.int32)
    xt = np.stack([xb, np.zeros(n, int)], 1).astype(np.int32)
    res = oracle.solve(a, b, xs, xt, oracle.OracleParams(cost_kind=kind))
    assert abs(res.objective - opt) <= 1e-8 * opt


def test_purification_with_non_integer_costs():
    rng = np.random.default_rng(90)
    m, n = 12, 15
    xs = rng.integers(0, 9, (m, 2)).astype(np.int32)
    xt = rng.integers(0, 9, (n, 2)).astype(np.int32)
    rows = np.repeat(np.arange(m), 6)
    cols = rng.integers(0, n, rows.size)
    flows = rng.uniform(0.01, 1.0, rows.size)
    c = oracle.costs(xs, xt, rows, cols, 2)
    r2, c2, f2 = oracle.purify_to_forest(rows, cols, flows, c, m, n)
    assert oracle.is_forest(r2, c2, m, n)
    np.testing.assert_allclose(np.bincount(r2, weights=f2, minlength=m),
                               np.bincount(rows, weights=flows, minlength=m), atol=1e-12)
    np.testing.assert_allclose(np.bincount(c2, weights=f2, minlength=n),
                               np.bincount(cols, weights=flows, minlength=n), atol=1e-12)
    assert float(oracle.costs(xs, xt, r2, c2, 2) @ f2) <= float(c @ flows) * (1 + 1e-12)
