"""Degenerate and edge cases of whole solves through the C-ABI, against the
CPU oracle or a closed form, and the errors the boundary must report."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2206_11009_amd as otip
    c = otip.Context(0)
    yield c
    c.close()


def certified(res, a, b, xs, xt):
    m, n = len(a), len(b)
    assert res.status == 0, res.info
    assert res.rel_gap <= 1e-6 and res.marginal_residual <= 1e-8, res.info
    assert len(res.flows) <= m + n - 1
    assert oracle.is_forest(res.rows, res.cols, m, n)
    rs = np.zeros(m)
    cs = np.zeros(n)
    np.add.at(rs, res.rows, res.flows)
    np.add.at(cs, res.cols, res.flows)
    assert np.abs(rs - a).sum() + np.abs(cs - b).sum() <= 1e-8 * (a.sum() + b.sum())
    c = oracle.sq_costs(xs, xt, res.rows, res.cols)
    assert abs(float((c * res.flows).sum()) - res.objective) <= 1e-12 * max(1, abs(res.objective))


def masses(rng, k):
    v = rng.uniform(0.1, 1.0, k)
    return v / v.sum()


@pytest.mark.parametrize("m,n,seed", [(37, 23, 0), (23, 37, 1), (64, 5, 2), (5, 64, 3),
                                      (200, 130, 4)])
def test_rectangular_point_clouds(ctx, m, n, seed):
    """m != n, points anywhere in a box (not grids)."""
    import paper_2206_11009_amd as otip
    rng = np.random.default_rng(seed)
    xs = rng.integers(-300, 300, (m, 2)).astype(np.int32)
    xt = rng.integers(-300, 300, (n, 2)).astype(np.int32)
    a, b = masses(rng, m), masses(rng, n)
    res = otip.otip_solve(ctx, a, b, xs, xt)
    certified(res, a, b, xs, xt)
    ref = oracle.solve(a, b, xs, xt)
    assert abs(res.objective - ref.objective) <= 1e-6 * abs(ref.objective)


@pytest.mark.parametrize("m,n", [(1, 1), (1, 7), (7, 1), (2, 2)])
def test_tiny_and_single_row_or_column(ctx, m, n):
    """One source (or target): the plan is forced; its cost is the closed form."""
    import paper_2206_11009_amd as otip
    rng = np.random.default_rng(m * 10 + n)
    xs = rng.integers(0, 20, (m, 2)).astype(np.int32)
    xt = rng.integers(0, 20, (n, 2)).astype(np.int32)
    a, b = masses(rng, m), masses(rng, n)
    res = otip.otip_solve(ctx, a, b, xs, xt)
    certified(res, a, b, xs, xt)
    C = ((xs[:, None, :].astype(np.int64) - xt[None, :, :]) ** 2).sum(-1)
    if m == 1:
        assert res.objective == pytest.approx(float((C[0] * b).sum()), rel=1e-12)
    elif n == 1:
        assert res.objective == pytest.approx(float((C[:, 0] * a).sum()), rel=1e-12)
    else:
        assert abs(res.objective - oracle.solve(a, b, xs, xt).objective) <= 1e-9


def test_identical_supports_cost_zero(ctx):
    """Same points and masses on both sides: the optimum is 0 (the identity plan)."""
    import paper_2206_11009_amd as otip
    rng = np.random.default_rng(7)
    xs = rng.integers(0, 50, (150, 2)).astype(np.int32)
    a = masses(rng, 150)
    res = otip.otip_solve(ctx, a, a.copy(), xs, xs.copy())
    certified(res, a, a, xs, xs)
    assert abs(res.objective) <= 1e-12


def test_duplicate_points_and_ties(ctx):
    """Many coincident points: costs with massive ties, several optimal plans."""
    import paper_2206_11009_amd as otip
    rng = np.random.default_rng(8)
    xs = rng.integers(0, 4, (90, 2)).astype(np.int32)
    xt = rng.integers(0, 4, (70, 2)).astype(np.int32)
    a, b = masses(rng, 90), masses(rng, 70)
    res = otip.otip_solve(ctx, a, b, xs, xt)
    certified(res, a, b, xs, xt)
    ref = oracle.solve(a, b, xs, xt)
    assert abs(res.objective - ref.objective) <= 1e-6 * max(1e-12, abs(ref.objective)) + 1e-12


def test_masses_over_many_orders_of_magnitude(ctx):
    import paper_2206_11009_amd as otip
    rng = np.random.default_rng(9)
    m = n = 120
    xs = rng.integers(0, 40, (m, 2)).astype(np.int32)
    xt = rng.integers(0, 40, (n, 2)).astype(np.int32)
    a = 10.0 ** rng.uniform(-9, 0, m)
    b = 10.0 ** rng.uniform(-9, 0, n)
    b *= a.sum() / b.sum()
    res = otip.otip_solve(ctx, a, b, xs, xt)
    certified(res, a, b, xs, xt)
    ref = oracle.solve(a, b, xs, xt)
    assert abs(res.objective - ref.objective) <= 1e-6 * abs(ref.objective)


def test_largest_coordinates(ctx):
    """Coordinates at the documented limits (costs near 2^31)."""
    import paper_2206_11009_amd as otip
    rng = np.random.default_rng(10)
    lim = 1 << 14
    xs = rng.integers(-lim, lim + 1, (40, 2)).astype(np.int32)
    xt = rng.integers(-lim, lim + 1, (30, 2)).astype(np.int32)
    xs[0] = (-lim, -lim)
    xt[0] = (lim, lim)
    a, b = masses(rng, 40), masses(rng, 30)
    res = otip.otip_solve(ctx, a, b, xs, xt)
    certified(res, a, b, xs, xt)
    ref = oracle.solve(a, b, xs, xt)
    assert abs(res.objective - ref.objective) <= 1e-6 * abs(ref.objective)


@pytest.mark.parametrize("case", ["negative_mass", "nan_mass", "inf_mass", "unbalanced",
                                  "all_zero", "coordinate_range", "empty"])
def test_invalid_inputs_are_rejected(ctx, case):
    import paper_2206_11009_amd as otip
    rng = np.random.default_rng(11)
    m, n = 12, 9
    xs = rng.integers(0, 10, (m, 2)).astype(np.int32)
    xt = rng.integers(0, 10, (n, 2)).astype(np.int32)
    a, b = masses(rng, m), masses(rng, n)
    if case == "negative_mass":
        a[3] = -a[3]
    elif case == "inf_mass":
        b[2] = np.inf
    elif case == "all_zero":
        a[:] = 0.0
        b[:] = 0.0
    elif case == "nan_mass":
        a[0] = np.nan
    elif case == "unbalanced":
        a = a * 1.01
    elif case == "coordinate_range":
        xs[4, 1] = (1 << 14) + 1
    elif case == "empty":
        a, xs = a[:0], xs[:0]
    with pytest.raises(otip.OtipError) as e:
        otip.otip_solve(ctx, a, b, xs, xt)
    assert e.value.code == otip.OTIP_EINVAL
    # the context is still usable
    xs2 = rng.integers(0, 10, (m, 2)).astype(np.int32)
    assert otip.otip_solve(ctx, masses(rng, m), masses(rng, n), xs2, xt).status == 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_zero_masses_are_dropped_and_restored(ctx, seed):
    """Zero-mass rows and columns (the marginals lie in R+): the optimum is the
    one without them, they get no flow, and their c-transform duals keep every
    reduced cost of the full problem >= r_min (the certificate holds for it)."""
    import paper_2206_11009_amd as otip
    rng = np.random.default_rng(20 + seed)
    m, n = 60, 45
    xs = rng.integers(0, 30, (m, 2)).astype(np.int32)
    xt = rng.integers(0, 30, (n, 2)).astype(np.int32)
    a, b = masses(rng, m), masses(rng, n)
    zr = rng.choice(m, 7, replace=False)
    zc = rng.choice(n, 5, replace=False)
    if seed == 2:
        zc = np.append(zc, n - 1)           # the gauge column is dropped too
    a[zr] = 0.0
    b[zc] = 0.0
    b *= a.sum() / b.sum()
    res = otip.otip_solve(ctx, a, b, xs, xt)
    certified(res, a, b, xs, xt)
    assert len(res.y) == m and len(res.z) == n and res.z[n - 1] == 0.0
    assert not np.isin(res.rows, zr).any() and not np.isin(res.cols, zc).any()
    ki, kj = np.flatnonzero(a > 0), np.flatnonzero(b > 0)
    ref = oracle.solve(a[ki], b[kj], xs[ki], xt[kj])
    assert abs(res.objective - ref.objective) <= 1e-6 * abs(ref.objective)
    C = ((xs[:, None, :].astype(np.int64) - xt[None, :, :]) ** 2).sum(-1)
    r = C - res.y[:, None] - res.z[None, :]
    tol = 1e-9 * C.max()
    assert r[zr].min() >= -tol and r[:, zc].min() >= -tol
    bound = a @ res.y + b @ res.z + a.sum() * min(0.0, r.min())
    assert (res.objective - bound) / max(1.0, res.objective) <= 1e-6
