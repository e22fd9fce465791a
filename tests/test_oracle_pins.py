"""Pins of the CPU oracle to things other than itself.

Each test checks an oracle function against what the paper or the mathematics
fixes independently: explicit Kronecker matrices (Section 2.1), the block
structure of the normal matrix (Section 3.5), the Schur complement identities
and weak diagonal dominance (Section 4), the unreduced Newton block system
(eq. redsystem), brute-force pricing, and exact optima of transport problems
(enumeration of permutations, Hungarian algorithm, a simplex/IPM LP solver, and
closed forms: 1-D monotone coupling, translation, product marginals).
"""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linear_sum_assignment, linprog

import oracle
import oracle.ipm as I
from oracle import _cscan
from synthetic import config_instance, grid_coords

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def explicit_A(m, n):
    """A = [e_n^T (x) I_m ; I_n (x) e_m^T] as a dense matrix (eq. Astructure)."""
    return np.vstack([np.kron(np.ones((1, n)), np.eye(m)), np.kron(np.eye(n), np.ones((1, m)))])


def explicit_costs(xs, xt):
    """m x n integer squared distances, from a plain double loop."""
    m, n = len(xs), len(xt)
    C = np.zeros((m, n), np.int64)
    for i in range(m):
        for j in range(n):
            C[i, j] = sum((int(xs[i][d]) - int(xt[j][d])) ** 2 for d in range(2))
    return C


def random_support(rng, m, n, psi):
    idx = np.sort(rng.choice(m * n, size=psi, replace=False))
    return idx, idx % m, idx // m


# --------------------------------------------------------------- Section 2.1
def test_kronecker_products_match_explicit_matrix():
    rng = np.random.default_rng(1)
    m, n = 5, 7
    A = explicit_A(m, n)
    assert np.linalg.matrix_rank(A) == m + n - 1          # rank deficient by 1
    idx, rows, cols = random_support(rng, m, n, 17)
    vals = rng.standard_normal(17)
    x = np.zeros(m * n)
    x[idx] = vals
    ra, rb = oracle.A_apply(vals, rows, cols, m, n)
    np.testing.assert_allclose(np.concatenate([ra, rb]), A @ x, rtol=0, atol=1e-14)
    # A_1 x = X e_n, A_2 x = X^T e_m with X = reshape(x, m, n) column-wise
    X = x.reshape((m, n), order="F")
    np.testing.assert_allclose(ra, X.sum(1), atol=1e-14)
    np.testing.assert_allclose(rb, X.sum(0), atol=1e-14)
    y, z = rng.standard_normal(m), rng.standard_normal(n)
    np.testing.assert_allclose(oracle.AT_apply(y, z, rows, cols),
                               (A.T @ np.concatenate([y, z]))[idx], atol=1e-14)


# --------------------------------------------------------------- Section 3.5
def test_normal_matrix_blocks():
    rng = np.random.default_rng(2)
    m, n = 6, 4
    idx, rows, cols = random_support(rng, m, n, 15)
    theta = rng.uniform(0.1, 3.0, 15)
    Ared = explicit_A(m, n)[:, idx]
    K = Ared @ np.diag(theta) @ Ared.T
    M, N, V = oracle.normal_blocks(theta, rows, cols, m, n)
    Vd = V.toarray()
    np.testing.assert_allclose(K[:m, :m], np.diag(M), atol=1e-14)
    np.testing.assert_allclose(K[m:, m:], np.diag(N), atol=1e-14)
    np.testing.assert_allclose(K[:m, m:], Vd, atol=1e-14)
    # eq. matrix_relations: V e = M e, V^T e = N e
    np.testing.assert_allclose(Vd.sum(1), M, atol=1e-13)
    np.testing.assert_allclose(Vd.sum(0), N, atol=1e-13)


# --------------------------------------------------------------- Section 4
@pytest.mark.parametrize("m,n", [(7, 5), (5, 7)])
def test_schur_complements_and_diagonal_dominance(m, n):
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([np.arange(m) + (np.arange(m) % n) * m,
                                    (np.arange(n) % m) + np.arange(n) * m,
                                    rng.choice(m * n, 12, replace=False)]))
    rows, cols = idx % m, idx // m
    theta = rng.uniform(0.2, 5.0, idx.size)
    Ared = explicit_A(m, n)[:, idx]
    K = Ared @ np.diag(theta) @ Ared.T
    Kmm, Kmn, Knn = K[:m, :m], K[:m, m:], K[m:, m:]
    SM_ref = Knn - Kmn.T @ np.linalg.solve(Kmm, Kmn)
    SN_ref = Kmm - Kmn @ np.linalg.solve(Knn, Kmn.T)
    M, N, V = oracle.normal_blocks(theta, rows, cols, m, n)
    SM = oracle.schur_complement(M, N, V, "M").toarray()
    SN = oracle.schur_complement(M, N, V, "N").toarray()
    np.testing.assert_allclose(SM, SM_ref, atol=1e-12)
    np.testing.assert_allclose(SN, SN_ref, atol=1e-12)
    # S_M e = 0 and weak diagonal dominance holds with equality (eq. diagdom)
    for S in (SM, SN):
        np.testing.assert_allclose(S.sum(1), 0.0, atol=1e-12)
        off = np.abs(S).sum(1) - np.abs(np.diag(S))
        np.testing.assert_allclose(np.abs(np.diag(S)) - off, 0.0, atol=1e-12)
    # both Schur solution formulas (second block through S_M; first through
    # S_N with alpha_1 = S_N^-1 (beta_1 - V N^-1 beta_2)) solve K alpha = beta
    beta = K @ rng.standard_normal(m + n)
    a2 = np.linalg.lstsq(SM, beta[m:] - V.T.toarray() @ (beta[:m] / M), rcond=None)[0]
    a1 = (beta[:m] - V.toarray() @ a2) / M
    np.testing.assert_allclose(K @ np.concatenate([a1, a2]), beta, atol=1e-10)
    b1 = np.linalg.lstsq(SN, beta[:m] - V.toarray() @ (beta[m:] / N), rcond=None)[0]
    b2 = (beta[m:] - V.T.toarray() @ b1) / N
    np.testing.assert_allclose(K @ np.concatenate([b1, b2]), beta, atol=1e-10)


# --------------------------------------------------------------- eq. redsystem
@pytest.mark.parametrize("mode", ["direct", "pcg"])
def test_newton_direction_solves_unreduced_block_system(mode):
    rng = np.random.default_rng(4)
    m, n = 6, 5
    idx = np.unique(np.concatenate([np.arange(m) + (np.arange(m) % n) * m,
                                    (np.arange(n) % m) + np.arange(n) * m,
                                    rng.choice(m * n, 10, replace=False)]))
    st = I._State()
    st.m, st.n, st.zeta = m, n, 1.0
    st.xs = rng.integers(0, 5, (m, 2)).astype(np.int32)
    st.xt = rng.integers(0, 5, (n, 2)).astype(np.int32)
    st.a, st.b = rng.uniform(0.5, 1, m), rng.uniform(0.5, 1, n)
    st.b *= st.a.sum() / st.b.sum()
    I._set_support(st, idx, rng.uniform(0.1, 1, idx.size), rng.uniform(0.1, 1, idx.size))
    st.y, st.z = rng.standard_normal(m), rng.standard_normal(n)
    st.droptol = 1e-4
    st.theta = st.p / st.s
    r1a, r1b = rng.standard_normal(m) * 1e-2, rng.standard_normal(n) * 1e-2
    shift = (r1a.sum() - r1b.sum()) / n          # keep [e; -e]^T r1 = 0 (sum a = sum b)
    r1b = r1b + shift
    r2 = rng.standard_normal(st.psi) * 1e-2
    r3 = rng.standard_normal(st.psi) * 1e-2
    P = oracle.OracleParams(cg_max_iter=5000)
    sys_ = I._build_system(st, st.theta, mode, P)
    dp, dy, dz, ds = I._newton(st, sys_, r1a, r1b, r2, r3, 1e-13)
    psi = st.psi
    Ared = explicit_A(m, n)[:, st.idx]
    K = np.zeros((2 * psi + m + n, 2 * psi + m + n))
    K[:m + n, :psi] = Ared
    K[m + n:m + n + psi, psi:psi + m + n] = Ared.T
    K[m + n:m + n + psi, psi + m + n:] = np.eye(psi)
    K[m + n + psi:, :psi] = np.diag(st.s)
    K[m + n + psi:, psi + m + n:] = np.diag(st.p)
    rhs = np.concatenate([r1a, r1b, r2, r3])
    sol = np.linalg.lstsq(K, rhs, rcond=None)[0]
    np.testing.assert_allclose(K @ sol, rhs, atol=1e-10)   # consistent system
    np.testing.assert_allclose(dp, sol[:psi], atol=1e-9)
    np.testing.assert_allclose(ds, sol[psi + m + n:], atol=1e-9)
    # dy is unique up to the gauge (t e_m, -t e_n): compare A^T dy
    np.testing.assert_allclose(dy[st.rows] + dz[st.cols],
                               Ared.T @ sol[psi:psi + m + n], atol=1e-9)


# --------------------------------------------------------------- Section 3.4
def brute_price(xs, xt, y, z, support, kmax):
    m, n = len(xs), len(xt)
    C = explicit_costs(xs, xt).astype(np.float64)
    R = (C - y[:, None]) - z[None, :]
    r = R.reshape(-1, order="F")                   # vec: idx = i + j*m
    mask = np.ones(m * n, bool)
    mask[support] = False
    cand = np.nonzero(mask & (r < 0))[0]
    order = np.lexsort((cand, r[cand]))
    cand = cand[order]
    return cand[:kmax], r[cand[:kmax]], len(cand)


@pytest.mark.parametrize("integer_duals", [False, True])
@pytest.mark.parametrize("kmax", [0, 1, 7, 10_000])
def test_pricing_matches_brute_force(integer_duals, kmax):
    rng = np.random.default_rng(5 + kmax)
    m, n = 13, 11
    xs = rng.integers(0, 9, (m, 2)).astype(np.int32)
    xt = rng.integers(0, 9, (n, 2)).astype(np.int32)
    if integer_duals:       # many exact ties: the index tie-break decides
        y, z = rng.integers(0, 30, m).astype(float), rng.integers(0, 30, n).astype(float)
    else:
        y, z = rng.uniform(0, 40, m), rng.uniform(0, 40, n)
    support = np.sort(rng.choice(m * n, 20, replace=False))
    idx, r, nneg = _cscan.price(xs, xt, y, z, support, kmax)
    bidx, br, bneg = brute_price(xs, xt, y, z, support, kmax)
    assert nneg == bneg
    np.testing.assert_array_equal(idx, bidx)
    np.testing.assert_array_equal(r, br)


def test_rmin_matches_brute_force():
    rng = np.random.default_rng(6)
    xs = rng.integers(0, 9, (9, 2)).astype(np.int32)
    xt = rng.integers(0, 9, (12, 2)).astype(np.int32)
    y, z = rng.uniform(0, 40, 9), rng.uniform(0, 40, 12)
    R = (explicit_costs(xs, xt) - y[:, None]) - z[None, :]
    v, arg = _cscan.rmin(xs, xt, y, z)
    flat = R.reshape(-1, order="F")
    assert v == flat.min() and arg == int(np.argmin(flat))


# --------------------------------------------------------------- Section 3.2 (end)
def test_initial_support_threshold_and_cover():
    rng = np.random.default_rng(7)
    xs = rng.integers(0, 12, (40, 2)).astype(np.int32)
    xt = rng.integers(0, 12, (30, 2)).astype(np.int32)
    m, n = 40, 30
    idx, T = oracle.initial_support(xs, xt, 5.0)
    C = explicit_costs(xs, xt)
    target = math.ceil(5.0 * (m + n - 1))
    assert (C <= T).sum() >= target and (C <= T - 1).sum() < target
    want = set(np.nonzero((C <= T).reshape(-1, order="F"))[0].tolist())
    for i in range(m):
        want.add(i + int(np.argmin(C[i])) * m)
    for j in range(n):
        want.add(int(np.argmin(C[:, j])) + j * m)
    assert set(idx.tolist()) == want
    assert np.all(np.diff(idx) > 0)


# --------------------------------------------------------------- exact optima
def check_invariants(res, a, b, xs, xt):
    m, n = len(a), len(b)
    assert res.status == "optimal"
    assert res.marginal_residual <= 1e-8
    assert res.rel_gap <= 1e-6
    assert len(res.flows) <= m + n - 1
    assert oracle.is_forest(res.rows, res.cols, m, n)
    # complementary slackness on the plan's support: sum p |r| is a small part
    # of the objective
    c = oracle.sq_costs(xs, xt, res.rows, res.cols)
    red = c - res.y[res.rows] - res.z[res.cols]
    assert (res.flows * np.abs(red)).sum() <= 1e-6 * max(1.0, abs(res.objective))


@pytest.mark.parametrize("n", [3, 5, 7])
def test_uniform_marginals_vs_permutation_enumeration(n):
    """Birkhoff: with a = b = e/n an optimal plan is a permutation matrix / n."""
    rng = np.random.default_rng(100 + n)
    xs = rng.integers(0, 10, (n, 2)).astype(np.int32)
    xt = rng.integers(0, 10, (n, 2)).astype(np.int32)
    C = explicit_costs(xs, xt)
    best = min(sum(C[i, s[i]] for i in range(n)) for s in itertools.permutations(range(n)))
    a = np.full(n, 1.0 / n)
    res = oracle.solve(a, a.copy(), xs, xt)
    assert abs(res.objective - best / n) <= 1e-9 * max(1.0, best / n)
    check_invariants(res, a, a, xs, xt)


def test_uniform_marginals_vs_hungarian():
    rng = np.random.default_rng(11)
    n = 60
    xs = rng.integers(0, 30, (n, 2)).astype(np.int32)
    xt = rng.integers(0, 30, (n, 2)).astype(np.int32)
    C = explicit_costs(xs, xt)
    r, c = linear_sum_assignment(C)
    opt = C[r, c].sum() / n
    a = np.full(n, 1.0 / n)
    res = oracle.solve(a, a.copy(), xs, xt)
    assert abs(res.objective - opt) <= 1e-8 * opt
    check_invariants(res, a, a, xs, xt)


def lp_optimum(a, b, xs, xt):
    m, n = len(a), len(b)
    c = explicit_costs(xs, xt).reshape(-1, order="F").astype(float)
    A = sp.vstack([sp.kron(np.ones((1, n)), sp.eye(m)), sp.kron(sp.eye(n), np.ones((1, m)))])
    r = linprog(c, A_eq=A, b_eq=np.concatenate([a, b]), bounds=(0, None), method="highs",
                options=dict(primal_feasibility_tolerance=1e-10, dual_feasibility_tolerance=1e-10))
    assert r.status == 0
    return r.fun


@pytest.mark.parametrize("k", [0, 1, 2])
def test_gaussian_16x16_vs_lp_solver(k):
    inst = config_instance("c1", k)
    res = oracle.solve(inst.a, inst.b, inst.xs, inst.xt)
    ref = lp_optimum(inst.a, inst.b, inst.xs, inst.xt)
    assert abs(res.objective - ref) <= 1e-7 * ref
    check_invariants(res, inst.a, inst.b, inst.xs, inst.xt)


def test_rectangular_random_points_vs_lp_solver():
    rng = np.random.default_rng(12)
    m, n = 23, 37
    xs = rng.integers(0, 20, (m, 2)).astype(np.int32)
    xt = rng.integers(0, 20, (n, 2)).astype(np.int32)
    a = rng.uniform(0.2, 1.0, m); a /= a.sum()
    b = rng.uniform(0.2, 1.0, n); b /= b.sum()
    res = oracle.solve(a, b, xs, xt)
    ref = lp_optimum(a, b, xs, xt)
    assert abs(res.objective - ref) <= 1e-7 * ref
    check_invariants(res, a, b, xs, xt)


def monotone_1d(xa, a, xb, b):
    """Optimal cost of 1-D transport with convex cost: north-west corner rule on
    sorted positions (the monotone coupling)."""
    ia, ib = np.argsort(xa, kind="stable"), np.argsort(xb, kind="stable")
    xa, a, xb, b = xa[ia], a[ia].astype(float).copy(), xb[ib], b[ib].astype(float).copy()
    i = j = 0
    cost = 0.0
    while i < len(a) and j < len(b):
        t = min(a[i], b[j])
        cost += t * float(xa[i] - xb[j]) ** 2
        a[i] -= t
        b[j] -= t
        if a[i] <= 1e-300:
            i += 1
        else:
            j += 1
    return cost


def test_one_dimensional_monotone_coupling():
    rng = np.random.default_rng(13)
    m, n = 30, 45
    xa = rng.integers(0, 100, m)
    xb = rng.integers(0, 100, n)
    a = rng.uniform(0.1, 1, m); a /= a.sum()
    b = rng.uniform(0.1, 1, n); b /= b.sum()
    xs = np.stack([xa, np.zeros(m, int)], 1).astype(np.int32)
    xt = np.stack([xb, np.zeros(n, int)], 1).astype(np.int32)
    res = oracle.solve(a, b, xs, xt)
    opt = monotone_1d(xa, a, xb, b)
    assert abs(res.objective - opt) <= 1e-8 * opt
    check_invariants(res, a, b, xs, xt)


def test_product_marginals_separate():
    """a = a_x (x) a_y, b = b_x (x) b_y on a grid: the squared cost separates, so
    OPT = W(a_x, b_x) + W(a_y, b_y) (each a 1-D monotone coupling)."""
    rng = np.random.default_rng(14)
    side = 12
    ax, ay, bx, by = (rng.uniform(0.1, 1, side) for _ in range(4))
    ax, ay, bx, by = ax / ax.sum(), ay / ay.sum(), bx / bx.sum(), by / by.sum()
    xy = grid_coords(side)               # pixel i at (i // side, i % side)
    a = np.outer(ax, ay).reshape(-1)
    b = np.outer(bx, by).reshape(-1)
    pos = np.arange(side)
    opt = monotone_1d(pos, ax, pos, bx) + monotone_1d(pos, ay, pos, by)
    res = oracle.solve(a, b, xy, xy.copy())
    assert abs(res.objective - opt) <= 1e-8 * opt
    check_invariants(res, a, b, xy, xy)


def test_translation():
    """b(x) = a(x - t) with both supports inside the grid: OPT = |t|^2 sum(a)
    (Jensen's inequality gives the lower bound, the shift attains it)."""
    side, t = 14, (2, 3)
    rng = np.random.default_rng(15)
    img = np.zeros((side, side))
    img[1:8, 2:9] = rng.uniform(0.2, 1.0, (7, 7))
    sh = np.zeros_like(img)
    sh[1 + t[0]:8 + t[0], 2 + t[1]:9 + t[1]] = img[1:8, 2:9]
    a = img.reshape(-1) + 1e-12
    b = sh.reshape(-1) + 1e-12
    b *= a.sum() / b.sum()
    xy = grid_coords(side)
    res = oracle.solve(a, b, xy, xy.copy())
    opt = (t[0] ** 2 + t[1] ** 2) * a.sum()
    assert abs(res.objective - opt) <= 1e-6 * opt
    assert res.marginal_residual <= 1e-8 and res.rel_gap <= 1e-6


def test_identical_marginals_cost_zero():
    inst = config_instance("c1", 3)
    res = oracle.solve(inst.a, inst.a.copy(), inst.xs, inst.xt)
    assert abs(res.objective) <= 1e-12
    assert res.marginal_residual <= 1e-8


def test_single_source():
    rng = np.random.default_rng(16)
    xs = np.array([[3, 4]], np.int32)
    xt = rng.integers(0, 10, (20, 2)).astype(np.int32)
    b = rng.uniform(0.1, 1, 20); b /= b.sum()
    res = oracle.solve(np.array([1.0]), b, xs, xt)
    opt = float((explicit_costs(xs, xt)[0] * b).sum())
    assert abs(res.objective - opt) <= 1e-12 * opt


# --------------------------------------------------------------- purification
def test_purification_gives_forest_with_same_marginals_and_no_more_cost():
    rng = np.random.default_rng(17)
    m, n = 9, 8
    xs = rng.integers(0, 6, (m, 2)).astype(np.int32)
    xt = rng.integers(0, 6, (n, 2)).astype(np.int32)
    a = rng.uniform(0.1, 1, m); a /= a.sum()
    b = rng.uniform(0.1, 1, n); b /= b.sum()
    P = np.outer(a, b)                       # fully dense feasible plan
    rows, cols = np.nonzero(P)
    flows = P[rows, cols]
    costs = explicit_costs(xs, xt)[rows, cols]
    r2, c2, f2 = oracle.purify_to_forest(rows, cols, flows, costs, m, n)
    assert oracle.is_forest(r2, c2, m, n) and len(f2) <= m + n - 1
    ra, rb = oracle.A_apply(f2, r2, c2, m, n)
    np.testing.assert_allclose(ra, a, atol=1e-15)
    np.testing.assert_allclose(rb, b, atol=1e-15)
    assert (explicit_costs(xs, xt)[r2, c2] * f2).sum() <= (costs * flows).sum() + 1e-15


# --------------------------------------------------------------- Thm 2 / Cor. 1
def _is_chordal(adj):
    """Maximum cardinality search, then check the ordering is a perfect
    elimination ordering (Tarjan & Yannakakis)."""
    n = len(adj)
    weight = [0] * n
    order, seen = [], [False] * n
    for _ in range(n):
        v = max((u for u in range(n) if not seen[u]), key=lambda u: weight[u])
        seen[v] = True
        order.append(v)
        for u in adj[v]:
            if not seen[u]:
                weight[u] += 1
    pos = {v: k for k, v in enumerate(order)}
    for v in order:
        earlier = [u for u in adj[v] if pos[u] < pos[v]]
        if earlier:
            p = max(earlier, key=lambda u: pos[u])
            if not set(earlier) - {p} <= set(adj[p]):
                return False
    return True


def test_schur_pattern_of_forest_support_is_chordal():
    """Corollary 1: on an acyclic support the Schur complement pattern is chordal,
    so a perfect elimination ordering factorises it with zero fill."""
    rng = np.random.default_rng(18)
    m, n = 15, 12
    # random spanning tree of the bipartite graph
    nodes = list(range(m + n))
    rng.shuffle(nodes)
    edges = []
    for k in range(1, m + n):
        v = nodes[k]
        cands = [u for u in nodes[:k] if (u < m) != (v < m)]
        if not cands:
            continue
        u = cands[rng.integers(len(cands))]
        i, j = (u, v - m) if u < m else (v, u - m)
        edges.append(i + j * m)
    idx = np.unique(edges)
    rows, cols = idx % m, idx // m
    assert oracle.is_forest(rows, cols, m, n)
    M, N, V = oracle.normal_blocks(rng.uniform(0.5, 2, idx.size), rows, cols, m, n)
    S = oracle.schur_complement(M, N, V, "M").tocoo()
    adj = [set() for _ in range(n)]
    for r_, c_ in zip(S.row, S.col):
        if r_ != c_:
            adj[r_].add(c_)
    assert _is_chordal(adj)


# --------------------------------------------------------------- Section 4.2
def _brute_fill(pattern):
    """Entries of the strictly lower factor from symbolic elimination on a
    dense boolean matrix: eliminating k joins every pair of its later
    neighbours (the elimination graph)."""
    P = pattern.copy()
    n = P.shape[0]
    total = 0
    for k in range(n):
        later = np.nonzero(P[k + 1:, k])[0] + k + 1
        total += later.size
        for a in later:
            P[later, a] = True
            P[a, later] = True
    return total


def _random_spd(rng, n, density):
    A = sp.random(n, n, density=density, random_state=int(rng.integers(1 << 30)))
    A = A + A.T
    return (A + sp.diags(np.asarray(abs(A).sum(1)).ravel() + 1.0)).tocsr()


@pytest.mark.parametrize("n,density", [(1, 1.0), (7, 0.3), (60, 0.08), (200, 0.02)])
def test_ldl_reconstructs_the_matrix_and_counts_the_symbolic_fill(n, density):
    """L D L^T equals the permuted matrix, and the stored entries of L are
    exactly those of symbolic elimination (so the fill statistic is the true
    one)."""
    rng = np.random.default_rng(n)
    A = _random_spd(rng, n, density)
    perm = rng.permutation(n)
    F = _cscan.LDL(A, perm, 1e-12)
    assert F.n_inf == 0
    L, d = F.factors()
    Ap = A[perm][:, perm].toarray()
    np.testing.assert_allclose((L @ sp.diags(d) @ L.T).toarray(), Ap, rtol=0, atol=1e-12 * abs(Ap).max())
    assert np.allclose(np.diag(L.toarray()), 1.0) and sp.triu(L, 1).nnz == 0
    assert F.nnz_L - n == _brute_fill(Ap != 0.0)
    b = rng.standard_normal(n)
    np.testing.assert_allclose(A @ F.solve(b), b, atol=1e-10)


def test_ldl_infinite_pivot_grounds_each_component():
    """A weighted graph Laplacian is singular once per connected component: the
    factorisation replaces exactly that many pivots by +inf (the paper's
    modified factorisation) and returns a solution of every consistent
    system, equal to the minimum-norm one up to a constant per component."""
    rng = np.random.default_rng(3)
    blocks = []
    for size in (9, 14, 6):
        W = sp.random(size, size, density=0.5, random_state=int(rng.integers(1 << 30)))
        W = W + W.T + sp.diags(np.ones(size - 1), 1) + sp.diags(np.ones(size - 1), -1)  # connected
        W = sp.csr_matrix(W - sp.diags(W.diagonal()))
        blocks.append(sp.diags(np.asarray(W.sum(1)).ravel()) - W)
    S = sp.block_diag(blocks).tocsr()
    n = S.shape[0]
    comp = np.repeat(np.arange(3), [9, 14, 6])
    F = _cscan.LDL(S, rng.permutation(n), 1e-10)
    assert F.n_inf == 3
    b = rng.standard_normal(n)
    b -= (np.bincount(comp, b) / np.bincount(comp))[comp]  # consistent: zero sum per component
    x = F.solve(b)
    np.testing.assert_allclose(S @ x, b, atol=1e-10)
    x_pinv = np.linalg.pinv(S.toarray()) @ b
    shift = x - x_pinv
    for c in range(3):
        assert np.ptp(shift[comp == c]) < 1e-9


def test_ldl_of_forest_schur_complement_has_zero_fill_under_a_perfect_ordering():
    """Corollary 1 with the factor itself: the Schur complement of an acyclic
    support, ordered by a perfect elimination ordering (reversed maximum
    cardinality search), factorises with no entry outside its own pattern."""
    rng = np.random.default_rng(21)
    m, n = 18, 14
    nodes = list(range(m + n))
    rng.shuffle(nodes)
    edges = []
    for k in range(1, m + n):
        v = nodes[k]
        cands = [u for u in nodes[:k] if (u < m) != (v < m)]
        if cands:
            u = cands[rng.integers(len(cands))]
            i, j = (u, v - m) if u < m else (v, u - m)
            edges.append(i + j * m)
    idx = np.unique(edges)
    rows, cols = idx % m, idx // m
    M, N, V = oracle.normal_blocks(rng.uniform(0.5, 2, idx.size), rows, cols, m, n)
    S = oracle.schur_complement(M, N, V, "M").tocsr()
    adj = [set(S[r].indices) - {r} for r in range(n)]
    weight, order, seen = [0] * n, [], [False] * n
    for _ in range(n):
        v = max((u for u in range(n) if not seen[u]), key=lambda u: weight[u])
        seen[v] = True
        order.append(v)
        for u in adj[v]:
            if not seen[u]:
                weight[u] += 1
    peo = np.array(order[::-1])
    F = _cscan.LDL(S, peo, 1e-12)
    assert F.nnz_L == sp.tril(S).nnz


# --------------------------------------------------------------- Section 3.4
def _norm_dist(xs, xt, kind):
    """m x n distances in the cost's norm, and the squared 2-norm, by numpy."""
    d = xs[:, None, :].astype(np.int64) - xt[None, :, :].astype(np.int64)
    sq = (d * d).sum(-1)
    if kind == 1:
        return np.abs(d).sum(-1).astype(float), sq
    if kind == 3:
        return np.abs(d).max(-1).astype(float), sq
    return np.sqrt(sq), sq


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
@pytest.mark.parametrize("radius", [0.05, 0.2, 0.5])
def test_heuristic_subset_is_the_disk_of_the_largest_distance(kind, radius):
    """J = {cost key < L} holds exactly the pairs closer than radius * D, with D
    the largest distance of the points' bounding box in the cost's norm (so J
    is the same fraction of all pairs at every image side, Section 5.1)."""
    side = 24
    xs = grid_coords(side)
    xt = grid_coords(side)
    L = I.heuristic_key_limit(xs, xt, radius, kind)
    dist, sq = _norm_dist(xs, xt, kind)
    D = {0: math.sqrt(2) * (side - 1), 2: math.sqrt(2) * (side - 1), 1: 2 * (side - 1),
         3: side - 1}[kind]
    key = sq if kind in (0, 2) else dist.astype(np.int64)
    inside = dist < radius * D
    np.testing.assert_array_equal(key < L, inside)


@pytest.mark.parametrize("kind", [0, 2])
@pytest.mark.parametrize("kmax", [1, 9, 10_000])
def test_heuristic_pricing_is_pricing_restricted_to_the_subset(kind, kmax):
    """Pricing over J equals a brute-force sort of the reduced costs of J's
    variables outside the support; a limit above every key is the full scan."""
    rng = np.random.default_rng(30 + kmax + kind)
    m, n = 17, 14
    xs = rng.integers(0, 12, (m, 2)).astype(np.int32)
    xt = rng.integers(0, 12, (n, 2)).astype(np.int32)
    y, z = rng.uniform(0, 60, m), rng.uniform(0, 60, n)
    support = np.sort(rng.choice(m * n, 25, replace=False))
    L = 30
    _, sq = _norm_dist(xs, xt, kind)
    c = np.sqrt(sq) if kind == 2 else sq.astype(float)
    r = (c - y[:, None]) - z[None, :]
    idx_all = np.arange(m * n)
    rv = r.reshape(-1, order="F")
    keyv = sq.reshape(-1, order="F")
    ok = (rv < 0) & (keyv < L) & ~np.isin(idx_all, support)
    cand = idx_all[ok]
    cand = cand[np.lexsort((cand, rv[cand]))]
    idx, rr, nneg = _cscan.price(xs, xt, y, z, support, kmax, kind, key_limit=L)
    assert nneg == cand.size
    np.testing.assert_array_equal(idx, cand[:kmax])
    np.testing.assert_array_equal(rr, rv[cand[:kmax]])
    full = _cscan.price(xs, xt, y, z, support, kmax, kind)
    above = _cscan.price(xs, xt, y, z, support, kmax, kind, key_limit=int(sq.max()) + 1)
    for u, v in zip(full, above):
        np.testing.assert_array_equal(u, v)


@pytest.mark.parametrize("k,kind", [(0, 0), (1, 0), (2, 1)])
def test_heuristic_pricing_solve_reaches_the_lp_optimum(k, kind):
    """With heuristic pricing (3 iterations on J, then a full scan) the method
    still ends at the optimum: the stop test's pricing and the certificate scan
    every variable."""
    inst = config_instance("c1", k)
    P = oracle.OracleParams(heur_radius=0.15, heur_run=3, cost_kind=kind)
    hist = []
    res = oracle.solve(inst.a, inst.b, inst.xs, inst.xt, P, log=hist.append)
    assert any(h.get("heuristic") for h in hist) and not all(h.get("heuristic") for h in hist)
    if kind == 0:
        ref = lp_optimum(inst.a, inst.b, inst.xs, inst.xt)
    else:
        ref = oracle.solve(inst.a, inst.b, inst.xs, inst.xt,
                           oracle.OracleParams(cost_kind=kind)).objective
    assert abs(res.objective - ref) <= 1e-7 * ref
    assert res.rel_gap <= 1e-6 and res.marginal_residual <= 1e-8


# --------------------------------------------------------------- Sections 4.2, 4.3 remarks
def test_ordering_is_reused_while_the_pattern_stays_inside_it():
    """The symbolic part (ordering) of the factorisation is kept while the
    Schur pattern shrinks and recomputed when it grows; the factor it gives is
    exact either way."""
    rng = np.random.default_rng(40)
    n = 80
    A = _random_spd(rng, n, 0.06)
    cache = {}
    F1 = I.direct_factor(A, 1e-12, cache)
    assert cache.get("reused", 0) == 0
    # drop some off-diagonal pairs (symmetric): pattern shrinks -> reused
    C = sp.triu(A, 1).tocoo()
    keep = rng.random(C.nnz) > 0.3
    U = sp.coo_matrix((C.data[keep], (C.row[keep], C.col[keep])), shape=A.shape)
    B = U + U.T
    B = (B + sp.diags(np.asarray(abs(B).sum(1)).ravel() + 1.0)).tocsr()
    F2 = I.direct_factor(B, 1e-12, cache)
    assert cache["reused"] == 1
    b = rng.standard_normal(n)
    np.testing.assert_allclose(B @ F2.solve(b), b, atol=1e-10)
    np.testing.assert_allclose(A @ F1.solve(b), b, atol=1e-10)
    # a new off-diagonal pair outside the pattern -> a new ordering
    i, j = np.argwhere((A.toarray() == 0) & ~np.eye(n, dtype=bool))[0]
    E = sp.coo_matrix(([0.5, 0.5], ([i, j], [j, i])), shape=A.shape)
    G = (A + E + sp.diags(np.full(n, 1.0))).tocsr()
    I.direct_factor(G, 1e-12, cache)
    assert cache["reused"] == 1


def test_forced_switch_back_to_cg_still_reaches_the_optimum():
    """A switch to the direct solver at iteration 4 and a forced return to CG
    at iteration 8 (remark of Section 4.3): the following iterations run CG and
    the solve ends at the LP optimum."""
    inst = config_instance("c1", 1)
    hist = []
    P = oracle.OracleParams(force_switch_at=4, force_switch_back_at=8)
    res = oracle.solve(inst.a, inst.b, inst.xs, inst.xt, P, log=hist.append)
    assert res.switches_back == 1
    solvers = [h["solver"] for h in hist]
    k = next(q for q, h in enumerate(hist) if h.get("switch_back"))
    assert hist[k]["it"] == 8 and solvers[k - 1] == "direct"
    ref = lp_optimum(inst.a, inst.b, inst.xs, inst.xt)
    assert abs(res.objective - ref) <= 1e-7 * ref
    check_invariants(res, inst.a, inst.b, inst.xs, inst.xt)


def test_switch_back_rule_alternating_solvers_reach_the_optimum():
    """Thresholds that make the support-drop rule fire at every chance and the
    growth rule at any growth of the support: the solvers alternate while
    columns enter, and the method still converges."""
    inst = config_instance("c1", 2)
    hist = []
    P = oracle.OracleParams(switch_drop=-10.0, switch_back_grow=1e-9, max_iter=300)
    res = oracle.solve(inst.a, inst.b, inst.xs, inst.xt, P, log=hist.append)
    assert res.switches_back >= 3
    ref = lp_optimum(inst.a, inst.b, inst.xs, inst.xt)
    assert abs(res.objective - ref) <= 1e-7 * ref
    check_invariants(res, inst.a, inst.b, inst.xs, inst.xt)
