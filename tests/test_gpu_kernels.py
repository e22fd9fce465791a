"""Kernel-level parity of the HIP library against the CPU oracle (through the
C-ABI).  Pricing selections are compared bit for bit (the oracle is fed the
same FP64 duals); sums are compared to rounding."""
import numpy as np
import pytest

import oracle
from oracle import _cscan
from synthetic import config_instance, grid_coords

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2206_11009_amd as otip
    c = otip.Context(0)
    yield c
    c.close()


def bitmap_of(support, m, n):
    words = np.zeros((m * n + 31) // 32, np.uint32)
    s = np.asarray(support, np.int64)
    np.bitwise_or.at(words, s >> 5, (np.uint32(1) << (s & 31).astype(np.uint32)))
    return words.view(np.int32)


def price_both(ctx, xs, xt, y, z, support, kmax):
    import paper_2206_11009_amd as otip
    m, n = len(xs), len(xt)
    bm = bitmap_of(support, m, n) if len(support) else None
    oi, oj, orr, nneg = otip.otip_price(ctx, xs, xt, y, z, bm, kmax)
    g_idx = oi.cpu().numpy().astype(np.int64) + oj.cpu().numpy().astype(np.int64) * m
    g_r = orr.cpu().numpy()
    o_idx, o_r, o_neg = _cscan.price(xs, xt, y, z, np.sort(np.asarray(support, np.int64)), kmax)
    return g_idx, g_r, nneg, o_idx, o_r, o_neg


@pytest.mark.parametrize("m,n,kmax,seed", [(13, 11, 7, 0), (300, 257, 300, 1), (1000, 700, 50, 2),
                                           (64, 64, 100000, 3), (257, 129, 0, 4)])
def test_pricing_bit_exact_random(ctx, m, n, kmax, seed):
    rng = np.random.default_rng(seed)
    xs = rng.integers(0, 60, (m, 2)).astype(np.int32)
    xt = rng.integers(0, 60, (n, 2)).astype(np.int32)
    y = rng.uniform(0, 900, m)
    z = rng.uniform(0, 900, n)
    support = rng.choice(m * n, size=min(m * n // 3, 5000), replace=False)
    g_idx, g_r, g_neg, o_idx, o_r, o_neg = price_both(ctx, xs, xt, y, z, support, kmax)
    assert g_neg == o_neg
    np.testing.assert_array_equal(g_idx, o_idx)
    np.testing.assert_array_equal(g_r, o_r)


def test_pricing_ties_broken_by_index(ctx):
    """Integer duals make many reduced costs exactly equal; the selection at
    the cut must follow the variable index."""
    rng = np.random.default_rng(9)
    m, n = 400, 300
    xs = rng.integers(0, 20, (m, 2)).astype(np.int32)
    xt = rng.integers(0, 20, (n, 2)).astype(np.int32)
    y = rng.integers(0, 200, m).astype(float)
    z = rng.integers(0, 200, n).astype(float)
    for kmax in (1, 17, 999, 5000):
        g_idx, g_r, g_neg, o_idx, o_r, o_neg = price_both(ctx, xs, xt, y, z, [], kmax)
        assert g_neg == o_neg
        np.testing.assert_array_equal(g_idx, o_idx)
        np.testing.assert_array_equal(g_r, o_r)


def test_pricing_grid_64x64_full_size(ctx):
    """64x64 grids (16.8M variables) with duals near the optimum's scale."""
    inst = config_instance("c2", 0)
    m = inst.m
    rng = np.random.default_rng(3)
    c0 = oracle.sq_costs(inst.xs, inst.xt, np.arange(m), np.arange(m)).astype(float)
    y = rng.uniform(0, 50, m) + c0
    z = rng.uniform(0, 50, m)
    support = rng.choice(m * m, 50000, replace=False)
    g_idx, g_r, g_neg, o_idx, o_r, o_neg = price_both(ctx, inst.xs, inst.xt, y, z, support, m)
    assert g_neg == o_neg
    np.testing.assert_array_equal(g_idx, o_idx)
    np.testing.assert_array_equal(g_r, o_r)


def price_both_prec(ctx, xs, xt, y, z, support, kmax, precision):
    import paper_2206_11009_amd as otip
    m, n = len(xs), len(xt)
    bm = bitmap_of(support, m, n) if len(support) else None
    oi, oj, orr, nneg = otip.otip_price(ctx, xs, xt, y, z, bm, kmax, precision=precision)
    g_idx = oi.cpu().numpy().astype(np.int64) + oj.cpu().numpy().astype(np.int64) * m
    return g_idx, orr.cpu().numpy(), nneg


@pytest.mark.parametrize("cfg", ["c3", "c5"])
def test_pricing_full_size_fp64_and_mixed(ctx, cfg):
    """The 128 x 128 (268M variables) and 256 x 256 (4.29e9 variables, a
    537 MB support bitmap) scans select the oracle's m columns bit for bit, in
    FP64 and in the FP32 scan with its FP64 re-check, on duals at the scale of
    the optimum's (many reduced costs negative and inside the FP32 band)."""
    import paper_2206_11009_amd as otip
    inst = config_instance(cfg, 0)
    m = inst.m
    rng = np.random.default_rng(31)
    c0 = oracle.sq_costs(inst.xs, inst.xt, np.arange(m), np.arange(m)).astype(float)
    y = rng.uniform(0, 60, m) + c0
    z = rng.uniform(0, 60, m)
    support = np.unique(rng.choice(m * m, 10 * m, replace=False))
    o_idx, o_r, o_neg = _cscan.price(inst.xs, inst.xt, y, z, support, m)
    assert o_neg > m
    for prec in (otip.OTIP_FP64, otip.OTIP_MIXED):
        g_idx, g_r, g_neg = price_both_prec(ctx, inst.xs, inst.xt, y, z, support, m, prec)
        assert g_neg == o_neg, prec
        np.testing.assert_array_equal(g_idx, o_idx)
        np.testing.assert_array_equal(g_r, o_r)


def test_pricing_variable_indices_above_2_32(ctx):
    """m = 65536 sources, n = 70000 targets: variable indices i + j m reach
    4.6e9, beyond 32 bits."""
    rng = np.random.default_rng(47)
    m, n = 65536, 70000
    xs = rng.integers(0, 300, (m, 2)).astype(np.int32)
    xt = rng.integers(0, 300, (n, 2)).astype(np.int32)
    y = rng.uniform(0, 3000, m)
    z = rng.uniform(0, 3000, n)
    support = np.unique(rng.integers(0, m * n, 200000))
    g_idx, g_r, g_neg, o_idx, o_r, o_neg = price_both(ctx, xs, xt, y, z, support, m)
    assert o_neg > m and o_idx.max() > 2 ** 32
    assert g_neg == o_neg
    np.testing.assert_array_equal(g_idx, o_idx)
    np.testing.assert_array_equal(g_r, o_r)


def test_rmin(ctx):
    import paper_2206_11009_amd as otip
    rng = np.random.default_rng(5)
    xs = rng.integers(0, 60, (333, 2)).astype(np.int32)
    xt = rng.integers(0, 60, (517, 2)).astype(np.int32)
    y, z = rng.uniform(0, 900, 333), rng.uniform(0, 900, 517)
    v, arg = otip.otip_rmin(ctx, xs, xt, y, z)
    ov, oarg = _cscan.rmin(xs, xt, y, z)
    assert v == ov and arg == oarg


@pytest.mark.parametrize("m,n", [(1000, 300), (1024, 64), (3000, 130)])
def test_kron_apply_dense(ctx, m, n):
    import torch
    import paper_2206_11009_amd as otip
    rng = np.random.default_rng(m)
    X = rng.standard_normal((m, n))
    Xt = torch.as_tensor(np.ascontiguousarray(X.T), device="cuda:0")   # vec(X) contiguous
    rs = torch.empty(m, dtype=torch.float64, device="cuda:0")
    cs = torch.empty(n, dtype=torch.float64, device="cuda:0")
    otip.otip_kron_apply(ctx, Xt, rs, cs)
    vals = rng.standard_normal(m * n)
    rows, cols = np.arange(m * n) % m, np.arange(m * n) // m
    ra, rb = oracle.A_apply(X.reshape(-1, order="F"), rows, cols, m, n)
    np.testing.assert_allclose(rs.cpu().numpy(), ra, rtol=1e-12, atol=1e-11)
    np.testing.assert_allclose(cs.cpu().numpy(), rb, rtol=1e-12, atol=1e-11)
    y = torch.as_tensor(rng.standard_normal(m), device="cuda:0")
    z = torch.as_tensor(rng.standard_normal(n), device="cuda:0")
    Y = torch.empty((n, m), dtype=torch.float64, device="cuda:0")
    otip.otip_kron_apply_t(ctx, y, z, Y)
    ref = oracle.AT_apply(y.cpu().numpy(), z.cpu().numpy(), rows, cols)
    np.testing.assert_array_equal(Y.cpu().numpy().reshape(-1), ref)
    del vals


def test_schur_matches_oracle(ctx):
    import paper_2206_11009_amd as otip
    inst = config_instance("c1", 2)
    m, n = inst.m, inst.n
    idx, _ = oracle.initial_support(inst.xs, inst.xt, 5.0)
    rng = np.random.default_rng(1)
    extra = rng.choice(m * n, 400, replace=False)
    idx = np.unique(np.concatenate([idx, extra]))
    theta = rng.uniform(0.1, 10.0, idx.size)
    rp, ci, va, M, N = otip.otip_schur(ctx, m, n, idx, theta)
    rows, cols = idx % m, idx // m
    Mo, No, V = oracle.normal_blocks(theta, rows, cols, m, n)
    S = oracle.schur_complement(Mo, No, V, "M").toarray()
    G = np.zeros((n, n))
    rp, ci, va = rp.cpu().numpy(), ci.cpu().numpy(), va.cpu().numpy()
    for j in range(n):
        for e in range(rp[j], rp[j + 1]):
            G[j, ci[e]] = va[e]
    np.testing.assert_allclose(M.cpu().numpy(), Mo, rtol=1e-13)
    np.testing.assert_allclose(N.cpu().numpy(), No, rtol=1e-13)
    scale = np.abs(S).max()
    np.testing.assert_allclose(G, S, atol=1e-12 * scale)
    # pattern: exactly the nonzero structure of V^T V, column indices sorted
    pat = (V.T @ V).toarray() != 0
    assert ((G != 0) | np.eye(n, dtype=bool)).sum() >= pat.sum() - n
    for j in range(n):
        assert np.all(np.diff(ci[rp[j]:rp[j + 1]]) > 0)
    assert np.array_equal(G, G.T)   # exactly symmetric


@pytest.mark.parametrize("cfg,extra", [("c2", 20000), ("c3", 40000)])
def test_schur_matches_oracle_full_size(ctx, cfg, extra):
    """S_M at n = 4096 (rows accumulated in LDS) and n = 16384 (the merge of
    source lists used above 8192 targets), on the initial support plus random
    far entries (rows of S spanning more than 8192 columns), against the
    oracle's sparse N - V^T M^-1 V."""
    import scipy.sparse as sp
    import paper_2206_11009_amd as otip
    inst = config_instance(cfg, 0)
    m, n = inst.m, inst.n
    idx, _ = oracle.initial_support(inst.xs, inst.xt, 5.0)
    rng = np.random.default_rng(17)
    idx = np.unique(np.concatenate([idx, rng.choice(m * n, extra, replace=False)]))
    theta = np.exp(rng.uniform(-8.0, 8.0, idx.size))      # IPM-like spread of Theta
    rp, ci, va, M, N = otip.otip_schur(ctx, m, n, idx, theta)
    rp, ci, va = rp.cpu().numpy(), ci.cpu().numpy()[:rp[-1]], va.cpu().numpy()[:rp[-1]]
    G = sp.csr_matrix((va, ci, rp), shape=(n, n))
    rows, cols = idx % m, idx // m
    Mo, No, V = oracle.normal_blocks(theta, rows, cols, m, n)
    S = oracle.schur_complement(Mo, No, V, "M").tocsr()
    np.testing.assert_allclose(M.cpu().numpy(), Mo, rtol=1e-13)
    np.testing.assert_allclose(N.cpu().numpy(), No, rtol=1e-13)
    D = (G - S).tocoo()
    scale = abs(S).max()
    assert abs(D.data).max() <= 1e-12 * scale
    # the pattern holds every pair of targets sharing a source, sorted per row
    P = (V.T @ V).tocsr()
    P.data[:] = 1.0
    Gp = G.copy()
    Gp.data[:] = 1.0
    assert (P - P.multiply(Gp)).count_nonzero() == 0
    assert all(np.all(np.diff(ci[rp[j]:rp[j + 1]]) > 0) for j in range(n))
    assert (G - G.T).count_nonzero() == 0
    spans = np.array([ci[rp[j + 1] - 1] - ci[rp[j]] for j in range(n)])
    if n > 8192:
        assert spans.max() > 8192
    # zero row sums (eq. diagdom)
    assert abs(np.asarray(G.sum(axis=1)).ravel()).max() <= 1e-12 * scale


@pytest.mark.parametrize("m,n,kmax,seed", [(300, 257, 300, 1), (1000, 700, 50, 2), (64, 64, 100000, 3),
                                           (257, 129, 0, 4)])
def test_mixed_pricing_identical_to_fp64(ctx, m, n, kmax, seed):
    """FP32 scan + FP64 re-check returns exactly the FP64 selection and count."""
    import paper_2206_11009_amd as otip
    rng = np.random.default_rng(seed)
    xs = rng.integers(0, 60, (m, 2)).astype(np.int32)
    xt = rng.integers(0, 60, (n, 2)).astype(np.int32)
    y, z = rng.uniform(0, 900, m), rng.uniform(0, 900, n)
    support = rng.choice(m * n, size=min(m * n // 3, 5000), replace=False)
    bm = bitmap_of(support, m, n)
    oi, oj, orr, nneg = otip.otip_price(ctx, xs, xt, y, z, bm, kmax, otip.OTIP_MIXED)
    o_idx, o_r, o_neg = _cscan.price(xs, xt, y, z, np.sort(support.astype(np.int64)), kmax)
    assert nneg == o_neg
    g_idx = oi.cpu().numpy().astype(np.int64) + oj.cpu().numpy().astype(np.int64) * m
    np.testing.assert_array_equal(g_idx, o_idx)
    np.testing.assert_array_equal(orr.cpu().numpy(), o_r)


def test_mixed_pricing_near_zero_band(ctx):
    """Duals placed so that many reduced costs sit inside the FP32 margin of 0."""
    import paper_2206_11009_amd as otip
    inst = config_instance("c2", 1)
    m = inst.m
    rng = np.random.default_rng(8)
    c0 = oracle.sq_costs(inst.xs, inst.xt, np.arange(m), np.arange(m)).astype(float)
    y = c0 + rng.integers(0, 3, m).astype(float) + rng.uniform(-1e-6, 1e-6, m)
    z = np.zeros(m)
    for kmax in (0, 7, m):
        oi, oj, orr, nneg = otip.otip_price(ctx, inst.xs, inst.xt, y, z, None, kmax, otip.OTIP_MIXED)
        o_idx, o_r, o_neg = _cscan.price(inst.xs, inst.xt, y, z, np.zeros(0, np.int64), kmax)
        assert nneg == o_neg
        g_idx = oi.cpu().numpy().astype(np.int64) + oj.cpu().numpy().astype(np.int64) * m
        np.testing.assert_array_equal(g_idx, o_idx)
        np.testing.assert_array_equal(orr.cpu().numpy(), o_r)
