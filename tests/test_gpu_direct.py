"""The direct solver of the Newton step after the switch (Section 4.2) alone,
through the C-ABI: the library's dense FP64 L D L^T with the infinite-pivot
rule on oracle-built Schur complements, against CPU solves."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import oracle.ipm as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2206_11009_amd as otip
    c = otip.Context(0)
    yield c
    c.close()


def schur_small(n_side, seed):
    m = n = n_side
    rng = np.random.default_rng(seed)
    idx = np.unique(np.concatenate([np.arange(m) + np.arange(m) * m,
                                    (np.arange(m) + 1) % m + np.arange(m) * m,
                                    rng.choice(m * n, 4 * m, replace=False)]))
    theta = np.exp(rng.uniform(-3, 3, idx.size))
    M, N, V = oracle.normal_blocks(theta, idx % m, idx // m, m, n)
    S = oracle.schur_complement(M, N, V, "M").tocsr()
    S.sort_indices()
    return S, rng


def run_case(ctx, S, rng, substitution):
    import paper_2206_11009_amd as otip
    n = S.shape[0]
    b = rng.standard_normal(n)
    b -= b.mean()                      # in the range of S (connected support)
    x, ninf, nnzl = otip.otip_ldl_solve(ctx, S.indptr, S.indices, S.data, b,
                                        substitution=substitution)
    x = x.cpu().numpy()
    assert ninf == 1
    assert n <= nnzl <= n * (n + 1) // 2
    r = S @ x - b
    assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(b)
    # the CPU factorisation of the oracle: the same solution up to the null vector e
    F = I.direct_factor(S, 1e-12)
    xc = F.solve(b)
    d = x - xc
    assert np.ptp(d) <= 1e-7 * max(1.0, np.abs(xc).max())


@pytest.mark.parametrize("substitution", [False, True])
def test_direct_solve_n100(ctx, substitution):
    S, rng = schur_small(100, 3)
    run_case(ctx, S, rng, substitution)


@pytest.mark.parametrize("substitution", [False, True])
def test_direct_solve_n2025_and_split_n4096(ctx, substitution):
    """n = 2025 (45 x 45, below the size where the inverse's top level is not
    formed) and n = 4096 (64 x 64, where the solves apply L21 between the two
    halves' inverses)."""
    for side in (45, 64):
        S, rng = grid_schur(side, side)
        run_case(ctx, S, rng, substitution)


def grid_schur(side, seed):
    """Schur complement (M-side) of a side x side grid pair: the initial support
    plus 5 m random entries, theta log-uniform over [e^-3, e^3]."""
    m = n = side * side
    rng = np.random.default_rng(seed)
    xs = np.stack([np.arange(m) // side, np.arange(m) % side], 1).astype(np.int32)
    idx, _ = oracle.initial_support(xs, xs, 5.0)
    idx = np.unique(np.concatenate([idx, rng.choice(m * n, 5 * m, replace=False)]))
    theta = np.exp(rng.uniform(-3.0, 3.0, idx.size))
    M, N, V = oracle.normal_blocks(theta, idx % m, idx // m, m, n)
    S = oracle.schur_complement(M, N, V, "M").tocsr()
    S.sort_indices()
    return S, rng


def solve_both_ways(ctx, S, rng):
    """The solve with the explicit inverse and by substitution: each leaves a
    residual at rounding level, and the two agree up to the null vector e."""
    import paper_2206_11009_amd as otip
    b = rng.standard_normal(S.shape[0])
    b -= b.mean()                      # in the range of S (connected support)
    xs = []
    for substitution in (False, True):
        x, ninf, _ = otip.otip_ldl_solve(ctx, S.indptr, S.indices, S.data, b,
                                         substitution=substitution)
        x = x.cpu().numpy()
        assert ninf == 1
        assert np.linalg.norm(S @ x - b) <= 1e-9 * np.linalg.norm(b)
        xs.append(x)
    assert np.ptp(xs[0] - xs[1]) <= 1e-7 * max(1.0, np.abs(xs[1]).max())


def test_direct_solve_ragged_update_n4900(ctx):
    """n = 4900 (70 x 70): trailing updates of 128 x 64 tiles with ragged last
    tile rows and columns (4644 = 36 * 128 + 36 rows after the first group of
    panels).  The oracle's sparse factorisation of this order takes most of a
    minute on the CPU, so the checks are the residual and the agreement of the
    two solve paths (the oracle is compared at n = 4096)."""
    S, rng = grid_schur(70, 70)
    solve_both_ways(ctx, S, rng)


def test_direct_solve_ragged_update_n9409(ctx):
    """n = 9409 (97 x 97): larger trailing triangles (9153 = 71 * 128 + 65 rows
    after the first group: the last tile row holds one full and one ragged
    64-row half)."""
    S, rng = grid_schur(97, 97)
    solve_both_ways(ctx, S, rng)


def test_direct_solve_is_deterministic(ctx):
    """The same factorisation and solve twice give the same bits (each panel
    workgroup reads its rows of A21 before any of its waves overwrites them
    with L21)."""
    import paper_2206_11009_amd as otip
    S, rng = grid_schur(97, 97)
    b = rng.standard_normal(S.shape[0])
    b -= b.mean()
    x1, _, _ = otip.otip_ldl_solve(ctx, S.indptr, S.indices, S.data, b)
    x2, _, _ = otip.otip_ldl_solve(ctx, S.indptr, S.indices, S.data, b)
    np.testing.assert_array_equal(x1.cpu().numpy(), x2.cpu().numpy())


def test_direct_solve_two_components_two_infinite_pivots(ctx):
    """A block-diagonal Schur complement of two disconnected supports: two
    infinite pivots, and every consistent right-hand side is solved."""
    import paper_2206_11009_amd as otip
    S1, rng = schur_small(60, 8)
    S2, _ = schur_small(40, 9)
    S = sp.block_diag([S1, S2]).tocsr()
    S.sort_indices()
    b = rng.standard_normal(100)
    b[:60] -= b[:60].mean()
    b[60:] -= b[60:].mean()
    x, ninf, _ = otip.otip_ldl_solve(ctx, S.indptr, S.indices, S.data, b)
    assert ninf == 2
    np.testing.assert_allclose(S @ x.cpu().numpy(), b, atol=1e-9 * np.linalg.norm(b))
