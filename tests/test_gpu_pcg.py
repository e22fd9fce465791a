"""The Newton step's preconditioned CG alone (otip_pcg) on Schur complements
that the oracle builds (Section 4): the residual bound it promises, the same
image S x as the oracle's own PCG, iteration counts close to the oracle's (the
same Jacobi preconditioner, so the same iterates in exact arithmetic), both
storage precisions, the SpMV's two lane-group shapes, both forms of the
iteration (one launch, or two for a matrix beyond 96 MB), ragged sizes,
degenerate matrices and rejected inputs."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from synthetic import config_instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2206_11009_amd as otip
    c = otip.Context(0)
    yield c
    c.close()


def schur_case(m, n, per_row, seed, spread=2.0):
    """S_M of a random support with per_row entries per source row (plus a
    cover of every column), theta log-uniform over 10^[-spread, spread]."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(m), per_row)
    cols = rng.integers(0, n, rows.size)
    rows = np.concatenate([rows, rng.integers(0, m, n)])
    cols = np.concatenate([cols, np.arange(n)])
    idx = np.unique(rows + cols.astype(np.int64) * m)
    r, c = idx % m, idx // m
    theta = 10.0 ** rng.uniform(-spread, spread, idx.size)
    M, N, V = oracle.normal_blocks(theta, r, c, m, n)
    S = oracle.schur_complement(M, N, V, "M").tocsr()
    S.sort_indices()
    x_true = rng.standard_normal(n)
    b = S @ x_true                      # in the range of S by construction
    return S, b


def run(ctx, S, b, rtol, maxit=1000, precision=0):
    import paper_2206_11009_amd as otip
    import torch
    rp = torch.as_tensor(S.indptr.astype(np.int32), device="cuda:0")
    ci = torch.as_tensor(S.indices.astype(np.int32), device="cuda:0")
    va = torch.as_tensor(S.data, device="cuda:0")
    x, res = otip.otip_pcg(ctx, rp, ci, va, b, rtol=rtol, maxit=maxit, precision=precision)
    return x.cpu().numpy(), res


@pytest.mark.parametrize("m,n,per_row,seed", [(300, 257, 3, 0),    # deg < 48: 16 lanes per row
                                              (120, 131, 40, 1),   # 64 lanes per row
                                              (64, 1031, 6, 2)])   # ragged, many rows
@pytest.mark.parametrize("precision", [0, 1])
def test_pcg_meets_its_bound_and_matches_the_oracle(ctx, m, n, per_row, seed, precision):
    S, b = schur_case(m, n, per_row, seed)
    rtol = 1e-8
    x, res = run(ctx, S, b, rtol, precision=precision)
    assert res.status == 0, res.status
    nb = np.linalg.norm(b)
    true_res = np.linalg.norm(b - S @ x)
    # the FP64 form stops on the recurrence residual, which drifts from the
    # true one by rounding; the mixed form stops on the true FP64 residual
    assert true_res <= (1.5 if precision == 0 else 1.0) * rtol * nb + 1e-13 * nb
    d = 1.0 / S.diagonal()
    xo, its_o, ok = oracle.ipm.pcg(S, b, rtol, 1000, lambda r: d * r)
    assert ok
    # x may differ from the oracle's in the null space of S; S x may not
    assert np.linalg.norm(S @ (x - xo)) <= 3 * rtol * nb
    if precision == 0:
        assert abs(res.iterations - its_o) <= 2 + 0.1 * its_o, (res.iterations, its_o)
        assert res.spmv_launches == res.iterations
        assert res.spmv_bytes == 12.0 * S.nnz + 100.0 * S.shape[0]   # a cache-resident S
        assert res.spmv_seconds > 0.0


def test_pcg_two_launch_form_beyond_96_mb(ctx):
    """A Schur matrix of about 11.5M nonzeros (138 MB of values and columns):
    the CG takes its two-launch form (timed SpMV bytes 12 nnz + 36 n), meets
    its bound, and matches the oracle's image and iteration count."""
    S, b = schur_case(20000, 20000, 24, 11, spread=4.0)
    assert 12.0 * S.nnz > 96.0 * (1 << 20)
    rtol = 1e-8
    x, res = run(ctx, S, b, rtol)
    assert res.status == 0, res.status
    nb = np.linalg.norm(b)
    assert np.linalg.norm(b - S @ x) <= 1.5 * rtol * nb + 1e-13 * nb
    d = 1.0 / S.diagonal()
    xo, its_o, ok = oracle.ipm.pcg(S, b, rtol, 1000, lambda r: d * r)
    assert ok
    assert np.linalg.norm(S @ (x - xo)) <= 3 * rtol * nb
    assert abs(res.iterations - its_o) <= 2 + 0.1 * its_o, (res.iterations, its_o)
    assert res.spmv_launches == res.iterations
    assert res.spmv_bytes == 12.0 * S.nnz + 36.0 * S.shape[0]


def test_pcg_on_the_solver_shaped_schur_of_a_grid_problem(ctx):
    """S_M of the oracle's initial support of a 16x16 problem (the solver's own
    pattern), with IPM-like theta spread over twelve orders of magnitude."""
    inst = config_instance("c1", 3)
    m, n = inst.m, inst.n
    idx, _ = oracle.initial_support(inst.xs, inst.xt, 5.0)
    rng = np.random.default_rng(5)
    theta = 10.0 ** rng.uniform(-6, 6, idx.size)
    M, N, V = oracle.normal_blocks(theta, idx % m, idx // m, m, n)
    S = oracle.schur_complement(M, N, V, "M").tocsr()
    S.sort_indices()
    ncomp, lab = oracle.ipm._components(idx % m, idx // m, m, n)
    b = rng.standard_normal(n)
    labn = lab[m:]
    b -= (np.bincount(labn, weights=b, minlength=ncomp) / np.maximum(
        np.bincount(labn, minlength=ncomp), 1))[labn]     # mean zero per component
    x, res = run(ctx, S, b, 1e-6)
    assert res.status == 0
    assert np.linalg.norm(b - S @ x) <= 1.5e-6 * np.linalg.norm(b)


def test_iteration_limit_and_degenerate_matrices(ctx):
    import paper_2206_11009_amd as otip
    S, b = schur_case(200, 300, 4, 7, spread=5.0)
    x, res = run(ctx, S, b, 1e-14, maxit=3)
    assert res.status == otip.OTIP_EMAXITER and res.iterations == 3
    # 1 x 1
    S1 = sp.csr_matrix(np.array([[4.0]]))
    x, res = run(ctx, S1, np.array([2.0]), 1e-12)
    assert res.status == 0 and x[0] == pytest.approx(0.5, rel=1e-15)
    # b = 0: converged at once, x = 0
    x, res = run(ctx, S, np.zeros(S.shape[0]), 1e-6)
    assert res.status == 0 and res.iterations == 0 and not x.any()
    # a diagonal matrix: one iteration (the Jacobi preconditioner is exact)
    D = sp.diags(np.linspace(1.0, 9.0, 777)).tocsr()
    bb = np.random.default_rng(8).standard_normal(777)
    x, res = run(ctx, D, bb, 1e-12)
    assert res.status == 0 and res.iterations == 1
    np.testing.assert_allclose(x, bb / D.diagonal(), rtol=1e-14)


@pytest.mark.parametrize("case", ["col_range", "rowptr_decreasing", "rowptr_end", "rtol"])
def test_pcg_rejects_bad_input(ctx, case):
    import paper_2206_11009_amd as otip
    import torch
    S, b = schur_case(40, 50, 3, 9)
    rp = S.indptr.astype(np.int32).copy()
    ci = S.indices.astype(np.int32).copy()
    rtol = 1e-6
    if case == "col_range":
        ci[7] = 50
    elif case == "rowptr_decreasing":
        rp[10], rp[11] = rp[11], rp[10] - 1
    elif case == "rowptr_end":
        rp[-1] -= 1
    else:
        rtol = 0.0
    with pytest.raises(otip.OtipError) as e:
        otip.otip_pcg(ctx, torch.as_tensor(rp, device="cuda:0"),
                      torch.as_tensor(ci, device="cuda:0"),
                      torch.as_tensor(S.data, device="cuda:0"), b, rtol=rtol)
    assert e.value.code == otip.OTIP_EINVAL
    x, res = run(ctx, S, b, 1e-6)      # the context is still usable
    assert res.status == 0
