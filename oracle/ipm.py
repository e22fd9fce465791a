"""CPU oracle of the interior-point-inspired column-generation method.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): plain FP64 numpy/scipy,
written from the paper, unblocked, in the paper's step order.  The HIP library
never imports this module and this module never imports the library.

Problem (Section 2.1, Kantorovich LP):  min c^T p  s.t.  A p = f = [a; b],
p >= 0, with A = [e_n^T (x) I_m ; I_n (x) e_m^T] and p = vec(P) column-wise, so
variable idx = i + j*m (0-based) moves mass from source i to target j.

One outer iteration (Section 3.2; the step order of the paper's commented
"SparseIPM" listing):

1. residuals on the support ("index"):  r1 = f - A_red p,
   r2 = c_red - A_red^T y - s,  mu = p^T s / psi                (eq. redsystem)
2. stop test (Section 3.2, end), then the a-posteriori pricing check
3. Newton direction from the normal equations (eq. normalequationsipm)
   A Theta A^T dy = r1 + A Theta (r2 - P^{-1} r3),  Theta = diag(p/s),
   solved through a Schur complement of [[M, V], [V^T, N]] (Sections 3.5, 4):
   predictor, Mehrotra corrector and Gondzio centrality correctors
   (Section 3.3)
4. step to the boundary scaled by 0.995, separately for primal and dual
5. pricing: the most negative reduced costs c - A^T y outside the support
   enter with p = s = sqrt(mu); small p leave (Section 3.2, update phase);
   at most m of each per iteration
6. iterative solver (preconditioned CG) until the support shrinks fast, then a
   direct LDL^T-type factorisation (Sections 4.2-4.3)

Readings of points the paper leaves open are the fields of ``OracleParams``;
each names the passage it settles.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.sparse.csgraph import connected_components

from . import _cscan
from .purify import purify_to_forest, forest_flows


@dataclass
class OracleParams:
    # Section 5.2: tolerances and limits used in the paper's experiments.
    tol: float = 1e-6
    cg_tol_pred: float = 1e-6
    cg_tol_corr: float = 1e-3
    max_iter: int = 200
    cg_max_iter: int = 1000
    max_corr: int = 3
    # Section 3.3: step to the boundary scaled by a constant close to 1.
    step_scale: float = 0.995
    # Section 3.2 (initial support "three to ten times" m+n-1): factor used.
    kappa: float = 5.0
    # Section 4.3: relative drop of psi over the last 5 iterations triggers the
    # switch; "sufficiently large" read as >= 10 %, and the factor must not be
    # denser than switch_fill * nnz(S).
    switch_window: int = 5
    switch_drop: float = 0.1
    switch_fill: float = 20.0
    # Section 3.3 (multiple centrality correctors, symmetric neighbourhood):
    # target box [beta_min, beta_max] * sigma*mu, trial step alpha + delta,
    # accept a corrector that raises min(alpha_p, alpha_d) by >= accept.
    mcc_beta_min: float = 0.1
    mcc_beta_max: float = 10.0
    mcc_delta: float = 0.1
    mcc_accept: float = 0.01
    # Section 3.2: removal of small p "when the IPM is near convergence":
    # near = max(rel r1, rel r2) <= remove_gate; small = p < remove_rel*min(a_i, b_j).
    remove_gate: float = 1e-3
    remove_rel: float = 1e-6
    # Section 4.2: an incomplete factorisation with a drop tolerance lowered
    # whenever a solve needs too many CG iterations, diagonal lifted for safety.
    # The paper names incomplete Cholesky; this oracle uses SuperLU's threshold
    # incomplete LU in symmetric mode (natural order, diagonal pivots) as the
    # stand-in: on the symmetric, weakly diagonally dominant Schur complement it
    # drops entries by the same threshold rule, but its factors are not exactly
    # L and L^T, hence the flexible (Polak-Ribiere) CG in ``pcg``.
    droptol0: float = 1e-2
    droptol_min: float = 1e-6
    droptol_cg_limit: int = 100
    diag_lift: float = 1e-8
    # Section 4.2: a pivot d_k <= pivot_tol * S_kk of the singular
    # factorisation is replaced by +inf ("modified Cholesky" option).
    pivot_tol: float = 1e-12
    # a-posteriori pricing check after the stop test (Section 3.2: "could also
    # check"): re-enter columns while sum(a)*|r| > cert_rel*max(1, |c^T p|).
    cert_rel: float = 1e-7
    # final primal projection onto A p = f on the support (see ``_polish``).
    polish_tol: float = 1e-12
    polish_steps: int = 4
    # after purification, flows below drop_rel * min(a_i, b_j) are taken as zero
    drop_rel: float = 1e-7
    # Inexact-Newton safeguard: the Schur residual left by CG becomes primal
    # infeasibility of the step (A dp - r1 equals it), so CG must also reach
    # ||res|| <= cg_eta * max(||r1||, cg_floor * (1 + ||f||)).  A solve that
    # cannot within cg_max_iter switches the method to the direct solver
    # (Section 4.2: CG struggles in the late, ill-conditioned iterations).
    cg_eta: float = 0.1
    cg_floor: float = 1e-9
    # "auto" = CG then switch (Section 4.3); "pcg" or "direct" force one solver.
    linear_solver: str = "auto"
    # "ic" (the incomplete factorisation above, Section 4.2) or "jacobi".
    preconditioner: str = "ic"
    # stop-test complementarity term: "relative" = psi*mu/max(1,|c^T p|);
    # "absolute" = mu exactly as printed in Section 3.2.
    stop_mu: str = "relative"
    # force the switch at this iteration (host-forced test hook); -1 = never
    force_switch_at: int = -1
    # exact power-of-two scaling of masses (mean source mass ~1) and costs
    # (largest cost <= 1) before solving; the paper is silent on scaling, and
    # its sqrt(mu) insertion presumes p and s of comparable size.
    scale: bool = True
    # cap on the number of entering columns per iteration; <= 0 means m
    # (Section 3.2: at most m variables enter or leave per iteration)
    enter_cap: int = 0
    # cost between pixels (Section 5.1): 0 squared 2-norm (this project's
    # default workload), 1 the 1-norm, 2 the 2-norm, 3 the inf-norm of the
    # integer offset (see ``costs``)
    cost_kind: int = 0
    # Section 3.4, heuristic pricing: price only J = {c < C_max} for heur_run
    # consecutive iterations, then the full vector once.  C_max scales with the
    # image side (Section 5.1) through the largest distance D between points:
    # J = pairs closer than heur_radius * D in the cost's own norm (see
    # ``heuristic_key_limit``).  0 = off (every iteration prices all m n).
    heur_radius: float = 0.0
    heur_run: int = 3
    # Section 4.3 remark: after a switch made by the support-drop rule, return
    # to CG once psi has grown by this fraction over the switch window; 0 =
    # never.  force_switch_back_at >= 0 returns at that iteration (test hook).
    switch_back_grow: float = 0.0
    force_switch_back_at: int = -1
    # Section 4.2 remark: keep the symbolic part of the factorisation (the
    # fill-reducing ordering) across support updates while the pattern of the
    # Schur complement stays inside the one it was computed for.
    reuse_ordering: bool = True


@dataclass
class OracleResult:
    status: str
    rows: np.ndarray
    cols: np.ndarray
    flows: np.ndarray
    y: np.ndarray
    z: np.ndarray
    objective: float
    dual_bound: float
    rel_gap: float
    marginal_residual: float
    r_min: float
    iterations: int
    cg_iterations: int
    direct_iterations: int
    max_fill_pct: float
    history: list = field(default_factory=list)
    switches_back: int = 0
    orderings_reused: int = 0
    seconds: float = 0.0


# ---------------------------------------------------------------------------
# Kronecker-structured products (Section 2.1) and costs
# ---------------------------------------------------------------------------

def sq_costs(xs, xt, rows, cols):
    """Integer squared Euclidean cost of the variables (rows[k], cols[k])."""
    d = xs[rows].astype(np.int64) - xt[cols].astype(np.int64)
    return (d * d).sum(axis=1)


def costs(xs, xt, rows, cols, kind=0):
    """C_ij of the variables (rows[k], cols[k]) for a cost kind of Section 5.1,
    from the integer offset d = x_i - x'_j: 0 |d|_2^2, 1 |d|_1, 2 |d|_2 (the
    correctly rounded square root of the exact integer |d|_2^2), 3 |d|_inf.
    Returned as doubles (exact for kinds 0, 1, 3)."""
    d = xs[rows].astype(np.int64) - xt[cols].astype(np.int64)
    if kind == 0:
        return (d * d).sum(axis=1).astype(np.float64)
    if kind == 1:
        return np.abs(d).sum(axis=1).astype(np.float64)
    if kind == 2:
        return np.sqrt((d * d).sum(axis=1).astype(np.float64))
    if kind == 3:
        return np.abs(d).max(axis=1).astype(np.float64)
    raise ValueError("cost kind must be 0, 1, 2 or 3")


def cost_span(xs, xt, kind=0):
    """Largest integer cost key over all pairs' bounding box: the cost itself
    for kinds 0, 1, 3 and the squared norm for kind 2 (its square root is
    increasing, so thresholds on it select the same sets)."""
    span = np.maximum(xs.max(0).astype(np.int64), xt.max(0).astype(np.int64)) - \
        np.minimum(xs.min(0).astype(np.int64), xt.min(0).astype(np.int64))
    if kind == 1:
        return int(span.sum())
    if kind == 3:
        return int(span.max())
    return int((span * span).sum())


def A_apply(vals, rows, cols, m, n):
    """A_red x: row sums (A_1 x = X e_n) and column sums (A_2 x = X^T e_m) of the
    sparse m x n array with entries vals at (rows, cols) (Section 2.1)."""
    return (np.bincount(rows, weights=vals, minlength=m),
            np.bincount(cols, weights=vals, minlength=n))


def AT_apply(y, z, rows, cols):
    """A_red^T [y; z]: entry (i, j) is y_i + z_j (A_1^T u = vec(u e_n^T),
    A_2^T w = vec(e_m w^T), Section 2.1)."""
    return y[rows] + z[cols]


def normal_blocks(theta, rows, cols, m, n):
    """Blocks of A Theta A^T = [[M, V], [V^T, N]] (Section 3.5, eq. normaleq):
    vec(V) = theta on the support, M and N the row and column sums of V."""
    M = np.bincount(rows, weights=theta, minlength=m)
    N = np.bincount(cols, weights=theta, minlength=n)
    V = sp.csr_matrix((theta, (rows, cols)), shape=(m, n))
    return M, N, V


def schur_complement(M, N, V, side):
    """S_M = N - V^T M^-1 V (side 'M') or S_N = M - V N^-1 V^T (side 'N')
    (Section 4)."""
    if side == "M":
        return (sp.diags(N) - V.T @ sp.diags(1.0 / M) @ V).tocsr()
    return (sp.diags(M) - V @ sp.diags(1.0 / N) @ V.T).tocsr()


# ---------------------------------------------------------------------------
# Linear solvers for the Schur system (Section 4.2)
# ---------------------------------------------------------------------------

class SchurSolver:
    """Holds one iteration's Schur complement and solves with it.

    The Schur complement is singular (rank deficient by one per connected
    component of the support graph, Section 4).  For CG the right-hand side is
    projected onto the range (mean-zero on every component) before solving.
    """

    def __init__(self, S, comp, ncomp, mode, params, droptol, factor=None, cache=None):
        self.S = S
        self.comp = comp
        self.ncomp = ncomp
        self.mode = mode
        self.params = params
        self.cg_iters = 0
        self.max_cg_in_solve = 0
        self.fill = 0.0
        self.lu = factor
        self.prec = None
        self.failed = False
        n = S.shape[0]
        if mode == "direct":
            if self.lu is None:
                self.lu = direct_factor(S, params.pivot_tol, cache)
            self.fill = 100.0 * self.lu.nnz_L / float(n * n)
        else:
            if params.preconditioner == "ic":
                d = S.diagonal()
                Sl = (S + sp.diags(params.diag_lift * d)).tocsc()
                self.prec = spla.spilu(Sl, drop_tol=droptol, fill_factor=50.0,
                                       permc_spec="NATURAL", diag_pivot_thresh=0.0,
                                       options=dict(SymmetricMode=True))
            else:
                self.dinv = 1.0 / S.diagonal()

    def _project(self, r):
        if self.ncomp == 1:
            return r - r.mean()
        sums = np.bincount(self.comp, weights=r, minlength=self.ncomp)
        cnt = np.bincount(self.comp, minlength=self.ncomp)
        return r - (sums / cnt)[self.comp]

    def _apply_prec(self, r):
        if self.prec is not None:
            return self.prec.solve(r)
        return self.dinv * r

    def solve(self, rhs, tol, atol=math.inf):
        if self.mode == "direct":
            x = self.lu.solve(rhs)
            # one step of iterative refinement against the unshifted matrix
            x = x + self.lu.solve(rhs - self.S @ x)
            return x
        b = self._project(rhs)
        x, its, ok = pcg(self.S, b, tol, self.params.cg_max_iter, self._apply_prec, atol)
        self.cg_iters += its
        self.max_cg_in_solve = max(self.max_cg_in_solve, its)
        if not ok:
            self.failed = True
        return x


def min_degree_order(S):
    """Fill-reducing symmetric ordering: SuperLU's multiple minimum degree on
    the pattern of S (a library ordering stands in for the paper's AMD; any
    ordering gives the same solution up to rounding)."""
    n = S.shape[0]
    P = S.tocsr().copy()
    P.data = np.full(P.data.shape, -1.0)
    P = P - sp.diags(P.diagonal()) + sp.diags(np.asarray(abs(P).sum(1)).ravel() + 1.0)
    lu = spla.splu(P.tocsc(), permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    return np.argsort(lu.perm_c)


def direct_factor(S, pivtol, cache=None):
    """Exact L D L^T of the Schur complement after a minimum-degree ordering,
    with the infinite-pivot rule for vanishing pivots (Section 4.2).  With a
    cache (a dict), the ordering of an earlier factorisation is reused while the
    pattern of S lies inside the pattern it was computed for (the remark of
    Section 4.2 on updating the symbolic factorisation instead of redoing it):
    any symmetric ordering gives the same factorisation up to rounding, and one
    computed for a superset pattern gives no more fill than on that superset."""
    pat = S.tocsr().copy()
    pat.data = np.ones_like(pat.data)
    if cache is not None and cache.get("pattern") is not None and \
            cache["pattern"].shape == pat.shape and \
            (pat - pat.multiply(cache["pattern"])).count_nonzero() == 0:
        cache["reused"] = cache.get("reused", 0) + 1
        return _cscan.LDL(S, cache["perm"], pivtol)
    perm = min_degree_order(S)
    if cache is not None:
        cache["pattern"], cache["perm"] = pat, perm
    return _cscan.LDL(S, perm, pivtol)


def pcg(S, b, tol, maxit, prec, atol=math.inf):
    """Preconditioned CG (flexible Polak-Ribiere form, robust to the slight
    asymmetry of a threshold incomplete factorisation); stops when
    ||b - S x|| <= min(tol * ||b||, atol).  Returns (x, iterations, converged)."""
    x = np.zeros_like(b)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, True
    target = min(tol * nb, atol)
    r = b.copy()
    zv = prec(r)
    d = zv.copy()
    rz = r @ zv
    its = 0
    while its < maxit:
        q = S @ d
        dq = d @ q
        if not dq > 0.0:
            break
        alpha = rz / dq
        x += alpha * d
        r_old = r
        r = r - alpha * q
        its += 1
        if np.linalg.norm(r) <= target:
            return x, its, True
        zn = prec(r)
        rz_new = r @ zn
        if rz == 0.0:
            break
        beta = (zn @ (r - r_old)) / rz
        rz = rz_new
        d = zn + beta * d
    return x, its, bool(np.linalg.norm(r) <= target)


# ---------------------------------------------------------------------------
# The method
# ---------------------------------------------------------------------------

def heuristic_key_limit(xs, xt, radius, kind=0):
    """Integer bound L of the heuristic subset J = {cost key < L} (Section 3.4).
    The cost key is the cost itself, or the squared norm for the 2-norm.  With
    D the largest distance between points in the cost's norm, J holds the pairs
    closer than radius * D: for the squared and 2-norm costs the key is the
    squared 2-norm, so L = ceil(radius^2 * Dsq) (Dsq the largest squared
    distance); for the 1- and inf-norm L = ceil(radius * D).  Double arithmetic
    left to right, then the ceiling: for an integer key k and real t, k < t if
    and only if k < ceil(t)."""
    span = float(cost_span(xs, xt, kind))
    if kind in (0, 2):
        return int(math.ceil(radius * radius * span))
    return int(math.ceil(radius * span))


def initial_support(xs, xt, kappa, kind=0):
    """Section 3.2 (end): the variables of small cost, about kappa*(m+n-1) of
    them -- all (i, j) with c_ij <= T for the smallest integer T reaching that
    count -- plus the cheapest target of every source and the cheapest source of
    every target so that every row and column of the plan is covered.  For the
    2-norm the threshold is on the squared norm (the same sets)."""
    m, n = xs.shape[0], xt.shape[0]
    target = int(math.ceil(kappa * (m + n - 1)))
    cmax = cost_span(xs, xt, kind)
    hist = _cscan.cost_hist(xs, xt, cmax, kind)
    cum = np.cumsum(hist)
    T = int(np.searchsorted(cum, min(target, m * n)))
    base = _cscan.collect_le(xs, xt, T, int(cum[T]), kind)
    ra, ca = _cscan.row_col_argmin(xs, xt, kind)
    extra = np.concatenate([np.arange(m) + ra * m, ca + np.arange(n) * m])
    return np.unique(np.concatenate([base, extra])), T


def _max_step(x, dx):
    neg = dx < 0.0
    if not neg.any():
        return math.inf
    return float(np.min(-x[neg] / dx[neg]))


class _State:
    kind = 0  # cost kind (squared Euclidean unless the solve sets another)


def _components(rows, cols, m, n):
    g = sp.csr_matrix((np.ones(rows.shape[0]), (rows, m + cols)), shape=(m + n, m + n))
    ncomp, lab = connected_components(g, directed=False)
    return ncomp, lab


def _build_system(st, theta, mode, params, factor=None):
    m, n = st.m, st.n
    M, N, V = normal_blocks(theta, st.rows, st.cols, m, n)
    side = "M" if n <= m else "N"
    S = schur_complement(M, N, V, side)
    ncomp, lab = _components(st.rows, st.cols, m, n)
    comp = lab[m:] if side == "M" else lab[:m]
    # relabel compactly
    _, comp = np.unique(comp, return_inverse=True)
    cache = getattr(st, "symbolic", None) if params.reuse_ordering else None
    solver = SchurSolver(S, comp, int(comp.max()) + 1, mode, params, st.droptol, factor, cache)
    return M, N, V, side, solver


def _newton(st, sys, r1a, r1b, r2, r3, tol, atol=math.inf):
    """Solve eq. redsystem through the normal equations and a Schur complement
    (Sections 3.1, 3.5, 4).  Returns (dp, dy, dz, ds)."""
    M, N, V, side, solver = sys
    w = st.theta * (r2 - r3 / st.p)
    wa, wb = A_apply(w, st.rows, st.cols, st.m, st.n)
    beta1 = r1a + wa
    beta2 = r1b + wb
    if side == "M":
        dz = solver.solve(beta2 - V.T @ (beta1 / M), tol, atol)
        dy = (beta1 - V @ dz) / M
    else:
        dy = solver.solve(beta1 - V @ (beta2 / N), tol, atol)
        dz = (beta2 - V.T @ dy) / N
    ds = r2 - AT_apply(dy, dz, st.rows, st.cols)
    dp = (r3 - st.p * ds) / st.s
    return dp, dy, dz, ds


def _steps(st, dp, ds, scale):
    ap = min(1.0, scale * _max_step(st.p, dp))
    ad = min(1.0, scale * _max_step(st.s, ds))
    return ap, ad


def _starting_point(st, params):
    """Mehrotra's starting-point heuristic on the restricted LP (Theta = I):
    least-norm p~ with A p~ = f, least-squares duals for c, then shifts that make
    p and s positive and balanced.  The paper leaves the starting point open."""
    ones = np.ones(st.psi)
    st.theta = ones
    sys = _build_system(st, ones, "direct", params)
    M, N, V, side, solver = sys

    def normal_solve(b1, b2):
        if side == "M":
            dz = solver.solve(b2 - V.T @ (b1 / M), 0.0)
            dy = (b1 - V @ dz) / M
        else:
            dy = solver.solve(b1 - V @ (b2 / N), 0.0)
            dz = (b2 - V.T @ dy) / N
        return dy, dz

    wy, wz = normal_solve(st.a, st.b)
    pt = AT_apply(wy, wz, st.rows, st.cols)
    ca, cb = A_apply(st.c, st.rows, st.cols, st.m, st.n)
    ly, lz = normal_solve(ca, cb)
    stil = st.c - AT_apply(ly, lz, st.rows, st.cols)
    dp = max(-1.5 * pt.min(), 0.0)
    dsv = max(-1.5 * stil.min(), 0.0)
    ph = pt + dp
    sh = stil + dsv
    ps = float(ph @ sh)
    dph = 0.5 * ps / sh.sum() if sh.sum() > 0 else 0.0
    dsh = 0.5 * ps / ph.sum() if ph.sum() > 0 else 0.0
    p = ph + dph
    s = sh + dsh
    # a degenerate start (all products zero) gets a unit shift
    if not (p.min() > 0 and s.min() > 0):
        p = np.maximum(p, 1e-8 * max(1.0, np.abs(p).max()))
        s = np.maximum(s, 1e-8 * max(1.0, np.abs(s).max()))
    st.p, st.s, st.y, st.z = p, s, ly, lz


def _set_support(st, idx, p, s):
    order = np.argsort(idx, kind="stable")
    st.idx = idx[order]
    st.p = p[order]
    st.s = s[order]
    st.rows = st.idx % st.m
    st.cols = st.idx // st.m
    st.c = costs(st.xs, st.xt, st.rows, st.cols, st.kind) * st.zeta
    st.psi = st.idx.shape[0]


def _polish(st, params):
    """Final primal projection onto A p = f restricted to the support: the
    Newton step with r2 = r3 = 0 and unit primal step, dp = Theta A^T (A Theta A^T)^-1 r1,
    repeated until ||A p - f||_1 / ||f||_1 <= polish_tol."""
    for _ in range(params.polish_steps):
        ra, rb = A_apply(st.p, st.rows, st.cols, st.m, st.n)
        r1a, r1b = st.a - ra, st.b - rb
        rel = (np.abs(r1a).sum() + np.abs(r1b).sum()) / (st.a.sum() + st.b.sum())
        if rel <= params.polish_tol:
            break
        st.theta = st.p / st.s
        sys = _build_system(st, st.theta, "direct", params)
        M, N, V, side, solver = sys
        if side == "M":
            dz = solver.solve(r1b - V.T @ (r1a / M), 0.0)
            dy = (r1a - V @ dz) / M
        else:
            dy = solver.solve(r1a - V @ (r1b / N), 0.0)
            dz = (r1b - V.T @ dy) / N
        st.p = np.maximum(st.p + st.theta * AT_apply(dy, dz, st.rows, st.cols), 0.0)


def solve(a, b, xs, xt, params: OracleParams | None = None, log=None) -> OracleResult:
    """Solve the Kantorovich LP with the cost of ``params.cost_kind`` (default
    squared Euclidean) between integer coordinates xs (m x 2) and xt (n x 2),
    marginals a and b (sum a = sum b)."""
    P = params or OracleParams()
    t0 = time.perf_counter()
    st = _State()
    st.kind = int(P.cost_kind)
    if st.kind not in (0, 1, 2, 3):
        raise ValueError("cost kind must be 0, 1, 2 or 3")
    st.a = np.asarray(a, np.float64)
    st.b = np.asarray(b, np.float64)
    st.xs = np.ascontiguousarray(xs, np.int32)
    st.xt = np.ascontiguousarray(xt, np.int32)
    st.m, st.n = st.a.shape[0], st.b.shape[0]
    m, n = st.m, st.n
    if not (np.all(st.a > 0) and np.all(st.b > 0)):
        raise ValueError("marginals must be strictly positive")
    if abs(st.a.sum() - st.b.sum()) > 1e-12 * st.a.sum():
        raise ValueError("sum(a) != sum(b)")
    st.droptol = P.droptol0
    # exact power-of-two scaling: p_s = omega p, c_s = zeta c, duals y_s = zeta y
    st.omega, st.zeta = 1.0, 1.0
    if P.scale:
        cmax = max(1.0, float(cost_span(st.xs, st.xt, st.kind)))
        if st.kind == 2:
            cmax = max(1.0, math.sqrt(cmax))
        st.omega = 2.0 ** round(math.log2(m / st.a.sum()))
        st.zeta = 2.0 ** -math.ceil(math.log2(cmax))
        st.a = st.a * st.omega
        st.b = st.b * st.omega
    f_norm = math.sqrt(float(st.a @ st.a + st.b @ st.b))
    kcap = m if P.enter_cap <= 0 else P.enter_cap

    st.heur_limit = heuristic_key_limit(st.xs, st.xt, P.heur_radius, st.kind) \
        if P.heur_radius > 0.0 else 0
    st.symbolic = {}
    st.forced_switch_done = st.forced_back_done = st.switched_by_drop = False
    st.switches_back = 0
    idx0, _T = initial_support(st.xs, st.xt, P.kappa, st.kind)
    _set_support(st, idx0, np.ones(idx0.shape[0]), np.ones(idx0.shape[0]))
    _starting_point(st, P)

    mode = "direct" if P.linear_solver == "direct" else "pcg"
    psi_hist = []
    hist = []
    cg_total = 0
    direct_its = 0
    max_fill = 0.0
    status = "maxiter"
    cg_failed = False
    it = 0
    tol_int = P.tol
    while True:
        status, it, cg_failed, mode, cg_total, direct_its, max_fill = _iterate(
            st, P, tol_int, it, mode, psi_hist, hist, cg_total, direct_its, max_fill, cg_failed,
            f_norm, kcap, log)
        result = _finalize(st, P, status, it, cg_total, direct_its, max_fill, hist, t0)
        # the certified gap decides: tighten the internal tolerance and resume
        if result.rel_gap <= P.tol or it >= P.max_iter or tol_int <= 1e-13:
            if result.rel_gap > P.tol:
                result.status = "maxiter"
            return result
        tol_int = max(tol_int * 0.1, 1e-13)


def _iterate(st, P, tol_int, it, mode, psi_hist, hist, cg_total, direct_its, max_fill, cg_failed,
             f_norm, kcap, log):
    """Outer iterations from `it` until the stop test passes (and the
    a-posteriori pricing finds nothing significant) or max_iter."""
    m, n = st.m, st.n
    status = "maxiter"
    while it < P.max_iter:
        # 1. residuals of eq. redsystem
        ra, rb = A_apply(st.p, st.rows, st.cols, m, n)
        r1a, r1b = st.a - ra, st.b - rb
        r2 = st.c - AT_apply(st.y, st.z, st.rows, st.cols) - st.s
        mu = float(st.p @ st.s) / st.psi
        prim = float(st.c @ st.p)
        rel1 = math.sqrt(float(r1a @ r1a + r1b @ r1b)) / (1.0 + f_norm)
        rel2 = float(np.linalg.norm(r2)) / (1.0 + float(np.linalg.norm(st.c)))
        relmu = st.psi * mu / max(1.0, abs(prim)) if P.stop_mu == "relative" else mu
        psi_hist.append(st.psi)
        rec = dict(it=it, psi=st.psi, mu=mu, rel_r1=rel1, rel_r2=rel2, rel_mu=relmu,
                   solver=mode, primal=prim)
        hist.append(rec)
        # 2. stop test, then the a-posteriori pricing check
        if max(rel1, rel2, relmu) < tol_int:
            sel, rsel, _ = _cscan.price(st.xs, st.xt, st.y / st.zeta, st.z / st.zeta,
                                        st.idx, kcap, st.kind)
            big = np.abs(rsel * st.zeta) * st.a.sum() > P.cert_rel * max(1.0, abs(prim))
            if not big.any():
                return "optimal", it + 1, cg_failed, mode, cg_total, direct_its, max_fill
            sm = math.sqrt(mu)
            rec["cert_added"] = int(big.sum())
            _set_support(st, np.concatenate([st.idx, sel[big]]),
                         np.concatenate([st.p, np.full(int(big.sum()), sm)]),
                         np.concatenate([st.s, np.full(int(big.sum()), sm)]))
            it += 1
            continue
        # 6a. switch back to CG (remark of Section 4.3)
        factor = None
        just_back = False
        if mode == "direct" and P.linear_solver == "auto":
            w = P.switch_window
            back = None
            if P.force_switch_back_at >= 0 and it >= P.force_switch_back_at \
                    and not st.forced_back_done:
                st.forced_back_done = True
                back = "forced"
            elif P.switch_back_grow > 0.0 and st.switched_by_drop and len(psi_hist) > w and \
                    (psi_hist[-1] - psi_hist[-1 - w]) / psi_hist[-1 - w] >= P.switch_back_grow:
                back = "support growing"
            if back:
                mode = "pcg"
                st.switched_by_drop = False
                st.switches_back += 1
                cg_failed = False
                just_back = True
                rec["switch_back"] = back
        # 6b. switch test (Section 4.3)
        if mode == "pcg" and not just_back and P.linear_solver == "auto":
            w = P.switch_window
            forced = P.force_switch_at >= 0 and it >= P.force_switch_at and \
                not st.forced_switch_done
            force = forced or cg_failed
            drop_ok = len(psi_hist) > w and \
                (psi_hist[-1 - w] - psi_hist[-1]) / psi_hist[-1 - w] >= P.switch_drop
            if force or drop_ok:
                st.theta = st.p / st.s
                M_, N_, V_ = normal_blocks(st.theta, st.rows, st.cols, m, n)
                S_ = schur_complement(M_, N_, V_, "M" if n <= m else "N")
                lu = direct_factor(S_, P.pivot_tol,
                                   st.symbolic if P.reuse_ordering else None)
                nnz_lower = (S_.nnz + S_.shape[0]) / 2.0
                if force or lu.nnz_L <= P.switch_fill * nnz_lower:
                    mode = "direct"
                    factor = lu
                    st.forced_switch_done = st.forced_switch_done or forced
                    st.switched_by_drop = not force
        # 3. Newton direction
        st.theta = st.p / st.s
        sys = _build_system(st, st.theta, mode, P, factor)
        solver = sys[4]
        # predictor (affine scaling, sigma = 0)
        r3 = -st.p * st.s
        r1n = math.sqrt(float(r1a @ r1a + r1b @ r1b))
        atol = P.cg_eta * max(r1n, P.cg_floor * (1.0 + f_norm))
        dpa, dya, dza, dsa = _newton(st, sys, r1a, r1b, r2, r3, P.cg_tol_pred, atol)
        apa, ada = _steps(st, dpa, dsa, 1.0)
        apa, ada = min(1.0, apa), min(1.0, ada)
        mu_aff = float((st.p + apa * dpa) @ (st.s + ada * dsa)) / st.psi
        sigma = (mu_aff / mu) ** 3 if mu > 0 else 0.0
        # Mehrotra corrector
        r3 = sigma * mu - st.p * st.s - dpa * dsa
        dp, dy, dz, ds = _newton(st, sys, r1a, r1b, r2, r3, P.cg_tol_pred, atol)
        ap, ad = _steps(st, dp, ds, P.step_scale)
        # Gondzio multiple centrality correctors
        ncorr = 0
        zero_m = np.zeros(m)
        zero_n = np.zeros(n)
        zero_psi = np.zeros(st.psi)
        while ncorr < P.max_corr and min(ap, ad) < 1.0:
            atp = min(1.0, ap + P.mcc_delta)
            atd = min(1.0, ad + P.mcc_delta)
            v = (st.p + atp * dp) * (st.s + atd * ds)
            lo, hi = P.mcc_beta_min * sigma * mu, P.mcc_beta_max * sigma * mu
            rc = np.clip(v, lo, hi) - v
            rc = np.maximum(rc, -hi)
            cdp, cdy, cdz, cds = _newton(st, sys, zero_m, zero_n, zero_psi, rc,
                                         P.cg_tol_corr, atol)
            ndp, ndy, ndz, nds = dp + cdp, dy + cdy, dz + cdz, ds + cds
            nap, nad = _steps(st, ndp, nds, P.step_scale)
            if min(nap, nad) >= min(ap, ad) + P.mcc_accept:
                dp, dy, dz, ds, ap, ad = ndp, ndy, ndz, nds, nap, nad
                ncorr += 1
            else:
                break
        cg_total += solver.cg_iters
        cg_failed = solver.failed
        if mode == "direct":
            direct_its += 1
            max_fill = max(max_fill, solver.fill)
        elif solver.max_cg_in_solve > P.droptol_cg_limit:
            st.droptol = max(P.droptol_min, st.droptol / 10.0)
        rec.update(alpha_p=ap, alpha_d=ad, sigma=sigma, ncorr=ncorr, cg=solver.cg_iters)
        # 4. update
        st.p = st.p + ap * dp
        st.s = st.s + ad * ds
        st.y = st.y + ad * dy
        st.z = st.z + ad * dz
        mu_new = float(st.p @ st.s) / st.psi
        # 5. pricing and support update; heuristic pricing (Section 3.4):
        # iterations it with it mod (heur_run + 1) < heur_run scan only J
        heur = P.heur_radius > 0.0 and it % (P.heur_run + 1) < P.heur_run
        sel, rsel, nneg = _cscan.price(st.xs, st.xt, st.y / st.zeta, st.z / st.zeta,
                                       st.idx, kcap, st.kind,
                                       st.heur_limit if heur else 0)
        keep = np.ones(st.psi, dtype=bool)
        if max(rel1, rel2) <= P.remove_gate:
            thr = P.remove_rel * np.minimum(st.a[st.rows], st.b[st.cols])
            cand = np.nonzero(st.p < thr)[0]
            cand = cand[np.lexsort((st.idx[cand], st.p[cand]))]
            rdeg = np.bincount(st.rows, minlength=m)
            cdeg = np.bincount(st.cols, minlength=n)
            removed = 0
            for e in cand.tolist():
                if removed >= m:
                    break
                i, j = st.rows[e], st.cols[e]
                if rdeg[i] > 1 and cdeg[j] > 1:
                    keep[e] = False
                    rdeg[i] -= 1
                    cdeg[j] -= 1
                    removed += 1
        sm = math.sqrt(mu_new)
        k = sel.shape[0]
        rec.update(added=int(k), removed=int((~keep).sum()), n_negative=nneg, heuristic=heur)
        _set_support(st, np.concatenate([st.idx[keep], sel]),
                     np.concatenate([st.p[keep], np.full(k, sm)]),
                     np.concatenate([st.s[keep], np.full(k, sm)]))
        if log:
            log(rec)
        it += 1
    return status, it, cg_failed, mode, cg_total, direct_its, max_fill


def _finalize(st, P, status, it, cg_total, direct_its, max_fill, hist, t0):
    """Final primal projection, purification to a basic plan, dual certificate.
    Leaves the iterate scaled and usable for further iterations."""
    m, n = st.m, st.n
    saved = (st.a, st.b, st.p, st.y, st.z)
    _polish(st, P)
    saved = (st.a, st.b, st.p.copy(), st.y, st.z)
    # undo the scaling
    a, b = st.a / st.omega, st.b / st.omega
    pu = st.p / st.omega
    yu, zu = st.y / st.zeta, st.z / st.zeta
    st.a, st.b, st.p, st.y, st.z = saved
    # purification to a basic plan: first with numerically-zero flows removed
    # before any cycle is cancelled (fast); if the forest's exact flows are not
    # nonnegative, again with every positive flow
    for predrop in (True, False):
        keep = pu > 0.0
        if predrop:
            keep &= pu >= P.drop_rel * np.minimum(a[st.rows], b[st.cols])
        rows, cols, flows = purify_to_forest(st.rows[keep], st.cols[keep], pu[keep],
                                             costs(st.xs, st.xt, st.rows[keep],
                                                   st.cols[keep], st.kind), m, n)
        # the forest's flows as the marginals determine them, kept only if
        # they stay nonnegative
        big = flows >= P.drop_rel * np.minimum(a[rows], b[cols])
        exact, _imb = forest_flows(rows[big], cols[big], a, b)
        if exact.size and exact.min() >= -1e-12 * exact.max():
            rows, cols, flows = rows[big], cols[big], np.maximum(exact, 0.0)
            break
    order = np.argsort(rows + cols * m, kind="stable")
    rows, cols, flows = rows[order], cols[order], flows[order]
    cvals = costs(st.xs, st.xt, rows, cols, st.kind)
    objective = math.fsum((cvals * flows).tolist())
    suma = a.sum()

    def bound(yv, zv):
        rm, _ = _cscan.rmin(st.xs, st.xt, yv, zv, st.kind)
        return math.fsum((a * yv).tolist()) + math.fsum((b * zv).tolist()) + suma * min(0.0, rm), rm

    # gauge: z_{n-1} = 0 (adding t to y and -t to z leaves c - A^T y unchanged)
    g = zu[n - 1]
    y = yu + g
    z = zu - g
    dual, r_min = bound(y, z)
    # dual recovery after termination (Section 3.3): duals of the basic plan,
    # y_i + z_j = C_ij on its forest edges, each tree anchored at the
    # interior-point dual of its smallest node; kept if their bound is stronger
    yb, zb = basis_duals(rows, cols, cvals, y, z, m, n)
    dual_b, r_min_b = bound(yb, zb)
    if dual_b > dual:
        y, z, dual, r_min = yb, zb, dual_b, r_min_b
    ra, rb = A_apply(flows, rows, cols, m, n)
    marg = (np.abs(ra - a).sum() + np.abs(rb - b).sum()) / (a.sum() + b.sum())
    rel_gap = (objective - dual) / max(1.0, abs(objective))
    return OracleResult(status=status, rows=rows, cols=cols, flows=flows, y=y, z=z,
                        objective=objective, dual_bound=dual, rel_gap=rel_gap,
                        marginal_residual=float(marg), r_min=r_min, iterations=it,
                        cg_iterations=cg_total, direct_iterations=direct_its,
                        max_fill_pct=max_fill, history=hist,
                        switches_back=st.switches_back,
                        orderings_reused=st.symbolic.get("reused", 0),
                        seconds=time.perf_counter() - t0)


def basis_duals(rows, cols, costs, y0, z0, m, n):
    """Duals of a basic plan: y_i + z_j = C_ij on every edge of its forest; the
    smallest node of each tree keeps its value from (y0, z0); gauge z_{n-1} = 0."""
    pot = np.concatenate([y0, z0]).astype(np.float64)
    adj = [[] for _ in range(m + n)]
    for k, (i, j) in enumerate(zip(rows.tolist(), cols.tolist())):
        adj[i].append((m + j, k))
        adj[m + j].append((i, k))
    seen = np.zeros(m + n, bool)
    for r in range(m + n):
        if seen[r]:
            continue
        seen[r] = True
        stack = [r]
        while stack:
            u = stack.pop()
            for v, k in adj[u]:
                if not seen[v]:
                    seen[v] = True
                    pot[v] = costs[k] - pot[u]
                    stack.append(v)
    g = pot[m + n - 1]
    return pot[:m] + g, pot[m:] - g
