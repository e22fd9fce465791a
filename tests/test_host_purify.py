"""The library's host purification (csrc/purify.cpp, built here with g++ and
called through a small C wrapper) against the oracle's purification of the
same plan.  Both implement one reading of Section 2.2 (maximum-flow spanning
forest, cycle cancelling in the cost non-increasing direction with the
non-forest edge decreasing on a tie, bottleneck at the lowest variable index,
then the forest's flows from the marginals by leaf elimination), so the basic
plans must agree: same support, flows to rounding.  Plans are mixtures of
vertex plans, so they have many cycles, and the integer costs of the 1- and
inf-norms make most cycle costs exactly zero."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from oracle.purify import forest_flows, purify_to_forest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2206_11009_amd", "csrc", "purify.cpp")

WRAPPER = r"""
#include <cstddef>
#include <cstdint>
#include <vector>
namespace otip {
void purify_plan(int m, int n, const std::vector<int32_t> &rows, const std::vector<int32_t> &cols,
                 const std::vector<double> &flows, const std::vector<double> &costs,
                 const std::vector<double> &a, const std::vector<double> &b, double drop_rel,
                 std::vector<int32_t> &orows, std::vector<int32_t> &ocols,
                 std::vector<double> &oflows);
}
extern "C" int64_t purify_c(int m, int n, int64_t k, const int32_t *rows, const int32_t *cols,
                            const double *flows, const double *costs, const double *a,
                            const double *b, double drop_rel, int32_t *orow, int32_t *ocol,
                            double *oflow) {
    std::vector<int32_t> r(rows, rows + k), c(cols, cols + k), R, C;
    std::vector<double> f(flows, flows + k), w(costs, costs + k), av(a, a + m), bv(b, b + n), F;
    otip::purify_plan(m, n, r, c, f, w, av, bv, drop_rel, R, C, F);
    for (std::size_t q = 0; q < F.size(); ++q) {
        orow[q] = R[q];
        ocol[q] = C[q];
        oflow[q] = F[q];
    }
    return (int64_t)F.size();
}
"""


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("purify")
    w = d / "wrapper.cpp"
    w.write_text(WRAPPER)
    so = d / "libpurify_host.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", str(so), str(w), SRC],
                   check=True)
    L = ctypes.CDLL(str(so))
    L.purify_c.restype = ctypes.c_int64
    return L


def library(L, rows, cols, flows, costs, a, b, drop_rel=1e-7):
    m, n, k = len(a), len(b), len(flows)
    i32 = lambda x: np.ascontiguousarray(x, np.int32)
    f64 = lambda x: np.ascontiguousarray(x, np.float64)
    r, c, f, w, av, bv = i32(rows), i32(cols), f64(flows), f64(costs), f64(a), f64(b)
    orow = np.empty(m + n + k, np.int32)
    ocol = np.empty(m + n + k, np.int32)
    ofl = np.empty(m + n + k, np.float64)
    p = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    cnt = L.purify_c(m, n, ctypes.c_int64(k), p(r), p(c), p(f), p(w), p(av), p(bv),
                     ctypes.c_double(drop_rel), p(orow), p(ocol), p(ofl))
    return orow[:cnt], ocol[:cnt], ofl[:cnt]


def oracle_plan(rows, cols, flows, costs, a, b, drop_rel=1e-7):
    """The oracle's final purification steps (as its solve takes them)."""
    m = len(a)
    for predrop in (True, False):
        keep = flows > 0.0
        if predrop:
            keep &= flows >= drop_rel * np.minimum(a[rows], b[cols])
        r, c, f = purify_to_forest(rows[keep], cols[keep], flows[keep], costs[keep], m, len(b))
        big = f >= drop_rel * np.minimum(a[r], b[c])
        exact, _ = forest_flows(r[big], c[big], a, b)
        if exact.size and exact.min() >= -1e-12 * exact.max():
            r, c, f = r[big], c[big], np.maximum(exact, 0.0)
            break
    order = np.argsort(r + c.astype(np.int64) * m, kind="stable")
    return r[order], c[order], f[order]


def mixture_plan(rng, a, b, parts):
    """A convex combination of north-west-corner plans on random orderings of
    rows and columns: feasible for (a, b), with many cycles."""
    m, n = len(a), len(b)
    P = np.zeros((m, n))
    wts = rng.uniform(0.5, 1.0, parts)
    wts /= wts.sum()
    for w in wts:
        ia, ib = rng.permutation(m), rng.permutation(n)
        aa, bb = a[ia].copy(), b[ib].copy()
        i = j = 0
        while i < m and j < n:
            t = min(aa[i], bb[j])
            P[ia[i], ib[j]] += w * t
            aa[i] -= t
            bb[j] -= t
            if aa[i] <= 1e-300:
                i += 1
            else:
                j += 1
    r, c = np.nonzero(P)
    return r.astype(np.int64), c.astype(np.int64), P[r, c]


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_host_purification_matches_oracle(lib, kind, seed):
    rng = np.random.default_rng(300 + 10 * kind + seed)
    m, n = int(rng.integers(8, 40)), int(rng.integers(8, 40))
    xs = rng.integers(0, 6, (m, 2)).astype(np.int32)   # few distinct offsets: many cost ties
    xt = rng.integers(0, 6, (n, 2)).astype(np.int32)
    a = rng.uniform(0.2, 1.0, m)
    a /= a.sum()
    b = rng.uniform(0.2, 1.0, n)
    b /= b.sum()
    rows, cols, flows = mixture_plan(rng, a, b, 6)
    costs = oracle.costs(xs, xt, rows, cols, kind)
    r1, c1, f1 = library(lib, rows, cols, flows, costs, a, b)
    r2, c2, f2 = oracle_plan(rows, cols, flows, costs, a, b)
    assert len(r1) <= m + n - 1 and oracle.is_forest(r1, c1, m, n)
    np.testing.assert_array_equal(r1, r2)
    np.testing.assert_array_equal(c1, c2)
    np.testing.assert_allclose(f1, f2, rtol=1e-13, atol=1e-16)
    # marginals kept, cost not raised
    np.testing.assert_allclose(np.bincount(r1, weights=f1, minlength=m), a, atol=1e-14)
    np.testing.assert_allclose(np.bincount(c1, weights=f1, minlength=n), b, atol=1e-14)
    c_in = float(costs @ flows)
    c_out = float(oracle.costs(xs, xt, r1, c1, kind) @ f1)
    assert c_out <= c_in * (1 + 1e-12) + 1e-15


def test_host_purification_of_a_basic_plan_is_the_identity(lib):
    """A plan that is already a forest comes back unchanged (order by index)."""
    rng = np.random.default_rng(7)
    m, n = 15, 11
    a = rng.uniform(0.1, 1.0, m)
    a /= a.sum()
    b = rng.uniform(0.1, 1.0, n)
    b /= b.sum()
    rows, cols, flows = mixture_plan(rng, a, b, 1)
    costs = rng.uniform(0, 5, rows.size)
    r1, c1, f1 = library(lib, rows, cols, flows, costs, a, b)
    order = np.argsort(rows + cols * m)
    np.testing.assert_array_equal(r1, rows[order])
    np.testing.assert_array_equal(c1, cols[order])
    np.testing.assert_allclose(f1, flows[order], rtol=1e-12, atol=1e-16)
