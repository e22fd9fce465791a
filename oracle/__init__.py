"""Reference oracle for the interior-point-inspired column-generation method
for discrete optimal transport (Zanetti & Gondzio, arXiv 2206.11009).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import, call or link anything in this package.  The HIP
library is independent of it: the two share no code, no headers and no
constants; only the seeded input generators in ``synthetic`` feed both.

Contents
--------
* ``ipm``     -- the method in plain FP64 numpy/scipy, in the paper's step order
                 (Sections 2-4), with kernel-level pieces (Kronecker products,
                 normal-matrix blocks, Schur complement, Newton direction).
* ``scan.c``  -- plain C loops over all m*n variables: pricing with a bounded
                 heap, the full reduced-cost minimum, cost histograms
                 (loaded through ``_cscan``).
* ``purify``  -- cycle cancelling of a plan to an acyclic (basic) support.

Every function cites the passage it follows.  Each is pinned by the CPU tests
to something other than itself (closed forms, brute force, library LP solvers,
the paper's identities); see ``tests/test_oracle_pins.py``.
"""
from . import _cscan  # noqa: F401
from .ipm import (OracleParams, OracleResult, solve, initial_support, sq_costs, costs,  # noqa: F401
                  A_apply, AT_apply, normal_blocks, schur_complement)
from .purify import purify_to_forest, is_forest  # noqa: F401


def build():
    """Compile the oracle's C scans (gcc)."""
    return _cscan.build(force=True)
