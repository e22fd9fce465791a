"""Checkpoint and resume through the C-ABI (otip_state_save / otip_state_load):
a solve stopped by the iteration limit and resumed takes exactly the steps of
one uninterrupted solve (bit-identical plan, duals, objective and counters),
before and after the switch to the direct solver and on a problem with
zero masses; records of another problem or damaged records are refused."""
import struct

import numpy as np
import pytest

from synthetic import config_instance

pytestmark = pytest.mark.gpu

HEADER = 120  # bytes before the support-size history in the record (layout version 2)


@pytest.fixture(scope="module")
def ctx():
    import paper_2206_11009_amd as otip
    c = otip.Context(0)
    yield c
    c.close()


def solve(ctx, inst, **kw):
    import paper_2206_11009_amd as otip
    return otip.otip_solve(ctx, inst.a, inst.b, inst.xs, inst.xt, prm=otip.params(**kw))


def same(r1, r2):
    assert r1.status == r2.status
    assert r1.iterations == r2.iterations
    assert r1.cg_iterations == r2.cg_iterations
    assert r1.direct_iterations == r2.direct_iterations
    assert r1.objective == r2.objective
    np.testing.assert_array_equal(r1.rows, r2.rows)
    np.testing.assert_array_equal(r1.cols, r2.cols)
    np.testing.assert_array_equal(r1.flows, r2.flows)
    np.testing.assert_array_equal(r1.y, r2.y)
    np.testing.assert_array_equal(r1.z, r2.z)


@pytest.fixture(scope="module")
def reference(ctx):
    inst = config_instance("c1", 4)
    r1 = solve(ctx, inst)
    r2 = solve(ctx, inst)
    assert r1.status == 0
    same(r1, r2)          # the solver is deterministic: the premise of the checks below
    return inst, r1


@pytest.mark.parametrize("stop", [3, 9, 17])
def test_resume_takes_the_same_steps(ctx, reference, stop):
    import paper_2206_11009_amd as otip
    inst, full = reference
    assert stop < full.iterations
    part = solve(ctx, inst, max_iter=stop)
    assert part.status == otip.OTIP_EMAXITER and part.iterations == stop
    rec = otip.otip_state_save(ctx)
    assert rec[:8] == b"OTIPCKP1"
    otip.otip_state_load(ctx, rec)
    resumed = solve(ctx, inst)
    same(resumed, full)


def test_resume_after_the_direct_switch_and_of_a_converged_solve(ctx, reference):
    import paper_2206_11009_amd as otip
    inst, full = reference
    assert full.direct_iterations >= 2
    stop = full.iterations - full.direct_iterations + 1   # one direct iteration done
    part = solve(ctx, inst, max_iter=stop)
    assert part.direct_iterations >= 1
    otip.otip_state_load(ctx, otip.otip_state_save(ctx))
    same(solve(ctx, inst), full)
    # the record of a converged solve resumes to the same result at once
    otip.otip_state_load(ctx, otip.otip_state_save(ctx))
    same(solve(ctx, inst), full)


def test_resume_with_zero_masses(ctx):
    import paper_2206_11009_amd as otip
    inst = config_instance("c1", 5)
    a, b = inst.a.copy(), inst.b.copy()
    a[[3, 70, 200]] = 0.0
    b[[0, 128]] = 0.0
    b *= a.sum() / b.sum()
    full = otip.otip_solve(ctx, a, b, inst.xs, inst.xt)
    assert full.status == 0
    part = otip.otip_solve(ctx, a, b, inst.xs, inst.xt, prm=otip.params(max_iter=8))
    assert part.status == otip.OTIP_EMAXITER
    otip.otip_state_load(ctx, otip.otip_state_save(ctx))
    same(otip.otip_solve(ctx, a, b, inst.xs, inst.xt), full)


def test_records_of_another_problem_or_damaged_are_refused(ctx, reference):
    import paper_2206_11009_amd as otip
    inst, full = reference
    solve(ctx, inst, max_iter=5)
    rec = otip.otip_state_save(ctx)
    # another problem of the same size: refused when the solve starts
    other = config_instance("c1", 6)
    otip.otip_state_load(ctx, rec)
    with pytest.raises(otip.OtipError) as e:
        solve(ctx, other)
    assert e.value.code == otip.OTIP_EINVAL
    # damaged records: refused on load ...
    for bad in (rec[:-8], rec + b"\0" * 8, b"XXXXXXXX" + rec[8:], rec[:50]):
        with pytest.raises(otip.OtipError) as e:
            otip.otip_state_load(ctx, bad)
        assert e.value.code == otip.OTIP_EINVAL
    # ... or before anything reaches the device (a support index past m*n)
    hist_len = struct.unpack_from("<q", rec, HEADER - 8)[0]
    m, n = struct.unpack_from("<ii", rec, 12)
    assert (m, n) == (inst.m, inst.n)
    at = HEADER + 8 * hist_len
    bad = bytearray(rec)
    struct.pack_into("<Q", bad, at, m * n)
    otip.otip_state_load(ctx, bytes(bad))
    with pytest.raises(otip.OtipError) as e:
        solve(ctx, inst)
    assert e.value.code == otip.OTIP_EINVAL
    # the context is still usable and holds no stale record
    same(solve(ctx, inst), full)


def test_save_before_any_solve_is_an_error():
    import paper_2206_11009_amd as otip
    c = otip.Context(0)
    try:
        with pytest.raises(otip.OtipError) as e:
            otip.otip_state_save(c)
        assert e.value.code == otip.OTIP_EINVAL
    finally:
        c.close()
