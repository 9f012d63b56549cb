"""Pins of the oracle's frozen-smoothing mode (used by derivative checks).

With the HC iteration count of every step frozen, the timestep is a smooth
function of sigma, of the gradient rows and of the initial state, so central
finite differences of the oracle are the reference for the discrete adjoint.
The frozen mode must therefore (a) reproduce a free run exactly when given
that run's own counts, and (b) run exactly m iterations of the Sec. 3.3
update, whatever the tolerance would have decided.
"""
import numpy as np

import oracle
from paper_2403_01161_amd.inputs import box_center, icosphere, ou_gradient_table


def _sim(**kw):
    L = (12, 12, 12)
    V, T = icosphere(2, 2.6, box_center(L))
    base = dict(tau=0.9, sigma=0.02, radius=2.6, vertices=V, triangles=T)
    base.update(kw)
    return oracle.Oracle(L, **base), T


def _table(n):
    A = ou_gradient_table(n, 5.0, 1e-3, seed=7)
    A[:, 1] += 4e-3
    return A


def test_frozen_counts_of_free_run_reproduce_it_exactly():
    A = _table(15)
    free, _ = _sim(A0=A[0])
    counts = []
    for n in range(len(A)):
        free.step(A[n])
        counts.append(free.last_iters())
    assert max(counts) >= 2 and min(counts) >= 1  # both branches of the exit test occur
    frozen, _ = _sim(A0=A[0])
    frozen.freeze_iters(counts)
    frozen.step_table(A)
    assert np.array_equal(frozen.vertices(), free.vertices())
    assert np.array_equal(frozen.populations(), free.populations())


def test_frozen_count_runs_exactly_m_iterations():
    # one step with m = 3 frozen equals: the same step without smoothing,
    # then three HC iterations with a tolerance that is never met
    A = _table(1)
    raw, T = _sim(A0=A[0], reg_max_iter=0)
    raw.step(A[0])
    expect, it, _ = oracle.hc(raw.vertices(), T, tol=-1.0, max_iter=3)
    assert it == 3
    fz, _ = _sim(A0=A[0])
    fz.freeze_iters([3])
    fz.step(A[0])
    assert fz.last_iters() == 3
    assert np.array_equal(fz.vertices(), expect)
    assert np.array_equal(fz.populations(), raw.populations())


def test_frozen_zero_is_no_smoothing_and_schedule_expires():
    A = _table(4)
    a, _ = _sim(A0=A[0])
    a.freeze_iters([0, 0])
    b, _ = _sim(A0=A[0], reg_max_iter=0)
    a.step_table(A[:2])
    b.step_table(A[:2])
    assert np.array_equal(a.vertices(), b.vertices())
    a.step(A[2])  # schedule used up: the tolerance test decides again
    assert a.last_iters() >= 1


def test_freeze_rejects_negative_counts():
    a, _ = _sim()
    try:
        a.freeze_iters([1, -1])
    except oracle.OracleError as e:
        assert e.code == -1
    else:
        raise AssertionError("negative count accepted")
