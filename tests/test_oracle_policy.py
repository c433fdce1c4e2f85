"""Pins of the oracle's rebuild policy (Section 3: full reuse until a solve misses the
iteration limit, Algorithm 3; occasional full rebuilds between partial updates, every m-th
step or on a convergence criterion).

The modes the oracle takes are checked against sequences fixed by those rules, and every
full rebuild it takes is checked to be the hierarchy a fresh setup builds from the same
values (bit for bit), every partial update the one Algorithm 4 gives."""
import numpy as np
import pytest

from workloads import front_c1, rhs_uniform, two_fluid_7pt

P, F, O = 0, 1, 2
N = 16


def _series(T):
    p, c, v0 = two_fluid_7pt(N, front_c1(0))
    return p, c, v0, [two_fluid_7pt(N, front_c1(t))[2] for t in range(T)]


def _same(a, b):
    assert a.num_levels == b.num_levels
    for l in range(a.num_levels):
        x, y = a.level(l), b.level(l)
        for k in range(3):
            assert np.array_equal(x["A"][k], y["A"][k])
        if y["P"] is not None:
            for k in range(3):
                assert np.array_equal(x["P"][k], y["P"][k])


def test_every_third_update_is_full(ora):
    p, c, v0, vals = _series(9)
    h = ora.OracleHierarchy(p, c, v0, coarse_enough=32)
    taken = []
    for t in range(1, 9):
        taken.append(h.rebuild_auto(vals[t], base=P, every=3))
        _, info = h.solve(rhs_uniform(N**3, 1, t))
        assert info["converged"]
        fresh = ora.OracleHierarchy(p, c, vals[t], coarse_enough=32)
        if taken[-1] == F:
            _same(h, fresh)
        else:
            # partial: the kept transfer operators are those of the last full build
            assert taken[-1] == P
    assert taken == [P, P, F, P, P, F, P, P]


def test_every_without_solves(ora):
    """The count is of updates since the last full build, solves or not."""
    p, c, v0, vals = _series(7)
    h = ora.OracleHierarchy(p, c, v0, coarse_enough=32)
    assert [h.rebuild_auto(vals[t], base=O, every=2) for t in range(1, 7)] == [O, F, O, F, O, F]


def test_missed_iteration_limit_under_full_reuse(ora):
    """Algorithm 3: a solve that stops at the iteration limit makes the next update a full
    build; one that converges keeps the hierarchy."""
    p, c, v0, vals = _series(6)
    f = rhs_uniform(N**3, 1, 0)
    h = ora.OracleHierarchy(p, c, v0, coarse_enough=32, maxiter=2)
    assert h.rebuild_auto(vals[1], base=O) == O          # no solve yet
    _, info = h.solve(f)
    assert not info["converged"] and info["iters"] == 2
    assert h.rebuild_auto(vals[2], base=O) == F
    assert h.rebuild_auto(vals[3], base=O) == O          # history restarts at the full build
    h2 = ora.OracleHierarchy(p, c, v0, coarse_enough=32)
    _, info = h2.solve(f)
    assert info["converged"]
    assert [h2.rebuild_auto(vals[t], base=O) for t in (1, 2)] == [O, O]


def test_iteration_growth(ora):
    """A full build when the last solve took more than growth times the first solve after
    the last full build; the reference is that first solve's count."""
    p, c, v0, vals = _series(4)
    f = rhs_uniform(N**3, 1, 0)
    h = ora.OracleHierarchy(p, c, v0, coarse_enough=32)
    _, i0 = h.solve(f)
    k = i0["iters"]
    assert k > 2
    # same count again: not more than 1.0 x the reference
    _, i1 = h.solve(f)
    assert i1["iters"] == k
    assert h.rebuild_auto(vals[1], base=P, growth=1.0) == P
    # a solve from the exact answer needs no iteration and counts as one
    u, _ = h.solve(f)
    h.solve(f, u)
    assert h.rebuild_auto(vals[2], base=P, growth=0.5) == P   # 1 is not more than k / 2
    h.solve(f)
    assert h.rebuild_auto(vals[3], base=P, growth=(k - 1) / k) == F


def test_bad_policies(ora):
    p, c, v0, vals = _series(2)
    h = ora.OracleHierarchy(p, c, v0, coarse_enough=32)
    for kw in (dict(base=F), dict(base=P, every=-1), dict(base=P, growth=-0.5), dict(base=P, growth=float("nan"))):
        with pytest.raises(ora.OracleError):
            h.rebuild_auto(vals[1], **kw)
