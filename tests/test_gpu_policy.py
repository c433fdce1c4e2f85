"""Rebuild policy on the device: which update each step takes, and that a full setup it
triggers is the hierarchy a fresh setup builds from the same values."""
import numpy as np
import pytest

from tests.gpu_util import T
from workloads import front_c1, rhs_uniform, two_fluid_7pt

pytestmark = pytest.mark.gpu


def same_hierarchy(g, h):
    assert g.num_levels == h.num_levels
    for l in range(g.num_levels):
        a, b = g.level(l), h.level(l)
        for k in (0, 1, 2):
            assert np.array_equal(a["A"][k], b["A"][k]), (l, k)
        if b["agg"] is not None:
            assert np.array_equal(a["agg"], b["agg"]), l
        if b["P"] is not None:
            for k in (0, 1, 2):
                assert np.array_equal(a["P"][k], b["P"][k]), (l, k)


def test_every_third_update_is_a_full_setup():
    from paper_2108_02054_amd import AMG
    from paper_2108_02054_amd.amg import FULL, PARTIAL, policy

    p, c, v0 = two_fluid_7pt(32, front_c1(0))
    vals = [two_fluid_7pt(32, front_c1(t))[2] for t in range(8)]
    n = len(p) - 1
    g = AMG(T(p), T(c), T(v0))
    pol = policy(PARTIAL, every=3)
    taken = []
    for t in range(1, 8):
        taken.append(g.rebuild_auto(T(vals[t]), pol))
        _, info = g.solve(T(rhs_uniform(n, 1, t)))
        assert info["converged"]
        if taken[-1] == FULL:
            fresh = AMG(T(p), T(c), T(vals[t]))
            same_hierarchy(g, fresh)
            fresh.close()
    assert taken == [PARTIAL, PARTIAL, FULL, PARTIAL, PARTIAL, FULL, PARTIAL]
    g.close()


def test_growth_and_missed_convergence_trigger_full_setups():
    from paper_2108_02054_amd import AMG
    from paper_2108_02054_amd.amg import FULL, OPERATOR_ONLY, PARTIAL, policy

    p, c, v0 = two_fluid_7pt(32, front_c1(0))
    v1, v2 = (two_fluid_7pt(32, front_c1(t))[2] for t in (2, 4))
    n = len(p) - 1
    f = T(rhs_uniform(n, 1, 1))
    g = AMG(T(p), T(c), T(v0))
    g.solve(f)                                                     # the reference solve
    assert g.rebuild_auto(T(v1), policy(PARTIAL, growth=10.0)) == PARTIAL
    g.solve(f)
    assert g.rebuild_auto(T(v2), policy(PARTIAL, growth=0.5)) == FULL  # any solve exceeds half the reference
    g.close()
    # full reuse: a solve cut off by the iteration limit makes the next update a full setup
    g = AMG(T(p), T(c), T(v0), maxiter=3)
    g.solve(f)
    assert g.rebuild_auto(T(v2), policy(OPERATOR_ONLY)) == FULL
    _, info = g.solve(f)
    assert not info["converged"]
    g.close()
    g = AMG(T(p), T(c), T(v0))
    g.solve(f)
    assert g.rebuild_auto(T(v1), policy(OPERATOR_ONLY)) == OPERATOR_ONLY
    _, info = g.solve(f)
    assert info["converged"]
    g.close()
