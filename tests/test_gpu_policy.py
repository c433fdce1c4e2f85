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


def _borderline(hist_iters, converged, ref, growth, maxiter):
    """Whether the next decision could flip if the last solve took one iteration more or
    less (the device and the oracle may differ by one)."""
    if hist_iters is None:
        return False
    if growth > 0 and ref and abs(hist_iters - growth * ref) <= 1.0:
        return True
    return abs(hist_iters - maxiter) <= 1 and converged


@pytest.mark.parametrize("base,every,growth,maxiter", [(0, 4, 0.0, 100), (0, 3, 0.0, 100), (2, 0, 0.0, 100),
                                                       (2, 3, 0.0, 100)])
def test_policy_series_matches_oracle(base, every, growth, maxiter):
    """The same rebuild policy on the device and in the oracle over a 32^3 two-fluid series
    (interface three cells per step): the same mode at every step and iterations within
    one.  The series are chosen so that no decision is within one iteration of a threshold
    (the growth rule, whose thresholds these series approach within one iteration, is
    checked by the oracle's pins and the host logic)."""
    import oracle
    from paper_2108_02054_amd import AMG
    from paper_2108_02054_amd.amg import policy
    from workloads import front_moving

    N = 32
    p, c, v0 = two_fluid_7pt(N, front_moving(N, 0))
    vals = [two_fluid_7pt(N, front_moving(N, 3 * t))[2] for t in range(12)]
    print(f"case policy base={base} every={every} growth={growth}", flush=True)
    g = AMG(T(p), T(c), T(v0), maxiter=maxiter)
    o = oracle.OracleHierarchy(p, c, v0, maxiter=maxiter)
    pol = policy(base, every=every, growth=growth)
    last, conv, ref = None, True, None
    compared = 0
    modes = []
    for t in range(1, 12):
        if _borderline(last, conv, ref, growth, maxiter):
            break
        mg = g.rebuild_auto(T(vals[t]), pol)
        mo = o.rebuild_auto(vals[t], base, every, growth)
        assert mg == mo, (t, mg, mo)
        f = rhs_uniform(N**3, 1, t)
        _, ig = g.solve(T(f))
        _, io = o.solve(f)
        assert ig["converged"] == io["converged"], t
        assert abs(ig["iters"] - io["iters"]) <= 1, (t, ig, io)
        if mo == 1 or ref is None:  # the first solve after the last full build
            ref = io["iters"]
        last, conv = io["iters"], io["converged"]
        modes.append(mo)
        compared += 1
    assert compared == 11, compared
    assert 1 in modes
    g.close()
