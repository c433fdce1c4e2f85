"""Device blocks that the library frees are handed to its next allocations on the same
stream (it keeps them per stream and size class).  A hierarchy rebuilt after a history of
full-reuse updates, partial updates, full rebuilds and another context created and
destroyed on the same stream must equal, bit for bit, one set up fresh on the same values,
and solve alike: a block handed out while still in use would break that."""
import numpy as np
import pytest

from tests.gpu_util import T
from workloads import rhs_uniform, two_fluid_7pt

pytestmark = pytest.mark.gpu


def _same_levels(g, h):
    assert g.num_levels == h.num_levels
    for l in range(h.num_levels):
        a, b = g.level(l), h.level(l)
        for k in range(3):
            assert np.array_equal(a["A"][k], b["A"][k]), (l, k)
        if b["P"] is not None:
            for k in range(3):
                assert np.array_equal(a["P"][k], b["P"][k]), (l, k)
            assert np.array_equal(a["m"], b["m"]), l


def test_full_rebuild_after_mixed_history_equals_fresh_setup():
    from paper_2108_02054_amd import AMG, FULL, OPERATOR_ONLY
    N = 24
    mats = [two_fluid_7pt(N, f) for f in (0.3, 0.45, 0.6, 0.75)]
    p, c, v0 = mats[0]
    print(f"case two-fluid N={N} mixed history", flush=True)
    g = AMG(T(p), T(c), T(v0))
    for i in range(1, len(mats)):
        v = mats[i][2]
        g.rebuild_ex(T(v), OPERATOR_ONLY)
        other = AMG(T(p), T(c), T(mats[i - 1][2]))  # a second context on the same stream
        g.rebuild(T(v))
        other.close()
        g.rebuild_ex(T(v), FULL)
        fresh = AMG(T(p), T(c), T(v))
        _same_levels(g, fresh)
        f = rhs_uniform(len(p) - 1, 2, i)
        u, info = g.solve(T(f))
        uf, info_f = fresh.solve(T(f))
        assert info["converged"] and info["iters"] == info_f["iters"], (info, info_f)
        assert np.array_equal(u.cpu().numpy(), uf.cpu().numpy())
        fresh.close()
    g.close()
