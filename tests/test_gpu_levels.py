"""Aggregation bit-exact per level on identical input: every level's operator A_l of an
oracle hierarchy is handed to the device as a level-0 matrix with that level's strength
threshold eps_0 * 2^-l (and at most two aggregation steps, so that the coarsest level
stays small enough for the dense inverse); the device's level-0 strength flags,
aggregates and prolongator pattern must equal the oracle's level l bit for bit (and the
prolongator values to 1e-14).  This separates the setup's integer decisions from the
rounding differences that coarse operators computed on two machines carry."""
import math

import numpy as np
import pytest

from tests.gpu_util import T, rel_max
from workloads import front_c1, lognormal_27pt, two_fluid_7pt
from workloads.poisson import coupled4_7pt

pytestmark = pytest.mark.gpu

CASES = [
    ("tf32", lambda: two_fluid_7pt(32, front_c1(4)), dict(eps_strong=0.08)),
    ("tf24_plain", lambda: two_fluid_7pt(24, 0.45), dict(eps_strong=0.08, aggregation=1)),
    ("ln27_20", lambda: lognormal_27pt(20, 3), dict(eps_strong=0.02)),
    ("coupled4_12", lambda: coupled4_7pt(12, 3), dict(eps_strong=0.08, aggregation=1, block_size=4)),
]


@pytest.mark.parametrize("name,make,prm", CASES, ids=[c[0] for c in CASES])
def test_aggregation_per_level_identical_input(name, make, prm):
    import oracle
    from paper_2108_02054_amd import AMG
    p, c, v = make()
    o = oracle.OracleHierarchy(p, c, v, coarse_enough=128, **prm)  # deep enough for three levels
    assert o.num_levels >= 3
    for l in range(o.num_levels - 1):
        ol = o.level(l)
        Ap, Ac, Av = ol["A"]
        eps = math.ldexp(prm["eps_strong"], -l)
        print(f"case {name} level {l} n={ol['n']} eps={eps}", flush=True)
        g = AMG(T(Ap), T(Ac), T(Av), **{**prm, "eps_strong": eps, "max_levels": 3, "coarse_enough": 1})
        assert g.num_levels >= 2
        gl = g.level(0)
        assert np.array_equal(gl["strong"], ol["strong"]), f"strength differs on level {l}"
        assert np.array_equal(gl["agg"], ol["agg"]), f"aggregates differ on level {l}"
        assert gl["P"][3] == ol["P"][3]
        for k in (0, 1):
            assert np.array_equal(gl["P"][k], ol["P"][k]), f"P pattern differs on level {l}"
        assert rel_max(gl["P"][2], ol["P"][2]) <= 1e-14, l
        g.close()
    o.close()
