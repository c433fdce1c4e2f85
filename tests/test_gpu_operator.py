"""The Krylov operator entry point (y = A x by the level-0 SpMV kernel the CG uses) against
SciPy on every storage form: the 7-point marching kernel, the windowed 27-point diagonal
storage, CSR row blocks, the node-group kernel of block systems, and the CSR form after an
operator-only update (whose values differ from the hierarchy's)."""
import numpy as np
import pytest
import scipy.sparse as sp

from tests.dense import random_spd_graph
from tests.gpu_util import T
from workloads import lognormal_27pt, two_fluid_7pt
from workloads.poisson import coupled4_7pt

pytestmark = pytest.mark.gpu

CASES = [
    ("tf7_march", lambda: two_fluid_7pt(40, 0.45), {}, 7),
    ("ln27_window", lambda: lognormal_27pt(16, 1), dict(eps_strong=0.02), 27),
    ("random_csr", lambda: random_spd_graph(3000, 5, 3), {}, 0),
    ("coupled4_node", lambda: coupled4_7pt(10, 2), dict(block_size=4, aggregation=1), 0),
]


@pytest.mark.parametrize("name,make,prm,ndiag", CASES, ids=[c[0] for c in CASES])
def test_apply_operator_matches_scipy(name, make, prm, ndiag):
    from paper_2108_02054_amd import AMG, OPERATOR_ONLY
    p, c, v = make()
    n = len(p) - 1
    print(f"case {name} n={n}", flush=True)
    g = AMG(T(p), T(c), T(v), **prm)
    assert g.level_format(0) == ndiag
    x = np.random.default_rng(7).standard_normal(n)
    y = g.apply_operator(T(x)).cpu().numpy()
    ref = sp.csr_matrix((v, c, p), shape=(n, n)) @ x
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    v2 = v * (1.0 + 0.25 * np.random.default_rng(8).random(len(v)))   # any new values
    g.rebuild_ex(T(v2), OPERATOR_ONLY)
    y2 = g.apply_operator(T(x)).cpu().numpy()
    ref2 = sp.csr_matrix((v2, c, p), shape=(n, n)) @ x
    assert np.abs(y2 - ref2).max() <= 1e-13 * np.abs(ref2).max()
    g.close()


def test_apply_operator_rejects_aliasing():
    from paper_2108_02054_amd import AMG, AmgError
    p, c, v = two_fluid_7pt(8, 0.5)
    g = AMG(T(p), T(c), T(v), coarse_enough=20)
    x = T(np.ones(len(p) - 1))
    with pytest.raises(AmgError) as e:
        g.apply_operator(x, x)
    assert e.value.code == -1
