"""Pins of the oracle's Galerkin products, prolongator and partial rebuild (Algorithms 1, 4).

Each check compares against something other than the oracle's own sparse code: dense
NumPy products, closed forms, and invariants of the Galerkin product.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from tests.dense import csr, dense, random_spd_graph
from workloads import front_moving, neumann_7pt, pattern_7pt, two_fluid_7pt


def _levels(h):
    return [h.level(l) for l in range(h.num_levels)]


CASES = [
    ("tf4", lambda: two_fluid_7pt(4, 0.5)),
    ("tf6", lambda: two_fluid_7pt(6, 0.45)),
    ("box345", lambda: two_fluid_7pt(3, 0.5, ny=4, nz=5)),
    ("rand60", lambda: random_spd_graph(60, 4, 1)),
    ("rand200", lambda: random_spd_graph(200, 3, 2)),
]


@pytest.mark.parametrize("name,make", CASES)
@pytest.mark.parametrize("aggregation", [0, 1])
def test_rap_dense_brute_force(ora, name, make, aggregation):
    """A_{l+1} = P_l^T A_l P_l equals the dense triple product on every level."""
    p, c, v = make()
    h = ora.OracleHierarchy(p, c, v, coarse_enough=4, aggregation=aggregation)
    L = _levels(h)
    assert len(L) >= 2
    for l in range(len(L) - 1):
        A = dense(*L[l]["A"])
        Pp, Pc, Pv, nc = L[l]["P"]
        P = dense(Pp, Pc, Pv, shape=(L[l]["n"], nc))
        Ac = dense(*L[l + 1]["A"])
        ref = P.T @ A @ P
        assert np.abs(Ac - ref).max() <= 1e-14 * np.abs(ref).max()
        # structural pattern: every stored entry of the dense product's support is present
        assert np.all((ref != 0) <= (csr(*L[l + 1]["A"]).toarray() != 0) | (ref == 0))


def _agg_prolongator(n_fine_1d, size):
    """1-D aggregates of `size` consecutive points, unnormalised."""
    m = n_fine_1d // size
    P = np.zeros((n_fine_1d, m))
    for i in range(n_fine_1d):
        P[i, i // size] = 1.0
    return P


def _to_csr(M):
    S = sp.csr_matrix(M)
    S.sort_indices()
    return S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64)


def test_rap_closed_form_1d(ora):
    """tridiag(-1,2,-1) of size 3m with aggregates of 3 gives tridiag(-1,2,-1) of size m."""
    m = 7
    n = 3 * m
    A = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    P = _agg_prolongator(n, 3)
    h = ora.OracleHierarchy(*_to_csr(A), transfer=[(*_to_csr(P), m)], coarse_enough=1)
    Ac = dense(*h.level(1)["A"])
    expect = 2 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)
    assert np.array_equal(Ac, expect)


def test_rap_closed_form_3d(ora):
    """Constant 7-point operator on (3m)^3 with 3x3x3 block aggregates: A_c = 9 A_{m^3}
    exactly (Kronecker-sum argument: p^T L p = L_m and p^T p = 3 I)."""
    m = 3
    N = 3 * m
    p, c, v = two_fluid_7pt(N, front=0.0)  # density 1 everywhere
    p1 = _agg_prolongator(N, 3)
    P = np.kron(np.kron(p1, p1), p1)  # index x fastest == kron(z, y, x) ordering
    h = ora.OracleHierarchy(p, c, v, transfer=[(*_to_csr(P), m**3)], coarse_enough=1)
    Ac = dense(*h.level(1)["A"])
    pm, cm, vm = two_fluid_7pt(m, front=0.0)
    assert np.array_equal(Ac, 9.0 * dense(pm, cm, vm))


def test_coarse_symmetry(ora):
    p, c, v = two_fluid_7pt(12, 0.4)
    h = ora.OracleHierarchy(p, c, v, coarse_enough=20)
    for lv in _levels(h):
        A = csr(*lv["A"])
        S = (A != 0).astype(int)
        assert (S != S.T).nnz == 0
        d = A - A.T
        assert (abs(d).max() if d.nnz else 0.0) <= 1e-14 * abs(A).max()


def test_near_nullspace(ora):
    """Pure Neumann operator (A 1 = 0): every Galerkin operator keeps the constant in its
    null space, and the smoothed prolongator reproduces constants exactly up to rounding
    (the filtered matrix preserves row sums).  Needs every node aggregated: an isolated
    node has an empty prolongator row, which breaks P 1 = 1 by construction."""
    p, c, v = neumann_7pt(8, seed=3)
    h = ora.OracleHierarchy(p, c, v, coarse_enough=10, check=False)
    for l, lv in enumerate(_levels(h)):
        if lv["agg"] is not None:
            assert np.all(lv["agg"] >= 0), l
        A = csr(*lv["A"])
        one = np.ones(A.shape[0])
        assert np.abs(A @ one).max() <= 1e-13 * abs(A).max(), l
        if lv["P"] is not None:
            Pp, Pc, Pv, nc = lv["P"]
            P = csr(Pp, Pc, Pv, shape=(lv["n"], nc))
            agg = lv["agg"]
            s = P @ np.ones(nc)
            assert np.abs(s[agg >= 0] - 1.0).max() <= 1e-13
            assert np.all(s[agg < 0] == 0)


def test_tentative_reproduces_constants(ora):
    p, c, v = two_fluid_7pt(10, 0.5)
    h = ora.OracleHierarchy(p, c, v, coarse_enough=10, aggregation=1)
    lv = h.level(0)
    Pp, Pc, Pv, nc = lv["P"]
    s = csr(Pp, Pc, Pv, shape=(lv["n"], nc)) @ np.ones(nc)
    assert np.array_equal(s, (lv["agg"] >= 0).astype(float))


def _snapshot(h):
    out = []
    for lv in _levels(h):
        out.append((lv["A"][2].copy(), None if lv["m"] is None else lv["m"].copy()))
    return out, h.coarse_factor()


def test_partial_at_step0_equals_setup(ora):
    """Alg. 4 applied to the matrix the hierarchy was built from reproduces every level,
    smoother and coarse factor bit for bit."""
    p, c, v = two_fluid_7pt(12, front_moving(12, 0))
    h = ora.OracleHierarchy(p, c, v, coarse_enough=30)
    before, Lb = _snapshot(h)
    h.rebuild(v, mode=0)
    after, La = _snapshot(h)
    for (a0, m0), (a1, m1) in zip(before, after):
        assert np.array_equal(a0, a1)
        assert (m0 is None and m1 is None) or np.array_equal(m0, m1)
    assert np.array_equal(Lb, La)


@pytest.mark.parametrize("smoother", [0, 1])
def test_partial_scaling_power_of_two(ora, smoother):
    """rebuild(2A) = 2 rebuild(A) exactly; the smoother diagonal halves exactly."""
    p, c, v = two_fluid_7pt(12, front_moving(12, 0))
    _, _, v2 = two_fluid_7pt(12, front_moving(12, 3))
    h = ora.OracleHierarchy(p, c, v, coarse_enough=30, smoother=smoother)
    h.rebuild(v2, 0)
    a, _ = _snapshot(h)
    h.rebuild(2.0 * v2, 0)
    b, _ = _snapshot(h)
    for (a0, m0), (a1, m1) in zip(a, b):
        assert np.array_equal(2.0 * a0, a1)
        if m0 is not None:
            assert np.array_equal(0.5 * m0, m1)


def test_partial_linearity(ora):
    """The Galerkin update is linear in the fine values (to rounding)."""
    p, c, v = two_fluid_7pt(10, front_moving(10, 0))
    _, _, va = two_fluid_7pt(10, front_moving(10, 2))
    _, _, vb = two_fluid_7pt(10, front_moving(10, 5))
    h = ora.OracleHierarchy(p, c, v, coarse_enough=20)
    res = []
    for w in (va, vb, va + vb):
        h.rebuild(w, 0)
        res.append([lv["A"][2].copy() for lv in _levels(h)])
    for A, B, AB in zip(*res):
        assert np.abs(AB - (A + B)).max() <= 1e-15 * np.abs(AB).max() * 4


def test_partial_keeps_transfer_full_rebuilds_it(ora):
    p, c, v = two_fluid_7pt(12, front_moving(12, 0))
    _, _, v2 = two_fluid_7pt(12, front_moving(12, 4))
    h = ora.OracleHierarchy(p, c, v, coarse_enough=30)
    P0 = h.level(0)["P"][2].copy()
    h.rebuild(v2, 0)
    assert np.array_equal(h.level(0)["P"][2], P0)
    # the partial operators are the Galerkin products with the old P and the new A
    lv0, lv1 = h.level(0), h.level(1)
    Pp, Pc, Pv, nc = lv0["P"]
    P = dense(Pp, Pc, Pv, shape=(lv0["n"], nc))
    ref = P.T @ dense(p, c, v2) @ P
    assert np.abs(dense(*lv1["A"]) - ref).max() <= 1e-14 * np.abs(ref).max()
    h.rebuild(v2, 1)
    h2 = ora.OracleHierarchy(p, c, v2, coarse_enough=30)
    assert np.array_equal(h.level(0)["P"][2], h2.level(0)["P"][2])


def test_operator_only_update(ora):
    """Algorithm 3 (full reuse) changes only the Krylov operator; the hierarchy stays."""
    p, c, v = two_fluid_7pt(10, front_moving(10, 0))
    _, _, v2 = two_fluid_7pt(10, front_moving(10, 4))
    h = ora.OracleHierarchy(p, c, v, coarse_enough=20)
    A1 = h.level(1)["A"][2].copy()
    h.rebuild(v2, 2)
    assert np.array_equal(h.level(0)["A"][2], v)
    assert np.array_equal(h.level(1)["A"][2], A1)
    assert np.array_equal(h.outer_values(), v2)


def test_pattern_check_rejects_unsorted(ora):
    p, c, v = pattern_7pt(3)[0], pattern_7pt(3)[1].copy(), np.ones(len(pattern_7pt(3)[1]))
    c[1], c[2] = c[2], c[1]
    with pytest.raises(ora.OracleError):
        ora.OracleHierarchy(p, c, v)
