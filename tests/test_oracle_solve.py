"""Pins of the oracle's smoother, coarse solver, V-cycle (Algorithm 2) and PCG."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from tests.dense import csr, dense, random_spd_graph
from workloads import front_c1, rhs_uniform, two_fluid_7pt


def test_spai0_diagonal_matrix_is_exact_inverse(ora):
    n = 50
    d = np.linspace(1.0, 7.0, n)
    p = np.arange(n + 1, dtype=np.int32)
    c = np.arange(n, dtype=np.int32)
    # single level (n <= coarse_enough): m is still computed on non-coarsest levels only,
    # so force two levels with a prescribed transfer
    P = np.zeros((n, 1))
    P[:, 0] = 1.0
    import scipy.sparse as sp
    S = sp.csr_matrix(P)
    h = ora.OracleHierarchy(p, c, d, transfer=[(S.indptr, S.indices, S.data, 1)], smoother=1,
                            coarse_enough=0)
    # d / (d * d): the exact inverse up to two roundings
    assert np.abs(h.level(0)["m"] * d - 1.0).max() <= 4.5e-16


@pytest.mark.parametrize("smoother", [0, 1])
def test_smoother_formulas(ora, smoother):
    """Jacobi: m = omega / diag.  SPAI0: m minimises ||I - diag(m) A||_F (checked by the
    optimality condition: any perturbation of one entry increases the norm)."""
    p, c, v = random_spd_graph(40, 4, 5)
    h = ora.OracleHierarchy(p, c, v, coarse_enough=5, smoother=smoother)
    A = dense(p, c, v)
    m = h.level(0)["m"]
    if smoother == 0:
        assert np.array_equal(m, 0.72 / np.diag(A))
    else:
        I = np.eye(len(m))

        def f(mm):
            return np.sum((I - mm[:, None] * A) ** 2)

        base = f(m)
        for i in range(0, len(m), 7):
            for s in (1e-4, -1e-4):
                mm = m.copy()
                mm[i] *= 1 + s
                assert f(mm) > base


def test_coarse_cholesky_and_solve(ora):
    p, c, v = two_fluid_7pt(8, 0.5)
    h = ora.OracleHierarchy(p, c, v, coarse_enough=100)
    top = h.num_levels - 1
    Ac = dense(*h.level(top)["A"])
    L = h.coarse_factor()
    assert np.allclose(L @ L.T, Ac, rtol=0, atol=1e-13 * np.abs(Ac).max())
    assert np.all(np.triu(L, 1) == 0)


def test_single_level_pcg_is_direct(ora):
    """n <= coarse_enough: the preconditioner is the exact inverse, one iteration."""
    p, c, v = two_fluid_7pt(6, 0.5)
    h = ora.OracleHierarchy(p, c, v, coarse_enough=500)
    assert h.num_levels == 1
    f = rhs_uniform(216, 1, 0)
    u, info = h.solve(f)
    assert info["iters"] == 1 and info["converged"]
    x = np.linalg.solve(dense(p, c, v), f)
    assert np.abs(u - x).max() <= 1e-12 * np.abs(x).max()


@pytest.mark.parametrize("smoother", [0, 1])
def test_vcycle_symmetric_positive(ora, smoother):
    p, c, v = two_fluid_7pt(10, 0.5)
    h = ora.OracleHierarchy(p, c, v, coarse_enough=30, smoother=smoother)
    assert h.num_levels >= 3
    g = np.random.default_rng(0)
    for _ in range(4):
        x, y = g.standard_normal(1000), g.standard_normal(1000)
        Bx, By = h.vcycle(x), h.vcycle(y)
        assert abs(x @ By - y @ Bx) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(By)
        assert x @ Bx > 0


def test_vcycle_two_grid_identity(ora):
    """For a two-level hierarchy with one pre- and one post-sweep, B = (I - E) A^{-1} where
    E = (I - M A)(I - P A_c^{-1} P^T A)(I - M A) is the textbook two-grid error operator."""
    p, c, v = random_spd_graph(120, 3, 11)
    h = ora.OracleHierarchy(p, c, v, coarse_enough=60, max_levels=2)
    assert h.num_levels == 2
    A = dense(p, c, v)
    l0 = h.level(0)
    Pp, Pc, Pv, nc = l0["P"]
    P = dense(Pp, Pc, Pv, shape=(120, nc))
    Ac = dense(*h.level(1)["A"])
    M = np.diag(l0["m"])
    I = np.eye(120)
    E = (I - M @ A) @ (I - P @ np.linalg.solve(Ac, P.T @ A)) @ (I - M @ A)
    B_ref = (I - E) @ np.linalg.inv(A)
    B = np.column_stack([h.vcycle(I[:, j]) for j in range(120)])
    assert np.abs(B - B_ref).max() <= 1e-10 * np.abs(B_ref).max()


@pytest.mark.parametrize("smoother", [0, 1])
@pytest.mark.parametrize("aggregation", [0, 1])
def test_pcg_against_sparse_direct(ora, smoother, aggregation):
    N = 16
    p, c, v = two_fluid_7pt(N, front_c1(3))
    h = ora.OracleHierarchy(p, c, v, coarse_enough=50, smoother=smoother, aggregation=aggregation)
    f = rhs_uniform(N**3, 1, 3)
    u, info = h.solve(f)
    assert info["converged"] and info["rel_res_true"] <= 1e-8
    A = csr(p, c, v)
    assert np.linalg.norm(f - A @ u) / np.linalg.norm(f) <= 1e-8
    x = spla.spsolve(A.tocsc(), f)
    # error bounded by cond * rtol; cond(A) of the two-fluid operator ~ 1e5 here
    assert np.linalg.norm(u - x) <= 1e-2 * np.linalg.norm(x)


def test_pcg_zero_rhs_and_initial_guess(ora):
    p, c, v = two_fluid_7pt(8, 0.5)
    h = ora.OracleHierarchy(p, c, v, coarse_enough=30)
    u, info = h.solve(np.zeros(512), u=np.ones(512))
    assert np.all(u == 0) and info["iters"] == 0
    f = rhs_uniform(512, 1, 0)
    x = spla.spsolve(csr(p, c, v).tocsc(), f)
    u, info = h.solve(f, u=x)
    assert info["iters"] == 0 and info["converged"]


def test_pcg_maxiter_not_converged(ora):
    p, c, v = two_fluid_7pt(12, 0.5)
    h = ora.OracleHierarchy(p, c, v, coarse_enough=30, maxiter=2)
    u, info = h.solve(rhs_uniform(12**3, 1, 0))
    assert not info["converged"] and info["iters"] == 2 and info["rel_res_true"] > 1e-8


def test_not_spd_coarse(ora):
    """An indefinite matrix with a positive diagonal fails in the coarse factorisation."""
    n = 40
    A = 2.0 * np.eye(n)
    A[0, 1] = A[1, 0] = 5.0
    import scipy.sparse as sp
    S = sp.csr_matrix(A)
    with pytest.raises(ora.OracleError) as e:
        ora.OracleHierarchy(S.indptr, S.indices, S.data, coarse_enough=100)
    assert e.value.code == -5


def test_full_reuse_iterations_grow_partial_does_not(ora):
    """Table 2 behaviour on a moving-interface series: after the interface moved, reusing
    the whole hierarchy costs far more iterations than the partial update, which stays
    close to a full rebuild (one-cell move of a density-1000 column)."""
    N = 24
    p, c, v0 = two_fluid_7pt(N, 0.3)
    _, _, v1 = two_fluid_7pt(N, 0.3 + 1 / N)
    f = rhs_uniform(N**3, 2, 1)
    full = ora.OracleHierarchy(p, c, v0, coarse_enough=100)
    full.rebuild(v1, 2)
    _, it_full_reuse = full.solve(f)
    part = ora.OracleHierarchy(p, c, v0, coarse_enough=100)
    part.rebuild(v1, 0)
    _, it_part = part.solve(f)
    fresh = ora.OracleHierarchy(p, c, v1, coarse_enough=100)
    _, it_fresh = fresh.solve(f)
    assert it_part["converged"] and it_fresh["converged"]
    assert it_full_reuse["iters"] > 2 * it_part["iters"]
    assert it_part["iters"] <= it_fresh["iters"] + 3
