"""Pins of the oracle's BiCGStab (the paper's Krylov method for its non-symmetric systems),
its LU coarse solve, and the non-symmetric convection-diffusion series."""
import numpy as np
import scipy.sparse as sp

from tests.dense import dense
from workloads import rhs_uniform, two_fluid_7pt
from workloads.poisson import convdiff_7pt


def test_convdiff_generator():
    """Peclet 0 is the constant Laplacian bit for bit; otherwise the operator is a
    non-symmetric, weakly row-diagonally-dominant M-matrix on the 7-point pattern whose
    symmetric part is the Laplacian plus a non-negative diagonal."""
    p, c, v = convdiff_7pt(6, 3)
    q, d, u = two_fluid_7pt(6, 0.5, rho_heavy=1.0)
    p0, c0, v0 = convdiff_7pt(6, 3, peclet=0.0)
    assert np.array_equal(p0, q) and np.array_equal(c0, d) and np.array_equal(v0, u)
    assert np.array_equal(p, q) and np.array_equal(c, d)
    A = sp.csr_matrix((v, c, p)).toarray()
    L = sp.csr_matrix((u, d, q)).toarray()
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 0) and np.all(np.diag(A) > 0)
    assert np.all(np.diag(A) - np.abs(off).sum(axis=1) >= -1e-12)
    assert np.abs(A - A.T).max() > 0.1
    # first-order upwinding: A = L + h * (upwind convection), whose off-diagonal part is
    # one-sided per direction, so (A + A^T)/2 - L has non-positive off-diagonals and
    # zero row sums in the interior
    S = 0.5 * (A + A.T) - L
    assert np.all(S - np.diag(np.diag(S)) <= 1e-15)
    # a turning flow: the series changes with t but keeps its pattern
    assert not np.array_equal(convdiff_7pt(6, 4)[2], v)


def test_bicgstab_matches_dense_solve(ora):
    p, c, v = convdiff_7pt(8, 5)
    n = len(p) - 1
    f = rhs_uniform(n, 6, 5)
    h = ora.OracleHierarchy(p, c, v, coarse_enough=60, rtol=1e-11)
    assert h.num_levels >= 2
    u, info = h.solve_bicgstab(f)
    x = np.linalg.solve(dense(p, c, v), f)
    assert info["converged"] and info["rel_res_true"] <= 1e-11
    assert np.linalg.norm(u - x) / np.linalg.norm(x) <= 1e-9


def test_bicgstab_single_level_is_one_step(ora):
    """n <= coarse_enough: the preconditioner is the exact inverse, so s = r - alpha A M r
    vanishes at the first half step."""
    p, c, v = convdiff_7pt(5, 2)
    n = len(p) - 1
    f = rhs_uniform(n, 6, 2)
    h = ora.OracleHierarchy(p, c, v, coarse_enough=200)
    assert h.num_levels == 1
    u, info = h.solve_bicgstab(f)
    x = np.linalg.solve(dense(p, c, v), f)
    assert info["iters"] == 1 and info["converged"]
    assert np.linalg.norm(u - x) / np.linalg.norm(x) <= 1e-12


def test_coarse_lu_of_a_nonsymmetric_operator(ora):
    p, c, v = convdiff_7pt(8, 1)
    h = ora.OracleHierarchy(p, c, v, coarse_enough=100)
    top = h.num_levels - 1
    Ac = dense(*h.level(top)["A"])
    assert np.abs(Ac - Ac.T).max() > 1e-6
    LU = h.coarse_factor()
    L = np.tril(LU, -1) + np.eye(len(LU))
    U = np.triu(LU)
    assert np.allclose(L @ U, Ac, rtol=0, atol=1e-13 * np.abs(Ac).max())


def test_bicgstab_on_an_spd_system_agrees_with_cg(ora):
    p, c, v = two_fluid_7pt(10, 0.45)
    n = len(p) - 1
    f = rhs_uniform(n, 1, 3)
    h = ora.OracleHierarchy(p, c, v, coarse_enough=50, rtol=1e-10)
    ub, ib = h.solve_bicgstab(f)
    uc, ic = h.solve(f)
    assert ib["converged"] and ic["converged"]
    assert np.linalg.norm(ub - uc) / np.linalg.norm(uc) <= 1e-8
    # BiCGStab applies two V-cycles per iteration
    assert ib["iters"] <= ic["iters"]


def test_bicgstab_zero_rhs_and_exact_guess(ora):
    p, c, v = convdiff_7pt(6, 0)
    n = len(p) - 1
    h = ora.OracleHierarchy(p, c, v, coarse_enough=50)
    u, info = h.solve_bicgstab(np.zeros(n), np.ones(n))
    assert info["converged"] and info["iters"] == 0 and not u.any()
    x = np.linalg.solve(dense(p, c, v), np.ones(n))
    u, info = h.solve_bicgstab(np.ones(n), x)
    assert info["converged"] and info["iters"] == 0


def test_partial_rebuild_of_the_nonsymmetric_series(ora):
    """Algorithm 4 on the turning flow: a partial update from step 0 to step 3 keeps P and
    gives the same Galerkin operators as R (A P) formed densely, and BiCGStab converges."""
    p, c, v0 = convdiff_7pt(8, 0)
    v3 = convdiff_7pt(8, 3)[2]
    n = len(p) - 1
    h = ora.OracleHierarchy(p, c, v0, coarse_enough=40)
    h.rebuild(v3, 0)
    A = dense(p, c, v3)
    for l in range(h.num_levels - 1):
        lv = h.level(l)
        P = dense(*lv["P"][:3], shape=(lv["n"], lv["P"][3]))
        Ac = P.T @ A @ P
        got = dense(*h.level(l + 1)["A"])
        assert np.abs(got - Ac).max() <= 1e-12 * np.abs(Ac).max()
        A = Ac
    u, info = h.solve_bicgstab(rhs_uniform(n, 6, 3))
    assert info["converged"]
