"""Pins of the oracle's differentiable form: A(theta) assembly and the adjoint gradient.

L(theta) = 0.5 ||u - u_t||^2 with A(theta) u = f and k = exp(theta) per cell.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from tests.dense import csr
from workloads import logcoef_inputs, pattern_7pt, two_fluid_7pt


def test_assembly_constant_coefficient(ora):
    """theta = 0: every face coefficient is 1 and every boundary face adds 1, which is the
    constant-density operator."""
    N = 5
    v = ora.assemble_logcoef7(N, N, N, np.zeros(N**3))
    _, _, ref = two_fluid_7pt(N, 0.0)
    assert np.array_equal(v, ref)


def test_assembly_homogeneous_symmetric_rowsums(ora):
    nx, ny, nz = 4, 5, 3
    g = np.random.default_rng(0)
    th = g.normal(0, 0.5, nx * ny * nz)
    p, c, _ = pattern_7pt(nx, ny, nz)
    v = ora.assemble_logcoef7(nx, ny, nz, th)
    A = csr(p, c, v).toarray()
    assert np.array_equal(A, A.T)
    # k -> 2k scales the operator by exactly 2 (harmonic means and ghost terms are
    # degree-1 homogeneous)
    v2 = ora.assemble_logcoef7(nx, ny, nz, th + np.log(2.0))
    assert np.abs(v2 - 2 * v).max() <= 1e-14 * np.abs(v).max()
    # row sums: only the ghost faces remain, k_c per missing neighbour
    nmiss = 6 - (np.diff(p) - 1)
    assert np.allclose(A.sum(axis=1), nmiss * np.exp(th), rtol=1e-12, atol=1e-13)


def _solve(p, c, v, b):
    return spla.spsolve(csr(p, c, v).tocsc(), b)


def _loss_grad(ora, N, th, f, ut):
    p, c, _ = pattern_7pt(N)
    v = ora.assemble_logcoef7(N, N, N, th)
    u = _solve(p, c, v, f)
    lam = _solve(p, c, v, u - ut)
    g = ora.adjoint_logcoef7(N, N, N, th, u, lam)
    return 0.5 * np.sum((u - ut) ** 2), g, u


def test_gradient_sum_identity(ora):
    """theta -> theta + s scales A by e^s, so u -> e^-s u and
    sum_c dL/dtheta_c = -u^T (u - u_t)."""
    N = 8
    th, f, ut, _ = logcoef_inputs(N)
    _, g, u = _loss_grad(ora, N, th, f, ut)
    want = -u @ (u - ut)
    assert abs(g.sum() - want) <= 1e-10 * abs(want)


def test_gradient_central_differences(ora):
    N = 8
    th, f, ut, cells = logcoef_inputs(N)
    L0, g, _ = _loss_grad(ora, N, th, f, ut)
    h = 1e-6
    for c in cells:
        e = np.zeros_like(th)
        e[c] = h
        Lp = _loss_grad(ora, N, th + e, f, ut)[0]
        Lm = _loss_grad(ora, N, th - e, f, ut)[0]
        fd = (Lp - Lm) / (2 * h)
        assert abs(g[c] - fd) <= 1e-6 * np.abs(g).max() + 1e-9, (c, g[c], fd)


def test_gradient_with_amg_solves(ora):
    """Same gradient with the oracle's AMG-preconditioned CG at a tight tolerance."""
    N = 8
    th, f, ut, _ = logcoef_inputs(N)
    p, c, _ = pattern_7pt(N)
    v = ora.assemble_logcoef7(N, N, N, th)
    h = ora.OracleHierarchy(p, c, v, coarse_enough=50, rtol=1e-13)
    u, i1 = h.solve(f)
    lam, i2 = h.solve(u - ut)
    assert i1["converged"] and i2["converged"]
    g = ora.adjoint_logcoef7(N, N, N, th, u, lam)
    _, g_ref, _ = _loss_grad(ora, N, th, f, ut)
    assert np.abs(g - g_ref).max() <= 1e-9 * np.abs(g_ref).max()
