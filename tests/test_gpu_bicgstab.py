"""BiCGStab on the device against the oracle's, on the non-symmetric convection-diffusion
series: hierarchy parity after a partial rebuild, iterations and solution."""
import numpy as np
import pytest

from tests.gpu_util import T, both, compare_levels, rel_fro
from workloads import rhs_uniform, two_fluid_7pt
from workloads.poisson import convdiff_7pt

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(16, 16, 16), (24, 16, 12), (33, 17, 9)])
@pytest.mark.parametrize("precision", [0, 1])
def test_bicgstab_partial_rebuild_parity(shape, precision):
    nx, ny, nz = shape
    p, c, v0 = convdiff_7pt(nx, 0, ny=ny, nz=nz)
    v3 = convdiff_7pt(nx, 3, ny=ny, nz=nz)[2]
    n = len(p) - 1
    print(f"case convdiff {shape} precision {precision}", flush=True)
    g, o = both(p, c, v0, precision=precision)
    g.rebuild(T(v3))
    o.rebuild(v3, 0)
    if precision == 0:
        compare_levels(g, o, tol=1e-10)
    f = rhs_uniform(n, 6, 3)
    u, info = g.solve_bicgstab(T(f))
    uo, io = o.solve_bicgstab(f)
    assert info["converged"] and info["rel_res_true"] <= 1e-8, info
    assert io["converged"]
    assert abs(info["iters"] - io["iters"]) <= (1 if precision == 0 else 3), (info, io)
    assert rel_fro(u.cpu().numpy(), uo) <= 1e-6
    if g.level_format(0):
        assert g.diagonals_read(0) == g.level_format(0)  # not symmetric: every diagonal read
    g.close()
    o.close()


def test_bicgstab_on_spd_matches_cg():
    p, c, v = two_fluid_7pt(32, 0.45)
    n = len(p) - 1
    f = T(rhs_uniform(n, 1, 2))
    from paper_2108_02054_amd import AMG
    g = AMG(T(p), T(c), T(v))
    ub, ib = g.solve_bicgstab(f)
    uc, ic = g.solve(f)
    assert ib["converged"] and ic["converged"]
    assert rel_fro(ub.cpu().numpy(), uc.cpu().numpy()) <= 1e-7
    g.close()


def test_bicgstab_series_64_and_edge_cases():
    """A 64^3 turning-flow series with partial reuse converges every step; a zero
    right-hand side returns zero at once; an exact initial guess takes no iteration."""
    from paper_2108_02054_amd import AMG
    p, c, v0 = convdiff_7pt(64, 0)
    n = len(p) - 1
    g = AMG(T(p), T(c), T(v0))
    its = []
    for t in range(1, 4):
        g.rebuild(T(convdiff_7pt(64, t)[2]))
        _, info = g.solve_bicgstab(T(rhs_uniform(n, 6, t)))
        assert info["converged"] and info["rel_res_true"] <= 1e-8
        its.append(info["iters"])
    print("iterations", its, flush=True)
    u, info = g.solve_bicgstab(T(np.zeros(n)))
    assert info["converged"] and info["iters"] == 0 and not u.any().item()
    f = T(rhs_uniform(n, 6, 3))
    x, _ = g.solve_bicgstab(f)
    _, info = g.solve_bicgstab(f, x.clone())
    assert info["converged"] and info["iters"] <= 1
    g.close()


def test_bicgstab_full_reuse_matches_oracle():
    """Algorithm 3 (only the Krylov operator changes) under BiCGStab: the products use the
    CSR form of the new operator, the V-cycle the old hierarchy; iterations and solution
    follow the oracle's."""
    p, c, v0 = convdiff_7pt(16, 0)
    v4 = convdiff_7pt(16, 4)[2]
    n = len(p) - 1
    g, o = both(p, c, v0)
    from paper_2108_02054_amd.amg import OPERATOR_ONLY
    g.rebuild_ex(T(v4), OPERATOR_ONLY)
    o.rebuild(v4, 2)
    f = rhs_uniform(n, 6, 4)
    u, info = g.solve_bicgstab(T(f))
    uo, io = o.solve_bicgstab(f)
    assert info["converged"] and io["converged"]
    assert abs(info["iters"] - io["iters"]) <= 1, (info, io)
    assert rel_fro(u.cpu().numpy(), uo) <= 1e-6
    g.close()
    o.close()


def test_bicgstab_single_level_converges_at_the_half_step():
    """With one level the preconditioner is the exact inverse, so the first step's half
    step already solves the system (alpha = 1, s = 0): the device-side test of ||s|| ends
    the solve there with x = alpha p^ only, after one iteration, as the oracle does; the
    solution matches a dense solve of the non-symmetric system."""
    p, c, v = convdiff_7pt(6, 2, ny=6, nz=6)
    n = len(p) - 1
    g, o = both(p, c, v, coarse_enough=400)
    assert g.num_levels == 1
    f = rhs_uniform(n, 6, 1)
    u, info = g.solve_bicgstab(T(f))
    uo, io = o.solve_bicgstab(f)
    assert info["converged"] and info["iters"] == 1, info
    assert io["iters"] == 1
    A = np.zeros((n, n))
    for i in range(n):
        A[i, c[p[i]:p[i + 1]]] = v[p[i]:p[i + 1]]
    ud = np.linalg.solve(A, f)
    assert np.abs(u.cpu().numpy() - ud).max() <= 1e-12 * np.abs(ud).max()
    assert rel_fro(u.cpu().numpy(), uo) <= 1e-12
    g.close()
    o.close()
