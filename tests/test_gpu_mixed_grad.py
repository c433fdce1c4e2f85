"""The two added forms on the GPU: mixed precision (FP32 hierarchy and V-cycle under FP64
CG) and the differentiable solve (adjoint on the reused hierarchy)."""
import numpy as np
import pytest
import torch

from tests.gpu_util import T, both, rel_fro, rel_max
from workloads import front_c1, front_moving, logcoef_inputs, pattern_7pt, rhs_uniform, two_fluid_7pt

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,flex", [(32, 0), (48, 1)])
def test_mixed_precision_solve(N, flex):
    """Patterns and aggregates as in FP64 (setup decisions are FP64); FP32 operator values
    within FP32 rounding of the FP64 oracle; the solve still reaches 1e-8."""
    p, c, v0 = two_fluid_7pt(N, front_moving(N, 0))
    _, _, v1 = two_fluid_7pt(N, front_moving(N, 2))
    g, o = both(p, c, v0, precision=1, flexible_cg=flex)
    g.rebuild(T(v1))
    o.rebuild(v1, 0)
    errs = []
    for l in range(o.num_levels):
        gl, ol = g.level(l), o.level(l)
        assert np.array_equal(gl["A"][1], ol["A"][1])
        if ol["agg"] is not None:
            assert np.array_equal(gl["agg"], ol["agg"])
        errs.append(rel_fro(gl["A"][2], ol["A"][2]))
        assert errs[-1] <= 1e-5, (l, errs[-1])
    f = rhs_uniform(N**3, 3, 2)
    u, info = g.solve(T(f))
    uo, io = o.solve(f)
    print(f"mixed N={N}: level errors {['%.1e' % e for e in errs]} iters {info['iters']} vs fp64 oracle "
          f"{io['iters']}", flush=True)
    assert info["converged"] and info["rel_res_true"] <= 1e-8
    assert info["iters"] <= io["iters"] + 5
    assert rel_fro(u.cpu().numpy(), uo) <= 1e-5


@pytest.mark.parametrize("case,flex", [("tf7", 0), ("tf7", 1), ("ln27", 0), ("ln27", 1)])
def test_mixed_last_sweep_writes_fp64_z(monkeypatch, case, flex):
    """In mixed precision the last FP32 sweep of level 0 (plane marching for the 7-point
    operator, two-row windows for the 27-point one) writes z widened to FP64 and forms the
    CG's r.z (and, flexible, r.z_old) itself; the solve agrees with the form that widens z
    in a separate pass, and its true residual is confirmed on the host."""
    import scipy.sparse as sp

    from paper_2108_02054_amd import AMG

    if case == "tf7":
        N = 48
        p, c, v0 = two_fluid_7pt(N, front_moving(N, 0))
        v1 = two_fluid_7pt(N, front_moving(N, 2))[2]
        prm = dict()
    else:
        from workloads import lognormal_27pt
        N = 40
        p, c, v0 = lognormal_27pt(N, 0)
        v1 = lognormal_27pt(N, 2)[2]
        prm = dict(eps_strong=0.02)
    n = len(p) - 1
    f = rhs_uniform(n, 3, 2)
    print(f"case {case} flexible {flex}", flush=True)

    def run():
        g = AMG(T(p), T(c), T(v0), precision=1, flexible_cg=flex, **prm)
        g.rebuild(T(v1))
        u, info = g.solve(T(f))
        g.close()
        return u.cpu().numpy(), info

    uf, inf_f = run()
    monkeypatch.setenv("AMGMI_NO_RZ32", "1")
    us, inf_s = run()
    A = sp.csr_matrix((v1, c, p), shape=(n, n))
    for u, info in ((uf, inf_f), (us, inf_s)):
        assert info["converged"]
        res = np.linalg.norm(f - A @ u) / np.linalg.norm(f)
        assert res <= 1.01e-8, res
    assert abs(inf_f["iters"] - inf_s["iters"]) <= 1
    assert rel_fro(uf, us) <= 1e-6, rel_fro(uf, us)


def test_logcoef_assembly_parity():
    import oracle
    from paper_2108_02054_amd import logcoef7_assemble
    for (nx, ny, nz) in [(8, 8, 8), (5, 7, 3), (1, 4, 6), (17, 9, 5)]:
        th = np.random.default_rng(nx * 100 + ny).normal(0, 0.5, nx * ny * nz)
        vg = logcoef7_assemble(T(th), nx, ny, nz).cpu().numpy()
        vo = oracle.assemble_logcoef7(nx, ny, nz, th)
        assert rel_max(vg, vo) <= 1e-14, (nx, ny, nz)
        # pattern implied by the kernel is the generator's: constant theta gives A(0) exactly
        p, c, _ = pattern_7pt(nx, ny, nz)
        assert len(vg) == len(c)


def test_adjoint_kernel_parity():
    import oracle
    from paper_2108_02054_amd import logcoef7_adjoint
    nx, ny, nz = 9, 6, 4
    g = np.random.default_rng(2)
    th, u, lam = (g.standard_normal(nx * ny * nz) for _ in range(3))
    gg = logcoef7_adjoint(T(th), T(u), T(lam), nx, ny, nz).cpu().numpy()
    go = oracle.adjoint_logcoef7(nx, ny, nz, th, u, lam)
    assert rel_max(gg, go) <= 1e-13


def _loss_and_grad(amg, th, f, ut, N):
    from paper_2108_02054_amd import AMGSolve
    theta = T(th).requires_grad_(True)
    u = AMGSolve.apply(theta, T(f), amg, (N, N, N))
    loss = 0.5 * torch.sum((u - T(ut)) ** 2)
    loss.backward()
    return float(loss), theta.grad.cpu().numpy(), u.detach().cpu().numpy()


@pytest.mark.parametrize("N,rtol", [(16, 1e-12), (64, 1e-11)])
def test_autograd_gradient(N, rtol):
    """Gradient w.r.t. per-cell log-coefficients: closed-form sum identity, the oracle's
    gradient, and central finite differences (h = 1e-6) at 16 seeded cells."""
    import oracle
    from paper_2108_02054_amd import AMG, logcoef7_assemble
    th, f, ut, cells = logcoef_inputs(N)
    p, c, _ = pattern_7pt(N)
    v = logcoef7_assemble(T(th), N, N, N)
    amg = AMG(T(p), T(c), v, rtol=rtol, maxiter=300)
    L0, g, u = _loss_and_grad(amg, th, f, ut, N)
    want = -u @ (u - ut)
    assert abs(g.sum() - want) <= 1e-8 * abs(want)
    vo = oracle.assemble_logcoef7(N, N, N, th)
    o = oracle.OracleHierarchy(p, c, vo, rtol=rtol, maxiter=300)
    uo, _ = o.solve(f)
    lo, _ = o.solve(uo - ut)
    go = oracle.adjoint_logcoef7(N, N, N, th, uo, lo)
    assert rel_max(g, go) <= 1e-8
    h = 1e-6
    from paper_2108_02054_amd import AMGSolve
    worst = 0.0
    for cell in cells:
        Ls = []
        for s in (1.0, -1.0):
            t2 = th.copy()
            t2[cell] += s * h
            with torch.no_grad():
                uu = AMGSolve.apply(T(t2), T(f), amg, (N, N, N))
            Ls.append(0.5 * float(torch.sum((uu - T(ut)) ** 2)))
        fd = (Ls[0] - Ls[1]) / (2 * h)
        err = abs(g[cell] - fd)
        worst = max(worst, err / np.abs(g).max())
        assert err <= 1e-4 * np.abs(g).max() + 1e-8, (cell, g[cell], fd)
    print(f"N={N}: FD worst relative error {worst:.2e}", flush=True)


def test_autograd_restores_values_for_backward():
    """Two forward passes before one backward: the backward pass reloads A(theta) of its
    own forward pass into the hierarchy."""
    from paper_2108_02054_amd import AMG, AMGSolve, logcoef7_assemble
    N = 12
    th, f, ut, _ = logcoef_inputs(N)
    p, c, _ = pattern_7pt(N)
    amg = AMG(T(p), T(c), logcoef7_assemble(T(th), N, N, N), rtol=1e-12, maxiter=300)
    theta = T(th).requires_grad_(True)
    u1 = AMGSolve.apply(theta, T(f), amg, (N, N, N))
    _ = AMGSolve.apply(T(th + 0.3), T(f), amg, (N, N, N))
    (0.5 * torch.sum((u1 - T(ut)) ** 2)).backward()
    g1 = theta.grad.cpu().numpy()
    amg2 = AMG(T(p), T(c), logcoef7_assemble(T(th), N, N, N), rtol=1e-12, maxiter=300)
    _, g2, _ = _loss_and_grad(amg2, th, f, ut, N)
    assert rel_max(g1, g2) <= 1e-9
