"""Parity with the oracle at the full sizes of the benchmark series (GPU).

* two-fluid 192^3 (7.1 M rows), the series whose FP64 and mixed-precision steps are
  compared: setup at step 0, partial update to the last step (29);
* 27-point lognormal 160^3 (4.1 M rows, 109 M entries, eps 0.02) with the FP32 hierarchy,
  and in FP64: setup at step 0, partial update to step 39;
* the differentiable solve at 128^3: the gradient against the oracle's and against
  central finite differences at 16 seeded cells.

FP64 levels are compared with the oracle's bit for bit where the kernels keep the oracle's
summation order and within 1e-10 otherwise (normwise and max-entry), aggregates and
patterns bit for bit; V-cycle outputs and solutions entry by entry (largest difference
over the largest entry); the true residual is recomputed on the host with SciPy.  For the
mixed form the error of every result against the FP64 oracle is printed (per-level
||dA_l||_F / ||A_l||_F, the smoother diagonal, the V-cycle output, the solution, the final
residual and the iterations) and bounded loosely: its parity is not pinned beyond the
final residual, which must reach 1e-8 as in FP64.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from tests.gpu_util import T, bitwise_levels, compare_levels, rel_fro, rel_max
from workloads import CONFIGS, front_moving, logcoef_inputs, pattern_7pt, rhs_uniform, series_matrix

pytestmark = pytest.mark.gpu


def host_rel_res(p, c, v, f, u):
    A = sp.csr_matrix((v, c, p), shape=(len(p) - 1, len(p) - 1))
    return float(np.linalg.norm(f - A @ u) / np.linalg.norm(f))


def mixed_errors(g, o):
    """Per-level relative errors of the FP32 hierarchy against the FP64 oracle."""
    out = []
    for l in range(o.num_levels):
        gl, ol = g.level(l), o.level(l)
        assert np.array_equal(gl["A"][0], ol["A"][0]) and np.array_equal(gl["A"][1], ol["A"][1]), l
        if ol["agg"] is not None:
            assert np.array_equal(gl["agg"], ol["agg"]), l
        e = {"A": rel_fro(gl["A"][2], ol["A"][2])}
        if ol["P"] is not None:
            e["m"] = rel_max(gl["m"], ol["m"])
        out.append(e)
    return out


def check_solution(p, c, v, f, u, info, uo, io, tol_u, tol_iters):
    res = host_rel_res(p, c, v, f, u)
    assert info["converged"] and res <= 1e-8 * (1 + 1e-2), (res, info)
    assert abs(res - info["rel_res_true"]) <= 1e-2 * 1e-8, (res, info["rel_res_true"])
    assert abs(info["iters"] - io["iters"]) <= tol_iters, (info, io)
    assert rel_max(u, uo) <= tol_u and rel_fro(u, uo) <= tol_u
    return res


def run_series(cfg_id, t_last, precisions):
    """Setup at step 0 and a partial update to t_last, on the device in each precision
    and in the oracle; returns what the checks need."""
    import oracle
    from paper_2108_02054_amd import AMG
    cfg = CONFIGS[cfg_id]
    p, c, v0 = series_matrix(cfg_id, 0)
    _, _, vt = series_matrix(cfg_id, t_last)
    n = len(p) - 1
    f = rhs_uniform(n, cfg_id, t_last)
    o = oracle.OracleHierarchy(p, c, v0, eps_strong=cfg["eps_strong"])
    o.rebuild(vt, 0)
    r = np.random.default_rng(7).uniform(-1, 1, n)
    zo = o.vcycle(r)
    uo, io = o.solve(f)
    Tp, Tc, Tv0, Tvt, Tf, Tr = T(p), T(c), T(v0), T(vt), T(f), T(r)
    out = {}
    for prec in precisions:
        print(f"case config {cfg_id} ({cfg['name']}) precision {prec} step 0 -> {t_last}", flush=True)
        g = AMG(Tp, Tc, Tv0, eps_strong=cfg["eps_strong"], precision=prec)
        g.rebuild(Tvt)
        z = g.vcycle(Tr).cpu().numpy()
        u, info = g.solve(Tf)
        torch.cuda.synchronize()
        out[prec] = (g, z, u.cpu().numpy(), info)
    return p, c, vt, f, o, zo, uo, io, out


def test_two_fluid_192_fp64_and_mixed():
    p, c, vt, f, o, zo, uo, io, out = run_series(3, 29, (0, 1))
    g, z, u, info = out[0]
    compare_levels(g, o, tol=1e-10)
    assert bitwise_levels(g, o) is None
    assert rel_max(z, zo) <= 1e-11, rel_max(z, zo)
    res = check_solution(p, c, vt, f, u, info, uo, io, 1e-6, 1)
    print(f"192^3 FP64: iters {info['iters']} (oracle {io['iters']}), host rel res {res:.3e}, "
          f"u max diff {rel_max(u, uo):.1e}, z max diff {rel_max(z, zo):.1e}", flush=True)
    g.close()
    g, z, u, info = out[1]
    errs = mixed_errors(g, o)
    for l, e in enumerate(errs):
        assert e["A"] <= 1e-5 and e.get("m", 0.0) <= 1e-5, (l, e)
    assert rel_max(z, zo) <= 1e-3, rel_max(z, zo)
    res = check_solution(p, c, vt, f, u, info, uo, io, 1e-3, 5)
    print(f"192^3 mixed vs FP64 oracle: level errors {[{k: float('%.1e' % x) for k, x in e.items()} for e in errs]}, "
          f"z {rel_max(z, zo):.1e}, iters {info['iters']} (oracle {io['iters']}), host rel res {res:.3e}, "
          f"u {rel_max(u, uo):.1e}", flush=True)
    g.close()


def test_lognormal_27pt_160_mixed_and_fp64():
    p, c, vt, f, o, zo, uo, io, out = run_series(5, 39, (1, 0))
    g, z, u, info = out[1]
    errs = mixed_errors(g, o)
    for l, e in enumerate(errs):
        assert e["A"] <= 1e-5 and e.get("m", 0.0) <= 1e-5, (l, e)
    assert rel_max(z, zo) <= 1e-3, rel_max(z, zo)
    res = check_solution(p, c, vt, f, u, info, uo, io, 1e-3, 5)
    print(f"160^3 27-point mixed vs FP64 oracle: level errors "
          f"{[{k: float('%.1e' % x) for k, x in e.items()} for e in errs]}, z {rel_max(z, zo):.1e}, iters "
          f"{info['iters']} (oracle {io['iters']}), host rel res {res:.3e}, u {rel_max(u, uo):.1e}", flush=True)
    g.close()
    g, z, u, info = out[0]
    compare_levels(g, o, tol=1e-10)
    assert rel_max(z, zo) <= 1e-10, rel_max(z, zo)
    res = check_solution(p, c, vt, f, u, info, uo, io, 1e-6, 1)
    print(f"160^3 27-point FP64: iters {info['iters']} (oracle {io['iters']}), host rel res {res:.3e}, "
          f"u {rel_max(u, uo):.1e}, bitwise levels: {bitwise_levels(g, o) or 'all'}", flush=True)
    g.close()


def test_gradient_128():
    """Series 4 at 128^3: sum identity, the oracle's gradient (both at rtol 1e-11) and
    central finite differences (h = 1e-6) at 16 seeded cells."""
    import oracle
    from paper_2108_02054_amd import AMG, AMGSolve, logcoef7_assemble
    N, rtol = 128, 1e-11
    th, f, ut, cells = logcoef_inputs(N)
    p, c, _ = pattern_7pt(N)
    print("case gradient 128^3", flush=True)
    v = logcoef7_assemble(T(th), N, N, N)
    amg = AMG(T(p), T(c), v, rtol=rtol, maxiter=300)
    theta = T(th).requires_grad_(True)
    u = AMGSolve.apply(theta, T(f), amg, (N, N, N))
    loss = 0.5 * torch.sum((u - T(ut)) ** 2)
    loss.backward()
    g = theta.grad.cpu().numpy()
    un = u.detach().cpu().numpy()
    want = -un @ (un - ut)
    assert abs(g.sum() - want) <= 1e-8 * abs(want)
    vo = oracle.assemble_logcoef7(N, N, N, th)
    o = oracle.OracleHierarchy(p, c, vo, rtol=rtol, maxiter=300)
    uo, _ = o.solve(f)
    lo, _ = o.solve(uo - ut)
    go = oracle.adjoint_logcoef7(N, N, N, th, uo, lo)
    assert rel_max(un, uo) <= 1e-8
    assert rel_max(g, go) <= 1e-8, rel_max(g, go)
    h = 1e-6
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
    print(f"128^3 gradient: vs oracle {rel_max(g, go):.1e}, FD worst {worst:.1e}", flush=True)
    amg.close()
