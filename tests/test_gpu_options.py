"""A grid of option combinations on small problems, each against the oracle: the solve's
iterations and solution, after a partial rebuild.  It exercises the kernel families
together (diagonal storage with the marching or windowed forms, row blocks, the coarse
tail, two-byte columns, mixed precision, SPAI0, plain aggregation, extra sweeps, flexible
CG, BiCGStab) in combinations the focused tests do not pin one by one."""
import numpy as np
import pytest

from tests.gpu_util import T, both, rel_fro
from workloads import front_c1, lognormal_27pt, rhs_uniform, two_fluid_7pt
from workloads.poisson import convdiff_7pt

pytestmark = pytest.mark.gpu

# (name, matrix series, params, krylov)
CASES = [
    ("tf7_spai0", "tf7", dict(smoother=1), "cg"),
    ("tf7_plain", "tf7", dict(aggregation=1), "cg"),
    ("tf7_sweeps22", "tf7", dict(npre=2, npost=2), "cg"),
    ("tf7_sweeps02", "tf7", dict(npre=0, npost=2), "cg"),
    ("tf7_flex_mixed", "tf7", dict(flexible_cg=1, precision=1), "cg"),
    ("tf7_mixed_spai0", "tf7", dict(precision=1, smoother=1), "cg"),
    ("tf7_coarse_small", "tf7", dict(coarse_enough=16), "cg"),
    ("box_plain_mixed", "box", dict(aggregation=1, precision=1), "cg"),
    ("ln27_sweeps22", "ln27", dict(eps_strong=0.02, npre=2, npost=2), "cg"),
    ("ln27_spai0_mixed", "ln27", dict(eps_strong=0.02, smoother=1, precision=1), "cg"),
    ("cd7_bicg_spai0", "cd7", dict(smoother=1), "bicg"),
    ("cd7_bicg_plain_mixed", "cd7", dict(aggregation=1, precision=1), "bicg"),
    ("cd7_bicg_sweeps22", "cd7", dict(npre=2, npost=2), "bicg"),
]


def series(kind):
    if kind == "tf7":
        p, c, v0 = two_fluid_7pt(20, front_c1(0))
        return p, c, v0, two_fluid_7pt(20, front_c1(3))[2]
    if kind == "box":
        p, c, v0 = two_fluid_7pt(29, 0.4, ny=13, nz=11)
        return p, c, v0, two_fluid_7pt(29, 0.47, ny=13, nz=11)[2]
    if kind == "ln27":
        p, c, v0 = lognormal_27pt(14, 0)
        return p, c, v0, lognormal_27pt(14, 2)[2]
    p, c, v0 = convdiff_7pt(18, 0, ny=14, nz=11)
    return p, c, v0, convdiff_7pt(18, 3, ny=14, nz=11)[2]


@pytest.mark.parametrize("name,kind,prm,krylov", CASES, ids=[c[0] for c in CASES])
def test_option_grid_against_oracle(name, kind, prm, krylov):
    p, c, v0, v1 = series(kind)
    n = len(p) - 1
    print(f"case {name}", flush=True)
    g, o = both(p, c, v0, **prm)
    g.rebuild(T(v1))
    o.rebuild(v1, 0)
    f = rhs_uniform(n, 1, 5)
    if krylov == "bicg":
        u, info = g.solve_bicgstab(T(f))
        uo, io = o.solve_bicgstab(f)
    else:
        u, info = g.solve(T(f))
        uo, io = o.solve(f)
    mixed = prm.get("precision", 0) == 1
    assert info["converged"] and info["rel_res_true"] <= 1e-8, info
    assert io["converged"]
    assert abs(info["iters"] - io["iters"]) <= (3 if mixed else 1), (info, io)
    assert rel_fro(u.cpu().numpy(), uo) <= 1e-6
    g.close()
    o.close()
