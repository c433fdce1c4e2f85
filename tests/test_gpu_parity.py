"""HIP path vs the oracle, through the C interface (ctypes binding), on the same seeded
inputs.  Aggregates, strength flags and sparsity patterns must match bit for bit;
FP64 operator values within 1e-10 relative (normwise and max-entry); solves to the
1e-8 true relative residual with the oracle's iteration count +-1."""
import numpy as np
import pytest
import torch

from tests.dense import random_spd_graph
from tests.gpu_util import T, bitwise_levels, both, compare_levels, dev, rel_fro, rel_max
from workloads import (front_c1, front_moving, lognormal_27pt, rhs_uniform, two_fluid_7pt)

pytestmark = pytest.mark.gpu

SETUP_CASES = {
    "tf16": (lambda: two_fluid_7pt(16, front_c1(0)), dict(coarse_enough=32)),
    "tf32_c1": (lambda: two_fluid_7pt(32, front_c1(0)), dict()),
    "box_5x7x9": (lambda: two_fluid_7pt(5, 0.5, ny=7, nz=9), dict(coarse_enough=8)),
    "box_33x17x9": (lambda: two_fluid_7pt(33, 0.4, ny=17, nz=9), dict()),
    "rand500": (lambda: random_spd_graph(500, 4, 3), dict(coarse_enough=20)),
    "ln27_10": (lambda: lognormal_27pt(10, 0), dict(eps_strong=0.02, coarse_enough=16)),
    "tf24_plain": (lambda: two_fluid_7pt(24, 0.45), dict(aggregation=1)),
    "tf24_spai0": (lambda: two_fluid_7pt(24, 0.45), dict(smoother=1)),
}


@pytest.mark.parametrize("name", list(SETUP_CASES))
def test_setup_parity(name):
    make, prm = SETUP_CASES[name]
    p, c, v = make()
    print(f"case {name} n={len(p) - 1}", flush=True)
    g, o = both(p, c, v, **prm)
    compare_levels(g, o, tol=1e-10)


@pytest.mark.parametrize("name", ["tf32_c1", "box_33x17x9", "rand500", "tf24_spai0"])
def test_setup_fp64_bitwise(name):
    """Stronger than required: the FP64 hierarchy is bitwise the oracle's, because every
    Galerkin entry is summed in the oracle's order with separately rounded operations."""
    make, prm = SETUP_CASES[name]
    p, c, v = make()
    g, o = both(p, c, v, **prm)
    assert bitwise_levels(g, o) is None


def test_partial_rebuild_parity():
    N = 32
    p, c, v0 = two_fluid_7pt(N, front_c1(0))
    g, o = both(p, c, v0)
    for t in (2, 5, 9):
        _, _, vt = two_fluid_7pt(N, front_c1(t))
        g.rebuild(T(vt))
        o.rebuild(vt, 0)
        compare_levels(g, o, tol=1e-10)
        assert bitwise_levels(g, o) is None
    # the coarse inverse matches the inverse of the oracle's coarsest operator
    top = o.num_levels - 1
    Ac = np.zeros((o.dims(top)[0],) * 2)
    ptr, col, val = o.level(top)["A"]
    for i in range(len(ptr) - 1):
        Ac[i, col[ptr[i]:ptr[i + 1]]] = val[ptr[i]:ptr[i + 1]]
    assert rel_max(g.coarse_inverse(), np.linalg.inv(Ac)) <= 1e-11


def _snapshot(g):
    return [(g.level(l)["A"][2].copy(), None if g.level(l)["m"] is None else g.level(l)["m"].copy())
            for l in range(g.num_levels)], g.coarse_inverse()


def test_step0_partial_equals_setup_gpu():
    p, c, v = two_fluid_7pt(32, front_c1(0))
    from paper_2108_02054_amd import AMG
    g = AMG(T(p), T(c), T(v))
    a, ia = _snapshot(g)
    g.rebuild(T(v))
    b, ib = _snapshot(g)
    for (x0, m0), (x1, m1) in zip(a, b):
        assert np.array_equal(x0, x1)
        assert (m0 is None and m1 is None) or np.array_equal(m0, m1)
    assert np.array_equal(ia, ib)


@pytest.mark.parametrize("smoother", [0, 1])
def test_power_of_two_scaling_gpu(smoother):
    from paper_2108_02054_amd import AMG
    p, c, v = two_fluid_7pt(24, front_moving(24, 0))
    _, _, v2 = two_fluid_7pt(24, front_moving(24, 3))
    g = AMG(T(p), T(c), T(v), smoother=smoother)
    g.rebuild(T(v2))
    a, ia = _snapshot(g)
    g.rebuild(T(2.0 * v2))
    b, ib = _snapshot(g)
    for (x0, m0), (x1, m1) in zip(a, b):
        assert np.array_equal(2.0 * x0, x1)
        if m0 is not None:
            assert np.array_equal(0.5 * m0, m1)
    assert np.array_equal(0.5 * ia, ib)


@pytest.mark.parametrize("N,prm", [(16, dict(coarse_enough=32)), (32, dict()), (48, dict(smoother=1))])
def test_solve_parity(N, prm):
    p, c, v = two_fluid_7pt(N, front_c1(4))
    g, o = both(p, c, v, **prm)
    f = rhs_uniform(N**3, 1, 4)
    u, info = g.solve(T(f))
    uo, io = o.solve(f)
    print(f"N={N} gpu {info} oracle {io}", flush=True)
    assert info["converged"] and info["rel_res_true"] <= 1e-8
    assert abs(info["iters"] - io["iters"]) <= 1
    assert rel_fro(u.cpu().numpy(), uo) <= 1e-6


def test_vcycle_parity():
    p, c, v = two_fluid_7pt(32, 0.5)
    g, o = both(p, c, v)
    r = np.random.default_rng(5).standard_normal(32**3)
    z = g.vcycle(T(r)).cpu().numpy()
    zo = o.vcycle(r)
    assert rel_fro(z, zo) <= 1e-12


def test_single_level_direct():
    p, c, v = two_fluid_7pt(5, 0.5)
    g, o = both(p, c, v, coarse_enough=200)
    assert g.num_levels == 1
    f = rhs_uniform(125, 1, 0)
    u, info = g.solve(T(f))
    assert info["iters"] == 1 and info["converged"]
    uo, _ = o.solve(f)
    assert rel_max(u.cpu().numpy(), uo) <= 1e-12


def test_transfer_closed_forms_gpu():
    import scipy.sparse as sp
    from paper_2108_02054_amd import AMG

    def to_csr(M):
        S = sp.csr_matrix(M)
        S.sort_indices()
        return S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64)

    def agg1d(n, s):
        P = np.zeros((n, n // s))
        P[np.arange(n), np.arange(n) // s] = 1.0
        return P

    m = 7
    A = 2 * np.eye(3 * m) - np.eye(3 * m, k=1) - np.eye(3 * m, k=-1)
    Pp, Pc, Pv = to_csr(agg1d(3 * m, 3))
    g = AMG(*(T(a) for a in to_csr(A)), transfer=[(T(Pp), T(Pc), T(Pv), m)], coarse_enough=1)
    lv = g.level(1)
    Ac = np.zeros((m, m))
    for i in range(m):
        Ac[i, lv["A"][1][lv["A"][0][i]:lv["A"][0][i + 1]]] = lv["A"][2][lv["A"][0][i]:lv["A"][0][i + 1]]
    assert np.array_equal(Ac, 2 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1))

    m = 3
    p, c, v = two_fluid_7pt(3 * m, 0.0)
    p1 = agg1d(3 * m, 3)
    Pp, Pc, Pv = to_csr(np.kron(np.kron(p1, p1), p1))
    g = AMG(T(p), T(c), T(v), transfer=[(T(Pp), T(Pc), T(Pv), m**3)], coarse_enough=1)
    pm, cm, vm = two_fluid_7pt(m, 0.0)
    lv = g.level(1)
    assert np.array_equal(lv["A"][0], pm) and np.array_equal(lv["A"][1], cm)
    assert np.array_equal(lv["A"][2], 9.0 * vm)


def test_full_reuse_and_full_rebuild_modes():
    from paper_2108_02054_amd import AMG, FULL, OPERATOR_ONLY
    N = 24
    p, c, v0 = two_fluid_7pt(N, 0.3)
    _, _, v1 = two_fluid_7pt(N, 0.3 + 1 / N)
    f = rhs_uniform(N**3, 2, 1)
    g, o = both(p, c, v0, coarse_enough=100)
    g.rebuild_ex(T(v1), OPERATOR_ONLY)
    o.rebuild(v1, 2)
    _, ig = g.solve(T(f))
    _, io = o.solve(f)
    print("full reuse", ig, io, flush=True)
    assert ig["converged"] == io["converged"]
    assert abs(ig["iters"] - io["iters"]) <= 2
    # the hierarchy is untouched by the operator-only update
    assert np.array_equal(g.level(0)["A"][2], v0)
    g.rebuild_ex(T(v1), FULL)
    fresh = AMG(T(p), T(c), T(v1), coarse_enough=100)
    for l in range(fresh.num_levels):
        a, b = g.level(l), fresh.level(l)
        assert np.array_equal(a["A"][2], b["A"][2]) and np.array_equal(a["A"][1], b["A"][1])
        if a["agg"] is not None:
            assert np.array_equal(a["agg"], b["agg"])


def test_pattern_change_same_size_keeps_transfer():
    """New pattern, same n: P_l kept, Galerkin patterns recomputed.  Reference: the oracle
    with the GPU's (kept) transfer operators prescribed."""
    import oracle
    from paper_2108_02054_amd import AMG
    N = 10
    p, c, v = two_fluid_7pt(N, 0.5)
    g = AMG(T(p), T(c), T(v), coarse_enough=20)
    Ps = [g.level(l)["P"] for l in range(g.num_levels - 1)]
    p2, c2, v2 = lognormal_27pt(N, 0)
    g.set_pattern(T(p2), T(c2))
    g.rebuild(T(v2), pattern_changed=True)
    o = oracle.OracleHierarchy(p2, c2, v2, transfer=Ps, coarse_enough=20)
    assert g.num_levels == o.num_levels
    for l in range(o.num_levels):
        gl, ol = g.level(l), o.level(l)
        assert np.array_equal(gl["A"][0], ol["A"][0]) and np.array_equal(gl["A"][1], ol["A"][1])
        assert rel_max(gl["A"][2], ol["A"][2]) <= 1e-10
    f = rhs_uniform(N**3, 5, 0)
    _, info = g.solve(T(f))
    assert info["converged"]


def test_pattern_change_new_size_runs_full_setup():
    from paper_2108_02054_amd import AMG
    p, c, v = two_fluid_7pt(10, 0.5)
    g = AMG(T(p), T(c), T(v), coarse_enough=20)
    p2, c2, v2 = two_fluid_7pt(12, 0.5)
    g.set_pattern(T(p2), T(c2))
    g.rebuild(T(v2), pattern_changed=True)
    fresh = AMG(T(p2), T(c2), T(v2), coarse_enough=20)
    assert g.num_levels == fresh.num_levels
    for l in range(g.num_levels):
        assert np.array_equal(g.level(l)["A"][2], fresh.level(l)["A"][2])


def test_error_paths():
    from paper_2108_02054_amd import AMG, AmgError
    p, c, v = two_fluid_7pt(6, 0.5)
    g = AMG(T(p), T(c), T(v), coarse_enough=20)
    with pytest.raises(AmgError) as e:
        g.rebuild(T(v), pattern_changed=True)
    assert e.value.code == -1
    c_bad = c.copy()
    c_bad[1], c_bad[2] = c_bad[2], c_bad[1]
    with pytest.raises(AmgError) as e:
        AMG(T(p), T(c_bad), T(v))
    assert e.value.code == -1
    v_bad = v.copy()
    v_bad[p[3]:p[4]][c[p[3]:p[4]] == 3] = -1.0
    with pytest.raises(AmgError) as e:
        AMG(T(p), T(c), T(v_bad))
    assert e.value.code == -5
    # drop one entry of a symmetric pair: not structurally symmetric
    keep = np.ones(len(c), bool)
    row0 = slice(p[0], p[1])
    k = p[0] + int(np.where(c[row0] == 1)[0][0])
    keep[k] = False
    counts = np.diff(p) - np.bincount(np.repeat(np.arange(len(p) - 1), np.diff(p))[~keep], minlength=len(p) - 1)
    p_ns = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    with pytest.raises(AmgError) as e:
        AMG(T(p_ns), T(c[keep]), T(v[keep]), coarse_enough=20)
    assert e.value.code == -4
    g2 = AMG(T(p), T(c), T(v), coarse_enough=20, maxiter=1)
    _, info = g2.solve(T(rhs_uniform(216, 1, 0)))
    assert not info["converged"] and info["iters"] == 1
    # NaN values in a partial update surface as a failed coarse factorisation at the solve
    vn = v.copy()
    vn[5] = np.nan
    g.rebuild(T(vn))
    with pytest.raises(AmgError) as e:
        g.solve(T(rhs_uniform(216, 1, 0)))
    assert e.value.code == -5


def test_determinism():
    from paper_2108_02054_amd import AMG
    p, c, v = two_fluid_7pt(32, front_c1(3))
    f = T(rhs_uniform(32**3, 1, 3))
    a = AMG(T(p), T(c), T(v))
    b = AMG(T(p), T(c), T(v))
    assert bitwise_levels_gpu(a, b)
    ua, ia = a.solve(f)
    ub, ib = b.solve(f)
    assert ia == ib and torch.equal(ua, ub)


def bitwise_levels_gpu(a, b):
    for l in range(a.num_levels):
        x, y = a.level(l), b.level(l)
        if not (np.array_equal(x["A"][2], y["A"][2]) and (x["m"] is None or np.array_equal(x["m"], y["m"]))):
            return False
    return True


def test_zero_rhs_and_exact_guess():
    p, c, v = two_fluid_7pt(8, 0.5)
    g, o = both(p, c, v, coarse_enough=30)
    u, info = g.solve(T(np.zeros(512)), T(np.ones(512)))
    assert info["iters"] == 0 and float(u.abs().max()) == 0.0


def test_lane_group_kernels_parity(monkeypatch):
    """The lane-group fallbacks (used where rows are too long to stage in LDS) give the
    same hierarchy and solve as the staged kernels."""
    monkeypatch.setenv("AMGMI_ROW_KERNELS", "lanes")
    p, c, v0 = two_fluid_7pt(32, front_c1(0))
    _, _, v1 = two_fluid_7pt(32, front_c1(5))
    g, o = both(p, c, v0)
    g.rebuild(T(v1))
    o.rebuild(v1, 0)
    compare_levels(g, o, tol=1e-10)
    assert bitwise_levels(g, o) is None
    f = rhs_uniform(32**3, 1, 5)
    u, info = g.solve(T(f))
    uo, io = o.solve(f)
    assert info["converged"] and abs(info["iters"] - io["iters"]) <= 1
    assert rel_fro(u.cpu().numpy(), uo) <= 1e-6


GALERKIN_FORMS = ["pos", "pos:4", "pos:16", "pos:64", "pos:4:2", "pos:8:2", "pos:32:2", "pos16", "pos16:4:2",
                  "lanes", "nodia"]


@pytest.mark.parametrize("form", GALERKIN_FORMS)
@pytest.mark.parametrize("smoother", [0, 1])
def test_galerkin_forms_parity(monkeypatch, form, smoother):
    """Every Galerkin form (the position-map form at several lanes per row, with one or
    two terms per lane and entry, with one- and two-byte positions, the lane-group kernels,
    and with level 0 in CSR rather than diagonal storage) gives the oracle's FP64 hierarchy bit for bit after a partial
    rebuild, with the fused value ingest and smoother diagonal, on 7-point and 27-point
    patterns."""
    if form == "nodia":  # level 0 in CSR
        monkeypatch.setenv("AMGMI_NO_DIA", "1")
    else:
        monkeypatch.setenv("AMGMI_GALERKIN", form)
    print(f"form {form} smoother {smoother}", flush=True)
    p, c, v0 = two_fluid_7pt(32, front_c1(0))
    _, _, v1 = two_fluid_7pt(32, front_c1(5))
    g, o = both(p, c, v0, smoother=smoother)
    g.rebuild(T(v1))
    o.rebuild(v1, 0)
    assert bitwise_levels(g, o) is None
    p, c, v0 = lognormal_27pt(12, 0)
    _, _, v1 = lognormal_27pt(12, 3)
    g, o = both(p, c, v0, smoother=smoother, eps_strong=0.02, coarse_enough=16)
    g.rebuild(T(v1))
    o.rebuild(v1, 0)
    assert bitwise_levels(g, o) is None


@pytest.mark.parametrize("npre,npost,precision", [(1, 1, 0), (2, 2, 0), (0, 1, 0), (1, 1, 1)])
def test_coarse_tail_matches_level_kernels(monkeypatch, npre, npost, precision):
    """The one-workgroup coarse tail computes the same V-cycle as the per-level kernels
    (Algorithm 2; the row sums differ only in their order), and both match the oracle."""
    p, c, v = two_fluid_7pt(32, 0.5)
    r = np.random.default_rng(7).standard_normal(32**3)
    prm = dict(npre=npre, npost=npost, precision=precision, coarse_enough=128)  # a 19-row coarsest level
    g = __import__("paper_2108_02054_amd").AMG(T(p), T(c), T(v), **prm)
    assert g.level_storage(g.num_levels - 1)["tail"] == 1  # the coarsest level (27 rows) runs in the tail
    z_tail = g.vcycle(T(r)).cpu().numpy()
    monkeypatch.setenv("AMGMI_NO_TAIL", "1")
    h = __import__("paper_2108_02054_amd").AMG(T(p), T(c), T(v), **prm)
    assert h.level_storage(h.num_levels - 1)["tail"] == 0
    z_sep = h.vcycle(T(r)).cpu().numpy()
    tol = 1e-12 if precision == 0 else 1e-5
    assert rel_fro(z_tail, z_sep) <= tol
    if precision == 0:
        import oracle
        o = oracle.OracleHierarchy(p, c, v, npre=npre, npost=npost, coarse_enough=128)
        assert rel_fro(z_tail, o.vcycle(r)) <= 1e-12


@pytest.mark.parametrize("case,precision", [("tf32", 0), ("tf32", 1), ("ln27", 0), ("box", 0)])
def test_diagonal_storage_matches_csr(monkeypatch, case, precision):
    """The level-0 kernels on the diagonal storage of a stencil operator compute the same
    V-cycle and solve as the CSR kernels (row sums in a different order only)."""
    from paper_2108_02054_amd import AMG

    if case == "tf32":
        p, c, v0 = two_fluid_7pt(32, front_c1(0))
        v1 = two_fluid_7pt(32, front_c1(4))[2]
        prm = dict()
    elif case == "ln27":
        p, c, v0 = lognormal_27pt(16, 0)
        v1 = lognormal_27pt(16, 2)[2]
        prm = dict(eps_strong=0.02)
    else:
        p, c, v0 = two_fluid_7pt(33, 0.4, ny=17, nz=9)
        v1 = two_fluid_7pt(33, 0.45, ny=17, nz=9)[2]
        prm = dict()
    prm["precision"] = precision
    n = len(p) - 1
    r = np.random.default_rng(11).standard_normal(n)
    f = rhs_uniform(n, 1, 3)

    def run():
        g = AMG(T(p), T(c), T(v0), **prm)
        g.rebuild(T(v1))
        z = g.vcycle(T(r)).cpu().numpy()
        u, info = g.solve(T(f))
        out = (z, u.cpu().numpy(), info)
        g.close()
        return out

    zd, ud, idia = run()
    monkeypatch.setenv("AMGMI_NO_DIA", "1")
    zc, uc, icsr = run()
    tol = 1e-12 if precision == 0 else 1e-5
    assert rel_fro(zd, zc) <= tol
    assert idia["converged"] and icsr["converged"]
    assert abs(idia["iters"] - icsr["iters"]) <= 1
    assert rel_fro(ud, uc) <= 1e-7


@pytest.mark.parametrize("case", ["tf32", "ln27", "aniso"])
@pytest.mark.parametrize("precision", [0, 1])
def test_symmetric_diagonal_read_is_exact(monkeypatch, case, precision):
    """Once a solve has seen symmetric values, the level-0 kernels read each sub-diagonal
    entry of the diagonal storage as its mirror on the super-diagonal: the same numbers in
    the same order, so V-cycles, iterates and iteration counts equal those of the full read
    bit for bit.  Values made unsymmetric in one entry are caught at the rebuild and read in
    full."""
    from paper_2108_02054_amd import AMG

    if case == "tf32":
        p, c, v0 = two_fluid_7pt(32, front_c1(0))
        v1 = two_fluid_7pt(32, front_c1(4))[2]
        prm, nd = dict(), 7
    elif case == "ln27":
        p, c, v0 = lognormal_27pt(16, 0)
        v1 = lognormal_27pt(16, 2)[2]
        prm, nd = dict(eps_strong=0.02), 27
    else:
        p, c, v0 = two_fluid_7pt(33, 0.4, ny=17, nz=9)
        v1 = two_fluid_7pt(33, 0.45, ny=17, nz=9)[2]
        prm, nd = dict(), 7
    prm["precision"] = precision
    n = len(p) - 1
    r = np.random.default_rng(12).standard_normal(n)
    f1, f2 = rhs_uniform(n, 1, 3), rhs_uniform(n, 2, 4)
    # one off-diagonal entry of a middle row scaled: the pattern stays, the values are not
    # symmetric any more
    row = n // 2
    k = next(t for t in range(p[row], p[row + 1]) if c[t] != row)
    v1_bad = v1.copy()
    v1_bad[k] *= 1.0 + 1e-6

    def run(vals):
        g = AMG(T(p), T(c), T(v0), **prm)
        assert g.level_format(0) == nd
        g.rebuild(T(vals))
        u1, i1 = g.solve(T(f1))
        z = g.vcycle(T(r)).cpu().numpy()
        u2, i2 = g.solve(T(f2))
        out = (g.diagonals_read(0), z, u1.cpu().numpy(), u2.cpu().numpy(), i1["iters"], i2["iters"])
        g.close()
        return out

    sym = run(v1)
    bad = run(v1_bad)
    monkeypatch.setenv("AMGMI_NO_DIA_SYM", "1")
    full = run(v1)
    full_bad = run(v1_bad)
    assert sym[0] == (nd + 1) // 2 and full[0] == nd
    assert bad[0] == nd and full_bad[0] == nd
    for a, b in ((sym, full), (bad, full_bad)):
        for x, y in zip(a[1:4], b[1:4]):
            assert np.array_equal(x, y)
        assert a[4:] == b[4:]


@pytest.mark.parametrize("shape", [(32, 32, 32), (33, 17, 9), (260, 3, 5), (5, 6, 40)])
@pytest.mark.parametrize("precision", [0, 1])
def test_marching_kernels_match_row_kernels(monkeypatch, shape, precision):
    """The 7-point marching kernels (a workgroup walks planes of the grid, neighbours from
    registers and LDS) give every row the same result as the one-row-per-thread kernels:
    V-cycles agree bit for bit; solves, whose dot products are grouped differently, agree
    in iterations and to the solver tolerance.  Shapes: whole segments; a plane that is
    not a whole number of segments with an odd last chunk of planes; lines longer than a
    workgroup (every -+b neighbour from global memory); planes shorter than a workgroup."""
    from paper_2108_02054_amd import AMG

    nx, ny, nz = shape
    p, c, v0 = two_fluid_7pt(nx, 0.4, ny=ny, nz=nz)
    v1 = two_fluid_7pt(nx, 0.47, ny=ny, nz=nz)[2]
    n = len(p) - 1
    r = np.random.default_rng(13).standard_normal(n)
    f = rhs_uniform(n, 1, 3)
    print(f"case {shape} precision {precision}", flush=True)

    def run():
        g = AMG(T(p), T(c), T(v0), precision=precision)
        assert g.level_format(0) == 7
        g.rebuild(T(v1))
        u1, i1 = g.solve(T(f))
        z = g.vcycle(T(r)).cpu().numpy()
        out = (z, u1.cpu().numpy(), i1)
        g.close()
        return out

    zm, um, im = run()
    monkeypatch.setenv("AMGMI_NO_MARCH", "1")
    zr, ur, ir = run()
    assert np.array_equal(zm, zr)
    assert im["converged"] and ir["converged"]
    assert abs(im["iters"] - ir["iters"]) <= 1
    assert rel_fro(um, ur) <= 1e-7


@pytest.mark.parametrize("case", ["ln27_16", "ln27_17", "ln27_20", "tf7_nomarch"])
@pytest.mark.parametrize("precision", [0, 1])
def test_windowed_kernels_match_row_kernels(monkeypatch, case, precision):
    """The windowed diagonal-storage kernels (vector entries of each offset cluster staged
    in LDS per workgroup; with 27 diagonals two FP64 or four FP32 rows per thread) give
    every row the one-row-per-thread result bit for bit: the 27-point operator on grids
    whose plane is and is not a multiple of a workgroup and whose row count is odd (17^3:
    the last thread has one row), and a 7-point operator with the marching kernels
    switched off."""
    from paper_2108_02054_amd import AMG

    if case.startswith("ln27"):
        N = int(case.split("_")[1])
        p, c, v0 = lognormal_27pt(N, 0)
        v1 = lognormal_27pt(N, 2)[2]
        prm = dict(eps_strong=0.02)
    else:
        monkeypatch.setenv("AMGMI_NO_MARCH", "1")
        p, c, v0 = two_fluid_7pt(33, 0.4, ny=17, nz=9)
        v1 = two_fluid_7pt(33, 0.45, ny=17, nz=9)[2]
        prm = dict()
    prm["precision"] = precision
    monkeypatch.setenv("AMGMI_WIN_ALL", "1")  # the V-cycle kernels too
    n = len(p) - 1
    r = np.random.default_rng(14).standard_normal(n)
    f = rhs_uniform(n, 1, 3)
    print(f"case {case} precision {precision}", flush=True)

    def run():
        g = AMG(T(p), T(c), T(v0), **prm)
        g.rebuild(T(v1))
        u1, i1 = g.solve(T(f))
        z = g.vcycle(T(r)).cpu().numpy()
        out = (z, u1.cpu().numpy(), i1)
        g.close()
        return out

    zw, uw, iw = run()
    monkeypatch.setenv("AMGMI_NO_WIN", "1")
    zr, ur, ir = run()
    assert np.array_equal(zw, zr)
    assert iw["converged"] and ir["converged"]
    assert abs(iw["iters"] - ir["iters"]) <= 1
    assert rel_fro(uw, ur) <= 1e-7


@pytest.mark.parametrize("N", [16, 17, 20, 84])
def test_two_row_krylov_spmv_is_exact(monkeypatch, N):
    """The 27-point Krylov SpMV with two rows per thread (one 16-byte load per diagonal for
    both rows' entries, windows of 512 rows) gives y = A x equal bit for bit to the one-row
    windowed kernel's and the one-row-per-thread kernel's, with the full read and with the
    symmetric read, for an even row count, an odd one (17^3, whose last thread has one row)
    and counts that are not a multiple of 512; y also agrees with a host product.  At 84^3
    the windowed initial and final residual runs on 1158 workgroups, more than the 1024
    partials of the bounded grids, and its true residual agrees with the row kernel's."""
    import scipy.sparse as sp

    from paper_2108_02054_amd import AMG

    p, c, v0 = lognormal_27pt(N, 0)
    v1 = lognormal_27pt(N, 2)[2]
    n = len(p) - 1
    x = np.random.default_rng(16).standard_normal(n)
    f = rhs_uniform(n, 1, 3)
    print(f"N {N} n {n}", flush=True)

    def run():
        g = AMG(T(p), T(c), T(v0), eps_strong=0.02)
        g.rebuild(T(v1))
        y_full = g.apply_operator(T(x)).cpu().numpy()
        u, info = g.solve(T(f))
        y_sym = g.apply_operator(T(x)).cpu().numpy()
        out = (y_full, y_sym, g.diagonals_read(0), u.cpu().numpy(), info)
        g.close()
        return out

    two = run()
    monkeypatch.setenv("AMGMI_NO_WIN2", "1")
    one = run()
    monkeypatch.setenv("AMGMI_NO_WIN", "1")
    row = run()
    assert two[2] == 14 and one[2] == 14 and row[2] == 14
    for other in (one, row):
        assert np.array_equal(two[0], other[0])
        assert np.array_equal(two[1], other[1])
        assert abs(two[4]["iters"] - other[4]["iters"]) <= 1
        assert rel_fro(two[3], other[3]) <= 1e-7
    assert np.array_equal(two[0], two[1])
    A = sp.csr_matrix((v1, c, p), shape=(n, n))
    assert rel_max(two[0], A @ x) <= 1e-13
    assert two[4]["converged"]
    res = np.linalg.norm(f - A @ two[3]) / np.linalg.norm(f)
    assert abs(two[4]["rel_res_true"] - res) <= 1e-3 * res, (two[4]["rel_res_true"], res)


@pytest.mark.parametrize("precision", [0, 1])
def test_two_byte_columns_change_nothing(monkeypatch, precision):
    """The row-block kernels reading two-byte block-relative column indices (64^3: level 0's
    P and R and level 1's operator qualify) give the int32 kernels' results bit for bit."""
    from paper_2108_02054_amd import AMG

    p, c, v0 = two_fluid_7pt(64, front_moving(64, 0))
    v1 = two_fluid_7pt(64, front_moving(64, 2))[2]
    n = len(p) - 1
    r = np.random.default_rng(15).standard_normal(n)
    f = rhs_uniform(n, 2, 2)

    def run():
        g = AMG(T(p), T(c), T(v0), precision=precision)
        g.rebuild(T(v1))
        u, info = g.solve(T(f))
        z = g.vcycle(T(r)).cpu().numpy()
        out = (z, u.cpu().numpy(), info["iters"])
        g.close()
        return out

    a = run()
    monkeypatch.setenv("AMGMI_NO_C16", "1")
    b = run()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_full_size_128_partial_rebuild_and_solve():
    """At the benchmark's full size (two-fluid 128^3, the configuration bench.py times,
    with the diagonal storage and the default launch shapes): after a partial rebuild to a
    later step, every level's aggregates and patterns match the oracle's bit for bit and
    its FP64 values too (summed in the oracle's order); the solve converges to 1e-8 in the
    oracle's iteration count +-1 with a solution within 1e-6."""
    N = 128
    p, c, v0 = two_fluid_7pt(N, front_moving(N, 0))
    v5 = two_fluid_7pt(N, front_moving(N, 5))[2]
    print("case two-fluid 128^3 step 0 -> 5", flush=True)
    g, o = both(p, c, v0)
    assert g.level_format(0) == 7
    g.rebuild(T(v5))
    o.rebuild(v5, 0)
    compare_levels(g, o, tol=1e-10)
    assert bitwise_levels(g, o) is None
    f = rhs_uniform(N**3, 2, 5)
    u, info = g.solve(T(f))
    uo, io = o.solve(f)
    assert info["converged"] and info["rel_res_true"] <= 1e-8
    assert abs(info["iters"] - io["iters"]) <= 1
    assert rel_fro(u.cpu().numpy(), uo) <= 1e-6


@pytest.mark.parametrize("precision,flexible", [(0, 0), (1, 0), (0, 1)])
def test_host_mirror_matches_copy(monkeypatch, precision, flexible):
    """The CG update kernels write the ||r||^2 partials and the breakdown flag straight into
    mapped host memory; the solve then takes exactly the decisions, iterations and iterates
    it takes when they are copied back after the kernel (over several solves and rebuilds)."""
    from paper_2108_02054_amd import AMG

    p, c, v0 = two_fluid_7pt(32, front_c1(0))
    vals = [two_fluid_7pt(32, front_c1(t))[2] for t in (1, 2, 3)]

    def run():
        g = AMG(T(p), T(c), T(v0), precision=precision, flexible_cg=flexible)
        out = []
        for t, vt in enumerate(vals):
            g.rebuild(T(vt))
            u, info = g.solve(T(rhs_uniform(32**3, 1, t)))
            out.append((info["iters"], info["converged"], u.cpu().numpy()))
        g.close()
        return out

    mapped = run()
    monkeypatch.setenv("AMGMI_NO_HOST_WRITE", "1")
    copied = run()
    for (im, cm, um), (ic, cc, uc) in zip(mapped, copied):
        assert cm and cc and im == ic
        assert np.array_equal(um, uc)



@pytest.mark.parametrize("dims,precision", [((5, 5, 6), 0), ((9, 9, 9), 0), ((12, 12, 12), 0), ((8, 16, 16), 0),
                                            ((9, 9, 9), 1)])
def test_blocked_coarse_inverse(dims, precision):
    """Coarsest levels above the 128 rows one workgroup's LDS holds are inverted by the
    blocked Gauss-Jordan kernels (64-pivot blocks, ragged last block): a one-level hierarchy
    (150 to 2048 rows) is a direct solve, one CG iteration, and its inverse matches NumPy's
    (of the FP32-rounded operator in mixed precision)."""
    from paper_2108_02054_amd import AMG
    nx, ny, nz = dims
    n = nx * ny * nz
    p, c, v = two_fluid_7pt(nx, 0.45, ny=ny, nz=nz)
    print(f"case blocked coarse inverse n={n} precision {precision}", flush=True)
    g = AMG(T(p), T(c), T(v), coarse_enough=2048, precision=precision)
    assert g.num_levels == 1
    A = np.zeros((n, n))
    for i in range(n):
        A[i, c[p[i]:p[i + 1]]] = v[p[i]:p[i + 1]] if precision == 0 else v[p[i]:p[i + 1]].astype(np.float32)
    assert rel_max(g.coarse_inverse(), np.linalg.inv(A)) <= 1e-11
    f = rhs_uniform(n, 1, 0)
    u, info = g.solve(T(f))
    assert info["converged"] and info["iters"] <= (1 if precision == 0 else 3)
    print(f"n={n}: coarse inverse {g.phase_times()['coarse']:.3f} ms at setup", flush=True)
    g.close()


def test_coarse_inverse_beside_the_solve(monkeypatch):
    """The blocked inverse of a partial update runs on the context's side stream: its traced
    time reads right after the update; exported then it is the inverse of the new coarsest
    operator; two updates in a
    row followed by a solve give the oracle's iterations; a NaN value makes the next CG and
    BiCGStab solves report a coarsest operator that is not SPD."""
    import oracle
    from paper_2108_02054_amd import AMG, AmgError
    monkeypatch.setenv("AMGMI_NO_TAIL", "1")  # the side stream serves only levels outside a tail
    p, c, v0 = two_fluid_7pt(32, front_c1(0))
    _, _, v1 = two_fluid_7pt(32, front_c1(2))
    _, _, v2 = two_fluid_7pt(32, front_c1(4))
    print("case coarse inverse beside the solve (32^3)", flush=True)
    g = AMG(T(p), T(c), T(v0))
    nL = g.dims(g.num_levels - 1)[0]
    assert nL > 128, nL  # the blocked inverse
    g.trace(["coarse_inv"], level=-1)
    g.rebuild(T(v1))
    t = g.trace_read()  # its events were recorded on the side stream: read before any solve
    assert t["coarse_inv"][1] == 1 and t["coarse_inv"][0] > 0, t
    g.trace([], level=0)
    L = g.level(g.num_levels - 1)
    Ap, Ac, Av = L["A"]
    A = np.zeros((nL, nL))
    for i in range(nL):
        A[i, Ac[Ap[i]:Ap[i + 1]]] = Av[Ap[i]:Ap[i + 1]]
    assert rel_max(g.coarse_inverse(), np.linalg.inv(A)) <= 1e-11
    g.rebuild(T(v2))
    o = oracle.OracleHierarchy(p, c, v0)
    o.rebuild(v2, 0)
    f = rhs_uniform(32**3, 1, 4)
    u, info = g.solve(T(f))
    uo, io = o.solve(f)
    assert info["converged"] and abs(info["iters"] - io["iters"]) <= 1
    assert rel_max(u.cpu().numpy(), uo) <= 1e-6
    vn = v2.copy()
    vn[7] = np.nan
    for solver in ("solve", "solve_bicgstab"):
        g.rebuild(T(vn))
        with pytest.raises(AmgError) as e:
            getattr(g, solver)(T(f))
        assert e.value.code == -5, (solver, e.value)
    g.rebuild(T(v2))  # the context stays usable
    u, info = g.solve(T(f))
    assert info["converged"]
    g.close()


def test_coarsest_level_too_large_for_the_dense_inverse():
    from paper_2108_02054_amd import AMG, AmgError
    p, c, v = two_fluid_7pt(13, 0.45)  # 2197 rows in one level
    with pytest.raises(AmgError) as e:
        AMG(T(p), T(c), T(v), coarse_enough=4096)
    assert e.value.code == -1 and "dense inverse" in str(e.value)


def test_trace_every_brackets_a_sample():
    """amg_trace_every: with every = 4 only launches 1, 5, 9, ... of a traced class on a
    level are timed (each solve of k iterations launches the Krylov SpMV k times), the
    counts start again at each amg_trace call, and the solution does not change."""
    from paper_2108_02054_amd import AMG

    p, c, v0 = two_fluid_7pt(32, front_c1(0))
    _, _, v1 = two_fluid_7pt(32, front_c1(2))
    f = rhs_uniform(32**3, 1, 2)
    g = AMG(T(p), T(c), T(v0))
    g.rebuild(T(v1))
    g.trace(["cg_pq"], level=0)
    u1, i1 = g.solve(T(f))
    all_ = g.trace_read()["cg_pq"]
    assert all_[1] == i1["iters"] and all_[0] > 0
    g.trace(["cg_pq"], level=0, every=4)
    u2, i2 = g.solve(T(f))
    u3, i3 = g.solve(T(f))
    some = g.trace_read()["cg_pq"]
    assert some[1] == (i2["iters"] + i3["iters"] + 3) // 4, (some, i2["iters"], i3["iters"])
    assert some[0] > 0
    g.trace([], level=0)
    assert torch.equal(u1, u2) and torch.equal(u2, u3)
    with pytest.raises(Exception):
        g.trace(["cg_pq"], level=0, every=0)
    g.close()
