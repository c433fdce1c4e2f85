"""Systems with 4 unknowns per node (the paper's 4x4-block systems, Section 4) on the
device against the oracle: node aggregation bit-exact (node matrix of block norms,
strength, MIS-2, expansion to the unknowns), coarse operators and block Jacobi smoothers
within 1e-10, partial rebuilds over a series, CG and BiCGStab solves, sweep counts, both
row-kernel families, mixed precision, argument errors, and the full-size coupled
56^3-node system that bench.py times."""
import numpy as np
import pytest
import scipy.sparse as sp

from tests.dense import random_spd_graph
from tests.gpu_util import T, both, compare_levels, rel_fro, rel_max
from workloads import rhs_uniform, two_fluid_7pt
from workloads.poisson import coupled4_7pt

pytestmark = pytest.mark.gpu

B = 4
BLOCK = dict(block_size=B, aggregation=1)


@pytest.mark.parametrize("N", [9, 13])
def test_block_setup_parity(N):
    """13^3 nodes = 8788 rows: several 256-row tiles and a ragged tail."""
    p, c, v = coupled4_7pt(N, 2)
    print(f"case coupled4 N={N}", flush=True)
    g, o = both(p, c, v, coarse_enough=128, **BLOCK)
    compare_levels(g, o, tol=1e-10)
    assert g.num_levels >= 3
    g.close()
    o.close()


@pytest.mark.parametrize("seed", [0, 1])
def test_block_kronecker_random_graph(seed):
    pp, cc, vv = random_spd_graph(400, 4, seed)
    rg = np.random.default_rng(seed)
    M = rg.uniform(-1.0, 1.0, size=(B, B))
    K = M @ M.T + B * np.eye(B)
    A = sp.kron(sp.csr_matrix((vv, cc, pp), shape=(400, 400)), sp.csr_matrix(K), format="csr")
    A.sort_indices()
    p, c, v = A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy()
    print(f"case kron seed={seed}", flush=True)
    g, o = both(p, c, v, coarse_enough=32, **BLOCK)
    compare_levels(g, o, tol=1e-10)
    g.close()
    o.close()


@pytest.mark.parametrize("bs", [2, 3, 4, 6])
def test_node_pair_loads(monkeypatch, bs):
    """The node-group residual, sweeps and Krylov product with two adjacent positions per
    lane (even block sizes; odd ones keep one position per lane) form the row sums of the
    one-position form in another order: the product matches SciPy's, and the V-cycle and
    the solve match those of the one-position kernels and the oracle's V-cycle."""
    pp, cc, vv = random_spd_graph(300, 5, 3)
    rg = np.random.default_rng(bs)
    M = rg.uniform(-1.0, 1.0, size=(bs, bs))
    K = M @ M.T + bs * np.eye(bs)
    A = sp.kron(sp.csr_matrix((vv, cc, pp), shape=(300, 300)), sp.csr_matrix(K), format="csr")
    A.sort_indices()
    p, c, v = A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy()
    prm = dict(block_size=bs, aggregation=1, coarse_enough=64)
    print(f"case kron bs={bs}", flush=True)
    g, o = both(p, c, v, **prm)
    x = np.random.default_rng(1).standard_normal(A.shape[0])
    y = g.apply_operator(T(x)).cpu().numpy()
    assert rel_max(y, A @ x) <= 1e-14
    r = np.random.default_rng(2).standard_normal(A.shape[0])
    z = g.vcycle(T(r)).cpu().numpy()
    u, info = g.solve(T(r))
    monkeypatch.setenv("AMGMI_NO_NODE_PAIRS", "1")
    h = __import__("paper_2108_02054_amd").AMG(T(p), T(c), T(v), **prm)
    z1 = h.vcycle(T(r)).cpu().numpy()
    u1, info1 = h.solve(T(r))
    if bs % 2:
        assert np.array_equal(z, z1) and np.array_equal(u.cpu().numpy(), u1.cpu().numpy())
    else:
        assert rel_fro(z, z1) <= 1e-13
        assert rel_fro(u.cpu().numpy(), u1.cpu().numpy()) <= 1e-9
    assert rel_fro(z, o.vcycle(r)) <= 1e-10
    assert info["converged"] and abs(info["iters"] - info1["iters"]) <= 1, (info, info1)
    for m in (g, h, o):
        m.close()


def _kron_system(n, deg, seed, bs, isolate=()):
    pp, cc, vv = random_spd_graph(n, deg, seed)
    G = sp.csr_matrix((vv, cc, pp), shape=(n, n)).tolil()
    for i in isolate:  # a node with its diagonal block only: it joins no aggregate
        d = G[i, i]
        G[i, :] = 0
        G[:, i] = 0
        G[i, i] = d
    G = G.tocsr()
    G.eliminate_zeros()
    rg = np.random.default_rng(seed + bs)
    M = rg.uniform(-1.0, 1.0, size=(bs, bs))
    K = M @ M.T + bs * np.eye(bs)
    A = sp.kron(G, sp.csr_matrix(K), format="csr")
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy()


@pytest.mark.parametrize("case", ["coupled4", "kron3", "kron2_isolated", "mixed"])
def test_node_galerkin_product(monkeypatch, case):
    """A partial update of a block system forms A_{l+1} = R_l A_l P_l in one pass over A_l's
    B x B blocks (Section 4's block values; Alg. 4): bit for bit the scalar position-map
    product's and the oracle's row-by-row product's coarse operators and block smoothers,
    also when a node joins no aggregate (its values then reach the hierarchy by a copy) and
    in the FP32 hierarchy (same solve as the scalar product's)."""
    from paper_2108_02054_amd import AMG
    if case in ("coupled4", "mixed"):
        p, c, v0 = coupled4_7pt(12, 0)
        v1 = coupled4_7pt(12, 3)[2]
        prm = dict(block_size=4, aggregation=1, coarse_enough=128, precision=1 if case == "mixed" else 0)
    else:
        bs = 3 if case == "kron3" else 2
        p, c, v0 = _kron_system(400, 5, 4, bs, isolate=(7, 123) if "isolated" in case else ())
        rg = np.random.default_rng(9)
        v1 = v0 * (1.0 + 0.1 * rg.uniform(size=v0.shape))
        v1 = 0.5 * (v1 + sp.csr_matrix((v1, c, p)).T.tocsr().sorted_indices().data)  # still symmetric
        prm = dict(block_size=bs, aggregation=1, coarse_enough=32)
    print(f"case node galerkin {case}", flush=True)
    g = AMG(T(p), T(c), T(v0), **prm)
    L = g.num_levels
    assert L >= 2
    g.rebuild(T(v1))  # (the first partial update forms the plans)
    assert [g.level_storage(l)["node_galerkin"] for l in range(L - 1)] == [1] * (L - 1)
    monkeypatch.setenv("AMGMI_NO_NODE_GAL", "1")
    h = AMG(T(p), T(c), T(v0), **prm)
    h.rebuild(T(v1))
    assert h.level_storage(0)["node_galerkin"] == 0
    f = rhs_uniform(len(p) - 1, 7, 2)
    u, info = g.solve(T(f))
    uh, ih = h.solve(T(f))
    assert info["converged"] and info["iters"] == ih["iters"], (info, ih)
    assert np.array_equal(u.cpu().numpy(), uh.cpu().numpy())
    if case == "mixed":
        g.close()
        h.close()
        return
    for l in range(L):
        a, b = g.level(l), h.level(l)
        assert np.array_equal(a["A"][2], b["A"][2]), l
        if a["P"] is not None:
            assert np.array_equal(a["m"], b["m"]), l
    import oracle
    o = oracle.OracleHierarchy(p, c, v0, **{k: x for k, x in prm.items() if k != "precision"})
    o.rebuild(v1, 0)
    assert o.num_levels == L
    for l in range(L):
        assert np.array_equal(g.level(l)["A"][2], o.level(l)["A"][2]), l
    for m in (g, h, o):
        m.close()


@pytest.mark.parametrize("case", ["coupled4", "kron3", "kron2_isolated", "mixed"])
def test_node_transfers(monkeypatch, case):
    """The block V-cycle's prolongation through the aggregate of each node (P_l =
    P_node (x) I_B with unit values, Section 4's node aggregation) gives the V-cycle of the
    CSR prolongation bit for bit, the oracle's V-cycle and the same solve, also with nodes
    outside every aggregate and in FP32."""
    from paper_2108_02054_amd import AMG
    if case in ("coupled4", "mixed"):
        p, c, v = coupled4_7pt(12, 1)
        prm = dict(block_size=4, aggregation=1, coarse_enough=128, precision=1 if case == "mixed" else 0)
    else:
        bs = 3 if case == "kron3" else 2
        p, c, v = _kron_system(400, 5, 4, bs, isolate=(7, 123) if "isolated" in case else ())
        prm = dict(block_size=bs, aggregation=1, coarse_enough=32)
    print(f"case node transfers {case}", flush=True)
    g = AMG(T(p), T(c), T(v), **prm)
    L = g.num_levels
    assert [g.level_storage(l)["node_transfer"] for l in range(L - 1)] == [1] * (L - 1)
    monkeypatch.setenv("AMGMI_NO_NODE_TRANSFER", "1")
    h = AMG(T(p), T(c), T(v), **prm)
    assert h.level_storage(0)["node_transfer"] == 0
    r = np.random.default_rng(3).standard_normal(len(p) - 1)
    z, zh = g.vcycle(T(r)).cpu().numpy(), h.vcycle(T(r)).cpu().numpy()
    assert np.array_equal(z, zh)
    f = rhs_uniform(len(p) - 1, 7, 5)
    u, info = g.solve(T(f))
    uh, ih = h.solve(T(f))
    assert info["converged"] and info["iters"] == ih["iters"], (info, ih)
    assert np.array_equal(u.cpu().numpy(), uh.cpu().numpy())
    if case != "mixed":
        import oracle
        o = oracle.OracleHierarchy(p, c, v, **{k: x for k, x in prm.items() if k != "precision"})
        assert rel_fro(z, o.vcycle(r)) <= 1e-10
        o.close()
    g.close()
    h.close()


def test_block_partial_series_and_solves():
    N = 14
    p, c, v0 = coupled4_7pt(N, 0)
    n = len(p) - 1
    print("case coupled4 N=14 series", flush=True)
    g, o = both(p, c, v0, **BLOCK)
    for t in (1, 2, 3):
        v = coupled4_7pt(N, t)[2]
        g.rebuild(T(v))
        o.rebuild(v, 0)
        compare_levels(g, o, tol=1e-10)
        f = rhs_uniform(n, 7, t)
        u, info = g.solve(T(f))
        uo, io = o.solve(f)
        assert info["converged"] and info["rel_res_true"] <= 1e-8, info
        assert abs(info["iters"] - io["iters"]) <= 1, (info, io)
        assert rel_fro(u.cpu().numpy(), uo) <= 1e-6
    u, info = g.solve_bicgstab(T(f))
    uo, io = o.solve_bicgstab(f)
    assert info["converged"] and io["converged"]
    assert abs(info["iters"] - io["iters"]) <= 1, (info, io)
    assert rel_fro(u.cpu().numpy(), uo) <= 1e-6
    g.close()
    o.close()


def test_block_mixed_precision():
    N = 12
    p, c, v0 = coupled4_7pt(N, 0)
    v1 = coupled4_7pt(N, 2)[2]
    print("case coupled4 N=12 mixed", flush=True)
    g, o = both(p, c, v0, precision=1, **BLOCK)
    g.rebuild(T(v1))
    o.rebuild(v1, 0)
    f = rhs_uniform(len(p) - 1, 7, 2)
    u, info = g.solve(T(f))
    uo, io = o.solve(f)
    assert info["converged"] and info["rel_res_true"] <= 1e-8
    assert abs(info["iters"] - io["iters"]) <= 3, (info, io)
    assert rel_fro(u.cpu().numpy(), uo) <= 1e-6
    g.close()
    o.close()


@pytest.mark.parametrize("env,first", [({}, 0), ({"AMGMI_TAIL_SOLO": "128"}, 2), ({"AMGMI_TAIL_NNZ": "200000"}, 1)])
def test_block_coarse_tail(monkeypatch, env, first):
    """The one-workgroup coarse tail on a block system.  A coarsest level alone goes to it only
    up to 64 rows (this system's has 88); forced onto that level (the restriction into it and
    the dense solve), or onto the last two levels (the block smoother applied from LDS as well),
    it computes the V-cycle of the separate launches (row sums in another order) and of the
    oracle (Algorithm 2)."""
    N = 13
    p, c, v = coupled4_7pt(N, 1)
    for k, x in env.items():
        monkeypatch.setenv(k, x)
    print(f"case coupled4 N=13 tail env={env}", flush=True)
    g, o = both(p, c, v, coarse_enough=128, **BLOCK)
    L = g.num_levels
    assert L == 3 and g.dims(L - 1)[0] == 88
    assert [g.level_storage(l)["tail"] for l in range(L)] == [int(first > 0 and l >= first) for l in range(L)]
    r = np.random.default_rng(11).standard_normal(len(p) - 1)
    z = g.vcycle(T(r)).cpu().numpy()
    monkeypatch.setenv("AMGMI_NO_TAIL", "1")
    h = __import__("paper_2108_02054_amd").AMG(T(p), T(c), T(v), coarse_enough=128, **BLOCK)
    assert h.level_storage(L - 1)["tail"] == 0
    z_sep = h.vcycle(T(r)).cpu().numpy()
    assert rel_fro(z, z_sep) <= 1e-12
    assert rel_fro(z, o.vcycle(r)) <= 1e-10
    for x in (g, h, o):
        x.close()


@pytest.mark.parametrize("kernels,npre,npost", [("default", 2, 2), ("default", 0, 2), ("lanes", 1, 1)])
def test_block_sweeps_and_kernel_families(monkeypatch, kernels, npre, npost):
    if kernels == "lanes":
        monkeypatch.setenv("AMGMI_ROW_KERNELS", "lanes")
    N = 11
    p, c, v0 = coupled4_7pt(N, 0)
    v1 = coupled4_7pt(N, 3)[2]
    print(f"case coupled4 N=11 {kernels} npre={npre} npost={npost}", flush=True)
    g, o = both(p, c, v0, npre=npre, npost=npost, **BLOCK)
    g.rebuild(T(v1))
    o.rebuild(v1, 0)
    compare_levels(g, o, tol=1e-10)
    f = rhs_uniform(len(p) - 1, 7, 3)
    u, info = g.solve(T(f))
    uo, io = o.solve(f)
    assert info["converged"] and io["converged"]
    assert abs(info["iters"] - io["iters"]) <= 1, (info, io)
    assert rel_fro(u.cpu().numpy(), uo) <= 1e-6
    r = np.random.default_rng(5).standard_normal(len(p) - 1)
    z = g.vcycle(T(r)).cpu().numpy()
    assert rel_fro(z, o.vcycle(r)) <= 1e-10
    g.close()
    o.close()


def test_block_argument_errors():
    from paper_2108_02054_amd import AMG, AmgError
    p, c, v = coupled4_7pt(3, 0)
    for bad, code in ((dict(block_size=B, aggregation=0), -1),    # needs plain aggregation
                      (dict(block_size=5, aggregation=1), -1),    # 108 rows
                      (dict(block_size=9, aggregation=1), -1),
                      (dict(block_size=0, aggregation=1), -1),
                      (dict(block_size=B, aggregation=1, smoother=1), -1),
                      (dict(block_size=B, aggregation=1, flexible_cg=1), -1)):
        with pytest.raises(AmgError) as e:
            AMG(T(p), T(c), T(v), coarse_enough=8, **bad)
        assert e.value.code == code, bad
    sp_, sc, sv = two_fluid_7pt(4, 0.5)                           # no full 2x2 blocks
    with pytest.raises(AmgError) as e:
        AMG(T(sp_), T(sc), T(sv), coarse_enough=4, block_size=2, aggregation=1)
    assert e.value.code == -4
    with pytest.raises(AmgError) as e:                              # also on a single level
        AMG(T(sp_), T(sc), T(sv), coarse_enough=128, block_size=2, aggregation=1)
    assert e.value.code == -4
    g = AMG(T(p), T(c), T(v), coarse_enough=8, **BLOCK)            # still usable afterwards
    _, info = g.solve(T(rhs_uniform(len(p) - 1, 7, 0)))
    assert info["converged"]
    g1 = AMG(T(p), T(c), T(v), coarse_enough=128, **BLOCK)         # one level: a direct solve
    assert g1.num_levels == 1
    _, info = g1.solve(T(rhs_uniform(len(p) - 1, 7, 0)))
    assert info["converged"] and info["iters"] == 1


def test_full_size_coupled4_56_partial_rebuild_and_solve():
    """The configuration bench.py times for block systems (56^3 nodes, 702,464 rows,
    19.4M entries): after a partial rebuild to a later step every level matches the
    oracle (aggregates and patterns bit for bit, values within 1e-10) and the solve agrees."""
    N = 56
    p, c, v0 = coupled4_7pt(N, 0)
    v5 = coupled4_7pt(N, 5)[2]
    print("case coupled4 56^3 step 0 -> 5", flush=True)
    g, o = both(p, c, v0, **BLOCK)
    print(f"level-0 format {g.level_format(0)}", flush=True)
    g.rebuild(T(v5))
    o.rebuild(v5, 0)
    compare_levels(g, o, tol=1e-10)
    f = rhs_uniform(len(p) - 1, 7, 5)
    u, info = g.solve(T(f))
    uo, io = o.solve(f)
    assert info["converged"] and info["rel_res_true"] <= 1e-8
    assert abs(info["iters"] - io["iters"]) <= 1, (info, io)
    assert rel_fro(u.cpu().numpy(), uo) <= 1e-6
    g.close()
    o.close()


def test_block_rebuild_modes():
    """Full reuse keeps the hierarchy (the Krylov operator alone takes the new values) and
    a full rebuild equals a fresh setup, with block smoothers."""
    from paper_2108_02054_amd import AMG, FULL, OPERATOR_ONLY
    N = 10
    p, c, v0 = coupled4_7pt(N, 0)
    v1 = coupled4_7pt(N, 4)[2]
    f = rhs_uniform(len(p) - 1, 7, 4)
    print("case coupled4 N=10 modes", flush=True)
    g, o = both(p, c, v0, **BLOCK)
    g.rebuild_ex(T(v1), OPERATOR_ONLY)
    o.rebuild(v1, 2)
    _, ig = g.solve(T(f))
    _, io = o.solve(f)
    assert ig["converged"] == io["converged"]
    assert abs(ig["iters"] - io["iters"]) <= 2, (ig, io)
    assert np.array_equal(g.level(0)["A"][2], v0)
    g.rebuild_ex(T(v1), FULL)
    fresh = AMG(T(p), T(c), T(v1), **BLOCK)
    for l in range(fresh.num_levels):
        a, b = g.level(l), fresh.level(l)
        assert np.array_equal(a["A"][2], b["A"][2]) and np.array_equal(a["A"][1], b["A"][1])
        if a["P"] is not None:
            assert np.array_equal(a["m"], b["m"])
    g.close()
    o.close()


def test_block_pattern_change_same_size():
    """A new full-block pattern with the same row count keeps P_l (node aggregates) and
    recomputes the Galerkin patterns (reference: the oracle with those transfer operators);
    a pattern without full blocks is refused."""
    import oracle
    from paper_2108_02054_amd import AMG, AmgError
    from workloads import lognormal_27pt
    N = 8
    p, c, v = coupled4_7pt(N, 0)
    g = AMG(T(p), T(c), T(v), coarse_enough=16, **BLOCK)
    Ps = [g.level(l)["P"] for l in range(g.num_levels - 1)]
    lp, lc, lv = lognormal_27pt(N, 0)
    K = np.array([[3.0, 0.5, 0.2, 0.1], [0.5, 2.0, 0.3, 0.2], [0.2, 0.3, 2.5, 0.4], [0.1, 0.2, 0.4, 1.5]])
    A2 = sp.kron(sp.csr_matrix((lv, lc, lp), shape=(N**3, N**3)), sp.csr_matrix(K), format="csr")
    A2.sort_indices()
    p2, c2, v2 = A2.indptr.astype(np.int32), A2.indices.astype(np.int32), A2.data.copy()
    print("case coupled4 N=8 pattern change", flush=True)
    g.set_pattern(T(p2), T(c2))
    g.rebuild(T(v2), pattern_changed=True)
    o = oracle.OracleHierarchy(p2, c2, v2, transfer=Ps, coarse_enough=16, **BLOCK)
    assert g.num_levels == o.num_levels
    for l in range(o.num_levels):
        gl, ol = g.level(l), o.level(l)
        assert np.array_equal(gl["A"][0], ol["A"][0]) and np.array_equal(gl["A"][1], ol["A"][1])
        assert rel_fro(gl["A"][2], ol["A"][2]) <= 1e-10
        if ol["P"] is not None:
            assert rel_fro(gl["m"], ol["m"]) <= 1e-10
    f = rhs_uniform(len(p2) - 1, 7, 1)
    u, info = g.solve(T(f))
    uo, io = o.solve(f)
    assert info["converged"] and abs(info["iters"] - io["iters"]) <= 1, (info, io)
    sp3, sc3, _ = two_fluid_7pt(N, 0.5, nz=4 * N)                   # same n, scalar pattern
    g.set_pattern(T(sp3), T(sc3))
    with pytest.raises(AmgError) as e:
        g.rebuild(T(np.ones(len(sc3))), pattern_changed=True)
    assert e.value.code == -4
