"""Pins of the oracle for systems with several unknowns per node.

For its monolithic block systems the paper runs plain (non-smoothed) aggregation and
damped Jacobi on 4x4-block matrices (Section 4), where every value is a block.  The
oracle aggregates nodes (strength and MIS-2 on the matrix of block Frobenius norms;
unknown b of a node goes to unknown b of the node's aggregate) and smooths with damped
block Jacobi (omega times the inverse of each node's diagonal block).  The checks use the
Kronecker identity (L (x) K with plain transfer operators P (x) I gives coarse operators
(P^T L P) (x) K and smoother blocks omega / l_ii K^{-1}), node norms and block inverses
computed in NumPy, dense triple products, the textbook two-grid error operator and
structural invariants.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from tests.dense import dense, random_spd_graph
from workloads import two_fluid_7pt
from workloads.poisson import coupled4_7pt, rhs_uniform

B = 4


def _spd_block(seed):
    g = np.random.default_rng(seed)
    M = g.uniform(-1.0, 1.0, size=(B, B))
    K = M @ M.T + B * np.eye(B)
    assert np.all(K != 0.0)
    return K


def _kron(p, c, v, K):
    n = len(p) - 1
    A = sp.kron(sp.csr_matrix((v, c, p), shape=(n, n)), sp.csr_matrix(K), format="csr")
    A.sort_indices()
    assert A.nnz == len(v) * B * B
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy()


def _expand(agg_node):
    a = np.repeat(agg_node.astype(np.int64), B) * B + np.tile(np.arange(B), len(agg_node))
    return np.where(np.repeat(agg_node, B) >= 0, a, -1)


SCALARS = [
    ("tf6", lambda: two_fluid_7pt(6, 0.45)),
    ("rand80", lambda: random_spd_graph(80, 3, 4)),
    ("rand120", lambda: random_spd_graph(120, 4, 5)),
]


@pytest.mark.parametrize("name,make", SCALARS)
def test_kronecker_aggregates_are_the_scalar_ones(ora, name, make):
    """Node norms of L (x) K are |l_ij| ||K||_F, so the strength test and the MIS-2 see
    the scalar graph of L: the node aggregates are those of L, repeated per unknown."""
    p, c, v = make()
    ap, ac, av = _kron(p, c, v, _spd_block(1))
    hs = ora.OracleHierarchy(p, c, v, aggregation=1, coarse_enough=4)
    hb = ora.OracleHierarchy(ap, ac, av, aggregation=1, block_size=B, coarse_enough=4 * B)
    s0, b0 = hs.level(0), hb.level(0)
    assert np.array_equal(b0["agg"], _expand(s0["agg"]))
    # strong flag of a dof entry = flag of its node entry
    n = len(p) - 1
    node_flag = {}
    for i in range(n):
        for k in range(p[i], p[i + 1]):
            node_flag[(i, int(c[k]))] = bool(s0["strong"][k])
    bp, bc = b0["A"][0], b0["A"][1]
    for r in range(n * B):
        for k in range(bp[r], bp[r + 1]):
            j = int(bc[k])
            if j // B != r // B:
                assert b0["strong"][k] == node_flag[(r // B, j // B)]
    assert hb.num_levels == hs.num_levels


@pytest.mark.parametrize("name,make", SCALARS)
def test_kronecker_coarse_operator_closed_form(ora, name, make):
    """Plain P = P_s (x) I on L (x) K gives A_1 = (P_s^T L P_s) (x) K."""
    p, c, v = make()
    K = _spd_block(2)
    ap, ac, av = _kron(p, c, v, K)
    hs = ora.OracleHierarchy(p, c, v, aggregation=1, coarse_enough=4)
    hb = ora.OracleHierarchy(ap, ac, av, aggregation=1, block_size=B, coarse_enough=4 * B)
    Pp, Pc, Pv, nc = hs.level(0)["P"]
    P = dense(Pp, Pc, Pv, shape=(len(p) - 1, nc))
    L = dense(p, c, v)
    ref = np.kron(P.T @ L @ P, K)
    got = dense(*hb.level(1)["A"])
    assert got.shape == ref.shape
    assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)


def test_node_strength_from_numpy_norms(ora):
    """Coupled blocks that differ per node: node norms taken in NumPy, the oracle's
    scalar aggregation run on that node matrix, expanded per unknown."""
    N = 4
    p, c, v = coupled4_7pt(N, 3, front=0.45)
    n = len(p) - 1
    nn = n // B
    rows, cols, vals = [], [], []
    for I in range(nn):
        r0 = I * B
        blk_cols = c[p[r0]:p[r0 + 1]][::B] // B
        for g, J in enumerate(blk_cols):
            blk = np.array([v[p[r0 + b] + g * B:p[r0 + b] + g * B + B] for b in range(B)])
            rows.append(I)
            cols.append(J)
            vals.append(np.linalg.norm(blk))
    Nm = sp.csr_matrix((vals, (rows, cols)), shape=(nn, nn))
    Nm.sort_indices()
    eps = 0.08
    strong_n, agg_n, nc_n = ora.aggregate(Nm.indptr.astype(np.int32), Nm.indices.astype(np.int32),
                                          Nm.data, eps)
    h = ora.OracleHierarchy(p, c, v, aggregation=1, block_size=B, eps_strong=eps, coarse_enough=16)
    L0 = h.level(0)
    assert np.array_equal(L0["agg"], _expand(agg_n))
    assert h.level(1)["n"] == nc_n * B


def test_block_structure_on_every_level(ora):
    """Coarse unknown b of aggregate a is row B a + b; every coarse operator is made of
    full B x B blocks, so the next level aggregates nodes again; A_{l+1} = P^T A_l P."""
    p, c, v = coupled4_7pt(6, 2, front=0.4)
    h = ora.OracleHierarchy(p, c, v, aggregation=1, block_size=B, coarse_enough=8)
    assert h.num_levels >= 3
    for l in range(h.num_levels):
        L = h.level(l)
        Ap, Ac, Av = L["A"]
        n = L["n"]
        assert n % B == 0
        for I in range(n // B):
            base = Ac[Ap[I * B]:Ap[I * B + 1]]
            assert len(base) % B == 0
            assert np.array_equal(base[::B] % B, np.zeros(len(base) // B, dtype=base.dtype))
            for b in range(B):
                assert np.array_equal(Ac[Ap[I * B + b]:Ap[I * B + b + 1]], base)
        if L["P"] is not None:
            a = L["agg"].reshape(-1, B)
            iso = a[:, 0] < 0                       # isolated nodes: no aggregate at all
            assert np.all(a[iso] < 0)
            assert np.all(a[~iso] % B == np.arange(B))
            a0 = a[~iso] // B
            assert np.all(a0 == a0[:, :1])
            Pp, Pc, Pv, nc = L["P"]
            P = dense(Pp, Pc, Pv, shape=(n, nc))
            ref = P.T @ dense(Ap, Ac, Av) @ P
            got = dense(*h.level(l + 1)["A"])
            assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)


def test_partial_rebuild_keeps_node_aggregates(ora):
    p, c, v0 = coupled4_7pt(6, 0, front=0.4)
    _, _, v1 = coupled4_7pt(6, 5, front=0.6)
    h = ora.OracleHierarchy(p, c, v0, aggregation=1, block_size=B, coarse_enough=8)
    agg0 = h.level(0)["agg"].copy()
    P0 = h.level(0)["P"]
    h.rebuild(v1, ora.OracleHierarchy.PARTIAL)
    L = h.level(0)
    assert np.array_equal(L["agg"], agg0)
    assert all(np.array_equal(a, b) for a, b in zip(L["P"][:3], P0[:3]))
    Pm = dense(*P0[:3], shape=(len(p) - 1, P0[3]))
    ref = Pm.T @ dense(p, c, v1) @ Pm
    got = dense(*h.level(1)["A"])
    assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)


def test_block_size_argument_errors(ora):
    p, c, v = coupled4_7pt(3, 0)
    with pytest.raises(ora.OracleError):           # needs plain aggregation
        ora.OracleHierarchy(p, c, v, aggregation=0, block_size=B)
    with pytest.raises(ora.OracleError):           # 108 rows, not a multiple of 5
        ora.OracleHierarchy(p, c, v, aggregation=1, block_size=5, coarse_enough=4)
    with pytest.raises(ora.OracleError):
        ora.OracleHierarchy(p, c, v, aggregation=1, block_size=0)
    with pytest.raises(ora.OracleError):           # block SPAI0 is not defined here
        ora.OracleHierarchy(p, c, v, aggregation=1, block_size=B, smoother=1, coarse_enough=8)
    sp_, sc, sv = two_fluid_7pt(4, 0.5)             # scalar 7-point: no full 2x2 blocks
    with pytest.raises(ora.OracleError):
        ora.OracleHierarchy(sp_, sc, sv, aggregation=1, block_size=2, coarse_enough=4)


def test_node_aggregation_converges_faster_than_scalar(ora):
    """On the strongly coupled system, node aggregation with block Jacobi needs clearly fewer
    PCG iterations than scalar aggregation with point Jacobi on the same matrix."""
    p, c, v = coupled4_7pt(16, 0)
    f = rhs_uniform(len(p) - 1, 7, 0)
    hb = ora.OracleHierarchy(p, c, v, aggregation=1, block_size=B)
    hs = ora.OracleHierarchy(p, c, v, aggregation=1)
    _, ib = hb.solve(f)
    _, is_ = hs.solve(f)
    assert ib["converged"] and is_["converged"]
    assert ib["iters"] * 3 < is_["iters"] * 2


@pytest.mark.parametrize("name,make", SCALARS)
def test_block_smoother_kronecker(ora, name, make):
    """On L (x) K the diagonal block of node i is l_ii K: M_i = omega / l_ii K^{-1}."""
    p, c, v = make()
    K = _spd_block(3)
    ap, ac, av = _kron(p, c, v, K)
    omega = 0.72
    h = ora.OracleHierarchy(ap, ac, av, aggregation=1, block_size=B, coarse_enough=4 * B)
    m = h.level(0)["m"].reshape(-1, B, B)
    Ld = dense(p, c, v).diagonal()
    ref = (omega / Ld)[:, None, None] * np.linalg.inv(K)[None]
    assert np.abs(m - ref).max() <= 1e-14 * np.abs(ref).max()


def test_block_smoother_inverts_diagonal_blocks(ora):
    p, c, v = coupled4_7pt(6, 11, front=0.5)
    omega = 0.6
    h = ora.OracleHierarchy(p, c, v, aggregation=1, block_size=B, coarse_enough=8, jacobi_omega=omega)
    assert h.num_levels >= 3
    for l in range(h.num_levels - 1):
        L = h.level(l)
        A = dense(*L["A"])
        m = L["m"].reshape(-1, B, B)
        for I in range(L["n"] // B):
            D = A[I * B:I * B + B, I * B:I * B + B]
            assert np.abs(D @ m[I] - omega * np.eye(B)).max() <= 1e-13


def _nonsym_kron():
    """L (x) K with a non-symmetric K (SPD part plus a skew part): diagonal blocks that are
    not symmetric, so a transposed block product would show."""
    p, c, v = random_spd_graph(40, 3, 7)
    K = _spd_block(4)
    K = K + np.triu(np.full((B, B), 0.7), 1) - np.tril(np.full((B, B), 0.7), -1)
    return _kron(p, c, v, K)


@pytest.mark.parametrize("make", [lambda: coupled4_7pt(4, 5, front=0.5), _nonsym_kron],
                         ids=["coupled4", "nonsym_kron"])
def test_block_vcycle_two_grid_identity(ora, make):
    """Two levels, one pre- and one post-sweep of block Jacobi M = blockdiag(M_I):
    B = (I - E) A^{-1} with E = (I - M A)(I - P A_c^{-1} P^T A)(I - M A)."""
    p, c, v = make()
    n = len(p) - 1
    h = ora.OracleHierarchy(p, c, v, aggregation=1, block_size=B, max_levels=2, coarse_enough=4 * B)
    assert h.num_levels == 2
    A = dense(p, c, v)
    l0 = h.level(0)
    Pp, Pc, Pv, nc = l0["P"]
    P = dense(Pp, Pc, Pv, shape=(n, nc))
    Ac = dense(*h.level(1)["A"])
    m = l0["m"].reshape(-1, B, B)
    M = np.zeros((n, n))
    for I in range(n // B):
        M[I * B:I * B + B, I * B:I * B + B] = m[I]
    Id = np.eye(n)
    E = (Id - M @ A) @ (Id - P @ np.linalg.solve(Ac, P.T @ A)) @ (Id - M @ A)
    B_ref = (Id - E) @ np.linalg.inv(A)
    Bm = np.column_stack([h.vcycle(Id[:, j]) for j in range(n)])
    assert np.abs(Bm - B_ref).max() <= 1e-10 * np.abs(B_ref).max()
