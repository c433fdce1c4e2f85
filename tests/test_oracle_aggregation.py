"""Pins of the oracle's strength test and aggregation (transfer operators of Algorithm 1).

Checked against the definitions by brute force: dense distance matrices of the strong
graph, independence at distance >= 3, maximality, connectivity, and a dense greedy
independent set of the squared graph computed independently in NumPy.
"""
import numpy as np
import pytest

from tests.dense import dense, distances, random_spd_graph, strong_graph
from workloads import lognormal_27pt, pattern_27pt, two_fluid_7pt

SPLITMIX_FIRST = [  # SplitMix64 outputs for seed 0 (published sequence), i.e. the
    # finaliser applied to k * 0x9E3779B97F4A7C15 for k = 1, 2, 3
    0xE220A8397B1DCDAF,
    0x6E789E6AA1B965F4,
    0x06C45D188009454F,
]


def test_mix64_is_splitmix_finaliser(ora):
    golden = 0x9E3779B97F4A7C15
    for k, want in enumerate(SPLITMIX_FIRST, start=1):
        assert ora.mix64((k * golden) % 2**64) == want


def _check_aggregation(p, c, v, strong, agg, nc):
    n = len(p) - 1
    S = strong_graph(p, c, strong)
    assert np.array_equal(S, S.T)
    isolated = ~S.any(axis=1)
    assert np.all(agg[isolated] == -1)
    assert np.all(agg[~isolated] >= 0)
    assert set(np.unique(agg[agg >= 0]).tolist()) == set(range(nc))
    D = distances(S, max_d=4)
    # every aggregate is connected in S and has a centre within distance 2 of all members
    # (pass-2 nodes hang off a pass-1 node of the root), so the root set is recoverable:
    roots = []
    for a in range(nc):
        members = np.where(agg == a)[0]
        sub = D[np.ix_(members, members)]
        assert np.all(sub <= 4), "aggregate not connected within radius"
        centre = [m for m, row in zip(members, sub) if np.all(D[m, members] <= 2)]
        assert centre, "no centre"
        roots.append(centre)
    return D, roots


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_aggregation_properties_random(ora, seed):
    p, c, v = random_spd_graph(80, 3, seed)
    strong, agg, nc = ora.aggregate(p, c, v, 0.08)
    _check_aggregation(p, c, v, strong, agg, nc)


def _greedy_mis2_dense(S, prio):
    """Greedy maximal independent set of the squared strong graph, by decreasing
    priority, computed from the dense distance matrix."""
    n = S.shape[0]
    D = distances(S, max_d=2)
    iso = ~S.any(axis=1)
    roots = []
    blocked = np.zeros(n, dtype=bool)
    for i in sorted(np.where(~iso)[0], key=lambda i: -prio[i]):
        if not blocked[i]:
            roots.append(i)
            blocked |= D[i] <= 2
    return sorted(roots)


@pytest.mark.parametrize("make", [
    lambda: random_spd_graph(90, 3, 7),
    lambda: random_spd_graph(150, 2, 8),
    lambda: two_fluid_7pt(6, 0.5),
    lambda: two_fluid_7pt(5, 0.3, ny=3, nz=4),
])
def test_mis2_matches_dense_greedy(ora, make):
    p, c, v = make()
    strong, agg, nc = ora.aggregate(p, c, v, 0.08)
    S = strong_graph(p, c, strong)
    prio = [ora.mix64(i) for i in range(len(p) - 1)]
    roots = _greedy_mis2_dense(S, prio)
    assert len(roots) == nc
    # roots are numbered in increasing node order, and a root labels itself
    assert [agg[r] for r in roots] == list(range(nc))
    D = distances(S, max_d=3)
    R = np.array(roots)
    sub = D[np.ix_(R, R)]
    assert np.all(sub[~np.eye(len(R), dtype=bool)] >= 3)
    # pass 1: strong neighbours of a root carry its label; pass 2 as specified
    for r in roots:
        assert np.all(agg[S[r]] == agg[r])
    pass1 = np.full(len(agg), -1)
    for r in roots:
        pass1[r] = agg[r]
        pass1[S[r]] = agg[r]
    A = dense(p, c, v)
    for i in np.where((pass1 < 0) & S.any(axis=1))[0]:
        cand = [j for j in np.where(S[i])[0] if pass1[j] >= 0]
        assert cand
        w = {j: A[i, j] * A[j, i] for j in cand}
        best = max(w.values())
        want = min(pass1[j] for j in cand if w[j] == best)
        assert agg[i] == want


def test_strength_constant_7pt_all_strong(ora):
    """Constant 7-point operator: a_ij^2 / (a_ii a_jj) >= 1/36 > 0.08^2, all strong."""
    p, c, v = two_fluid_7pt(5, 0.0)
    strong, agg, nc = ora.aggregate(p, c, v, 0.08)
    off = np.array([c[k] != i for i in range(len(p) - 1) for k in range(p[i], p[i + 1])])
    assert np.all(strong[off]) and not np.any(strong[~off])


def test_strength_anisotropic(ora):
    """-eps u_xx - u_yy - u_zz with eps = 1e-3: x-couplings weak, others strong."""
    N = 5
    p, c, _ = two_fluid_7pt(N, 0.0)
    v = np.zeros(len(c))
    for i in range(N**3):
        d = 0.0
        for k in range(p[i], p[i + 1]):
            j = c[k]
            if j == i:
                continue
            w = 1e-3 if abs(j - i) == 1 else 1.0
            v[k] = -w
            d += w
        v[p[i] + list(c[p[i]:p[i + 1]]).index(i)] = d + 2.0
    strong, _, _ = ora.aggregate(p, c, v, 0.08)
    for i in range(N**3):
        for k in range(p[i], p[i + 1]):
            j = c[k]
            if j != i:
                assert strong[k] == (abs(j - i) != 1)


def test_27pt_equal_weights_threshold(ora):
    """Constant 27-point operator: a_ij^2 / (a_ii a_jj) = 1/676.  Everything is isolated at
    eps = 0.08 (0.0064 > 1/676) and everything is strong at eps = 0.02 (0.0004 < 1/676)."""
    N = 4
    p, c, _ = pattern_27pt(N)
    v = np.where(np.repeat(np.arange(N**3), np.diff(p)) == c, 26.0, -1.0)
    _, agg, nc = ora.aggregate(p, c, v, 0.08)
    assert nc == 0 and np.all(agg == -1)
    strong, agg, nc = ora.aggregate(p, c, v, 0.02)
    assert nc > 0 and np.all(agg >= 0)


def test_lognormal_27pt_aggregates(ora):
    p, c, v = lognormal_27pt(6, 0)
    strong, agg, nc = ora.aggregate(p, c, v, 0.02)
    _check_aggregation(p, c, v, strong, agg, nc)
