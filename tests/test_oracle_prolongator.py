"""Pins of the oracle's smoothed prolongator (transfer operators of Algorithm 1, Section 2;
smoothed aggregation with a lumped filtered operator, Vanek-Mandel-Brezina 1996).

The prolongator is P = P_tent - omega D_F^-1 A_F P_tent, with A_F the filtered operator
(weak couplings of a non-isolated row added onto its diagonal), omega = (4/3)/rho and rho
the Gershgorin bound of D_F^-1 A_F.  Three kinds of check fix it:

* closed forms where rho, omega and the diagonal scale are known by hand: constant-
  coefficient Laplacians whose couplings are all strong (rho = 2, omega = 2/3, P[i, J] =
  delta - (2/(3d)) (d delta - #neighbours of i in J)) and an anisotropic operator whose
  weak x-couplings are lumped onto the diagonal (d_F = 4 in the interior);
* a dense NumPy construction from A, the strength flags and the aggregates on ragged grids
  and random graphs, compared entry by entry, together with the structural union pattern
  (explicit zeros kept);
* sensitivity: the expected values built with a wrong omega or without the 1/d_F scale
  differ from the oracle's by far more than the tolerance, so those mistakes cannot pass.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from tests.dense import dense, random_spd_graph
from workloads import lognormal_27pt, two_fluid_7pt

TOL = 1e-15


def _tridiag(n):
    A = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    S = sp.csr_matrix(A)
    S.sort_indices()
    return S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64)


def _level0(ora, p, c, v, **kw):
    h = ora.OracleHierarchy(p, c, v, **kw)
    lv = h.level(0)
    assert lv["P"] is not None and lv["agg"] is not None
    Pp, Pc, Pv, nc = lv["P"]
    P = dense(Pp, Pc, Pv, shape=(lv["n"], nc))
    return lv, P, (Pp, Pc, Pv, nc)


def _neighbour_counts(A, agg, nc, strong_mask=None):
    """cnt[i, J] = number of off-diagonal neighbours j of i (strong ones if a mask is given)
    with agg(j) = J."""
    n = A.shape[0]
    cnt = np.zeros((n, nc))
    for i in range(n):
        for j in np.nonzero(A[i])[0]:
            if j == i or agg[j] < 0:
                continue
            if strong_mask is not None and not strong_mask[i, j]:
                continue
            cnt[i, agg[j]] += 1
    return cnt


def _rel(P, E):
    return np.abs(P - E).max() / np.abs(E).max()


def test_closed_form_1d_laplacian(ora):
    """tridiag(-1, 2, -1): every coupling strong (1 > 0.08^2 * 4), the interior Gershgorin
    ratio (2 + 1 + 1) / 2 = 2 is the largest, so omega = 2/3 and the scale is 1/3: a row
    whose two neighbours share its aggregate keeps 1; a row with one neighbour outside gets
    2/3 in its own aggregate and 1/3 in the other; the boundary row gets 2/3 when its one
    neighbour shares its aggregate."""
    n = 40
    p, c, v = _tridiag(n)
    lv, P, _ = _level0(ora, p, c, v, coarse_enough=4)
    agg = lv["agg"]
    assert np.all(agg >= 0)
    nc = P.shape[1]
    E = np.zeros((n, nc))
    for i in range(n):
        E[i, agg[i]] += 1.0
        nbrs = [j for j in (i - 1, i + 1) if 0 <= j < n]
        E[i, agg[i]] -= 2.0 / 3.0
        for j in nbrs:
            E[i, agg[j]] += 1.0 / 3.0
    assert _rel(P, E) <= TOL
    interior = [i for i in range(1, n - 1) if agg[i - 1] == agg[i] == agg[i + 1]]
    edge = [i for i in range(1, n - 1) if (agg[i - 1] == agg[i]) != (agg[i + 1] == agg[i])]
    assert interior and edge
    assert np.all(np.abs(P[interior, agg[interior]] - 1.0) <= TOL)
    for i in edge:
        other = agg[i - 1] if agg[i - 1] != agg[i] else agg[i + 1]
        assert abs(P[i, agg[i]] - 2.0 / 3.0) <= TOL and abs(P[i, other] - 1.0 / 3.0) <= TOL


@pytest.mark.parametrize("dims", [(6, 6, 6), (5, 4, 7)])
def test_closed_form_3d_laplacian(ora, dims):
    """Constant 7-point operator with ghost closure: diagonal 6 on every row, all couplings
    strong (1/36 > 0.08^2), interior Gershgorin ratio 12/6 = 2, so omega = 2/3 and the
    scale is 1/9: P[i, J] = delta(agg_i, J) - (6 delta(agg_i, J) - cnt(i, J)) / 9."""
    nx, ny, nz = dims
    p, c, v = two_fluid_7pt(nx, 0.0, ny=ny, nz=nz)
    lv, P, _ = _level0(ora, p, c, v, coarse_enough=8)
    A = dense(p, c, v)
    assert np.all(np.diag(A) == 6.0)
    agg = lv["agg"]
    nc = P.shape[1]
    cnt = _neighbour_counts(A, agg, nc)
    E = -cnt * (-1.0 / 9.0)  # -(omega/d) * a_ij with a_ij = -1
    E[np.arange(len(agg)), agg] += 1.0 - 6.0 / 9.0
    assert _rel(P, E) <= TOL
    # rows whose six neighbours all share the aggregate reproduce the tentative 1 exactly
    full = [i for i in range(len(agg)) if cnt[i, agg[i]] == 6]
    if full:
        assert np.all(np.abs(P[full, agg[full]] - 1.0) <= TOL)


def _anisotropic(N, e):
    """-e u_xx - u_yy - u_zz, 7 points, Dirichlet ghost closure: diagonal 2e + 4 on every
    row."""
    p, c, _ = two_fluid_7pt(N, 0.0)
    v = np.zeros(len(c))
    for i in range(N**3):
        for k in range(p[i], p[i + 1]):
            j = c[k]
            if j != i:
                v[k] = -(e if abs(j - i) == 1 else 1.0)
        v[p[i] + list(c[p[i]:p[i + 1]]).index(i)] = 2 * e + 4.0
    return p, c, v


def test_closed_form_lumped_anisotropic(ora):
    """-e u_xx - u_yy - u_zz with e = 1e-2: x-couplings weak (1e-4 < 0.08^2 (4.02)^2), the
    others strong.  Lumping adds each weak -e onto the diagonal, so d_F = 4 + e (2 - x
    neighbours): 4 in the x-interior, 4 + e at the x-faces.  The largest Gershgorin ratio of
    D_F^-1 A_F is (4 + 4)/4 = 2 (rows with all four y/z neighbours, x-interior), so omega =
    2/3 and P[i, J] = delta(agg_i, J) - (2/3)/d_F(i) (d_F(i) delta(agg_i, J) - cnt_yz(i, J))."""
    N, e = 6, 1e-2
    p, c, v = _anisotropic(N, e)
    lv, P, _ = _level0(ora, p, c, v, coarse_enough=8)
    A = dense(p, c, v)
    n = N**3
    agg = lv["agg"]
    nc = P.shape[1]
    yz = np.zeros((n, n), dtype=bool)
    for i in range(n):
        for j in np.nonzero(A[i])[0]:
            yz[i, j] = j != i and abs(j - i) != 1
    # the oracle's strength flags are the y/z couplings (R2 closed form)
    S = np.zeros((n, n), dtype=bool)
    for i in range(n):
        for k in range(p[i], p[i + 1]):
            S[i, c[k]] = lv["strong"][k]
    assert np.array_equal(S, yz)
    cnt = _neighbour_counts(A, agg, nc, strong_mask=yz)
    x = np.arange(n) % N
    dF = 4.0 + e * ((x == 0).astype(float) + (x == N - 1).astype(float))
    scale = (2.0 / 3.0) / dF
    E = cnt * scale[:, None]
    E[np.arange(n), agg] += 1.0 - scale * dF
    assert _rel(P, E) <= TOL
    # without lumping (d_F = 2e + 4) the same rows would differ well above the tolerance
    scale_nolump = (2.0 / 3.0) / (2 * e + 4.0)
    E2 = cnt * scale_nolump
    E2[np.arange(n), agg] += 1.0 - scale_nolump * (2 * e + 4.0)
    assert _rel(P, E2) > 1e-4


def _dense_prolongator(A, strong_mask, agg, nc, omega_rule="gershgorin", scale=True):
    """P from its definition with dense NumPy: lumped filtered A_F, rho = max row sum of
    |D_F^-1 A_F|, omega = (4/3)/rho, P = P_tent - omega D_F^-1 A_F P_tent.  omega_rule and
    scale switch in the mistakes the sensitivity test looks for."""
    n = A.shape[0]
    iso = agg < 0
    F = np.zeros_like(A)
    for i in range(n):
        F[i, i] = A[i, i]
        if iso[i]:
            continue
        for j in np.nonzero(A[i])[0]:
            if j == i:
                continue
            if strong_mask[i, j]:
                F[i, j] = A[i, j]
            else:
                F[i, i] += A[i, j]
    d = np.diag(F)
    rho = (np.abs(F).sum(axis=1) / np.abs(d)).max()
    omega = {"gershgorin": 4.0 / 3.0 / rho, "one_over_rho": 1.0 / rho}[omega_rule]
    Pt = np.zeros((n, nc))
    Pt[np.where(~iso)[0], agg[~iso]] = 1.0
    D = (omega / d) if scale else np.full(n, omega)
    return Pt - D[:, None] * (F @ Pt), F, Pt


def _strong_mask(p, c, strong):
    n = len(p) - 1
    S = np.zeros((n, n), dtype=bool)
    for i in range(n):
        for k in range(p[i], p[i + 1]):
            S[i, c[k]] = strong[k]
    return S


CASES = [
    ("tf6", lambda: two_fluid_7pt(6, 0.45), {}),
    ("box345", lambda: two_fluid_7pt(3, 0.5, ny=4, nz=5), {}),
    ("tf_ragged", lambda: two_fluid_7pt(7, 0.33, ny=5, nz=6), {}),
    ("rand80", lambda: random_spd_graph(80, 3, 11), {}),
    ("rand200", lambda: random_spd_graph(200, 4, 12), {}),
    ("ln27", lambda: lognormal_27pt(5, 0), {"eps_strong": 0.02}),
]


@pytest.mark.parametrize("name,make,kw", CASES)
def test_dense_construction(ora, name, make, kw):
    """The oracle's level-0 prolongator equals the dense construction entry by entry, and its
    stored pattern is the structural union of P_tent and pattern(A_F) pattern(P_tent)."""
    p, c, v = make()
    lv, P, (Pp, Pc, Pv, nc) = _level0(ora, p, c, v, coarse_enough=4, **kw)
    A = dense(p, c, v)
    S = _strong_mask(p, c, lv["strong"])
    E, F, Pt = _dense_prolongator(A, S, lv["agg"], nc)
    assert _rel(P, E) <= TOL, name
    struct = ((F != 0).astype(int) @ (Pt != 0).astype(int) > 0) | (Pt != 0)
    stored = np.zeros_like(struct)
    for i in range(len(Pp) - 1):
        stored[i, Pc[Pp[i]:Pp[i + 1]]] = True
    assert np.array_equal(stored, struct), name
    for i in range(len(Pp) - 1):
        assert np.all(np.diff(Pc[Pp[i]:Pp[i + 1]]) > 0)


@pytest.mark.parametrize("name,make,kw", CASES[:4])
def test_mistakes_are_caught(ora, name, make, kw):
    """omega = 1/rho instead of (4/3)/rho, or omega without the 1/d_F scale, gives expected
    values far outside the tolerance, so the comparisons above would fail on either."""
    p, c, v = make()
    lv, P, (_, _, _, nc) = _level0(ora, p, c, v, coarse_enough=4, **kw)
    A = dense(p, c, v)
    S = _strong_mask(p, c, lv["strong"])
    wrong_omega, _, _ = _dense_prolongator(A, S, lv["agg"], nc, omega_rule="one_over_rho")
    no_scale, _, _ = _dense_prolongator(A, S, lv["agg"], nc, scale=False)
    assert _rel(P, wrong_omega) > 1e-3
    assert _rel(P, no_scale) > 1e-3


def test_coarser_levels_dense(ora):
    """The same construction on every level of a hierarchy (threshold halved per level)."""
    p, c, v = two_fluid_7pt(12, 0.4)
    h = ora.OracleHierarchy(p, c, v, coarse_enough=20)
    for l in range(h.num_levels - 1):
        lv = h.level(l)
        Pp, Pc, Pv, nc = lv["P"]
        P = dense(Pp, Pc, Pv, shape=(lv["n"], nc))
        Ap, Ac, Av = lv["A"]
        A = dense(Ap, Ac, Av)
        E, _, _ = _dense_prolongator(A, _strong_mask(Ap, Ac, lv["strong"]), lv["agg"], nc)
        assert _rel(P, E) <= 4 * TOL, l
