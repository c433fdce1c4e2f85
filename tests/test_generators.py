"""The seeded inputs: exact nnz formulas, symmetry, definiteness, interface motion, seeds."""
import numpy as np
import pytest

from tests.dense import csr
from workloads import (front_c1, front_moving, lognormal_27pt, logcoef_inputs, pattern_7pt,
                       pattern_27pt, rhs_uniform, two_fluid_7pt)


@pytest.mark.parametrize("N", [2, 3, 5, 16])
def test_7pt_nnz_and_sorted(N):
    p, c, _ = pattern_7pt(N)
    assert len(c) == 7 * N**3 - 6 * N**2
    for i in range(N**3):
        row = c[p[i]:p[i + 1]]
        assert np.all(np.diff(row) > 0) and i in row


@pytest.mark.parametrize("N", [3, 4, 6])
def test_27pt_nnz(N):
    p, c, _ = pattern_27pt(N)
    assert len(c) == (3 * N - 2) ** 3


def test_box_pattern_nnz():
    nx, ny, nz = 3, 4, 5
    p, c, _ = pattern_7pt(nx, ny, nz)
    assert len(c) == 7 * nx * ny * nz - 2 * (nx * ny + ny * nz + nx * nz)


@pytest.mark.parametrize("front", [0.0, 0.31, 0.55, 1.0])
def test_two_fluid_symmetric_spd(front):
    N = 6
    A = csr(*two_fluid_7pt(N, front)).toarray()
    assert np.array_equal(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0
    # constant density: the face coefficient 2/(1+1) = 1 everywhere, diagonal 6
    if front == 0.0:
        assert np.all(np.diag(A) == 6.0)
        off = A - np.diag(np.diag(A))
        assert set(np.unique(off)) <= {0.0, -1.0}


def test_two_fluid_coefficients():
    """Face between a heavy (1000) and a light (1) cell carries 2/1001; a heavy cell on the
    boundary gains 1/1000 per missing face."""
    N = 4
    p, c, v = two_fluid_7pt(N, front=0.5)  # heavy: x in {0,1}, z in {0,1,2}
    A = csr(p, c, v).toarray()
    i = 1 + N * (1 + N * 1)  # (x=1, y=1, z=1): heavy
    j = i + 1                # (x=2, ...): light
    assert A[i, j] == -2.0 / 1001.0
    corner = 0               # (0,0,0) heavy, 3 missing faces
    expect = 3 * (2.0 / 2000.0) + 3 * (1.0 / 1000.0)
    assert A[corner, corner] == pytest.approx(expect, rel=1e-15)


def test_front_motion():
    # 32^3 with x = 0.3 + 0.02 t: cells move in only on some steps
    heavy_cols = [int(np.sum((np.arange(32) + 0.5) / 32 < front_c1(t))) for t in range(10)]
    assert heavy_cols[0] == 10
    changed = [t for t in range(1, 10) if heavy_cols[t] != heavy_cols[t - 1]]
    assert changed == [2, 3, 5, 7, 8]
    # one cell per step
    N = 128
    cols = [int(np.sum((np.arange(N) + 0.5) / N < front_moving(N, t))) for t in range(5)]
    assert np.all(np.diff(cols) == 1)


def test_fixed_pattern_over_series():
    p0, c0, v0 = two_fluid_7pt(8, front_moving(8, 0))
    p1, c1, v1 = two_fluid_7pt(8, front_moving(8, 3))
    assert np.array_equal(p0, p1) and np.array_equal(c0, c1) and not np.array_equal(v0, v1)


def test_lognormal_27pt_symmetric_spd_and_drift():
    p, c, v0 = lognormal_27pt(5, 0)
    _, _, v1 = lognormal_27pt(5, 1)
    A = csr(p, c, v0).toarray()
    assert np.allclose(A, A.T, rtol=0, atol=1e-14 * np.abs(A).max())
    assert np.linalg.eigvalsh(A).min() > 0
    assert not np.array_equal(v0, v1)
    # drift is smooth in time: relative change per step is bounded
    assert np.max(np.abs(v1 - v0) / np.abs(v0)) < 0.5


def test_seeds_reproducible():
    a = rhs_uniform(100, 1, 3)
    b = rhs_uniform(100, 1, 3)
    c = rhs_uniform(100, 1, 4)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= -1 and a.max() <= 1
    th, f, ut, cells = logcoef_inputs(8)
    assert len(set(cells.tolist())) == 16
    assert abs(th.std() - 0.5) < 0.1


def test_coupled4_matches_loop_assembly():
    """The 4x4-block coupled system against a loop over nodes and faces."""
    from workloads.poisson import coupled4_7pt, coupling_blocks
    N, t, front = 3, 7, 0.5
    p, c, v = coupled4_7pt(N, t, front=front)
    A = np.zeros((4 * N ** 3, 4 * N ** 3))
    for i in range(len(p) - 1):
        A[i, c[p[i]:p[i + 1]]] = v[p[i]:p[i + 1]]
    Kh, Kl = coupling_blocks(t)
    ref = np.zeros_like(A)

    def cell(x, y, z):
        heavy = (x + 0.5) / N < front and (z + 0.5) / N < 0.6
        return (1000.0 if heavy else 1.0), (Kh if heavy else Kl)

    for z in range(N):
        for y in range(N):
            for x in range(N):
                I = x + N * (y + N * z)
                ri, Ki = cell(x, y, z)
                for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    X, Y, Z = x + d[0], y + d[1], z + d[2]
                    if 0 <= X < N and 0 <= Y < N and 0 <= Z < N:
                        rj, Kj = cell(X, Y, Z)
                        J = X + N * (Y + N * Z)
                        w, K = 2.0 / (ri + rj), 0.5 * (Ki + Kj)
                        ref[4 * I:4 * I + 4, 4 * J:4 * J + 4] = -w * K
                    else:
                        w, K = 1.0 / ri, Ki
                    ref[4 * I:4 * I + 4, 4 * I:4 * I + 4] += w * K
    assert np.allclose(A, ref, rtol=1e-14, atol=0.0)
    assert np.array_equal(np.diff(p), np.repeat(np.diff(p)[::4], 4))
    assert np.all(np.linalg.eigvalsh(Kh) > 0) and np.all(np.linalg.eigvalsh(Kl) > 0)
    assert np.linalg.eigvalsh(A).min() > 0
