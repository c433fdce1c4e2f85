"""Seeded synthetic Poisson time series standing in for the paper's dam-break matrices.

The paper's experiments (Section 4) use matrices from a two-fluid dam-break simulation
that are not available here.  These generators keep what matters for the method: a
density jump of 1000 across a moving interface, a sparsity pattern fixed over a series
of time steps, and SPD systems.  Everything is produced on the host in float64 so that
every consumer sees identical bits.

Conventions
-----------
* Cell (x, y, z) of an nx*ny*nz grid has row index x + nx*(y + ny*z) (x fastest).
* Cell centres sit at ((x+1/2)/nx, (y+1/2)/ny, (z+1/2)/nz).
* CSR rows list their columns in increasing order; int32 row pointers and columns.
* Homogeneous Dirichlet closure by a ghost cell that carries the cell's own coefficient,
  so a missing neighbour adds the cell's own face coefficient to the diagonal.
* Seeds: numpy SeedSequence([2108, 2054, cfg_id, t, stream]).
"""
from __future__ import annotations

import numpy as np

SEED_ROOT = (2108, 2054)
STREAM_RHS, STREAM_UT, STREAM_THETA, STREAM_CELLS, STREAM_LOGN, STREAM_DRIFT = range(6)


def rng(cfg_id: int, t: int, stream: int) -> np.random.Generator:
    """Independent generator for (configuration, time step, stream)."""
    return np.random.default_rng(np.random.SeedSequence([*SEED_ROOT, cfg_id, t, stream]))


# ----------------------------------------------------------------------------- patterns

def _offsets(kind: str):
    if kind == "7pt":
        offs = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    elif kind == "27pt":
        offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    else:
        raise ValueError(kind)
    return offs


def _shift(a: np.ndarray, dx: int, dy: int, dz: int):
    """out[z,y,x] = a[z+dz, y+dy, x+dx] where in range, and the in-range mask."""
    nz, ny, nx = a.shape
    out = np.zeros_like(a)
    mask = np.zeros(a.shape, dtype=bool)
    zs = slice(max(0, -dz), nz - max(0, dz))
    ys = slice(max(0, -dy), ny - max(0, dy))
    xs = slice(max(0, -dx), nx - max(0, dx))
    zt = slice(max(0, dz), nz - max(0, -dz))
    yt = slice(max(0, dy), ny - max(0, -dy))
    xt = slice(max(0, dx), nx - max(0, -dx))
    out[zs, ys, xs] = a[zt, yt, xt]
    mask[zs, ys, xs] = True
    return out, mask


def stencil_pattern(nx: int, ny: int, nz: int, kind: str = "7pt"):
    """CSR pattern of a 7- or 27-point stencil.  Returns (row_ptr, col, mask) where
    mask[n, n_offsets] marks which stencil entries exist (row-major over offsets, in
    increasing column order), so dense per-offset values compress with ``v[mask]``."""
    offs = _offsets(kind)
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64).reshape(nz, ny, nx)
    cols = np.empty((n, len(offs)), dtype=np.int64)
    mask = np.empty((n, len(offs)), dtype=bool)
    for o, (dx, dy, dz) in enumerate(offs):
        s, m = _shift(idx, dx, dy, dz)
        cols[:, o] = s.reshape(-1)
        mask[:, o] = m.reshape(-1)
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("pattern exceeds int32 indexing")
    col = cols[mask].astype(np.int32)
    return row_ptr.astype(np.int32), col, mask


def pattern_7pt(nx, ny=None, nz=None):
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return stencil_pattern(nx, ny, nz, "7pt")


def pattern_27pt(nx, ny=None, nz=None):
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return stencil_pattern(nx, ny, nz, "27pt")


def _assemble(coef: np.ndarray, kind: str, pair, ghost: bool = True):
    """Values of a symmetric diffusion stencil from per-cell coefficients ``coef``
    ([nz,ny,nx]).  ``pair(c, n)`` gives the face coefficient between a cell and a
    neighbour; a_cn = -pair, a_cc = sum of pairs (+ own coefficient per missing
    neighbour when ``ghost``)."""
    nz, ny, nx = coef.shape
    offs = _offsets(kind)
    row_ptr, col, mask = stencil_pattern(nx, ny, nz, kind)
    n = nx * ny * nz
    dense = np.zeros((n, len(offs)), dtype=np.float64)
    diag = np.zeros(coef.shape, dtype=np.float64)
    n_missing = np.zeros(coef.shape, dtype=np.int64)
    centre = offs.index((0, 0, 0))
    for o, (dx, dy, dz) in enumerate(offs):
        if o == centre:
            continue
        cn, m = _shift(coef, dx, dy, dz)
        face = np.where(m, pair(coef, np.where(m, cn, coef)), 0.0)
        dense[:, o] = -face.reshape(-1)
        diag += face
        n_missing += ~m
    if ghost:
        diag += n_missing * pair(coef, coef)
    dense[:, centre] = diag.reshape(-1)
    return row_ptr, col, dense[mask]


# ----------------------------------------------------------------------------- C1-C3

def front_c1(t: int) -> float:
    """Interface position of the 32^3 series: x = 0.3 + 0.02 t."""
    return 0.3 + 0.02 * t


def front_moving(n_cells: int, t: int) -> float:
    """Interface that advances one cell per step: x = 0.3 + t / N."""
    return 0.3 + t / n_cells


def two_fluid_7pt(N: int, front: float, rho_heavy: float = 1000.0, zcut: float = 0.6,
                  ny: int | None = None, nz: int | None = None):
    """Two-fluid pressure Poisson operator -div(1/rho grad p) on a 7-point stencil.

    rho = rho_heavy inside the column x < front, z < zcut (no condition on y), else 1.
    The face coefficient is the harmonic mean of 1/rho on both sides, 2/(rho_a+rho_b).
    Returns (row_ptr int32, col int32, val float64)."""
    nx = N
    ny = N if ny is None else ny
    nz = N if nz is None else nz
    xc = (np.arange(nx) + 0.5) / nx
    zc = (np.arange(nz) + 0.5) / nz
    heavy = (xc[None, None, :] < front) & (zc[:, None, None] < zcut)
    rho = np.where(np.broadcast_to(heavy, (nz, ny, nx)), rho_heavy, 1.0)
    return _assemble(rho, "7pt", lambda a, b: 2.0 / (a + b))


def neumann_7pt(N: int, seed: int = 0, sigma: float = 0.3):
    """7-point operator with random positive face coefficients and no boundary terms:
    every row sums to zero, so the constant vector is in the null space."""
    g = np.random.default_rng(seed)
    k = np.exp(g.normal(0.0, sigma, size=(N, N, N)))
    return _assemble(k, "7pt", lambda a, b: 2.0 * a * b / (a + b), ghost=False)


# ----------------------------------------------------------------------------- C5

def lognormal_27pt(N: int, t: int, cfg_id: int = 5, sigma: float = 1.5,
                   period: int = 40):
    """27-point operator with lognormal coefficients drifting smoothly in time.

    k_c^t = exp(sigma * g_c + d_t(x_c)), g_c ~ N(0,1) i.i.d. (fixed over the series),
    d_t(x) = 0.5 sin(2 pi kappa.x + phi + 2 pi t / period), kappa in {1,2}^3 and
    phi ~ U[0, 2 pi) drawn once.  Face coefficient 2 k_c k_n / (k_c + k_n) for all 26
    neighbours; the pattern is fixed."""
    g = rng(cfg_id, 0, STREAM_LOGN).standard_normal((N, N, N))
    rd = rng(cfg_id, 0, STREAM_DRIFT)
    kappa = rd.integers(1, 3, size=3)
    phi = rd.uniform(0.0, 2.0 * np.pi)
    c = (np.arange(N) + 0.5) / N
    arg = (kappa[0] * c[None, None, :] + kappa[1] * c[None, :, None] + kappa[2] * c[:, None, None])
    drift = 0.5 * np.sin(2.0 * np.pi * arg + phi + 2.0 * np.pi * t / period)
    k = np.exp(sigma * g + drift)
    return _assemble(k, "27pt", lambda a, b: 2.0 * a * b / (a + b))


# ----------------------------------------------------------------------------- C4

def logcoef_inputs(N: int, cfg_id: int = 4, n_cells: int = 16):
    """Inputs of the differentiable solve: theta ~ N(0, 0.5^2) per cell, f ~ U[-1,1],
    u_t ~ N(0,1), and ``n_cells`` distinct cells for the finite-difference check.
    The operator values A(theta) are not built here (that is part of the method)."""
    n = N ** 3
    theta = rng(cfg_id, 0, STREAM_THETA).normal(0.0, 0.5, size=n)
    f = rng(cfg_id, 0, STREAM_RHS).uniform(-1.0, 1.0, size=n)
    u_t = rng(cfg_id, 0, STREAM_UT).standard_normal(n)
    cells = rng(cfg_id, 0, STREAM_CELLS).choice(n, size=n_cells, replace=False)
    return theta, f, u_t, np.sort(cells)


def logcoef_theta(N: int, t: int, cfg_id: int = 4, step: float = 0.02) -> np.ndarray:
    """Log-coefficients of step t of the differentiable series: theta_0 of logcoef_inputs
    moved t steps along one seeded N(0, 1) direction (``step`` per step), as an outer
    optimisation would move them; the pattern stays."""
    theta0 = logcoef_inputs(N, cfg_id)[0]
    if t == 0:
        return theta0
    d = rng(cfg_id, 0, STREAM_DRIFT).standard_normal(N ** 3)
    return theta0 + (step * t) * d


def rhs_uniform(n: int, cfg_id: int, t: int) -> np.ndarray:
    """Right-hand side of step t: U[-1, 1]."""
    return rng(cfg_id, t, STREAM_RHS).uniform(-1.0, 1.0, size=n)


# ----------------------------------------------------------------------------- C7 (4x4 blocks)

def coupling_blocks(t: int, period: int = 40):
    """The two SPD 4x4 coupling matrices of step t (heavy fluid, light fluid):
    K = L L^T + I/2 with L lower triangular, its off-diagonal part turning with
    phi_t = 2 pi t / period (light fluid: half the scale, a quarter turn ahead).  The
    blocks are strongly coupled: a point (scalar) Jacobi sweep does not smooth this
    system, a block Jacobi sweep does."""
    phi = 2.0 * np.pi * t / period
    out = []
    for scale, shift in ((1.0, 0.0), (0.5, 0.5 * np.pi)):
        c, s = np.cos(phi + shift), np.sin(phi + shift)
        L = np.array([[1.0, 0.0, 0.0, 0.0],
                      [0.4 * c, 1.0, 0.0, 0.0],
                      [0.3 * s, 0.2 * c, 1.0, 0.0],
                      [0.5 * c * s, 0.3 * s, 0.4 * c, 0.6]]) * scale
        out.append(L @ L.T + 0.5 * np.eye(4))
    return out


def coupled4_7pt(N: int, t: int, front: float | None = None, rho_heavy: float = 1000.0,
                 zcut: float = 0.6, period: int = 40):
    """A monolithic system with 4 unknowns per grid node on the 7-point node graph:
    unknown b of node I is row 4 I + b (node-major), every stored block is a full 4x4
    block.  Face (I, J) couples the nodes by -w_IJ K_IJ, w_IJ the two-fluid face
    coefficient of two_fluid_7pt and K_IJ = (K_I + K_J) / 2 with K_c the heavy or light
    coupling matrix of coupling_blocks(t); the diagonal block is the sum of the node's
    w_IJ K_IJ plus w_II K_I per missing neighbour (ghost closure).  A sum of Kronecker
    products (e_I - e_J)(e_I - e_J)^T (x) w K with SPD K, so SPD.  The front moves one
    cell per step as in the two-fluid series.  Returns (row_ptr, col, val)."""
    B = 4
    nx = ny = nz = N
    front = front_moving(N, t) if front is None else front
    xc = (np.arange(nx) + 0.5) / nx
    zc = (np.arange(nz) + 0.5) / nz
    heavy = np.broadcast_to((xc[None, None, :] < front) & (zc[:, None, None] < zcut), (nz, ny, nx))
    rho = np.where(heavy, rho_heavy, 1.0)
    Kh, Kl = coupling_blocks(t, period)
    Kc = np.where(heavy[..., None, None], Kh, Kl)                 # [nz,ny,nx,4,4]
    offs = _offsets("7pt")
    centre = offs.index((0, 0, 0))
    nptr, ncol, mask = stencil_pattern(nx, ny, nz, "7pt")
    nn = nx * ny * nz
    blocks = np.zeros((nn, len(offs), B, B))
    diag = np.zeros((nz, ny, nx, B, B))
    for o, (dx, dy, dz) in enumerate(offs):
        if o == centre:
            continue
        rn, m = _shift(rho, dx, dy, dz)
        w = np.where(m, 2.0 / (rho + np.where(m, rn, rho)), 1.0 / rho)
        Kn = np.empty_like(Kc)
        for a in range(B):
            for b in range(B):
                Kn[..., a, b], _ = _shift(Kc[..., a, b], dx, dy, dz)
        Kf = np.where(m[..., None, None], 0.5 * (Kc + Kn), Kc)
        face = w[..., None, None] * Kf
        blocks[:, o] = np.where(m[..., None, None], -face, 0.0).reshape(nn, B, B)
        diag += face                                              # ghost closure when ~m
    blocks[:, centre] = diag.reshape(nn, B, B)
    # dof row 4I+b lists, for each stored node column J (increasing), columns 4J..4J+3
    nblk = np.diff(nptr).astype(np.int64)
    row_len = np.repeat(nblk * B, B)
    row_ptr = np.zeros(nn * B + 1, dtype=np.int64)
    np.cumsum(row_len, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("pattern exceeds int32 indexing")
    nodes_of = np.repeat(np.arange(nn), nblk)                     # node of each stored block
    kept = blocks[mask]                                           # [nblocks, 4, 4], row-major per node
    jcol = ncol.astype(np.int64)
    # gather per node: row b of the node -> [blocks of the node] x [4 columns]
    col = np.empty(int(row_ptr[-1]), dtype=np.int64)
    val = np.empty(int(row_ptr[-1]), dtype=np.float64)
    start = nptr[:-1].astype(np.int64)
    for b in range(B):
        rows = np.arange(nn) * B + b
        base = row_ptr[rows]                                      # first entry of each dof row
        pos = base[nodes_of] + (np.arange(len(nodes_of)) - start[nodes_of]) * B
        for q in range(B):
            col[pos + q] = jcol * B + q
            val[pos + q] = kept[:, b, q]
    return row_ptr.astype(np.int32), col.astype(np.int32), val


# ----------------------------------------------------------------------------- presets

CONFIGS = {
    1: dict(name="two_fluid_7pt_32", N=32, steps=10, kind="two_fluid", front="c1",
            eps_strong=0.08, precision="fp64"),
    2: dict(name="two_fluid_7pt_128", N=128, steps=50, kind="two_fluid", front="moving",
            eps_strong=0.08, precision="fp64"),
    3: dict(name="two_fluid_7pt_192", N=192, steps=30, kind="two_fluid", front="moving",
            eps_strong=0.08, precision="mixed"),
    4: dict(name="logcoef_7pt", N=(64, 128), steps=1, kind="logcoef", eps_strong=0.08,
            precision="fp64"),
    5: dict(name="lognormal_27pt_160", N=160, steps=40, kind="lognormal27",
            eps_strong=0.02, precision="mixed"),
    6: dict(name="convdiff_7pt_128", N=128, steps=40, kind="convdiff", eps_strong=0.08,
            precision="fp64"),
    7: dict(name="coupled4_7pt_56", N=56, steps=40, kind="coupled4", eps_strong=0.08,
            precision="fp64", block_size=4, aggregation=1),
}


def series_matrix(cfg_id: int, t: int, N: int | None = None):
    """Matrix of step t of configuration ``cfg_id`` (C1, C2, C3, C5, C6)."""
    c = CONFIGS[cfg_id]
    N = c["N"] if N is None else N
    if c["kind"] == "two_fluid":
        front = front_c1(t) if c["front"] == "c1" else front_moving(N, t)
        return two_fluid_7pt(N, front)
    if c["kind"] == "lognormal27":
        return lognormal_27pt(N, t, cfg_id=cfg_id)
    if c["kind"] == "convdiff":
        return convdiff_7pt(N, t)
    if c["kind"] == "coupled4":
        return coupled4_7pt(N, t)
    raise ValueError(f"configuration {cfg_id} has no matrix series")


# ----------------------------------------------------------------------------- C6 (non-symmetric)

def convdiff_velocity(N: int, t: int, peclet: float = 1.0, period: int = 40, nz: int | None = None):
    """Cell velocities of the convection-diffusion series, shape [nz, 3]: a flow turning in
    the x-y plane with period ``period`` steps, w = peclet*N*(1 + 0.5 sin(2 pi z)) *
    (cos phi_t, sin phi_t, 0.25), phi_t = 2 pi t / period (constant in x and y)."""
    nz = N if nz is None else nz
    zc = (np.arange(nz) + 0.5) / nz
    phi = 2.0 * np.pi * t / period
    amp = peclet * N * (1.0 + 0.5 * np.sin(2.0 * np.pi * zc))
    return amp[:, None] * np.array([np.cos(phi), np.sin(phi), 0.25])[None, :]


def convdiff_7pt(N: int, t: int, peclet: float = 1.0, period: int = 40, ny: int | None = None,
                 nz: int | None = None):
    """Non-symmetric 7-point convection-diffusion operator -lap u + w.grad u on the unit
    cube (h = 1/N), first-order upwind convection, scaled by h^2: row c has diagonal
    6 + h(|w_x| + |w_y| + |w_z|) and, towards the neighbour in direction -+e_d, the entry
    -1 - h max(+-w_d, 0) (the upwind side carries the convection); homogeneous Dirichlet
    closure (a missing neighbour's entry is dropped, the diagonal keeps its 6).  A
    diagonally dominant M-matrix with the 7-point pattern; at peclet = 0 it is the
    constant-coefficient Laplacian of two_fluid_7pt with rho_heavy = 1.  Returns
    (row_ptr int32, col int32, val float64)."""
    nx = N
    ny = N if ny is None else ny
    nz = N if nz is None else nz
    h = 1.0 / N
    w = convdiff_velocity(N, t, peclet, period, nz)           # [nz, 3]
    wz = np.broadcast_to(w[:, None, None, :], (nz, ny, nx, 3))
    offs = _offsets("7pt")
    row_ptr, col, mask = stencil_pattern(nx, ny, nz, "7pt")
    n = nx * ny * nz
    dense = np.zeros((n, len(offs)), dtype=np.float64)
    centre = offs.index((0, 0, 0))
    diag = np.full((nz, ny, nx), 6.0)
    for d in range(3):
        diag = diag + h * np.abs(wz[..., d])
    for o, e in enumerate(offs):
        if o == centre:
            continue
        d = int(np.flatnonzero(e)[0])
        sgn = e[d]                                            # -1: neighbour behind, +1: ahead
        conv = h * np.maximum(-sgn * wz[..., d], 0.0)         # upwind side only
        dense[:, o] = (-1.0 - conv).reshape(-1)
    dense[:, centre] = diag.reshape(-1)
    return row_ptr, col, dense[mask]
