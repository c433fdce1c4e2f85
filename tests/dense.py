"""Dense brute-force helpers for the tests (NumPy / SciPy only)."""
import numpy as np
import scipy.sparse as sp


def csr(ptr, col, val, shape=None):
    n = len(ptr) - 1
    if shape is None:
        shape = (n, n)
    return sp.csr_matrix((np.asarray(val), np.asarray(col), np.asarray(ptr)), shape=shape)


def dense(ptr, col, val, shape=None):
    return csr(ptr, col, val, shape).toarray()


def strong_graph(ptr, col, strong):
    """Adjacency (dense bool) of the strong graph from per-entry flags."""
    n = len(ptr) - 1
    S = np.zeros((n, n), dtype=bool)
    for i in range(n):
        for k in range(ptr[i], ptr[i + 1]):
            if strong[k]:
                S[i, col[k]] = True
    return S


def distances(S, max_d=3):
    """All-pairs shortest path lengths in the graph S, capped at max_d+1 (dense BFS by
    boolean matrix powers)."""
    n = S.shape[0]
    D = np.full((n, n), max_d + 1, dtype=np.int64)
    reach = np.eye(n, dtype=bool)
    D[reach] = 0
    frontier = reach.copy()
    for d in range(1, max_d + 1):
        nxt = (frontier.astype(np.int64) @ S.astype(np.int64)) > 0
        new = nxt & (D > d)
        D[new] = d
        frontier = nxt
    return D


def random_spd_graph(n, deg, seed):
    """Symmetric positive definite M-matrix on a random graph (structurally symmetric,
    sorted CSR): negative off-diagonals, diagonal = row sum of |off| + a random shift."""
    g = np.random.default_rng(seed)
    W = np.zeros((n, n))
    for i in range(n):
        nb = g.choice(n, size=deg, replace=False)
        for j in nb:
            if j != i:
                w = g.uniform(0.1, 2.0)
                W[i, j] = W[j, i] = w
    A = -W
    A[np.diag_indices(n)] = W.sum(axis=1) + g.uniform(0.01, 0.5, size=n)
    M = sp.csr_matrix(A)
    M.sort_indices()
    # keep explicit structure: every (i, j) with W != 0 plus the diagonal
    return M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64)
