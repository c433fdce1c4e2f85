"""Helpers shared by the GPU parity tests."""
import numpy as np
import torch

ORACLE_KEYS = {"smoother", "aggregation", "jacobi_omega", "eps_strong", "coarse_enough", "max_levels", "npre",
               "npost", "rtol", "maxiter", "flexible_cg", "block_size"}


def dev():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch.device("cuda:0")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def both(p, c, v, **params):
    """The same matrix through the HIP library and through the oracle."""
    import oracle
    from paper_2108_02054_amd import AMG

    g = AMG(T(p), T(c), T(v), **params)
    o = oracle.OracleHierarchy(p, c, v, **{k: x for k, x in params.items() if k in ORACLE_KEYS})
    return g, o


def rel_max(a, b):
    s = np.abs(b).max()
    return float(np.abs(a - b).max() / (s if s > 0 else 1.0))


def rel_fro(a, b):
    s = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (s if s > 0 else 1.0))


def compare_levels(g, o, tol=1e-10, values=True, print_report=False):
    """Patterns and aggregates bit-exact, values within tol (normwise and max-entry)."""
    assert g.num_levels == o.num_levels, (g.num_levels, o.num_levels)
    worst = 0.0
    for l in range(o.num_levels):
        gl, ol = g.level(l), o.level(l)
        assert gl["n"] == ol["n"], l
        for k in (0, 1):
            assert np.array_equal(gl["A"][k], ol["A"][k]), f"A pattern differs on level {l}"
        if ol["agg"] is not None:
            assert np.array_equal(gl["agg"], ol["agg"]), f"aggregates differ on level {l}"
            assert np.array_equal(gl["strong"], ol["strong"]), f"strength differs on level {l}"
        if ol["P"] is not None:
            assert gl["P"][3] == ol["P"][3]
            for k in (0, 1):
                assert np.array_equal(gl["P"][k], ol["P"][k]), f"P pattern differs on level {l}"
        if values:
            e = max(rel_max(gl["A"][2], ol["A"][2]), rel_fro(gl["A"][2], ol["A"][2]))
            worst = max(worst, e)
            assert e <= tol, (l, e)
            if ol["P"] is not None:
                assert rel_max(gl["P"][2], ol["P"][2]) <= tol, l
                assert rel_max(gl["m"], ol["m"]) <= tol, l
        if print_report:
            print(f"level {l}: n={ol['n']} nnz={len(ol['A'][1])}", flush=True)
    return worst


def bitwise_levels(g, o):
    for l in range(o.num_levels):
        gl, ol = g.level(l), o.level(l)
        if not np.array_equal(gl["A"][2], ol["A"][2]):
            return f"A values level {l}"
        if ol["P"] is not None:
            if not np.array_equal(gl["P"][2], ol["P"][2]):
                return f"P values level {l}"
            if not np.array_equal(gl["m"], ol["m"]):
                return f"smoother level {l}"
    return None
