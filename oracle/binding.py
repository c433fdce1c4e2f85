"""ctypes binding of ``liboracle.so`` (built from ``amg_oracle.cpp`` with g++)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "amg_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

ORA_OK = 0


class OracleError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"oracle status {code}: {msg}")
        self.code = code


def build(verbose: bool = False) -> str:
    """Compile the oracle with g++ (no HIP headers involved)."""
    cmd = ["g++", "-std=c++17", "-O2", "-march=native", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class OracleParams(C.Structure):
    _fields_ = [
        ("smoother", C.c_int),
        ("aggregation", C.c_int),
        ("jacobi_omega", C.c_double),
        ("eps_strong", C.c_double),
        ("coarse_enough", C.c_int),
        ("max_levels", C.c_int),
        ("npre", C.c_int),
        ("npost", C.c_int),
        ("rtol", C.c_double),
        ("maxiter", C.c_int),
        ("flexible_cg", C.c_int),
        ("block_size", C.c_int),
    ]


class OracleInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("rel_res_true", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        P, I32, I64, D, U8 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint8
        pi32, pd, pu8, pi64 = C.POINTER(I32), C.POINTER(D), C.POINTER(U8), C.POINTER(I64)
        L.ora_last_error.restype = C.c_char_p
        L.ora_mix64.restype = C.c_uint64
        L.ora_mix64.argtypes = [C.c_uint64]
        L.ora_params_default.argtypes = [C.POINTER(OracleParams)]
        L.ora_num_threads.restype = C.c_int
        L.ora_set_num_threads.argtypes = [C.c_int]
        L.ora_aggregate.argtypes = [I32, pi32, pi32, pd, D, pu8, pi32, pi32]
        L.ora_setup.argtypes = [C.POINTER(P), I32, pi32, pi32, pd, C.POINTER(OracleParams)]
        L.ora_setup_transfer.argtypes = [C.POINTER(P), I32, pi32, pi32, pd, C.c_int,
                                         C.POINTER(pi32), C.POINTER(pi32), C.POINTER(pd), pi32,
                                         C.POINTER(OracleParams)]
        L.ora_rebuild.argtypes = [P, pd, C.c_int]
        L.ora_rebuild_auto.argtypes = [P, pd, C.c_int, C.c_int, C.c_double, C.POINTER(C.c_int)]
        L.ora_solve.argtypes = [P, pd, pd, C.POINTER(OracleInfo)]
        L.ora_solve_bicgstab.argtypes = [P, pd, pd, C.POINTER(OracleInfo)]
        L.ora_vcycle.argtypes = [P, pd, pd]
        L.ora_num_levels.argtypes = [P]
        L.ora_level_dims.argtypes = [P, C.c_int, pi64]
        L.ora_export_level.argtypes = [P, C.c_int, pi32, pu8, pi32, pi32, pd, pi32, pi32, pd, pd]
        L.ora_export_outer.argtypes = [P, pd]
        L.ora_export_coarse_factor.argtypes = [P, pd]
        L.ora_destroy.argtypes = [P]
        L.ora_assemble_logcoef7.argtypes = [C.c_int, C.c_int, C.c_int, pd, pd]
        L.ora_adjoint_logcoef7.argtypes = [C.c_int, C.c_int, C.c_int, pd, pd, pd, pd]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


def _check(st: int):
    if st != ORA_OK:
        raise OracleError(st, lib().ora_last_error().decode())


def default_params(**kw) -> OracleParams:
    p = OracleParams()
    lib().ora_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def mix64(i: int) -> int:
    return int(lib().ora_mix64(i))


def num_threads() -> int:
    return int(lib().ora_num_threads())


def set_num_threads(t: int):
    lib().ora_set_num_threads(int(t))


def _csr(row_ptr, col, val):
    return (np.ascontiguousarray(row_ptr, dtype=np.int32), np.ascontiguousarray(col, dtype=np.int32),
            np.ascontiguousarray(val, dtype=np.float64))


def aggregate(row_ptr, col, val, eps):
    """Strength flags (per stored entry), aggregate labels and the number of aggregates."""
    row_ptr, col, val = _csr(row_ptr, col, val)
    n = len(row_ptr) - 1
    strong = np.zeros(len(col), dtype=np.uint8)
    agg = np.zeros(n, dtype=np.int32)
    nc = C.c_int32(0)
    _check(lib().ora_aggregate(n, _p(row_ptr, C.c_int32), _p(col, C.c_int32), _p(val, C.c_double),
                               float(eps), _p(strong, C.c_uint8), _p(agg, C.c_int32), C.byref(nc)))
    return strong.astype(bool), agg, int(nc.value)


def assemble_logcoef7(nx, ny, nz, theta):
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    n = nx * ny * nz
    nnz = 7 * n - 2 * (nx * ny + ny * nz + nx * nz)
    val = np.zeros(nnz, dtype=np.float64)
    _check(lib().ora_assemble_logcoef7(nx, ny, nz, _p(theta, C.c_double), _p(val, C.c_double)))
    return val


def adjoint_logcoef7(nx, ny, nz, theta, u, lam):
    theta, u, lam = (np.ascontiguousarray(a, dtype=np.float64) for a in (theta, u, lam))
    g = np.zeros(nx * ny * nz, dtype=np.float64)
    _check(lib().ora_adjoint_logcoef7(nx, ny, nz, _p(theta, C.c_double), _p(u, C.c_double),
                                      _p(lam, C.c_double), _p(g, C.c_double)))
    return g


class OracleHierarchy:
    """An oracle AMG hierarchy (Algorithm 1), updatable by Algorithms 3 and 4."""

    PARTIAL, FULL, OPERATOR_ONLY = 0, 1, 2

    def __init__(self, row_ptr, col, val, transfer=None, check=True, **params):
        self.row_ptr, self.col, val = _csr(row_ptr, col, val)
        self.n = len(self.row_ptr) - 1
        self.params = default_params(**params)
        h = C.c_void_p()
        L = lib()
        if transfer is None:
            st = L.ora_setup(C.byref(h), self.n, _p(self.row_ptr, C.c_int32), _p(self.col, C.c_int32),
                             _p(val, C.c_double), C.byref(self.params))
        else:
            Ps = [_csr(*t[:3]) for t in transfer]
            ncs = np.array([t[3] for t in transfer], dtype=np.int32)
            k = len(Ps)
            pp = (C.POINTER(C.c_int32) * max(k, 1))(*[_p(a[0], C.c_int32) for a in Ps])
            pc = (C.POINTER(C.c_int32) * max(k, 1))(*[_p(a[1], C.c_int32) for a in Ps])
            pv = (C.POINTER(C.c_double) * max(k, 1))(*[_p(a[2], C.c_double) for a in Ps])
            self._keep = Ps
            st = L.ora_setup_transfer(C.byref(h), self.n, _p(self.row_ptr, C.c_int32),
                                      _p(self.col, C.c_int32), _p(val, C.c_double), k, pp, pc, pv,
                                      _p(ncs, C.c_int32), C.byref(self.params))
        self.h = h
        self.status = st
        if check:
            try:
                _check(st)
            except OracleError:
                self.close()
                raise

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().ora_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        self.close()

    def rebuild(self, val, mode: int = 0):
        val = np.ascontiguousarray(val, dtype=np.float64)
        _check(lib().ora_rebuild(self.h, _p(val, C.c_double), int(mode)))

    def rebuild_auto(self, val, base: int = 0, every: int = 0, growth: float = 0.0) -> int:
        """The update the rebuild policy picks from this hierarchy's history, applied; returns
        the mode taken (0 partial, 1 full, 2 operator only)."""
        val = np.ascontiguousarray(val, dtype=np.float64)
        m = C.c_int(-1)
        _check(lib().ora_rebuild_auto(self.h, _p(val, C.c_double), int(base), int(every), float(growth),
                                      C.byref(m)))
        return m.value

    def solve(self, f, u=None):
        f = np.ascontiguousarray(f, dtype=np.float64)
        u = np.zeros(self.n) if u is None else np.array(u, dtype=np.float64, copy=True)
        info = OracleInfo()
        _check(lib().ora_solve(self.h, _p(f, C.c_double), _p(u, C.c_double), C.byref(info)))
        return u, dict(iters=info.iters, converged=bool(info.converged), rel_res_true=info.rel_res_true)

    def solve_bicgstab(self, f, u=None):
        """BiCGStab with the V-cycle on the right (the paper's Krylov method)."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        u = np.zeros(self.n) if u is None else np.array(u, dtype=np.float64, copy=True)
        info = OracleInfo()
        _check(lib().ora_solve_bicgstab(self.h, _p(f, C.c_double), _p(u, C.c_double), C.byref(info)))
        return u, dict(iters=info.iters, converged=bool(info.converged), rel_res_true=info.rel_res_true)

    def vcycle(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.zeros(self.n)
        _check(lib().ora_vcycle(self.h, _p(r, C.c_double), _p(z, C.c_double)))
        return z

    @property
    def num_levels(self) -> int:
        return int(lib().ora_num_levels(self.h))

    def dims(self, l):
        d = np.zeros(4, dtype=np.int64)
        _check(lib().ora_level_dims(self.h, l, _p(d, C.c_int64)))
        return [int(x) for x in d]

    def level(self, l):
        """Dict with A (ptr, col, val), P (ptr, col, val, nc) or None, agg, strong, m."""
        n, nnzA, nc, nnzP = self.dims(l)
        coarsest = l == self.num_levels - 1
        Ap, Ac, Av = np.zeros(n + 1, np.int32), np.zeros(nnzA, np.int32), np.zeros(nnzA)
        agg = np.full(n, -2, np.int32)
        strong = np.zeros(nnzA, np.uint8)
        m = np.zeros(n * max(1, self.params.block_size))   # block_size x block_size per node
        Pp = np.zeros(n + 1, np.int32) if not coarsest else None
        Pc = np.zeros(nnzP, np.int32) if not coarsest else None
        Pv = np.zeros(nnzP) if not coarsest else None
        _check(lib().ora_export_level(self.h, l, _p(agg, C.c_int32), _p(strong, C.c_uint8),
                                      _p(Ap, C.c_int32), _p(Ac, C.c_int32), _p(Av, C.c_double),
                                      _p(Pp, C.c_int32), _p(Pc, C.c_int32), _p(Pv, C.c_double),
                                      _p(m, C.c_double)))
        out = dict(n=n, A=(Ap, Ac, Av), agg=None, strong=None, m=None, P=None)
        if not coarsest:
            out["P"] = (Pp, Pc, Pv, nc)
            out["m"] = m
            if not (agg == -2).all():
                out["agg"] = agg
                out["strong"] = strong.astype(bool)
        return out

    def outer_values(self):
        v = np.zeros(len(self.col))
        _check(lib().ora_export_outer(self.h, _p(v, C.c_double)))
        return v

    def coarse_factor(self):
        nL = self.dims(self.num_levels - 1)[0]
        L = np.zeros((nL, nL))
        _check(lib().ora_export_coarse_factor(self.h, _p(L, C.c_double)))
        return L
