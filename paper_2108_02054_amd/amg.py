"""ctypes binding of libamgmi.so (include/amg.h), the gfx950 partial-reuse AMG library.

Argument marshalling only: every step of setup, rebuild and solve runs in the HIP
library.  Tensors must be contiguous CUDA (HIP) tensors: int32 patterns, float64 values.
Work is enqueued on the torch stream that is current when the hierarchy is built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("AMGMI_LIB") or os.path.join(HERE, "libamgmi.so")

AMG_OK = 0
STATUS = {0: "AMG_OK", -1: "AMG_ERR_ARG", -2: "AMG_ERR_HIP", -3: "AMG_ERR_OOM", -4: "AMG_ERR_PATTERN",
          -5: "AMG_ERR_NOT_SPD", -6: "AMG_ERR_BREAKDOWN", -7: "AMG_ERR_STATE"}
PARTIAL, FULL, OPERATOR_ONLY = 0, 1, 2

EXPORTED = [
    "amg_params_default", "amg_setup", "amg_setup_transfer", "amg_rebuild", "amg_set_pattern",
    "amg_rebuild_ex", "amg_solve", "amg_vcycle", "amg_destroy", "amg_last_error", "amg_num_levels",
    "amg_level_dims", "amg_level_format", "amg_export_level", "amg_export_coarse_inverse", "amg_phase_times",
    "amg_logcoef7_assemble", "amg_logcoef7_adjoint", "amg_trace", "amg_trace_every", "amg_trace_read", "amg_policy_pick",
    "amg_rebuild_auto", "amg_solve_bicgstab", "amg_apply_operator", "amg_trace_read_levels", "amg_level_storage",
    "amg_apply_operator_noalloc",
]
MODE_NAMES = {PARTIAL: "partial", FULL: "full", OPERATOR_ONLY: "operator_only"}
KERNEL_CLASSES = ["galerkin_ap", "galerkin_rap", "smoother", "coarse_inv", "cg_pq", "cg_update", "cg_rz",
                  "cg_init", "smooth0_res", "jacobi", "restrict", "prolong", "coarse_gemv", "cast", "tail",
                  "bicg_spmv"]


class AmgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


# amg_params.alloc / dealloc: the device allocator a context takes its memory from
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


def _torch_alloc(nbytes, stream, user):
    """A block from PyTorch's caching allocator on the context's stream (user: the device
    index); NULL when it has none, which the library reports as AMG_ERR_OOM."""
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), device=int(user or 0), stream=int(stream or 0))
    except Exception:  # out of memory: the library raises its own error
        return None


def _torch_free(ptr, nbytes, stream, user):
    try:
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:  # interpreter shutdown: torch already torn down
        pass


_TORCH_ALLOC = ALLOC_FN(_torch_alloc)
_TORCH_FREE = FREE_FN(_torch_free)


class AmgParams(C.Structure):
    _fields_ = [
        ("smoother", C.c_int),
        ("aggregation", C.c_int),
        ("jacobi_omega", C.c_double),
        ("eps_strong", C.c_double),
        ("coarse_enough", C.c_int),
        ("max_levels", C.c_int),
        ("npre", C.c_int),
        ("npost", C.c_int),
        ("precision", C.c_int),
        ("rtol", C.c_double),
        ("maxiter", C.c_int),
        ("flexible_cg", C.c_int),
        ("block_size", C.c_int),
        ("alloc", ALLOC_FN),
        ("dealloc", FREE_FN),
        ("alloc_user", C.c_void_p),
    ]


class AmgPolicy(C.Structure):
    _fields_ = [("base", C.c_int), ("every", C.c_int), ("growth", C.c_double)]


def policy(base: int = PARTIAL, every: int = 0, growth: float = 0.0) -> AmgPolicy:
    return AmgPolicy(int(base), int(every), float(growth))


def policy_pick(pol: AmgPolicy, updates: int, iters_ref: int, last_iters: int, last_converged: int) -> int:
    """The mode the rebuild policy picks for a history (host logic of the library)."""
    m = C.c_int(-1)
    code = lib().amg_policy_pick(C.byref(pol), int(updates), int(iters_ref), int(last_iters),
                                 int(last_converged), C.byref(m))
    if code != AMG_OK:
        raise AmgError(code, "invalid rebuild policy")
    return m.value


class AmgSolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("rel_res_true", C.c_double)]


_lib = None


def lib():
    """Load the in-tree library; fails loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        V, I32, I64, D, I = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_int
        pP = C.POINTER(V)
        L.amg_params_default.argtypes = [C.POINTER(AmgParams)]
        L.amg_setup.argtypes = [pP, I32, I64, V, V, V, C.POINTER(AmgParams), V]
        L.amg_setup_transfer.argtypes = [pP, I32, I64, V, V, V, I, C.POINTER(V), C.POINTER(V), C.POINTER(V),
                                         C.POINTER(I32), C.POINTER(I64), C.POINTER(AmgParams), V]
        L.amg_rebuild.argtypes = [V, V, I]
        L.amg_set_pattern.argtypes = [V, I32, I64, V, V]
        L.amg_rebuild_ex.argtypes = [V, V, I]
        L.amg_solve.argtypes = [V, V, V, C.POINTER(AmgSolveInfo)]
        L.amg_solve_bicgstab.argtypes = [V, V, V, C.POINTER(AmgSolveInfo)]
        L.amg_vcycle.argtypes = [V, V, V]
        L.amg_apply_operator.argtypes = [V, V, V]
        L.amg_apply_operator_noalloc.argtypes = [V, V, V]
        L.amg_destroy.argtypes = [V]
        L.amg_last_error.argtypes = [V]
        L.amg_last_error.restype = C.c_char_p
        L.amg_num_levels.argtypes = [V, C.POINTER(I)]
        L.amg_level_dims.argtypes = [V, I, C.POINTER(I64)]
        L.amg_level_format.argtypes = [V, I, C.POINTER(I), C.POINTER(I), C.POINTER(I)]
        L.amg_export_level.argtypes = [V, I] + [V] * 9
        L.amg_export_coarse_inverse.argtypes = [V, V]
        L.amg_phase_times.argtypes = [V, C.POINTER(D)]
        L.amg_logcoef7_assemble.argtypes = [I32, I32, I32, V, V, V]
        L.amg_logcoef7_adjoint.argtypes = [I32, I32, I32, V, V, V, V, V]
        L.amg_trace.argtypes = [V, C.c_uint, I]
        L.amg_trace_every.argtypes = [V, I]
        L.amg_trace_read.argtypes = [V, C.POINTER(D), C.POINTER(I64)]
        L.amg_trace_read_levels.argtypes = [V, I, C.POINTER(D), C.POINTER(I64)]
        L.amg_level_storage.argtypes = [V, I, C.POINTER(I)]
        L.amg_policy_pick.argtypes = [C.POINTER(AmgPolicy), I, I, I, I, C.POINTER(I)]
        L.amg_rebuild_auto.argtypes = [V, V, C.POINTER(AmgPolicy), C.POINTER(I)]
        for name in EXPORTED:
            getattr(L, name).restype = C.c_int if name != "amg_last_error" else C.c_char_p
        _lib = L
    return _lib


def default_params(**kw) -> AmgParams:
    p = AmgParams()
    lib().amg_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(f"unknown AMG parameter {k!r}")
        setattr(p, k, v)
    return p


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class AMG:
    """A device-resident AMG hierarchy for a series of matrices with one pattern.

    allocator="torch" (the default) gives the library PyTorch's caching allocator for all
    its device memory (torch.cuda.memory_allocated() then counts the hierarchy);
    allocator="library" lets it use a stream-ordered pool of its own; a tuple (ALLOC_FN,
    FREE_FN[, user]) passes the caller's own callbacks."""

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, transfer=None,
                 allocator: str = "torch", **params):
        _dev(row_ptr, torch.int32, "row_ptr")
        _dev(col, torch.int32, "col")
        _dev(val, torch.float64, "val")
        self.n = row_ptr.numel() - 1
        self.nnz = col.numel()
        if val.numel() != self.nnz:
            raise ValueError("val and col lengths differ")
        self.params = default_params(**params)
        if allocator == "torch":
            self.params.alloc = _TORCH_ALLOC
            self.params.dealloc = _TORCH_FREE
            self.params.alloc_user = C.c_void_p(val.device.index or 0)
        elif isinstance(allocator, tuple):  # (ALLOC_FN, FREE_FN[, user]) of the caller's
            self.params.alloc, self.params.dealloc = allocator[0], allocator[1]
            self.params.alloc_user = C.c_void_p(allocator[2] if len(allocator) > 2 else None)
        elif allocator != "library":
            raise ValueError(f"allocator must be 'torch', 'library' or (alloc, dealloc), not {allocator!r}")
        self.allocator = allocator
        self.device = val.device
        self._stream = _stream()
        ctx = C.c_void_p()
        L = lib()
        if transfer is None:
            st = L.amg_setup(C.byref(ctx), self.n, self.nnz, _ptr(row_ptr), _ptr(col), _ptr(val),
                             C.byref(self.params), self._stream)
        else:
            k = len(transfer)
            Ps = [(_dev(p, torch.int32, "P_ptr"), _dev(c, torch.int32, "P_col"),
                   _dev(v, torch.float64, "P_val"), int(nc)) for p, c, v, nc in transfer]
            arr = lambda xs: (C.c_void_p * max(k, 1))(*[x.data_ptr() for x in xs])  # noqa: E731
            pp, pc, pv = arr([t[0] for t in Ps]), arr([t[1] for t in Ps]), arr([t[2] for t in Ps])
            ncs = (C.c_int32 * max(k, 1))(*[t[3] for t in Ps])
            nnzs = (C.c_int64 * max(k, 1))(*[t[1].numel() for t in Ps])
            st = L.amg_setup_transfer(C.byref(ctx), self.n, self.nnz, _ptr(row_ptr), _ptr(col), _ptr(val), k,
                                      pp, pc, pv, ncs, nnzs, C.byref(self.params), self._stream)
        if st != AMG_OK:
            raise AmgError(st, L.amg_last_error(None).decode())
        self.ctx = ctx
        self._values_token = None

    # -------------------------------------------------------------- lifecycle
    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            lib().amg_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != AMG_OK:
            raise AmgError(st, lib().amg_last_error(self.ctx).decode())

    # -------------------------------------------------------------- strategies
    def rebuild(self, val: torch.Tensor, pattern_changed: bool = False):
        """Algorithm 4 (partial reuse) for new values; asynchronous on the stream."""
        _dev(val, torch.float64, "val")
        self._values_token = None
        self._check(lib().amg_rebuild(self.ctx, _ptr(val), int(bool(pattern_changed))))

    def rebuild_ex(self, val: torch.Tensor, mode: int):
        _dev(val, torch.float64, "val")
        self._values_token = None
        self._check(lib().amg_rebuild_ex(self.ctx, _ptr(val), int(mode)))

    def rebuild_auto(self, val: torch.Tensor, pol: AmgPolicy) -> int:
        """New values with the mode the rebuild policy picks from this hierarchy's history
        (updates since its last full setup, first and last solve's iterations); returns it."""
        _dev(val, torch.float64, "val")
        self._values_token = None
        m = C.c_int(-1)
        self._check(lib().amg_rebuild_auto(self.ctx, _ptr(val), C.byref(pol), C.byref(m)))
        return m.value

    def set_pattern(self, row_ptr: torch.Tensor, col: torch.Tensor):
        _dev(row_ptr, torch.int32, "row_ptr")
        _dev(col, torch.int32, "col")
        self._check(lib().amg_set_pattern(self.ctx, row_ptr.numel() - 1, col.numel(), _ptr(row_ptr), _ptr(col)))
        self.n, self.nnz = row_ptr.numel() - 1, col.numel()

    def solve(self, f: torch.Tensor, u: torch.Tensor | None = None):
        """PCG with one V-cycle per iteration.  Returns (u, info)."""
        _dev(f, torch.float64, "f")
        if u is None:
            u = torch.zeros_like(f)
        else:
            _dev(u, torch.float64, "u")
        info = AmgSolveInfo()
        self._check(lib().amg_solve(self.ctx, _ptr(f), _ptr(u), C.byref(info)))
        return u, dict(iters=info.iters, converged=bool(info.converged), rel_res_true=info.rel_res_true)

    def solve_bicgstab(self, f: torch.Tensor, u: torch.Tensor | None = None):
        """BiCGStab with the V-cycle on the right (non-symmetric operators).  Returns (u, info)."""
        _dev(f, torch.float64, "f")
        if u is None:
            u = torch.zeros_like(f)
        else:
            _dev(u, torch.float64, "u")
        info = AmgSolveInfo()
        self._check(lib().amg_solve_bicgstab(self.ctx, _ptr(f), _ptr(u), C.byref(info)))
        return u, dict(iters=info.iters, converged=bool(info.converged), rel_res_true=info.rel_res_true)

    def apply_operator(self, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
        """y = A x by the level-0 Krylov SpMV kernel (asynchronous on the stream)."""
        _dev(x, torch.float64, "x")
        y = torch.empty_like(x) if y is None else y
        _dev(y, torch.float64, "y")
        self._check(lib().amg_apply_operator(self.ctx, _ptr(x), _ptr(y)))
        return y

    def vcycle(self, r: torch.Tensor) -> torch.Tensor:
        _dev(r, torch.float64, "r")
        z = torch.empty_like(r)
        self._check(lib().amg_vcycle(self.ctx, _ptr(r), _ptr(z)))
        return z

    # -------------------------------------------------------------- introspection
    @property
    def num_levels(self) -> int:
        L = C.c_int()
        self._check(lib().amg_num_levels(self.ctx, C.byref(L)))
        return L.value

    def dims(self, l: int):
        d = (C.c_int64 * 5)()
        self._check(lib().amg_level_dims(self.ctx, l, d))
        return [int(x) for x in d]

    def level_format(self, l: int) -> int:
        """Diagonals of level l's diagonal storage (0: CSR kernels)."""
        nd = C.c_int()
        self._check(lib().amg_level_format(self.ctx, l, C.byref(nd), None, None))
        return nd.value

    def diagonals_read(self, l: int) -> int:
        """Diagonals the solve kernels read per row of level l's diagonal storage: half of
        them (plus the main one) once a solve has seen symmetric values."""
        nd, nr = C.c_int(), C.c_int()
        self._check(lib().amg_level_format(self.ctx, l, C.byref(nd), C.byref(nr), None))
        return nr.value

    def march_plane(self, l: int) -> int:
        """Plane stride of the 7-point marching kernels on level l (0: not used)."""
        nd, pl = C.c_int(), C.c_int()
        self._check(lib().amg_level_format(self.ctx, l, C.byref(nd), None, C.byref(pl)))
        return pl.value

    def level(self, l: int):
        """Host copies of level l: dict with A (ptr, col, val), P (ptr, col, val, nc) or
        None, agg, strong, m."""
        n, nnzA, nc, nnzP, _ = self.dims(l)
        coarsest = l == self.num_levels - 1
        Ap, Ac, Av = np.zeros(n + 1, np.int32), np.zeros(nnzA, np.int32), np.zeros(nnzA)
        agg = np.full(n, -2, np.int32)
        strong = np.full(nnzA, 2, np.uint8)
        m = np.zeros(n * max(1, self.params.block_size))   # block_size x block_size per node
        P = None if coarsest else (np.zeros(n + 1, np.int32), np.zeros(nnzP, np.int32), np.zeros(nnzP))
        vp = lambda a: C.c_void_p(a.ctypes.data) if a is not None else None  # noqa: E731
        self._check(lib().amg_export_level(
            self.ctx, l, vp(agg), vp(strong), vp(Ap), vp(Ac), vp(Av),
            vp(P[0]) if P else None, vp(P[1]) if P else None, vp(P[2]) if P else None,
            vp(m) if not coarsest else None))
        out = dict(n=n, A=(Ap, Ac, Av), agg=None, strong=None, m=None, P=None)
        if not coarsest:
            out["P"] = (*P, nc)
            out["m"] = m
        if not (agg == -2).all():
            out["agg"] = agg
        if not (strong == 2).all():
            out["strong"] = strong.astype(bool)
        return out

    def coarse_inverse(self) -> np.ndarray:
        nL = self.dims(self.num_levels - 1)[0]
        M = np.zeros((nL, nL))
        self._check(lib().amg_export_coarse_inverse(self.ctx, C.c_void_p(M.ctypes.data)))
        return M

    def trace(self, classes, level: int = 0, every: int = 1):
        """Time the launches of the named kernel classes on `level` with HIP events: every
        launch, or with `every` > 1 only each every-th one per class and level."""
        mask = 0
        for name in classes:
            mask |= 1 << KERNEL_CLASSES.index(name)
        self._check(lib().amg_trace(self.ctx, mask, level))
        self._check(lib().amg_trace_every(self.ctx, every))

    def trace_read(self) -> dict:
        """{class: (total ms, launches)} since the previous read."""
        ms = (C.c_double * 16)()
        cnt = (C.c_int64 * 16)()
        self._check(lib().amg_trace_read(self.ctx, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_CLASSES) if cnt[i]}

    def trace_read_levels(self) -> list:
        """Per level: {class: (total ms, launches)} since the previous read."""
        L = self.num_levels
        K = len(KERNEL_CLASSES)
        ms = (C.c_double * (L * K))()
        cnt = (C.c_int64 * (L * K))()
        self._check(lib().amg_trace_read_levels(self.ctx, L, ms, cnt))
        return [{k: (ms[l * K + i], cnt[l * K + i]) for i, k in enumerate(KERNEL_CLASSES) if cnt[l * K + i]}
                for l in range(L)]

    def level_storage(self, l: int) -> dict:
        """Column format and launch shape of level l's operators in the solve kernels."""
        out = (C.c_int * 10)()
        self._check(lib().amg_level_storage(self.ctx, l, out))
        return dict(A_c16=out[0], P_c16=out[1], R_c16=out[2], A_rpb=out[3], P_rpb=out[4], R_rpb=out[5],
                    tail=out[6], value_bytes=out[7], node_galerkin=out[8], node_transfer=out[9])

    def phase_times(self) -> dict:
        out = (C.c_double * 8)()
        self._check(lib().amg_phase_times(self.ctx, out))
        keys = ["aggregation", "prolongator", "symbolic", "galerkin", "smoother", "coarse", "total"]
        return dict(zip(keys, list(out)[:7]))


# ------------------------------------------------------------------ differentiable form

def logcoef7_assemble(theta: torch.Tensor, nx: int, ny: int, nz: int) -> torch.Tensor:
    """Values of the 7-point operator A(theta) on the sorted 7-point pattern."""
    _dev(theta, torch.float64, "theta")
    if theta.numel() != nx * ny * nz:
        raise ValueError("theta has the wrong size")
    nnz = 7 * nx * ny * nz - 2 * (nx * ny + ny * nz + nx * nz)
    val = torch.empty(nnz, dtype=torch.float64, device=theta.device)
    st = lib().amg_logcoef7_assemble(nx, ny, nz, _ptr(theta), _ptr(val), _stream())
    if st != AMG_OK:
        raise AmgError(st, lib().amg_last_error(None).decode())
    return val


def logcoef7_adjoint(theta, u, lam, nx: int, ny: int, nz: int) -> torch.Tensor:
    for t, nm in ((theta, "theta"), (u, "u"), (lam, "lambda")):
        _dev(t, torch.float64, nm)
    g = torch.empty_like(theta)
    st = lib().amg_logcoef7_adjoint(nx, ny, nz, _ptr(theta), _ptr(u), _ptr(lam), _ptr(g), _stream())
    if st != AMG_OK:
        raise AmgError(st, lib().amg_last_error(None).decode())
    return g


class AMGSolve(torch.autograd.Function):
    """u = A(theta)^{-1} f for the 7-point log-coefficient operator, differentiable in
    theta and f.  The forward pass assembles A(theta) on the device and runs the partial
    update (Algorithm 4) of ``amg`` before the solve; the backward pass solves the adjoint
    system on the same hierarchy (A is symmetric) and scatters -lambda (dA/dtheta) u."""

    @staticmethod
    def forward(ctx, theta, f, amg: AMG, grid):
        nx, ny, nz = grid
        val = logcoef7_assemble(theta.detach().contiguous(), nx, ny, nz)
        amg.rebuild(val)
        token = object()
        amg._values_token = token
        u, info = amg.solve(f.detach().contiguous())
        if not info["converged"]:
            raise AmgError(-6, f"forward solve did not converge ({info})")
        ctx.amg, ctx.grid, ctx.token = amg, grid, token
        ctx.save_for_backward(theta, u, val)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        theta, u, val = ctx.saved_tensors
        amg = ctx.amg
        if amg._values_token is not ctx.token:  # the hierarchy moved on: restore A(theta)
            amg.rebuild(val)
            amg._values_token = ctx.token
        lam, info = amg.solve(grad_u.detach().contiguous())
        if not info["converged"]:
            raise AmgError(-6, f"adjoint solve did not converge ({info})")
        g = logcoef7_adjoint(theta.detach().contiguous(), u, lam, *ctx.grid)
        return g, lam, None, None
