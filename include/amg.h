/*
 * amg.h -- C interface of the MI355X (gfx950) partial-reuse AMG library.
 *
 * The library solves A u = f for a sequence of sparse SPD matrices that share one
 * sparsity pattern (a non-steady-state problem, one matrix per time step).  A smoothed-
 * aggregation hierarchy is built once (Algorithm 1 of Demidov, "Partial Reuse AMG Setup
 * Cost Amortization Strategy for the Solution of Non-Steady State Problems", Section 2).
 * On later steps the transfer operators P_l and R_l = P_l^T are kept while every level's
 * Galerkin operator A_{l+1} = R_l A_l P_l, smoother and the coarsest direct solver are
 * rebuilt (Algorithm 4, Section 3); the Galerkin products reuse the sparsity pattern
 * computed at setup, so only their numeric phase runs (the extension proposed in
 * Section 5).  The solve is CG preconditioned by one V-cycle (Algorithm 2 and the last
 * paragraph of Section 2).
 *
 * Conventions for every entry point:
 *  - Matrices are CSR with 0-based int32 row pointers and columns, columns sorted
 *    ascending and unique within a row, a stored positive diagonal, a structurally
 *    symmetric pattern and SPD values.
 *  - Pointers are DEVICE pointers unless marked (host).  Inputs are borrowed for the
 *    duration of the call; the library copies what it keeps.
 *  - All device work is enqueued on the HIP stream given to amg_setup (NULL: the null
 *    stream), except the blocked inverse of a coarsest level of more than 128 rows after a
 *    partial update, which runs on a stream the context owns (ordered after the update's
 *    work on the given stream) so that it overlaps the start of the next solve; every later
 *    use of the hierarchy on the given stream waits for it, and amg_destroy for all of the
 *    context's work.  The caller's buffers must be ready on the given stream.
 *  - Every call returns an amg_status and never throws across the interface.  After a
 *    HIP runtime error, and after any failure of a call that replaces the hierarchy (a full
 *    rebuild, AMG_FULL or a size change; a pattern change), the context is unusable: every
 *    later call on it returns AMG_ERR_STATE, and only amg_last_error and amg_destroy
 *    remain.  Other failures (invalid arguments, a CG breakdown, a failed allocation before
 *    anything changed) leave the context as it was.  amg_last_error() describes the last
 *    failure of a context.
 *  - Device memory: from the caller's allocator when amg_params.alloc/dealloc are set
 *    (e.g. PyTorch's caching allocator), else from a stream-ordered pool private to the
 *    context (see amg_setup).
 */
#ifndef AMGMI_AMG_H
#define AMGMI_AMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amg_ctx amg_ctx;

typedef enum {
    AMG_OK = 0,
    AMG_ERR_ARG = -1,       /* invalid argument (NULL, size, unsorted/out-of-range columns) */
    AMG_ERR_HIP = -2,       /* HIP runtime error */
    AMG_ERR_OOM = -3,       /* device allocation failed */
    AMG_ERR_PATTERN = -4,   /* pattern not structurally symmetric, or changed unexpectedly */
    AMG_ERR_NOT_SPD = -5,   /* non-positive diagonal or coarse pivot */
    AMG_ERR_BREAKDOWN = -6, /* CG breakdown: p.Ap <= 0 or a non-finite scalar */
    AMG_ERR_STATE = -7      /* context unusable after an earlier HIP error or failed replacement */
} amg_status;

/* How amg_rebuild_ex updates the hierarchy for new matrix values (same pattern). */
typedef enum {
    AMG_PARTIAL = 0,       /* Algorithm 4: keep P_l, R_l; rebuild A_{l+1}, smoothers, coarse solver */
    AMG_FULL = 1,          /* Algorithm 1 from scratch (aggregation, P_l, patterns, everything) */
    AMG_OPERATOR_ONLY = 2  /* Algorithm 3 (full reuse): only the Krylov operator changes */
} amg_rebuild_mode;

typedef struct {
    int smoother;         /* 0: damped Jacobi m_i = omega/a_ii; 1: SPAI0 m_i = a_ii / sum_j a_ij^2 */
    int aggregation;      /* 0: smoothed aggregation; 1: plain aggregation (P = tentative) */
    double jacobi_omega;  /* Jacobi damping (0.72) */
    double eps_strong;    /* strength threshold on level 0, halved per level (0.08) */
    int coarse_enough;    /* stop coarsening at <= this many rows (1024; the coarsest level
                           * gets a dense inverse, which takes at most 2048 rows) */
    int max_levels;       /* (12) */
    int npre, npost;      /* Jacobi/SPAI0 sweeps before and after the coarse correction (1, 1) */
    int precision;        /* 0: FP64 everywhere; 1: FP32 hierarchy and V-cycle under FP64 CG */
    double rtol;          /* stop when ||f - A u||_2 / ||f||_2 <= rtol, true residual (1e-8) */
    int maxiter;          /* (100) */
    int flexible_cg;      /* 1: beta = r.(z - z_old) / rho_old (robust to an inexact B) */
    int block_size;       /* unknowns per node (1).  B in 2..8 describes a system whose unknown b
                           * of node I is row I*B + b and whose stored entries form full B x B
                           * blocks (every row of a node lists the same columns, in groups of B
                           * starting at a multiple of B), as in the paper's 4x4-block systems
                           * (Section 4): the nodes are aggregated on the matrix of block
                           * Frobenius norms, unknown b of a node joins unknown b of its
                           * aggregate, and the smoother is damped block Jacobi, omega times
                           * the inverse of each node's diagonal block (AMG_ERR_NOT_SPD at
                           * setup for a singular one; after a partial update it shows as a
                           * breakdown of the next solve).  Needs aggregation = 1, smoother =
                           * 0, flexible_cg = 0 and n divisible by B (AMG_ERR_ARG otherwise);
                           * a matrix without full blocks gives AMG_ERR_PATTERN. */
    /* Device allocator of the context (both NULL, the default: the library's own).  alloc
     * returns a block of at least `bytes` bytes usable by work enqueued on `stream` (the
     * context's stream) after the call, or NULL when it has none (the call then fails with
     * AMG_ERR_OOM); dealloc receives each block back with the size asked for, once the
     * library has enqueued its last use of it on `stream` (stream-ordered: the block may be
     * reused by later work on that stream, not by other streams before it completes).
     * user is passed through.  Called only from the thread that called the library; both
     * must be set or both NULL (AMG_ERR_ARG). */
    void* (*alloc)(size_t bytes, void* stream, void* user);
    void (*dealloc)(void* ptr, size_t bytes, void* stream, void* user);
    void* alloc_user;
} amg_params;

typedef struct {          /* host struct filled by amg_solve */
    int iters;            /* CG iterations taken */
    int converged;        /* 1 when the true relative residual reached rtol */
    double rel_res_true;  /* ||f - A u|| / ||f|| of the returned u */
} amg_solve_info;

/* Fill *p (host) with the defaults listed above. */
amg_status amg_params_default(amg_params* p);

/* Algorithm 1 on the device.  n rows, nnz entries; row_ptr[n+1], col[nnz], val[nnz] are
 * device arrays; p is a host struct (NULL: defaults).  Synchronises the stream (coarse
 * sizes are needed on the host).  *out receives a new context on AMG_OK, NULL otherwise.
 * Device memory: with p->alloc set, every block comes from the caller's allocator.
 * Otherwise the context creates a stream-ordered pool of its own on the current device
 * (hipMemPoolCreate; it keeps freed memory, release threshold UINT64_MAX, so repeated
 * setups reuse it instead of mapping it anew; no other pool is changed) and keeps the
 * blocks it frees, per size class (at most 12.5 % padding), for its next allocations; the
 * kept blocks never exceed the context's own peak of live device memory.  A failed
 * allocation hands back the kept blocks of this context, then of every context of the
 * library, trims their pools and retries.  amg_destroy frees everything and destroys the
 * pool. */
amg_status amg_setup(amg_ctx** out, int32_t n, int64_t nnz, const int32_t* row_ptr,
                     const int32_t* col, const double* val, const amg_params* p, void* hip_stream);

/* Algorithm 1 with prescribed transfer operators (test hook for closed-form Galerkin
 * products): level l < nlev uses P_l with n_l rows, nc[l] columns and nnzP[l] entries
 * (device CSR arrays P_ptr[l], P_col[l], P_val[l]; the pointer arrays and nc, nnzP are
 * host arrays).  The level reached after them is the coarsest. */
amg_status amg_setup_transfer(amg_ctx** out, int32_t n, int64_t nnz, const int32_t* row_ptr,
                              const int32_t* col, const double* val, int nlev,
                              const int32_t* const* P_ptr, const int32_t* const* P_col,
                              const double* const* P_val, const int32_t* nc, const int64_t* nnzP,
                              const amg_params* p, void* hip_stream);

/* New values val[nnz] (device) for the current pattern.  pattern_changed == 0 runs
 * Algorithm 4 (numeric Galerkin products on the cached patterns, smoothers, coarse
 * inverse) without any host synchronisation.  pattern_changed != 0 is valid only after
 * amg_set_pattern: with the same n the transfer operators are kept and the Galerkin
 * patterns are recomputed before the partial update; with a different n a full setup runs
 * (a size change, Section 3).  Non-zero without a pending pattern returns AMG_ERR_ARG. */
amg_status amg_rebuild(amg_ctx* c, const double* val, int pattern_changed);

/* Register a new pattern (device arrays, n rows, nnz entries, borrowed for the call and
 * copied) for the next amg_rebuild(..., 1).  Section 3 notes that the pattern of
 * discretised PDE matrices seldom changes between steps and that a change of size (e.g. by
 * adaptive remeshing) needs a full rebuild; with the same n this library keeps the transfer
 * operators and recomputes only the Galerkin patterns.  Nothing is checked or changed until
 * that rebuild (which validates the pattern).  Errors: AMG_ERR_ARG for a NULL context or
 * array, n <= 0, nnz <= 0 or nnz >= 2^31; AMG_ERR_OOM. */
amg_status amg_set_pattern(amg_ctx* c, int32_t n, int64_t nnz, const int32_t* row_ptr,
                           const int32_t* col);

/* New values with an explicit update mode (see amg_rebuild_mode). */
amg_status amg_rebuild_ex(amg_ctx* c, const double* val, amg_rebuild_mode m);

/* Rebuild policy layered on amg_rebuild_ex (Section 3: full reuse until a solve misses the
 * iteration limit, Algorithm 3; an occasional full rebuild between partial updates).
 *   base:   AMG_PARTIAL or AMG_OPERATOR_ONLY, the mode used when no trigger fires;
 *   every:  > 0: a full setup as the every-th update after the last full setup (0: off);
 *   growth: > 0: a full setup when the last solve took more than growth times the
 *           iterations of the first solve after the last full setup (0: off).
 * With the AMG_OPERATOR_ONLY base a solve that did not converge also triggers one. */
typedef struct {
    amg_rebuild_mode base;
    int every;
    double growth;
} amg_policy;

/* The mode the policy p (host) picks, host logic only: updates = updates since the last
 * full setup (0 right after it), iters_ref = iterations of the first solve after it (0:
 * none yet), last_iters / last_converged = the last solve (last_iters 0: none yet).
 * *mode (host) receives AMG_FULL or p->base.  Errors: AMG_ERR_ARG for NULL pointers, a
 * base other than AMG_PARTIAL / AMG_OPERATOR_ONLY, every < 0 or growth < 0 (or NaN). */
amg_status amg_policy_pick(const amg_policy* p, int updates, int iters_ref, int last_iters, int last_converged,
                           amg_rebuild_mode* mode);

/* amg_rebuild_ex(c, val, m) with m = amg_policy_pick(p, ...) on c's history (updates since
 * its last full setup, the first and the last solve's iterations); *taken (host, may be
 * NULL) receives m.  Errors: those of amg_policy_pick and amg_rebuild_ex. */
amg_status amg_rebuild_auto(amg_ctx* c, const double* val, const amg_policy* p, amg_rebuild_mode* taken);

/* CG preconditioned by one V-cycle per iteration (the V-cycle of Algorithm 2 used as the
 * preconditioner of a Krylov method, last paragraph of Section 2).  f[n] (device, read),
 * u[n] (device, in: initial guess, out: solution).  info (host) may be NULL.  Returns after convergence
 * or maxiter: one 16-byte device-to-host read per iteration decides the stop.  Not
 * converging is not an error (info->converged = 0). */
amg_status amg_solve(amg_ctx* c, const double* f, double* u, amg_solve_info* info);

/* BiCGStab (van der Vorst) with one V-cycle applied on the right per half step: the
 * paper's Krylov method, for non-symmetric operators (Section 4).  Arguments, stopping
 * rule (true relative residual, maxiter, restart from the true residual when the
 * recursive one reached rtol but the true one did not) and info as for amg_solve; each
 * iteration applies the V-cycle and the Krylov operator twice, forms its scalars (alpha,
 * omega, beta, the half-step test) on the device and reads the ||r||^2 partials and the
 * breakdown flags back once.  A zero or non-finite r^.r, r^.v, t.t or omega returns
 * AMG_ERR_BREAKDOWN.  The coarsest level's inverse is formed without pivoting and needs
 * positive elimination pivots (diagonally dominant M-matrices have them). */
amg_status amg_solve_bicgstab(amg_ctx* c, const double* f, double* u, amg_solve_info* info);

/* One V-cycle z = B r from a zero initial guess (Algorithm 2: pre-smoothing, restriction,
 * recursion, the coarsest direct solve, prolongation, post-smoothing; r, z: device, n
 * entries, z overwritten; asynchronous on the stream).  AMG_ERR_ARG for NULL arguments. */
amg_status amg_vcycle(amg_ctx* c, const double* r, double* z);

/* y = A x with the Krylov operator (the values of the last update, pattern of level 0),
 * by the kernel the CG applies on its first iteration (the level-0 SpMV of Section 2's
 * Krylov loop): x, y device arrays of n entries, distinct; asynchronous on the stream.
 * For measurements and checks; it overwrites the CG's work vectors.  AMG_ERR_ARG for
 * NULL or aliased arguments. */
amg_status amg_apply_operator(amg_ctx* c, const double* x, double* y);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): amg_apply_operator with the same kernels
 * and results, whose scratch (the copy of p the Krylov SpMV writes and its block partials)
 * lives in a static device array of the library instead of the context's CG vectors.  The
 * call allocates nothing and never touches the CG's work vectors.  The array holds
 * 2^23 + 2^20 doubles (72 MiB) on every device the library is used on, from the library's
 * load to the end of the process; its address on a device is looked up on the first call
 * there.  Limits: n <= 2^23 rows, and the SpMV's grid within the partial region; beyond
 * them AMG_ERR_ARG with a message.  The context's device must be current (AMG_ERR_ARG
 * otherwise).  All calls on one device share the array: calls that overlap on a device
 * (other streams, other threads) race and must be serialised by the caller.  Asynchronous
 * on the context's stream; AMG_ERR_ARG for NULL or aliased x, y; AMG_ERR_STATE on a broken
 * context. */
amg_status amg_apply_operator_noalloc(amg_ctx* c, const double* x, double* y);

/* Release the context: waits for its stream, frees all its device memory (to the caller's
 * allocator, or by destroying its private pool), its pinned host buffers and events.
 * Valid on a broken context.  AMG_ERR_ARG for NULL.  (Not a step of the paper; the end of
 * the time loop of Algorithms 3 and 4.) */
amg_status amg_destroy(amg_ctx* c);

/* Description of the last failure of c (or of the last failed amg_setup when c is NULL). */
const char* amg_last_error(const amg_ctx* c);

/* ---- introspection (tests and reports) ---- */
amg_status amg_num_levels(const amg_ctx* c, int* L);

/* dims[0..4] = { n_l, nnz(A_l), n_{l+1} (0 on the coarsest), nnz(P_l), nnz(A_l P_l) } */
amg_status amg_level_dims(const amg_ctx* c, int l, int64_t* dims);

/* Storage of level l's operator in the solve kernels: *ndiag (host) receives the number of
 * stored diagonals when the level is kept in diagonal storage (the finest level of a
 * stencil operator: at most 32 distinct column offsets, well filled; the values are
 * refreshed from the CSR copy after every rebuild), or 0 when the CSR kernels are used.
 * *nread (host, may be NULL) receives the number of diagonals the solve kernels read per
 * row: (ndiag+1)/2 when the offsets are symmetric and the values last refreshed were
 * found symmetric (the solve reads each sub-diagonal entry as its mirror; known from the
 * first solve after a rebuild on), else ndiag.  *plane (host, may be NULL) receives the
 * plane stride a when the level-0 kernels of a 7-point operator (offsets -a, -b, -1, 0,
 * 1, b, a) walk the grid plane by plane (two planes per workgroup, neighbours within a
 * plane from LDS), else 0.
 * Errors: AMG_ERR_ARG for a NULL ndiag or l out of range. */
amg_status amg_level_format(const amg_ctx* c, int l, int* ndiag, int* nread, int* plane);

/* Copy level l to host arrays (any may be NULL).  agg[n_l], strong[nnz(A_l)] exist on
 * aggregated levels; P on non-coarsest levels; m (smoother diagonal, n_l values; with
 * block_size B > 1 the n_l / B blocks omega * D_I^{-1}, row-major, n_l * B values) on
 * non-coarsest levels.  In mixed precision A_val/P_val/m are the FP32 values widened to FP64.
 * Synchronises the stream. */
amg_status amg_export_level(const amg_ctx* c, int l, int32_t* agg, uint8_t* strong, int32_t* A_ptr,
                            int32_t* A_col, double* A_val, int32_t* P_ptr, int32_t* P_col,
                            double* P_val, double* m);

/* Dense inverse of the coarsest operator (host, n_L * n_L, row-major). */
amg_status amg_export_coarse_inverse(const amg_ctx* c, double* inv);

/* Milliseconds of the phases of the last setup or rebuild (host out[8]):
 * {strength+aggregation, prolongator+transpose, symbolic Galerkin, numeric Galerkin,
 *  smoother, coarse inverse, total, 0}.  Synchronises the stream. */
amg_status amg_phase_times(const amg_ctx* c, double* out);

/* ---- per-kernel timing (reports and roofline measurements) ---- */

typedef enum {
    AMG_K_GALERKIN_AP = 0,   /* numeric A_l P_l */
    AMG_K_GALERKIN_RAP = 1,  /* numeric R_l (A_l P_l) */
    AMG_K_SMOOTHER = 2,      /* smoother diagonal */
    AMG_K_COARSE_INV = 3,    /* densify + inverse of the coarsest operator */
    AMG_K_CG_PQ = 4,         /* p = z + beta p, q = A p, p.q (the Krylov operator SpMV) */
    AMG_K_CG_UPDATE = 5,     /* x += alpha p, r -= alpha q, r.r */
    AMG_K_CG_RZ = 6,         /* r.z */
    AMG_K_CG_INIT = 7,       /* r = f - A x, r.r, f.f */
    AMG_K_SMOOTH0_RES = 8,   /* first pre-smoothing sweep fused with the residual */
    AMG_K_JACOBI = 9,        /* one smoothing sweep */
    AMG_K_RESTRICT = 10,     /* f_{l+1} = R_l r_l */
    AMG_K_PROLONG = 11,      /* u_l += P_l u_{l+1} */
    AMG_K_COARSE_GEMV = 12,  /* u_L = A_L^{-1} f_L */
    AMG_K_CAST = 13,         /* FP64 <-> FP32 conversions of the mixed-precision form */
    AMG_K_TAIL = 14,         /* restriction into the coarse tail and Algorithm 2 on all its levels */
    AMG_K_BICG_SPMV = 15,    /* BiCGStab's products with the Krylov operator (v = A p^, t = A s^) */
    AMG_K_COUNT = 16
} amg_kernel_class;

/* Bracket every launch of the kernel classes in `mask` (bit k = class k) on level `level`
 * (-1: every level; the CG kernels count as level 0) with HIP events on the context's
 * stream.  mask = 0 turns tracing off. */
amg_status amg_trace(amg_ctx* c, unsigned mask, int level);

/* Bracket only every `every`-th launch (1, 1 + every, ...) of each traced class on each
 * level; the others run with no events, so a timing of live launches adds little to the
 * work it times (each bracketed launch holds the stream for its timestamps).  Counts start
 * again at this call and at amg_trace.  AMG_ERR_ARG for every < 1.  Default 1. */
amg_status amg_trace_every(amg_ctx* c, int every);

/* Milliseconds and launch counts per class (host arrays of AMG_K_COUNT) accumulated since
 * the previous read; resets them.  Synchronises the stream. */
amg_status amg_trace_read(amg_ctx* c, double* ms, int64_t* launches);

/* The same per level: ms and launches (host arrays of nlev * AMG_K_COUNT, row-major by
 * level; the CG kernels count as level 0, launches on levels >= nlev as level nlev - 1).
 * AMG_ERR_ARG for NULL arrays or nlev <= 0.  Synchronises the stream. */
amg_status amg_trace_read_levels(amg_ctx* c, int nlev, double* ms, int64_t* launches);

/* How level l is stored for the solve kernels (host out[10]): {A_l, P_l, R_l read with
 * two-byte column offsets (1) or int32 columns (0) by the row-block kernels; rows per
 * LDS-staged block of A_l, P_l, R_l (0: lane-group kernels); 1 when the level is part of the
 * one-workgroup coarse tail; value bytes of the hierarchy (8 FP64, 4 FP32); 1 when a
 * partial update forms A_{l+1} from A_l's B x B blocks in one pass (block systems whose
 * P_l is the node aggregation's, Section 4's block value type; known once the first
 * partial update after a setup or a pattern change has run), 0 otherwise; 1 when the
 * V-cycle's prolongation from level l + 1 reads one aggregate index per node instead of
 * P_l's row pointers, columns and values (the same block systems)}.  For reports of the bytes the kernels move.  AMG_ERR_ARG for NULL
 * out or l out of range. */
amg_status amg_level_storage(const amg_ctx* c, int l, int* out);

/* ---- differentiable form: 7-point operator with per-cell log-coefficients ---- */

/* val[nnz] (device) = A(theta) on the sorted 7-point pattern of an nx*ny*nz grid (cell
 * x + nx*(y + ny*z)): a_cj = -2 k_c k_j / (k_c + k_j) with k = exp(theta), and
 * a_cc = sum_j 2 k_c k_j / (k_c + k_j) + (number of missing neighbours) * k_c. */
amg_status amg_logcoef7_assemble(int32_t nx, int32_t ny, int32_t nz, const double* theta,
                                 double* val, void* hip_stream);

/* grad[c] (device) = -lambda^T (dA/dtheta_c) u for the operator above (the gradient of a
 * loss L(u) when lambda = A^{-1} dL/du, A symmetric). */
amg_status amg_logcoef7_adjoint(int32_t nx, int32_t ny, int32_t nz, const double* theta,
                                const double* u, const double* lambda, double* grad,
                                void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* AMGMI_AMG_H */
