// amg_internal.h -- hierarchy layout and kernel launchers of the gfx950 AMG library.
//
// Everything lives in device memory for the lifetime of a context; nothing is moved
// between host and device after setup except a few scalars per CG iteration.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "amg.h"

namespace amgmi {

// ------------------------------------------------------------------ error handling
struct Fail {
    amg_status st;
    std::string msg;
};

[[noreturn]] void throw_hip(hipError_t e, const char* expr, const char* file, int line);

#define HIP_CHECK(x)                                                                   \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) ::amgmi::throw_hip(e_, #x, __FILE__, __LINE__);          \
    } while (0)

#define HIP_LAUNCH_CHECK() HIP_CHECK(hipGetLastError())

// ------------------------------------------------------------------ memory
// Device memory of one context.  With the caller's allocator (amg_params.alloc/dealloc)
// every block comes from it and goes back to it when the library frees it.  Otherwise the
// context owns a private stream-ordered pool (hipMemPoolCreate, set to keep what it has,
// destroyed with the context) and keeps the blocks it frees, per size class, for its next
// allocations: a full setup allocates nearly the same sizes in the same order every time,
// so its temporaries and its new hierarchy come from these blocks rather than from the
// pool, whose host cost per call was measured to grow from microseconds to ~0.1 ms once
// long-lived buffers were interleaved with setups.  The kept blocks are bounded by the
// context's own peak of live device memory; past it they all go back to the pool.
struct DevMem {
    void* (*hook_alloc)(size_t, void*, void*) = nullptr;
    void (*hook_free)(void*, size_t, void*, void*) = nullptr;
    void* hook_user = nullptr;
    hipStream_t s = nullptr;
    hipMemPool_t pool = nullptr;                // private pool (no caller allocator)
    std::unordered_map<void*, size_t> live;     // block -> bytes (the class size when kept)
    std::map<size_t, std::vector<void*>> kept;  // freed blocks by size class
    size_t live_bytes = 0, kept_bytes = 0, peak_bytes = 0;
    std::mutex mu;
};

// Allocations made between the construction and destruction of a MemScope use its DevMem
// (every entry point that takes a context opens one); outside any scope dalloc/dfree go
// straight to hipMallocAsync/hipFreeAsync.
struct MemScope {
    DevMem* prev;
    explicit MemScope(DevMem* m);
    ~MemScope();
    MemScope(const MemScope&) = delete;
    MemScope& operator=(const MemScope&) = delete;
};
void* dalloc(size_t bytes, hipStream_t s);
void dfree(void* p, hipStream_t s);
void mem_init(DevMem& m, hipStream_t s, void* (*a)(size_t, void*, void*), void (*f)(void*, size_t, void*, void*),
              void* user);
void mem_release(DevMem& m);  // kept blocks back, stream synchronised, private pool destroyed

template <typename T>
T* dnew(size_t n, hipStream_t s) {
    return static_cast<T*>(dalloc(n * sizeof(T) + (n == 0 ? 8 : 0), s));
}

// ------------------------------------------------------------------ layout
// CSR in HBM: int32 row pointers and columns (every size of the configurations fits),
// FP64 values plus an optional FP32 shadow used by the mixed-precision hierarchy.
struct Csr {
    int32_t nrows = 0, ncols = 0;
    int64_t nnz = 0;
    int32_t* ptr = nullptr;
    int32_t* col = nullptr;
    double* val = nullptr;
    float* val32 = nullptr;
    // Launch shape of the row kernels: rows per LDS-staged block (0: rows too long to
    // stage, use lane groups) and the lane-group width.
    int rpb = 0;
    int g = 8;
    // Two-byte column indices for the row-block kernels: col = cblk[row block] + c16[k]
    // (null when some block's columns span more than 65535)
    uint16_t* c16 = nullptr;
    int32_t* cblk = nullptr;
    template <typename T>
    T* v() const;
};
template <>
inline double* Csr::v<double>() const { return val; }
template <>
inline float* Csr::v<float>() const { return val32; }

// A Galerkin product C = L B in the position-map form: lanes per output row g, LDS
// accumulators per row cap, and the cached position map (for every product term l * b of
// a C row, in the row-by-row product's order, the position of its column in the C row;
// one byte each when every C row is shorter than 256, else two), with each row's first
// term at off[row].  g == 0: the product uses the lane-group kernels.
struct GalShape {
    int g = 0;
    int cap = 0;
    int epl = 2;                // L entries per lane per chunk
    int wide = 0;               // 1: two-byte positions
    int tpl = 1;                // B terms per lane loaded per entry of a batch (1 or 2)
    // device arrays owned by the hierarchy
    void* pos = nullptr;        // position map, one entry per term
    int64_t* off = nullptr;     // nrows + 1 term offsets
    int32_t* bst = nullptr;     // per L entry: start of its B row
    uint16_t* tof = nullptr;    // per L entry: its first term's offset within the row
    int32_t* dpos = nullptr;    // per L row: index of its diagonal entry (C = A P only)
    int64_t terms = 0;
};

// Galerkin product of a block system whose transfer operator is P_l = P_node (x) I_B with
// unit values (node aggregation, plain): block (J, L) of A_{l+1} is the sum, over the fine
// nodes I of aggregate J in ascending order, of the sum of the blocks (I, K) of A_l with K
// in aggregate L in ascending K -- the row-by-row product's order, so the result is that
// product's bit for bit.  One term per block of A_l, grouped by the coarse block it feeds.
struct NodeGal {
    int32_t* tptr = nullptr;  // per coarse block (+1): its first term
    int32_t* toff = nullptr;  // per term: index of the fine block's (0, 0) value
    int32_t* tlen = nullptr;  // per term: 2 * the fine rows' length, + 1 when it starts a new fine node
    int32_t* cout = nullptr;  // per coarse block: index of its (0, 0) value
    int32_t* clen = nullptr;  // per coarse block: the coarse rows' length
    int64_t nblk = 0;         // coarse blocks (0: no plan, the scalar product runs)
    int64_t nterm = 0;
    bool complete = false;    // every block of A_l is some term's (the product can ingest values)
};

struct Level {
    Csr A;       // A_l
    Csr P, R;    // P_l and R_l = P_l^T (empty on the coarsest level)
    Csr AP;      // cached pattern (and values) of A_l P_l, the first Galerkin factor
    int32_t* agg = nullptr;      // aggregate of each row (setup product, kept for export)
    // block systems: node pattern of A_l (node row pointers, node columns), read by the
    // node-group kernels in place of A_l's own index arrays
    int32_t* nptr = nullptr;
    int32_t* ncol = nullptr;
    bool node_pairs = true;      // node-group kernels take two adjacent positions per lane (even B)
    NodeGal ngal;                // block systems: node Galerkin plan of A_{l+1} = R_l A_l P_l
    // block systems whose P_l is P_node (x) I_B with unit values: the aggregate of every
    // node (-1: none), for the node prolongation (null: the CSR prolongation runs)
    int32_t* nagg = nullptr;
    uint8_t* strong = nullptr;   // strength flag per stored entry of A_l
    double* m = nullptr;         // smoother diagonal
    float* m32 = nullptr;
    // V-cycle work vectors in the hierarchy precision
    void* u = nullptr;
    void* f = nullptr;
    void* r = nullptr;
    void* t = nullptr;
    // Galerkin kernels: lane-group widths (A_l P_l rows; A_{l+1} rows) and the gathered
    // kernel's shapes for A_l P_l and R_l (A_l P_l)
    int gAP = 8, gRAP = 32;
    GalShape galAP, galRAP;
    template <typename T>
    T* mv() const;
};
template <>
inline double* Level::mv<double>() const { return m; }
template <>
inline float* Level::mv<float>() const { return m32; }

// Device scalar slots.
enum Scal {
    S_RHO = 0,    // r.z of the current iteration
    S_PQ = 1,     // p.Ap
    S_FLAG = 2,   // 1: CG breakdown
    S_COARSE = 3, // coarse factorisation status: 0 ok, 1 not SPD
    S_BETA = 4,
    S_ALPHA = 5,
    S_RHO_USED = 6,  // the rho of the current iteration's alpha (beta's denominator)
    S_ASYM = 7,      // diagonal storage: 0 when the last refreshed values are symmetric
    S_COUNT = 8
};

// Reductions store one partial per block into a region; the consumer adds them in block
// order.  Every region holds up to `cap` partials (full grids of the level-0 kernels;
// bounded grids use at most RED_BLOCKS <= cap); P_RR and P_FF sit right after the scalars
// so the host reads them, and the scalars, with one copy.
enum PartRegion { P_RZ = 0, P_RZOLD = 1, P_PQ = 2, P_RR = 3, P_FF = 4 };
constexpr int RED_BLOCKS = 1024;

struct RedScratch {
    // [P_RZ cap][P_RZOLD cap][P_PQ cap][scalars S_COUNT][P_RR cap][P_FF cap]: the scalars
    // and the ||r||^2 and ||f||^2 partials are adjacent, so one copy brings them to the host
    double* part = nullptr;
    int cap = 0;
    // device address of the host mirror (mapped, coherent pinned memory): the CG update
    // kernels write their ||r||^2 partials and the breakdown flag there directly
    double* host = nullptr;
    __host__ __device__ double* region(int k) const {
        if (k <= P_PQ) return part + (size_t)k * cap;
        if (k == P_RR) return part + 3 * (size_t)cap + S_COUNT;
        return part + 4 * (size_t)cap + S_COUNT;
    }
    __host__ __device__ double* scal() const { return part + 3 * (size_t)cap; }
    static size_t doubles(int cap) { return 5 * (size_t)cap + S_COUNT; }
    // the host mirror of [scalars, P_RR, P_FF]
    static size_t host_doubles(int cap) { return S_COUNT + 2 * (size_t)cap; }
};

// Row-block kernels: RB_THREADS threads, at most RB_CAP nonzeros staged in LDS per block.
constexpr int RB_THREADS = 256;
constexpr int RB_CAP = 2048;
constexpr int RB_MIN_BLOCKS = 1024;

int lane_group(double avg_per_row);  // power of two in [2, 64]
int pick_rows_per_block(const int32_t* host_ptr, int32_t nrows);  // 0: no row blocking
int red_grid_rows(int nrows, int rpb, int g);
int full_grid_rows(int nrows, int rpb, int g);
int red_grid_elems(int64_t n);

// ------------------------------------------------------------------ solve kernels
template <typename T>
void launch_spmv(const Csr& A, const T* x, T* y, const T* m2, T* y2, hipStream_t s);
template <typename T>
void launch_residual(const Csr& A, const T* f, const T* u, T* r, hipStream_t s);
template <typename T>
void launch_jacobi(const Csr& A, const T* m, const T* f, const T* u, T* uout, hipStream_t s);
template <typename T>
void launch_smooth0_residual(const Csr& A, const T* m, const T* f, T* u, T* r, hipStream_t s);
template <typename T>
void launch_prolong_add(const Csr& P, const T* uc, T* u, hipStream_t s);
// Diagonal storage of the finest operator when its pattern has few distinct column
// offsets (a stencil): entry (i, i + off[d]) at val[d * n + i], absent entries 0.  The
// level-0 solve kernels stream it without any index arrays.
constexpr int DIA_MAX = 32;
struct DiaOff {
    int off[DIA_MAX];
    // 1: the values are symmetric, so the solve kernels read each sub-diagonal entry
    // A(i, j) as the super-diagonal entry A(j, i) and never touch the lower diagonals
    int sym;
};
// Windowed form of the diagonal-storage kernels: the offsets fall into at most
// WIN_MAX_CL clusters (a stencil's planes); a workgroup of TPB rows stages, per cluster,
// the vector entries of rows [i0 + lo, i0 + TPB + lo + span) in LDS.
constexpr int WIN_MAX_CL = 4;
constexpr int WIN_CAP = 4096;   // LDS entries per workgroup (all windows)
struct WinPlan {
    int ncl = 0;                // 0: not used
    int lo[WIN_MAX_CL] = {0, 0, 0, 0};    // smallest offset of the cluster
    int len[WIN_MAX_CL] = {0, 0, 0, 0};   // window length: TPB + span of the cluster
    int base[WIN_MAX_CL] = {0, 0, 0, 0};  // start of the window in LDS
    int total = 0;                        // LDS entries of all windows
    bool all = false;                     // also the V-cycle kernels (else the Krylov SpMV only)
    bool two = false;                     // two rows per thread fit (27 diagonals)
    unsigned char cl[DIA_MAX] = {};       // cluster of each diagonal
};
struct Dia {
    int ndiag = 0;              // 0: not used
    DiaOff off{};
    bool symoff = false;        // the offsets are -k..k-symmetric and include 0
    // 7-point marching kernels: offsets -a, -b, -1, 0, 1, b, a; march_a == 0: not used
    int march_a = 0, march_b = 0;
    WinPlan win;                // windowed kernels for other stencils (ncl == 0: not used)
    double* val = nullptr;      // FP64 values (Krylov operator and FP64 V-cycle)
    float* val32 = nullptr;     // FP32 values (mixed-precision V-cycle)
    uint8_t* slot = nullptr;    // diagonal of every stored entry of A_0
    template <typename T>
    const T* v() const;
};
template <>
inline const double* Dia::v<double>() const { return val; }
template <>
inline const float* Dia::v<float>() const { return val32; }

// Start and stop events that the next launch of a timed kernel (the Krylov SpMV) records
// itself, set by the host's kernel trace and cleared by the launch.
struct KernelEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local KernelEvents g_kernel_events;

// Launches kernel k; when the host's trace asked for this kernel's own timing, the launch
// records its start and stop events itself (hipExtLaunchKernel), so that they bracket the
// kernel's execution and not the dispatch gap before it.
template <typename F, typename... Args>
void timed_launch(F k, unsigned grid, unsigned block, unsigned shmem, hipStream_t s, Args... args) {
    if (g_kernel_events.start != nullptr) {
        const KernelEvents e = g_kernel_events;
        g_kernel_events = KernelEvents{};
        hipExtLaunchKernelGGL(k, dim3(grid), dim3(block), shmem, s, e.start, e.stop, 0, args...);
    } else {
        hipLaunchKernelGGL(k, dim3(grid), dim3(block), shmem, s, args...);
    }
}

std::vector<int> dia_offsets(const Csr& A, hipStream_t s);
// Two-byte column indices of A for its row blocks (A.rpb > 0): writes cblk (one base per
// block) and sets *wide when a block's columns span more than 65535; then c16.
void launch_c16_bases(const Csr& A, int32_t* cblk, int* wide, hipStream_t s);
void launch_c16_fill(const Csr& A, const int32_t* cblk, uint16_t* c16, hipStream_t s);

// Workgroups of the 7-point marching kernels for n rows with plane stride a.
int march_blocks(int n, int a);
// Window plan for the sorted offsets (clusters split at gaps wider than a workgroup), or
// ncl = 0 when they need more clusters or LDS than the windowed kernels have.
WinPlan win_plan(const std::vector<int>& offs);

// BiCGStab vector kernels (kernels_krylov.hip).  Partials: part[q * nb + workgroup].
// The step's scalars live on the device (BiScal slots, formed by launch_bi_scal from the
// partials of the kernel before), so a step runs with one host round trip: the update
// copies the slots and the r.r partials to the host mirror (host[0..nb) partials,
// host[2 RED_BLOCKS + k] slot k).
enum BiScal { BS_RHO = 0, BS_ALPHA = 1, BS_OMEGA = 2, BS_BETA = 3, BS_HALF = 4, BS_BAD = 5, BS_COUNT = 8 };
// launch_bi_scal stages: RESET (rho = value, alpha = omega = 1, flags cleared); BETA (from
// the r^.r partials: beta, then rho); ALPHA (from r^.v: alpha = rho / r^.v); HALF (from s.s:
// the half step has converged when ||s|| <= tol); OMEGA (from t.s and t.t: omega)
enum BiStage { BI_RESET = 0, BI_BETA = 1, BI_ALPHA = 2, BI_HALF = 3, BI_OMEGA = 4 };
// BS_BAD bits: a zero or non-finite r^.r, r^.v, t.t or omega
enum BiBad { BI_BAD_RHO = 1, BI_BAD_RV = 2, BI_BAD_TT = 4, BI_BAD_OMEGA = 8 };
int bi_grid(int64_t n);
void launch_bi_residual(int64_t n, const double* f, const double* y, double* r, double* part, int nb, hipStream_t s);
void launch_bi_dots(int64_t n, const double* a, const double* b, const double* c, const double* d, double* part,
                    int nb, hipStream_t s);
void launch_bi_scal(int stage, double* sc, const double* part, int nb, double value, double tol, hipStream_t s);
void launch_bi_direction(int64_t n, const double* r, const double* v, const double* sc, int first, double* p,
                         hipStream_t s);
void launch_bi_half(int64_t n, const double* r, const double* v, const double* sc, double* sv, double* part, int nb,
                    hipStream_t s);
void launch_bi_update(int64_t n, const double* ph, const double* sh, const double* sv, const double* t,
                      const double* rh, const double* sc, double* x, double* r, double* rho_part, double* host, int nb,
                      hipStream_t s);
void launch_dia_slots(const Csr& A, const Dia& D, hipStream_t s);
template <typename T>
void launch_dia_scatter(const Csr& A, const Dia& D, const double* val, T* dval, hipStream_t s);
// scal[S_ASYM] = 0 when every stored sub-diagonal entry equals its mirror (bit for bit), 1
// otherwise; needs D.symoff and the FP64 values just scattered.
template <typename T>
void launch_dia_gather(const Csr& A, const Dia& D, const T* dval, T* val, hipStream_t s);
void launch_dia_symcheck(int n, const Dia& D, double* scal, hipStream_t s);
template <typename T>
void launch_dia_smooth0_residual(int n, const Dia& D, const T* m, const T* f, T* u, T* r, hipStream_t s);
template <typename T>
void launch_dia_residual(int n, const Dia& D, const T* f, const T* u, T* r, hipStream_t s);
template <typename T>
void launch_dia_jacobi(int n, const Dia& D, const T* m, const T* f, const T* u, T* uout, hipStream_t s);
int launch_dia_update_smooth0(int n, const Dia& D, const double* p, const double* q, double* x, const double* r,
                              double* rn, const double* m, double* u, double* rv, const RedScratch& rs,
                              hipStream_t s);
int launch_cg_update_cast(int n, const double* p, const double* q, double* x, double* r, float* r32,
                          const RedScratch& rs, hipStream_t s);
int launch_dia_cg_init(int n, const Dia& D, const double* f, const double* x, double* r, const RedScratch& rs,
                       hipStream_t s);
int launch_dia_jacobi_rz(int n, const Dia& D, const double* m, const double* r, const double* u, double* z,
                         int flexible, const RedScratch& rs, hipStream_t s);
// Mixed precision: the last FP32 sweep u + M (f - A u) written to z in FP64, with the r.z
// partials of the FP64 residual r; returns the partial count, or 0 when D has no marching
// or windowed form for it (nothing launched).
int launch_dia_jacobi_rz32(int n, const Dia& D, const float* m, const float* f, const float* u, const double* r,
                           double* z, int flexible, const RedScratch& rs, hipStream_t s);
int launch_dia_cg_pq(int n, const Dia& D, const double* z, const double* pold, double* pnew, double* q, int first,
                     const RedScratch& rs, hipStream_t s);

// The coarse tail of the V-cycle: the restriction into level t, then Algorithm 2 on levels
// t .. L (the last one solved with the dense inverse) in one workgroup, writing u_t.
constexpr int TAIL_MAX_LEVELS = 6;
constexpr int TAIL_MAX_ROWS = 2048;        // rows of all tail levels together
constexpr int64_t TAIL_MAX_NNZ = 16384;    // stored entries the tail reads (A, P, R and R_{t-1})
constexpr int TAIL_SOLO_ROWS = 64;         // largest coarsest level that a tail may hold alone
constexpr size_t TAIL_SMEM_MAX = 3 * TAIL_MAX_ROWS * sizeof(double);
template <typename T>
struct TailLevel {
    int n = 0;
    int soff = 0;               // LDS offset (elements) of the level's f, u, w vectors
    const int* Aptr = nullptr;
    const int* Acol = nullptr;
    const T* Aval = nullptr;
    const T* m = nullptr;
    const int* Rptr = nullptr;  // R_l and P_l: empty on the coarsest tail level
    const int* Rcol = nullptr;
    const T* Rval = nullptr;
    const int* Pptr = nullptr;
    const int* Pcol = nullptr;
    const T* Pval = nullptr;
};
template <typename T>
struct TailArgs {
    int nlev = 0;
    int npre = 1, npost = 1;
    int bs = 1;                    // unknowns per node: > 1 smooths with B x B blocks (m: B per row)
    const int* rin_ptr = nullptr;  // R_{t-1} and r_{t-1}
    const int* rin_col = nullptr;
    const T* rin_val = nullptr;
    const T* rin = nullptr;
    T* uout = nullptr;             // u_t
    const double* cinv = nullptr;  // dense inverse of the coarsest operator
    TailLevel<T> lv[TAIL_MAX_LEVELS];
};
template <typename T>
void launch_vcycle_tail(const TailArgs<T>& a, hipStream_t s);

template <typename T>
void launch_coarse_gemv(int n, const double* inv, const T* f, T* u, const double* bad, hipStream_t s);
void launch_cast_d2f(int64_t n, const double* a, float* b, hipStream_t s);
void launch_cast_f2d(int64_t n, const float* a, double* b, hipStream_t s);
void launch_copy(int64_t n, const double* a, double* b, hipStream_t s);

// CG pieces (FP64); each reducing launcher returns the number of partials it wrote.
int launch_cg_init(const Csr& A, const double* val, const double* f, const double* x, double* r,
                   const RedScratch& rs, hipStream_t s);
int launch_jacobi_rz(const Csr& A, const double* m, const double* r, const double* u, double* z, int flexible,
                     const RedScratch& rs, hipStream_t s);
int launch_cast_rz(int n, const float* z32, const double* r, double* z, int flexible, const RedScratch& rs,
                   hipStream_t s);
int launch_cg_rz(int n, const double* r, const double* z, const RedScratch& rs, hipStream_t s);
void launch_fin_rz(int nb, int flexible, int first, const RedScratch& rs, hipStream_t s);
void launch_fin_pq(int nb, const RedScratch& rs, hipStream_t s);
int launch_cg_pq(const Csr& A, const double* val, const double* z, const double* pold, double* pnew, double* q,
                 int first, const RedScratch& rs, hipStream_t s);
int launch_cg_update(int n, const double* p, const double* q, double* x, double* r, const RedScratch& rs,
                     hipStream_t s);

// ------------------------------------------------------------------ Galerkin / smoother
template <typename T>
void launch_smoother_diag(const Csr& A, int kind, double omega, T* m, hipStream_t s);
template <typename T>
bool launch_galerkin_ap(const Csr& A, const Csr& P, const Csr& AP, int g, GalShape gs, int kind, double omega, T* m,
                        const double* ain, hipStream_t s, const Dia* dia = nullptr);
template <typename T>
void launch_galerkin_rap(const Csr& R, const Csr& AP, const Csr& Ac, int g, GalShape gs, hipStream_t s);
GalShape pick_galerkin_shape(int32_t nrows, int64_t nnzL, int64_t terms, int maxlen_c, int gforce, int tforce);
// count_galerkin_terms writes the term offsets gs.off (nrows + 1) and returns the number
// of terms (and the most in one row); build_galerkin_posmap fills gs.pos, gs.bst, gs.tof
// and, if allocated, gs.dpos (all allocated by the caller in between).
int64_t count_galerkin_terms(const Csr& L, const Csr& B, int64_t* off, int64_t* max_row, hipStream_t s);
bool galerkin_terms_fit(int64_t max_row);
void build_galerkin_posmap(const Csr& L, const Csr& B, const Csr& C, const GalShape& gs, hipStream_t s);

// ------------------------------------------------------------------ setup
// flags: device int[8], see SetupFlag.
enum SetupFlag {
    F_ARG = 0,
    F_PATTERN = 1,
    F_NOT_SPD = 2,
    F_UNDECIDED = 3,
    F_NOAGG = 4,
    F_BLOCK = 5,
    F_NODEGAL = 6,   // block system: P_l is not P_node (x) I_B with unit values (no node Galerkin plan)
    F_NODEPART = 7,  // block system: some node belongs to no aggregate
    F_COUNT = 8
};

void launch_validate(const Csr& A, int32_t* diag_pos, int* flags, hipStream_t s);
void launch_strength(const Csr& A, const int32_t* diag_pos, double eps2, uint8_t* strong, int32_t* tpos,
                     uint8_t* isolated, int* flags, hipStream_t s);
// distance-2 maximal independent set; returns the number of roots (host sync per round)
void run_mis2(const Csr& A, const uint8_t* strong, const uint8_t* isolated, uint8_t* state, int* flags,
              int* h_flags, hipStream_t s);
int32_t run_aggregate(const Csr& A, const uint8_t* strong, const int32_t* tpos, const uint8_t* state,
                      int32_t* agg, int* flags, int* h_flags, hipStream_t s);
void build_prolongator(const Csr& A, const uint8_t* strong, const int32_t* diag_pos, const int32_t* agg,
                       int32_t nc, int plain, Csr& P, hipStream_t s);
void build_transpose(const Csr& P, Csr& R, hipStream_t s);
void symbolic_spgemm(const Csr& A, const Csr& B, Csr& C, hipStream_t s);
void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s);
// Systems with B unknowns per node (unknown b of node I is row I*B + b): the node matrix
// of block Frobenius norms (its arrays are dnew allocations of the caller; for a pattern
// without values, its pattern only), and the expansion of node aggregates and strength
// flags to the unknowns.
void build_node_matrix(const Csr& A, int B, Csr& Nm, int* flags, int* h_flags, hipStream_t s);
template <typename T>
void launch_block_inv(const Level& L, int B, double omega, T* m, int* flags, hipStream_t s);
template <typename T>
void launch_block_apply(int n, int B, const T* m, const T* r, const T* uin, T* uout, hipStream_t s);
// Node-group products on level L of a block system (L.nptr, L.ncol: its node pattern).
// node_grid(nn): workgroups that give every node group its own (the reduction scratch is
// sized for it, so the Krylov product runs without a grid-stride second pass).
int node_grid(int nn);
template <typename T>
void launch_node_residual(const Level& L, int B, const T* f, const T* u, T* r, hipStream_t s);
template <typename T>
void launch_node_sweep(const Level& L, int B, const T* m, const T* f, const T* uin, T* uout, hipStream_t s);
int launch_node_cg_pq(const Level& L, int B, const double* val, const double* z, const double* pold, double* pnew,
                      double* q, int first, const RedScratch& rs, hipStream_t s);
// z = uin + M (r - A uin) on level 0 with the r.z partials; returns their count.
int launch_node_sweep_rz(const Level& L, int B, const double* m, const double* r, const double* uin, double* z,
                         const RedScratch& rs, hipStream_t s);
void launch_node_expand(const Csr& A, int B, const Csr& Nm, const uint8_t* nstrong, const int32_t* nagg,
                        uint8_t* strong, int32_t* agg, hipStream_t s);
// Node Galerkin plan of levels L -> N (block size B; N's node pattern built): the aggregate
// of every fine node from P (flags[F_NODEGAL] when P is not of the unit Kronecker form,
// flags[F_NODEPART] for a node outside every aggregate), then per coarse node the terms'
// coarse positions (tpos per block of A_l) and counts (cnt per coarse block), then, with
// g.tptr formed from the counts, the terms themselves (cur, last: scratch per coarse block).
void launch_node_gal_agg(const Csr& P, int B, int32_t* nagg, int* flags, hipStream_t s);
void launch_node_gal_count(const Level& L, const Level& N, int B, const int32_t* nagg, int32_t* tpos, int32_t* cnt,
                           int* flags, hipStream_t s);
void launch_node_gal_fill(const Level& L, const Level& N, int B, const int32_t* tpos, const NodeGal& g, int32_t* cur,
                          int32_t* last, hipStream_t s);
// Prolongation of a block system with P_l = P_node (x) I_B (L.nagg set): u_l += P_l uc,
// one thread per fine row.
template <typename T>
void launch_node_prolong(const Level& L, int B, const T* uc, T* u, hipStream_t s);
// A_{l+1} = R_l A_l P_l by the node plan: the values of A_l from aval, or, with lin, from
// the caller's FP64 array, stored into a64 (and a32 when given) as they are read.
template <typename T>
void launch_node_rap(const NodeGal& g, int B, const T* aval, const double* lin, double* a64, float* a32, T* cval,
                     hipStream_t s);
void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s);
int64_t max_i64(const int64_t* in, int64_t n, hipStream_t s);  // synchronises

// ------------------------------------------------------------------ coarse solve
constexpr int COARSE_LDS_MAX = 128;      // dense FP64 inverse held in one workgroup's LDS
constexpr int COARSE_GLOBAL_MAX = 2048;  // larger coarsest levels: blocked, many workgroups
constexpr size_t COARSE_WORK_DOUBLES = 2 * 64 * 64;  // scratch of the blocked inverse
template <typename T>
void launch_densify(const Csr& A, double* D, hipStream_t s);
// In-place inverse of the dense n x n coarsest operator (Gauss-Jordan, positive pivots;
// scal[S_COARSE] = 1 when one is not).  work: COARSE_WORK_DOUBLES doubles, needed when
// n > COARSE_LDS_MAX.
void launch_dense_inverse(int n, double* D, double* scal, double* work, hipStream_t s);

// ------------------------------------------------------------------ differentiable form
void launch_logcoef7_assemble(int nx, int ny, int nz, const double* theta, double* val, hipStream_t s);
void launch_logcoef7_adjoint(int nx, int ny, int nz, const double* theta, const double* u, const double* lam,
                             double* grad, hipStream_t s);

// XCD-aware block index: hardware dispatches workgroups round-robin over the 8 XCDs;
// this gives every XCD a contiguous range of logical blocks so that neighbouring rows
// (and the vector entries they gather) share one L2.
__device__ inline int xcd_block() {
    const int b = blockIdx.x, nb = gridDim.x;
    const int per = nb >> 3, rem = nb & 7;
    const int x = b & 7, i = b >> 3;
    return x * per + (x < rem ? x : rem) + i;
}

}  // namespace amgmi

struct amg_ctx {
    amg_params prm{};
    hipStream_t stream = nullptr;
    std::vector<amgmi::Level> lv;
    // Krylov operator values (pattern of lv[0].A).  Aliases lv[0].A.val until full reuse
    // (Algorithm 3) gives the Krylov solver newer values than the hierarchy.
    double* outer_val = nullptr;
    double* outer_own = nullptr;
    int32_t nL = 0;
    int tail = 0;                 // first level of the fused coarse tail (0: none)
    amgmi::Dia dia;               // diagonal storage of A_0 (ndiag 0: CSR kernels)
    double* cinv = nullptr;       // dense inverse of the coarsest operator (FP64)
    double* cwork = nullptr;      // scratch of its blocked inverse (more than COARSE_LDS_MAX rows)
    // CG state
    double *x = nullptr, *r = nullptr, *r2 = nullptr, *z = nullptr, *zold = nullptr, *pa = nullptr, *pb = nullptr,
           *q = nullptr;
    amgmi::RedScratch rs{};
    double* h_red = nullptr;      // pinned host mirror of the scalars and the P_RR, P_FF partials
    // BiCGStab: one more vector (the hierarchy's) and mapped host memory for its partials
    double* bi_t = nullptr;
    double* bi_sc = nullptr;      // BiCGStab's device scalars (BS_COUNT)
    double* bi_part = nullptr;    // its device partials (6 regions of RED_BLOCKS)
    double* bi_w = nullptr;       // the p copy the diagonal-storage SpMV writes (unused here)
    double* h_bi = nullptr;
    double* d_bi = nullptr;
    int* d_flags = nullptr;       // setup flags
    int* h_flags = nullptr;       // pinned
    // pending pattern for amg_rebuild(..., pattern_changed)
    int32_t pend_n = 0;
    int64_t pend_nnz = 0;
    int32_t* pend_ptr = nullptr;
    int32_t* pend_col = nullptr;
    bool transfer_given = false;
    // rebuild-policy history: updates since the last full setup, iterations of the first
    // solve after it (0: not yet), the last solve's iterations and convergence
    int pol_updates = 0, pol_iters_ref = 0, pol_last_iters = 0, pol_last_conv = 0;
    // allocations: the hierarchy (released by a full rebuild) and the context's own
    std::vector<void*> hier_allocs;
    std::vector<void*> own_allocs;
    amgmi::DevMem mem;            // where the device memory of this context comes from
    int device = 0;               // the device current at amg_setup
    // phase times of the last setup / rebuild (Table 1 breakdown)
    double phase_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    bool phase_pending = false;   // partial rebuild: times still to be read from ev[]
    hipEvent_t ev[4]{};
    hipEvent_t ev_read = nullptr;  // completion of the per-iteration scalar read
    // The blocked inverse of the coarsest operator (more than COARSE_LDS_MAX rows) of a
    // partial update runs on a stream of the context's own (side, default priority),
    // ordered after the update's Galerkin products by ev_fork, so that it overlaps the
    // start of the next solve; every use of the inverse, or of its pivot flag, on the
    // context's stream first waits for ev_inv (wait_coarse).
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_inv = nullptr;
    bool cinv_pending = false;
    // per-kernel tracing (amg_trace): every trace_every-th launch of a traced class on a
    // level is bracketed (trace_seen counts them per class and level, levels above 63 as 63)
    unsigned trace_mask = 0;
    int trace_level = -1;
    int trace_every = 1;
    std::array<std::array<int64_t, 64>, 16> trace_seen{};
    std::vector<hipEvent_t> ev_pool;
    struct Traced {
        int cls;
        int level;
        hipEvent_t a, b;
    };
    std::vector<Traced> traced;
    // set while a full setup or a pattern change replaces the hierarchy: a failure then
    // leaves the context unusable (broken)
    bool replacing = false;
    // the partial update wrote A_0's new values straight into the diagonal storage: the CSR
    // value arrays of level 0 are formed from it when they are read (exports)
    bool a0_csr_stale = false;
    // block systems: the node Galerkin plans are built by the first partial update after a
    // setup or a pattern change (a series of full setups never needs them)
    bool ngal_ready = false;
    // mixed precision: the last level-0 sweep writes z in FP64 with r.z (off with
    // AMGMI_NO_RZ32: a separate widening pass)
    bool rz32 = true;
    bool broken = false;
    std::string err;
};
