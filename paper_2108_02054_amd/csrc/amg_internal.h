// amg_internal.h -- hierarchy layout and kernel launchers of the gfx950 AMG library.
//
// Everything lives in device memory for the lifetime of a context; nothing is moved
// between host and device after setup except a few scalars per CG iteration.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
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
void* dalloc(size_t bytes, hipStream_t s);
void dfree(void* p, hipStream_t s);

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
    template <typename T>
    T* v() const;
};
template <>
inline double* Csr::v<double>() const { return val; }
template <>
inline float* Csr::v<float>() const { return val32; }

struct Level {
    Csr A;       // A_l
    Csr P, R;    // P_l and R_l = P_l^T (empty on the coarsest level)
    Csr AP;      // cached pattern (and values) of A_l P_l, the first Galerkin factor
    int32_t* agg = nullptr;      // aggregate of each row (setup product, kept for export)
    uint8_t* strong = nullptr;   // strength flag per stored entry of A_l
    double* m = nullptr;         // smoother diagonal
    float* m32 = nullptr;
    // V-cycle work vectors in the hierarchy precision
    void* u = nullptr;
    void* f = nullptr;
    void* r = nullptr;
    void* t = nullptr;
    // lane-group widths of the row kernels
    int gA = 8, gP = 4, gR = 32, gAP = 8, gRAP = 32;
    template <typename T>
    T* mv() const;
};
template <>
inline double* Level::mv<double>() const { return m; }
template <>
inline float* Level::mv<float>() const { return m32; }

// Device scalar slots used by the CG kernels.
enum Scal {
    S_FF = 0,     // ||f||^2
    S_RR = 1,     // ||r||^2
    S_RHO = 2,    // r.z
    S_PQ = 3,     // p.Ap
    S_BETA = 4,
    S_FLAG = 5,   // 1: breakdown
    S_RZOLD = 6,  // r.z_old (flexible CG)
    S_COARSE = 7, // coarse factorisation status: 0 ok, 1 not SPD
    S_COUNT = 8
};

// Reductions run on a fixed grid so that every partial sum, and therefore the result,
// is independent of scheduling: the last block to finish adds the partials in order.
constexpr int RED_BLOCKS = 2048;
constexpr int RED_THREADS = 256;
constexpr int RED_MAXK = 2;

int lane_group(double avg_per_row);  // power of two in [2, 64]

// ------------------------------------------------------------------ solve kernels
struct RedScratch {
    double* part;      // RED_MAXK * RED_BLOCKS
    unsigned* ticket;  // one counter
    double* scal;      // S_COUNT device scalars
};

template <typename T>
void launch_spmv(const Csr& A, int g, const T* x, T* y, hipStream_t s);
template <typename T>
void launch_residual(const Csr& A, int g, const T* f, const T* u, T* r, hipStream_t s);
template <typename T>
void launch_jacobi(const Csr& A, int g, const T* m, const T* f, const T* u, T* uout, hipStream_t s);
template <typename T>
void launch_smooth0_residual(const Csr& A, int g, const T* m, const T* f, T* u, T* r, hipStream_t s);
template <typename T>
void launch_prolong_add(const Csr& P, int g, const T* uc, T* u, hipStream_t s);
template <typename T>
void launch_coarse_gemv(int n, const double* inv, const T* f, T* u, hipStream_t s);
void launch_cast_d2f(int64_t n, const double* a, float* b, hipStream_t s);
void launch_cast_f2d(int64_t n, const float* a, double* b, hipStream_t s);
void launch_copy(int64_t n, const double* a, double* b, hipStream_t s);

// CG pieces (FP64).  See amg_api.hip for the iteration they form.
void launch_cg_init(const Csr& A, const double* outer_val, int g, const double* f, const double* x,
                    double* r, const RedScratch& rs, hipStream_t s);
void launch_cg_rz(int n, const double* r, const double* z, const double* zold, int flexible, int first,
                  const RedScratch& rs, hipStream_t s);
void launch_cg_pq(const Csr& A, const double* outer_val, int g, const double* z, const double* pold,
                  double* pnew, double* q, int first, const RedScratch& rs, hipStream_t s);
void launch_cg_update(int n, const double* p, const double* q, double* x, double* r, const RedScratch& rs,
                      hipStream_t s);

// ------------------------------------------------------------------ Galerkin / smoother
template <typename T>
void launch_smoother_diag(const Csr& A, int kind, double omega, T* m, hipStream_t s);
template <typename T>
void launch_galerkin_ap(const Csr& A, const Csr& P, const Csr& AP, int g, hipStream_t s);
template <typename T>
void launch_galerkin_rap(const Csr& R, const Csr& AP, const Csr& Ac, int g, hipStream_t s);

// ------------------------------------------------------------------ setup
// flags: device int[8], see SetupFlag.
enum SetupFlag { F_ARG = 0, F_PATTERN = 1, F_NOT_SPD = 2, F_UNDECIDED = 3, F_NOAGG = 4, F_COUNT = 8 };

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

// ------------------------------------------------------------------ coarse solve
constexpr int COARSE_LDS_MAX = 128;      // dense FP64 inverse held in one workgroup's LDS
constexpr int COARSE_GLOBAL_MAX = 8192;  // larger coarsest levels work in global memory
template <typename T>
void launch_densify(const Csr& A, double* D, hipStream_t s);
void launch_dense_inverse(int n, double* D, double* scal, hipStream_t s);

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
    double* cinv = nullptr;       // dense inverse of the coarsest operator (FP64)
    // CG state
    double *x = nullptr, *r = nullptr, *z = nullptr, *zold = nullptr, *pa = nullptr, *pb = nullptr,
           *q = nullptr;
    amgmi::RedScratch rs{};
    double* h_scal = nullptr;     // pinned host copy of the scalar slots
    int* d_flags = nullptr;       // setup flags
    int* h_flags = nullptr;       // pinned
    // pending pattern for amg_rebuild(..., pattern_changed)
    int32_t pend_n = 0;
    int64_t pend_nnz = 0;
    int32_t* pend_ptr = nullptr;
    int32_t* pend_col = nullptr;
    bool transfer_given = false;
    // allocations: the hierarchy (released by a full rebuild) and the context's own
    std::vector<void*> hier_allocs;
    std::vector<void*> own_allocs;
    // phase times of the last setup / rebuild (Table 1 breakdown)
    double phase_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    bool phase_pending = false;   // partial rebuild: times still to be read from ev[]
    hipEvent_t ev[4]{};
    // per-kernel tracing (amg_trace)
    unsigned trace_mask = 0;
    int trace_level = -1;
    std::vector<hipEvent_t> ev_pool;
    struct Traced {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<Traced> traced;
    bool broken = false;
    std::string err;
};
