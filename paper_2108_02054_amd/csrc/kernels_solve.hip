// kernels_solve.hip -- V-cycle (Algorithm 2) and preconditioned-CG kernels for gfx950.
//
// Every kernel here is bandwidth bound (about 0.17 flop per byte).  The main form is the
// row-block kernel: a workgroup owns `rpb` consecutive rows whose nonzeros (at most
// RB_CAP, chosen per matrix at setup) are streamed with fully coalesced loads, multiplied
// by the gathered vector entries and staged in LDS; one thread per row then adds its
// row's products in column order and applies the kernel's epilogue.  Rows too long to
// stage fall back to lane-group kernels (G lanes per row, cross-lane butterfly sums).
//
// Reductions never use fences or atomics (an agent-scope fence writes back and
// invalidates the per-XCD L2 caches): each block stores one partial sum into a fixed slot
// and the consumer -- the next kernel, or the host -- adds the slots in block order.  The
// number of blocks is a fixed function of the size, so every result is bitwise
// reproducible.
#include <algorithm>
#include <climits>
#include <vector>

#include <type_traits>

#include <hip/hip_ext.h>

#include "amg_internal.h"

namespace amgmi {

constexpr int TPB = 256;
static_assert(RB_THREADS == TPB, "row-block kernels use one thread per staged row");

template <int G, typename T>
__device__ __forceinline__ T group_sum(T s) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
    return s;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T s) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}

#define AMG_WITH_G(g, ...)                                                  \
    do {                                                                    \
        switch (g) {                                                        \
            case 2: { constexpr int G = 2; __VA_ARGS__; } break;            \
            case 4: { constexpr int G = 4; __VA_ARGS__; } break;            \
            case 8: { constexpr int G = 8; __VA_ARGS__; } break;            \
            case 16: { constexpr int G = 16; __VA_ARGS__; } break;          \
            case 32: { constexpr int G = 32; __VA_ARGS__; } break;          \
            case 64: { constexpr int G = 64; __VA_ARGS__; } break;          \
            default: throw Fail{AMG_ERR_ARG, "unsupported lane group"};     \
        }                                                                   \
    } while (0)

thread_local KernelEvents g_kernel_events;

static inline unsigned grid_for(int64_t items, int per_block) {
    int64_t b = (items + per_block - 1) / per_block;
    return (unsigned)(b > 0 ? b : 1);
}

// ------------------------------------------------------------------ row-block staging

// One staging pass group: U strided entries per thread.  Every column and value load is
// issued before the first gather and every gather before the first product, so a thread
// keeps U loads of each kind in flight instead of walking its entries one round trip at a
// time.  Indices past the block's range are clamped to its last entry (in bounds, their
// products dropped).
template <int U, typename T, class C, class X>
__device__ __forceinline__ void rb_stage(int k0, int k1, C colat, const T* __restrict__ val, X xget, T* sp) {
    int jj[U];
    T vv[U], xx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int k = min(k0 + u * RB_THREADS + (int)threadIdx.x, k1 - 1);
        jj[u] = colat(k);
        vv[u] = val[k];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) xx[u] = xget(jj[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int k = k0 + u * RB_THREADS + (int)threadIdx.x;
        if (k < k1) sp[k - k0] = vv[u] * xx[u];
    }
}

// Loads ptr[row0 .. row1] into sptr and val[k] * xget(col(k)) for the block's nonzeros into
// sp.  The block's entry range comes from two uniform loads of ptr, so the entry loads do
// not wait for the pointer stage; one barrier at the end publishes both.  Every thread of
// the block must call it.
template <typename T, class C, class X>
__device__ __forceinline__ void rb_load_core(int row0, int row1, const int* __restrict__ ptr, C colat,
                                             const T* __restrict__ val, X xget, int* sptr, T* sp) {
    const int nr = row1 - row0;
    for (int i = threadIdx.x; i <= nr; i += RB_THREADS) sptr[i] = ptr[row0 + i];
    const int k0 = ptr[row0];
    const int k1 = min(ptr[row1], k0 + RB_CAP);  // blocks are sized within RB_CAP
    // as many load slots per thread as the block needs (a clamped slot still costs its
    // loads): 5 passes are common (rows of 30-40 entries in blocks of 32 rows)
    const int passes = (k1 - k0 + RB_THREADS - 1) / RB_THREADS;
    static_assert(RB_CAP / RB_THREADS == 8, "stage variants cover 1 to 8 passes");
    if (passes > 6)
        rb_stage<8>(k0, k1, colat, val, xget, sp);
    else if (passes > 5)
        rb_stage<6>(k0, k1, colat, val, xget, sp);
    else if (passes > 4)
        rb_stage<5>(k0, k1, colat, val, xget, sp);
    else if (passes > 2)
        rb_stage<4>(k0, k1, colat, val, xget, sp);
    else if (passes > 0)
        rb_stage<2>(k0, k1, colat, val, xget, sp);
    __syncthreads();
}

template <typename T, class X>
__device__ __forceinline__ void rb_load(int row0, int row1, const int* __restrict__ ptr, const int* __restrict__ col,
                                        const T* __restrict__ val, X xget, int* sptr, T* sp) {
    rb_load_core(row0, row1, ptr, [&](int k) { return col[k]; }, val, xget, sptr, sp);
}

// Column indices as the row-block kernels of the V-cycle read them: int32, or two bytes
// relative to a base per row block (rows of a block reach nearby columns: aggregates of
// neighbouring nodes), which saves 2 of the 12 bytes an FP64 entry costs.
struct ColSrc {
    const int* __restrict__ col;
    const uint16_t* __restrict__ c16;
    const int* __restrict__ cblk;
};
inline ColSrc colsrc(const Csr& A) { return ColSrc{A.col, A.c16, A.cblk}; }

template <typename T, class X>
__device__ __forceinline__ void rb_load(int row0, int row1, const int* __restrict__ ptr, const ColSrc& cs, int blk,
                                        const T* __restrict__ val, X xget, int* sptr, T* sp) {
    if (cs.c16 != nullptr) {
        const int cb = cs.cblk[blk];
        rb_load_core(row0, row1, ptr, [&](int k) { return cb + (int)cs.c16[k]; }, val, xget, sptr, sp);
    } else {
        rb_load_core(row0, row1, ptr, [&](int k) { return cs.col[k]; }, val, xget, sptr, sp);
    }
}

// One base per row block: the smallest column of its rows (rows are sorted, so the
// first entry of each); *wide = 1 when a block's columns span more than two bytes.
__global__ __launch_bounds__(TPB) void k_c16_bases(int n, int rpb, const int* __restrict__ ptr,
                                                   const int* __restrict__ col, int* __restrict__ cblk,
                                                   int* __restrict__ wide) {
    const int b = blockIdx.x * TPB + threadIdx.x;
    const int nb = (n + rpb - 1) / rpb;
    if (b >= nb) return;
    const int r0 = b * rpb, r1 = min(r0 + rpb, n);
    int lo = INT_MAX, hi = INT_MIN;
    for (int r = r0; r < r1; ++r)
        if (ptr[r] < ptr[r + 1]) {
            lo = min(lo, col[ptr[r]]);
            hi = max(hi, col[ptr[r + 1] - 1]);
        }
    if (lo > hi) lo = hi = 0;  // no entries
    cblk[b] = lo;
    if ((int64_t)hi - lo > 65535) wide[0] = 1;
}

__global__ __launch_bounds__(TPB) void k_c16_fill(int n, int rpb, const int* __restrict__ ptr,
                                                  const int* __restrict__ col, const int* __restrict__ cblk,
                                                  uint16_t* __restrict__ c16) {
    const int r = blockIdx.x * TPB + threadIdx.x;
    if (r >= n) return;
    const int base = cblk[r / rpb];
    for (int k = ptr[r]; k < ptr[r + 1]; ++k) c16[k] = (uint16_t)(col[k] - base);
}

void launch_c16_bases(const Csr& A, int32_t* cblk, int* wide, hipStream_t s) {
    const int nb = (A.nrows + A.rpb - 1) / A.rpb;
    timed_launch(k_c16_bases, (unsigned)((nb + TPB - 1) / TPB), TPB, 0, s, A.nrows, A.rpb, A.ptr, A.col, cblk, wide);
    HIP_LAUNCH_CHECK();
}
void launch_c16_fill(const Csr& A, const int32_t* cblk, uint16_t* c16, hipStream_t s) {
    timed_launch(k_c16_fill, (unsigned)((A.nrows + TPB - 1) / TPB), TPB, 0, s, A.nrows, A.rpb, A.ptr, A.col, cblk, c16);
    HIP_LAUNCH_CHECK();
}

// Threads per staged row: a block of rpb rows gives each row RB_THREADS / rpb threads
// (at most a wavefront), which add strided subsets of the row and combine them with a
// fixed butterfly; with one thread per row the sum is in plain column order.
__device__ __forceinline__ int rb_tpr(int rpb) {
    const int t = RB_THREADS / rpb;
    return t > 64 ? 64 : t;
}

// Sum of row r (local) of the staged block; `lane` is the thread's index within the row.
template <typename T>
__device__ __forceinline__ T rb_rowsum(const int* sptr, const T* sp, int r, int lane, int tpr) {
    const int k0 = sptr[0], e = sptr[r + 1] - k0;
    T s = 0;
    for (int q = sptr[r] - k0 + lane; q < e; q += tpr) s += sp[q];
    for (int o = tpr >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o, tpr);
    return s;
}

// Contiguous range of row blocks handled by this (XCD-remapped) block of a bounded grid.
__device__ __forceinline__ void rb_range(int nrb, int& rb0, int& rb1) {
    const int per = (nrb + (int)gridDim.x - 1) / (int)gridDim.x;
    const int lb = xcd_block();
    rb0 = lb * per;
    rb1 = min(rb0 + per, nrb);
}

// Deterministic block sum of K values; thread 0 stores them at dst[q][slot].
template <int K>
__device__ __forceinline__ void block_store(double (&v)[K], double* const (&dst)[K], int slot) {
    __shared__ double sm[K][RB_THREADS / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const double x = wave_sum(v[q]);
        if (lane == 0) sm[q][w] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            double s = 0.0;
            for (int i = 0; i < RB_THREADS / 64; ++i) s += sm[q][i];
            dst[q][slot] = s;
        }
    }
}

// Sum of p[0..nb) by one block of FIN_THREADS threads in a fixed order (four independent
// strided accumulators per thread, then a fixed tree); returned to every thread.
constexpr int FIN_THREADS = 1024;
__device__ __forceinline__ double block_sum(const double* __restrict__ p, int nb) {
    __shared__ double sm[FIN_THREADS / 64];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    int i = threadIdx.x;
    for (; i + 3 * FIN_THREADS < nb; i += 4 * FIN_THREADS) {
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] += p[i + u * FIN_THREADS];
    }
    for (int u = 0; i < nb; i += FIN_THREADS, ++u) a[u & 3] += p[i];
    double s = (a[0] + a[1]) + (a[2] + a[3]);
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < FIN_THREADS / 64; ++k) t += sm[k];
    __syncthreads();
    return t;
}

// Where the CG update kernels put their ||r||^2 partials: straight into the host mirror
// when there is one (workgroup 0 also copies the breakdown flag there), else P_RR.
__device__ __forceinline__ double* rr_dest(const RedScratch& rs, bool bad) {
    if (rs.host == nullptr) return rs.region(P_RR);
    if (blockIdx.x == 0 && threadIdx.x == 0) rs.host[S_FLAG] = bad ? 1.0 : 0.0;
    return rs.host + S_COUNT;
}

// ------------------------------------------------------------------ V-cycle kernels

// The row-block V-cycle kernels below read their own row's epilogue operands (m, f, u)
// before the staging barrier, so those loads overlap the entry loads instead of following
// them.

// y = A x; with m2 given also y2 = m2 * y (the restriction forms the coarse level's first
// smoothing sweep u = m f from zero at the same time).
template <typename T>
__global__ __launch_bounds__(RB_THREADS) void k_rb_spmv(int n, int rpb, const int* __restrict__ ptr,
                                                        ColSrc cs, const T* __restrict__ val,
                                                        const T* __restrict__ x, T* __restrict__ y,
                                                        const T* __restrict__ m2, T* __restrict__ y2) {
    __shared__ int sptr[RB_THREADS + 1];
    __shared__ T sp[RB_CAP];
    const int row0 = xcd_block() * rpb;
    if (row0 >= n) return;
    const int row1 = min(row0 + rpb, n);
    const int tpr = rb_tpr(rpb), r = threadIdx.x / tpr, lane = threadIdx.x & (tpr - 1);
    const bool own = r < row1 - row0 && lane == 0;
    const T mi = (own && m2 != nullptr) ? m2[row0 + r] : T(0);
    rb_load(row0, row1, ptr, cs, xcd_block(), val, [&](int j) { return x[j]; }, sptr, sp);
    if (r < row1 - row0) {
        const T v = rb_rowsum(sptr, sp, r, lane, tpr);
        if (lane == 0) {
            y[row0 + r] = v;
            if (m2 != nullptr) y2[row0 + r] = mi * v;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(RB_THREADS) void k_rb_residual(int n, int rpb, const int* __restrict__ ptr,
                                                            ColSrc cs, const T* __restrict__ val,
                                                            const T* __restrict__ f, const T* __restrict__ u,
                                                            T* __restrict__ r) {
    __shared__ int sptr[RB_THREADS + 1];
    __shared__ T sp[RB_CAP];
    const int row0 = xcd_block() * rpb;
    if (row0 >= n) return;
    const int row1 = min(row0 + rpb, n);
    const int tpr = rb_tpr(rpb), t = threadIdx.x / tpr, lane = threadIdx.x & (tpr - 1);
    const bool own = t < row1 - row0 && lane == 0;
    const T fi = own ? f[row0 + t] : T(0);
    rb_load(row0, row1, ptr, cs, xcd_block(), val, [&](int j) { return u[j]; }, sptr, sp);
    if (t < row1 - row0) {
        const T v = rb_rowsum(sptr, sp, t, lane, tpr);
        if (lane == 0) r[row0 + t] = fi - v;
    }
}

// One damped-Jacobi / SPAI0 sweep: uout = u + m (f - A u)
template <typename T>
__global__ __launch_bounds__(RB_THREADS) void k_rb_jacobi(int n, int rpb, const int* __restrict__ ptr,
                                                          ColSrc cs, const T* __restrict__ val,
                                                          const T* __restrict__ m, const T* __restrict__ f,
                                                          const T* __restrict__ u, T* __restrict__ uout) {
    __shared__ int sptr[RB_THREADS + 1];
    __shared__ T sp[RB_CAP];
    const int row0 = xcd_block() * rpb;
    if (row0 >= n) return;
    const int row1 = min(row0 + rpb, n);
    const int tpr = rb_tpr(rpb), t = threadIdx.x / tpr, lane = threadIdx.x & (tpr - 1);
    const bool own = t < row1 - row0 && lane == 0;
    const int i = row0 + t;
    const T ui = own ? u[i] : T(0), mi = own ? m[i] : T(0), fi = own ? f[i] : T(0);
    rb_load(row0, row1, ptr, cs, xcd_block(), val, [&](int j) { return u[j]; }, sptr, sp);
    if (t < row1 - row0) {
        const T v = rb_rowsum(sptr, sp, t, lane, tpr);
        if (lane == 0) uout[i] = ui + mi * (fi - v);
    }
}

// First pre-smoothing sweep from u = 0 (u = m f) fused with the residual r = f - A u; the
// neighbours' u_j = m_j f_j are formed from m and f.
template <typename T>
__global__ __launch_bounds__(RB_THREADS) void k_rb_smooth0_residual(int n, int rpb, const int* __restrict__ ptr,
                                                                    ColSrc cs,
                                                                    const T* __restrict__ val, const T* __restrict__ m,
                                                                    const T* __restrict__ f, T* __restrict__ u,
                                                                    T* __restrict__ r) {
    __shared__ int sptr[RB_THREADS + 1];
    __shared__ T sp[RB_CAP];
    const int row0 = xcd_block() * rpb;
    if (row0 >= n) return;
    const int row1 = min(row0 + rpb, n);
    const int tpr = rb_tpr(rpb), t = threadIdx.x / tpr, lane = threadIdx.x & (tpr - 1);
    const bool own = t < row1 - row0 && lane == 0;
    const int i = row0 + t;
    const T mi = own ? m[i] : T(0), fi = own ? f[i] : T(0);
    rb_load(row0, row1, ptr, cs, xcd_block(), val, [&](int j) { return m[j] * f[j]; }, sptr, sp);
    if (t < row1 - row0) {
        const T v = rb_rowsum(sptr, sp, t, lane, tpr);
        if (lane == 0) {
            u[i] = mi * fi;
            r[i] = fi - v;
        }
    }
}

// u += P uc (coarse-grid correction)
template <typename T>
__global__ __launch_bounds__(RB_THREADS) void k_rb_prolong_add(int n, int rpb, const int* __restrict__ ptr,
                                                               ColSrc cs, const T* __restrict__ val,
                                                               const T* __restrict__ uc, T* __restrict__ u) {
    __shared__ int sptr[RB_THREADS + 1];
    __shared__ T sp[RB_CAP];
    const int row0 = xcd_block() * rpb;
    if (row0 >= n) return;
    const int row1 = min(row0 + rpb, n);
    const int tpr = rb_tpr(rpb), t = threadIdx.x / tpr, lane = threadIdx.x & (tpr - 1);
    const bool own = t < row1 - row0 && lane == 0;
    const T ui = own ? u[row0 + t] : T(0);
    rb_load(row0, row1, ptr, cs, xcd_block(), val, [&](int j) { return uc[j]; }, sptr, sp);
    if (t < row1 - row0) {
        const T v = rb_rowsum(sptr, sp, t, lane, tpr);
        if (lane == 0) u[row0 + t] = ui + v;
    }
}

// Lane-group fallbacks (rows longer than a staged block).
template <int G>
__device__ __forceinline__ int group_row(int& lane) {
    lane = threadIdx.x & (G - 1);
    return (xcd_block() * TPB + (int)threadIdx.x) / G;
}

template <int G, typename T, int KIND>
__global__ __launch_bounds__(TPB) void k_lg(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                                            const T* __restrict__ val, const T* __restrict__ m,
                                            const T* __restrict__ f, const T* __restrict__ x, T* __restrict__ y,
                                            T* __restrict__ y2) {
    int lane;
    const int row = group_row<G>(lane);
    if (row >= n) return;
    const int b = ptr[row], e = ptr[row + 1];
    T s = 0;
    for (int k = b + lane; k < e; k += G) {
        const int j = col[k];
        s += val[k] * (KIND == 3 ? m[j] * f[j] : x[j]);
    }
    s = group_sum<G>(s);
    if (lane != 0) return;
    if constexpr (KIND == 0) {                                            // y = A x (, y2 = m y)
        y[row] = s;
        if (m != nullptr) y2[row] = m[row] * s;
    }
    if constexpr (KIND == 1) y[row] = f[row] - s;                         // r = f - A x
    if constexpr (KIND == 2) y[row] = x[row] + m[row] * (f[row] - s);     // Jacobi
    if constexpr (KIND == 3) {                                            // first sweep + residual
        y[row] = m[row] * f[row];
        y2[row] = f[row] - s;
    }
    if constexpr (KIND == 4) y[row] += s;                                 // u += P uc
}

// s = sum of a[j] * x[j] over j = j0, j0 + G, ... < n, added in that order; U pairs are
// loaded before they are added, so that a row of a few hundred entries costs a few round
// trips to memory rather than one per entry.
template <int G, typename T>
__device__ __forceinline__ double strided_dot(const double* __restrict__ a, const T* x, int j0, int n) {
    constexpr int U = 8;
    double s = 0.0;
    for (int jb = j0; jb < n; jb += U * G) {
        double av[U], xv[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int j = jb + k * G;
            av[k] = j < n ? a[j] : 0.0;
            xv[k] = j < n ? (double)x[j] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (jb + k * G < n) s += av[k] * xv[k];
    }
    return s;
}

// u = A^{-1} f on the coarsest level: one wavefront per row of the dense FP64 inverse; a
// NaN solution when the inverse's pivot flag *bad is set (a coarsest operator that is not
// SPD then surfaces as a breakdown of the Krylov method that applies the cycle).
template <typename T>
__global__ __launch_bounds__(TPB) void k_coarse_gemv(int n, const double* __restrict__ inv, const T* __restrict__ f,
                                                     T* __restrict__ u, const double* __restrict__ bad) {
    const int lane = threadIdx.x & 63;
    const int row = (blockIdx.x * TPB + (int)threadIdx.x) >> 6;
    if (row >= n) return;
    double s = strided_dot<64>(inv + (size_t)row * n, f, lane, n);
    s = wave_sum(s);
    if (lane == 0) u[row] = (*bad != 0.0) ? (T)__builtin_nan("") : (T)s;
}

__global__ void k_cast_d2f(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

__global__ void k_cast_f2d(int64_t n, const float* __restrict__ a, double* __restrict__ b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (double)a[i];
}

__global__ void k_copy(int64_t n, const double* __restrict__ a, double* __restrict__ b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

static inline unsigned ew_blocks(int64_t n) {
    int64_t b = (n + TPB - 1) / TPB;
    if (b > 8192) b = 8192;
    return (unsigned)(b > 0 ? b : 1);
}

#define AMG_RB_OR_LG(A, RBCALL, KIND, ...)                                                              \
    do {                                                                                                \
        if ((A).rpb > 0) {                                                                              \
            RBCALL;                                                                                     \
        } else {                                                                                        \
            AMG_WITH_G((A).g, (timed_launch(k_lg<G, T, KIND>, grid_for((int64_t)(A).nrows * G, TPB), TPB, 0, s, __VA_ARGS__))); \
        }                                                                                               \
        HIP_LAUNCH_CHECK();                                                                             \
    } while (0)

// The restriction and the prolongation go through timed_launch: when their class is
// traced the launch records its own events.
template <typename T>
void launch_spmv(const Csr& A, const T* x, T* y, const T* m2, T* y2, hipStream_t s) {
    if (A.rpb > 0) {
        timed_launch(k_rb_spmv<T>, grid_for(A.nrows, A.rpb), RB_THREADS, 0, s, A.nrows, A.rpb, (const int*)A.ptr,
                     colsrc(A), (const T*)A.v<T>(), x, y, m2, y2);
    } else {
        AMG_WITH_G(A.g, timed_launch(k_lg<G, T, 0>, grid_for((int64_t)A.nrows * G, TPB), TPB, 0, s, A.nrows,
                                     (const int*)A.ptr, (const int*)A.col, (const T*)A.v<T>(), m2, (const T*)nullptr,
                                     x, y, y2));
    }
    HIP_LAUNCH_CHECK();
}
template <typename T>
void launch_residual(const Csr& A, const T* f, const T* u, T* r, hipStream_t s) {
    AMG_RB_OR_LG(A, (timed_launch(k_rb_residual<T>, grid_for(A.nrows, A.rpb), RB_THREADS, 0, s, A.nrows, A.rpb, A.ptr, colsrc(A), A.v<T>(), f, u, r)),
                 1, A.nrows, A.ptr, A.col, A.v<T>(), nullptr, f, u, r, nullptr);
}
template <typename T>
void launch_jacobi(const Csr& A, const T* m, const T* f, const T* u, T* uout, hipStream_t s) {
    AMG_RB_OR_LG(A, (timed_launch(k_rb_jacobi<T>, grid_for(A.nrows, A.rpb), RB_THREADS, 0, s, A.nrows, A.rpb, A.ptr, colsrc(A), A.v<T>(), m, f, u, uout)),
                 2, A.nrows, A.ptr, A.col, A.v<T>(), m, f, u, uout, nullptr);
}
template <typename T>
void launch_smooth0_residual(const Csr& A, const T* m, const T* f, T* u, T* r, hipStream_t s) {
    AMG_RB_OR_LG(A, (timed_launch(k_rb_smooth0_residual<T>, grid_for(A.nrows, A.rpb), RB_THREADS, 0, s, A.nrows, A.rpb, A.ptr, colsrc(A), A.v<T>(), m, f, u, r)),
                 3, A.nrows, A.ptr, A.col, A.v<T>(), m, f, nullptr, u, r);
}
template <typename T>
void launch_prolong_add(const Csr& P, const T* uc, T* u, hipStream_t s) {
    if (P.rpb > 0) {
        timed_launch(k_rb_prolong_add<T>, grid_for(P.nrows, P.rpb), RB_THREADS, 0, s, P.nrows, P.rpb,
                     (const int*)P.ptr, colsrc(P), (const T*)P.v<T>(), uc, u);
    } else {
        AMG_WITH_G(P.g, timed_launch(k_lg<G, T, 4>, grid_for((int64_t)P.nrows * G, TPB), TPB, 0, s, P.nrows,
                                     (const int*)P.ptr, (const int*)P.col, (const T*)P.v<T>(), (const T*)nullptr,
                                     (const T*)nullptr, uc, u, (T*)nullptr));
    }
    HIP_LAUNCH_CHECK();
}
template <typename T>
void launch_coarse_gemv(int n, const double* inv, const T* f, T* u, const double* bad, hipStream_t s) {
    timed_launch(k_coarse_gemv<T>, grid_for((int64_t)n * 64, TPB), TPB, 0, s, n, inv, f, u, bad);
    HIP_LAUNCH_CHECK();
}
void launch_cast_d2f(int64_t n, const double* a, float* b, hipStream_t s) {
    timed_launch(k_cast_d2f, ew_blocks(n), TPB, 0, s, n, a, b);
    HIP_LAUNCH_CHECK();
}
void launch_cast_f2d(int64_t n, const float* a, double* b, hipStream_t s) {
    timed_launch(k_cast_f2d, ew_blocks(n), TPB, 0, s, n, a, b);
    HIP_LAUNCH_CHECK();
}
void launch_copy(int64_t n, const double* a, double* b, hipStream_t s) {
    timed_launch(k_copy, ew_blocks(n), TPB, 0, s, n, a, b);
    HIP_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ diagonal storage
//
// Level-0 kernels on the diagonal storage of A_0: one thread per row, the row's
// diagonals in increasing offset (that is, column) order, each term added to the row sum
// with a fused multiply-add; an absent entry is stored as 0, and a column outside [0, n)
// drops its term.  Values and vector entries are read with coalesced loads and no index
// arrays.  Reductions write one partial per workgroup (logical block order).
//
// Symmetric values (o.sym): the offsets are -k..k around a main diagonal in the middle,
// and the entry on diagonal d < nd/2 of row i is read as the entry on the mirrored
// diagonal nd-1-d of row j = i + off[d]; that is the same number, so the sum (same terms,
// same order) is the same to the bit, and only the main and upper diagonals are read.

template <typename T>
__device__ __forceinline__ T fmadd(T a, T b, T c) {
    if constexpr (std::is_same<T, double>::value)
        return __builtin_fma(a, b, c);
    else
        return __builtin_fmaf(a, b, c);
}

// ND > 0: the diagonal count as a compile-time constant (the loops unroll fully).  Every
// load is issued unconditionally (a column outside [0, n) reads row i's own entries
// instead) and an out-of-range term is dropped with a select, not a branch, so that all
// of a row's loads are in flight together.
template <int ND, typename T, typename X>
__device__ __forceinline__ T dia_row(int i, int n, int nd_rt, const DiaOff& o, const T* __restrict__ v, X xget) {
    const int nd = ND > 0 ? ND : nd_rt;
    T s = 0;
    if (o.sym) {
        const int h = nd >> 1;
#pragma unroll
        for (int d = 0; d < h; ++d) {
            const int j = i + o.off[d];
            const bool in = (unsigned)j < (unsigned)n;
            const int jj = in ? j : i;
            const T t = fmadd(v[(size_t)(nd - 1 - d) * n + jj], xget(jj), s);
            s = in ? t : s;
        }
#pragma unroll
        for (int d = h; d < nd; ++d) {
            const int j = i + o.off[d];
            const bool in = (unsigned)j < (unsigned)n;
            const T t = fmadd(v[(size_t)d * n + i], xget(in ? j : i), s);
            s = in ? t : s;
        }
        return s;
    }
#pragma unroll
    for (int d = 0; d < nd; ++d) {
        const int j = i + o.off[d];
        const bool in = (unsigned)j < (unsigned)n;
        const T t = fmadd(v[(size_t)d * n + i], xget(in ? j : i), s);
        s = in ? t : s;
    }
    return s;
}

// Calls f(std::integral_constant<int, ND>) with ND = 7 for the 7-point stencil, else 0.
template <typename F>
inline void dia_nd(int nd, F&& f) {
    if (nd == 7)
        f(std::integral_constant<int, 7>{});
    else
        f(std::integral_constant<int, 0>{});
}

// Refresh of the diagonal storage from A's CSR values.  Few diagonals: one thread per row
// writes its entries (each write coalesced across the rows of a wavefront).  Many (the
// 27-point operator): a row's entries are far apart for the threads of a wavefront, so a
// workgroup reads its rows' entries once, coalesced, into a diagonal-major LDS tile and
// writes each diagonal's run of rows (1.1 ms -> 0.5 ms per refresh at 160^3; the 7-point
// refresh stays faster per row).
template <typename T>
__global__ __launch_bounds__(TPB) void k_dia_scatter_rows(int n, const int* __restrict__ ptr,
                                                          const uint8_t* __restrict__ slot,
                                                          const double* __restrict__ val, T* __restrict__ dval) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n) return;
    for (int t = ptr[i]; t < ptr[i + 1]; ++t) dval[(size_t)slot[t] * n + i] = (T)val[t];
}

// The reverse: the CSR values of A_0 from its diagonal storage (the CSR copy is only
// formed on demand once the partial update writes the diagonal storage directly).
template <typename T>
__global__ __launch_bounds__(TPB) void k_dia_gather_rows(int n, const int* __restrict__ ptr,
                                                         const uint8_t* __restrict__ slot,
                                                         const T* __restrict__ dval, T* __restrict__ val) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n) return;
    for (int t = ptr[i]; t < ptr[i + 1]; ++t) val[t] = dval[(size_t)slot[t] * n + i];
}

constexpr int SC_ROWS = 128;
constexpr int SC_TILE_MIN_DIAG = 16;

template <typename T>
__global__ __launch_bounds__(TPB) void k_dia_scatter(int n, int nd, const int* __restrict__ ptr,
                                                     const uint8_t* __restrict__ slot, const double* __restrict__ val,
                                                     T* __restrict__ dval) {
    // absent entries stay 0 in the tile, as in the storage
    __shared__ int sptr[SC_ROWS + 1];
    __shared__ T tile[DIA_MAX * SC_ROWS];
    const int r0 = xcd_block() * SC_ROWS;
    if (r0 >= n) return;
    const int nr = min(SC_ROWS, n - r0);
    for (int i = threadIdx.x; i <= nr; i += TPB) sptr[i] = ptr[r0 + i];
    for (int e = threadIdx.x; e < nd * SC_ROWS; e += TPB) tile[e] = T(0);
    __syncthreads();
    const int e0 = sptr[0], e1 = sptr[nr];
    for (int e = e0 + (int)threadIdx.x; e < e1; e += TPB) {
        int lo = 0, hi = nr;  // the entry's row: sptr[lo] <= e < sptr[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (sptr[mid] <= e)
                lo = mid;
            else
                hi = mid;
        }
        tile[(int)slot[e] * SC_ROWS + lo] = (T)val[e];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nd * SC_ROWS; e += TPB) {
        const int d = e / SC_ROWS, r = e - d * SC_ROWS;
        if (r < nr) dval[(size_t)d * n + r0 + r] = tile[e];
    }
}

// Compares every sub-diagonal value with its mirror (absent entries are stored zeros, so
// the pattern is compared too).  k_dia_clear zeroes the flag in a launch of its own first;
// the check only ever stores 1, so the order of its stores does not matter.
__global__ void k_dia_clear(double* __restrict__ flag) {
    if (threadIdx.x == 0) flag[0] = 0.0;
}

__global__ __launch_bounds__(TPB) void k_dia_symcheck(int n, int nd, DiaOff o, const double* __restrict__ v,
                                                      double* __restrict__ flag) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n) return;
    bool bad = false;
    for (int d = 0; d < (nd >> 1); ++d) {
        const int j = i + o.off[d];
        if ((unsigned)j < (unsigned)n)
            bad |= __double_as_longlong(v[(size_t)d * n + i]) !=
                   __double_as_longlong(v[(size_t)(nd - 1 - d) * n + j]);
    }
    if (bad) flag[0] = 1.0;
}

template <typename T, int ND>
__global__ __launch_bounds__(TPB) void k_dia_smooth0_residual(int n, int nd, DiaOff o, const T* __restrict__ v,
                                                              const T* __restrict__ m, const T* __restrict__ f,
                                                              T* __restrict__ u, T* __restrict__ r) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n) return;
    const T s = dia_row<ND>(i, n, nd, o, v, [&](int j) { return m[j] * f[j]; });
    const T fi = f[i];
    u[i] = m[i] * fi;
    r[i] = fi - s;
}

template <typename T, int ND>
__global__ __launch_bounds__(TPB) void k_dia_residual(int n, int nd, DiaOff o, const T* __restrict__ v,
                                                      const T* __restrict__ f, const T* __restrict__ u,
                                                      T* __restrict__ r) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n) return;
    r[i] = f[i] - dia_row<ND>(i, n, nd, o, v, [&](int j) { return u[j]; });
}

template <typename T, int ND>
__global__ __launch_bounds__(TPB) void k_dia_jacobi(int n, int nd, DiaOff o, const T* __restrict__ v,
                                                    const T* __restrict__ m, const T* __restrict__ f,
                                                    const T* __restrict__ u, T* __restrict__ uout) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n) return;
    const T s = dia_row<ND>(i, n, nd, o, v, [&](int j) { return u[j]; });
    uout[i] = u[i] + m[i] * (f[i] - s);
}

template <int ND>
__global__ __launch_bounds__(TPB) void k_dia_jacobi_rz(int n, int nd, DiaOff o, const double* __restrict__ v,
                                                       const double* __restrict__ m, const double* __restrict__ r,
                                                       const double* __restrict__ u, double* __restrict__ z,
                                                       int flexible, RedScratch rs) {
    const int lb = xcd_block();
    const int i = lb * TPB + threadIdx.x;
    double loc[2] = {0.0, 0.0};
    if (i < n) {
        const double s = dia_row<ND>(i, n, nd, o, v, [&](int j) { return u[j]; });
        const double ri = r[i];
        const double zi = u[i] + m[i] * (ri - s);
        if (flexible) loc[1] += ri * z[i];
        z[i] = zi;
        loc[0] += ri * zi;
    }
    double* const dst[2] = {rs.region(P_RZ), rs.region(P_RZOLD)};
    block_store<2>(loc, dst, lb);
}

template <int ND, bool FIRST>
__global__ __launch_bounds__(TPB) void k_dia_cg_pq(int n, int nd, DiaOff o, const double* __restrict__ v,
                                                   const double* __restrict__ z, const double* __restrict__ pold,
                                                   double* __restrict__ pnew, double* __restrict__ q,
                                                   RedScratch rs) {
    const double beta = FIRST ? 0.0 : rs.scal()[S_BETA];
    auto pv = [&](int j) { return FIRST ? z[j] : __builtin_fma(beta, pold[j], z[j]); };
    const int lb = xcd_block();
    const int i = lb * TPB + threadIdx.x;
    double loc[1] = {0.0};
    if (i < n) {
        const double qi = dia_row<ND>(i, n, nd, o, v, pv);
        const double pi = pv(i);
        pnew[i] = pi;
        q[i] = qi;
        loc[0] += pi * qi;
    }
    double* const dst[1] = {rs.region(P_PQ)};
    block_store<1>(loc, dst, lb);
}

// The set of distinct column offsets (col - row) of a CSR pattern, in a 64-slot open-
// addressing table (DIA_EMPTY: free).  Each workgroup first collects its rows' offsets in
// LDS, then inserts them into the global table; flag[0] is set when the set outgrows
// DIA_MAX.  Integer compare-and-swap only: the resulting set does not depend on order.
constexpr int DIA_TAB = 64;
constexpr int DIA_EMPTY = INT_MIN;

__device__ __forceinline__ bool dia_insert(int* tab, int o) {
    unsigned h = ((unsigned)o * 2654435761u) >> 26;  // 6 bits
    for (int p = 0; p < DIA_TAB; ++p) {
        int* slot = tab + ((h + p) & (DIA_TAB - 1));
        const int cur = *slot;
        if (cur == o) return true;
        if (cur == DIA_EMPTY) {
            const int prev = atomicCAS(slot, DIA_EMPTY, o);
            if (prev == DIA_EMPTY || prev == o) return true;
        }
    }
    return false;
}

__global__ __launch_bounds__(TPB) void k_dia_offsets(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                                                     int* __restrict__ tab, int* __restrict__ flag) {
    __shared__ int st[DIA_TAB];
    __shared__ int over;
    if (threadIdx.x < DIA_TAB) st[threadIdx.x] = DIA_EMPTY;
    if (threadIdx.x == 0) over = 0;
    __syncthreads();
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i < n)
        for (int k = ptr[i]; k < ptr[i + 1]; ++k)
            if (!dia_insert(st, col[k] - i)) {
                over = 1;
                break;
            }
    __syncthreads();
    if (threadIdx.x < DIA_TAB && st[threadIdx.x] != DIA_EMPTY)
        if (!dia_insert(tab, st[threadIdx.x])) over = 1;
    __syncthreads();
    if (threadIdx.x == 0 && over) flag[0] = 1;
}

// Diagonal index of every stored entry, given the sorted offsets.
__global__ __launch_bounds__(TPB) void k_dia_slots(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                                                   int nd, DiaOff o, uint8_t* __restrict__ slot) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i >= n) return;
    for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
        const int off = col[k] - i;
        int lo = 0, hi = nd - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (o.off[mid] < off)
                lo = mid + 1;
            else
                hi = mid;
        }
        slot[k] = (uint8_t)lo;
    }
}

// The distinct offsets of A's pattern (sorted), or an empty list when there are more
// than DIA_MAX of them.
std::vector<int> dia_offsets(const Csr& A, hipStream_t s) {
    int* buf = dnew<int>(DIA_TAB + 1, s);
    std::vector<int> init(DIA_TAB + 1, DIA_EMPTY);
    init[DIA_TAB] = 0;
    HIP_CHECK(hipMemcpyAsync(buf, init.data(), init.size() * sizeof(int), hipMemcpyHostToDevice, s));
    timed_launch(k_dia_offsets, (unsigned)((A.nrows + TPB - 1) / TPB), TPB, 0, s, A.nrows, A.ptr, A.col, buf, buf + DIA_TAB);
    HIP_LAUNCH_CHECK();
    std::vector<int> h(DIA_TAB + 1);
    HIP_CHECK(hipMemcpyAsync(h.data(), buf, h.size() * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    dfree(buf, s);
    std::vector<int> offs;
    if (h[DIA_TAB] != 0) return offs;
    for (int q = 0; q < DIA_TAB; ++q)
        if (h[q] != DIA_EMPTY) offs.push_back(h[q]);
    if ((int)offs.size() > DIA_MAX) return {};
    std::sort(offs.begin(), offs.end());
    return offs;
}

void launch_dia_slots(const Csr& A, const Dia& D, hipStream_t s) {
    timed_launch(k_dia_slots, (unsigned)((A.nrows + TPB - 1) / TPB), TPB, 0, s, A.nrows, A.ptr, A.col, D.ndiag, D.off, D.slot);
    HIP_LAUNCH_CHECK();
}

// The CG update x += alpha p, r_new = r - alpha q (x does not move on breakdown) fused with
// the first V-cycle sweep from zero on level 0 and its residual: u = m r_new and
// rv = r_new - A u, where every neighbour's r_new is formed from r and q with the same
// operation as its owner row uses (so r is read, and r_new written to another buffer);
// ||r_new||^2 partials, one per workgroup.
template <int ND>
__global__ __launch_bounds__(TPB) void k_dia_update_smooth0(int n, int nd, DiaOff o, const double* __restrict__ v,
                                                            const double* __restrict__ p,
                                                            const double* __restrict__ q, double* __restrict__ x,
                                                            const double* __restrict__ r, double* __restrict__ rn,
                                                            const double* __restrict__ m, double* __restrict__ u,
                                                            double* __restrict__ rv, RedScratch rs) {
    const double* sc = rs.scal();
    const bool bad = sc[S_FLAG] != 0.0;
    const double alpha = sc[S_ALPHA];
    // on breakdown r_new = r - 0 q (r up to the sign of a zero entry; the solve stops there)
    const double step = bad ? 0.0 : alpha;
    auto rnew = [&](int j) { return __builtin_fma(-step, q[j], r[j]); };
    const int lb = xcd_block();
    const int i = lb * TPB + threadIdx.x;
    double loc[1] = {0.0};
    if (i < n) {
        const double s = dia_row<ND>(i, n, nd, o, v, [&](int j) { return m[j] * rnew(j); });
        const double ri = rnew(i);
        if (!bad) x[i] = __builtin_fma(alpha, p[i], x[i]);
        rn[i] = ri;
        u[i] = m[i] * ri;
        rv[i] = ri - s;
        loc[0] = ri * ri;
    }
    double* const dst[1] = {rr_dest(rs, bad)};
    block_store<1>(loc, dst, lb);
}

// r = f - A x on the diagonal storage, with ||r||^2 and ||f||^2 partials (bounded grid,
// host-summed).
template <int ND>
__global__ __launch_bounds__(TPB) void k_dia_cg_init(int n, int nd, DiaOff o, const double* __restrict__ v,
                                                     const double* __restrict__ f, const double* __restrict__ x,
                                                     double* __restrict__ r, RedScratch rs) {
    double loc[2] = {0.0, 0.0};
    for (int i = blockIdx.x * TPB + threadIdx.x; i < n; i += gridDim.x * TPB) {
        const double fi = f[i];
        const double ri = fi - dia_row<ND>(i, n, nd, o, v, [&](int j) { return x[j]; });
        r[i] = ri;
        loc[0] += ri * ri;
        loc[1] += fi * fi;
    }
    double* const dst[2] = {rs.region(P_RR), rs.region(P_FF)};
    block_store<2>(loc, dst, blockIdx.x);
}

static inline unsigned dia_blocks(int n) { return (unsigned)((n + TPB - 1) / TPB); }

// ------------------------------------------------------------------ 7-point marching form
//
// Level-0 kernels for a 7-point operator whose diagonals have the offsets -a, -b, -1, 0,
// 1, b, a (1 < b < a: a stencil on a grid of planes of a rows and lines of b rows).  The
// one-row-per-thread kernels above load the vector at all seven columns of a row and
// every load goes through the vector memory path on its own; here a workgroup owns TPB
// consecutive positions r of a plane and MZ consecutive planes (rows i = plane * a + r)
// and every vector entry is loaded about once: x(i -+ a) is the thread's own x of the
// planes before and after, x(i -+ 1) and x(i -+ b) are read from an LDS copy of the
// plane's segment (from global memory where they fall outside it), and with symmetric
// values the sub-diagonal entries U_1(i - 1), U_b(i - b) come from LDS copies of those
// diagonals, U_a(i - a) from the previous plane.  All global loads of the MZ planes are
// issued before the first is used.  Each row adds the same terms in the same order with
// the same fused multiply-adds as dia_row, so the row results equal the one-row-per-thread
// kernels' bit for bit; reduction partials are one per workgroup.
constexpr int MZ = 2;

int march_blocks(int n, int a) {
    const int64_t nseg = (a + TPB - 1) / TPB;
    const int64_t planes = ((int64_t)n + a - 1) / a;
    return (int)(nseg * ((planes + MZ - 1) / MZ));
}

template <bool SYM, typename T, typename XG, typename EP>
__device__ __forceinline__ void march7(int n, int a, int b, const T* __restrict__ v, XG xget, EP epi) {
    __shared__ T Xs[2][TPB];
    __shared__ T U1s[SYM ? 2 : 1][SYM ? TPB : 1], Ubs[SYM ? 2 : 1][SYM ? TPB : 1];
    const int nseg = (a + TPB - 1) / TPB;
    const int lb = xcd_block();
    const int t = threadIdx.x;
    const int r = (lb % nseg) * TPB + t;
    const bool own = r < a;  // positions past the plane only supply their x to neighbours
    const int64_t ib = (int64_t)(lb / nseg) * MZ * a + r;
    auto cl = [n](int64_t j) { return (j >= 0 && j < n) ? (int)j : 0; };  // loads stay in [0, n)
    const size_t sn = (size_t)n;
    const T* dm = v + 3 * sn;  // offset 0
    const T* d1 = v + 4 * sn;  // +1
    const T* db = v + 5 * sn;  // +b
    const T* da = v + 6 * sn;  // +a
    T X[MZ + 2], A0[MZ], A1[MZ], AB[MZ], AA[MZ + 1], LA[MZ], LB[MZ], L1[MZ];
    T XMB[MZ], AMB[MZ], XPB[MZ], XM1[MZ], AM1[MZ], XP1[MZ];
    const bool mb_out = t < b, pb_out = t + b >= TPB;
    AA[0] = SYM ? da[cl(ib - a)] : T(0);
#pragma unroll
    for (int k = 0; k < MZ + 2; ++k) X[k] = xget(cl(ib + (int64_t)(k - 1) * a));
#pragma unroll
    for (int k = 0; k < MZ; ++k) {
        const int64_t i = ib + (int64_t)k * a;
        const int ic = cl(i);
        A0[k] = dm[ic];
        A1[k] = d1[ic];
        AB[k] = db[ic];
        AA[k + 1] = da[ic];
        if constexpr (!SYM) {
            LA[k] = v[ic];
            LB[k] = v[sn + ic];
            L1[k] = v[2 * sn + ic];
        }
        XMB[k] = AMB[k] = XPB[k] = XM1[k] = AM1[k] = XP1[k] = T(0);
        if (mb_out) {
            const int jj = cl(i - b);
            XMB[k] = xget(jj);
            if constexpr (SYM) AMB[k] = db[jj];
        }
        if (pb_out) XPB[k] = xget(cl(i + b));
        if (t == 0) {
            const int jj = cl(i - 1);
            XM1[k] = xget(jj);
            if constexpr (SYM) AM1[k] = d1[jj];
        }
        if (t == TPB - 1) XP1[k] = xget(cl(i + 1));
    }
    const int tm1 = t > 0 ? t - 1 : t, tp1 = t < TPB - 1 ? t + 1 : t;
    const int tmb = mb_out ? t : t - b, tpb = pb_out ? t : t + b;
#pragma unroll
    for (int k = 0; k < MZ; ++k) {
        const int64_t i = ib + (int64_t)k * a;
        const int bf = k & 1;
        Xs[bf][t] = X[k + 1];
        if constexpr (SYM) {
            U1s[bf][t] = A1[k];
            Ubs[bf][t] = AB[k];
        }
        __syncthreads();
        const T x_m1 = t > 0 ? Xs[bf][tm1] : XM1[k];
        const T x_p1 = t < TPB - 1 ? Xs[bf][tp1] : XP1[k];
        const T x_mb = mb_out ? XMB[k] : Xs[bf][tmb];
        const T x_pb = pb_out ? XPB[k] : Xs[bf][tpb];
        T c_ma, c_mb, c_m1;
        if constexpr (SYM) {
            c_ma = AA[k];
            c_mb = mb_out ? AMB[k] : Ubs[bf][tmb];
            c_m1 = t > 0 ? U1s[bf][tm1] : AM1[k];
        } else {
            c_ma = LA[k];
            c_mb = LB[k];
            c_m1 = L1[k];
        }
        if (own && i < n) {
            T s = 0;
            s = i - a >= 0 ? fmadd(c_ma, X[k], s) : s;
            s = i - b >= 0 ? fmadd(c_mb, x_mb, s) : s;
            s = i - 1 >= 0 ? fmadd(c_m1, x_m1, s) : s;
            s = fmadd(A0[k], X[k + 1], s);
            s = i + 1 < n ? fmadd(A1[k], x_p1, s) : s;
            s = i + b < n ? fmadd(AB[k], x_pb, s) : s;
            s = i + a < n ? fmadd(AA[k + 1], X[k + 2], s) : s;
            epi((int)i, s, X[k + 1]);
        }
    }
}

template <bool SYM, typename T>
__global__ __launch_bounds__(TPB) void k_m7_smooth0_residual(int n, int a, int b, const T* __restrict__ v,
                                                             const T* __restrict__ m, const T* __restrict__ f,
                                                             T* __restrict__ u, T* __restrict__ r) {
    march7<SYM, T>(n, a, b, v, [&](int j) { return m[j] * f[j]; }, [&](int i, T s, T xc) {
        u[i] = xc;
        r[i] = f[i] - s;
    });
}

template <bool SYM, typename T>
__global__ __launch_bounds__(TPB) void k_m7_residual(int n, int a, int b, const T* __restrict__ v,
                                                     const T* __restrict__ f, const T* __restrict__ u,
                                                     T* __restrict__ r) {
    march7<SYM, T>(n, a, b, v, [&](int j) { return u[j]; }, [&](int i, T s, T) { r[i] = f[i] - s; });
}

template <bool SYM, typename T>
__global__ __launch_bounds__(TPB) void k_m7_jacobi(int n, int a, int b, const T* __restrict__ v,
                                                   const T* __restrict__ m, const T* __restrict__ f,
                                                   const T* __restrict__ u, T* __restrict__ uout) {
    march7<SYM, T>(n, a, b, v, [&](int j) { return u[j]; },
                   [&](int i, T s, T xc) { uout[i] = xc + m[i] * (f[i] - s); });
}

template <bool SYM>
__global__ __launch_bounds__(TPB) void k_m7_jacobi_rz(int n, int a, int b, const double* __restrict__ v,
                                                      const double* __restrict__ m, const double* __restrict__ r,
                                                      const double* __restrict__ u, double* __restrict__ z,
                                                      int flexible, RedScratch rs) {
    double loc[2] = {0.0, 0.0};
    march7<SYM, double>(n, a, b, v, [&](int j) { return u[j]; }, [&](int i, double s, double xc) {
        const double ri = r[i];
        const double zi = xc + m[i] * (ri - s);
        if (flexible) loc[1] += ri * z[i];
        z[i] = zi;
        loc[0] += ri * zi;
    });
    double* const dst[2] = {rs.region(P_RZ), rs.region(P_RZOLD)};
    block_store<2>(loc, dst, xcd_block());
}

// Mixed precision: the last FP32 sweep of level 0 writes z in FP64 (its FP32 value widened,
// as k_cast_rz does) and forms the CG's r.z with the FP64 residual r in the same pass.
template <bool SYM>
__global__ __launch_bounds__(TPB) void k_m7_jacobi_rz32(int n, int a, int b, const float* __restrict__ v,
                                                        const float* __restrict__ m, const float* __restrict__ f,
                                                        const float* __restrict__ u, const double* __restrict__ r,
                                                        double* __restrict__ z, int flexible, RedScratch rs) {
    double loc[2] = {0.0, 0.0};
    march7<SYM, float>(n, a, b, v, [&](int j) { return u[j]; }, [&](int i, float s, float xc) {
        const float z32 = xc + m[i] * (f[i] - s);
        const double ri = r[i];
        const double zi = (double)z32;
        if (flexible) loc[1] += ri * z[i];
        z[i] = zi;
        loc[0] += ri * zi;
    });
    double* const dst[2] = {rs.region(P_RZ), rs.region(P_RZOLD)};
    block_store<2>(loc, dst, xcd_block());
}

template <bool SYM, bool FIRST>
__global__ __launch_bounds__(TPB) void k_m7_cg_pq(int n, int a, int b, const double* __restrict__ v,
                                                  const double* __restrict__ z, const double* __restrict__ pold,
                                                  double* __restrict__ pnew, double* __restrict__ q, RedScratch rs) {
    const double beta = FIRST ? 0.0 : rs.scal()[S_BETA];
    double loc[1] = {0.0};
    march7<SYM, double>(
        n, a, b, v, [&](int j) { return FIRST ? z[j] : __builtin_fma(beta, pold[j], z[j]); },
        [&](int i, double s, double xc) {
            pnew[i] = xc;
            q[i] = s;
            loc[0] += xc * s;
        });
    double* const dst[1] = {rs.region(P_PQ)};
    block_store<1>(loc, dst, xcd_block());
}

template <bool SYM>
__global__ __launch_bounds__(TPB) void k_m7_update_smooth0(int n, int a, int b, const double* __restrict__ v,
                                                           const double* __restrict__ p,
                                                           const double* __restrict__ q, double* __restrict__ x,
                                                           const double* __restrict__ r, double* __restrict__ rn,
                                                           const double* __restrict__ m, double* __restrict__ u,
                                                           double* __restrict__ rv, RedScratch rs) {
    const double* sc = rs.scal();
    const bool bad = sc[S_FLAG] != 0.0;
    const double alpha = sc[S_ALPHA];
    const double step = bad ? 0.0 : alpha;
    double loc[1] = {0.0};
    march7<SYM, double>(
        n, a, b, v, [&](int j) { return m[j] * __builtin_fma(-step, q[j], r[j]); },
        [&](int i, double s, double xc) {
            const double ri = __builtin_fma(-step, q[i], r[i]);
            if (!bad) x[i] = __builtin_fma(alpha, p[i], x[i]);
            rn[i] = ri;
            u[i] = xc;
            rv[i] = ri - s;
            loc[0] += ri * ri;
        });
    double* const dst[1] = {rr_dest(rs, bad)};
    block_store<1>(loc, dst, xcd_block());
}

// ------------------------------------------------------------------ windowed form
//
// Level-0 kernels for other stencils in diagonal storage (the 27-point operator): the
// offsets fall into a few clusters (the grid planes below, at and above a row), and a
// workgroup of TPB consecutive rows stages, per cluster, the vector entries its rows
// reach through that cluster (rows [i0 + lo, i0 + TPB + lo + span)) in LDS with
// coalesced loads, so each vector entry is loaded about (TPB + span) / TPB times per
// cluster instead of once per diagonal.  The matrix entries are loaded as in dia_row
// (all before the barrier), and each row adds the same terms in the same order with the
// same fused multiply-adds, so its result is the one-row-per-thread kernels' bit for bit.

WinPlan win_plan(const std::vector<int>& offs) {
    WinPlan w;
    const int nd = (int)offs.size();
    if (nd == 0 || nd > DIA_MAX) return w;
    int k = 0, start = 0, total = 0;
    for (int d = 0; d <= nd; ++d) {
        if (d == nd || (d > start && offs[(size_t)d] - offs[(size_t)d - 1] > TPB)) {
            if (k == WIN_MAX_CL) return WinPlan{};
            w.lo[k] = offs[(size_t)start];
            w.len[k] = TPB + (offs[(size_t)d - 1] - offs[(size_t)start]);
            w.base[k] = total;
            total += w.len[k];
            for (int q = start; q < d; ++q) w.cl[q] = (unsigned char)k;
            ++k;
            start = d;
        }
    }
    if (total > WIN_CAP) return WinPlan{};
    w.ncl = k;
    w.total = total;
    // two rows per thread: windows TPB entries longer
    w.two = nd == 27 && total + k * TPB <= WIN_CAP;
    return w;
}

template <int ND, bool SYM, typename T, typename XG, typename EP>
__device__ __forceinline__ void win_rows(int n, int nd_rt, const DiaOff& o, const WinPlan& w,
                                         const T* __restrict__ v, XG xget, EP epi) {
    extern __shared__ __align__(16) unsigned char win_smem[];  // w.total entries, sized at launch
    T* X = reinterpret_cast<T*>(win_smem);
    const int nd = ND > 0 ? ND : nd_rt;
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)xcd_block() * TPB;
    for (int k = 0; k < w.ncl; ++k)
        for (int e = t; e < w.len[k]; e += TPB) {
            const int64_t j = i0 + w.lo[k] + e;
            X[w.base[k] + e] = (j >= 0 && j < n) ? xget((int)j) : T(0);
        }
    const int64_t i = i0 + t;
    const bool row = i < n;
    const int ii = row ? (int)i : 0;
    const size_t sn = (size_t)n;
    // the row's matrix entries (one-row-per-thread order; mirrored reads when symmetric)
    auto coef = [&](int d) {
        const int off = o.off[d];
        const int64_t j = i + off;
        const int jj = (j >= 0 && j < n) ? (int)j : ii;
        return (SYM && off < 0) ? v[(size_t)(nd - 1 - d) * sn + jj] : v[(size_t)d * sn + ii];
    };
    constexpr int NA = ND > 0 ? ND : 1;
    T A[NA];
    if constexpr (ND > 0) {
#pragma unroll
        for (int d = 0; d < ND; ++d) A[d] = coef(d);
    }
    __syncthreads();
    if (!row) return;
    T s = 0, xc = 0;
#pragma unroll
    for (int d = 0; d < (ND > 0 ? ND : DIA_MAX); ++d) {
        if (ND == 0 && d >= nd) break;
        const int off = o.off[d];
        const int k = w.cl[d];
        const T x = X[w.base[k] + (off - w.lo[k]) + t];
        if (off == 0) xc = x;
        const int64_t j = i + off;
        const bool in = j >= 0 && j < n;
        T a;
        if constexpr (ND > 0)
            a = A[d];
        else
            a = coef(d);
        s = in ? fmadd(a, x, s) : s;
    }
    epi((int)i, s, xc);
}

// R rows per thread (27 diagonals, R = 2): a workgroup of TPB threads owns R TPB
// consecutive rows, thread t the rows i .. i + R - 1 with i = i0 + R t, and fetches each
// diagonal's entries of its rows with one load (16 bytes in FP64, 8 in FP32): the own-row run
// (i .. i + R - 1) and, for a mirrored sub-diagonal entry, the run (i + off ..
// i + off + R - 1) of the super-diagonal, aligned to one value for any off.  The windows
// are (R - 1) TPB entries longer.  Each row adds the same terms in the same order with the
// same fused multiply-adds as win_rows, so the results are equal bit for bit.  A
// workgroup whose runs all lie inside [0, n) loads them whole (the offsets are sorted, so
// the first and last bound them); the others load entry by entry.  (Four FP32 rows per
// thread, one 16-byte load per diagonal, measured slower: 160^3 first sweep + residual
// 106 against 90 us, sweep 94 against 84; the longer windows and 130 VGPRs cost more than
// the loads saved.)
template <typename T, int R>
struct WRun {
    typedef T v __attribute__((ext_vector_type(R)));
    typedef v u __attribute__((aligned(sizeof(T))));
};

// entries j .. j + R - 1 of the diagonal array p; an entry outside [0, n) reads entry 0
// and is not used
template <int R, typename T>
__device__ __forceinline__ typename WRun<T, R>::v wp_run_edge(const T* __restrict__ p, int64_t j, int n) {
    typename WRun<T, R>::v r;
#pragma unroll
    for (int q = 0; q < R; ++q) r[q] = p[(j + q >= 0 && j + q < n) ? j + q : 0];
    return r;
}

// the R row sums step together: without this point the scheduler runs the first row's
// chain through all diagonals first and keeps the other rows' window values live (FP64,
// two rows: 226 VGPRs against 125, and half the waves per SIMD)
template <int R, typename T>
__device__ __forceinline__ void wp_step(T (&s)[R]) {
    static_assert(R == 2, "two row sums");
    asm volatile("" : "+v"(s[0]), "+v"(s[1]));
}

template <int R, int ND, bool SYM, typename T, typename XG, typename EP>
__device__ __forceinline__ void win_rows_r(int n, const DiaOff& o, const WinPlan& w, const T* __restrict__ v,
                                           XG xget, EP epi) {
    static_assert(ND > 0, "several rows per thread need the diagonal count at compile time");
    static_assert(R == 2, "two rows per thread");
    typedef typename WRun<T, R>::v PR;
    typedef typename WRun<T, R>::u PRu;
    extern __shared__ __align__(16) unsigned char win_smem[];  // w.total + (R - 1) w.ncl TPB entries
    T* X = reinterpret_cast<T*>(win_smem);
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)xcd_block() * (R * TPB);
    for (int k = 0; k < w.ncl; ++k)
        for (int e = t; e < w.len[k] + (R - 1) * TPB; e += TPB) {
            const int64_t j = i0 + w.lo[k] + e;
            X[w.base[k] + k * (R - 1) * TPB + e] = (j >= 0 && j < n) ? xget((int)j) : T(0);
        }
    const int64_t i = i0 + R * t;
    const size_t sn = (size_t)n;
    const bool inner = i0 + min(o.off[0], 0) >= 0 && i0 + R * TPB + max(o.off[ND - 1], 0) <= n;
    PR A[ND];
    if (inner) {
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const int off = o.off[d];
            A[d] = *reinterpret_cast<const PRu*>((SYM && off < 0) ? v + (size_t)(ND - 1 - d) * sn + (i + off)
                                                                 : v + (size_t)d * sn + i);
        }
    } else {
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const int off = o.off[d];
            A[d] = (SYM && off < 0) ? wp_run_edge<R>(v + (size_t)(ND - 1 - d) * sn, i + off, n)
                                    : wp_run_edge<R>(v + (size_t)d * sn, i, n);
        }
    }
    __syncthreads();
    if (i >= n) return;
    T sum[R], xc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) sum[q] = xc[q] = T(0);
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const int off = o.off[d];
        const int k = w.cl[d];
        const T* xp = X + w.base[k] + k * (R - 1) * TPB + (off - w.lo[k]) + R * t;
        const int64_t j = i + off;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const T x = xp[q];
            if (off == 0) xc[q] = x;
            sum[q] = (j + q >= 0 && j + q < n) ? fmadd(A[d][q], x, sum[q]) : sum[q];
        }
        wp_step<R>(sum);
    }
#pragma unroll
    for (int q = 0; q < R; ++q)
        if (i + q < n) epi((int)i + q, sum[q], xc[q]);
}

// The windowed row loop with R rows per thread (R > 1: win_rows_r, ND > 0).
template <int R, int ND, bool SYM, typename T, typename XG, typename EP>
__device__ __forceinline__ void win_any(int n, int nd, const DiaOff& o, const WinPlan& w, const T* __restrict__ v,
                                        XG xget, EP epi) {
    if constexpr (R > 1)
        win_rows_r<R, ND, SYM, T>(n, o, w, v, xget, epi);
    else
        win_rows<ND, SYM, T>(n, nd, o, w, v, xget, epi);
}

template <int ND, bool SYM, int R, typename T>
__global__ __launch_bounds__(TPB) void k_w_smooth0_residual(int n, int nd, DiaOff o, WinPlan w,
                                                            const T* __restrict__ v, const T* __restrict__ m,
                                                            const T* __restrict__ f, T* __restrict__ u,
                                                            T* __restrict__ r) {
    win_any<R, ND, SYM, T>(n, nd, o, w, v, [&](int j) { return m[j] * f[j]; }, [&](int i, T s, T xc) {
        u[i] = xc;
        r[i] = f[i] - s;
    });
}

template <int ND, bool SYM, int R, typename T>
__global__ __launch_bounds__(TPB) void k_w_residual(int n, int nd, DiaOff o, WinPlan w, const T* __restrict__ v,
                                                    const T* __restrict__ f, const T* __restrict__ u,
                                                    T* __restrict__ r) {
    win_any<R, ND, SYM, T>(n, nd, o, w, v, [&](int j) { return u[j]; }, [&](int i, T s, T) { r[i] = f[i] - s; });
}

template <int ND, bool SYM, int R, typename T>
__global__ __launch_bounds__(TPB) void k_w_jacobi(int n, int nd, DiaOff o, WinPlan w, const T* __restrict__ v,
                                                  const T* __restrict__ m, const T* __restrict__ f,
                                                  const T* __restrict__ u, T* __restrict__ uout) {
    win_any<R, ND, SYM, T>(n, nd, o, w, v, [&](int j) { return u[j]; },
                         [&](int i, T s, T xc) { uout[i] = xc + m[i] * (f[i] - s); });
}

template <int ND, bool SYM, int R>
__global__ __launch_bounds__(TPB) void k_w_jacobi_rz(int n, int nd, DiaOff o, WinPlan w, const double* __restrict__ v,
                                                     const double* __restrict__ m, const double* __restrict__ r,
                                                     const double* __restrict__ u, double* __restrict__ z,
                                                     int flexible, RedScratch rs) {
    double loc[2] = {0.0, 0.0};
    win_any<R, ND, SYM, double>(n, nd, o, w, v, [&](int j) { return u[j]; }, [&](int i, double s, double xc) {
        const double ri = r[i];
        const double zi = xc + m[i] * (ri - s);
        if (flexible) loc[1] += ri * z[i];
        z[i] = zi;
        loc[0] += ri * zi;
    });
    double* const dst[2] = {rs.region(P_RZ), rs.region(P_RZOLD)};
    block_store<2>(loc, dst, xcd_block());
}

// k_m7_jacobi_rz32 in the windowed form.
template <int ND, bool SYM, int R>
__global__ __launch_bounds__(TPB) void k_w_jacobi_rz32(int n, int nd, DiaOff o, WinPlan w, const float* __restrict__ v,
                                                       const float* __restrict__ m, const float* __restrict__ f,
                                                       const float* __restrict__ u, const double* __restrict__ r,
                                                       double* __restrict__ z, int flexible, RedScratch rs) {
    double loc[2] = {0.0, 0.0};
    win_any<R, ND, SYM, float>(n, nd, o, w, v, [&](int j) { return u[j]; }, [&](int i, float s, float xc) {
        const float z32 = xc + m[i] * (f[i] - s);
        const double ri = r[i];
        const double zi = (double)z32;
        if (flexible) loc[1] += ri * z[i];
        z[i] = zi;
        loc[0] += ri * zi;
    });
    double* const dst[2] = {rs.region(P_RZ), rs.region(P_RZOLD)};
    block_store<2>(loc, dst, xcd_block());
}

// k_dia_cg_init in the windowed form: r = f - A x, partials of r.r and f.f.
template <int ND, bool SYM, int R>
__global__ __launch_bounds__(TPB) void k_w_cg_init(int n, int nd, DiaOff o, WinPlan w, const double* __restrict__ v,
                                                   const double* __restrict__ f, const double* __restrict__ x,
                                                   double* __restrict__ r, RedScratch rs) {
    double loc[2] = {0.0, 0.0};
    win_any<R, ND, SYM, double>(n, nd, o, w, v, [&](int j) { return x[j]; }, [&](int i, double s, double) {
        const double fi = f[i];
        const double ri = fi - s;
        r[i] = ri;
        loc[0] += ri * ri;
        loc[1] += fi * fi;
    });
    double* const dst[2] = {rs.region(P_RR), rs.region(P_FF)};
    block_store<2>(loc, dst, xcd_block());
}

template <int ND, bool SYM, int R, bool FIRST>
__global__ __launch_bounds__(TPB) void k_w_cg_pq(int n, int nd, DiaOff o, WinPlan w, const double* __restrict__ v,
                                                 const double* __restrict__ z, const double* __restrict__ pold,
                                                 double* __restrict__ pnew, double* __restrict__ q, RedScratch rs) {
    const double beta = FIRST ? 0.0 : rs.scal()[S_BETA];
    double loc[1] = {0.0};
    win_any<R, ND, SYM, double>(
        n, nd, o, w, v, [&](int j) { return FIRST ? z[j] : __builtin_fma(beta, pold[j], z[j]); },
        [&](int i, double s, double xc) {
            pnew[i] = xc;
            q[i] = s;
            loc[0] += xc * s;
        });
    double* const dst[1] = {rs.region(P_PQ)};
    block_store<1>(loc, dst, xcd_block());
}

template <int ND, bool SYM, int R>
__global__ __launch_bounds__(TPB) void k_w_update_smooth0(int n, int nd, DiaOff o, WinPlan w,
                                                          const double* __restrict__ v, const double* __restrict__ p,
                                                          const double* __restrict__ q, double* __restrict__ x,
                                                          const double* __restrict__ r, double* __restrict__ rn,
                                                          const double* __restrict__ m, double* __restrict__ u,
                                                          double* __restrict__ rv, RedScratch rs) {
    const double* sc = rs.scal();
    const bool bad = sc[S_FLAG] != 0.0;
    const double alpha = sc[S_ALPHA];
    const double step = bad ? 0.0 : alpha;
    double loc[1] = {0.0};
    win_any<R, ND, SYM, double>(
        n, nd, o, w, v, [&](int j) { return m[j] * __builtin_fma(-step, q[j], r[j]); },
        [&](int i, double s, double xc) {
            const double ri = __builtin_fma(-step, q[i], r[i]);
            if (!bad) x[i] = __builtin_fma(alpha, p[i], x[i]);
            rn[i] = ri;
            u[i] = xc;
            rv[i] = ri - s;
            loc[0] += ri * ri;
        });
    double* const dst[1] = {rr_dest(rs, bad)};
    block_store<1>(loc, dst, xcd_block());
}

// Rows per thread of the windowed kernels: two with 27 diagonals and room for the longer
// windows (WinPlan::two, off with AMGMI_NO_WIN2), else one.
template <typename T>
inline int win_rows_per_thread(const Dia& D) {
    return (D.win.ncl > 0 && D.ndiag == 27 && D.win.two) ? 2 : 1;
}

template <typename T>
inline int win_blocks(int n, const Dia& D) {
    const int r = win_rows_per_thread<T>(D);
    return (int)(((int64_t)n + r * TPB - 1) / (r * TPB));
}

template <typename T>
inline unsigned win_bytes(const Dia& D) {
    const int r = win_rows_per_thread<T>(D);
    return (unsigned)((size_t)(D.win.total + (r - 1) * D.win.ncl * TPB) * sizeof(T));
}

// Runs f(std::integral_constant<int, ND>, std::bool_constant<SYM>,
// std::integral_constant<int, R>) for the windowed form of a kernel in T when D has one
// (ND = 27 for the 27-point stencil, else 0; R = win_rows_per_thread<T>(D), launched on
// win_blocks<T>(n, D) workgroups with win_bytes<T>(D) of LDS).
// `gains`: the kernel reads two or more FP64 vectors per neighbour (the Krylov SpMV, the
// CG update fused with the first sweep, the FP64 first sweep).  With one row per thread
// the windows win only there: the sweeps that read one vector per neighbour, and the FP32
// ones, measured faster without them (27-point, 160^3: last sweep 176 against 231 us), so
// they use one-row windows only when D.win.all is set.  With several rows per thread
// every windowed kernel is faster than one row per thread (27-point, 160^3, two rows:
// FP32 first sweep + residual 89 against 106 us, FP32 sweep 82 against 96, FP64 last
// sweep + r.z 157 against 172), so the windows are then used for all.
template <typename T, typename F>
inline bool win_call(const Dia& D, F&& f, bool gains = false) {
    const int rows = win_rows_per_thread<T>(D);
    if (D.win.ncl == 0 || !(gains || D.win.all || rows > 1)) return false;
    auto with_nd = [&](auto S) {
        if (D.ndiag == 27) {
            if (rows == 2)
                f(std::integral_constant<int, 27>{}, S, std::integral_constant<int, 2>{});
            else
                f(std::integral_constant<int, 27>{}, S, std::integral_constant<int, 1>{});
        } else {
            f(std::integral_constant<int, 0>{}, S, std::integral_constant<int, 1>{});
        }
    };
    if (D.off.sym)
        with_nd(std::true_type{});
    else
        with_nd(std::false_type{});
    return true;
}

// Runs f(std::bool_constant<SYM>) for the marching form when D has one.
template <typename F>
inline bool march_call(const Dia& D, F&& f) {
    if (D.march_a == 0) return false;
    if (D.off.sym)
        f(std::true_type{});
    else
        f(std::false_type{});
    return true;
}


template <typename T>
void launch_dia_scatter(const Csr& A, const Dia& D, const double* val, T* dval, hipStream_t s) {
    if (D.ndiag >= SC_TILE_MIN_DIAG)
        timed_launch(k_dia_scatter<T>, grid_for(A.nrows, SC_ROWS), TPB, 0, s, A.nrows, D.ndiag, A.ptr, D.slot, val, dval);
    else
        timed_launch(k_dia_scatter_rows<T>, dia_blocks(A.nrows), TPB, 0, s, A.nrows, A.ptr, D.slot, val, dval);
    HIP_LAUNCH_CHECK();
}

template <typename T>
void launch_dia_gather(const Csr& A, const Dia& D, const T* dval, T* val, hipStream_t s) {
    timed_launch(k_dia_gather_rows<T>, dia_blocks(A.nrows), TPB, 0, s, A.nrows, (const int*)A.ptr,
                 (const uint8_t*)D.slot, dval, val);
    HIP_LAUNCH_CHECK();
}
template void launch_dia_gather<double>(const Csr&, const Dia&, const double*, double*, hipStream_t);
template void launch_dia_gather<float>(const Csr&, const Dia&, const float*, float*, hipStream_t);

void launch_dia_symcheck(int n, const Dia& D, double* scal, hipStream_t s) {
    timed_launch(k_dia_clear, 1, 64, 0, s, scal + S_ASYM);
    HIP_LAUNCH_CHECK();
    if (n == 0) return;
    timed_launch(k_dia_symcheck, dia_blocks(n), TPB, 0, s, n, D.ndiag, D.off, D.val, scal + S_ASYM);
    HIP_LAUNCH_CHECK();
}

template <typename T>
void launch_dia_smooth0_residual(int n, const Dia& D, const T* m, const T* f, T* u, T* r, hipStream_t s) {
    if (march_call(D, [&](auto S) {
            timed_launch(k_m7_smooth0_residual<decltype(S)::value, T>, march_blocks(n, D.march_a), TPB, 0, s, n, D.march_a, D.march_b, D.v<T>(), m, f, u, r);
        })) {
        HIP_LAUNCH_CHECK();
        return;
    }
    if (win_call<T>(D, [&](auto K, auto S, auto R) {
            timed_launch(k_w_smooth0_residual<decltype(K)::value, decltype(S)::value, decltype(R)::value, T>, win_blocks<T>(n, D), TPB, win_bytes<T>(D), s, n, D.ndiag, D.off, D.win, D.v<T>(), m, f, u, r);
        }, std::is_same<T, double>::value)) {
        HIP_LAUNCH_CHECK();
        return;
    }
    dia_nd(D.ndiag, [&](auto K) {
        timed_launch(k_dia_smooth0_residual<T, decltype(K)::value>, dia_blocks(n), TPB, 0, s, n, D.ndiag, D.off, D.v<T>(), m, f, u, r);
    });
    HIP_LAUNCH_CHECK();
}
template <typename T>
void launch_dia_residual(int n, const Dia& D, const T* f, const T* u, T* r, hipStream_t s) {
    if (march_call(D, [&](auto S) {
            timed_launch(k_m7_residual<decltype(S)::value, T>, march_blocks(n, D.march_a), TPB, 0, s, n, D.march_a, D.march_b, D.v<T>(), f, u, r);
        })) {
        HIP_LAUNCH_CHECK();
        return;
    }
    if (win_call<T>(D, [&](auto K, auto S, auto R) {
            timed_launch(k_w_residual<decltype(K)::value, decltype(S)::value, decltype(R)::value, T>, win_blocks<T>(n, D), TPB, win_bytes<T>(D), s, n, D.ndiag, D.off, D.win, D.v<T>(), f, u, r);
        })) {
        HIP_LAUNCH_CHECK();
        return;
    }
    dia_nd(D.ndiag, [&](auto K) {
        timed_launch(k_dia_residual<T, decltype(K)::value>, dia_blocks(n), TPB, 0, s, n, D.ndiag, D.off, D.v<T>(), f, u, r);
    });
    HIP_LAUNCH_CHECK();
}
template <typename T>
void launch_dia_jacobi(int n, const Dia& D, const T* m, const T* f, const T* u, T* uout, hipStream_t s) {
    if (march_call(D, [&](auto S) {
            timed_launch(k_m7_jacobi<decltype(S)::value, T>, march_blocks(n, D.march_a), TPB, 0, s, n, D.march_a, D.march_b, D.v<T>(), m, f, u, uout);
        })) {
        HIP_LAUNCH_CHECK();
        return;
    }
    if (win_call<T>(D, [&](auto K, auto S, auto R) {
            timed_launch(k_w_jacobi<decltype(K)::value, decltype(S)::value, decltype(R)::value, T>, win_blocks<T>(n, D), TPB, win_bytes<T>(D), s, n, D.ndiag, D.off, D.win, D.v<T>(), m, f, u, uout);
        })) {
        HIP_LAUNCH_CHECK();
        return;
    }
    dia_nd(D.ndiag, [&](auto K) {
        timed_launch(k_dia_jacobi<T, decltype(K)::value>, dia_blocks(n), TPB, 0, s, n, D.ndiag, D.off, D.v<T>(), m, f, u, uout);
    });
    HIP_LAUNCH_CHECK();
}
int launch_dia_cg_init(int n, const Dia& D, const double* f, const double* x, double* r, const RedScratch& rs,
                       hipStream_t s) {
    const int nbw = win_blocks<double>(n, D);
    if (win_call<double>(D, [&](auto K, auto S, auto R) {
            if (nbw > rs.cap) throw Fail{AMG_ERR_ARG, "reduction scratch too small"};
            timed_launch(k_w_cg_init<decltype(K)::value, decltype(S)::value, decltype(R)::value>, nbw, TPB, win_bytes<double>(D), s, n, D.ndiag, D.off, D.win, D.val, f, x, r, rs);
        })) {
        HIP_LAUNCH_CHECK();
        return nbw;
    }
    const int nb = red_grid_elems(n);
    dia_nd(D.ndiag, [&](auto K) {
        timed_launch(k_dia_cg_init<decltype(K)::value>, nb, TPB, 0, s, n, D.ndiag, D.off, D.val, f, x, r, rs);
    });
    HIP_LAUNCH_CHECK();
    return nb;
}
int launch_dia_jacobi_rz(int n, const Dia& D, const double* m, const double* r, const double* u, double* z,
                         int flexible, const RedScratch& rs, hipStream_t s) {
    if (D.march_a > 0) {
        const int nb = march_blocks(n, D.march_a);
        if (nb > rs.cap) throw Fail{AMG_ERR_ARG, "reduction scratch too small"};
        march_call(D, [&](auto S) {
            timed_launch(k_m7_jacobi_rz<decltype(S)::value>, nb, TPB, 0, s, n, D.march_a, D.march_b, D.val, m, r, u, z,
                                                                   flexible, rs);
        });
        HIP_LAUNCH_CHECK();
        return nb;
    }
    const int nbw = win_blocks<double>(n, D);
    if (win_call<double>(D, [&](auto K, auto S, auto R) {
            if (nbw > rs.cap) throw Fail{AMG_ERR_ARG, "reduction scratch too small"};
            timed_launch(k_w_jacobi_rz<decltype(K)::value, decltype(S)::value, decltype(R)::value>, nbw, TPB, win_bytes<double>(D), s, n, D.ndiag, D.off, D.win, D.val, m, r, u, z, flexible, rs);
        })) {
        HIP_LAUNCH_CHECK();
        return nbw;
    }
    const int nb = (int)dia_blocks(n);
    if (nb > rs.cap) throw Fail{AMG_ERR_ARG, "reduction scratch too small"};
    dia_nd(D.ndiag, [&](auto K) {
        timed_launch(k_dia_jacobi_rz<decltype(K)::value>, nb, TPB, 0, s, n, D.ndiag, D.off, D.val, m, r, u, z, flexible, rs);
    });
    HIP_LAUNCH_CHECK();
    return nb;
}
int launch_dia_jacobi_rz32(int n, const Dia& D, const float* m, const float* f, const float* u, const double* r,
                           double* z, int flexible, const RedScratch& rs, hipStream_t s) {
    if (D.march_a > 0) {
        const int nb = march_blocks(n, D.march_a);
        if (nb > rs.cap) throw Fail{AMG_ERR_ARG, "reduction scratch too small"};
        march_call(D, [&](auto S) {
            timed_launch(k_m7_jacobi_rz32<decltype(S)::value>, nb, TPB, 0, s, n, D.march_a, D.march_b, D.val32, m, f, u,
                         r, z, flexible, rs);
        });
        HIP_LAUNCH_CHECK();
        return nb;
    }
    const int nbw = win_blocks<float>(n, D);
    if (win_call<float>(D, [&](auto K, auto S, auto R) {
            if (nbw > rs.cap) throw Fail{AMG_ERR_ARG, "reduction scratch too small"};
            timed_launch(k_w_jacobi_rz32<decltype(K)::value, decltype(S)::value, decltype(R)::value>, nbw, TPB,
                         win_bytes<float>(D), s, n, D.ndiag, D.off, D.win, D.val32, m, f, u, r, z, flexible, rs);
        })) {
        HIP_LAUNCH_CHECK();
        return nbw;
    }
    return 0;
}
int launch_dia_cg_pq(int n, const Dia& D, const double* z, const double* pold, double* pnew, double* q, int first,
                     const RedScratch& rs, hipStream_t s) {
    if (D.march_a > 0) {
        const int nb = march_blocks(n, D.march_a);
        if (nb > rs.cap) throw Fail{AMG_ERR_ARG, "reduction scratch too small"};
        march_call(D, [&](auto S) {
            constexpr bool SYM = decltype(S)::value;
            if (first)
                timed_launch(k_m7_cg_pq<SYM, true>, nb, TPB, 0, s, n, D.march_a, D.march_b, (const double*)D.val, z,
                             pold, pnew, q, rs);
            else
                timed_launch(k_m7_cg_pq<SYM, false>, nb, TPB, 0, s, n, D.march_a, D.march_b, (const double*)D.val, z,
                             pold, pnew, q, rs);
        });
        HIP_LAUNCH_CHECK();
        return nb;
    }
    const int nbw = win_blocks<double>(n, D);
    if (win_call<double>(D, [&](auto K, auto S, auto R) {
            constexpr int NDK = decltype(K)::value;
            constexpr bool SYM = decltype(S)::value;
            constexpr int RK = decltype(R)::value;
            if (nbw > rs.cap) throw Fail{AMG_ERR_ARG, "reduction scratch too small"};
            if (first)
                timed_launch(k_w_cg_pq<NDK, SYM, RK, true>, nbw, TPB, win_bytes<double>(D), s, n, D.ndiag, D.off, D.win, (const double*)D.val,
                             z, pold, pnew, q, rs);
            else
                timed_launch(k_w_cg_pq<NDK, SYM, RK, false>, nbw, TPB, win_bytes<double>(D), s, n, D.ndiag, D.off, D.win, (const double*)D.val,
                             z, pold, pnew, q, rs);
        }, true)) {
        HIP_LAUNCH_CHECK();
        return nbw;
    }
    const int nb = (int)dia_blocks(n);
    if (nb > rs.cap) throw Fail{AMG_ERR_ARG, "reduction scratch too small"};
    dia_nd(D.ndiag, [&](auto K) {
        if (first)
            timed_launch(k_dia_cg_pq<decltype(K)::value, true>, nb, TPB, 0, s, n, D.ndiag, D.off, (const double*)D.val,
                         z, pold, pnew, q, rs);
        else
            timed_launch(k_dia_cg_pq<decltype(K)::value, false>, nb, TPB, 0, s, n, D.ndiag, D.off, (const double*)D.val,
                         z, pold, pnew, q, rs);
    });
    HIP_LAUNCH_CHECK();
    return nb;
}

int launch_dia_update_smooth0(int n, const Dia& D, const double* p, const double* q, double* x, const double* r,
                              double* rn, const double* m, double* u, double* rv, const RedScratch& rs,
                              hipStream_t s) {
    if (D.march_a > 0) {
        const int nb = march_blocks(n, D.march_a);
        if (nb > rs.cap) throw Fail{AMG_ERR_ARG, "reduction scratch too small"};
        march_call(D, [&](auto S) {
            timed_launch(k_m7_update_smooth0<decltype(S)::value>, nb, TPB, 0, s, n, D.march_a, D.march_b, D.val, p, q, x, r,
                                                                        rn, m, u, rv, rs);
        });
        HIP_LAUNCH_CHECK();
        return nb;
    }
    const int nbw = win_blocks<double>(n, D);
    if (win_call<double>(D, [&](auto K, auto S, auto R) {
            if (nbw > rs.cap) throw Fail{AMG_ERR_ARG, "reduction scratch too small"};
            timed_launch(k_w_update_smooth0<decltype(K)::value, decltype(S)::value, decltype(R)::value>, nbw, TPB, win_bytes<double>(D), s, n, D.ndiag, D.off, D.win, D.val, p, q, x, r, rn, m, u, rv, rs);
        }, true)) {
        HIP_LAUNCH_CHECK();
        return nbw;
    }
    const int nb = (int)dia_blocks(n);
    if (nb > rs.cap) throw Fail{AMG_ERR_ARG, "reduction scratch too small"};
    dia_nd(D.ndiag, [&](auto K) {
        timed_launch(k_dia_update_smooth0<decltype(K)::value>, nb, TPB, 0, s, n, D.ndiag, D.off, D.val, p, q, x, r, rn, m, u, rv, rs);
    });
    HIP_LAUNCH_CHECK();
    return nb;
}

// ------------------------------------------------------------------ coarse tail
//
// The last levels of the V-cycle (Algorithm 2 from the level reached by a restriction down
// to the direct solve and back up) are small, so one workgroup runs them all, with every
// vector of those levels in LDS and __syncthreads() between the steps.  This replaces a
// dozen launches, each of which would occupy a few CUs for a few microseconds, by one.
// Rows: TAIL_G lanes each, adding their products and combining them with a butterfly.

constexpr int TAIL_THREADS = 1024;
constexpr int TAIL_G = 8;

template <typename T>
__device__ __forceinline__ T tail_row(const int* __restrict__ ptr, const int* __restrict__ col,
                                      const T* __restrict__ val, const T* x, int i, int g) {
    constexpr int U = 8;  // entries per lane loaded together
    const int b = ptr[i], e = ptr[i + 1];
    T s = 0;
    for (int k0 = b + g; k0 < e; k0 += U * TAIL_G) {
        int cc[U];
        T vv[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int k = k0 + j * TAIL_G;
            if (k < e) {
                cc[j] = col[k];
                vv[j] = val[k];
            }
        }
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (k0 + j * TAIL_G < e) s += vv[j] * x[cc[j]];
    }
    return group_sum<TAIL_G, T>(s);
}

// Block smoother product (M x)_i on a tail level with bs unknowns per node: row i of its
// node's block times the node's entries of x, in column order.
template <typename T>
__device__ __forceinline__ T tail_mblock(const T* __restrict__ m, const T* x, int i, int bs) {
    const int base = i - i % bs;
    const T* mi = m + (size_t)i * bs;
    T d = 0;
    for (int q = 0; q < bs; ++q) d = d + mi[q] * x[base + q];
    return d;
}

// One smoothing sweep u <- u + m (f - A u) on a tail level (through w); with blocks
// (bs > 1) the residual goes to w first and u <- u + M w follows.
template <typename T>
__device__ __forceinline__ void tail_sweep(const TailLevel<T>& L, int bs, const T* f, T* u, T* w, int r0, int g) {
    constexpr int RS = TAIL_THREADS / TAIL_G;
    if (bs > 1) {
        for (int i = r0; i < L.n; i += RS) {
            const T au = tail_row<T>(L.Aptr, L.Acol, L.Aval, u, i, g);
            if (g == 0) w[i] = f[i] - au;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < L.n; i += TAIL_THREADS) u[i] = u[i] + tail_mblock<T>(L.m, w, i, bs);
        __syncthreads();
        return;
    }
    for (int i = r0; i < L.n; i += RS) {
        const T au = tail_row<T>(L.Aptr, L.Acol, L.Aval, u, i, g);
        if (g == 0) w[i] = u[i] + L.m[i] * (f[i] - au);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < L.n; i += TAIL_THREADS) u[i] = w[i];
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(TAIL_THREADS) void k_vcycle_tail(TailArgs<T> a) {
    extern __shared__ __align__(16) unsigned char tail_smem[];
    T* sm = reinterpret_cast<T*>(tail_smem);  // level l: f, u, w at sm + a.lv[l].soff
    const int g = threadIdx.x & (TAIL_G - 1);
    const int r0 = threadIdx.x / TAIL_G;
    constexpr int RS = TAIL_THREADS / TAIL_G;  // rows per pass
    // restriction into the first tail level
    {
        T* f0 = sm + a.lv[0].soff;
        for (int i = r0; i < a.lv[0].n; i += RS) {
            const T v = tail_row<T>(a.rin_ptr, a.rin_col, a.rin_val, a.rin, i, g);
            if (g == 0) f0[i] = v;
        }
    }
    __syncthreads();
    for (int l = 0; l + 1 < a.nlev; ++l) {
        const TailLevel<T>& L = a.lv[l];
        const int n = L.n;
        T* f = sm + L.soff;
        T* u = f + n;
        T* w = u + n;
        // pre-smoothing from u = 0: the first sweep is u = m f (u = M f with blocks)
        for (int i = threadIdx.x; i < n; i += TAIL_THREADS)
            u[i] = a.npre > 0 ? (a.bs > 1 ? tail_mblock<T>(L.m, f, i, a.bs) : L.m[i] * f[i]) : (T)0;
        __syncthreads();
        for (int it = 1; it < a.npre; ++it) tail_sweep<T>(L, a.bs, f, u, w, r0, g);
        // residual into w, restricted to the next level
        for (int i = r0; i < n; i += RS) {
            const T au = tail_row<T>(L.Aptr, L.Acol, L.Aval, u, i, g);
            if (g == 0) w[i] = f[i] - au;
        }
        __syncthreads();
        T* fn = sm + a.lv[l + 1].soff;
        for (int i = r0; i < a.lv[l + 1].n; i += RS) {
            const T v = tail_row<T>(L.Rptr, L.Rcol, L.Rval, w, i, g);
            if (g == 0) fn[i] = v;
        }
        __syncthreads();
    }
    {
        // coarsest level: the dense inverse, applied in FP64
        const TailLevel<T>& L = a.lv[a.nlev - 1];
        const int nc = L.n;
        const T* f = sm + L.soff;
        T* u = sm + L.soff + nc;
        for (int i = r0; i < nc; i += RS) {
            double s = strided_dot<TAIL_G>(a.cinv + (size_t)i * nc, f, g, nc);
            s = group_sum<TAIL_G, double>(s);
            if (g == 0) u[i] = (T)s;
        }
        __syncthreads();
    }
    for (int l = a.nlev - 2; l >= 0; --l) {
        const TailLevel<T>& L = a.lv[l];
        const int n = L.n;
        T* f = sm + L.soff;
        T* u = f + n;
        T* w = u + n;
        const T* uc = sm + a.lv[l + 1].soff + a.lv[l + 1].n;
        for (int i = r0; i < n; i += RS) {  // u_l += P_l u_{l+1}
            const T v = tail_row<T>(L.Pptr, L.Pcol, L.Pval, uc, i, g);
            if (g == 0) u[i] = u[i] + v;
        }
        __syncthreads();
        for (int it = 0; it < a.npost; ++it) tail_sweep<T>(L, a.bs, f, u, w, r0, g);
    }
    {
        const T* u0 = sm + a.lv[0].soff + a.lv[0].n;
        for (int i = threadIdx.x; i < a.lv[0].n; i += TAIL_THREADS) a.uout[i] = u0[i];
    }
}

template <typename T>
void launch_vcycle_tail(const TailArgs<T>& a, hipStream_t s) {
    if (a.nlev < 1 || a.nlev > TAIL_MAX_LEVELS) throw Fail{AMG_ERR_ARG, "coarse tail: level count"};
    // the LDS layout: level l's f, u, w at soff, soff + n, soff + 2n
    size_t need = 0;
    for (int l = 0; l < a.nlev; ++l) {
        if ((size_t)a.lv[l].soff != need) throw Fail{AMG_ERR_ARG, "coarse tail: LDS layout"};
        need += 3 * (size_t)a.lv[l].n;
    }
    const size_t sm = need * sizeof(T);
    if (sm > TAIL_SMEM_MAX) throw Fail{AMG_ERR_ARG, "coarse tail too large"};
    timed_launch(k_vcycle_tail<T>, 1, TAIL_THREADS, sm, s, a);
    HIP_LAUNCH_CHECK();
}

#define AMG_INST(T)                                                                                 \
    template void launch_spmv<T>(const Csr&, const T*, T*, const T*, T*, hipStream_t);              \
    template void launch_residual<T>(const Csr&, const T*, const T*, T*, hipStream_t);              \
    template void launch_jacobi<T>(const Csr&, const T*, const T*, const T*, T*, hipStream_t);      \
    template void launch_smooth0_residual<T>(const Csr&, const T*, const T*, T*, T*, hipStream_t);  \
    template void launch_prolong_add<T>(const Csr&, const T*, T*, hipStream_t);                     \
    template void launch_coarse_gemv<T>(int, const double*, const T*, T*, const double*, hipStream_t); \
    template void launch_vcycle_tail<T>(const TailArgs<T>&, hipStream_t);                          \
    template void launch_dia_scatter<T>(const Csr&, const Dia&, const double*, T*, hipStream_t);    \
    template void launch_dia_smooth0_residual<T>(int, const Dia&, const T*, const T*, T*, T*, hipStream_t); \
    template void launch_dia_residual<T>(int, const Dia&, const T*, const T*, T*, hipStream_t);     \
    template void launch_dia_jacobi<T>(int, const Dia&, const T*, const T*, const T*, T*, hipStream_t);
AMG_INST(double)
AMG_INST(float)
#undef AMG_INST

// ------------------------------------------------------------------ CG kernels (FP64)
//
// Scalars flow through partial sums: the kernels that form r.z and p.q write one partial
// per block (full grids, indexed by logical block), a one-block finalize kernel adds them
// in order and forms beta or alpha on the device; ||r||^2 and ||f||^2 come from bounded
// grids (at most RED_BLOCKS partials) that the host adds after its one copy per iteration.

int red_grid_elems(int64_t n) {
    const int64_t b = (n + TPB - 1) / TPB;
    return (int)(b < 1 ? 1 : (b > RED_BLOCKS ? RED_BLOCKS : b));
}

int full_grid_rows(int nrows, int rpb, int g) {
    const int64_t b = rpb > 0 ? (nrows + (int64_t)rpb - 1) / rpb : ((int64_t)nrows * g + TPB - 1) / TPB;
    return (int)(b < 1 ? 1 : b);
}

int red_grid_rows(int nrows, int rpb, int g) {
    const int b = full_grid_rows(nrows, rpb, g);
    return b > RED_BLOCKS ? RED_BLOCKS : b;
}

// r = f - A x, with ||r||^2 and ||f||^2 partials (bounded grid, host-summed).
template <int G>
__global__ __launch_bounds__(RB_THREADS) void k_cg_init(int n, int rpb, const int* __restrict__ ptr,
                                                        const int* __restrict__ col, const double* __restrict__ val,
                                                        const double* __restrict__ f, const double* __restrict__ x,
                                                        double* __restrict__ r, RedScratch rs) {
    __shared__ int sptr[RB_THREADS + 1];
    __shared__ double sp[RB_CAP];
    double loc[2] = {0.0, 0.0};
    if (rpb > 0) {
        int rb0, rb1;
        rb_range((n + rpb - 1) / rpb, rb0, rb1);
        const int tpr = rb_tpr(rpb), t = threadIdx.x / tpr, lane = threadIdx.x & (tpr - 1);
        for (int rb = rb0; rb < rb1; ++rb) {
            const int row0 = rb * rpb, row1 = min(row0 + rpb, n);
            rb_load(row0, row1, ptr, col, val, [&](int j) { return x[j]; }, sptr, sp);
            if (t < row1 - row0) {
                const double v = rb_rowsum(sptr, sp, t, lane, tpr);
                if (lane == 0) {
                    const int i = row0 + t;
                    const double fi = f[i], ri = fi - v;
                    r[i] = ri;
                    loc[0] += ri * ri;
                    loc[1] += fi * fi;
                }
            }
            __syncthreads();
        }
    } else {
        const int lane = threadIdx.x & (G - 1);
        const int groups = gridDim.x * (TPB / G);
        for (int row = (blockIdx.x * TPB + (int)threadIdx.x) / G; row < n; row += groups) {
            const int b = ptr[row], e = ptr[row + 1];
            double s = 0.0;
            for (int k = b + lane; k < e; k += G) s += val[k] * x[col[k]];
            s = group_sum<G>(s);
            if (lane == 0) {
                const double fi = f[row], ri = fi - s;
                r[row] = ri;
                loc[0] += ri * ri;
                loc[1] += fi * fi;
            }
        }
    }
    double* const dst[2] = {rs.region(P_RR), rs.region(P_FF)};
    block_store<2>(loc, dst, blockIdx.x);
}

// Last post-smoothing sweep of the level-0 V-cycle (FP64) fused with the CG dot products:
// z = u + m (r - A u) (the level-0 right-hand side is the CG residual r), r.z and, for
// flexible CG, r.z_old with z_old read from z before it is overwritten.  Full grid.
template <int G>
__global__ __launch_bounds__(RB_THREADS) void k_jacobi_rz(int n, int rpb, const int* __restrict__ ptr,
                                                          const int* __restrict__ col, const double* __restrict__ val,
                                                          const double* __restrict__ m, const double* __restrict__ r,
                                                          const double* __restrict__ u, double* __restrict__ z,
                                                          int flexible, RedScratch rs) {
    __shared__ int sptr[RB_THREADS + 1];
    __shared__ double sp[RB_CAP];
    double loc[2] = {0.0, 0.0};
    auto emit = [&](int i, double s) {
        const double ri = r[i];
        const double zi = u[i] + m[i] * (ri - s);
        if (flexible) loc[1] += ri * z[i];
        z[i] = zi;
        loc[0] += ri * zi;
    };
    const int lb = xcd_block();
    if (rpb > 0) {
        const int row0 = lb * rpb, row1 = min(row0 + rpb, n);
        rb_load(row0, row1, ptr, col, val, [&](int j) { return u[j]; }, sptr, sp);
        const int tpr = rb_tpr(rpb), t = threadIdx.x / tpr, lane = threadIdx.x & (tpr - 1);
        if (t < row1 - row0) {
            const double v = rb_rowsum(sptr, sp, t, lane, tpr);
            if (lane == 0) emit(row0 + t, v);
        }
    } else {
        const int lane = threadIdx.x & (G - 1);
        const int row = (lb * TPB + (int)threadIdx.x) / G;
        if (row < n) {
            const int b = ptr[row], e = ptr[row + 1];
            double s = 0.0;
            for (int k = b + lane; k < e; k += G) s += val[k] * u[col[k]];
            s = group_sum<G>(s);
            if (lane == 0) emit(row, s);
        }
    }
    double* const dst[2] = {rs.region(P_RZ), rs.region(P_RZOLD)};
    block_store<2>(loc, dst, lb);
}

// Mixed precision: z = (double) z32 fused with the same dot products (bounded grid).
__global__ __launch_bounds__(TPB) void k_cast_rz(int n, const float* __restrict__ z32, const double* __restrict__ r,
                                                 double* __restrict__ z, int flexible, RedScratch rs) {
    double loc[2] = {0.0, 0.0};
    for (int i = blockIdx.x * TPB + threadIdx.x; i < n; i += gridDim.x * TPB) {
        const double ri = r[i];
        const double zi = (double)z32[i];
        if (flexible) loc[1] += ri * z[i];
        z[i] = zi;
        loc[0] += ri * zi;
    }
    double* const dst[2] = {rs.region(P_RZ), rs.region(P_RZOLD)};
    block_store<2>(loc, dst, blockIdx.x);
}

// r.z (used when the V-cycle has no post-smoothing sweep to fuse it into).
__global__ __launch_bounds__(TPB) void k_cg_rz(int n, const double* __restrict__ r, const double* __restrict__ z,
                                               RedScratch rs) {
    double loc[1] = {0.0};
    for (int i = blockIdx.x * TPB + threadIdx.x; i < n; i += gridDim.x * TPB) loc[0] += r[i] * z[i];
    double* const dst[1] = {rs.region(P_RZ)};
    block_store<1>(loc, dst, blockIdx.x);
}

// rho_new = sum of the r.z partials; beta = (rho_new [- r.z_old]) / rho_old with rho_old
// the rho of the last alpha (so re-running it after a restart is harmless); rho = rho_new.
__global__ __launch_bounds__(FIN_THREADS) void k_fin_rz(int nb, int flexible, int first, RedScratch rs) {
    const double rz = block_sum(rs.region(P_RZ), nb);
    const double rzo = flexible ? block_sum(rs.region(P_RZOLD), nb) : 0.0;
    if (threadIdx.x == 0) {
        double* sc = rs.scal();
        sc[S_BETA] = first ? 0.0 : (flexible ? rz - rzo : rz) / sc[S_RHO_USED];
        sc[S_RHO] = rz;
    }
}

// p.q = sum of its partials; alpha = rho / p.q, or the breakdown flag (p.q <= 0 or a
// non-finite rho), in which case alpha = 0.
__global__ __launch_bounds__(FIN_THREADS) void k_fin_pq(int nb, RedScratch rs) {
    const double pq = block_sum(rs.region(P_PQ), nb);
    if (threadIdx.x == 0) {
        double* sc = rs.scal();
        const double rho = sc[S_RHO];
        const bool bad = !(pq > 0.0) || !isfinite(rho);
        sc[S_RHO_USED] = rho;
        sc[S_PQ] = pq;
        sc[S_ALPHA] = bad ? 0.0 : rho / pq;
        sc[S_FLAG] = bad ? 1.0 : 0.0;
    }
}

// p_new = z + beta p_old (p_new = z on the first iteration), q = A p_new, p_new.q partials
// (full grid).  Neighbours' p_new entries are formed with the same fma as the owner row,
// so q is A applied to exactly the stored p_new.
template <int G>
__global__ __launch_bounds__(RB_THREADS) void k_cg_pq(int n, int rpb, const int* __restrict__ ptr,
                                                      const int* __restrict__ col, const double* __restrict__ val,
                                                      const double* __restrict__ z, const double* __restrict__ pold,
                                                      double* __restrict__ pnew, double* __restrict__ q, int first,
                                                      RedScratch rs) {
    __shared__ int sptr[RB_THREADS + 1];
    __shared__ double sp[RB_CAP];
    const double beta = first ? 0.0 : rs.scal()[S_BETA];
    auto pv = [&](int j) { return first ? z[j] : __builtin_fma(beta, pold[j], z[j]); };
    double loc[1] = {0.0};
    const int lb = xcd_block();
    if (rpb > 0) {
        const int row0 = lb * rpb, row1 = min(row0 + rpb, n);
        rb_load(row0, row1, ptr, col, val, pv, sptr, sp);
        const int tpr = rb_tpr(rpb), t = threadIdx.x / tpr, lane = threadIdx.x & (tpr - 1);
        if (t < row1 - row0) {
            const double qi = rb_rowsum(sptr, sp, t, lane, tpr);
            if (lane == 0) {
                const int i = row0 + t;
                const double pi = pv(i);
                pnew[i] = pi;
                q[i] = qi;
                loc[0] += pi * qi;
            }
        }
    } else {
        const int lane = threadIdx.x & (G - 1);
        const int row = (lb * TPB + (int)threadIdx.x) / G;
        if (row < n) {
            const int b = ptr[row], e = ptr[row + 1];
            double s = 0.0;
            for (int k = b + lane; k < e; k += G) s += val[k] * pv(col[k]);
            s = group_sum<G>(s);
            if (lane == 0) {
                const double pi = pv(row);
                pnew[row] = pi;
                q[row] = s;
                loc[0] += pi * s;
            }
        }
    }
    double* const dst[1] = {rs.region(P_PQ)};
    block_store<1>(loc, dst, lb);
}

// x += alpha p; r -= alpha q; ||r||^2 partials (bounded grid).  On breakdown nothing moves.
__global__ __launch_bounds__(TPB) void k_cg_update(int n, const double* __restrict__ p, const double* __restrict__ q,
                                                   double* __restrict__ x, double* __restrict__ r, RedScratch rs) {
    const double* sc = rs.scal();
    const bool bad = sc[S_FLAG] != 0.0;
    const double alpha = sc[S_ALPHA];
    double loc[1] = {0.0};
    for (int i = blockIdx.x * TPB + threadIdx.x; i < n; i += gridDim.x * TPB) {
        double ri = r[i];
        if (!bad) {
            x[i] = __builtin_fma(alpha, p[i], x[i]);
            ri = __builtin_fma(-alpha, q[i], ri);
            r[i] = ri;
        }
        loc[0] += ri * ri;
    }
    double* const dst[1] = {rr_dest(rs, bad)};
    block_store<1>(loc, dst, blockIdx.x);
}

// The same update, also storing r in FP32 for the mixed-precision V-cycle (bounded grid).
__global__ __launch_bounds__(TPB) void k_cg_update_cast(int n, const double* __restrict__ p,
                                                        const double* __restrict__ q, double* __restrict__ x,
                                                        double* __restrict__ r, float* __restrict__ r32,
                                                        RedScratch rs) {
    const double* sc = rs.scal();
    const bool bad = sc[S_FLAG] != 0.0;
    const double alpha = sc[S_ALPHA];
    double loc[1] = {0.0};
    for (int i = blockIdx.x * TPB + threadIdx.x; i < n; i += gridDim.x * TPB) {
        double ri = r[i];
        if (!bad) {
            x[i] = __builtin_fma(alpha, p[i], x[i]);
            ri = __builtin_fma(-alpha, q[i], ri);
            r[i] = ri;
        }
        r32[i] = (float)ri;
        loc[0] += ri * ri;
    }
    double* const dst[1] = {rr_dest(rs, bad)};
    block_store<1>(loc, dst, blockIdx.x);
}

int launch_cg_init(const Csr& A, const double* val, const double* f, const double* x, double* r, const RedScratch& rs,
                   hipStream_t s) {
    const int nb = red_grid_rows(A.nrows, A.rpb, A.g);
    AMG_WITH_G(A.g, timed_launch(k_cg_init<G>, nb, RB_THREADS, 0, s, A.nrows, A.rpb, A.ptr, A.col, val, f, x, r, rs));
    HIP_LAUNCH_CHECK();
    return nb;
}
int launch_jacobi_rz(const Csr& A, const double* m, const double* r, const double* u, double* z, int flexible,
                     const RedScratch& rs, hipStream_t s) {
    const int nb = full_grid_rows(A.nrows, A.rpb, A.g);
    if (nb > rs.cap) throw Fail{AMG_ERR_ARG, "reduction scratch too small"};
    AMG_WITH_G(A.g, timed_launch(k_jacobi_rz<G>, nb, RB_THREADS, 0, s, A.nrows, A.rpb, A.ptr, A.col, A.val, m, r, u, z, flexible, rs));
    HIP_LAUNCH_CHECK();
    return nb;
}
int launch_cast_rz(int n, const float* z32, const double* r, double* z, int flexible, const RedScratch& rs,
                   hipStream_t s) {
    const int nb = red_grid_elems(n);
    timed_launch(k_cast_rz, nb, TPB, 0, s, n, z32, r, z, flexible, rs);
    HIP_LAUNCH_CHECK();
    return nb;
}
int launch_cg_rz(int n, const double* r, const double* z, const RedScratch& rs, hipStream_t s) {
    const int nb = red_grid_elems(n);
    timed_launch(k_cg_rz, nb, TPB, 0, s, n, r, z, rs);
    HIP_LAUNCH_CHECK();
    return nb;
}
void launch_fin_rz(int nb, int flexible, int first, const RedScratch& rs, hipStream_t s) {
    timed_launch(k_fin_rz, 1, FIN_THREADS, 0, s, nb, flexible, first, rs);
    HIP_LAUNCH_CHECK();
}
void launch_fin_pq(int nb, const RedScratch& rs, hipStream_t s) {
    timed_launch(k_fin_pq, 1, FIN_THREADS, 0, s, nb, rs);
    HIP_LAUNCH_CHECK();
}
int launch_cg_pq(const Csr& A, const double* val, const double* z, const double* pold, double* pnew, double* q,
                 int first, const RedScratch& rs, hipStream_t s) {
    const int nb = full_grid_rows(A.nrows, A.rpb, A.g);
    if (nb > rs.cap) throw Fail{AMG_ERR_ARG, "reduction scratch too small"};
    AMG_WITH_G(A.g, timed_launch(k_cg_pq<G>, nb, RB_THREADS, 0, s, A.nrows, A.rpb, (const int*)A.ptr, (const int*)A.col,
                                 val, z, pold, pnew, q, first, rs));
    HIP_LAUNCH_CHECK();
    return nb;
}
int launch_cg_update(int n, const double* p, const double* q, double* x, double* r, const RedScratch& rs,
                     hipStream_t s) {
    const int nb = red_grid_elems(n);
    timed_launch(k_cg_update, nb, TPB, 0, s, n, p, q, x, r, rs);
    HIP_LAUNCH_CHECK();
    return nb;
}
int launch_cg_update_cast(int n, const double* p, const double* q, double* x, double* r, float* r32,
                          const RedScratch& rs, hipStream_t s) {
    const int nb = red_grid_elems(n);
    timed_launch(k_cg_update_cast, nb, TPB, 0, s, n, p, q, x, r, r32, rs);
    HIP_LAUNCH_CHECK();
    return nb;
}

}  // namespace amgmi
