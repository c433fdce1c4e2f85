// kernels_solve.hip -- V-cycle (Algorithm 2) and preconditioned-CG kernels for gfx950.
//
// Row kernels give each CSR row a group of G lanes (G a power of two dividing the
// 64-wide wavefront, picked per matrix from its mean row length): the G lanes read the
// row's entries contiguously, gather x, and reduce with a butterfly of cross-lane
// shuffles.  Every kernel is bandwidth bound (about 0.17 flop per byte), so the design
// goals are coalesced CSR streams, few passes over the vectors, and XCD-local gathers.
#include "amg_internal.h"

namespace amgmi {

constexpr int TPB = 256;

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

static inline unsigned row_blocks(int64_t rows, int G) {
    int64_t b = (rows * G + TPB - 1) / TPB;
    return (unsigned)(b > 0 ? b : 1);
}

// Row handled by this lane group (XCD-local block order), and the lane within it.
template <int G>
__device__ __forceinline__ int group_row(int& lane) {
    lane = threadIdx.x & (G - 1);
    return (xcd_block() * TPB + (int)threadIdx.x) / G;
}

// ------------------------------------------------------------------ SpMV family

template <int G, typename T>
__global__ __launch_bounds__(TPB) void k_spmv(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                                              const T* __restrict__ val, const T* __restrict__ x,
                                              T* __restrict__ y) {
    int lane;
    const int row = group_row<G>(lane);
    if (row >= n) return;
    const int b = ptr[row], e = ptr[row + 1];
    T s = 0;
    for (int k = b + lane; k < e; k += G) s += val[k] * x[col[k]];
    s = group_sum<G>(s);
    if (lane == 0) y[row] = s;
}

// r = f - A u
template <int G, typename T>
__global__ __launch_bounds__(TPB) void k_residual(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                                                  const T* __restrict__ val, const T* __restrict__ f,
                                                  const T* __restrict__ u, T* __restrict__ r) {
    int lane;
    const int row = group_row<G>(lane);
    if (row >= n) return;
    const int b = ptr[row], e = ptr[row + 1];
    T s = 0;
    for (int k = b + lane; k < e; k += G) s += val[k] * u[col[k]];
    s = group_sum<G>(s);
    if (lane == 0) r[row] = f[row] - s;
}

// One damped-Jacobi / SPAI0 sweep: uout = u + m (f - A u)
template <int G, typename T>
__global__ __launch_bounds__(TPB) void k_jacobi(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                                                const T* __restrict__ val, const T* __restrict__ m,
                                                const T* __restrict__ f, const T* __restrict__ u,
                                                T* __restrict__ uout) {
    int lane;
    const int row = group_row<G>(lane);
    if (row >= n) return;
    const int b = ptr[row], e = ptr[row + 1];
    T s = 0;
    for (int k = b + lane; k < e; k += G) s += val[k] * u[col[k]];
    s = group_sum<G>(s);
    if (lane == 0) uout[row] = u[row] + m[row] * (f[row] - s);
}

// First pre-smoothing sweep from u = 0 (u = m f) fused with the residual r = f - A u:
// the neighbours' u_j = m_j f_j are recomputed from m and f instead of re-read.
template <int G, typename T>
__global__ __launch_bounds__(TPB) void k_smooth0_residual(int n, const int* __restrict__ ptr,
                                                          const int* __restrict__ col, const T* __restrict__ val,
                                                          const T* __restrict__ m, const T* __restrict__ f,
                                                          T* __restrict__ u, T* __restrict__ r) {
    int lane;
    const int row = group_row<G>(lane);
    if (row >= n) return;
    const int b = ptr[row], e = ptr[row + 1];
    T s = 0;
    for (int k = b + lane; k < e; k += G) {
        const int j = col[k];
        s += val[k] * (m[j] * f[j]);
    }
    s = group_sum<G>(s);
    if (lane == 0) {
        const T fi = f[row];
        u[row] = m[row] * fi;
        r[row] = fi - s;
    }
}

// u += P uc (coarse-grid correction)
template <int G, typename T>
__global__ __launch_bounds__(TPB) void k_prolong_add(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                                                     const T* __restrict__ val, const T* __restrict__ uc,
                                                     T* __restrict__ u) {
    int lane;
    const int row = group_row<G>(lane);
    if (row >= n) return;
    const int b = ptr[row], e = ptr[row + 1];
    T s = 0;
    for (int k = b + lane; k < e; k += G) s += val[k] * uc[col[k]];
    s = group_sum<G>(s);
    if (lane == 0) u[row] += s;
}

// u = A^{-1} f on the coarsest level: one wavefront per row of the dense FP64 inverse.
template <typename T>
__global__ __launch_bounds__(TPB) void k_coarse_gemv(int n, const double* __restrict__ inv, const T* __restrict__ f,
                                                     T* __restrict__ u) {
    const int lane = threadIdx.x & 63;
    const int row = (blockIdx.x * TPB + (int)threadIdx.x) >> 6;
    if (row >= n) return;
    const double* a = inv + (size_t)row * n;
    double s = 0.0;
    for (int j = lane; j < n; j += 64) s += a[j] * (double)f[j];
    s = wave_sum(s);
    if (lane == 0) u[row] = (T)s;
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

template <typename T>
void launch_spmv(const Csr& A, int g, const T* x, T* y, hipStream_t s) {
    AMG_WITH_G(g, k_spmv<G, T><<<row_blocks(A.nrows, G), TPB, 0, s>>>(A.nrows, A.ptr, A.col, A.v<T>(), x, y));
    HIP_LAUNCH_CHECK();
}
template <typename T>
void launch_residual(const Csr& A, int g, const T* f, const T* u, T* r, hipStream_t s) {
    AMG_WITH_G(g, k_residual<G, T><<<row_blocks(A.nrows, G), TPB, 0, s>>>(A.nrows, A.ptr, A.col, A.v<T>(), f, u, r));
    HIP_LAUNCH_CHECK();
}
template <typename T>
void launch_jacobi(const Csr& A, int g, const T* m, const T* f, const T* u, T* uout, hipStream_t s) {
    AMG_WITH_G(g, k_jacobi<G, T><<<row_blocks(A.nrows, G), TPB, 0, s>>>(A.nrows, A.ptr, A.col, A.v<T>(), m, f, u, uout));
    HIP_LAUNCH_CHECK();
}
template <typename T>
void launch_smooth0_residual(const Csr& A, int g, const T* m, const T* f, T* u, T* r, hipStream_t s) {
    AMG_WITH_G(g, k_smooth0_residual<G, T><<<row_blocks(A.nrows, G), TPB, 0, s>>>(A.nrows, A.ptr, A.col, A.v<T>(), m, f, u, r));
    HIP_LAUNCH_CHECK();
}
template <typename T>
void launch_prolong_add(const Csr& P, int g, const T* uc, T* u, hipStream_t s) {
    AMG_WITH_G(g, k_prolong_add<G, T><<<row_blocks(P.nrows, G), TPB, 0, s>>>(P.nrows, P.ptr, P.col, P.v<T>(), uc, u));
    HIP_LAUNCH_CHECK();
}
template <typename T>
void launch_coarse_gemv(int n, const double* inv, const T* f, T* u, hipStream_t s) {
    k_coarse_gemv<T><<<row_blocks(n, 64), TPB, 0, s>>>(n, inv, f, u);
    HIP_LAUNCH_CHECK();
}
void launch_cast_d2f(int64_t n, const double* a, float* b, hipStream_t s) {
    k_cast_d2f<<<ew_blocks(n), TPB, 0, s>>>(n, a, b);
    HIP_LAUNCH_CHECK();
}
void launch_cast_f2d(int64_t n, const float* a, double* b, hipStream_t s) {
    k_cast_f2d<<<ew_blocks(n), TPB, 0, s>>>(n, a, b);
    HIP_LAUNCH_CHECK();
}
void launch_copy(int64_t n, const double* a, double* b, hipStream_t s) {
    k_copy<<<ew_blocks(n), TPB, 0, s>>>(n, a, b);
    HIP_LAUNCH_CHECK();
}

#define AMG_INST(T)                                                                                      \
    template void launch_spmv<T>(const Csr&, int, const T*, T*, hipStream_t);                            \
    template void launch_residual<T>(const Csr&, int, const T*, const T*, T*, hipStream_t);              \
    template void launch_jacobi<T>(const Csr&, int, const T*, const T*, const T*, T*, hipStream_t);      \
    template void launch_smooth0_residual<T>(const Csr&, int, const T*, const T*, T*, T*, hipStream_t);  \
    template void launch_prolong_add<T>(const Csr&, int, const T*, T*, hipStream_t);                     \
    template void launch_coarse_gemv<T>(int, const double*, const T*, T*, hipStream_t);
AMG_INST(double)
AMG_INST(float)
#undef AMG_INST

// ------------------------------------------------------------------ reductions
//
// Each kernel below runs on a grid of min(RED_BLOCKS, rows needed) blocks, fixed for a
// given n.  A block sums its threads' partials in a fixed tree, writes one partial per
// block, and the last block to arrive (ticket counter) adds the partials in block order.
// The result is therefore bitwise reproducible run to run.

template <int K>
__device__ bool block_reduce_last(double (&v)[K], const RedScratch rs, double (&tot)[K]) {
    __shared__ double sm[K][RED_THREADS / 64];
    __shared__ int is_last;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        double x = wave_sum(v[q]);
        if (lane == 0) sm[q][w] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            double s = 0.0;
            for (int i = 0; i < RED_THREADS / 64; ++i) s += sm[q][i];
            rs.part[q * RED_BLOCKS + blockIdx.x] = s;
        }
        __threadfence();
        const unsigned t = atomicAdd(rs.ticket, 1u);
        is_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
#pragma unroll
    for (int q = 0; q < K; ++q) {
        double s = 0.0;
        for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x)
            s += __hip_atomic_load(&rs.part[q * RED_BLOCKS + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s = wave_sum(s);
        __syncthreads();
        if (lane == 0) sm[q][w] = s;
        __syncthreads();
        double t = 0.0;
        for (int i = 0; i < RED_THREADS / 64; ++i) t += sm[q][i];
        tot[q] = t;
    }
    if (threadIdx.x == 0) *rs.ticket = 0u;
    return true;
}

static inline unsigned red_blocks(int64_t rows, int G) {
    int64_t b = (rows * G + RED_THREADS - 1) / RED_THREADS;
    if (b > RED_BLOCKS) b = RED_BLOCKS;
    return (unsigned)(b > 0 ? b : 1);
}

// r = f - A x with ||r||^2 and ||f||^2.
template <int G>
__global__ __launch_bounds__(RED_THREADS) void k_cg_init(int n, const int* __restrict__ ptr,
                                                         const int* __restrict__ col, const double* __restrict__ val,
                                                         const double* __restrict__ f, const double* __restrict__ x,
                                                         double* __restrict__ r, RedScratch rs) {
    const int lane = threadIdx.x & (G - 1);
    const int groups = gridDim.x * (RED_THREADS / G);
    double loc[2] = {0.0, 0.0};
    for (int row = (blockIdx.x * RED_THREADS + (int)threadIdx.x) / G; row < n; row += groups) {
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
    double tot[2];
    if (block_reduce_last<2>(loc, rs, tot) && threadIdx.x == 0) {
        rs.scal[S_RR] = tot[0];
        rs.scal[S_FF] = tot[1];
    }
}

// rho_new = r.z (and r.z_old for flexible CG); beta = (rho_new [- r.z_old]) / rho_old.
__global__ __launch_bounds__(RED_THREADS) void k_cg_rz(int n, const double* __restrict__ r,
                                                       const double* __restrict__ z,
                                                       const double* __restrict__ zold, int flexible, int first,
                                                       RedScratch rs) {
    double loc[2] = {0.0, 0.0};
    for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += gridDim.x * RED_THREADS) {
        loc[0] += r[i] * z[i];
        if (flexible) loc[1] += r[i] * zold[i];
    }
    double tot[2];
    if (block_reduce_last<2>(loc, rs, tot) && threadIdx.x == 0) {
        if (!first) {
            const double num = flexible ? tot[0] - tot[1] : tot[0];
            rs.scal[S_BETA] = num / rs.scal[S_RHO];
        }
        rs.scal[S_RHO] = tot[0];
    }
}

// p_new = z + beta p_old (p_new = z on the first iteration), q = A p_new, and p_new.q.
// Neighbours' p_new entries are formed from z and p_old with the same fma as the owner
// row, so q is exactly A applied to the stored p_new.
template <int G>
__global__ __launch_bounds__(RED_THREADS) void k_cg_pq(int n, const int* __restrict__ ptr,
                                                       const int* __restrict__ col, const double* __restrict__ val,
                                                       const double* __restrict__ z, const double* __restrict__ pold,
                                                       double* __restrict__ pnew, double* __restrict__ q, int first,
                                                       RedScratch rs) {
    const int lane = threadIdx.x & (G - 1);
    const int groups = gridDim.x * (RED_THREADS / G);
    const double beta = first ? 0.0 : rs.scal[S_BETA];
    double loc[1] = {0.0};
    for (int row = (blockIdx.x * RED_THREADS + (int)threadIdx.x) / G; row < n; row += groups) {
        const int b = ptr[row], e = ptr[row + 1];
        double s = 0.0;
        if (first) {
            for (int k = b + lane; k < e; k += G) s += val[k] * z[col[k]];
        } else {
            for (int k = b + lane; k < e; k += G) {
                const int j = col[k];
                s += val[k] * __builtin_fma(beta, pold[j], z[j]);
            }
        }
        s = group_sum<G>(s);
        if (lane == 0) {
            const double pi = first ? z[row] : __builtin_fma(beta, pold[row], z[row]);
            pnew[row] = pi;
            q[row] = s;
            loc[0] += pi * s;
        }
    }
    double tot[1];
    if (block_reduce_last<1>(loc, rs, tot) && threadIdx.x == 0) rs.scal[S_PQ] = tot[0];
}

// alpha = rho / p.q; x += alpha p; r -= alpha q; ||r||^2.  On breakdown (p.q <= 0 or a
// non-finite rho) nothing is updated and the flag is raised.
__global__ __launch_bounds__(RED_THREADS) void k_cg_update(int n, const double* __restrict__ p,
                                                           const double* __restrict__ q, double* __restrict__ x,
                                                           double* __restrict__ r, RedScratch rs) {
    const double rho = rs.scal[S_RHO], pq = rs.scal[S_PQ];
    const bool bad = !(pq > 0.0) || !isfinite(rho);
    const double alpha = bad ? 0.0 : rho / pq;
    double loc[1] = {0.0};
    for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += gridDim.x * RED_THREADS) {
        double ri = r[i];
        if (!bad) {
            x[i] += alpha * p[i];
            ri -= alpha * q[i];
            r[i] = ri;
        }
        loc[0] += ri * ri;
    }
    double tot[1];
    if (block_reduce_last<1>(loc, rs, tot) && threadIdx.x == 0) {
        rs.scal[S_RR] = tot[0];
        rs.scal[S_FLAG] = bad ? 1.0 : 0.0;
    }
}

void launch_cg_init(const Csr& A, const double* outer_val, int g, const double* f, const double* x, double* r,
                    const RedScratch& rs, hipStream_t s) {
    AMG_WITH_G(g, k_cg_init<G><<<red_blocks(A.nrows, G), RED_THREADS, 0, s>>>(A.nrows, A.ptr, A.col, outer_val, f, x, r, rs));
    HIP_LAUNCH_CHECK();
}
void launch_cg_rz(int n, const double* r, const double* z, const double* zold, int flexible, int first,
                  const RedScratch& rs, hipStream_t s) {
    k_cg_rz<<<red_blocks(n, 1), RED_THREADS, 0, s>>>(n, r, z, zold, flexible, first, rs);
    HIP_LAUNCH_CHECK();
}
void launch_cg_pq(const Csr& A, const double* outer_val, int g, const double* z, const double* pold, double* pnew,
                  double* q, int first, const RedScratch& rs, hipStream_t s) {
    AMG_WITH_G(g, k_cg_pq<G><<<red_blocks(A.nrows, G), RED_THREADS, 0, s>>>(A.nrows, A.ptr, A.col, outer_val, z, pold, pnew, q, first, rs));
    HIP_LAUNCH_CHECK();
}
void launch_cg_update(int n, const double* p, const double* q, double* x, double* r, const RedScratch& rs,
                      hipStream_t s) {
    k_cg_update<<<red_blocks(n, 1), RED_THREADS, 0, s>>>(n, p, q, x, r, rs);
    HIP_LAUNCH_CHECK();
}

}  // namespace amgmi
