// BiCGStab vector kernels (FP64): the paper's Krylov method for its non-symmetric
// systems (van der Vorst's BiCGStab, the V-cycle applied on the right).  The matrix
// products go through the level-0 SpMV launcher and the preconditioner through the
// V-cycle; these kernels do the vector updates and the dot products.  Every dot product
// is reduced deterministically: a bounded grid, each thread adding its entries in index
// order, a fixed wavefront and workgroup tree, one partial per workgroup written to
// mapped host memory, which the host adds in workgroup order.
#include "amg_internal.h"

namespace amgmi {

namespace {

constexpr int KT = 256;  // threads per workgroup

__device__ __forceinline__ double kwave_sum(double s) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}

// Workgroup sums of K values; thread 0 writes them to part[q * nb + blockIdx.x].
template <int K>
__device__ __forceinline__ void kblock_store(double (&v)[K], double* part, int nb) {
    __shared__ double sm[K][KT / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const double x = kwave_sum(v[q]);
        if (lane == 0) sm[q][w] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            double s = 0.0;
            for (int i = 0; i < KT / 64; ++i) s += sm[q][i];
            part[(size_t)q * nb + blockIdx.x] = s;
        }
    }
}

// Entries i, i + stride, ... of this thread; each workgroup covers a contiguous range
// of rows so that its partial is the sum over that range.
struct Range {
    int64_t b, e;
};
__device__ __forceinline__ Range block_range(int64_t n) {
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t b = per * blockIdx.x;
    return {b < n ? b : n, b + per < n ? b + per : n};
}

// r = f - y (y = A x), partials r.r and f.f
__global__ __launch_bounds__(KT) void k_bi_residual(int64_t n, const double* __restrict__ f,
                                                     const double* __restrict__ y, double* __restrict__ r,
                                                     double* __restrict__ part) {
    const Range R = block_range(n);
    double loc[2] = {0.0, 0.0};
    for (int64_t i = R.b + threadIdx.x; i < R.e; i += KT) {
        const double fi = f[i];
        const double ri = fi - y[i];
        r[i] = ri;
        loc[0] += ri * ri;
        loc[1] += fi * fi;
    }
    kblock_store<2>(loc, part, gridDim.x);
}

// partials a.b (and c.d when c != nullptr)
__global__ __launch_bounds__(KT) void k_bi_dots(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                                                 const double* __restrict__ c, const double* __restrict__ d,
                                                 double* __restrict__ part) {
    const Range R = block_range(n);
    double loc[2] = {0.0, 0.0};
    for (int64_t i = R.b + threadIdx.x; i < R.e; i += KT) {
        loc[0] += a[i] * b[i];
        if (c != nullptr) loc[1] += c[i] * d[i];
    }
    kblock_store<2>(loc, part, gridDim.x);
}

// p = r (first step) or p = r + beta (p - omega v)
__global__ __launch_bounds__(KT) void k_bi_direction(int64_t n, const double* __restrict__ r,
                                                      const double* __restrict__ v, double beta, double omega,
                                                      int first, double* __restrict__ p) {
    for (int64_t i = blockIdx.x * (int64_t)KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT)
        p[i] = first ? r[i] : r[i] + beta * (p[i] - omega * v[i]);
}

// s = r - alpha v, partial s.s
__global__ __launch_bounds__(KT) void k_bi_half(int64_t n, const double* __restrict__ r, const double* __restrict__ v,
                                                 double alpha, double* __restrict__ s, double* __restrict__ part) {
    const Range R = block_range(n);
    double loc[2] = {0.0, 0.0};
    for (int64_t i = R.b + threadIdx.x; i < R.e; i += KT) {
        const double si = r[i] - alpha * v[i];
        s[i] = si;
        loc[0] += si * si;
    }
    kblock_store<2>(loc, part, gridDim.x);
}

// x += alpha p^ (a converged half step)
__global__ __launch_bounds__(KT) void k_bi_xhalf(int64_t n, const double* __restrict__ ph, double alpha,
                                                  double* __restrict__ x) {
    for (int64_t i = blockIdx.x * (int64_t)KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT)
        x[i] += alpha * ph[i];
}

// x = x + alpha p^ + omega s^, r = s - omega t, partials r^.r and r.r
__global__ __launch_bounds__(KT) void k_bi_update(int64_t n, const double* __restrict__ ph,
                                                   const double* __restrict__ sh, const double* __restrict__ s,
                                                   const double* __restrict__ t, const double* __restrict__ rh,
                                                   double alpha, double omega, double* __restrict__ x,
                                                   double* __restrict__ r, double* __restrict__ part) {
    const Range R = block_range(n);
    double loc[2] = {0.0, 0.0};
    for (int64_t i = R.b + threadIdx.x; i < R.e; i += KT) {
        x[i] = x[i] + alpha * ph[i] + omega * sh[i];
        const double ri = s[i] - omega * t[i];
        r[i] = ri;
        loc[0] += rh[i] * ri;
        loc[1] += ri * ri;
    }
    kblock_store<2>(loc, part, gridDim.x);
}

inline unsigned vec_blocks(int64_t n) {
    const int64_t b = (n + KT - 1) / KT;
    return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

}  // namespace

int bi_grid(int64_t n) { return red_grid_elems(n); }

void launch_bi_residual(int64_t n, const double* f, const double* y, double* r, double* part, int nb, hipStream_t s) {
    k_bi_residual<<<nb, KT, 0, s>>>(n, f, y, r, part);
    HIP_LAUNCH_CHECK();
}
void launch_bi_dots(int64_t n, const double* a, const double* b, const double* c, const double* d, double* part,
                    int nb, hipStream_t s) {
    k_bi_dots<<<nb, KT, 0, s>>>(n, a, b, c, d, part);
    HIP_LAUNCH_CHECK();
}
void launch_bi_direction(int64_t n, const double* r, const double* v, double beta, double omega, int first, double* p,
                         hipStream_t s) {
    k_bi_direction<<<vec_blocks(n), KT, 0, s>>>(n, r, v, beta, omega, first, p);
    HIP_LAUNCH_CHECK();
}
void launch_bi_half(int64_t n, const double* r, const double* v, double alpha, double* sv, double* part, int nb,
                    hipStream_t s) {
    k_bi_half<<<nb, KT, 0, s>>>(n, r, v, alpha, sv, part);
    HIP_LAUNCH_CHECK();
}
void launch_bi_xhalf(int64_t n, const double* ph, double alpha, double* x, hipStream_t s) {
    k_bi_xhalf<<<vec_blocks(n), KT, 0, s>>>(n, ph, alpha, x);
    HIP_LAUNCH_CHECK();
}
void launch_bi_update(int64_t n, const double* ph, const double* sh, const double* sv, const double* t,
                      const double* rh, double alpha, double omega, double* x, double* r, double* part, int nb,
                      hipStream_t s) {
    k_bi_update<<<nb, KT, 0, s>>>(n, ph, sh, sv, t, rh, alpha, omega, x, r, part);
    HIP_LAUNCH_CHECK();
}

}  // namespace amgmi
