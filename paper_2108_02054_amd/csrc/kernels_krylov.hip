// BiCGStab vector kernels (FP64): the paper's Krylov method for its non-symmetric
// systems (van der Vorst's BiCGStab, the V-cycle applied on the right).  The matrix
// products go through the level-0 SpMV launcher and the preconditioner through the
// V-cycle; these kernels do the vector updates, the dot products and the step's scalars.
// Every dot product is reduced deterministically: a bounded grid, each thread adding its
// entries in index order, a fixed wavefront and workgroup tree, one partial per workgroup;
// a one-workgroup kernel adds the partials in a fixed order into the scalars the next
// kernels read (alpha, omega, beta), and only the ||r||^2 partials, the flags and the
// scalars of the step reach the host, through mapped host memory, once per step.
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

// Sum of p[0..nb) by one workgroup in a fixed order (each thread its strided entries in
// index order, then a fixed wavefront and workgroup tree); returned to every thread.
__device__ __forceinline__ double kblock_sum(const double* __restrict__ p, int nb) {
    __shared__ double sm[KT / 64];
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += KT) a += p[i];
    a = kwave_sum(a);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = a;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < KT / 64; ++w) s += sm[w];
    __syncthreads();
    return s;
}

// The scalars of one BiCGStab step, formed on the device from the partials of the kernel
// before (one workgroup), so that the step runs with no host round trip; see BiScal.
__global__ __launch_bounds__(KT) void k_bi_scal(int stage, double* __restrict__ sc, const double* __restrict__ part,
                                                 int nb, double value, double tol) {
    auto bad = [&](double x) { return x == 0.0 || !isfinite(x); };
    if (stage == BI_RESET) {
        if (threadIdx.x == 0) {
            sc[BS_RHO] = value;
            sc[BS_ALPHA] = sc[BS_OMEGA] = 1.0;
            sc[BS_BETA] = 0.0;
            sc[BS_HALF] = 0.0;
            sc[BS_BAD] = 0.0;
        }
        return;
    }
    const double a = kblock_sum(part, nb);
    const double b = stage == BI_OMEGA ? kblock_sum(part + nb, nb) : 0.0;
    if (threadIdx.x != 0) return;
    int flags = (int)sc[BS_BAD];
    if (stage == BI_BETA) {  // a = r^.r of the new residual
        if (bad(a)) flags |= BI_BAD_RHO;
        sc[BS_BETA] = (a / sc[BS_RHO]) * (sc[BS_ALPHA] / sc[BS_OMEGA]);
        sc[BS_RHO] = a;
    } else if (stage == BI_ALPHA) {  // a = r^.v
        if (bad(a)) flags |= BI_BAD_RV;
        sc[BS_ALPHA] = sc[BS_RHO] / a;
    } else if (stage == BI_HALF) {  // a = s.s; tol = rtol ||f||
        sc[BS_HALF] = sqrt(a) <= tol ? 1.0 : 0.0;
    } else if (stage == BI_OMEGA) {  // a = t.s, b = t.t
        if (bad(b)) flags |= BI_BAD_TT;
        const double w = a / b;
        if (bad(w)) flags |= BI_BAD_OMEGA;
        sc[BS_OMEGA] = w;
    }
    sc[BS_BAD] = (double)flags;
}

// p = r (first step) or p = r + beta (p - omega v)
__global__ __launch_bounds__(KT) void k_bi_direction(int64_t n, const double* __restrict__ r,
                                                      const double* __restrict__ v, const double* __restrict__ sc,
                                                      int first, double* __restrict__ p) {
    const double beta = sc[BS_BETA], omega = sc[BS_OMEGA];
    for (int64_t i = blockIdx.x * (int64_t)KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT)
        p[i] = first ? r[i] : r[i] + beta * (p[i] - omega * v[i]);
}

// s = r - alpha v, partial s.s
__global__ __launch_bounds__(KT) void k_bi_half(int64_t n, const double* __restrict__ r, const double* __restrict__ v,
                                                 const double* __restrict__ sc, double* __restrict__ s,
                                                 double* __restrict__ part) {
    const double alpha = sc[BS_ALPHA];
    const Range R = block_range(n);
    double loc[1] = {0.0};
    for (int64_t i = R.b + threadIdx.x; i < R.e; i += KT) {
        const double si = r[i] - alpha * v[i];
        s[i] = si;
        loc[0] += si * si;
    }
    kblock_store<1>(loc, part, gridDim.x);
}

// x = x + alpha p^ + omega s^, r = s - omega t, partials r^.r (device) and r.r (host
// mirror); after a converged half step only x += alpha p^.  Workgroup 0 copies the
// scalars and flags to the host mirror.
__global__ __launch_bounds__(KT) void k_bi_update(int64_t n, const double* __restrict__ ph,
                                                   const double* __restrict__ sh, const double* __restrict__ s,
                                                   const double* __restrict__ t, const double* __restrict__ rh,
                                                   const double* __restrict__ sc, double* __restrict__ x,
                                                   double* __restrict__ r, double* __restrict__ rho_part,
                                                   double* __restrict__ host) {
    const double alpha = sc[BS_ALPHA], omega = sc[BS_OMEGA];
    const bool half = sc[BS_HALF] != 0.0;
    const Range R = block_range(n);
    double loc[2] = {0.0, 0.0};
    if (half) {
        for (int64_t i = R.b + threadIdx.x; i < R.e; i += KT) x[i] += alpha * ph[i];
    } else {
        for (int64_t i = R.b + threadIdx.x; i < R.e; i += KT) {
            x[i] = x[i] + alpha * ph[i] + omega * sh[i];
            const double ri = s[i] - omega * t[i];
            r[i] = ri;
            loc[0] += rh[i] * ri;
            loc[1] += ri * ri;
        }
    }
    __shared__ double sm[2][KT / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const double xq = kwave_sum(loc[q]);
        if (lane == 0) sm[q][w] = xq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int i = 0; i < KT / 64; ++i) {
            a += sm[0][i];
            b += sm[1][i];
        }
        rho_part[blockIdx.x] = a;
        host[blockIdx.x] = b;
        if (blockIdx.x == 0)
            for (int k = 0; k < BS_COUNT; ++k) host[2 * RED_BLOCKS + k] = sc[k];
    }
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
void launch_bi_scal(int stage, double* sc, const double* part, int nb, double value, double tol, hipStream_t s) {
    k_bi_scal<<<1, KT, 0, s>>>(stage, sc, part, nb, value, tol);
    HIP_LAUNCH_CHECK();
}
void launch_bi_direction(int64_t n, const double* r, const double* v, const double* sc, int first, double* p,
                         hipStream_t s) {
    k_bi_direction<<<vec_blocks(n), KT, 0, s>>>(n, r, v, sc, first, p);
    HIP_LAUNCH_CHECK();
}
void launch_bi_half(int64_t n, const double* r, const double* v, const double* sc, double* sv, double* part, int nb,
                    hipStream_t s) {
    k_bi_half<<<nb, KT, 0, s>>>(n, r, v, sc, sv, part);
    HIP_LAUNCH_CHECK();
}
void launch_bi_update(int64_t n, const double* ph, const double* sh, const double* sv, const double* t,
                      const double* rh, const double* sc, double* x, double* r, double* rho_part, double* host, int nb,
                      hipStream_t s) {
    k_bi_update<<<nb, KT, 0, s>>>(n, ph, sh, sv, t, rh, sc, x, r, rho_part, host);
    HIP_LAUNCH_CHECK();
}

}  // namespace amgmi
