// kernels_block.hip -- systems with B unknowns per node (the paper's 4x4-block systems,
// Section 4, where every matrix value is a block): damped block Jacobi, whose smoother
// holds omega * D_I^{-1} for every node I (row-major, B*B values per node), and the
// node-group products (residual, sweep, Krylov SpMV) that read the level's node pattern.
// Unknown b of node I is row I*B + b; every stored entry belongs to a full B x B block.
//
// The inverse is Gauss-Jordan elimination with partial pivoting on [D_I | I], in the
// order of its definition (the first row of largest magnitude in the column is the pivot),
// with separately rounded products, so that in FP64 it reproduces the definition's
// rounding.  B is a compile-time constant (2..8): the working block stays in registers.
#include <algorithm>

#include <hip/hip_ext.h>

#include "amg_internal.h"

#pragma clang fp contract(off)

namespace amgmi {

constexpr int TPB_B = 256;

// One thread per node; its diagonal block is found in the node pattern (nptr, ncol: node
// I's rows hold B * B * nptr[I] entries before them, each row B * (nptr[I+1] - nptr[I])).
// Values are read in T (FP64, or the FP32 copies of a mixed hierarchy), the elimination
// runs in FP64 and the result is stored in T.  A zero pivot (singular block) sets
// flags[F_NOT_SPD] when flags is given; the block then holds non-finite values.
template <int B, typename T>
__global__ __launch_bounds__(TPB_B) void k_block_inv(int nn, const int* __restrict__ nptr,
                                                     const int* __restrict__ ncol, const T* __restrict__ val,
                                                     double omega, T* __restrict__ m, int* __restrict__ flags) {
    const int I = xcd_block() * TPB_B + threadIdx.x;
    if (I >= nn) return;
    double W[B][2 * B];
#pragma unroll
    for (int a = 0; a < B; ++a) {
#pragma unroll
        for (int q = 0; q < 2 * B; ++q) W[a][q] = (q == B + a) ? 1.0 : 0.0;
    }
    const int nb = nptr[I], ne = nptr[I + 1], len = B * (ne - nb);
    int g = nb;
    while (g < ne && ncol[g] < I) ++g;  // the diagonal block's position (absent: zero block)
    if (g < ne && ncol[g] == I) {
        const T* v = val + (size_t)B * B * nb + (size_t)B * (g - nb);
#pragma unroll
        for (int a = 0; a < B; ++a) {
#pragma unroll
            for (int q = 0; q < B; ++q) W[a][q] = (double)v[a * len + q];
        }
    }
    bool singular = false;
#pragma unroll
    for (int k = 0; k < B; ++k) {
        int piv = k;
        double best = fabs(W[k][k]);
#pragma unroll
        for (int a = k + 1; a < B; ++a) {
            const double v = fabs(W[a][k]);
            if (v > best) {
                best = v;
                piv = a;
            }
        }
        if (best == 0.0) singular = true;
        // swap rows k and piv (selects, so the block stays in registers)
#pragma unroll
        for (int a = k + 1; a < B; ++a) {
            if (a == piv) {
#pragma unroll
                for (int q = 0; q < 2 * B; ++q) {
                    const double t = W[k][q];
                    W[k][q] = W[a][q];
                    W[a][q] = t;
                }
            }
        }
        const double d = W[k][k];
#pragma unroll
        for (int q = 0; q < 2 * B; ++q) W[k][q] = W[k][q] / d;
#pragma unroll
        for (int a = 0; a < B; ++a) {
            if (a == k) continue;
            const double f = W[a][k];
#pragma unroll
            for (int q = 0; q < 2 * B; ++q) W[a][q] = W[a][q] - f * W[k][q];
        }
    }
    if (singular && flags != nullptr) atomicOr(&flags[F_NOT_SPD], 1);
    T* out = m + (size_t)I * B * B;
#pragma unroll
    for (int a = 0; a < B; ++a) {
#pragma unroll
        for (int q = 0; q < B; ++q) out[a * B + q] = (T)(omega * W[a][B + q]);
    }
}

// uout_i = uin_i + sum_q M_I[a][q] r_{I*B+q} for row i = I*B + a (uin == nullptr: zero);
// the block row product is summed in column order before it is added.
template <int B, typename T>
__global__ __launch_bounds__(TPB_B) void k_block_apply(int n, const T* __restrict__ m, const T* __restrict__ r,
                                                       const T* __restrict__ uin, T* __restrict__ uout) {
    const int i = xcd_block() * TPB_B + threadIdx.x;
    if (i >= n) return;
    const int base = i - i % B;
    const T* mi = m + (size_t)i * B;
    T s = 0;
#pragma unroll
    for (int q = 0; q < B; ++q) s = s + mi[q] * r[base + q];
    uout[i] = uin != nullptr ? uin[i] + s : s;
}

// ------------------------------------------------------------------ node-group products
//
// The rows of a node list the same columns (full blocks) and are consecutive in CSR, so
// with the node pattern (nptr, ncol) node I's rows hold B * B * nptr[I] entries before
// them, each row has len = B * (nptr[I+1] - nptr[I]) entries, and entry k of a row lies in
// column B * ncol[nptr[I] + k / B] + k % B: one 4-byte index per block instead of one
// per entry.  A group of NG lanes walks the row positions once and reads the B rows'
// values at the same offsets, coalesced across the group; every lane keeps B partial
// sums, a butterfly over the group leaves the B row sums in every lane, and lanes
// 0..B-1 finish one row each.  16 nodes per workgroup.
constexpr int NG = 16;
constexpr int NODES_PER_WG = TPB_B / NG;

__device__ __forceinline__ double bfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float bfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <int B, typename T>
__device__ __forceinline__ void node_rowsums(int I, int lane, const int* __restrict__ nptr,
                                             const int* __restrict__ ncol, const T* __restrict__ val,
                                             const T* __restrict__ x, T (&s)[B]) {
    const int nb = nptr[I];
    const int len = B * (nptr[I + 1] - nb);
    const T* v = val + (size_t)B * B * nb;
#pragma unroll
    for (int a = 0; a < B; ++a) s[a] = 0;
    int k = lane;
    for (; k + NG < len; k += 2 * NG) {  // two positions per pass: their loads in flight together
        const int k2 = k + NG;
        const int j1 = B * ncol[nb + k / B] + k % B, j2 = B * ncol[nb + k2 / B] + k2 % B;
        T v1[B], v2[B];
#pragma unroll
        for (int a = 0; a < B; ++a) {
            v1[a] = v[a * len + k];
            v2[a] = v[a * len + k2];
        }
        const T x1 = x[j1], x2 = x[j2];
#pragma unroll
        for (int a = 0; a < B; ++a) s[a] = bfma(v2[a], x2, bfma(v1[a], x1, s[a]));
    }
    if (k < len) {
        const T xj = x[B * ncol[nb + k / B] + k % B];
#pragma unroll
        for (int a = 0; a < B; ++a) s[a] = bfma(v[a * len + k], xj, s[a]);
    }
#pragma unroll
    for (int o = NG / 2; o > 0; o >>= 1) {
#pragma unroll
        for (int a = 0; a < B; ++a) s[a] += __shfl_xor(s[a], o, NG);
    }
}

// The same row sums with each lane taking two adjacent positions (k, k + 1), k even (B
// even): both lie in one block column, so one node column, one 2-element load of x and
// one 2-element load per row serve them, against two of each.  Rows of a node and the
// node's first entry start at even offsets, so every pair load is aligned to its size.
template <int B, typename T>
__device__ __forceinline__ void node_rowsums_pairs(int I, int lane, const int* __restrict__ nptr,
                                                   const int* __restrict__ ncol, const T* __restrict__ val,
                                                   const T* __restrict__ x, T (&s)[B]) {
    static_assert(B % 2 == 0, "pairs of positions need an even block size");
    typedef T T2 __attribute__((ext_vector_type(2)));
    const int nb = nptr[I];
    const int len = B * (nptr[I + 1] - nb);
    const T* v = val + (size_t)B * B * nb;
#pragma unroll
    for (int a = 0; a < B; ++a) s[a] = 0;
    const int np = len / 2;
    int h = lane;
    for (; h + NG < np; h += 2 * NG) {  // two pairs per pass: their loads in flight together
        const int k1 = 2 * h, k2 = 2 * (h + NG);
        const int j1 = B * ncol[nb + k1 / B] + k1 % B, j2 = B * ncol[nb + k2 / B] + k2 % B;
        T2 v1[B], v2[B];
#pragma unroll
        for (int a = 0; a < B; ++a) {
            v1[a] = *reinterpret_cast<const T2*>(v + a * len + k1);
            v2[a] = *reinterpret_cast<const T2*>(v + a * len + k2);
        }
        const T2 x1 = *reinterpret_cast<const T2*>(x + j1), x2 = *reinterpret_cast<const T2*>(x + j2);
#pragma unroll
        for (int a = 0; a < B; ++a)
            s[a] = bfma(v2[a].y, x2.y, bfma(v2[a].x, x2.x, bfma(v1[a].y, x1.y, bfma(v1[a].x, x1.x, s[a]))));
    }
    if (h < np) {
        const int k1 = 2 * h;
        const T2 x1 = *reinterpret_cast<const T2*>(x + B * ncol[nb + k1 / B] + k1 % B);
#pragma unroll
        for (int a = 0; a < B; ++a) {
            const T2 v1 = *reinterpret_cast<const T2*>(v + a * len + k1);
            s[a] = bfma(v1.y, x1.y, bfma(v1.x, x1.x, s[a]));
        }
    }
#pragma unroll
    for (int o = NG / 2; o > 0; o >>= 1) {
#pragma unroll
        for (int a = 0; a < B; ++a) s[a] += __shfl_xor(s[a], o, NG);
    }
}

// PR: pairs of positions (even B only)
template <int B, bool PR, typename T>
__device__ __forceinline__ void node_sums(int I, int lane, const int* __restrict__ nptr, const int* __restrict__ ncol,
                                          const T* __restrict__ val, const T* __restrict__ x, T (&s)[B]) {
    if constexpr (PR && B % 2 == 0)
        node_rowsums_pairs<B>(I, lane, nptr, ncol, val, x, s);
    else
        node_rowsums<B>(I, lane, nptr, ncol, val, x, s);
}

// s[lane] for lane < B, by selects (the array stays in registers)
template <int B, typename T>
__device__ __forceinline__ T pick(const T (&s)[B], int lane) {
    T v = s[0];
#pragma unroll
    for (int a = 1; a < B; ++a) v = lane == a ? s[a] : v;
    return v;
}

// r = f - A u
template <int B, bool PR, typename T>
__global__ __launch_bounds__(TPB_B) void k_node_residual(int nn, const int* __restrict__ nptr,
                                                         const int* __restrict__ ncol, const T* __restrict__ val,
                                                         const T* __restrict__ f, const T* __restrict__ u,
                                                         T* __restrict__ r) {
    const int I = xcd_block() * NODES_PER_WG + (int)threadIdx.x / NG;
    const int lane = threadIdx.x & (NG - 1);
    if (I >= nn) return;
    T s[B];
    node_sums<B, PR>(I, lane, nptr, ncol, val, u, s);
    if (lane < B) {
        const int i = I * B + lane;
        r[i] = f[i] - pick<B>(s, lane);
    }
}

// uout = uin + M (f - A uin): a residual and the block-diagonal product in one pass
template <int B, bool PR, typename T>
__global__ __launch_bounds__(TPB_B) void k_node_sweep(int nn, const int* __restrict__ nptr, const int* __restrict__ ncol,
                                                      const T* __restrict__ val, const T* __restrict__ m,
                                                      const T* __restrict__ f, const T* __restrict__ uin,
                                                      T* __restrict__ uout) {
    const int I = xcd_block() * NODES_PER_WG + (int)threadIdx.x / NG;
    const int lane = threadIdx.x & (NG - 1);
    if (I >= nn) return;
    T s[B];
    node_sums<B, PR>(I, lane, nptr, ncol, val, uin, s);
    if (lane < B) {
        const int i = I * B + lane;
        const T* mi = m + (size_t)i * B;
        T d = 0;
#pragma unroll
        for (int q = 0; q < B; ++q) d = d + mi[q] * (f[I * B + q] - s[q]);
        uout[i] = uin[i] + d;
    }
}

// The last post-sweep of a block system's level 0 with the CG's r.z partials (FP64): z =
// uin + M (r - A uin), one partial of r.z per workgroup (the full node grid).
template <int B, bool PR>
__global__ __launch_bounds__(TPB_B) void k_node_sweep_rz(int nn, const int* __restrict__ nptr,
                                                         const int* __restrict__ ncol, const double* __restrict__ val,
                                                         const double* __restrict__ m, const double* __restrict__ r,
                                                         const double* __restrict__ uin, double* __restrict__ z,
                                                         RedScratch rs) {
    const int I = xcd_block() * NODES_PER_WG + (int)threadIdx.x / NG;
    const int lane = threadIdx.x & (NG - 1);
    double loc = 0.0;
    if (I < nn) {
        double s[B];
        node_sums<B, PR>(I, lane, nptr, ncol, val, uin, s);
        if (lane < B) {
            const int i = I * B + lane;
            const double* mi = m + (size_t)i * B;
            double d = 0;
#pragma unroll
            for (int q = 0; q < B; ++q) d = d + mi[q] * (r[I * B + q] - s[q]);
            const double zi = uin[i] + d;
            z[i] = zi;
            loc += r[i] * zi;
        }
    }
    __shared__ double sm[TPB_B / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) loc += __shfl_xor(loc, o, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = loc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < TPB_B / 64; ++w) t += sm[w];
        rs.region(P_RZ)[blockIdx.x] = t;
    }
}

// p_new = z + beta p_old (z on the first iteration), elementwise.  The fma is the one the
// CG kernels of scalar systems use for the same update.
__global__ __launch_bounds__(TPB_B) void k_node_pupdate(int n, const double* __restrict__ z,
                                                        const double* __restrict__ pold, double* __restrict__ pnew,
                                                        int first, RedScratch rs) {
    const double beta = first ? 0.0 : rs.scal()[S_BETA];
    const int i = xcd_block() * TPB_B + threadIdx.x;
    if (i < n) pnew[i] = first ? z[i] : __builtin_fma(beta, pold[i], z[i]);
}

// q = A p and p.q partials (FP64), p formed by k_node_pupdate: one gathered vector per
// block column, one position per lane (the pair form measured slower here).  Bounded grid, nodes by grid stride: one partial per workgroup, in a
// fixed order.
template <int B>
__global__ __launch_bounds__(TPB_B) void k_node_cg_pq(int nn, const int* __restrict__ nptr,
                                                      const int* __restrict__ ncol, const double* __restrict__ val,
                                                      const double* __restrict__ p, double* __restrict__ q,
                                                      RedScratch rs) {
    const int lane = threadIdx.x & (NG - 1);
    double loc = 0.0;
    for (int I = blockIdx.x * NODES_PER_WG + (int)threadIdx.x / NG; I < nn; I += gridDim.x * NODES_PER_WG) {
        double s[B];
        node_rowsums<B>(I, lane, nptr, ncol, val, p, s);
        if (lane < B) {
            const int i = I * B + lane;
            const double qi = pick<B>(s, lane);
            q[i] = qi;
            loc += p[i] * qi;
        }
    }
    __shared__ double sm[TPB_B / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) loc += __shfl_xor(loc, o, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = loc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < TPB_B / 64; ++w) t += sm[w];
        rs.region(P_PQ)[blockIdx.x] = t;
    }
}

static unsigned bgrid(int64_t n) {
    const int64_t b = (n + TPB_B - 1) / TPB_B;
    return (unsigned)(b > 0 ? b : 1);
}

#define AMG_WITH_B(B_, ...)                                             \
    switch (B_) {                                                       \
        case 2: { constexpr int B = 2; __VA_ARGS__; } break;            \
        case 3: { constexpr int B = 3; __VA_ARGS__; } break;            \
        case 4: { constexpr int B = 4; __VA_ARGS__; } break;            \
        case 5: { constexpr int B = 5; __VA_ARGS__; } break;            \
        case 6: { constexpr int B = 6; __VA_ARGS__; } break;            \
        case 7: { constexpr int B = 7; __VA_ARGS__; } break;            \
        case 8: { constexpr int B = 8; __VA_ARGS__; } break;            \
        default: throw Fail{AMG_ERR_ARG, "block_size must be 1 .. 8"}; \
    }

static void need_nodes(const Level& L) {
    if (L.nptr == nullptr || L.ncol == nullptr) throw Fail{AMG_ERR_STATE, "node pattern missing"};
}

template <typename T>
void launch_block_inv(const Level& L, int B_, double omega, T* m, int* flags, hipStream_t s) {
    need_nodes(L);
    const int nn = L.A.nrows / B_;
    AMG_WITH_B(B_, timed_launch(k_block_inv<B, T>, bgrid(nn), TPB_B, 0, s, nn, L.nptr, L.ncol, L.A.v<T>(), omega, m, flags));
    HIP_LAUNCH_CHECK();
}

template <typename T>
void launch_block_apply(int n, int B_, const T* m, const T* r, const T* uin, T* uout, hipStream_t s) {
    AMG_WITH_B(B_, timed_launch(k_block_apply<B, T>, bgrid(n), TPB_B, 0, s, n, m, r, uin, uout));
    HIP_LAUNCH_CHECK();
}

int node_grid(int nn) { return (int)(((int64_t)nn + NODES_PER_WG - 1) / NODES_PER_WG); }

template <typename T>
void launch_node_residual(const Level& L, int B_, const T* f, const T* u, T* r, hipStream_t s) {
    need_nodes(L);
    const int nn = L.A.nrows / B_;
    const unsigned nb = (unsigned)std::max(1, node_grid(nn));
    AMG_WITH_B(B_, {
        if (L.node_pairs)
            timed_launch(k_node_residual<B, true, T>, nb, TPB_B, 0, s, nn, L.nptr, L.ncol, L.A.v<T>(), f, u, r);
        else
            timed_launch(k_node_residual<B, false, T>, nb, TPB_B, 0, s, nn, L.nptr, L.ncol, L.A.v<T>(), f, u, r);
    });
    HIP_LAUNCH_CHECK();
}

template <typename T>
void launch_node_sweep(const Level& L, int B_, const T* m, const T* f, const T* uin, T* uout, hipStream_t s) {
    need_nodes(L);
    const int nn = L.A.nrows / B_;
    const unsigned nb = (unsigned)std::max(1, node_grid(nn));
    AMG_WITH_B(B_, {
        if (L.node_pairs)
            timed_launch(k_node_sweep<B, true, T>, nb, TPB_B, 0, s, nn, L.nptr, L.ncol, L.A.v<T>(), m, f, uin, uout);
        else
            timed_launch(k_node_sweep<B, false, T>, nb, TPB_B, 0, s, nn, L.nptr, L.ncol, L.A.v<T>(), m, f, uin, uout);
    });
    HIP_LAUNCH_CHECK();
}

// The Krylov operator product of a block system (values `val` on the pattern of A): the
// direction update, then q = A p_new with the p.q partials.  Like the other Krylov SpMV
// launchers it takes the events that a kernel trace left for it, for the product (the
// elementwise update before it is not in them).
int launch_node_cg_pq(const Level& L, int B_, const double* val, const double* z, const double* pold, double* pnew,
                      double* q, int first, const RedScratch& rs, hipStream_t s) {
    need_nodes(L);
    const int n = L.A.nrows, nn = n / B_;
    const int nb = std::max(1, std::min(node_grid(nn), rs.cap));
    const KernelEvents e = g_kernel_events;
    g_kernel_events = KernelEvents{};
    timed_launch(k_node_pupdate, bgrid(n), TPB_B, 0, s, n, z, pold, pnew, first, rs);
    HIP_LAUNCH_CHECK();
    const double* p = pnew;
    auto go = [&](auto kern) {
        if (e.start != nullptr)
            hipExtLaunchKernelGGL(kern, dim3(nb), dim3(TPB_B), 0, s, e.start, e.stop, 0, nn, (const int*)L.nptr,
                                  (const int*)L.ncol, val, p, q, rs);
        else
            hipLaunchKernelGGL(kern, dim3(nb), dim3(TPB_B), 0, s, nn, (const int*)L.nptr, (const int*)L.ncol, val, p,
                               q, rs);
    };
    AMG_WITH_B(B_, go(k_node_cg_pq<B>));
    HIP_LAUNCH_CHECK();
    return nb;
}

int launch_node_sweep_rz(const Level& L, int B_, const double* m, const double* r, const double* uin, double* z,
                         const RedScratch& rs, hipStream_t s) {
    need_nodes(L);
    const int nn = L.A.nrows / B_;
    const int nb = std::max(1, node_grid(nn));
    if (nb > rs.cap) throw Fail{AMG_ERR_ARG, "reduction scratch too small"};
    AMG_WITH_B(B_, {
        if (L.node_pairs)
            timed_launch(k_node_sweep_rz<B, true>, nb, TPB_B, 0, s, nn, L.nptr, L.ncol, L.A.val, m, r, uin, z, rs);
        else
            timed_launch(k_node_sweep_rz<B, false>, nb, TPB_B, 0, s, nn, L.nptr, L.ncol, L.A.val, m, r, uin, z, rs);
    });
    HIP_LAUNCH_CHECK();
    return nb;
}

template void launch_node_residual<double>(const Level&, int, const double*, const double*, double*, hipStream_t);
template void launch_node_residual<float>(const Level&, int, const float*, const float*, float*, hipStream_t);
template void launch_node_sweep<double>(const Level&, int, const double*, const double*, const double*, double*,
                                        hipStream_t);
template void launch_node_sweep<float>(const Level&, int, const float*, const float*, const float*, float*,
                                       hipStream_t);
template void launch_block_inv<double>(const Level&, int, double, double*, int*, hipStream_t);
template void launch_block_inv<float>(const Level&, int, double, float*, int*, hipStream_t);
template void launch_block_apply<double>(int, int, const double*, const double*, const double*, double*, hipStream_t);
template void launch_block_apply<float>(int, int, const float*, const float*, const float*, float*, hipStream_t);

}  // namespace amgmi
