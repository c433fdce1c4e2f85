// kernels_block.hip -- systems with B unknowns per node (the paper's 4x4-block systems,
// Section 4, where every matrix value is a block): damped block Jacobi, whose smoother
// holds omega * D_I^{-1} for every node I (row-major, B*B values per node), the
// node-group products (residual, sweep, Krylov SpMV) that read the level's node pattern,
// and the Galerkin product of a partial update formed block by block.
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
// block column.  One node group per node, workgroups in XCD order like the sweeps', one
// partial per workgroup at its logical index; GS: a grid smaller than that (a reduction
// scratch with fewer slots than workgroups) takes the other nodes by grid stride.
template <int B, bool PR, bool GS>
__global__ __launch_bounds__(TPB_B) void k_node_cg_pq(int nn, const int* __restrict__ nptr,
                                                      const int* __restrict__ ncol, const double* __restrict__ val,
                                                      const double* __restrict__ p, double* __restrict__ q,
                                                      RedScratch rs) {
    const int lb = xcd_block();
    const int lane = threadIdx.x & (NG - 1);
    double loc = 0.0;
    for (int I = lb * NODES_PER_WG + (int)threadIdx.x / NG; I < nn; I += gridDim.x * NODES_PER_WG) {
        double s[B];
        node_sums<B, PR>(I, lane, nptr, ncol, val, p, s);
        if (lane < B) {
            const int i = I * B + lane;
            const double qi = pick<B>(s, lane);
            q[i] = qi;
            loc += p[i] * qi;
        }
        if constexpr (!GS) break;
    }
    __shared__ double sm[TPB_B / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) loc += __shfl_xor(loc, o, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = loc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < TPB_B / 64; ++w) t += sm[w];
        rs.region(P_PQ)[lb] = t;
    }
}

// ------------------------------------------------------------------ node Galerkin product
//
// With P_l = P_node (x) I_B and unit values, row I*B + a of A_l P_l sums, per aggregate L,
// the entries (a, c) of the blocks (I, K), K in L, in ascending K, and row J*B + a of
// R_l (A_l P_l) sums those row sums over the fine nodes I of aggregate J in ascending I.
// The plan lists, per block (J, L) of A_{l+1}, its terms -- the blocks (I, K) -- in the
// order (I, K), marking where a new fine node starts; lane (a, c) of the block's group adds
// the terms' entries (a, c) in that order, closing each fine node's sum before it adds the
// next one's: the products by the unit values are exact, so this is the row-by-row
// product's arithmetic.  The values are read once, in whole blocks of B consecutive
// entries per row.

// Aggregate of each fine node from P's rows, checking the unit Kronecker form.
template <int B>
__global__ __launch_bounds__(TPB_B) void k_ngal_agg(int nn, const int* __restrict__ Pptr, const int* __restrict__ Pcol,
                                                    const double* __restrict__ Pval, int* __restrict__ nagg,
                                                    int* __restrict__ flags) {
    const int I = blockIdx.x * TPB_B + threadIdx.x;
    if (I >= nn) return;
    const int c0 = Pptr[I * B + 1] - Pptr[I * B];
    bool ok = c0 == 0 || c0 == 1;
    int J = -1;
    if (ok && c0 == 1) {
        const int col0 = Pcol[Pptr[I * B]];
        ok = col0 % B == 0;
        J = col0 / B;
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int k = Pptr[I * B + b];
        const int cnt = Pptr[I * B + b + 1] - k;
        if (cnt != c0) ok = false;
        else if (ok && cnt == 1 && (Pcol[k] != J * B + b || Pval[k] != 1.0)) ok = false;
    }
    if (!ok) flags[F_NODEGAL] = 1;
    if (ok && J < 0) flags[F_NODEPART] = 1;
    nagg[I] = ok ? J : -1;
}

// One thread per coarse node J: the fine nodes of aggregate J are the columns / B of R's
// row J*B; each of their blocks (I, K) gets the position of aggregate(K) in J's coarse row.
template <int B>
__global__ __launch_bounds__(TPB_B) void k_ngal_count(int ncn, const int* __restrict__ Rptr,
                                                      const int* __restrict__ Rcol, const int* __restrict__ nptr,
                                                      const int* __restrict__ ncol, const int* __restrict__ nagg,
                                                      const int* __restrict__ cnptr, const int* __restrict__ cncol,
                                                      int* __restrict__ tpos, int* __restrict__ cnt,
                                                      int* __restrict__ flags) {
    const int J = blockIdx.x * TPB_B + threadIdx.x;
    if (J >= ncn) return;
    const int c0 = cnptr[J], c1 = cnptr[J + 1];
    for (int t = Rptr[J * B]; t < Rptr[J * B + 1]; ++t) {
        const int I = Rcol[t] / B;
        if (Rcol[t] % B != 0 || nagg[I] != J) flags[F_NODEGAL] = 1;
        for (int e = nptr[I]; e < nptr[I + 1]; ++e) {
            const int L = nagg[ncol[e]];
            int p = -1;
            if (L >= 0) {
                int lo = c0, hi = c1;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (cncol[mid] < L)
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                if (lo < c1 && cncol[lo] == L)
                    p = lo - c0;
                else
                    flags[F_NODEGAL] = 1;  // the coarse pattern lacks a block the product forms
            } else {
                flags[F_NODEPART] = 1;
            }
            tpos[e] = p;
            if (p >= 0) cnt[c0 + p] += 1;  // coarse row J is this thread's alone
        }
    }
}

template <int B>
__global__ __launch_bounds__(TPB_B) void k_ngal_fill(int ncn, const int* __restrict__ Rptr,
                                                     const int* __restrict__ Rcol, const int* __restrict__ nptr,
                                                     const int* __restrict__ cnptr, const int* __restrict__ tpos,
                                                     const int* __restrict__ tptr, int* __restrict__ toff,
                                                     int* __restrict__ tlen, int* __restrict__ cout,
                                                     int* __restrict__ clen, int* __restrict__ cur,
                                                     int* __restrict__ last) {
    const int J = blockIdx.x * TPB_B + threadIdx.x;
    if (J >= ncn) return;
    const int c0 = cnptr[J], c1 = cnptr[J + 1];
    for (int g = c0; g < c1; ++g) {
        cur[g] = tptr[g];
        last[g] = -1;
        cout[g] = B * B * c0 + (g - c0) * B;
        clen[g] = B * (c1 - c0);
    }
    for (int t = Rptr[J * B]; t < Rptr[J * B + 1]; ++t) {
        const int I = Rcol[t] / B;
        const int nb = nptr[I], len = B * (nptr[I + 1] - nb);
        for (int e = nb; e < nptr[I + 1]; ++e) {
            const int p = tpos[e];
            if (p < 0) continue;
            const int g = c0 + p;
            const int slot = cur[g]++;
            toff[slot] = B * B * nb + (e - nb) * B;
            tlen[slot] = 2 * len + (last[g] != I ? 1 : 0);
            last[g] = I;
        }
    }
}

// One lane per entry (a, c) of a coarse block, NGB >= B*B lanes per block.  The terms go
// in batches of U: a lane issues a batch's U value loads, then the next batch's plan loads,
// then adds the batch's values in order -- a coarse block's list (some forty terms for the
// block on the diagonal, two or three for the others) costs about one round trip to memory
// per batch.  lin, a64, a32 may be one array (the caller's values may be the hierarchy's
// own); each index is read and written by one lane only.
template <int B, int NGB, typename T>
__global__ __launch_bounds__(TPB_B) void k_node_rap(int64_t nblk, const int* __restrict__ tptr,
                                                    const int* __restrict__ toff, const int* __restrict__ tlen,
                                                    const int* __restrict__ cout, const int* __restrict__ clen,
                                                    const T* aval, const double* lin, double* a64, float* a32,
                                                    T* __restrict__ cval) {
    constexpr int U = 8;
    const int64_t t = (int64_t)xcd_block() * TPB_B + threadIdx.x;
    const int64_t g = t / NGB;
    const int q = (int)(t % NGB);
    if (g >= nblk || q >= B * B) return;
    const int a = q / B, c = q % B;
    const int k0 = tptr[g], k1 = tptr[g + 1];
    int o[U], lf[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const bool in = k0 + u < k1;
        o[u] = in ? toff[k0 + u] : 0;
        lf[u] = in ? tlen[k0 + u] : 0;
    }
    T acc = 0, part = 0;
    for (int k = k0; k < k1; k += U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            v[u] = 0;
            if (k + u < k1) {
                const int64_t idx = (int64_t)o[u] + (int64_t)a * (lf[u] >> 1) + c;
                if (lin != nullptr) {
                    const double x = lin[idx];
                    a64[idx] = x;
                    if (a32 != nullptr) a32[idx] = (float)x;
                    v[u] = (T)x;
                } else {
                    v[u] = aval[idx];
                }
            }
        }
        int on[U], ln[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int kk = k + U + u;
            const bool in = kk < k1;
            on[u] = in ? toff[kk] : 0;
            ln[u] = in ? tlen[kk] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (k + u < k1) {
                if ((lf[u] & 1) && k + u > k0) {  // a new fine node: its predecessor's sum is complete
                    acc = acc + part;
                    part = 0;
                }
                part = part + v[u];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            o[u] = on[u];
            lf[u] = ln[u];
        }
    }
    acc = acc + part;
    cval[(int64_t)cout[g] + (int64_t)a * clen[g] + c] = acc;
}

// ------------------------------------------------------------------ node prolongation
//
// With P_l = P_node (x) I_B and unit values, row I*B + b of P_l holds one 1 in column
// J*B + b (J the aggregate of node I) or nothing: the prolongation reads one aggregate
// index per node instead of a row pointer, a column and a value per row.  (A restriction
// of the same kind, eight lanes per aggregate walking its members, took 9.5 us per launch
// against 4.9 us for the LDS-staged CSR kernel on R_l, and is not used.)
template <typename T>
__global__ __launch_bounds__(TPB_B) void k_node_prolong(int n, int B, const int* __restrict__ nagg,
                                                        const T* __restrict__ uc, T* __restrict__ u) {
    const int i = xcd_block() * TPB_B + threadIdx.x;
    if (i >= n) return;
    const int J = nagg[i / B];
    const T add = J >= 0 ? uc[J * B + i % B] : (T)0;
    u[i] = u[i] + add;
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
    const int full = std::max(1, node_grid(nn));
    const int nb = std::min(full, rs.cap);
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
    AMG_WITH_B(B_, {
        if (nb < full)
            go(k_node_cg_pq<B, false, true>);
        else if (L.node_pairs)
            go(k_node_cg_pq<B, true, false>);
        else
            go(k_node_cg_pq<B, false, false>);
    });
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

template <typename T>
void launch_node_prolong(const Level& L, int B, const T* uc, T* u, hipStream_t s) {
    if (L.nagg == nullptr) throw Fail{AMG_ERR_STATE, "node transfer map missing"};
    const int n = L.A.nrows;
    timed_launch(k_node_prolong<T>, bgrid(n), TPB_B, 0, s, n, B, (const int*)L.nagg, uc, u);
    HIP_LAUNCH_CHECK();
}

template void launch_node_prolong<double>(const Level&, int, const double*, double*, hipStream_t);
template void launch_node_prolong<float>(const Level&, int, const float*, float*, hipStream_t);

void launch_node_gal_agg(const Csr& P, int B_, int32_t* nagg, int* flags, hipStream_t s) {
    const int nn = P.nrows / B_;
    AMG_WITH_B(B_, timed_launch(k_ngal_agg<B>, bgrid(nn), TPB_B, 0, s, nn, P.ptr, P.col, P.val, nagg, flags));
    HIP_LAUNCH_CHECK();
}

void launch_node_gal_count(const Level& L, const Level& N, int B_, const int32_t* nagg, int32_t* tpos, int32_t* cnt,
                           int* flags, hipStream_t s) {
    need_nodes(L);
    need_nodes(N);
    const int ncn = N.A.nrows / B_;
    AMG_WITH_B(B_, timed_launch(k_ngal_count<B>, bgrid(ncn), TPB_B, 0, s, ncn, L.R.ptr, L.R.col, L.nptr, L.ncol,
                                nagg, N.nptr, N.ncol, tpos, cnt, flags));
    HIP_LAUNCH_CHECK();
}

void launch_node_gal_fill(const Level& L, const Level& N, int B_, const int32_t* tpos, const NodeGal& g, int32_t* cur,
                          int32_t* last, hipStream_t s) {
    const int ncn = N.A.nrows / B_;
    AMG_WITH_B(B_, timed_launch(k_ngal_fill<B>, bgrid(ncn), TPB_B, 0, s, ncn, L.R.ptr, L.R.col, L.nptr, N.nptr, tpos,
                                g.tptr, g.toff, g.tlen, g.cout, g.clen, cur, last));
    HIP_LAUNCH_CHECK();
}

template <typename T>
void launch_node_rap(const NodeGal& g, int B_, const T* aval, const double* lin, double* a64, float* a32, T* cval,
                     hipStream_t s) {
    if (g.nblk <= 0) return;
    auto go = [&](auto kern, int ngb) {
        const int64_t threads = g.nblk * ngb;
        timed_launch(kern, (unsigned)((threads + TPB_B - 1) / TPB_B), TPB_B, 0, s, g.nblk, (const int*)g.tptr,
                     (const int*)g.toff, (const int*)g.tlen, (const int*)g.cout, (const int*)g.clen, aval, lin, a64,
                     a32, cval);
    };
    switch (B_) {
        case 2: go(k_node_rap<2, 4, T>, 4); break;
        case 3: go(k_node_rap<3, 16, T>, 16); break;
        case 4: go(k_node_rap<4, 16, T>, 16); break;
        case 5: go(k_node_rap<5, 32, T>, 32); break;
        case 6: go(k_node_rap<6, 64, T>, 64); break;
        case 7: go(k_node_rap<7, 64, T>, 64); break;
        case 8: go(k_node_rap<8, 64, T>, 64); break;
        default: throw Fail{AMG_ERR_ARG, "block_size must be 1 .. 8"};
    }
    HIP_LAUNCH_CHECK();
}

template void launch_node_rap<double>(const NodeGal&, int, const double*, const double*, double*, float*, double*,
                                      hipStream_t);
template void launch_node_rap<float>(const NodeGal&, int, const float*, const double*, double*, float*, float*,
                                     hipStream_t);
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
