// kernels_setup.hip -- AMG setup on the device (Algorithm 1, Section 2): strength of
// connection, aggregation by a distance-2 maximal independent set, smoothed prolongator,
// restriction R = P^T, Galerkin sparsity patterns, and the coarsest direct solver.
//
// The aggregation decisions are integer results driven by floating-point comparisons;
// they are made with separately rounded products (contraction off) in the same
// association as the definitions below, so that on the same input they are bit-exact
// and independent of scheduling.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_reduce.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>

#include "amg_internal.h"

#pragma clang fp contract(off)

namespace amgmi {

constexpr int TPB = 256;

static inline unsigned blocks_for(int64_t n) {
    int64_t b = (n + TPB - 1) / TPB;
    return (unsigned)(b > 0 ? b : 1);
}

// ------------------------------------------------------------------ input checks

// Rows: monotone pointers, sorted unique in-range columns, finite values and, for a
// square operator, a positive stored diagonal (diag_pos[i] = position of a_ii).
__global__ void k_validate(int n, int ncols, int64_t nnz, int need_diag, const int* __restrict__ ptr,
                           const int* __restrict__ col, const double* __restrict__ val, int* __restrict__ diag_pos,
                           int* __restrict__ flags) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i == 0 && (ptr[0] != 0 || (int64_t)ptr[n] != nnz)) atomicOr(&flags[F_ARG], 1);
    if (i >= n) return;
    const int b = ptr[i], e = ptr[i + 1];
    if (b > e || b < 0 || (int64_t)e > nnz) {
        atomicOr(&flags[F_ARG], 1);
        if (need_diag) diag_pos[i] = -1;
        return;
    }
    int d = -1, prev = -1;
    for (int k = b; k < e; ++k) {
        const int j = col[k];
        if (j < 0 || j >= ncols || j <= prev) atomicOr(&flags[F_ARG], 1);
        prev = j;
        if (val != nullptr && !isfinite(val[k])) atomicOr(&flags[F_ARG], 1);
        if (j == i) d = k;
    }
    if (!need_diag) return;
    diag_pos[i] = d;
    if (d < 0 || (val != nullptr && !(val[d] > 0.0))) atomicOr(&flags[F_NOT_SPD], 1);
}

void launch_validate(const Csr& A, int32_t* diag_pos, int* flags, hipStream_t s) {
    const int need_diag = diag_pos != nullptr ? 1 : 0;
    k_validate<<<blocks_for(A.nrows), TPB, 0, s>>>(A.nrows, A.ncols, A.nnz, need_diag, A.ptr, A.col, A.val,
                                                   diag_pos, flags);
    HIP_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ strength

// Entry k = (i,j), j != i, is strong when (a_ij * a_ji) > eps2 * |a_ii * a_jj|, with
// eps2 = eps * eps.  tpos[k] is the position of (j,i); a missing (j,i) means the pattern is
// not structurally symmetric.  A row without strong entries is isolated.
__global__ void k_strength(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                           const double* __restrict__ val, const int* __restrict__ diag_pos, double eps2,
                           uint8_t* __restrict__ strong, int* __restrict__ tpos, uint8_t* __restrict__ isolated,
                           int* __restrict__ flags) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n) return;
    const double aii = val[diag_pos[i]];
    bool any = false;
    for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
        const int j = col[k];
        if (j == i) {
            strong[k] = 0;
            tpos[k] = k;
            continue;
        }
        int lo = ptr[j], hi = ptr[j + 1] - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (col[mid] < i)
                lo = mid + 1;
            else
                hi = mid;
        }
        if (hi < lo || col[lo] != i) {
            atomicOr(&flags[F_PATTERN], 1);
            strong[k] = 0;
            tpos[k] = k;
            continue;
        }
        tpos[k] = lo;
        const double ajj = val[diag_pos[j]];
        const double lhs = val[k] * val[lo];
        const double rhs = eps2 * fabs(aii * ajj);
        const bool s = lhs > rhs;
        strong[k] = s ? 1 : 0;
        any = any || s;
    }
    isolated[i] = any ? 0 : 1;
}

void launch_strength(const Csr& A, const int32_t* diag_pos, double eps2, uint8_t* strong, int32_t* tpos,
                     uint8_t* isolated, int* flags, hipStream_t s) {
    k_strength<<<blocks_for(A.nrows), TPB, 0, s>>>(A.nrows, A.ptr, A.col, A.val, diag_pos, eps2, strong, tpos,
                                                   isolated, flags);
    HIP_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ MIS-2

// Priority of node i: the SplitMix64 finaliser (Steele, Lea, Flood 2014) of i, a
// bijection on 64-bit integers, so priorities never tie.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

enum : uint8_t { ST_UNDECIDED = 0, ST_ROOT = 1, ST_REMOVED = 2, ST_ISOLATED = 3 };

__global__ void k_mis_init(int n, const uint8_t* __restrict__ isolated, uint8_t* __restrict__ state) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i < n) state[i] = isolated[i] ? ST_ISOLATED : ST_UNDECIDED;
}

// m1[i] = max priority of an undecided node among i and its strong neighbours (0: none).
__global__ void k_mis_max1(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                           const uint8_t* __restrict__ strong, const uint8_t* __restrict__ state,
                           uint64_t* __restrict__ m1) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n) return;
    uint64_t m = state[i] == ST_UNDECIDED ? mix64((uint64_t)i) : 0;
    for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
        if (!strong[k]) continue;
        const int j = col[k];
        if (state[j] == ST_UNDECIDED) {
            const uint64_t p = mix64((uint64_t)j);
            m = p > m ? p : m;
        }
    }
    m1[i] = m;
}

// An undecided node whose priority is the largest among undecided nodes within strong
// distance 2 becomes a root.  (Repeating this round by round yields exactly the set a
// sequential greedy pass in decreasing priority order builds: every node of higher
// priority nearby has been decided before.)
__global__ void k_mis_max2(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                           const uint8_t* __restrict__ strong, const uint64_t* __restrict__ m1,
                           uint8_t* __restrict__ state) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n || state[i] != ST_UNDECIDED) return;
    uint64_t m = m1[i];
    for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
        if (!strong[k]) continue;
        const uint64_t p = m1[col[k]];
        m = p > m ? p : m;
    }
    if (m == mix64((uint64_t)i)) state[i] = ST_ROOT;
}

// c1[i] = i is a root or has a strong root neighbour.
__global__ void k_mis_cover1(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                             const uint8_t* __restrict__ strong, const uint8_t* __restrict__ state,
                             uint8_t* __restrict__ c1) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n) return;
    bool c = state[i] == ST_ROOT;
    for (int k = ptr[i]; k < ptr[i + 1] && !c; ++k)
        if (strong[k] && state[col[k]] == ST_ROOT) c = true;
    c1[i] = c ? 1 : 0;
}

// Undecided nodes within strong distance 2 of a root are removed; any node still
// undecided raises the flag for another round.
__global__ void k_mis_cover2(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                             const uint8_t* __restrict__ strong, const uint8_t* __restrict__ c1,
                             uint8_t* __restrict__ state, int* __restrict__ flags) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n || state[i] != ST_UNDECIDED) return;
    bool c = c1[i] != 0;
    for (int k = ptr[i]; k < ptr[i + 1] && !c; ++k)
        if (strong[k] && c1[col[k]]) c = true;
    if (c)
        state[i] = ST_REMOVED;
    else
        flags[F_UNDECIDED] = 1;
}

void run_mis2(const Csr& A, const uint8_t* strong, const uint8_t* isolated, uint8_t* state, int* flags,
              int* h_flags, hipStream_t s) {
    const int n = A.nrows;
    uint64_t* m1 = dnew<uint64_t>((size_t)n, s);
    uint8_t* c1 = dnew<uint8_t>((size_t)n, s);
    const unsigned nb = blocks_for(n);
    k_mis_init<<<nb, TPB, 0, s>>>(n, isolated, state);
    HIP_LAUNCH_CHECK();
    for (int round = 0;; ++round) {
        k_mis_max1<<<nb, TPB, 0, s>>>(n, A.ptr, A.col, strong, state, m1);
        k_mis_max2<<<nb, TPB, 0, s>>>(n, A.ptr, A.col, strong, m1, state);
        k_mis_cover1<<<nb, TPB, 0, s>>>(n, A.ptr, A.col, strong, state, c1);
        HIP_CHECK(hipMemsetAsync(flags + F_UNDECIDED, 0, sizeof(int), s));
        k_mis_cover2<<<nb, TPB, 0, s>>>(n, A.ptr, A.col, strong, c1, state, flags);
        HIP_LAUNCH_CHECK();
        HIP_CHECK(hipMemcpyAsync(h_flags, flags, F_COUNT * sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        if (!h_flags[F_UNDECIDED]) break;
        if (round > 4096) throw Fail{AMG_ERR_HIP, "MIS-2 did not terminate"};
    }
    dfree(m1, s);
    dfree(c1, s);
}

// ------------------------------------------------------------------ aggregation

// Pass 1: roots and their strong neighbours take the root's id (roots are at least 3
// apart, so at most one root is adjacent).
__global__ void k_agg_pass1(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                            const uint8_t* __restrict__ strong, const uint8_t* __restrict__ state,
                            const int* __restrict__ root_id, int* __restrict__ agg1) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n) return;
    int a = -1;
    if (state[i] == ST_ROOT) {
        a = root_id[i];
    } else if (state[i] != ST_ISOLATED) {
        for (int k = ptr[i]; k < ptr[i + 1]; ++k)
            if (strong[k] && state[col[k]] == ST_ROOT) a = root_id[col[k]];
    }
    agg1[i] = a;
}

// Pass 2: a node left over joins the pass-1 aggregate of its strong neighbour j with the
// largest a_ij * a_ji (ties: the smaller aggregate id).
__global__ void k_agg_pass2(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                            const double* __restrict__ val, const uint8_t* __restrict__ strong,
                            const int* __restrict__ tpos, const uint8_t* __restrict__ state,
                            const int* __restrict__ agg1, int* __restrict__ agg, int* __restrict__ flags) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n) return;
    const int a1 = agg1[i];
    if (a1 >= 0 || state[i] == ST_ISOLATED) {
        agg[i] = a1;
        return;
    }
    int best = -1;
    double best_w = 0.0;
    for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
        if (!strong[k]) continue;
        const int aj = agg1[col[k]];
        if (aj < 0) continue;
        const double w = val[k] * val[tpos[k]];
        if (best < 0 || w > best_w || (w == best_w && aj < best)) {
            best = aj;
            best_w = w;
        }
    }
    if (best < 0) atomicOr(&flags[F_NOAGG], 1);
    agg[i] = best;
}

__global__ void k_is_root(int n, const uint8_t* __restrict__ state, int* __restrict__ r) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i < n) r[i] = state[i] == ST_ROOT ? 1 : 0;
}

template <typename Tin, typename Tout>
static void scan_exclusive(const Tin* in, Tout* out, int64_t n, hipStream_t s) {
    size_t bytes = 0;
    HIP_CHECK(rocprim::exclusive_scan(nullptr, bytes, in, out, Tout(0), (size_t)n, rocprim::plus<Tout>(), s));
    void* tmp = dalloc(bytes, s);
    HIP_CHECK(rocprim::exclusive_scan(tmp, bytes, in, out, Tout(0), (size_t)n, rocprim::plus<Tout>(), s));
    dfree(tmp, s);
}

void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s) {
    scan_exclusive<int32_t, int32_t>(in, out, n, s);
}

void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
    scan_exclusive<int64_t, int64_t>(in, out, n, s);
}

int64_t max_i64(const int64_t* in, int64_t n, hipStream_t s) {
    int64_t* out = dnew<int64_t>(1, s);
    size_t bytes = 0;
    HIP_CHECK(rocprim::reduce(nullptr, bytes, in, out, (size_t)n, rocprim::maximum<int64_t>(), s));
    void* tmp = dalloc(bytes, s);
    HIP_CHECK(rocprim::reduce(tmp, bytes, in, out, (size_t)n, rocprim::maximum<int64_t>(), s));
    int64_t h = 0;
    HIP_CHECK(hipMemcpyAsync(&h, out, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    dfree(tmp, s);
    dfree(out, s);
    return h;
}

int32_t run_aggregate(const Csr& A, const uint8_t* strong, const int32_t* tpos, const uint8_t* state, int32_t* agg,
                      int* flags, int* h_flags, hipStream_t s) {
    const int n = A.nrows;
    const unsigned nb = blocks_for(n);
    int* isr = dnew<int>((size_t)n + 1, s);
    int* id = dnew<int>((size_t)n + 1, s);
    int* agg1 = dnew<int>((size_t)n, s);
    k_is_root<<<nb, TPB, 0, s>>>(n, state, isr);
    HIP_LAUNCH_CHECK();
    HIP_CHECK(hipMemsetAsync(isr + n, 0, sizeof(int), s));
    scan_exclusive<int, int>(isr, id, n + 1, s);
    k_agg_pass1<<<nb, TPB, 0, s>>>(n, A.ptr, A.col, strong, state, id, agg1);
    k_agg_pass2<<<nb, TPB, 0, s>>>(n, A.ptr, A.col, A.val, strong, tpos, state, agg1, agg, flags);
    HIP_LAUNCH_CHECK();
    int32_t nc = 0;
    HIP_CHECK(hipMemcpyAsync(&nc, id + n, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(h_flags, flags, F_COUNT * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    dfree(isr, s);
    dfree(id, s);
    dfree(agg1, s);
    if (h_flags[F_NOAGG]) throw Fail{AMG_ERR_PATTERN, "node left without an aggregate"};
    return nc;
}

// ------------------------------------------------------------------ block systems

// Node I owns rows I*B .. I*B+B-1.  Its rows must list the same columns, in groups of B
// consecutive columns starting at a multiple of B (full blocks); the node row then has
// one entry per group.  The input has passed k_validate, so every index is in range.
__global__ void k_node_count(int nn, int B, const int* __restrict__ ptr, const int* __restrict__ col,
                             int* __restrict__ cnt, int* __restrict__ flags) {
    const int I = xcd_block() * TPB + threadIdx.x;
    if (I >= nn) return;
    const int r0 = I * B;
    const int b0 = ptr[r0], len = ptr[r0 + 1] - b0;
    bool ok = len % B == 0;
    for (int c = 1; c < B && ok; ++c) {
        const int bc = ptr[r0 + c];
        if (ptr[r0 + c + 1] - bc != len) ok = false;
        for (int k = 0; k < len && ok; ++k)
            if (col[bc + k] != col[b0 + k]) ok = false;
    }
    for (int g = 0; g < len / B && ok; ++g) {
        const int c0 = col[b0 + g * B];
        if (c0 % B != 0) ok = false;
        for (int q = 1; q < B && ok; ++q)
            if (col[b0 + g * B + q] != c0 + q) ok = false;
    }
    if (!ok) atomicOr(&flags[F_BLOCK], 1);
    cnt[I] = ok ? len / B : 0;
}

// Entry (I, J) of the node matrix: the Frobenius norm of block (I, J), its squares summed
// over the block's rows in order and along each row in column order, then one square root.
__global__ void k_node_fill(int nn, int B, const int* __restrict__ ptr, const int* __restrict__ col,
                            const double* __restrict__ val, const int* __restrict__ Nptr, int* __restrict__ Ncol,
                            double* __restrict__ Nval) {
    const int I = xcd_block() * TPB + threadIdx.x;
    if (I >= nn) return;
    const int r0 = I * B;
    const int nb = Nptr[I], ng = Nptr[I + 1] - nb;
    for (int g = 0; g < ng; ++g) {
        Ncol[nb + g] = col[ptr[r0] + g * B] / B;
        if (val == nullptr) continue;  // the pattern only
        double ss = 0.0;
        for (int c = 0; c < B; ++c) {
            const double* v = val + ptr[r0 + c] + g * B;
            for (int q = 0; q < B; ++q) ss += v[q] * v[q];
        }
        Nval[nb + g] = sqrt(ss);
    }
}

// Unknown b of node I joins unknown b of the node's aggregate (none when the node is
// isolated); an entry of block (I, J) takes the strength flag of node entry (I, J).
__global__ void k_node_expand(int n, int B, const int* __restrict__ ptr, const int* __restrict__ Nptr,
                              const uint8_t* __restrict__ nstrong, const int* __restrict__ nagg,
                              uint8_t* __restrict__ strong, int* __restrict__ agg) {
    const int r = xcd_block() * TPB + threadIdx.x;
    if (r >= n) return;
    const int I = r / B;
    const int a = nagg[I];
    agg[r] = a >= 0 ? a * B + (r - I * B) : -1;
    const int b = ptr[r], nb = Nptr[I];
    for (int k = b; k < ptr[r + 1]; ++k) strong[k] = nstrong[nb + (k - b) / B];
}

void build_node_matrix(const Csr& A, int B, Csr& Nm, int* flags, int* h_flags, hipStream_t s) {
    if (B < 2 || A.nrows % B != 0) throw Fail{AMG_ERR_ARG, "block_size does not divide the row count"};
    const int nn = A.nrows / B;
    int* cnt = dnew<int>((size_t)nn + 1, s);
    k_node_count<<<blocks_for(nn), TPB, 0, s>>>(nn, B, A.ptr, A.col, cnt, flags);
    HIP_LAUNCH_CHECK();
    HIP_CHECK(hipMemsetAsync(cnt + nn, 0, sizeof(int), s));
    Nm.nrows = Nm.ncols = nn;
    Nm.ptr = dnew<int32_t>((size_t)nn + 1, s);
    scan_exclusive<int, int>(cnt, Nm.ptr, nn + 1, s);
    int32_t nnz = 0;
    HIP_CHECK(hipMemcpyAsync(&nnz, Nm.ptr + nn, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(h_flags, flags, F_COUNT * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    dfree(cnt, s);
    if (h_flags[F_BLOCK]) {
        dfree(Nm.ptr, s);
        Nm.ptr = nullptr;
        throw Fail{AMG_ERR_PATTERN, "block_size needs full blocks with the same columns in every row of a node"};
    }
    Nm.nnz = nnz;
    Nm.col = dnew<int32_t>((size_t)nnz, s);
    Nm.val = A.val != nullptr ? dnew<double>((size_t)nnz, s) : nullptr;
    k_node_fill<<<blocks_for(nn), TPB, 0, s>>>(nn, B, A.ptr, A.col, A.val, Nm.ptr, Nm.col, Nm.val);
    HIP_LAUNCH_CHECK();
}

void launch_node_expand(const Csr& A, int B, const Csr& Nm, const uint8_t* nstrong, const int32_t* nagg,
                        uint8_t* strong, int32_t* agg, hipStream_t s) {
    k_node_expand<<<blocks_for(A.nrows), TPB, 0, s>>>(A.nrows, B, A.ptr, Nm.ptr, nstrong, nagg, strong, agg);
    HIP_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ prolongator

// Filtered operator A_F (lumped): for a non-isolated row the diagonal is
// d_i = a_ii + sum of weak off-diagonal entries (column order), the strong entries are
// kept; an isolated row keeps a_ii only.  ratio_i = sum_j |aF_ij| / |d_i| (column order);
// rho = max_i ratio_i (exact, so order free) is accumulated on the IEEE bit pattern, which
// orders like the value for positive doubles.
__global__ void k_filter(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                         const double* __restrict__ val, const uint8_t* __restrict__ strong,
                         const int* __restrict__ diag_pos, const int* __restrict__ agg, double* __restrict__ dF,
                         unsigned long long* __restrict__ rho_bits) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n) return;
    const bool iso = agg[i] < 0;
    double d = val[diag_pos[i]];
    if (!iso)
        for (int k = ptr[i]; k < ptr[i + 1]; ++k)
            if (col[k] != i && !strong[k]) d += val[k];
    double s = 0.0;
    for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
        if (col[k] == i)
            s += fabs(d);
        else if (!iso && strong[k])
            s += fabs(val[k]);
    }
    dF[i] = d;
    const double ratio = s / fabs(d);
    atomicMax(rho_bits, (unsigned long long)__double_as_longlong(ratio));
}

// Number of distinct aggregates among the columns of row i of A_F (diagonal and strong
// entries); that is the length of row i of A_F P_tent and of the smoothed P.
__global__ void k_pcount(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                         const uint8_t* __restrict__ strong, const int* __restrict__ agg, int plain,
                         int* __restrict__ cnt) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n) return;
    if (agg[i] < 0) {
        cnt[i] = 0;
        return;
    }
    if (plain) {
        cnt[i] = 1;
        return;
    }
    const int b = ptr[i], e = ptr[i + 1];
    int c = 0;
    for (int k = b; k < e; ++k) {
        const int j = col[k];
        if (j != i && !strong[k]) continue;
        const int a = agg[j];
        bool seen = false;
        for (int q = b; q < k && !seen; ++q) {
            const int jq = col[q];
            if ((jq == i || strong[q]) && agg[jq] == a) seen = true;
        }
        if (!seen) ++c;
    }
    cnt[i] = c;
}

// Row i of P = P_tent - (omega / d_i) * (A_F P_tent), omega = (4/3) / rho.  Columns are
// the distinct aggregates of the row in increasing order; for column J the sum over the
// row's entries with aggregate J is taken in column order starting from 0.
__global__ void k_pfill(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                        const double* __restrict__ val, const uint8_t* __restrict__ strong,
                        const int* __restrict__ agg, const double* __restrict__ dF,
                        const unsigned long long* __restrict__ rho_bits, int plain, const int* __restrict__ Pptr,
                        int* __restrict__ Pcol, double* __restrict__ Pval) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n) return;
    const int ai = agg[i];
    if (ai < 0) return;
    int pos = Pptr[i];
    if (plain) {
        Pcol[pos] = ai;
        Pval[pos] = 1.0;
        return;
    }
    const double rho = __longlong_as_double((long long)*rho_bits);
    const double omega = (4.0 / 3.0) / rho;
    const double scale = omega / dF[i];
    const int b = ptr[i], e = ptr[i + 1];
    int last = -1;
    for (;;) {
        int J = 0x7fffffff;
        for (int k = b; k < e; ++k) {
            const int j = col[k];
            if (j != i && !strong[k]) continue;
            const int a = agg[j];
            if (a > last && a < J) J = a;
        }
        if (J == 0x7fffffff) break;
        double sJ = 0.0;
        for (int k = b; k < e; ++k) {
            const int j = col[k];
            if (j != i && !strong[k]) continue;
            if (agg[j] == J) sJ += (j == i) ? dF[i] : val[k];
        }
        const double pt = (J == ai) ? 1.0 : 0.0;
        Pcol[pos] = J;
        Pval[pos] = pt - scale * sJ;
        ++pos;
        last = J;
    }
}

void build_prolongator(const Csr& A, const uint8_t* strong, const int32_t* diag_pos, const int32_t* agg, int32_t nc,
                       int plain, Csr& P, hipStream_t s) {
    const int n = A.nrows;
    const unsigned nb = blocks_for(n);
    double* dF = nullptr;
    unsigned long long* rho_bits = nullptr;
    if (!plain) {
        dF = dnew<double>((size_t)n, s);
        rho_bits = dnew<unsigned long long>(1, s);
        HIP_CHECK(hipMemsetAsync(rho_bits, 0, sizeof(unsigned long long), s));
        k_filter<<<nb, TPB, 0, s>>>(n, A.ptr, A.col, A.val, strong, diag_pos, agg, dF, rho_bits);
        HIP_LAUNCH_CHECK();
    }
    int* cnt = dnew<int>((size_t)n + 1, s);
    k_pcount<<<nb, TPB, 0, s>>>(n, A.ptr, A.col, strong, agg, plain, cnt);
    HIP_LAUNCH_CHECK();
    HIP_CHECK(hipMemsetAsync(cnt + n, 0, sizeof(int), s));
    P.nrows = n;
    P.ncols = nc;
    P.ptr = dnew<int32_t>((size_t)n + 1, s);
    scan_exclusive<int, int>(cnt, P.ptr, n + 1, s);
    int32_t nnz = 0;
    HIP_CHECK(hipMemcpyAsync(&nnz, P.ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    P.nnz = nnz;
    P.col = dnew<int32_t>((size_t)nnz, s);
    P.val = dnew<double>((size_t)nnz, s);
    k_pfill<<<nb, TPB, 0, s>>>(n, A.ptr, A.col, A.val, strong, agg, dF, rho_bits, plain, P.ptr, P.col, P.val);
    HIP_LAUNCH_CHECK();
    dfree(cnt, s);
    if (dF) dfree(dF, s);
    if (rho_bits) dfree(rho_bits, s);
}

// ------------------------------------------------------------------ sorting helpers

template <typename K, typename V>
static void radix_sort_pairs(K* kin, K* kout, V* vin, V* vout, int64_t n, int end_bit, hipStream_t s) {
    size_t bytes = 0;
    HIP_CHECK(rocprim::radix_sort_pairs(nullptr, bytes, kin, kout, vin, vout, (size_t)n, 0u, (unsigned)end_bit, s));
    void* tmp = dalloc(bytes, s);
    HIP_CHECK(rocprim::radix_sort_pairs(tmp, bytes, kin, kout, vin, vout, (size_t)n, 0u, (unsigned)end_bit, s));
    dfree(tmp, s);
}

template <typename K>
static void radix_sort_keys(K* kin, K* kout, int64_t n, int end_bit, hipStream_t s) {
    size_t bytes = 0;
    HIP_CHECK(rocprim::radix_sort_keys(nullptr, bytes, kin, kout, (size_t)n, 0u, (unsigned)end_bit, s));
    void* tmp = dalloc(bytes, s);
    HIP_CHECK(rocprim::radix_sort_keys(tmp, bytes, kin, kout, (size_t)n, 0u, (unsigned)end_bit, s));
    dfree(tmp, s);
}

static int bits_for(uint64_t v) {
    int b = 1;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

// ptr[r] = number of keys (sorted, row-major key = r * ncols + c) with row < r.
__global__ void k_rowptr_from_keys(int nrows, int64_t nkeys, const uint64_t* __restrict__ keys, uint64_t ncols,
                                   int* __restrict__ ptr) {
    const int r = blockIdx.x * TPB + threadIdx.x;
    if (r > nrows) return;
    const uint64_t target = (uint64_t)r * ncols;
    int64_t lo = 0, hi = nkeys;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < target)
            lo = mid + 1;
        else
            hi = mid;
    }
    ptr[r] = (int)lo;
}

__global__ void k_cols_from_keys(int64_t nkeys, const uint64_t* __restrict__ keys, uint64_t ncols,
                                 int* __restrict__ col) {
    for (int64_t k = blockIdx.x * (int64_t)TPB + threadIdx.x; k < nkeys; k += (int64_t)gridDim.x * TPB)
        col[k] = (int)(keys[k] % ncols);
}

// ------------------------------------------------------------------ transpose

__global__ void k_transpose_keys(int n, const int* __restrict__ ptr, const int* __restrict__ col, uint64_t nrows,
                                 uint64_t* __restrict__ keys, int* __restrict__ idx) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i >= n) return;
    for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
        keys[k] = (uint64_t)col[k] * nrows + (uint64_t)i;
        idx[k] = k;
    }
}

__global__ void k_gather_vals(int64_t nnz, const int* __restrict__ idx, const double* __restrict__ v,
                              double* __restrict__ out) {
    for (int64_t k = blockIdx.x * (int64_t)TPB + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * TPB)
        out[k] = v[idx[k]];
}

static unsigned gs_blocks(int64_t n) {
    int64_t b = (n + TPB - 1) / TPB;
    if (b > 16384) b = 16384;
    return (unsigned)(b > 0 ? b : 1);
}

// R = P^T with sorted columns: sort the entries by (column, row).
void build_transpose(const Csr& P, Csr& R, hipStream_t s) {
    const int64_t nnz = P.nnz;
    R.nrows = P.ncols;
    R.ncols = P.nrows;
    R.nnz = nnz;
    R.ptr = dnew<int32_t>((size_t)R.nrows + 1, s);
    R.col = dnew<int32_t>((size_t)nnz, s);
    R.val = dnew<double>((size_t)nnz, s);
    uint64_t* k0 = dnew<uint64_t>((size_t)nnz, s);
    uint64_t* k1 = dnew<uint64_t>((size_t)nnz, s);
    int* i0 = dnew<int>((size_t)nnz, s);
    int* i1 = dnew<int>((size_t)nnz, s);
    k_transpose_keys<<<blocks_for(P.nrows), TPB, 0, s>>>(P.nrows, P.ptr, P.col, (uint64_t)P.nrows, k0, i0);
    HIP_LAUNCH_CHECK();
    const int eb = bits_for((uint64_t)P.ncols * (uint64_t)P.nrows);
    if (nnz > 0) radix_sort_pairs<uint64_t, int>(k0, k1, i0, i1, nnz, eb, s);
    k_rowptr_from_keys<<<blocks_for(R.nrows + 1), TPB, 0, s>>>(R.nrows, nnz, k1, (uint64_t)P.nrows, R.ptr);
    k_cols_from_keys<<<gs_blocks(nnz), TPB, 0, s>>>(nnz, k1, (uint64_t)P.nrows, R.col);
    k_gather_vals<<<gs_blocks(nnz), TPB, 0, s>>>(nnz, i1, P.val, R.val);
    HIP_LAUNCH_CHECK();
    dfree(k0, s);
    dfree(k1, s);
    dfree(i0, s);
    dfree(i1, s);
}

// ------------------------------------------------------------------ symbolic product

// Upper bound of the length of row i of A B (sum of the B row lengths it references).
__global__ void k_spgemm_ub(int n, const int* __restrict__ Aptr, const int* __restrict__ Acol,
                            const int* __restrict__ Bptr, int64_t* __restrict__ ub) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i > n) return;
    if (i == n) {
        ub[n] = 0;
        return;
    }
    int64_t c = 0;
    for (int k = Aptr[i]; k < Aptr[i + 1]; ++k) {
        const int j = Acol[k];
        c += Bptr[j + 1] - Bptr[j];
    }
    ub[i] = c;
}

__global__ void k_spgemm_expand(int n, const int* __restrict__ Aptr, const int* __restrict__ Acol,
                                const int* __restrict__ Bptr, const int* __restrict__ Bcol,
                                const int64_t* __restrict__ off, uint64_t ncols, uint64_t* __restrict__ keys) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n) return;
    int64_t pos = off[i];
    const uint64_t base = (uint64_t)i * ncols;
    for (int k = Aptr[i]; k < Aptr[i + 1]; ++k) {
        const int j = Acol[k];
        for (int q = Bptr[j]; q < Bptr[j + 1]; ++q) keys[pos++] = base + (uint64_t)Bcol[q];
    }
}

// Pattern of C = A B (structural: every product term creates its entry), sorted columns:
// expand all candidate (row, column) pairs, sort, and keep the unique ones.
void symbolic_spgemm(const Csr& A, const Csr& B, Csr& C, hipStream_t s) {
    const int n = A.nrows;
    int64_t* ub = dnew<int64_t>((size_t)n + 1, s);
    int64_t* off = dnew<int64_t>((size_t)n + 1, s);
    k_spgemm_ub<<<blocks_for(n + 1), TPB, 0, s>>>(n, A.ptr, A.col, B.ptr, ub);
    HIP_LAUNCH_CHECK();
    scan_exclusive<int64_t, int64_t>(ub, off, n + 1, s);
    int64_t total = 0;
    HIP_CHECK(hipMemcpyAsync(&total, off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (total >= ((int64_t)1 << 31)) throw Fail{AMG_ERR_ARG, "Galerkin product too large for int32 indexing"};
    C.nrows = n;
    C.ncols = B.ncols;
    C.ptr = dnew<int32_t>((size_t)n + 1, s);
    uint64_t* k0 = dnew<uint64_t>((size_t)total, s);
    uint64_t* k1 = dnew<uint64_t>((size_t)total, s);
    k_spgemm_expand<<<blocks_for(n), TPB, 0, s>>>(n, A.ptr, A.col, B.ptr, B.col, off, (uint64_t)B.ncols, k0);
    HIP_LAUNCH_CHECK();
    const int eb = bits_for((uint64_t)n * (uint64_t)B.ncols);
    if (total > 0) radix_sort_keys<uint64_t>(k0, k1, total, eb, s);
    // unique keys into k0
    int* nsel = dnew<int>(1, s);
    size_t bytes = 0;
    HIP_CHECK(rocprim::unique(nullptr, bytes, k1, k0, nsel, (size_t)total, rocprim::equal_to<uint64_t>(), s));
    void* tmp = dalloc(bytes, s);
    HIP_CHECK(rocprim::unique(tmp, bytes, k1, k0, nsel, (size_t)total, rocprim::equal_to<uint64_t>(), s));
    dfree(tmp, s);
    int nnz = 0;
    if (total > 0) {
        HIP_CHECK(hipMemcpyAsync(&nnz, nsel, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
    }
    C.nnz = nnz;
    C.col = dnew<int32_t>((size_t)nnz, s);
    k_rowptr_from_keys<<<blocks_for(n + 1), TPB, 0, s>>>(n, nnz, k0, (uint64_t)B.ncols, C.ptr);
    k_cols_from_keys<<<gs_blocks(nnz), TPB, 0, s>>>(nnz, k0, (uint64_t)B.ncols, C.col);
    HIP_LAUNCH_CHECK();
    dfree(nsel, s);
    dfree(k0, s);
    dfree(k1, s);
    dfree(ub, s);
    dfree(off, s);
}

// ------------------------------------------------------------------ coarsest level

template <typename T>
__global__ void k_densify(int n, const int* __restrict__ ptr, const int* __restrict__ col, const T* __restrict__ val,
                          double* __restrict__ D) {
    const int i = blockIdx.x;
    if (i >= n) return;
    for (int j = threadIdx.x; j < n; j += blockDim.x) D[(size_t)i * n + j] = 0.0;
    __syncthreads();
    for (int k = ptr[i] + threadIdx.x; k < ptr[i + 1]; k += blockDim.x) D[(size_t)i * n + col[k]] = (double)val[k];
}

template <typename T>
void launch_densify(const Csr& A, double* D, hipStream_t s) {
    k_densify<T><<<(unsigned)(A.nrows > 0 ? A.nrows : 1), 128, 0, s>>>(A.nrows, A.ptr, A.col, A.v<T>(), D);
    HIP_LAUNCH_CHECK();
}
template void launch_densify<double>(const Csr&, double*, hipStream_t);
template void launch_densify<float>(const Csr&, double*, hipStream_t);

// In-place inverse of an SPD matrix by Gauss-Jordan elimination without pivoting (the
// pivots are the positive LDL^T pivots of an SPD matrix; a non-positive or non-finite
// pivot reports "not SPD" in scal[S_COARSE]).  One workgroup, n <= COARSE_LDS_MAX: the
// matrix is held in LDS (128 x 128 FP64 = 128 KiB of the 160 KiB available).
__global__ __launch_bounds__(1024) void k_dense_inverse(int n, double* __restrict__ Mg, double* __restrict__ scal) {
    constexpr int CAP = COARSE_LDS_MAX;
    __shared__ double colk[CAP];
    __shared__ double rowk[CAP];
    __shared__ int bad;
    __shared__ double M[COARSE_LDS_MAX * COARSE_LDS_MAX];
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) M[e] = Mg[e];
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double p = M[(size_t)k * n + k];
        if (!(p > 0.0) || !isfinite(p)) {  // uniform: every thread reads the same pivot
            if (threadIdx.x == 0) bad = 1;
            break;
        }
        const double pinv = 1.0 / p;
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            colk[t] = M[(size_t)t * n + k];
            rowk[t] = (t == k) ? pinv : M[(size_t)k * n + t] * pinv;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
            const int i = e / n, j = e - i * n;
            double v;
            if (i == k)
                v = rowk[j];
            else if (j == k)
                v = -colk[i] * pinv;
            else
                v = M[e] - colk[i] * rowk[j];
            M[e] = v;
        }
        __syncthreads();
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) Mg[e] = M[e];
    if (threadIdx.x == 0) scal[S_COARSE] = bad ? 1.0 : 0.0;
}

// ------------------------------------------------------------------ blocked Gauss-Jordan
//
// Coarsest levels larger than COARSE_LDS_MAX are inverted in place by the same Gauss-Jordan
// elimination taken a block of BGJ pivots at a time.  With X = M_KK^{-1} for the pivot
// block K, one block step maps
//   M_KJ <- X M_KJ,   M_IJ <- M_IJ - M_IK X M_KJ,   M_IK <- -M_IK X,   M_KK <- X
// (I, J != K), which is the composition of the scalar steps of K's pivots.  Step k runs as
// two launches: k_bgj_pivot inverts M_KK (one workgroup, by the same block steps 16 pivots
// at a time: see bgj_invert_lds; every pivot checked positive) while other workgroups
// finish step k-1 (its row block, column block and diagonal block), then k_bgj_update
// applies the rank-BGJ update to every block (I, J) outside row and column K, forming
// X M_KJ itself; a last k_bgj_pivot finishes the last step.  X of two consecutive steps live in two slots of a scratch
// buffer.  The 64 x 64 x 64 block products run on the FP64 matrix cores: each of the 16
// waves of a workgroup owns one 16 x 16 tile of the product and accumulates it over 16
// steps of V_MFMA_F64_16X16X4F64.
constexpr int BGJ = 64;
constexpr int BGJ_THREADS = 1024;
constexpr int BGJ_RPT = BGJ * BGJ / BGJ_THREADS;  // tile elements per thread
// Row stride of a tile in LDS: 68 doubles put the 16 rows that an operand read of the
// matrix instruction touches in different banks (2-way at most), where 64 would put
// them all in one.
constexpr int BGJ_LD = 68;
typedef double bgj_v4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int bgj_size(int n, int b) { return min(BGJ, n - b * BGJ); }

// The i-th block index other than kp.
__device__ __forceinline__ int bgj_other(int i, int kp) { return i < kp ? i : i + 1; }

// A BGJ x BGJ tile spread over the threads: thread t holds rows t / BGJ + (BGJ_THREADS /
// BGJ) m (m < BGJ_RPT) of column t % BGJ.  Every global load of a tile is issued before any
// is used.
constexpr int BGJ_RSTEP = BGJ_THREADS / BGJ;

// Block (I, J) of the row-major n x n M (zero outside the matrix).
__device__ __forceinline__ void bgj_fetch(const double* __restrict__ M, int n, int I, int J, double (&v)[BGJ_RPT]) {
    const int bi = bgj_size(n, I), bj = bgj_size(n, J);
    const int r = threadIdx.x / BGJ, q = threadIdx.x % BGJ;
    const double* base = M + (size_t)(I * BGJ + r) * n + (size_t)J * BGJ + q;
#pragma unroll
    for (int m = 0; m < BGJ_RPT; ++m)
        v[m] = (r + BGJ_RSTEP * m < bi && q < bj) ? base[(size_t)(BGJ_RSTEP * m) * n] : 0.0;
}

// A tile stored densely (row stride BGJ), as X is.
__device__ __forceinline__ void bgj_fetch_dense(const double* __restrict__ X, double (&v)[BGJ_RPT]) {
#pragma unroll
    for (int m = 0; m < BGJ_RPT; ++m) v[m] = X[threadIdx.x + m * BGJ_THREADS];
}

// Into LDS s (row stride BGJ_LD).
__device__ __forceinline__ void bgj_put(double* s, const double (&v)[BGJ_RPT]) {
    const int r = threadIdx.x / BGJ, q = threadIdx.x % BGJ;
#pragma unroll
    for (int m = 0; m < BGJ_RPT; ++m) s[(r + BGJ_RSTEP * m) * BGJ_LD + q] = v[m];
}

// Writes the tile of registers v to block (I, J) of M.
__device__ __forceinline__ void bgj_store(double* __restrict__ M, int n, int I, int J, const double (&v)[BGJ_RPT]) {
    const int bi = bgj_size(n, I), bj = bgj_size(n, J);
    const int r = threadIdx.x / BGJ, q = threadIdx.x % BGJ;
    double* base = M + (size_t)(I * BGJ + r) * n + (size_t)J * BGJ + q;
#pragma unroll
    for (int m = 0; m < BGJ_RPT; ++m)
        if (r + BGJ_RSTEP * m < bi && q < bj) base[(size_t)(BGJ_RSTEP * m) * n] = v[m];
}

// The 16 x 16 tile of a b owned by this wave (tile row w / 4, tile column w % 4 for wave
// w), for BGJ x BGJ tiles a, b in LDS (row stride BGJ_LD).
// Lane l ends with entries (16 (w / 4) + l / 16 + 4 r, 16 (w % 4) + l % 16), r < 4 (the
// instruction's result layout: entry r of lane l is row l / 16 + 4 r, column l % 16).
__device__ __forceinline__ bgj_v4 bgj_mfma(const double* a, const double* b) {
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    const int i = 16 * (w >> 2) + (l & 15), j = 16 * (w & 3) + (l & 15), kk = l >> 4;
    bgj_v4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < BGJ / 4; ++s)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i * BGJ_LD + 4 * s + kk], b[(4 * s + kk) * BGJ_LD + j], acc, 0, 0, 0);
    return acc;
}

// Row and column of entry r of this lane's product tile.
__device__ __forceinline__ int bgj_out_row(int r) {
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    return 16 * (w >> 2) + (l >> 4) + 4 * r;
}
__device__ __forceinline__ int bgj_out_col() {
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    return 16 * (w & 3) + (l & 15);
}

// Writes sign * (this lane's product entries) to block (I, J) of M.
__device__ __forceinline__ void bgj_store_tile(double* __restrict__ M, int n, int I, int J, bgj_v4 acc, double sign) {
    const int bi = bgj_size(n, I), bj = bgj_size(n, J), j = bgj_out_col();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = bgj_out_row(r);
        if (i < bi && j < bj) M[(size_t)(I * BGJ + i) * n + (size_t)J * BGJ + j] = sign * acc[r];
    }
}

// Value of v in lane `lane` (uniform) of the wavefront.
__device__ __forceinline__ double bgj_lane(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), lane);
    const unsigned hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// 16 x 16 tile product on the FP64 matrix cores: c + sign * (a b), a and b tiles of an LDS
// matrix with row stride BGJ_LD, c and the result in the instruction's result layout (entry r
// of lane l is row l / 16 + 4 r, column l % 16).
__device__ __forceinline__ bgj_v4 bgj_tile_mm(const double* a, const double* b, bgj_v4 c, double sign) {
    const int l = threadIdx.x % 64, i = l & 15, kk = l >> 4;
#pragma unroll
    for (int s = 0; s < 4; ++s)
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(sign * a[i * BGJ_LD + 4 * s + kk], b[(4 * s + kk) * BGJ_LD + i], c, 0,
                                                  0, 0);
    return c;
}

__device__ __forceinline__ bgj_v4 bgj_tile_load(const double* t) {
    const int l = threadIdx.x % 64;
    bgj_v4 v;
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = t[((l >> 4) + 4 * r) * BGJ_LD + (l & 15)];
    return v;
}

__device__ __forceinline__ void bgj_tile_store(double* t, bgj_v4 v) {
    const int l = threadIdx.x % 64;
#pragma unroll
    for (int r = 0; r < 4; ++r) t[((l >> 4) + 4 * r) * BGJ_LD + (l & 15)] = v[r];
}

// In-place inverse of the BGJ x BGJ matrix D in LDS (row stride BGJ_LD) by Gauss-Jordan
// taken 16 pivots at a time, by the BGJ_THREADS = 16 wavefronts of the block.  For the
// 16-block S, wavefront 0 inverts D_SS in registers (lane i % 16 holds row i; the pivot
// row is read from its lane with readlane, so the 16 pivot steps need no barrier); then
// wavefront w updates tile (w / 4, w % 4) of the 4 x 4 tiling on the matrix cores:
//   D_SJ <- X D_SJ,   D_IS <- -D_IS X,   D_IJ <- D_IJ - D_IS (X D_SJ),   D_SS <- X.
// Only the 16-blocks that hold one of the first bk pivots are eliminated (rows and
// columns from bk on must be those of the identity).  A pivot that is not positive and
// finite sets *bad; the elimination runs on (the values are then meaningless).
__device__ void bgj_invert_lds(double* D, int bk, int* bad) {
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    const int TI = w >> 2, TJ = w & 3;
    for (int S = 0; 16 * S < bk; ++S) {
        double* X = D + 16 * S * BGJ_LD + 16 * S;
        if (w == 0) {
            const int i = l & 15;
            double e[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) e[j] = X[i * BGJ_LD + j];
            bool ok = true;
#pragma unroll
            for (int p = 0; p < 16; ++p) {
                const double piv = bgj_lane(e[p], p);
                ok = ok && piv > 0.0 && isfinite(piv);
                const double pinv = 1.0 / piv;
                // row p: e_pj / piv; other rows: e_ij - (e_ip / piv) e_pj
                const double sc = (i == p) ? pinv : 1.0;
                const double cf = (i == p) ? 0.0 : e[p] * pinv;
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    if (j == p) continue;
                    const double rpj = bgj_lane(e[j], p);
                    e[j] = fma(-cf, rpj, e[j] * sc);
                }
                e[p] = (i == p) ? pinv : -cf;
            }
            if (l < 16) {
#pragma unroll
                for (int j = 0; j < 16; ++j) X[i * BGJ_LD + j] = e[j];
            }
            if (!ok && l == 0) *bad = 1;
        }
        __syncthreads();
        const bool own = TI != S || TJ != S;
        bgj_v4 res = {0.0, 0.0, 0.0, 0.0};
        if (TI == S && TJ != S) {
            res = bgj_tile_mm(X, D + 16 * S * BGJ_LD + 16 * TJ, res, 1.0);
        } else if (TJ == S && TI != S) {
            res = bgj_tile_mm(D + 16 * TI * BGJ_LD + 16 * S, X, res, -1.0);
        } else if (own) {
            // T = X D_SJ in the result layout is the B operand of the next product as it
            // stands: entry s of lane j + 16 k is T(4 s + k, j).
            const bgj_v4 t = bgj_tile_mm(X, D + 16 * S * BGJ_LD + 16 * TJ, res, 1.0);
            res = bgj_tile_load(D + 16 * TI * BGJ_LD + 16 * TJ);
            const double* a = D + 16 * TI * BGJ_LD + 16 * S;
            const int i = l & 15, kk = l >> 4;
#pragma unroll
            for (int s = 0; s < 4; ++s) res = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[i * BGJ_LD + 4 * s + kk], t[s], res, 0, 0, 0);
        }
        __syncthreads();
        if (own) bgj_tile_store(D + 16 * TI * BGJ_LD + 16 * TJ, res);
        __syncthreads();
    }
}

// Inverse of the diagonal block K of M (bk x bk, padded with the identity), written
// densely to Xk; false (in every thread) if a pivot was not positive and finite.
__device__ bool bgj_invert_block(const double* __restrict__ M, int n, int K, double* __restrict__ Xk, double* D,
                                 int* bad) {
    const int bk = bgj_size(n, K);
    double v[BGJ_RPT];
    bgj_fetch(M, n, K, K, v);
    const int r = threadIdx.x / BGJ, q = threadIdx.x % BGJ;
#pragma unroll
    for (int m = 0; m < BGJ_RPT; ++m)
        if (r + BGJ_RSTEP * m >= bk) v[m] = (r + BGJ_RSTEP * m == q) ? 1.0 : 0.0;
    bgj_put(D, v);
    if (threadIdx.x == 0) *bad = 0;
    __syncthreads();
    bgj_invert_lds(D, bk, bad);
#pragma unroll
    for (int m = 0; m < BGJ_RPT; ++m) Xk[threadIdx.x + m * BGJ_THREADS] = D[(r + BGJ_RSTEP * m) * BGJ_LD + q];
    return *bad == 0;
}

__global__ __launch_bounds__(BGJ_THREADS) void k_bgj_pivot(int n, int k, double* __restrict__ M,
                                                           double* __restrict__ X, double* __restrict__ scal) {
    __shared__ double sa[BGJ * BGJ_LD];
    __shared__ double sb[BGJ * BGJ_LD];
    __shared__ int bad;
    const int nb = (n + BGJ - 1) / BGJ;
    const int w = blockIdx.x;
    if (w == 0) {
        if (k >= nb) return;
        const bool ok = bgj_invert_block(M, n, k, X + (size_t)(k & 1) * BGJ * BGJ, sa, &bad);
        if (threadIdx.x == 0 && (k == 0 || !ok)) scal[S_COARSE] = ok ? 0.0 : 1.0;
        return;
    }
    if (k == 0) return;
    const int kp = k - 1;  // finish the block step of kp
    double vx[BGJ_RPT], vb[BGJ_RPT];
    bgj_fetch_dense(X + (size_t)(kp & 1) * BGJ * BGJ, vx);
    if (w == 2 * nb - 1) {  // M_{kp kp} <- X
        bgj_store(M, n, kp, kp, vx);
        return;
    }
    const bool row = w < nb;
    const int O = bgj_other(row ? w - 1 : w - nb, kp);
    if (row) {  // M_{kp O} <- X M_{kp O}
        bgj_fetch(M, n, kp, O, vb);
        bgj_put(sa, vx);
        bgj_put(sb, vb);
        __syncthreads();
        bgj_store_tile(M, n, kp, O, bgj_mfma(sa, sb), 1.0);
    } else {  // M_{O kp} <- -M_{O kp} X
        bgj_fetch(M, n, O, kp, vb);
        bgj_put(sa, vb);
        bgj_put(sb, vx);
        __syncthreads();
        bgj_store_tile(M, n, O, kp, bgj_mfma(sa, sb), -1.0);
    }
}

// M_IJ <- M_IJ - M_IK (X M_KJ) for I, J != K = k; one workgroup per block (I, J).  All four
// operands are fetched at once; X M_KJ goes through LDS, M_IJ stays in registers.
__global__ __launch_bounds__(BGJ_THREADS) void k_bgj_update(int n, int k, double* __restrict__ M,
                                                            const double* __restrict__ X) {
    __shared__ double sx[BGJ * BGJ_LD];  // X, then M_IK
    __shared__ double sb[BGJ * BGJ_LD];  // M_KJ
    __shared__ double st[BGJ * BGJ_LD];  // X M_KJ
    const int nb = (n + BGJ - 1) / BGJ;
    const int w = blockIdx.x;
    const int I = bgj_other(w / (nb - 1), k), J = bgj_other(w % (nb - 1), k);
    const int bi = bgj_size(n, I), bj = bgj_size(n, J), j = bgj_out_col();
    double vx[BGJ_RPT], vk[BGJ_RPT], vi[BGJ_RPT], cur[4];
    bgj_fetch_dense(X + (size_t)(k & 1) * BGJ * BGJ, vx);
    bgj_fetch(M, n, k, J, vk);
    bgj_fetch(M, n, I, k, vi);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = bgj_out_row(r);
        cur[r] = (i < bi && j < bj) ? M[(size_t)(I * BGJ + i) * n + (size_t)J * BGJ + j] : 0.0;
    }
    bgj_put(sx, vx);
    bgj_put(sb, vk);
    __syncthreads();
    const bgj_v4 t = bgj_mfma(sx, sb);  // T = X M_KJ
#pragma unroll
    for (int r = 0; r < 4; ++r) st[bgj_out_row(r) * BGJ_LD + j] = t[r];
    __syncthreads();
    bgj_put(sx, vi);
    __syncthreads();
    const bgj_v4 acc = bgj_mfma(sx, st);  // M_IK T
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = bgj_out_row(r);
        if (i < bi && j < bj) M[(size_t)(I * BGJ + i) * n + (size_t)J * BGJ + j] = cur[r] - acc[r];
    }
}

void launch_dense_inverse(int n, double* D, double* scal, double* work, hipStream_t s) {
    if (n > COARSE_GLOBAL_MAX) throw Fail{AMG_ERR_ARG, "coarsest level too large for the dense inverse"};
    if (n <= COARSE_LDS_MAX) {
        k_dense_inverse<<<1, 1024, 0, s>>>(n, D, scal);
        HIP_LAUNCH_CHECK();
        return;
    }
    if (work == nullptr) throw Fail{AMG_ERR_ARG, "blocked coarse inverse without its scratch"};
    const int nb = (n + BGJ - 1) / BGJ;
    for (int k = 0; k <= nb; ++k) {
        k_bgj_pivot<<<k == 0 ? 1 : 2 * nb, BGJ_THREADS, 0, s>>>(n, k, D, work, scal);
        HIP_LAUNCH_CHECK();
        if (k < nb && nb > 1) {
            k_bgj_update<<<(nb - 1) * (nb - 1), BGJ_THREADS, 0, s>>>(n, k, D, work);
            HIP_LAUNCH_CHECK();
        }
    }
}

}  // namespace amgmi
