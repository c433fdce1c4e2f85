// kernels_galerkin.hip -- numeric phase of the Galerkin product A_{l+1} = R_l (A_l P_l)
// on patterns cached at setup, and the smoother diagonal (Algorithm 4, Section 3; the
// reuse of the product's sparsity pattern is the extension proposed in Section 5).
//
// Determinism: no atomics.  Each output entry is owned by one lane, which adds its
// product terms in the order a row-by-row (Gustavson) product visits them: increasing k
// along row i of the left factor, at most one matching entry per row of the right factor.
// Products and sums are rounded separately (contraction off), so FP64 results are
// bitwise reproducible and independent of the launch shape.
#include <type_traits>
#include <vector>

#include "amg_internal.h"

#pragma clang fp contract(off)

namespace amgmi {

constexpr int TPB = 256;

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

// Smoother diagonal of one level: damped Jacobi m_i = omega / a_ii, or SPAI0
// m_i = a_ii / sum_j a_ij^2 with the sum taken along the row in column order.
template <typename T>
__global__ __launch_bounds__(TPB) void k_smoother_diag(int n, const int* __restrict__ ptr,
                                                       const int* __restrict__ col, const T* __restrict__ val,
                                                       int kind, T omega, T* __restrict__ m) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n) return;
    T d = 0, s = 0;
    for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
        const T a = val[k];
        if (col[k] == i) d = a;
        s = s + a * a;
    }
    m[i] = (kind == 1) ? d / s : omega / d;
}

// AP = A P into the cached pattern of AP.  A group of G lanes per row of A; each lane
// owns entries J of the AP row and scans the P rows of the row's columns for J.
template <int G, typename T>
__global__ __launch_bounds__(TPB) void k_galerkin_ap(int n, const int* __restrict__ Aptr,
                                                     const int* __restrict__ Acol, const T* __restrict__ Aval,
                                                     const int* __restrict__ Pptr, const int* __restrict__ Pcol,
                                                     const T* __restrict__ Pval, const int* __restrict__ APptr,
                                                     const int* __restrict__ APcol, T* __restrict__ APval) {
    const int lane = threadIdx.x & (G - 1);
    const int row = (xcd_block() * TPB + (int)threadIdx.x) / G;
    if (row >= n) return;
    const int ab = Aptr[row], ae = Aptr[row + 1];
    const int se = APptr[row + 1];
    for (int s = APptr[row] + lane; s < se; s += G) {
        const int J = APcol[s];
        T acc = 0;
        for (int k = ab; k < ae; ++k) {
            const int j = Acol[k];
            const int pe = Pptr[j + 1];
            for (int q = Pptr[j]; q < pe; ++q) {
                const int c = Pcol[q];
                if (c >= J) {
                    if (c == J) acc = acc + Aval[k] * Pval[q];
                    break;
                }
            }
        }
        APval[s] = acc;
    }
}

// Position of column J in the sorted, non-empty row cols[b, e), or -1.
__device__ __forceinline__ int find_sorted(const int* __restrict__ cols, int b, int e, int J) {
    int lo = b, hi = e - 1;  // the lower bound of J lies in [lo, hi]
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cols[mid] < J)
            lo = mid + 1;
        else
            hi = mid;
    }
    return cols[lo] == J ? lo : -1;
}

// A_c = R (AP) into the cached pattern of A_c.  A group of G lanes per coarse row; each
// lane owns entries J of the row and walks the R row, finding J in each AP row.
template <int G, typename T>
__global__ __launch_bounds__(TPB) void k_galerkin_rap(int nc, const int* __restrict__ Rptr,
                                                      const int* __restrict__ Rcol, const T* __restrict__ Rval,
                                                      const int* __restrict__ APptr, const int* __restrict__ APcol,
                                                      const T* __restrict__ APval, const int* __restrict__ Cptr,
                                                      const int* __restrict__ Ccol, T* __restrict__ Cval) {
    const int lane = threadIdx.x & (G - 1);
    const int row = (xcd_block() * TPB + (int)threadIdx.x) / G;
    if (row >= nc) return;
    const int rb = Rptr[row], re = Rptr[row + 1];
    const int se = Cptr[row + 1];
    for (int s = Cptr[row] + lane; s < se; s += G) {
        const int J = Ccol[s];
        T acc = 0;
        for (int q = rb; q < re; ++q) {
            const int i = Rcol[q];
            const int b = APptr[i], e = APptr[i + 1];
            if (b == e) continue;
            const int pos = find_sorted(APcol, b, e, J);
            if (pos >= 0) acc = acc + Rval[q] * APval[pos];
        }
        Cval[s] = acc;
    }
}

// ------------------------------------------------------------------ LDS-staged forms
//
// A workgroup owns `rpb` consecutive rows of the left factor (rows chosen at setup so the
// staged data fits the caps below).  It stages the left factor's entries of those rows
// and, for each entry, the whole row of the right factor it references, in LDS; lanes
// then own output entries and add their terms from LDS in the fixed order above.

constexpr int GL_CAP_L = 512;   // staged entries of the left factor per block
constexpr int GL_CAP_C = 2048;  // staged entries of the referenced right-factor rows

// Exclusive prefix sum of v[0..count) in place, v[count] = total (count <= GL_CAP_L).
__device__ void block_exscan(int* v, int count, int* tmp) {
    constexpr int PER = (GL_CAP_L + TPB - 1) / TPB;
    const int t = threadIdx.x;
    const int b = t * PER;
    int loc = 0;
    for (int q = 0; q < PER; ++q)
        if (b + q < count) loc += v[b + q];
    tmp[t] = loc;
    __syncthreads();
    for (int off = 1; off < TPB; off <<= 1) {  // inclusive scan of the per-thread sums
        const int x = t >= off ? tmp[t - off] : 0;
        __syncthreads();
        tmp[t] += x;
        __syncthreads();
    }
    int run = t > 0 ? tmp[t - 1] : 0;
    for (int q = 0; q < PER; ++q)
        if (b + q < count) {
            const int x = v[b + q];
            v[b + q] = run;
            run += x;
        }
    if (t == TPB - 1) v[count] = tmp[TPB - 1];
    __syncthreads();
}

// Local row of a position given the staged row pointers (sorted, rows [0, nr)).
__device__ __forceinline__ int local_row(const int* sptr, int nr, int pos) {
    int lo = 0, hi = nr - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sptr[mid] <= pos)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Stages rows [row0, row1) of the left factor L and, for every entry (i, j), row j of the
// right factor B.  Returns through shared arrays: lptr (row pointers, rebased), lval (L
// values), lcol (L columns), boff (offset of each entry's B row in bcol/bval).
// With `lin` given, the left factor's values are read from the caller's FP64 array
// instead of Lval and copied to lout64 / loutT (either may be null) on the way: this is
// how new matrix values enter the hierarchy without a separate copy pass.
template <typename T>
__device__ void stage_pair(int row0, int row1, const int* __restrict__ Lptr, const int* __restrict__ Lcol,
                           const T* __restrict__ Lval, const int* __restrict__ Bptr, const int* __restrict__ Bcol,
                           const T* __restrict__ Bval, int* lptr, int* lcol, T* lval, int* boff, int* bst, int* bcol,
                           T* bval, int* tmp, const double* __restrict__ lin = nullptr,
                           double* __restrict__ lout64 = nullptr, T* __restrict__ loutT = nullptr) {
    const int nr = row1 - row0;
    for (int i = threadIdx.x; i <= nr; i += TPB) lptr[i] = Lptr[row0 + i];
    __syncthreads();
    const int k0 = lptr[0];
    const int nl = min(lptr[nr] - k0, GL_CAP_L);  // the host sizes blocks within the caps
    for (int t = threadIdx.x; t < nl; t += TPB) {
        const int j = Lcol[k0 + t];
        lcol[t] = j;
        if (lin != nullptr) {
            const double a = lin[k0 + t];
            if (lout64 != nullptr) lout64[k0 + t] = a;
            if (loutT != nullptr) loutT[k0 + t] = (T)a;
            lval[t] = (T)a;
        } else {
            lval[t] = Lval[k0 + t];
        }
        const int b = Bptr[j];
        bst[t] = b;
        boff[t] = Bptr[j + 1] - b;
    }
    __syncthreads();
    block_exscan(boff, nl, tmp);
    for (int t = threadIdx.x; t < nl; t += TPB) {
        const int o = boff[t], b = bst[t];
        const int len = min(boff[t + 1], GL_CAP_C) - o;
        for (int q = 0; q < len; ++q) {
            bcol[o + q] = Bcol[b + q];
            bval[o + q] = Bval[b + q];
        }
    }
    __syncthreads();
}

// AP = A P for rows [row0, row1) plus the smoother diagonal of those rows of A.
template <typename T>
__global__ __launch_bounds__(TPB) void k_galerkin_ap_lds(int n, int rpb, const int* __restrict__ Aptr,
                                                         const int* __restrict__ Acol, const T* __restrict__ Aval,
                                                         const int* __restrict__ Pptr, const int* __restrict__ Pcol,
                                                         const T* __restrict__ Pval, const int* __restrict__ APptr,
                                                         const int* __restrict__ APcol, T* __restrict__ APval,
                                                         int kind, T omega, T* __restrict__ m,
                                                         const double* __restrict__ Ain, double* __restrict__ Aout64,
                                                         T* __restrict__ AoutT) {
    __shared__ int lptr[TPB + 1];
    __shared__ int sptr[TPB + 1];
    __shared__ int lcol[GL_CAP_L];
    __shared__ T lval[GL_CAP_L];
    __shared__ int boff[GL_CAP_L + 1];
    __shared__ int bst[GL_CAP_L];
    __shared__ int bcol[GL_CAP_C];
    __shared__ T bval[GL_CAP_C];
    __shared__ int tmp[TPB];
    const int row0 = xcd_block() * rpb;
    if (row0 >= n) return;
    const int row1 = min(row0 + rpb, n), nr = row1 - row0;
    stage_pair<T>(row0, row1, Aptr, Acol, Aval, Pptr, Pcol, Pval, lptr, lcol, lval, boff, bst, bcol, bval, tmp, Ain,
                  Aout64, AoutT);
    for (int i = threadIdx.x; i <= nr; i += TPB) sptr[i] = APptr[row0 + i];
    __syncthreads();
    const int k0 = lptr[0];
    const int s0 = sptr[0], s1 = sptr[nr];
    for (int s = s0 + (int)threadIdx.x; s < s1; s += TPB) {
        const int r = local_row(sptr, nr, s);
        const int J = APcol[s];
        T acc = 0;
        for (int t = lptr[r] - k0; t < lptr[r + 1] - k0; ++t) {
            for (int q = boff[t]; q < boff[t + 1]; ++q) {
                const int c = bcol[q];
                if (c >= J) {
                    if (c == J) acc = acc + lval[t] * bval[q];
                    break;
                }
            }
        }
        APval[s] = acc;
    }
    if (m != nullptr && (int)threadIdx.x < nr) {
        const int r = threadIdx.x, i = row0 + r;
        T d = 0, ss = 0;
        for (int t = lptr[r] - k0; t < lptr[r + 1] - k0; ++t) {
            const T a = lval[t];
            if (lcol[t] == i) d = a;
            ss = ss + a * a;
        }
        m[i] = (kind == 1) ? d / ss : omega / d;
    }
}

// A_c = R (AP) for coarse rows [row0, row1).
template <typename T>
__global__ __launch_bounds__(TPB) void k_galerkin_rap_lds(int nc, int rpb, const int* __restrict__ Rptr,
                                                          const int* __restrict__ Rcol, const T* __restrict__ Rval,
                                                          const int* __restrict__ APptr,
                                                          const int* __restrict__ APcol,
                                                          const T* __restrict__ APval, const int* __restrict__ Cptr,
                                                          const int* __restrict__ Ccol, T* __restrict__ Cval) {
    __shared__ int lptr[TPB + 1];
    __shared__ int sptr[TPB + 1];
    __shared__ int lcol[GL_CAP_L];
    __shared__ T lval[GL_CAP_L];
    __shared__ int boff[GL_CAP_L + 1];
    __shared__ int bst[GL_CAP_L];
    __shared__ int bcol[GL_CAP_C];
    __shared__ T bval[GL_CAP_C];
    __shared__ int tmp[TPB];
    const int row0 = xcd_block() * rpb;
    if (row0 >= nc) return;
    const int row1 = min(row0 + rpb, nc), nr = row1 - row0;
    stage_pair<T>(row0, row1, Rptr, Rcol, Rval, APptr, APcol, APval, lptr, lcol, lval, boff, bst, bcol, bval, tmp);
    for (int i = threadIdx.x; i <= nr; i += TPB) sptr[i] = Cptr[row0 + i];
    __syncthreads();
    const int k0 = lptr[0];
    const int s0 = sptr[0], s1 = sptr[nr];
    for (int s = s0 + (int)threadIdx.x; s < s1; s += TPB) {
        const int r = local_row(sptr, nr, s);
        const int J = Ccol[s];
        T acc = 0;
        for (int t = lptr[r] - k0; t < lptr[r + 1] - k0; ++t) {
            const int b = boff[t], e = boff[t + 1];
            if (b == e) continue;
            const int pos = find_sorted(bcol, b, e, J);
            if (pos >= 0) acc = acc + lval[t] * bval[pos];
        }
        Cval[s] = acc;
    }
}

template <typename T>
void launch_smoother_diag(const Csr& A, int kind, double omega, T* m, hipStream_t s) {
    k_smoother_diag<T><<<row_blocks(A.nrows, 1), TPB, 0, s>>>(A.nrows, A.ptr, A.col, A.v<T>(), kind, (T)omega, m);
    HIP_LAUNCH_CHECK();
}

// AP = A P; with m != nullptr also the smoother diagonal of A, and with ain != nullptr
// the values of A are taken from ain (FP64) and stored into A's value arrays on the way.
// Only the staged form fuses these; it returns true when it did (m and A written).
template <typename T>
bool launch_galerkin_ap(const Csr& A, const Csr& P, const Csr& AP, int g, int rpb, int kind, double omega, T* m,
                        const double* ain, hipStream_t s) {
    if (rpb > 0) {
        double* out64 = (ain != nullptr && ain != A.val) ? A.val : nullptr;
        T* outT = nullptr;
        if constexpr (!std::is_same<T, double>::value) outT = ain != nullptr ? A.v<T>() : nullptr;
        k_galerkin_ap_lds<T><<<(unsigned)((A.nrows + rpb - 1) / rpb), TPB, 0, s>>>(
            A.nrows, rpb, A.ptr, A.col, A.v<T>(), P.ptr, P.col, P.v<T>(), AP.ptr, AP.col, AP.v<T>(), kind, (T)omega, m,
            ain, out64, outT);
        HIP_LAUNCH_CHECK();
        return true;
    }
    if (ain != nullptr) return false;  // the caller ingests the values first, then calls again
    AMG_WITH_G(g, k_galerkin_ap<G, T><<<row_blocks(A.nrows, G), TPB, 0, s>>>(
                      A.nrows, A.ptr, A.col, A.v<T>(), P.ptr, P.col, P.v<T>(), AP.ptr, AP.col, AP.v<T>()));
    HIP_LAUNCH_CHECK();
    return false;
}

template <typename T>
void launch_galerkin_rap(const Csr& R, const Csr& AP, const Csr& Ac, int g, int rpb, hipStream_t s) {
    if (rpb > 0) {
        k_galerkin_rap_lds<T><<<(unsigned)((R.nrows + rpb - 1) / rpb), TPB, 0, s>>>(
            R.nrows, rpb, R.ptr, R.col, R.v<T>(), AP.ptr, AP.col, AP.v<T>(), Ac.ptr, Ac.col, Ac.v<T>());
        HIP_LAUNCH_CHECK();
        return;
    }
    AMG_WITH_G(g, k_galerkin_rap<G, T><<<row_blocks(R.nrows, G), TPB, 0, s>>>(
                      R.nrows, R.ptr, R.col, R.v<T>(), AP.ptr, AP.col, AP.v<T>(), Ac.ptr, Ac.col, Ac.v<T>()));
    HIP_LAUNCH_CHECK();
}

// Rows per staged block for the product L B (0: the caps cannot be met, use lane groups):
// the largest power of two <= TPB such that every block stages at most GL_CAP_L entries of
// L and GL_CAP_C entries of the referenced B rows.  Host arrays.
int pick_galerkin_rpb(const int32_t* Lptr, const int32_t* Lcol, int32_t nrows, const int32_t* Bptr) {
    std::vector<int64_t> work((size_t)nrows + 1, 0);
    for (int32_t i = 0; i < nrows; ++i) {
        int64_t w = 0;
        for (int32_t k = Lptr[i]; k < Lptr[i + 1]; ++k) w += Bptr[Lcol[k] + 1] - Bptr[Lcol[k]];
        work[(size_t)i + 1] = work[i] + w;
    }
    for (int rpb = TPB; rpb >= 1; rpb >>= 1) {
        bool ok = true;
        for (int64_t r0 = 0; r0 < nrows && ok; r0 += rpb) {
            const int64_t r1 = r0 + rpb < nrows ? r0 + rpb : nrows;
            if ((int64_t)Lptr[r1] - Lptr[r0] > GL_CAP_L || work[r1] - work[r0] > GL_CAP_C) ok = false;
        }
        if (ok) return rpb;
    }
    return 0;
}

template void launch_smoother_diag<double>(const Csr&, int, double, double*, hipStream_t);
template void launch_smoother_diag<float>(const Csr&, int, double, float*, hipStream_t);
template bool launch_galerkin_ap<double>(const Csr&, const Csr&, const Csr&, int, int, int, double, double*,
                                         const double*, hipStream_t);
template bool launch_galerkin_ap<float>(const Csr&, const Csr&, const Csr&, int, int, int, double, float*,
                                        const double*, hipStream_t);
template void launch_galerkin_rap<double>(const Csr&, const Csr&, const Csr&, int, int, hipStream_t);
template void launch_galerkin_rap<float>(const Csr&, const Csr&, const Csr&, int, int, hipStream_t);

}  // namespace amgmi
