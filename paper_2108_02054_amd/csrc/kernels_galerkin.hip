// kernels_galerkin.hip -- numeric phase of the Galerkin product A_{l+1} = R_l (A_l P_l)
// on patterns cached at setup, and the smoother diagonal (Algorithm 4, Section 3; the
// reuse of the product's sparsity pattern is the extension proposed in Section 5).
//
// Determinism: no atomics.  Each output entry is owned by one lane, which adds its
// product terms in the order a row-by-row (Gustavson) product visits them: increasing k
// along row i of the left factor, at most one matching entry per row of the right factor.
// Products and sums are rounded separately (contraction off), so FP64 results are
// bitwise reproducible and independent of the launch shape.
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

template <typename T>
void launch_smoother_diag(const Csr& A, int kind, double omega, T* m, hipStream_t s) {
    k_smoother_diag<T><<<row_blocks(A.nrows, 1), TPB, 0, s>>>(A.nrows, A.ptr, A.col, A.v<T>(), kind, (T)omega, m);
    HIP_LAUNCH_CHECK();
}

template <typename T>
void launch_galerkin_ap(const Csr& A, const Csr& P, const Csr& AP, int g, hipStream_t s) {
    AMG_WITH_G(g, k_galerkin_ap<G, T><<<row_blocks(A.nrows, G), TPB, 0, s>>>(
                      A.nrows, A.ptr, A.col, A.v<T>(), P.ptr, P.col, P.v<T>(), AP.ptr, AP.col, AP.v<T>()));
    HIP_LAUNCH_CHECK();
}

template <typename T>
void launch_galerkin_rap(const Csr& R, const Csr& AP, const Csr& Ac, int g, hipStream_t s) {
    AMG_WITH_G(g, k_galerkin_rap<G, T><<<row_blocks(R.nrows, G), TPB, 0, s>>>(
                      R.nrows, R.ptr, R.col, R.v<T>(), AP.ptr, AP.col, AP.v<T>(), Ac.ptr, Ac.col, Ac.v<T>()));
    HIP_LAUNCH_CHECK();
}

template void launch_smoother_diag<double>(const Csr&, int, double, double*, hipStream_t);
template void launch_smoother_diag<float>(const Csr&, int, double, float*, hipStream_t);
template void launch_galerkin_ap<double>(const Csr&, const Csr&, const Csr&, int, hipStream_t);
template void launch_galerkin_ap<float>(const Csr&, const Csr&, const Csr&, int, hipStream_t);
template void launch_galerkin_rap<double>(const Csr&, const Csr&, const Csr&, int, hipStream_t);
template void launch_galerkin_rap<float>(const Csr&, const Csr&, const Csr&, int, hipStream_t);

}  // namespace amgmi
