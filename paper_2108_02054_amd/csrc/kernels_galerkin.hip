// kernels_galerkin.hip -- numeric phase of the Galerkin product A_{l+1} = R_l (A_l P_l)
// on patterns cached at setup, and the smoother diagonal (Algorithm 4, Section 3; the
// reuse of the product's sparsity pattern is the extension proposed in Section 5).
//
// Determinism: no atomics.  Each output entry is owned by one lane, which adds its
// product terms in the order a row-by-row (Gustavson) product visits them: increasing k
// along row i of the left factor, at most one matching entry per row of the right factor.
// Products and sums are rounded separately (contraction off), so FP64 results are
// bitwise reproducible and independent of the launch shape.
#include <algorithm>
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

// ------------------------------------------------------------------ position-map form
//
// The terms of row i of C = L B are l_t * b_e for the L entries t of row i in order and,
// for each, the entries e of B row Lcol[t] in order; this is the order in which a
// row-by-row product adds them.  The column of each term and so its position in the
// (cached, sorted) C row depend on the patterns alone: setup stores these positions once
// (the position map), and each numeric product only multiplies, and adds each term into
// its C entry, kept in LDS.  A group of G lanes per row of C walks the L entries in order;
// for entry t the lanes take the terms of B row Lcol[t], G at a time.  Positions within one
// B row are distinct, and the LDS operations of a wavefront complete in program order, so
// every entry of C receives its terms in the row-by-row order.  Each lane holds two L
// entries of a chunk (2G entries per chunk), and the terms of WF_AHEAD entries are loaded
// before they are added.  For C = A P the group also forms the smoother diagonal (the
// row's squares added in column order), and can take A's values from a new FP64 array,
// storing the hierarchy's copies on the way.

constexpr int WF_AHEAD = 4;            // L entries whose terms are loaded together
constexpr int WF_CAP_MAX = 4096;       // longest C row the form takes
constexpr size_t WF_SMEM_MAX = 65536;  // LDS per block

template <int G>
__device__ __forceinline__ int group_exscan(int v, int g, int& total) {
    int x = v;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        const int y = __shfl_up(x, o, G);
        if (g >= o) x += y;
    }
    total = __shfl(x, G - 1, G);
    return x - v;
}

template <typename T, int G, typename PT>
__global__ __launch_bounds__(TPB) void k_galerkin_pos(
    int nrows, int cap, const int* __restrict__ Lptr, const int* __restrict__ Lcol, const T* __restrict__ Lval,
    const int* __restrict__ Bptr, const T* __restrict__ Bval, const int* __restrict__ Cptr, T* __restrict__ Cval,
    const PT* __restrict__ pos, const int64_t* __restrict__ poff, int kind, T omega, T* __restrict__ m,
    const double* __restrict__ lin, double* __restrict__ lout64, T* __restrict__ loutT) {
    extern __shared__ __align__(16) unsigned char wf_smem[];
    const int g = threadIdx.x & (G - 1);
    T* sacc = reinterpret_cast<T*>(wf_smem) + (size_t)(threadIdx.x / G) * cap;
    const int row = (xcd_block() * TPB + (int)threadIdx.x) / G;
    if (row >= nrows) return;  // groups leave whole: G divides the wavefront
    const int sb = Cptr[row];
    const int len = min(Cptr[row + 1] - sb, cap);  // the host keeps every row within cap
    for (int q = g; q < len; q += G) sacc[q] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    T d = 0, ss = 0;
    const int le = Lptr[row + 1];
    const PT* prow = pos + poff[row];
    int carry = 0;  // terms of the row's earlier chunks
    for (int c0 = Lptr[row]; c0 < le; c0 += 2 * G) {
        // lane g holds L entries c0 + g (h = 0) and c0 + G + g (h = 1)
        int bst[2], blen[2], jj[2], toff[2];
        T lv[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int t = c0 + h * G + g;
            bst[h] = 0;
            blen[h] = 0;
            jj[h] = -1;
            lv[h] = 0;
            if (t < le) {
                const int j = Lcol[t];
                jj[h] = j;
                if (lin != nullptr) {
                    const double x = lin[t];
                    if (lout64 != nullptr) lout64[t] = x;
                    if (loutT != nullptr) loutT[t] = (T)x;
                    lv[h] = (T)x;
                } else {
                    lv[h] = Lval[t];
                }
                bst[h] = Bptr[j];
                blen[h] = Bptr[j + 1] - bst[h];
            }
        }
        int tot0, tot1;
        toff[0] = carry + group_exscan<G>(blen[0], g, tot0);
        toff[1] = carry + tot0 + group_exscan<G>(blen[1], g, tot1);
        carry += tot0 + tot1;
        const int nt = min(2 * G, le - c0);  // uniform across the group
        if (m != nullptr) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
                for (int q = 0; q < G && h * G + q < nt; ++q) {  // the row's squares in column order
                    const T a = __shfl(lv[h], q, G);
                    if (__shfl(jj[h], q, G) == row) d = a;
                    ss = ss + a * a;
                }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            for (int u0 = 0; u0 < G && h * G + u0 < nt; u0 += WF_AHEAD) {
                int ub[WF_AHEAD], ul[WF_AHEAD], uo[WF_AHEAD], up[WF_AHEAD];
                T uv[WF_AHEAD], bv[WF_AHEAD];
#pragma unroll
                for (int i = 0; i < WF_AHEAD; ++i) {  // first G terms of each entry, in flight together
                    const int u = u0 + i < G ? u0 + i : G - 1;
                    ub[i] = __shfl(bst[h], u, G);
                    ul[i] = (u0 + i < G && h * G + u0 + i < nt) ? __shfl(blen[h], u, G) : 0;
                    uo[i] = __shfl(toff[h], u, G);
                    uv[i] = __shfl(lv[h], u, G);
                    if (g < ul[i]) {
                        up[i] = (int)prow[uo[i] + g];
                        bv[i] = Bval[ub[i] + g];
                    }
                }
#pragma unroll
                for (int i = 0; i < WF_AHEAD; ++i) {
                    if (g < ul[i] && up[i] < len) sacc[up[i]] = sacc[up[i]] + uv[i] * bv[i];
                    for (int k = g + G; k < ul[i]; k += G) {  // rows of B longer than G
                        const int p = (int)prow[uo[i] + k];
                        const T b = Bval[ub[i] + k];
                        if (p < len) sacc[p] = sacc[p] + uv[i] * b;
                    }
                }
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int q = g; q < len; q += G) Cval[sb + q] = sacc[q];
    if (m != nullptr && g == 0) m[row] = (kind == 1) ? d / ss : omega / d;
}

// Terms per row of C = L B.
__global__ __launch_bounds__(TPB) void k_count_terms(int nrows, const int* __restrict__ Lptr,
                                                     const int* __restrict__ Lcol, const int* __restrict__ Bptr,
                                                     int64_t* __restrict__ cnt) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i > nrows) return;
    int64_t c = 0;
    if (i < nrows)
        for (int t = Lptr[i]; t < Lptr[i + 1]; ++t) c += Bptr[Lcol[t] + 1] - Bptr[Lcol[t]];
    cnt[i] = c;  // cnt[nrows] = 0, so the exclusive scan ends with the total
}

// The position map: 8 lanes per row of C, the L entries in order, the B row's terms
// across the lanes; each column is found in the sorted C row by binary search.  A column
// missing from the C row (which a consistent cached pattern never has) maps to the row
// length, which the numeric kernel skips.
template <typename PT>
__global__ __launch_bounds__(TPB) void k_posmap(int nrows, const int* __restrict__ Lptr,
                                                const int* __restrict__ Lcol, const int* __restrict__ Bptr,
                                                const int* __restrict__ Bcol, const int* __restrict__ Cptr,
                                                const int* __restrict__ Ccol, const int64_t* __restrict__ poff,
                                                PT* __restrict__ pos) {
    constexpr int G = 8;
    const int g = threadIdx.x & (G - 1);
    const int row = (xcd_block() * TPB + (int)threadIdx.x) / G;
    if (row >= nrows) return;
    const int cb = Cptr[row], ce = Cptr[row + 1];
    int64_t o = poff[row];
    for (int t = Lptr[row]; t < Lptr[row + 1]; ++t) {
        const int j = Lcol[t];
        const int b0 = Bptr[j], b1 = Bptr[j + 1];
        for (int e = b0 + g; e < b1; e += G) {
            const int J = Bcol[e];
            int lo = cb, hi = ce;  // lower bound of J in Ccol[cb, ce)
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (Ccol[mid] < J)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            const int p = (lo < ce && Ccol[lo] == J) ? lo - cb : ce - cb;
            pos[o + (e - b0)] = (PT)p;
        }
        o += b1 - b0;
    }
}

int64_t count_galerkin_terms(const Csr& L, const Csr& B, int64_t* off, hipStream_t s) {
    int64_t* cnt = dnew<int64_t>((size_t)L.nrows + 1, s);
    k_count_terms<<<row_blocks((int64_t)L.nrows + 1, 1), TPB, 0, s>>>(L.nrows, L.ptr, L.col, B.ptr, cnt);
    HIP_LAUNCH_CHECK();
    exclusive_scan_i64(cnt, off, (int64_t)L.nrows + 1, s);
    dfree(cnt, s);
    int64_t total = 0;
    HIP_CHECK(hipMemcpyAsync(&total, off + L.nrows, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    return total;
}

void build_galerkin_posmap(const Csr& L, const Csr& B, const Csr& C, const GalShape& gs, hipStream_t s) {
    if (gs.terms == 0) return;
    if (gs.wide)
        k_posmap<uint16_t><<<row_blocks(L.nrows, 8), TPB, 0, s>>>(L.nrows, L.ptr, L.col, B.ptr, B.col, C.ptr, C.col,
                                                                   gs.off, (uint16_t*)gs.pos);
    else
        k_posmap<uint8_t><<<row_blocks(L.nrows, 8), TPB, 0, s>>>(L.nrows, L.ptr, L.col, B.ptr, B.col, C.ptr, C.col,
                                                                  gs.off, (uint8_t*)gs.pos);
    HIP_LAUNCH_CHECK();
}

#define AMG_WITH_GS1(g, ...)                                                \
    do {                                                                    \
        switch (g) {                                                        \
            case 4: { constexpr int GG = 4; __VA_ARGS__; } break;           \
            case 8: { constexpr int GG = 8; __VA_ARGS__; } break;           \
            case 16: { constexpr int GG = 16; __VA_ARGS__; } break;         \
            case 32: { constexpr int GG = 32; __VA_ARGS__; } break;         \
            case 64: { constexpr int GG = 64; __VA_ARGS__; } break;         \
            default: throw Fail{AMG_ERR_ARG, "unsupported Galerkin lane count"}; \
        }                                                                   \
    } while (0)

// Launch shape of the position-map form for C = L B (host arrays): cap = the longest C
// row rounded up to a multiple of 8, and G = the power of two in [4, 64] nearest above the
// mean referenced B row length (so that most B rows take one pass of the group), raised
// until a block's LDS (TPB / G rows of cap FP64 accumulators) is within WF_SMEM_MAX.
// {0, ...}: the rows are too long for the form (lane-group kernels).  gforce forces G
// where the LDS allows.  The position map itself is built by the caller.
GalShape pick_galerkin_shape(const int32_t* Lptr, const int32_t* Lcol, int32_t nrows, const int32_t* Bptr,
                             const int32_t* Cptr, int gforce) {
    int maxlen = 0;
    for (int32_t i = 0; i < nrows; ++i) maxlen = std::max(maxlen, Cptr[i + 1] - Cptr[i]);
    if (maxlen > WF_CAP_MAX) return {};
    double refs = 0.0, tot = 0.0;
    for (int64_t k = 0; k < Lptr[nrows]; ++k) {
        refs += 1.0;
        tot += (double)(Bptr[Lcol[k] + 1] - Bptr[Lcol[k]]);
    }
    const double mean_b = refs > 0 ? tot / refs : 1.0;
    const int cap = std::max(8, (maxlen + 7) / 8 * 8);
    auto smem = [&](int G) { return (size_t)(TPB / G) * (size_t)cap * sizeof(double); };
    int G = 4;
    while (G < 64 && G < mean_b) G <<= 1;
    if (gforce == 4 || gforce == 8 || gforce == 16 || gforce == 32 || gforce == 64) G = gforce;
    while (G < 64 && smem(G) > WF_SMEM_MAX) G <<= 1;
    if (smem(G) > WF_SMEM_MAX) return {};
    GalShape gs;
    gs.g = G;
    gs.cap = cap;
    gs.wide = maxlen > 255 ? 1 : 0;
    return gs;
}

static size_t acc_smem(const GalShape& gs, size_t tsize) { return (size_t)(TPB / gs.g) * (size_t)gs.cap * tsize; }

template <typename T>
void launch_smoother_diag(const Csr& A, int kind, double omega, T* m, hipStream_t s) {
    k_smoother_diag<T><<<row_blocks(A.nrows, 1), TPB, 0, s>>>(A.nrows, A.ptr, A.col, A.v<T>(), kind, (T)omega, m);
    HIP_LAUNCH_CHECK();
}

// AP = A P; with m != nullptr also the smoother diagonal of A, and with ain != nullptr
// the values of A are taken from ain (FP64) and stored into A's value arrays on the way.
// Only the position-map form fuses these; it returns true when it did (m and A written).
template <typename T>
bool launch_galerkin_ap(const Csr& A, const Csr& P, const Csr& AP, int g, GalShape gs, int kind, double omega, T* m,
                        const double* ain, hipStream_t s) {
    if (gs.g > 0) {
        double* out64 = (ain != nullptr && ain != A.val) ? A.val : nullptr;
        T* outT = nullptr;
        if constexpr (!std::is_same<T, double>::value) outT = ain != nullptr ? A.v<T>() : nullptr;
        const size_t sm = acc_smem(gs, sizeof(T));
        if (gs.wide)
            AMG_WITH_GS1(gs.g, (k_galerkin_pos<T, GG, uint16_t><<<row_blocks(A.nrows, GG), TPB, sm, s>>>(
                                   A.nrows, gs.cap, A.ptr, A.col, A.v<T>(), P.ptr, P.v<T>(), AP.ptr, AP.v<T>(),
                                   (const uint16_t*)gs.pos, gs.off, kind, (T)omega, m, ain, out64, outT)));
        else
            AMG_WITH_GS1(gs.g, (k_galerkin_pos<T, GG, uint8_t><<<row_blocks(A.nrows, GG), TPB, sm, s>>>(
                                   A.nrows, gs.cap, A.ptr, A.col, A.v<T>(), P.ptr, P.v<T>(), AP.ptr, AP.v<T>(),
                                   (const uint8_t*)gs.pos, gs.off, kind, (T)omega, m, ain, out64, outT)));
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
void launch_galerkin_rap(const Csr& R, const Csr& AP, const Csr& Ac, int g, GalShape gs, hipStream_t s) {
    if (gs.g > 0) {
        const size_t sm = acc_smem(gs, sizeof(T));
        if (gs.wide)
            AMG_WITH_GS1(gs.g, (k_galerkin_pos<T, GG, uint16_t><<<row_blocks(R.nrows, GG), TPB, sm, s>>>(
                                   R.nrows, gs.cap, R.ptr, R.col, R.v<T>(), AP.ptr, AP.v<T>(), Ac.ptr, Ac.v<T>(),
                                   (const uint16_t*)gs.pos, gs.off, 0, (T)0, (T*)nullptr, nullptr, nullptr,
                                   (T*)nullptr)));
        else
            AMG_WITH_GS1(gs.g, (k_galerkin_pos<T, GG, uint8_t><<<row_blocks(R.nrows, GG), TPB, sm, s>>>(
                                   R.nrows, gs.cap, R.ptr, R.col, R.v<T>(), AP.ptr, AP.v<T>(), Ac.ptr, Ac.v<T>(),
                                   (const uint8_t*)gs.pos, gs.off, 0, (T)0, (T*)nullptr, nullptr, nullptr,
                                   (T*)nullptr)));
        HIP_LAUNCH_CHECK();
        return;
    }
    AMG_WITH_G(g, k_galerkin_rap<G, T><<<row_blocks(R.nrows, G), TPB, 0, s>>>(
                      R.nrows, R.ptr, R.col, R.v<T>(), AP.ptr, AP.col, AP.v<T>(), Ac.ptr, Ac.col, Ac.v<T>()));
    HIP_LAUNCH_CHECK();
}

template bool launch_galerkin_ap<double>(const Csr&, const Csr&, const Csr&, int, GalShape, int, double, double*,
                                         const double*, hipStream_t);
template bool launch_galerkin_ap<float>(const Csr&, const Csr&, const Csr&, int, GalShape, int, double, float*,
                                        const double*, hipStream_t);
template void launch_galerkin_rap<double>(const Csr&, const Csr&, const Csr&, int, GalShape, hipStream_t);
template void launch_galerkin_rap<float>(const Csr&, const Csr&, const Csr&, int, GalShape, hipStream_t);
template void launch_smoother_diag<double>(const Csr&, int, double, double*, hipStream_t);
template void launch_smoother_diag<float>(const Csr&, int, double, float*, hipStream_t);

}  // namespace amgmi
