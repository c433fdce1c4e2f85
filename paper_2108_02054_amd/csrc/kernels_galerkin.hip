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
// row-by-row product adds them.  Which B entries a row's terms read, and the position of
// each term's column in the (cached, sorted) C row, depend on the patterns alone, so setup
// stores them once: for every L entry its B row start and the offset of its first term
// within the row's terms, and for every term its position in the C row (the position
// map).  Each numeric product then only multiplies, and adds each term into its C entry,
// kept in LDS.  A group of G lanes per row of C loads a chunk of the row's L entries
// (EPL per lane) into LDS, then walks them in order, WF_AHEAD at a time: the lanes load
// those entries' terms (G per entry per pass) together, then add them entry by entry.
// Positions within one B row are distinct, and the LDS operations of a wavefront complete
// in program order, so every entry of C receives its terms in the row-by-row order.  For
// C = A P the group also forms the smoother diagonal (the row's squares added in column
// order), and can take A's values from a new FP64 array, storing the hierarchy's copies
// on the way.

constexpr int WF_LOADS = 8;            // B terms per lane loaded together
constexpr int WF_CAP_MAX = 4096;       // longest C row the form takes
constexpr int64_t WF_TERMS_MAX = 65535;  // most terms in one C row (two-byte term offsets)
constexpr size_t WF_SMEM_MAX = 65536;  // LDS per block

// One staged L entry: its B row start, first term (within the row) and term count.
struct alignas(16) WfEnt {
    int bs, to, len, pad;
};

template <typename T, int G, int EPL>
constexpr size_t wf_group_smem(int cap) {
    return (size_t)cap * sizeof(T) + (size_t)EPL * G * (sizeof(T) + sizeof(WfEnt));
}

template <typename T, int G, typename PT, int EPL, int TPL>
__global__ __launch_bounds__(TPB) void k_galerkin_pos(
    int nrows, int cap, const int* __restrict__ Lptr, const T* __restrict__ Lval, const int* __restrict__ Lbst,
    const uint16_t* __restrict__ Ltof, const T* __restrict__ Bval, const int* __restrict__ Cptr,
    T* __restrict__ Cval, const PT* __restrict__ pos, const int64_t* __restrict__ poff,
    const int* __restrict__ dpos, int kind, T omega, T* __restrict__ m, const double* __restrict__ lin,
    double* __restrict__ lout64, T* __restrict__ loutT, const uint8_t* __restrict__ dslot, int64_t dn,
    double* __restrict__ dout64, T* __restrict__ doutT) {
    extern __shared__ __align__(16) unsigned char wf_smem[];
    constexpr int NE = EPL * G;  // L entries per chunk
    const int g = threadIdx.x & (G - 1);
    const int gi = threadIdx.x / G;
    unsigned char* gbase = wf_smem + (size_t)gi * wf_group_smem<T, G, EPL>(cap);
    T* sacc = reinterpret_cast<T*>(gbase);
    T* elv = reinterpret_cast<T*>(gbase + (size_t)cap * sizeof(T));
    WfEnt* ent = reinterpret_cast<WfEnt*>(gbase + (size_t)cap * sizeof(T) + (size_t)NE * sizeof(T));
    const int row = (xcd_block() * TPB + (int)threadIdx.x) / G;
    if (row >= nrows) return;  // groups leave whole: G divides the wavefront
    const int sb = Cptr[row];
    const int len = min(Cptr[row + 1] - sb, cap);  // the host keeps every row within cap
    const int lb = Lptr[row], le = Lptr[row + 1];
    const int64_t p0 = poff[row];
    const int nterm = (int)(poff[row + 1] - p0);
    const int dp = m != nullptr ? dpos[row] : -1;
    const PT* prow = pos + p0;
    for (int q = g; q < len; q += G) sacc[q] = 0;
    T d = 0, ss = 0;
    for (int c0 = lb; c0 < le; c0 += NE) {
        const int nt = min(NE, le - c0);  // uniform across the group
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
            const int u = e * G + g;
            const int t = c0 + u;
            if (u < nt) {
                T lv;
                if (lin != nullptr) {
                    const double x = lin[t];
                    if (lout64 != nullptr) lout64[t] = x;
                    if (loutT != nullptr) loutT[t] = (T)x;
                    if (dslot != nullptr) {  // straight into the diagonal storage of L
                        const size_t q = (size_t)dslot[t] * (size_t)dn + (size_t)row;
                        dout64[q] = x;
                        if (doutT != nullptr) doutT[q] = (T)x;
                    }
                    lv = (T)x;
                } else {
                    lv = Lval[t];
                }
                const int to = Ltof[t];
                const int tn = t + 1 < le ? (int)Ltof[t + 1] : nterm;
                elv[u] = lv;
                WfEnt w;
                w.bs = Lbst[t];
                w.to = to;
                w.len = tn - to;
                w.pad = 0;
                ent[u] = w;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (m != nullptr)
            for (int u = 0; u < nt; ++u) {  // the row's squares in column order
                const T a = elv[u];
                if (c0 + u == dp) d = a;
                ss = ss + a * a;
            }
        // Batches of WF_AHEAD entries, double-buffered: the terms of the next batch are
        // loaded before the current batch is added.  Each lane loads TPL terms of every
        // entry of a batch (g, and g + G with TPL = 2), so B rows of up to TPL G terms
        // need no further round trip; TPL = 2 pays for it with half the entries per batch.
        constexpr int WF_AHEAD = WF_LOADS / TPL;
        int up[WF_AHEAD], ul[WF_AHEAD], uq[WF_AHEAD];
        T bv[WF_AHEAD], bw[WF_AHEAD];
        auto load = [&](int u0, int (&qp)[WF_AHEAD], int (&ql)[WF_AHEAD], T (&qv)[WF_AHEAD], int (&qq)[WF_AHEAD],
                        T (&qw)[WF_AHEAD]) {
#pragma unroll
            for (int i = 0; i < WF_AHEAD; ++i) {  // first 2G terms of each entry, in flight together
                const int u = u0 + i < nt ? u0 + i : nt - 1;
                const WfEnt w = ent[u];
                ql[i] = u0 + i < nt ? w.len : 0;
                if (g < ql[i]) {
                    qp[i] = (int)prow[w.to + g];
                    qv[i] = Bval[w.bs + g];
                }
                if (TPL > 1 && g + G < ql[i]) {
                    qq[i] = (int)prow[w.to + g + G];
                    qw[i] = Bval[w.bs + g + G];
                }
            }
        };
        load(0, up, ul, bv, uq, bw);
        for (int u0 = 0; u0 < nt; u0 += WF_AHEAD) {
            int up2[WF_AHEAD], ul2[WF_AHEAD], uq2[WF_AHEAD];
            T bv2[WF_AHEAD], bw2[WF_AHEAD];
            if (u0 + WF_AHEAD < nt) load(u0 + WF_AHEAD, up2, ul2, bv2, uq2, bw2);  // uniform across the group
#pragma unroll
            for (int i = 0; i < WF_AHEAD; ++i) {
                if (ul[i] == 0) continue;  // uniform across the group
                const T lv = elv[u0 + i];
                if (g < ul[i] && up[i] < len) sacc[up[i]] = sacc[up[i]] + lv * bv[i];
                if (TPL > 1 && g + G < ul[i] && uq[i] < len) sacc[uq[i]] = sacc[uq[i]] + lv * bw[i];
                if (ul[i] > TPL * G) {  // rows of B longer than TPL G
                    const WfEnt w = ent[u0 + i];
                    for (int k = g + TPL * G; k < ul[i]; k += G) {
                        const int p = (int)prow[w.to + k];
                        const T b = Bval[w.bs + k];
                        if (p < len) sacc[p] = sacc[p] + lv * b;
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < WF_AHEAD; ++i) {
                up[i] = up2[i];
                ul[i] = ul2[i];
                bv[i] = bv2[i];
                uq[i] = uq2[i];
                bw[i] = bw2[i];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
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

// Per L entry: its B row start and the offset of its first term within its row's terms.
__global__ __launch_bounds__(TPB) void k_entry_meta(int nrows, const int* __restrict__ Lptr,
                                                    const int* __restrict__ Lcol, const int* __restrict__ Bptr,
                                                    int* __restrict__ bst, uint16_t* __restrict__ tof) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= nrows) return;
    int o = 0;
    for (int t = Lptr[i]; t < Lptr[i + 1]; ++t) {
        const int b = Bptr[Lcol[t]];
        bst[t] = b;
        tof[t] = (uint16_t)o;
        o += Bptr[Lcol[t] + 1] - b;
    }
}

// Index of each row's diagonal entry (-1 if absent).
__global__ __launch_bounds__(TPB) void k_diag_index(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                                                    int* __restrict__ dpos) {
    const int i = xcd_block() * TPB + threadIdx.x;
    if (i >= n) return;
    int lo = ptr[i], hi = ptr[i + 1];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (col[mid] < i)
            lo = mid + 1;
        else
            hi = mid;
    }
    dpos[i] = (lo < ptr[i + 1] && col[lo] == i) ? lo : -1;
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

int64_t count_galerkin_terms(const Csr& L, const Csr& B, int64_t* off, int64_t* max_row, hipStream_t s) {
    int64_t* cnt = dnew<int64_t>((size_t)L.nrows + 1, s);
    k_count_terms<<<row_blocks((int64_t)L.nrows + 1, 1), TPB, 0, s>>>(L.nrows, L.ptr, L.col, B.ptr, cnt);
    HIP_LAUNCH_CHECK();
    exclusive_scan_i64(cnt, off, (int64_t)L.nrows + 1, s);
    *max_row = max_i64(cnt, (int64_t)L.nrows + 1, s);
    dfree(cnt, s);
    int64_t total = 0;
    HIP_CHECK(hipMemcpyAsync(&total, off + L.nrows, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    return total;
}

bool galerkin_terms_fit(int64_t max_row) { return max_row <= WF_TERMS_MAX; }

void build_galerkin_posmap(const Csr& L, const Csr& B, const Csr& C, const GalShape& gs, hipStream_t s) {
    if (L.nrows == 0) return;
    k_entry_meta<<<row_blocks(L.nrows, 1), TPB, 0, s>>>(L.nrows, L.ptr, L.col, B.ptr, gs.bst, gs.tof);
    HIP_LAUNCH_CHECK();
    if (gs.dpos != nullptr) {
        k_diag_index<<<row_blocks(L.nrows, 1), TPB, 0, s>>>(L.nrows, L.ptr, L.col, gs.dpos);
        HIP_LAUNCH_CHECK();
    }
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

// Launch shape of the position-map form for C = L B from its sizes (rows and entries of L,
// terms, the longest C row): cap = the longest C row rounded up to a multiple of 8; TPL =
// 2 terms per lane and entry for products of at least TPL2_MIN_ROWS rows (more rows per
// wavefront, fewer B rows left to a second round trip; measured at 128^3: level-0 A P
// 286 against 315 us, R (A P) 215 against 241 us), else 1 (small products want every lane
// on few rows); G = the power of two in [4, 64] nearest above the mean number of terms
// per L entry over TPL (the mean referenced B row length, so that most B rows take one
// pass of the group), or at least an eighth of the mean L row length, raised until a
// block's LDS (TPB / G rows of cap FP64 accumulators and the staged L entries) is within
// WF_SMEM_MAX.  {0, ...}: the rows are too long for the form (lane-group kernels).
// gforce and tforce force G and TPL where the LDS allows.  The position map itself is
// built by the caller.
constexpr int32_t TPL2_MIN_ROWS = 1 << 16;
GalShape pick_galerkin_shape(int32_t nrows, int64_t nnzL, int64_t terms, int maxlen, int gforce, int tforce) {
    if (maxlen > WF_CAP_MAX) return {};
    const double mean_b = nnzL > 0 ? (double)terms / (double)nnzL : 1.0;
    const int cap = std::max(8, (maxlen + 7) / 8 * 8);
    const double mean_l = nrows > 0 ? (double)nnzL / (double)nrows : 1.0;
    const int tpl = (tforce == 1 || tforce == 2) ? tforce : (nrows >= TPL2_MIN_ROWS ? 2 : 1);
    int G = 4;
    while (G < 64 && G * tpl < mean_b) G <<= 1;
    while (G < 64 && 8 * G <= mean_l) G <<= 1;  // long L rows: wider groups, fewer chunks
    if (gforce == 4 || gforce == 8 || gforce == 16 || gforce == 32 || gforce == 64) G = gforce;
    const int epl = mean_l > 2.0 * G ? 4 : 2;
    auto smem = [&](int g) {
        return (size_t)(TPB / g) * ((size_t)cap * sizeof(double) + (size_t)epl * g * (sizeof(double) + sizeof(WfEnt)));
    };
    while (G < 64 && smem(G) > WF_SMEM_MAX) G <<= 1;
    if (smem(G) > WF_SMEM_MAX) return {};
    GalShape gs;
    gs.g = G;
    gs.cap = cap;
    gs.epl = epl;
    gs.wide = maxlen > 255 ? 1 : 0;
    gs.tpl = tpl;
    return gs;
}

template <typename T>
static size_t acc_smem(const GalShape& gs) {
    return (size_t)(TPB / gs.g) * ((size_t)gs.cap * sizeof(T) + (size_t)gs.epl * gs.g * (sizeof(T) + sizeof(WfEnt)));
}

// Launches the position-map kernel for one product with the shape's template arguments.
template <typename T>
static void launch_pos(const Csr& L, const Csr& B, const Csr& C, const GalShape& gs, int kind, double omega, T* m,
                       const double* lin, double* lout64, T* loutT, hipStream_t s, const Dia* dia = nullptr) {
    const size_t sm = acc_smem<T>(gs);
    const int* dp = m != nullptr ? gs.dpos : nullptr;
    const uint8_t* dslot = dia != nullptr ? dia->slot : nullptr;
    double* d64 = dia != nullptr ? dia->val : nullptr;
    T* dT = nullptr;
    if constexpr (!std::is_same<T, double>::value)
        if (dia != nullptr) dT = dia->val32;
#define AMG_POS_LAUNCH(PT, EPL, TPL)                                                                      \
    AMG_WITH_GS1(gs.g, (k_galerkin_pos<T, GG, PT, EPL, TPL><<<row_blocks(L.nrows, GG), TPB, sm, s>>>(      \
                           L.nrows, gs.cap, L.ptr, L.v<T>(), gs.bst, gs.tof, B.v<T>(), C.ptr, C.v<T>(),     \
                           (const PT*)gs.pos, gs.off, dp, kind, (T)omega, m, lin, lout64, loutT, dslot,     \
                           (int64_t)L.nrows, d64, dT)))
#define AMG_POS_LAUNCH_T(PT, EPL)                  \
    do {                                           \
        if (gs.tpl == 2) AMG_POS_LAUNCH(PT, EPL, 2); \
        else AMG_POS_LAUNCH(PT, EPL, 1);           \
    } while (0)
    if (gs.wide) {
        if (gs.epl == 4) AMG_POS_LAUNCH_T(uint16_t, 4);
        else AMG_POS_LAUNCH_T(uint16_t, 2);
    } else {
        if (gs.epl == 4) AMG_POS_LAUNCH_T(uint8_t, 4);
        else AMG_POS_LAUNCH_T(uint8_t, 2);
    }
#undef AMG_POS_LAUNCH_T
#undef AMG_POS_LAUNCH
    HIP_LAUNCH_CHECK();
}

template <typename T>
void launch_smoother_diag(const Csr& A, int kind, double omega, T* m, hipStream_t s) {
    k_smoother_diag<T><<<row_blocks(A.nrows, 1), TPB, 0, s>>>(A.nrows, A.ptr, A.col, A.v<T>(), kind, (T)omega, m);
    HIP_LAUNCH_CHECK();
}

// AP = A P; with m != nullptr also the smoother diagonal of A, and with ain != nullptr
// the values of A are taken from ain (FP64) and stored on the way: into the diagonal
// storage `dia` when one is given (its FP64 and, in mixed precision, FP32 arrays), else
// into A's CSR value arrays.  Only the position-map form fuses these; it returns true when
// it did (m and the values written).
template <typename T>
bool launch_galerkin_ap(const Csr& A, const Csr& P, const Csr& AP, int g, GalShape gs, int kind, double omega, T* m,
                        const double* ain, hipStream_t s, const Dia* dia) {
    if (gs.g > 0) {
        const bool to_dia = dia != nullptr && ain != nullptr;
        double* out64 = (!to_dia && ain != nullptr && ain != A.val) ? A.val : nullptr;
        T* outT = nullptr;
        if constexpr (!std::is_same<T, double>::value) outT = (!to_dia && ain != nullptr) ? A.v<T>() : nullptr;
        launch_pos<T>(A, P, AP, gs, kind, omega, m, ain, out64, outT, s, to_dia ? dia : nullptr);
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
        launch_pos<T>(R, AP, Ac, gs, 0, 0.0, (T*)nullptr, nullptr, nullptr, (T*)nullptr, s);
        return;
    }
    AMG_WITH_G(g, k_galerkin_rap<G, T><<<row_blocks(R.nrows, G), TPB, 0, s>>>(
                      R.nrows, R.ptr, R.col, R.v<T>(), AP.ptr, AP.col, AP.v<T>(), Ac.ptr, Ac.col, Ac.v<T>()));
    HIP_LAUNCH_CHECK();
}

template bool launch_galerkin_ap<double>(const Csr&, const Csr&, const Csr&, int, GalShape, int, double, double*,
                                         const double*, hipStream_t, const Dia*);
template bool launch_galerkin_ap<float>(const Csr&, const Csr&, const Csr&, int, GalShape, int, double, float*,
                                        const double*, hipStream_t, const Dia*);
template void launch_galerkin_rap<double>(const Csr&, const Csr&, const Csr&, int, GalShape, hipStream_t);
template void launch_galerkin_rap<float>(const Csr&, const Csr&, const Csr&, int, GalShape, hipStream_t);
template void launch_smoother_diag<double>(const Csr&, int, double, double*, hipStream_t);
template void launch_smoother_diag<float>(const Csr&, int, double, float*, hipStream_t);

}  // namespace amgmi
