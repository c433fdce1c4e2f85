/*
 * amg_oracle.cpp -- plain FP64 CPU oracle for partial-reuse smoothed-aggregation AMG.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load this library.  The product path (the HIP library) never links,
 * loads or calls it, and the two share no source.
 *
 * What it computes, following Demidov, "Partial Reuse AMG Setup Cost Amortization
 * Strategy for the Solution of Non-Steady State Problems":
 *   - Algorithm 1 (AMG setup): per level transfer operators P_l, R_l = P_l^T, smoother
 *     S_l, Galerkin operator A_{l+1} = R_l A_l P_l; a direct solver on the coarsest level.
 *   - Algorithm 2 (V-cycle), used once per Krylov iteration as the preconditioner
 *     (Section 2, last paragraph).
 *   - Algorithm 3 (full reuse: the hierarchy is left as built) and Algorithm 4 (partial
 *     reuse: P_l, R_l kept; smoothers, Galerkin operators and the coarse solver rebuilt),
 *     and the choice between them and a full rebuild from the solves so far (Section 3).
 * The transfer operators are smoothed aggregation (Vanek, Mandel, Brezina 1996); the
 * paper's own runs use plain aggregation, available here as an option; for its systems
 * with 4x4 blocks (Section 4) the nodes are aggregated (block_size unknowns per node share
 * an aggregate, chosen on the matrix of block Frobenius norms).  The Krylov
 * methods are preconditioned CG for SPD systems and BiCGStab (the paper's method, for its
 * non-symmetric systems; van der Vorst 1992, the V-cycle applied on the right).  Details
 * the paper leaves open are fixed as follows and documented per function: strength test,
 * distance-2 maximal independent set with a fixed hash priority, aggregate assembly,
 * prolongator smoothing, Jacobi/SPAI0 diagonal, dense Cholesky on the coarsest level
 * when A_0 is symmetric and dense LU without pivoting otherwise.
 *
 * Semantics are sequential.  Row loops may run under OpenMP; rows are independent and
 * every reduction (dot products, norms, sums along a row) is taken in index order by
 * one thread, so results do not depend on the thread count.  Build with
 * -ffp-contract=off: each "c += a * b" below is a rounded product then a rounded sum.
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

enum Status {
    ORA_OK = 0,
    ORA_ERR_ARG = -1,
    ORA_ERR_OOM = -3,
    ORA_ERR_PATTERN = -4,
    ORA_ERR_NOT_SPD = -5,
    ORA_ERR_BREAKDOWN = -6,
};

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

struct Csr {
    int32_t n_rows = 0, n_cols = 0;
    std::vector<int32_t> ptr, col;
    std::vector<double> val;
    int64_t nnz() const { return (int64_t)col.size(); }
};

}  // namespace

extern "C" {

/* Parameters.  Layout mirrored by the oracle's Python binding. */
typedef struct {
    int smoother;          /* 0 damped Jacobi, 1 SPAI0 */
    int aggregation;       /* 0 smoothed aggregation, 1 plain aggregation (P = P_tent) */
    double jacobi_omega;   /* damping of the Jacobi smoother */
    double eps_strong;     /* strength threshold on level 0, halved on each coarser level */
    int coarse_enough;     /* stop coarsening once a level has at most this many rows */
    int max_levels;
    int npre, npost;       /* smoothing sweeps before / after the coarse correction */
    double rtol;           /* stop when ||f - A u|| / ||f|| <= rtol (true residual) */
    int maxiter;
    int flexible_cg;       /* 1: beta = r.(z - z_old) / rho_old */
    int block_size;        /* unknowns per node (1: scalar); > 1 needs plain aggregation */
} ora_params;

typedef struct {
    int iters;
    int converged;
    double rel_res_true;
} ora_info;

}  // extern "C"

namespace {

/* ------------------------------------------------------------------ sparse kernels */

/* y = A x */
void spmv(const Csr& A, const double* x, double* y) {
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < A.n_rows; ++i) {
        double s = 0.0;
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) s += A.val[k] * x[A.col[k]];
        y[i] = s;
    }
}

/* r = f - A u */
void residual(const Csr& A, const double* f, const double* u, double* r) {
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < A.n_rows; ++i) {
        double s = 0.0;
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) s += A.val[k] * u[A.col[k]];
        r[i] = f[i] - s;
    }
}

double dot(const std::vector<double>& a, const std::vector<double>& b) {
    double s = 0.0;
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
    return s;
}

double norm2(const std::vector<double>& a) { return std::sqrt(dot(a, a)); }

/* C = A B by Gustavson's row-by-row method.  The pattern is structural (an entry
 * exists when some product term touches it, whatever its value), columns are sorted,
 * and each entry is the sum of its product terms taken in the order (k along row i of
 * A, then m along row col(k) of B), starting from 0.0. */
Csr spgemm(const Csr& A, const Csr& B) {
    Csr C;
    C.n_rows = A.n_rows;
    C.n_cols = B.n_cols;
    C.ptr.assign((size_t)A.n_rows + 1, 0);
#pragma omp parallel
    {
        std::vector<int32_t> mark((size_t)B.n_cols, -1);
#pragma omp for schedule(static)
        for (int32_t i = 0; i < A.n_rows; ++i) {
            int32_t cnt = 0;
            for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                int32_t j = A.col[k];
                for (int32_t m = B.ptr[j]; m < B.ptr[j + 1]; ++m) {
                    int32_t c = B.col[m];
                    if (mark[c] != i) {
                        mark[c] = i;
                        ++cnt;
                    }
                }
            }
            C.ptr[(size_t)i + 1] = cnt;
        }
    }
    for (int32_t i = 0; i < A.n_rows; ++i) C.ptr[(size_t)i + 1] += C.ptr[i];
    C.col.resize((size_t)C.ptr[A.n_rows]);
    C.val.resize((size_t)C.ptr[A.n_rows]);
#pragma omp parallel
    {
        std::vector<int32_t> mark((size_t)B.n_cols, -1);
        std::vector<double> acc((size_t)B.n_cols, 0.0);
#pragma omp for schedule(static)
        for (int32_t i = 0; i < A.n_rows; ++i) {
            int32_t pos = C.ptr[i];
            for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                int32_t j = A.col[k];
                double a = A.val[k];
                for (int32_t m = B.ptr[j]; m < B.ptr[j + 1]; ++m) {
                    int32_t c = B.col[m];
                    if (mark[c] != i) {
                        mark[c] = i;
                        acc[c] = 0.0;
                        C.col[pos++] = c;
                    }
                    acc[c] += a * B.val[m];
                }
            }
            std::sort(C.col.begin() + C.ptr[i], C.col.begin() + C.ptr[(size_t)i + 1]);
            for (int32_t q = C.ptr[i]; q < C.ptr[(size_t)i + 1]; ++q) C.val[q] = acc[C.col[q]];
        }
    }
    return C;
}

/* B = A^T with sorted columns (counting sort by column). */
Csr transpose(const Csr& A) {
    Csr T;
    T.n_rows = A.n_cols;
    T.n_cols = A.n_rows;
    T.ptr.assign((size_t)A.n_cols + 1, 0);
    for (int64_t k = 0; k < A.nnz(); ++k) T.ptr[(size_t)A.col[k] + 1]++;
    for (int32_t c = 0; c < A.n_cols; ++c) T.ptr[(size_t)c + 1] += T.ptr[c];
    T.col.resize(A.col.size());
    T.val.resize(A.col.size());
    std::vector<int32_t> next(T.ptr.begin(), T.ptr.end() - 1);
    for (int32_t i = 0; i < A.n_rows; ++i)
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
            int32_t p = next[A.col[k]]++;
            T.col[p] = i;
            T.val[p] = A.val[k];
        }
    return T;
}

bool same_pattern(const Csr& a, const Csr& b) {
    return a.n_rows == b.n_rows && a.n_cols == b.n_cols && a.ptr == b.ptr && a.col == b.col;
}

/* --------------------------------------------------------------- input checks (O0) */

/* Square CSR with sorted unique in-range columns, a positive diagonal, finite values and
 * a structurally symmetric pattern.  Fills diag_pos (position of a_ii) and tpos (for
 * every stored (i,j), the position of (j,i)). */
int check_matrix(const Csr& A, std::vector<int64_t>& diag_pos, std::vector<int64_t>& tpos) {
    const int32_t n = A.n_rows;
    if (A.ptr[0] != 0) return fail(ORA_ERR_ARG, "row_ptr[0] != 0");
    for (int32_t i = 0; i < n; ++i)
        if (A.ptr[(size_t)i + 1] < A.ptr[i]) return fail(ORA_ERR_ARG, "row_ptr not monotone");
    diag_pos.assign((size_t)n, -1);
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
            int32_t j = A.col[k];
            if (j < 0 || j >= n) return fail(ORA_ERR_ARG, "column out of range");
            if (k > A.ptr[i] && A.col[(size_t)k - 1] >= j)
                return fail(ORA_ERR_PATTERN, "columns not sorted/unique in row " + std::to_string(i));
            if (!std::isfinite(A.val[k])) return fail(ORA_ERR_ARG, "non-finite value");
            if (j == i) diag_pos[i] = k;
        }
        if (diag_pos[i] < 0 || !(A.val[diag_pos[i]] > 0.0))
            return fail(ORA_ERR_NOT_SPD, "missing or non-positive diagonal in row " + std::to_string(i));
    }
    tpos.assign(A.col.size(), -1);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
            int32_t j = A.col[k];
            const int32_t* b = A.col.data() + A.ptr[j];
            const int32_t* e = A.col.data() + A.ptr[(size_t)j + 1];
            const int32_t* it = std::lower_bound(b, e, i);
            if (it == e || *it != i) return fail(ORA_ERR_PATTERN, "pattern not structurally symmetric");
            tpos[k] = A.ptr[j] + (it - b);
        }
    return ORA_OK;
}

/* ------------------------------------------------------- aggregation (setup, Alg. 1) */

/* Priority of node i in the distance-2 independent set: the SplitMix64 finaliser
 * (Steele, Lea, Flood 2014), a bijection on 64-bit integers, applied to i. */
uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Strength of connection (O1).  The off-diagonal entry k = (i,j) is strong when
 *   (a_ij * a_ji) > (eps * eps) * |a_ii * a_jj|
 * with exactly this association.  Row i is isolated when it has no strong entry. */
void strength(const Csr& A, double eps, const std::vector<int64_t>& diag_pos,
              const std::vector<int64_t>& tpos, std::vector<uint8_t>& strong) {
    strong.assign(A.col.size(), 0);
    const double eps2 = eps * eps;
    for (int32_t i = 0; i < A.n_rows; ++i) {
        double aii = A.val[diag_pos[i]];
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
            int32_t j = A.col[k];
            if (j == i) continue;
            double ajj = A.val[diag_pos[j]];
            double lhs = A.val[k] * A.val[tpos[k]];
            double rhs = eps2 * std::fabs(aii * ajj);
            strong[k] = lhs > rhs ? 1 : 0;
        }
    }
}

/* Aggregation (O2, O3).
 *  roots: the greedy distance-2 maximal independent set of the strong graph over
 *    non-isolated nodes, visiting nodes by decreasing mix64 priority; a node becomes a
 *    root when no root lies within strong-graph distance 2.
 *  ids: roots are numbered 0..nc-1 in increasing node order.
 *  pass 1: a root and each of its strong neighbours take the root's id.
 *  pass 2: every other non-isolated node takes the pass-1 id of the strong neighbour j
 *    with the largest a_ij * a_ji (ties: smaller id).
 *  isolated nodes: agg = -1. */
int aggregate(const Csr& A, const std::vector<uint8_t>& strong, const std::vector<int64_t>& tpos,
              std::vector<int32_t>& agg, int32_t& nc) {
    const int32_t n = A.n_rows;
    std::vector<uint8_t> isolated((size_t)n, 1);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
            if (strong[k]) isolated[i] = 0;

    std::vector<int32_t> order;
    for (int32_t i = 0; i < n; ++i)
        if (!isolated[i]) order.push_back(i);
    std::sort(order.begin(), order.end(),
              [](int32_t a, int32_t b) { return mix64((uint64_t)a) > mix64((uint64_t)b); });

    std::vector<uint8_t> is_root((size_t)n, 0), covered((size_t)n, 0);
    for (int32_t v : order) {
        if (covered[v]) continue;
        is_root[v] = 1;
        covered[v] = 1;
        for (int32_t k = A.ptr[v]; k < A.ptr[(size_t)v + 1]; ++k) {
            if (!strong[k]) continue;
            int32_t j = A.col[k];
            covered[j] = 1;
            for (int32_t q = A.ptr[j]; q < A.ptr[(size_t)j + 1]; ++q)
                if (strong[q]) covered[A.col[q]] = 1;
        }
    }

    agg.assign((size_t)n, -1);
    nc = 0;
    for (int32_t i = 0; i < n; ++i)
        if (is_root[i]) agg[i] = nc++;
    std::vector<int32_t> pass1(agg);
    for (int32_t r = 0; r < n; ++r) {
        if (!is_root[r]) continue;
        for (int32_t k = A.ptr[r]; k < A.ptr[(size_t)r + 1]; ++k)
            if (strong[k]) pass1[A.col[k]] = agg[r];
    }
    for (int32_t i = 0; i < n; ++i) {
        if (isolated[i] || pass1[i] >= 0) {
            agg[i] = pass1[i];
            continue;
        }
        int32_t best = -1;
        double best_w = 0.0;
        for (int32_t k = A.ptr[i]; k < A.ptr[(size_t)i + 1]; ++k) {
            if (!strong[k]) continue;
            int32_t j = A.col[k];
            if (pass1[j] < 0) continue;
            double w = A.val[k] * A.val[tpos[k]];
            if (best < 0 || w > best_w || (w == best_w && pass1[j] < best)) {
                best = pass1[j];
                best_w = w;
            }
        }
        if (best < 0) return fail(ORA_ERR_PATTERN, "node without an aggregate (MIS-2 not maximal)");
        agg[i] = best;
    }
    return ORA_OK;
}

/* Node matrix of a system with B unknowns per node (unknown b of node I is row I*B + b):
 * entry (I, J) is the Frobenius norm of the B x B block A(IB.., JB..), its squares added
 * row by row, column by column.  Every stored block must be full and the B rows of a node
 * must list the same columns.  map[k] = node entry of stored entry k. */
int node_matrix(const Csr& A, int B, Csr& Nm, std::vector<int64_t>& map) {
    if (A.n_rows % B != 0) return fail(ORA_ERR_ARG, "block_size does not divide the row count");
    const int32_t nn = A.n_rows / B;
    Nm = Csr();
    Nm.n_rows = Nm.n_cols = nn;
    Nm.ptr.assign((size_t)nn + 1, 0);
    map.assign(A.col.size(), 0);
    for (int32_t I = 0; I < nn; ++I) {
        const int32_t r0 = I * B;
        const int32_t b0 = A.ptr[r0], len = A.ptr[(size_t)r0 + 1] - b0;
        if (len % B != 0) return fail(ORA_ERR_PATTERN, "block_size needs full blocks");
        for (int c = 1; c < B; ++c) {
            const int32_t bc = A.ptr[(size_t)r0 + c];
            if (A.ptr[(size_t)r0 + c + 1] - bc != len) return fail(ORA_ERR_PATTERN, "block_size needs full blocks");
            for (int32_t k = 0; k < len; ++k)
                if (A.col[(size_t)bc + k] != A.col[(size_t)b0 + k])
                    return fail(ORA_ERR_PATTERN, "block_size needs full blocks");
        }
        for (int32_t g = 0; g < len / B; ++g) {
            const int32_t c0 = A.col[(size_t)b0 + g * B];
            if (c0 % B != 0) return fail(ORA_ERR_PATTERN, "block_size needs full blocks");
            for (int q = 1; q < B; ++q)
                if (A.col[(size_t)b0 + g * B + q] != c0 + q) return fail(ORA_ERR_PATTERN, "block_size needs full blocks");
            double ss = 0.0;
            for (int c = 0; c < B; ++c)
                for (int q = 0; q < B; ++q) {
                    const int64_t k = (int64_t)A.ptr[(size_t)r0 + c] + g * B + q;
                    ss += A.val[k] * A.val[k];
                    map[k] = (int64_t)Nm.col.size();
                }
            Nm.col.push_back(c0 / B);
            Nm.val.push_back(std::sqrt(ss));
        }
        Nm.ptr[(size_t)I + 1] = (int32_t)Nm.col.size();
    }
    return ORA_OK;
}

/* Tentative prolongator (O4): P_tent[i, agg(i)] = 1, empty row when agg(i) = -1. */
Csr tentative(const std::vector<int32_t>& agg, int32_t nc) {
    Csr P;
    P.n_rows = (int32_t)agg.size();
    P.n_cols = nc;
    P.ptr.assign(agg.size() + 1, 0);
    for (size_t i = 0; i < agg.size(); ++i) {
        P.ptr[i + 1] = P.ptr[i];
        if (agg[i] >= 0) {
            P.col.push_back(agg[i]);
            P.val.push_back(1.0);
            P.ptr[i + 1]++;
        }
    }
    return P;
}

/* Filtered operator (O5): non-isolated rows keep the diagonal and the strong entries;
 * weak off-diagonal entries are added onto the diagonal (row sums are preserved), the
 * diagonal being a_ii followed by the weak entries in column order.  Isolated rows
 * keep only the diagonal. */
Csr filtered(const Csr& A, const std::vector<uint8_t>& strong, const std::vector<int64_t>& diag_pos,
             const std::vector<int32_t>& agg) {
    Csr F;
    F.n_rows = F.n_cols = A.n_rows;
    F.ptr.assign((size_t)A.n_rows + 1, 0);
    for (int32_t i = 0; i < A.n_rows; ++i) {
        bool iso = agg[i] < 0;
        double d = A.val[diag_pos[i]];
        if (!iso)
            for (int32_t k = A.ptr[i]; k < A.ptr[(size_t)i + 1]; ++k)
                if (A.col[k] != i && !strong[k]) d += A.val[k];
        for (int32_t k = A.ptr[i]; k < A.ptr[(size_t)i + 1]; ++k) {
            int32_t j = A.col[k];
            if (j == i) {
                F.col.push_back(j);
                F.val.push_back(d);
            } else if (!iso && strong[k]) {
                F.col.push_back(j);
                F.val.push_back(A.val[k]);
            }
        }
        F.ptr[(size_t)i + 1] = (int32_t)F.col.size();
    }
    return F;
}

/* Smoothed prolongator (O6, O7):
 *   rho   = max_i sum_j |aF_ij| / |aF_ii|   (Gershgorin bound on D_F^-1 A_F)
 *   omega = (4/3) / rho
 *   P     = P_tent - (omega / aF_ii) * (A_F P_tent)    row by row
 * on the union pattern (explicit zeros kept). */
Csr smoothed_prolongator(const Csr& F, const Csr& Pt) {
    const int32_t n = F.n_rows;
    std::vector<double> dF((size_t)n, 0.0);
    double rho = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = F.ptr[i]; k < F.ptr[(size_t)i + 1]; ++k) {
            s += std::fabs(F.val[k]);
            if (F.col[k] == i) dF[i] = F.val[k];
        }
        double ratio = s / std::fabs(dF[i]);
        if (ratio > rho) rho = ratio;
    }
    const double omega = (4.0 / 3.0) / rho;
    Csr FP = spgemm(F, Pt);
    Csr P;
    P.n_rows = n;
    P.n_cols = Pt.n_cols;
    P.ptr.assign((size_t)n + 1, 0);
    for (int32_t i = 0; i < n; ++i) {
        double scale = omega / dF[i];
        int32_t a = Pt.ptr[i], ae = Pt.ptr[(size_t)i + 1];
        int32_t b = FP.ptr[i], be = FP.ptr[(size_t)i + 1];
        while (a < ae || b < be) {
            int32_t ca = a < ae ? Pt.col[a] : INT32_MAX;
            int32_t cb = b < be ? FP.col[b] : INT32_MAX;
            int32_t c = std::min(ca, cb);
            double pt = (ca == c) ? Pt.val[a++] : 0.0;
            double fp = (cb == c) ? FP.val[b++] : 0.0;
            P.col.push_back(c);
            P.val.push_back(pt - scale * fp);
        }
        P.ptr[(size_t)i + 1] = (int32_t)P.col.size();
    }
    return P;
}

/* ------------------------------------------------------------------ smoother (O10) */

/* Diagonal of the smoother S_l: damped Jacobi m_i = omega_J / a_ii, or SPAI0
 * m_i = a_ii / sum_j a_ij^2 (sum along the stored row in column order). */
void smoother_diag(const Csr& A, int kind, double omega, std::vector<double>& m) {
    m.assign((size_t)A.n_rows, 0.0);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < A.n_rows; ++i) {
        double d = 0.0, s = 0.0;
        for (int32_t k = A.ptr[i]; k < A.ptr[(size_t)i + 1]; ++k) {
            if (A.col[k] == i) d = A.val[k];
            s += A.val[k] * A.val[k];
        }
        m[i] = (kind == 1) ? d / s : omega / d;
    }
}

/* Damped block Jacobi for systems with B unknowns per node: M_I = omega * D_I^{-1}, D_I the
 * B x B diagonal block of node I, stored row-major at m[I*B*B ..].  The inverse is taken by
 * Gauss-Jordan elimination with partial pivoting on [D_I | I] (the first row of largest
 * magnitude in the column is the pivot); a zero pivot means D_I is singular. */
int block_smoother(const Csr& A, int B, double omega, std::vector<double>& m) {
    const int32_t nn = A.n_rows / B;
    m.assign((size_t)A.n_rows * B, 0.0);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int32_t I = 0; I < nn; ++I) {
        std::vector<double> W((size_t)B * 2 * B, 0.0);  // [D | I], row-major, 2B columns
        for (int a = 0; a < B; ++a) {
            const int32_t r = I * B + a;
            for (int32_t k = A.ptr[r]; k < A.ptr[(size_t)r + 1]; ++k)
                if (A.col[k] >= I * B && A.col[k] < I * B + B) W[(size_t)a * 2 * B + (A.col[k] - I * B)] = A.val[k];
            W[(size_t)a * 2 * B + B + a] = 1.0;
        }
        for (int k = 0; k < B; ++k) {
            int piv = k;
            for (int a = k + 1; a < B; ++a)
                if (std::fabs(W[(size_t)a * 2 * B + k]) > std::fabs(W[(size_t)piv * 2 * B + k])) piv = a;
            if (W[(size_t)piv * 2 * B + k] == 0.0) {
                bad = 1;
                break;
            }
            if (piv != k)
                for (int q = 0; q < 2 * B; ++q) std::swap(W[(size_t)k * 2 * B + q], W[(size_t)piv * 2 * B + q]);
            const double d = W[(size_t)k * 2 * B + k];
            for (int q = 0; q < 2 * B; ++q) W[(size_t)k * 2 * B + q] /= d;
            for (int a = 0; a < B; ++a) {
                if (a == k) continue;
                const double f = W[(size_t)a * 2 * B + k];
                for (int q = 0; q < 2 * B; ++q) W[(size_t)a * 2 * B + q] -= f * W[(size_t)k * 2 * B + q];
            }
        }
        for (int a = 0; a < B; ++a)
            for (int q = 0; q < B; ++q) m[((size_t)I * B + a) * B + q] = omega * W[(size_t)a * 2 * B + B + q];
    }
    return bad ? fail(ORA_ERR_NOT_SPD, "singular diagonal block") : ORA_OK;
}

/* u += M t: the scalar diagonal (B = 1) or the block diagonal, each row's block product
 * summed in column order before it is added. */
void smoother_apply(const std::vector<double>& m, int B, const std::vector<double>& t, std::vector<double>& u) {
    const int32_t n = (int32_t)u.size();
    if (B == 1) {
        for (int32_t i = 0; i < n; ++i) u[i] += m[i] * t[i];
        return;
    }
    for (int32_t i = 0; i < n; ++i) {
        const int32_t base = i - i % B;
        double s = 0.0;
        for (int q = 0; q < B; ++q) s += m[(size_t)i * B + q] * t[(size_t)base + q];
        u[i] += s;
    }
}

/* ------------------------------------------------------- coarsest solver (O11) */

/* Dense right-looking Cholesky A = L L^T of the coarsest operator (row-major, lower
 * triangle holds L).  A non-positive pivot means the operator is not SPD. */
int cholesky(const Csr& A, std::vector<double>& L) {
    const int32_t n = A.n_rows;
    L.assign((size_t)n * n, 0.0);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = A.ptr[i]; k < A.ptr[(size_t)i + 1]; ++k) L[(size_t)i * n + A.col[k]] = A.val[k];
    for (int32_t k = 0; k < n; ++k) {
        double piv = L[(size_t)k * n + k];
        if (!(piv > 0.0)) return fail(ORA_ERR_NOT_SPD, "non-positive pivot in the coarse Cholesky");
        double lkk = std::sqrt(piv);
        L[(size_t)k * n + k] = lkk;
        for (int32_t i = k + 1; i < n; ++i) L[(size_t)i * n + k] /= lkk;
        for (int32_t j = k + 1; j < n; ++j) {
            double ljk = L[(size_t)j * n + k];
            for (int32_t i = j; i < n; ++i) L[(size_t)i * n + j] -= L[(size_t)i * n + k] * ljk;
        }
    }
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j < n; ++j) L[(size_t)i * n + j] = 0.0;
    return ORA_OK;
}

/* x = (L L^T)^-1 b by forward then backward substitution. */
void cholesky_solve(const std::vector<double>& L, int32_t n, const double* b, double* x) {
    std::vector<double> y((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        double s = b[i];
        for (int32_t j = 0; j < i; ++j) s -= L[(size_t)i * n + j] * y[j];
        y[i] = s / L[(size_t)i * n + i];
    }
    for (int32_t i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int32_t j = i + 1; j < n; ++j) s -= L[(size_t)j * n + i] * x[j];
        x[i] = s / L[(size_t)i * n + i];
    }
}

/* Dense LU A = L U without pivoting (Doolittle: L unit lower, U upper, packed row-major
 * into one matrix) of a non-symmetric coarsest operator.  A non-positive or non-finite
 * pivot is rejected, as for the Cholesky pivots (the operators here are M-matrices whose
 * elimination pivots are positive). */
int lu_nopivot(const Csr& A, std::vector<double>& LU) {
    const int32_t n = A.n_rows;
    LU.assign((size_t)n * n, 0.0);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = A.ptr[i]; k < A.ptr[(size_t)i + 1]; ++k) LU[(size_t)i * n + A.col[k]] = A.val[k];
    for (int32_t k = 0; k < n; ++k) {
        const double piv = LU[(size_t)k * n + k];
        if (!(piv > 0.0) || !std::isfinite(piv)) return fail(ORA_ERR_NOT_SPD, "non-positive pivot in the coarse LU");
        for (int32_t i = k + 1; i < n; ++i) {
            const double lik = LU[(size_t)i * n + k] / piv;
            LU[(size_t)i * n + k] = lik;
            for (int32_t j = k + 1; j < n; ++j) LU[(size_t)i * n + j] -= lik * LU[(size_t)k * n + j];
        }
    }
    return ORA_OK;
}

/* x = (L U)^-1 b by forward (unit L) then backward substitution. */
void lu_solve(const std::vector<double>& LU, int32_t n, const double* b, double* x) {
    std::vector<double> y((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        double s = b[i];
        for (int32_t j = 0; j < i; ++j) s -= LU[(size_t)i * n + j] * y[j];
        y[i] = s;
    }
    for (int32_t i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int32_t j = i + 1; j < n; ++j) s -= LU[(size_t)i * n + j] * x[j];
        x[i] = s / LU[(size_t)i * n + i];
    }
}

/* True when every stored a_ij equals a_ji (same pattern assumed structurally symmetric). */
bool symmetric_values(const Csr& A) {
    for (int32_t i = 0; i < A.n_rows; ++i)
        for (int32_t k = A.ptr[i]; k < A.ptr[(size_t)i + 1]; ++k) {
            const int32_t j = A.col[k];
            const int32_t* b = A.col.data() + A.ptr[j];
            const int32_t* e = A.col.data() + A.ptr[(size_t)j + 1];
            const int32_t* q = std::lower_bound(b, e, i);
            if (q == e || *q != i || A.val[(size_t)(q - A.col.data())] != A.val[k]) return false;
        }
    return true;
}

/* --------------------------------------------------------------------- hierarchy */

struct Level {
    Csr A, P, R;
    std::vector<int32_t> agg;
    std::vector<uint8_t> strong;
    std::vector<double> m;
    std::vector<double> u, f, r, t;  // V-cycle work vectors
};

/* What the rebuild policy looks at (Section 3): updates since the last full build, the
 * iterations of the first solve after it (0: none yet), the last solve's iterations (0:
 * none yet; a solve that needed none counts as one) and whether it converged. */
struct History {
    int updates = 0;
    int iters_ref = 0;
    int last_iters = 0;
    int last_converged = 0;
};

struct Hierarchy {
    ora_params prm{};
    std::vector<Level> lv;
    Csr A_outer;            // the operator the Krylov solver iterates with
    std::vector<double> L;  // Cholesky factor of the coarsest operator, or its packed LU
    bool coarse_lu = false; // A_0 is not symmetric: L holds the coarsest operator's L U
    bool transfer_given = false;
    History hist;
};

const int kMaxDense = 8192;

/* Coarse factorisation and smoothers on every non-coarsest level. */
int finish_levels(Hierarchy& h) {
    for (size_t l = 0; l + 1 < h.lv.size(); ++l) {
        if (h.prm.block_size > 1) {
            int st = block_smoother(h.lv[l].A, h.prm.block_size, h.prm.jacobi_omega, h.lv[l].m);
            if (st) return st;
        } else {
            smoother_diag(h.lv[l].A, h.prm.smoother, h.prm.jacobi_omega, h.lv[l].m);
        }
    }
    Level& c = h.lv.back();
    if (c.A.n_rows > kMaxDense) return fail(ORA_ERR_ARG, "coarsest level too large for a dense solve");
    for (auto& l : h.lv) {
        l.u.assign((size_t)l.A.n_rows, 0.0);
        l.f.assign((size_t)l.A.n_rows, 0.0);
        l.r.assign((size_t)l.A.n_rows, 0.0);
        l.t.assign((size_t)l.A.n_rows, 0.0);
    }
    // Galerkin operators of a symmetric A_0 are symmetric up to rounding: Cholesky then
    h.coarse_lu = !symmetric_values(h.lv[0].A);
    return h.coarse_lu ? lu_nopivot(c.A, h.L) : cholesky(c.A, h.L);
}

/* Algorithm 1: build the hierarchy from A. */
int setup(Hierarchy& h, const Csr& A0) {
    h.hist = History{};
    h.lv.clear();
    h.lv.emplace_back();
    h.lv[0].A = A0;
    h.A_outer = A0;
    const ora_params& p = h.prm;
    if (p.block_size < 1 || (p.block_size > 1 && (p.aggregation != 1 || p.smoother != 0)))
        return fail(ORA_ERR_ARG, "block_size must be 1, or > 1 with plain aggregation and damped Jacobi");
    for (int l = 0;; ++l) {
        Level& cur = h.lv[(size_t)l];
        std::vector<int64_t> dpos, tpos;
        int st = check_matrix(cur.A, dpos, tpos);
        if (st) return st;
        if (cur.A.n_rows <= p.coarse_enough || l >= p.max_levels - 1) break;
        double eps = std::ldexp(p.eps_strong, -l);
        int32_t nc = 0;
        if (p.block_size > 1) {
            // systems: aggregate nodes (the strength test and MIS-2 on the node matrix of
            // block norms); unknown b of a node joins unknown b of its node's aggregate
            const int B = p.block_size;
            Csr Nm;
            std::vector<int64_t> map, ndpos, ntpos;
            st = node_matrix(cur.A, B, Nm, map);
            if (st) return st;
            st = check_matrix(Nm, ndpos, ntpos);
            if (st) return st;
            std::vector<uint8_t> nstrong;
            std::vector<int32_t> nagg;
            strength(Nm, eps, ndpos, ntpos, nstrong);
            int32_t ncn = 0;
            st = aggregate(Nm, nstrong, ntpos, nagg, ncn);
            if (st) return st;
            cur.agg.assign((size_t)cur.A.n_rows, -1);
            for (int32_t i = 0; i < cur.A.n_rows; ++i)
                if (nagg[(size_t)i / B] >= 0) cur.agg[(size_t)i] = nagg[(size_t)i / B] * B + i % B;
            cur.strong.assign(cur.A.col.size(), 0);
            for (size_t k = 0; k < cur.A.col.size(); ++k) cur.strong[k] = nstrong[(size_t)map[k]];
            nc = ncn * B;
        } else {
            strength(cur.A, eps, dpos, tpos, cur.strong);
            st = aggregate(cur.A, cur.strong, tpos, cur.agg, nc);
            if (st) return st;
        }
        if (nc == 0 || nc >= cur.A.n_rows) break;
        Csr Pt = tentative(cur.agg, nc);
        if (p.aggregation == 1) {
            cur.P = Pt;
        } else {
            Csr F = filtered(cur.A, cur.strong, dpos, cur.agg);
            cur.P = smoothed_prolongator(F, Pt);
        }
        cur.R = transpose(cur.P);
        Csr AP = spgemm(cur.A, cur.P);
        Csr Ac = spgemm(cur.R, AP);
        h.lv.emplace_back();
        h.lv.back().A = std::move(Ac);
    }
    return finish_levels(h);
}

/* Algorithm 4, update branch: keep P_l, R_l; rebuild smoothers, Galerkin operators
 * (whose patterns must not change) and the coarse factorisation. */
int partial_rebuild(Hierarchy& h, const double* val) {
    Csr& A0 = h.lv[0].A;
    std::copy(val, val + A0.nnz(), A0.val.begin());
    std::copy(val, val + A0.nnz(), h.A_outer.val.begin());
    for (size_t l = 0; l + 1 < h.lv.size(); ++l) {
        Csr AP = spgemm(h.lv[l].A, h.lv[l].P);
        Csr Ac = spgemm(h.lv[l].R, AP);
        if (!same_pattern(Ac, h.lv[l + 1].A)) return fail(ORA_ERR_PATTERN, "Galerkin pattern changed");
        h.lv[l + 1].A.val = std::move(Ac.val);
    }
    return finish_levels(h);
}

/* Algorithm 2: one V-cycle z = B r from a zero initial guess. */
void vcycle_level(Hierarchy& h, size_t l) {
    Level& L = h.lv[l];
    const int32_t n = L.A.n_rows;
    if (l + 1 == h.lv.size()) {
        if (h.coarse_lu)
            lu_solve(h.L, n, L.f.data(), L.u.data());
        else
            cholesky_solve(h.L, n, L.f.data(), L.u.data());
        return;
    }
    const ora_params& p = h.prm;
    std::fill(L.u.begin(), L.u.end(), 0.0);
    for (int s = 0; s < p.npre; ++s) {
        residual(L.A, L.f.data(), L.u.data(), L.t.data());
        smoother_apply(L.m, p.block_size, L.t, L.u);
    }
    residual(L.A, L.f.data(), L.u.data(), L.r.data());
    Level& C = h.lv[l + 1];
    spmv(L.R, L.r.data(), C.f.data());
    vcycle_level(h, l + 1);
    spmv(L.P, C.u.data(), L.t.data());
    for (int32_t i = 0; i < n; ++i) L.u[i] += L.t[i];
    for (int s = 0; s < p.npost; ++s) {
        residual(L.A, L.f.data(), L.u.data(), L.t.data());
        smoother_apply(L.m, p.block_size, L.t, L.u);
    }
}

void vcycle(Hierarchy& h, const double* r, double* z) {
    Level& L = h.lv[0];
    std::copy(r, r + L.A.n_rows, L.f.begin());
    vcycle_level(h, 0);
    std::copy(L.u.begin(), L.u.end(), z);
}

/* Preconditioned CG with one V-cycle as the preconditioner.  Stops when the true
 * relative residual ||f - A u|| / ||f|| is at most rtol. */
int pcg(Hierarchy& h, const double* fin, double* uin, ora_info* info) {
    const Csr& A = h.A_outer;
    const size_t n = (size_t)A.n_rows;
    const ora_params& p = h.prm;
    std::vector<double> f(fin, fin + n), x(uin, uin + n), r(n), z(n), zold(n), pv(n), q(n);
    info->iters = 0;
    info->converged = 0;
    info->rel_res_true = 0.0;
    double nf = norm2(f);
    if (nf == 0.0) {
        std::fill(uin, uin + n, 0.0);
        info->converged = 1;
        return ORA_OK;
    }
    residual(A, f.data(), x.data(), r.data());
    double res = norm2(r) / nf;
    if (res <= p.rtol) {
        info->converged = 1;
        info->rel_res_true = res;
        return ORA_OK;
    }
    vcycle(h, r.data(), z.data());
    pv = z;
    double rho = dot(r, z);
    int it = 0;
    while (it < p.maxiter) {
        ++it;
        spmv(A, pv.data(), q.data());
        double pq = dot(pv, q);
        if (!(pq > 0.0) || !std::isfinite(rho)) {
            info->iters = it;
            return fail(ORA_ERR_BREAKDOWN, "CG breakdown (p.Ap <= 0 or non-finite)");
        }
        double alpha = rho / pq;
        for (size_t i = 0; i < n; ++i) x[i] += alpha * pv[i];
        for (size_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
        res = norm2(r) / nf;
        if (res <= p.rtol) {
            residual(A, f.data(), x.data(), r.data());
            res = norm2(r) / nf;
            if (res <= p.rtol) {
                info->converged = 1;
                break;
            }
        }
        if (p.flexible_cg) zold = z;
        vcycle(h, r.data(), z.data());
        double rho_new = dot(r, z);
        double beta;
        if (p.flexible_cg) {
            double s = 0.0;
            for (size_t i = 0; i < n; ++i) s += r[i] * (z[i] - zold[i]);
            beta = s / rho;
        } else {
            beta = rho_new / rho;
        }
        rho = rho_new;
        for (size_t i = 0; i < n; ++i) pv[i] = z[i] + beta * pv[i];
    }
    if (!info->converged) {
        residual(A, f.data(), x.data(), r.data());
        res = norm2(r) / nf;
    }
    info->iters = it;
    info->rel_res_true = res;
    std::copy(x.begin(), x.end(), uin);
    return ORA_OK;
}

/* BiCGStab (van der Vorst 1992) with one V-cycle M applied on the right, the paper's
 * Krylov method for its non-symmetric systems.  With r^ = r_0 fixed: rho = r^.r;
 * beta = (rho / rho_prev)(alpha / omega); p = r + beta (p - omega v) (p = r at the first
 * step); p^ = M p; v = A p^; alpha = rho / r^.v; s = r - alpha v; s^ = M s; t = A s^;
 * omega = t.s / t.t; x += alpha p^ + omega s^; r = s - omega t.  When ||s|| or ||r||
 * reaches rtol the true residual f - A x is formed; if it is not small enough the method
 * restarts from it (r^ = r, p = v = 0).  A zero or non-finite rho, r^.v, t.t or omega is
 * a breakdown. */
int bicgstab(Hierarchy& h, const double* fin, double* uin, ora_info* info) {
    const Csr& A = h.A_outer;
    const size_t n = (size_t)A.n_rows;
    const ora_params& prm = h.prm;
    std::vector<double> f(fin, fin + n), x(uin, uin + n), r(n), rh(n), p(n, 0.0), v(n, 0.0), ph(n), s(n), sh(n),
        t(n);
    info->iters = 0;
    info->converged = 0;
    info->rel_res_true = 0.0;
    const double nf = norm2(f);
    if (nf == 0.0) {
        std::fill(uin, uin + n, 0.0);
        info->converged = 1;
        return ORA_OK;
    }
    residual(A, f.data(), x.data(), r.data());
    double res = norm2(r) / nf;
    if (res <= prm.rtol) {
        info->converged = 1;
        info->rel_res_true = res;
        return ORA_OK;
    }
    rh = r;
    double rho_prev = 1.0, alpha = 1.0, omega = 1.0;
    bool fresh = true;  // the first step after the start or a restart: p = r
    int it = 0;
    auto breakdown = [&](const char* what) {
        info->iters = it;
        return fail(ORA_ERR_BREAKDOWN, std::string("BiCGStab breakdown: ") + what);
    };
    // true residual; true (converged) or restart from it
    auto settle = [&]() {
        residual(A, f.data(), x.data(), r.data());
        res = norm2(r) / nf;
        if (res <= prm.rtol) return true;
        rh = r;
        std::fill(p.begin(), p.end(), 0.0);
        std::fill(v.begin(), v.end(), 0.0);
        rho_prev = alpha = omega = 1.0;
        fresh = true;
        return false;
    };
    while (it < prm.maxiter) {
        ++it;
        const double rho = dot(rh, r);
        if (rho == 0.0 || !std::isfinite(rho)) return breakdown("r^.r = 0");
        if (fresh) {
            p = r;
            fresh = false;
        } else {
            const double beta = (rho / rho_prev) * (alpha / omega);
            for (size_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        }
        vcycle(h, p.data(), ph.data());
        spmv(A, ph.data(), v.data());
        const double rv = dot(rh, v);
        if (rv == 0.0 || !std::isfinite(rv)) return breakdown("r^.v = 0");
        alpha = rho / rv;
        for (size_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        if (norm2(s) / nf <= prm.rtol) {
            for (size_t i = 0; i < n; ++i) x[i] += alpha * ph[i];
            if (settle()) {
                info->converged = 1;
                break;
            }
            continue;
        }
        vcycle(h, s.data(), sh.data());
        spmv(A, sh.data(), t.data());
        const double tt = dot(t, t);
        if (tt == 0.0 || !std::isfinite(tt)) return breakdown("t.t = 0");
        omega = dot(t, s) / tt;
        for (size_t i = 0; i < n; ++i) x[i] = x[i] + alpha * ph[i] + omega * sh[i];
        for (size_t i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
        rho_prev = rho;
        if (norm2(r) / nf <= prm.rtol) {
            if (settle()) {
                info->converged = 1;
                break;
            }
            continue;
        }
        if (omega == 0.0 || !std::isfinite(omega)) return breakdown("omega = 0");
    }
    if (!info->converged) {
        residual(A, f.data(), x.data(), r.data());
        res = norm2(r) / nf;
    }
    info->iters = it;
    info->rel_res_true = res;
    std::copy(x.begin(), x.end(), uin);
    return ORA_OK;
}

Csr make_csr(int32_t n_rows, int32_t n_cols, const int32_t* ptr, const int32_t* col, const double* val) {
    Csr A;
    A.n_rows = n_rows;
    A.n_cols = n_cols;
    A.ptr.assign(ptr, ptr + n_rows + 1);
    int64_t nnz = ptr[n_rows];
    A.col.assign(col, col + nnz);
    A.val.assign(val, val + nnz);
    return A;
}

/* ------------------------------------------- differentiable 7-point log-coefficients */

/* Face coefficient between cells with k = e^theta: harmonic mean 2 k_a k_b / (k_a + k_b);
 * a boundary face (ghost with the cell's own k) contributes k_a. */
inline double harm(double ka, double kb) { return 2.0 * ka * kb / (ka + kb); }

void neighbours7(int nx, int ny, int nz, int64_t c, int64_t nb[6], int& cnt) {
    int64_t x = c % nx, y = (c / nx) % ny, z = c / ((int64_t)nx * ny);
    cnt = 0;
    if (z > 0) nb[cnt++] = c - (int64_t)nx * ny;
    if (y > 0) nb[cnt++] = c - nx;
    if (x > 0) nb[cnt++] = c - 1;
    if (x < nx - 1) nb[cnt++] = c + 1;
    if (y < ny - 1) nb[cnt++] = c + nx;
    if (z < nz - 1) nb[cnt++] = c + (int64_t)nx * ny;
}

}  // namespace

/* ------------------------------------------------------------------ rebuild policy */

enum { MODE_PARTIAL = 0, MODE_FULL = 1, MODE_OPERATOR_ONLY = 2 };

/* Which update the next time step gets.  Algorithm 3 (full reuse) keeps the hierarchy
 * while the last solve converged within the iteration limit and rebuilds it otherwise.
 * Section 3 lets partial reuse rebuild from time to time as well: regularly, as the every-th
 * update after the last full build, or on a convergence criterion, here the last solve
 * needing more than growth times the iterations of the first solve after that build.
 * base is the update used when nothing asks for a rebuild (partial or operator only). */
int policy_mode(int base, int every, double growth, const History& hs) {
    if (base == MODE_OPERATOR_ONLY && hs.last_iters > 0 && !hs.last_converged) return MODE_FULL;
    if (every > 0 && hs.updates + 1 >= every) return MODE_FULL;
    if (growth > 0.0 && hs.iters_ref > 0 && hs.last_iters > 0 && (double)hs.last_iters > growth * (double)hs.iters_ref)
        return MODE_FULL;
    return base;
}

/* The solve's outcome enters the history (a failed solve counts as maxiter, unconverged). */
void record_solve(Hierarchy& h, int status, const ora_info& info) {
    History& hs = h.hist;
    hs.last_iters = status == ORA_OK ? std::max(info.iters, 1) : std::max(h.prm.maxiter, 1);
    hs.last_converged = status == ORA_OK ? info.converged : 0;
    if (hs.iters_ref == 0 && status == ORA_OK) hs.iters_ref = hs.last_iters;
}

/* =============================================================== exported interface */
extern "C" {

const char* ora_last_error(void) { return g_err.c_str(); }

uint64_t ora_mix64(uint64_t z) { return mix64(z); }

void ora_params_default(ora_params* p) {
    p->smoother = 0;
    p->aggregation = 0;
    p->jacobi_omega = 0.72;
    p->eps_strong = 0.08;
    p->coarse_enough = 1024;
    p->max_levels = 12;
    p->npre = 1;
    p->npost = 1;
    p->rtol = 1e-8;
    p->maxiter = 100;
    p->flexible_cg = 0;
    p->block_size = 1;
}

int ora_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* Strength flags and aggregates of one matrix (no hierarchy). */
int ora_aggregate(int32_t n, const int32_t* ptr, const int32_t* col, const double* val, double eps,
                  uint8_t* strong_out, int32_t* agg_out, int32_t* nc_out) {
    try {
        Csr A = make_csr(n, n, ptr, col, val);
        std::vector<int64_t> dpos, tpos;
        int st = check_matrix(A, dpos, tpos);
        if (st) return st;
        std::vector<uint8_t> strong;
        strength(A, eps, dpos, tpos, strong);
        std::vector<int32_t> agg;
        int32_t nc = 0;
        st = aggregate(A, strong, tpos, agg, nc);
        if (st) return st;
        if (strong_out) std::copy(strong.begin(), strong.end(), strong_out);
        if (agg_out) std::copy(agg.begin(), agg.end(), agg_out);
        *nc_out = nc;
        return ORA_OK;
    } catch (const std::bad_alloc&) {
        return fail(ORA_ERR_OOM, "out of memory");
    }
}

int ora_setup(void** out, int32_t n, const int32_t* ptr, const int32_t* col, const double* val,
              const ora_params* p) {
    *out = nullptr;
    if (n <= 0 || !ptr || !col || !val || !p) return fail(ORA_ERR_ARG, "bad argument");
    Hierarchy* h = new (std::nothrow) Hierarchy();
    if (!h) return fail(ORA_ERR_OOM, "out of memory");
    h->prm = *p;
    int st;
    try {
        st = setup(*h, make_csr(n, n, ptr, col, val));
    } catch (const std::bad_alloc&) {
        st = fail(ORA_ERR_OOM, "out of memory");
    }
    *out = h;  // kept on error too, so that the levels built so far can be inspected
    return st;
}

/* Hierarchy with prescribed transfer operators: level l uses P_l (n_l x nc[l]) for
 * l < nlev; the level reached after them is the coarsest. */
int ora_setup_transfer(void** out, int32_t n, const int32_t* ptr, const int32_t* col, const double* val,
                       int nlev, const int32_t* const* P_ptr, const int32_t* const* P_col,
                       const double* const* P_val, const int32_t* nc, const ora_params* p) {
    *out = nullptr;
    if (n <= 0 || nlev < 0 || !p) return fail(ORA_ERR_ARG, "bad argument");
    Hierarchy* h = new (std::nothrow) Hierarchy();
    if (!h) return fail(ORA_ERR_OOM, "out of memory");
    h->prm = *p;
    h->transfer_given = true;
    *out = h;
    try {
        h->lv.emplace_back();
        h->lv[0].A = make_csr(n, n, ptr, col, val);
        h->A_outer = h->lv[0].A;
        for (int l = 0; l < nlev; ++l) {
            Level& cur = h->lv[(size_t)l];
            std::vector<int64_t> dpos, tpos;
            int st = check_matrix(cur.A, dpos, tpos);
            if (st) return st;
            cur.P = make_csr(cur.A.n_rows, nc[l], P_ptr[l], P_col[l], P_val[l]);
            cur.R = transpose(cur.P);
            Csr AP = spgemm(cur.A, cur.P);
            Csr Ac = spgemm(cur.R, AP);
            h->lv.emplace_back();
            h->lv.back().A = std::move(Ac);
        }
        return finish_levels(*h);
    } catch (const std::bad_alloc&) {
        return fail(ORA_ERR_OOM, "out of memory");
    }
}

/* mode 0: partial reuse (Alg. 4); 1: full rebuild (Alg. 1); 2: operator only (Alg. 3). */
int ora_rebuild(void* hp, const double* val, int mode) {
    Hierarchy* h = (Hierarchy*)hp;
    if (!h || !val) return fail(ORA_ERR_ARG, "bad argument");
    try {
        if (mode == MODE_PARTIAL) {
            int st = partial_rebuild(*h, val);
            if (st == ORA_OK) ++h->hist.updates;
            return st;
        }
        if (mode == MODE_FULL) {
            if (h->transfer_given) return fail(ORA_ERR_ARG, "full rebuild of a prescribed-transfer hierarchy");
            Csr A = h->A_outer;
            std::copy(val, val + A.nnz(), A.val.begin());
            return setup(*h, A);
        }
        if (mode == MODE_OPERATOR_ONLY) {
            std::copy(val, val + h->A_outer.nnz(), h->A_outer.val.begin());
            ++h->hist.updates;
            return ORA_OK;
        }
    } catch (const std::bad_alloc&) {
        return fail(ORA_ERR_OOM, "out of memory");
    }
    return fail(ORA_ERR_ARG, "unknown rebuild mode");
}

/* The update the rebuild policy (base, every, growth; see policy_mode) picks from h's
 * history, applied with new values; *taken receives the mode. */
int ora_rebuild_auto(void* hp, const double* val, int base, int every, double growth, int* taken) {
    Hierarchy* h = (Hierarchy*)hp;
    if (!h || !val || (base != MODE_PARTIAL && base != MODE_OPERATOR_ONLY) || every < 0 || !(growth >= 0.0))
        return fail(ORA_ERR_ARG, "bad argument");
    const int m = policy_mode(base, every, growth, h->hist);
    if (taken) *taken = m;
    return ora_rebuild(hp, val, m);
}

int ora_solve(void* hp, const double* f, double* u, ora_info* info) {
    Hierarchy* h = (Hierarchy*)hp;
    if (!h || !f || !u || !info) return fail(ORA_ERR_ARG, "bad argument");
    int st = pcg(*h, f, u, info);
    record_solve(*h, st, *info);
    return st;
}

int ora_solve_bicgstab(void* hp, const double* f, double* u, ora_info* info) {
    Hierarchy* h = (Hierarchy*)hp;
    if (!h || !f || !u || !info) return fail(ORA_ERR_ARG, "bad argument");
    int st = bicgstab(*h, f, u, info);
    record_solve(*h, st, *info);
    return st;
}

int ora_vcycle(void* hp, const double* r, double* z) {
    Hierarchy* h = (Hierarchy*)hp;
    if (!h || !r || !z) return fail(ORA_ERR_ARG, "bad argument");
    vcycle(*h, r, z);
    return ORA_OK;
}

int ora_num_levels(void* hp) { return hp ? (int)((Hierarchy*)hp)->lv.size() : 0; }

/* dims = {n_l, nnz(A_l), n_{l+1} (0 on the coarsest), nnz(P_l)} */
int ora_level_dims(void* hp, int l, int64_t* dims) {
    Hierarchy* h = (Hierarchy*)hp;
    if (!h || l < 0 || l >= (int)h->lv.size()) return fail(ORA_ERR_ARG, "bad level");
    const Level& L = h->lv[(size_t)l];
    dims[0] = L.A.n_rows;
    dims[1] = L.A.nnz();
    dims[2] = L.P.n_cols;
    dims[3] = L.P.nnz();
    return ORA_OK;
}

/* Copy level l out (any pointer may be NULL).  strong/agg exist only on levels that
 * were aggregated; m only on non-coarsest levels. */
int ora_export_level(void* hp, int l, int32_t* agg, uint8_t* strong, int32_t* A_ptr, int32_t* A_col,
                     double* A_val, int32_t* P_ptr, int32_t* P_col, double* P_val, double* m) {
    Hierarchy* h = (Hierarchy*)hp;
    if (!h || l < 0 || l >= (int)h->lv.size()) return fail(ORA_ERR_ARG, "bad level");
    const Level& L = h->lv[(size_t)l];
    if (agg && !L.agg.empty()) std::copy(L.agg.begin(), L.agg.end(), agg);
    if (strong && !L.strong.empty()) std::copy(L.strong.begin(), L.strong.end(), strong);
    if (A_ptr) std::copy(L.A.ptr.begin(), L.A.ptr.end(), A_ptr);
    if (A_col) std::copy(L.A.col.begin(), L.A.col.end(), A_col);
    if (A_val) std::copy(L.A.val.begin(), L.A.val.end(), A_val);
    if (!L.P.ptr.empty()) {
        if (P_ptr) std::copy(L.P.ptr.begin(), L.P.ptr.end(), P_ptr);
        if (P_col) std::copy(L.P.col.begin(), L.P.col.end(), P_col);
        if (P_val) std::copy(L.P.val.begin(), L.P.val.end(), P_val);
    }
    if (m && !L.m.empty()) std::copy(L.m.begin(), L.m.end(), m);
    return ORA_OK;
}

/* Values of the outer (Krylov) operator. */
int ora_export_outer(void* hp, double* val) {
    Hierarchy* h = (Hierarchy*)hp;
    if (!h || !val) return fail(ORA_ERR_ARG, "bad argument");
    std::copy(h->A_outer.val.begin(), h->A_outer.val.end(), val);
    return ORA_OK;
}

/* Dense Cholesky factor of the coarsest operator (n_L x n_L, row-major). */
int ora_export_coarse_factor(void* hp, double* L) {
    Hierarchy* h = (Hierarchy*)hp;
    if (!h || !L) return fail(ORA_ERR_ARG, "bad argument");
    std::copy(h->L.begin(), h->L.end(), L);
    return ORA_OK;
}

void ora_destroy(void* hp) { delete (Hierarchy*)hp; }

/* Values of the 7-point operator A(theta) on the (sorted) 7-point pattern: face
 * coefficients are harmonic means of k = e^theta, boundary faces add k_c. */
int ora_assemble_logcoef7(int nx, int ny, int nz, const double* theta, double* val) {
    const int64_t n = (int64_t)nx * ny * nz;
    std::vector<double> k((size_t)n);
    for (int64_t c = 0; c < n; ++c) k[c] = std::exp(theta[c]);
    int64_t pos = 0;
    for (int64_t c = 0; c < n; ++c) {
        int64_t nb[6];
        int cnt;
        neighbours7(nx, ny, nz, c, nb, cnt);
        double diag = 0.0;
        int64_t diag_pos = -1;
        for (int q = 0; q < cnt; ++q) {
            if (nb[q] > c && diag_pos < 0) {
                diag_pos = pos++;
            }
            double w = harm(k[c], k[nb[q]]);
            val[pos++] = -w;
            diag += w;
        }
        if (diag_pos < 0) diag_pos = pos++;
        diag += (6 - cnt) * k[c];
        val[diag_pos] = diag;
    }
    return ORA_OK;
}

/* Gradient of L(u(theta)) with respect to theta, given u = A(theta)^-1 f and the adjoint
 * lambda = A^-1 dL/du:  g_c = -lambda^T (dA/dtheta_c) u, i.e.
 *   g_c = - sum_{faces (c,j)} [2 k_c k_j^2 / (k_c + k_j)^2] (lambda_c - lambda_j)(u_c - u_j)
 *         - (number of boundary faces of c) * k_c * lambda_c * u_c. */
int ora_adjoint_logcoef7(int nx, int ny, int nz, const double* theta, const double* u, const double* lam,
                         double* grad) {
    const int64_t n = (int64_t)nx * ny * nz;
    for (int64_t c = 0; c < n; ++c) {
        int64_t nb[6];
        int cnt;
        neighbours7(nx, ny, nz, c, nb, cnt);
        double kc = std::exp(theta[c]);
        double g = 0.0;
        for (int q = 0; q < cnt; ++q) {
            double kj = std::exp(theta[nb[q]]);
            double dw = 2.0 * kc * kj * kj / ((kc + kj) * (kc + kj));
            g -= dw * (lam[c] - lam[nb[q]]) * (u[c] - u[nb[q]]);
        }
        g -= (6 - cnt) * kc * lam[c] * u[c];
        grad[c] = g;
    }
    return ORA_OK;
}

}  // extern "C"
