// Driver for a sanitizer build of the oracle (test infrastructure, like the oracle itself):
// every entry point of amg_oracle.cpp runs on small ragged problems -- setup, the three
// update modes and the rebuild policy, CG and BiCGStab, the V-cycle, exports, prescribed
// transfer operators, plain aggregation with SPAI0, a system of 2 x 2 blocks, the
// log-coefficient assembly and its adjoint, and argument errors -- so that AddressSanitizer
// and UndefinedBehaviorSanitizer see each code path once.  Exit status 0 when every call
// returned what it should.
//
// Build (tests/test_oracle_sanitize.py):
//   g++ -std=c++17 -O1 -g -fsanitize=address,undefined -fno-sanitize-recover=all
//       -fno-omit-frame-pointer oracle/amg_oracle.cpp oracle/sanitize_main.cpp -o ora_san
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
typedef struct {
    int smoother;
    int aggregation;
    double jacobi_omega;
    double eps_strong;
    int coarse_enough;
    int max_levels;
    int npre, npost;
    double rtol;
    int maxiter;
    int flexible_cg;
    int block_size;
} ora_params;

typedef struct {
    int iters;
    int converged;
    double rel_res_true;
} ora_info;

const char* ora_last_error(void);
void ora_params_default(ora_params* p);
int ora_aggregate(int32_t n, const int32_t* ptr, const int32_t* col, const double* val, double eps,
                  uint8_t* strong_out, int32_t* agg_out, int32_t* nc_out);
int ora_setup(void** out, int32_t n, const int32_t* ptr, const int32_t* col, const double* val, const ora_params* p);
int ora_setup_transfer(void** out, int32_t n, const int32_t* ptr, const int32_t* col, const double* val, int nlev,
                       const int32_t* const* P_ptr, const int32_t* const* P_col, const double* const* P_val,
                       const int32_t* nc, const ora_params* p);
int ora_rebuild(void* hp, const double* val, int mode);
int ora_rebuild_auto(void* hp, const double* val, int base, int every, double growth, int* taken);
int ora_solve(void* hp, const double* f, double* u, ora_info* info);
int ora_solve_bicgstab(void* hp, const double* f, double* u, ora_info* info);
int ora_vcycle(void* hp, const double* r, double* z);
int ora_num_levels(void* hp);
int ora_level_dims(void* hp, int l, int64_t* dims);
int ora_export_level(void* hp, int l, int32_t* agg, uint8_t* strong, int32_t* A_ptr, int32_t* A_col, double* A_val,
                     int32_t* P_ptr, int32_t* P_col, double* P_val, double* m);
int ora_export_outer(void* hp, double* val);
int ora_export_coarse_factor(void* hp, double* L);
void ora_destroy(void* hp);
int ora_assemble_logcoef7(int nx, int ny, int nz, const double* theta, double* val);
int ora_adjoint_logcoef7(int nx, int ny, int nz, const double* theta, const double* u, const double* lam,
                         double* grad);
}

namespace {

int failures = 0;

void check(bool ok, const char* what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (%s)\n", what, ora_last_error());
        ++failures;
    }
}

struct Csr {
    std::vector<int32_t> ptr, col;
    std::vector<double> val;
    int32_t n() const { return (int32_t)ptr.size() - 1; }
};

// 7-point operator on nx x ny x nz cells: face weights w(x, y, z) of a two-valued
// coefficient (a heavy block in one corner), Dirichlet closure on the boundary, optionally
// a first-order upwind convection term (non-symmetric values).
Csr poisson7(int nx, int ny, int nz, double heavy, double conv) {
    Csr A;
    A.ptr.push_back(0);
    auto coef = [&](int x, int y, int z) { return (x < nx / 2 && z < nz / 2) ? 1.0 / heavy : 1.0; };
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int i = (z * ny + y) * nx + x;
                const int dx[6] = {0, 0, 0, 0, -1, 1}, dy[6] = {0, 0, -1, 1, 0, 0}, dz[6] = {-1, 1, 0, 0, 0, 0};
                double diag = 0.0;
                std::vector<std::pair<int, double>> row;
                for (int k = 0; k < 6; ++k) {
                    const int X = x + dx[k], Y = y + dy[k], Z = z + dz[k];
                    const double ci = coef(x, y, z);
                    if (X < 0 || Y < 0 || Z < 0 || X >= nx || Y >= ny || Z >= nz) {
                        diag += 2.0 * ci;
                        continue;
                    }
                    const double cj = coef(X, Y, Z);
                    const double w = 2.0 / (1.0 / ci + 1.0 / cj);
                    const double up = (k == 4) ? conv : 0.0;  // flow in +x: upwind neighbour x - 1
                    diag += w + up;
                    row.push_back({(Z * ny + Y) * nx + X, -w - up});
                }
                row.push_back({i, diag});
                for (size_t a = 0; a < row.size(); ++a)
                    for (size_t b = a + 1; b < row.size(); ++b)
                        if (row[b].first < row[a].first) std::swap(row[a], row[b]);
                for (auto& e : row) {
                    A.col.push_back(e.first);
                    A.val.push_back(e.second);
                }
                A.ptr.push_back((int32_t)A.col.size());
            }
    return A;
}

// L (x) K for an SPD 2 x 2 K: the node-major system of 2 x 2 blocks.
Csr kron2(const Csr& L, const double K[4]) {
    Csr A;
    A.ptr.push_back(0);
    for (int32_t I = 0; I < L.n(); ++I)
        for (int b = 0; b < 2; ++b) {
            for (int32_t k = L.ptr[I]; k < L.ptr[I + 1]; ++k)
                for (int c = 0; c < 2; ++c) {
                    A.col.push_back(L.col[k] * 2 + c);
                    A.val.push_back(L.val[k] * K[b * 2 + c]);
                }
            A.ptr.push_back((int32_t)A.col.size());
        }
    return A;
}

std::vector<double> rhs(int32_t n, uint64_t seed) {
    std::vector<double> f(n);
    for (int32_t i = 0; i < n; ++i) {
        seed = seed * 6364136223846793005ULL + 1442695040888963407ULL;
        f[i] = (double)(seed >> 11) / 9007199254740992.0 - 0.5;
    }
    return f;
}

void solve_all(void* h, int32_t n, bool bicgstab, const char* what) {
    const std::vector<double> f = rhs(n, 7);
    std::vector<double> u(n, 0.0), z(n);
    ora_info info{};
    check(ora_solve(h, f.data(), u.data(), &info) == 0 && info.converged == 1, what);
    check(ora_vcycle(h, f.data(), z.data()) == 0, what);
    if (bicgstab) {
        std::fill(u.begin(), u.end(), 0.0);
        check(ora_solve_bicgstab(h, f.data(), u.data(), &info) == 0 && info.converged == 1, what);
    }
}

void exports(void* h) {
    const int L = ora_num_levels(h);
    check(L >= 2, "several levels");
    for (int l = 0; l < L; ++l) {
        int64_t d[4];
        check(ora_level_dims(h, l, d) == 0, "level dims");
        std::vector<int32_t> agg(d[0]), Ap(d[0] + 1), Ac(d[1]), Pp(d[0] + 1), Pc(d[3] > 0 ? d[3] : 1);
        std::vector<uint8_t> strong(d[1]);
        std::vector<double> Av(d[1]), Pv(d[3] > 0 ? d[3] : 1), m(d[0]);
        const bool coarsest = l == L - 1;
        check(ora_export_level(h, l, agg.data(), strong.data(), Ap.data(), Ac.data(), Av.data(),
                               coarsest ? nullptr : Pp.data(), coarsest ? nullptr : Pc.data(),
                               coarsest ? nullptr : Pv.data(), coarsest ? nullptr : m.data()) == 0,
              "export level");
    }
    int64_t d[4];
    ora_level_dims(h, L - 1, d);
    std::vector<double> Lf(d[0] * d[0]);
    check(ora_export_coarse_factor(h, Lf.data()) == 0, "export coarse factor");
    int64_t d0[4];
    ora_level_dims(h, 0, d0);
    std::vector<double> outer(d0[1]);
    check(ora_export_outer(h, outer.data()) == 0, "export outer");
}

}  // namespace

int main() {
    ora_params p;
    ora_params_default(&p);
    p.coarse_enough = 24;

    // smoothed aggregation, damped Jacobi: setup, the three update modes, the policy
    const Csr A = poisson7(9, 7, 6, 1000.0, 0.0);
    const int32_t n = A.n();
    void* h = nullptr;
    check(ora_setup(&h, n, A.ptr.data(), A.col.data(), A.val.data(), &p) == 0, "setup");
    std::vector<double> v2(A.val);
    for (double& x : v2) x *= 1.5;
    check(ora_rebuild(h, v2.data(), 0) == 0, "partial update");
    solve_all(h, n, true, "solve after a partial update");
    check(ora_rebuild(h, A.val.data(), 2) == 0, "operator-only update");
    solve_all(h, n, false, "solve after an operator-only update");
    check(ora_rebuild(h, v2.data(), 1) == 0, "full update");
    exports(h);
    int taken = -1;
    for (int t = 0; t < 4; ++t) {
        check(ora_rebuild_auto(h, (t & 1) ? A.val.data() : v2.data(), 0, 3, 2.0, &taken) == 0, "policy update");
        solve_all(h, n, false, "solve under the policy");
    }
    check(ora_rebuild_auto(h, v2.data(), 2, 0, 0.0, &taken) == 0, "policy, full reuse");

    // prescribed transfer operators: level 0's P of this hierarchy
    {
        int64_t d[4];
        ora_level_dims(h, 0, d);
        std::vector<int32_t> agg(d[0]), Ap(d[0] + 1), Ac(d[1]), Pp(d[0] + 1), Pc(d[3]);
        std::vector<uint8_t> strong(d[1]);
        std::vector<double> Av(d[1]), Pv(d[3]), m(d[0]);
        ora_export_level(h, 0, agg.data(), strong.data(), Ap.data(), Ac.data(), Av.data(), Pp.data(), Pc.data(),
                         Pv.data(), m.data());
        const int32_t* pp[1] = {Pp.data()};
        const int32_t* pc[1] = {Pc.data()};
        const double* pv[1] = {Pv.data()};
        const int32_t nc[1] = {(int32_t)d[2]};
        void* ht = nullptr;
        check(ora_setup_transfer(&ht, n, A.ptr.data(), A.col.data(), A.val.data(), 1, pp, pc, pv, nc, &p) == 0,
              "setup with prescribed transfer operators");
        if (ht) {
            solve_all(ht, n, false, "solve with prescribed transfer operators");
            ora_destroy(ht);
        }
    }
    ora_destroy(h);

    // non-symmetric values (BiCGStab), plain aggregation with SPAI0, flexible CG
    {
        const Csr B = poisson7(8, 8, 5, 10.0, 0.3);
        ora_params q = p;
        q.aggregation = 1;
        q.smoother = 1;
        void* hb = nullptr;
        check(ora_setup(&hb, B.n(), B.ptr.data(), B.col.data(), B.val.data(), &q) == 0, "setup, non-symmetric");
        if (hb) {
            const std::vector<double> f = rhs(B.n(), 3);
            std::vector<double> u(B.n(), 0.0);
            ora_info info{};
            check(ora_solve_bicgstab(hb, f.data(), u.data(), &info) == 0 && info.converged == 1, "BiCGStab");
            ora_destroy(hb);
        }
        q = p;
        q.flexible_cg = 1;
        check(ora_setup(&hb, n, A.ptr.data(), A.col.data(), A.val.data(), &q) == 0, "setup, flexible CG");
        if (hb) {
            solve_all(hb, n, false, "flexible CG");
            ora_destroy(hb);
        }
    }

    // a system of 2 x 2 blocks: node aggregation, block Jacobi
    {
        const Csr Ls = poisson7(6, 5, 5, 1.0, 0.0);
        const double K[4] = {2.0, 0.5, 0.5, 1.0};
        const Csr B = kron2(Ls, K);
        ora_params q = p;
        q.aggregation = 1;
        q.block_size = 2;
        void* hb = nullptr;
        check(ora_setup(&hb, B.n(), B.ptr.data(), B.col.data(), B.val.data(), &q) == 0, "setup, 2 x 2 blocks");
        if (hb) {
            std::vector<double> vb(B.val);
            for (double& x : vb) x *= 0.75;
            check(ora_rebuild(hb, vb.data(), 0) == 0, "partial update, blocks");
            solve_all(hb, B.n(), false, "solve, blocks");
            ora_destroy(hb);
        }
    }

    // aggregation on its own
    {
        std::vector<uint8_t> strong(A.col.size());
        std::vector<int32_t> agg(n);
        int32_t nc = 0;
        check(ora_aggregate(n, A.ptr.data(), A.col.data(), A.val.data(), 0.08, strong.data(), agg.data(), &nc) == 0 &&
                  nc > 0 && nc < n,
              "aggregate");
    }

    // log-coefficient assembly and its adjoint
    {
        const int nx = 5, ny = 4, nz = 3, m = nx * ny * nz;
        std::vector<double> theta = rhs(m, 11);
        std::vector<double> val(7 * (size_t)m, 0.0);
        check(ora_assemble_logcoef7(nx, ny, nz, theta.data(), val.data()) == 0, "assemble log-coefficient");
        std::vector<double> u = rhs(m, 12), lam = rhs(m, 13), g(m);
        check(ora_adjoint_logcoef7(nx, ny, nz, theta.data(), u.data(), lam.data(), g.data()) == 0, "adjoint");
    }

    // argument errors return codes, not faults
    {
        void* hb = nullptr;
        check(ora_setup(&hb, n, nullptr, A.col.data(), A.val.data(), &p) != 0, "setup without row pointers");
        check(ora_rebuild(nullptr, A.val.data(), 0) != 0, "update without a hierarchy");
        check(ora_rebuild_auto(nullptr, A.val.data(), 0, 0, 0.0, nullptr) != 0, "policy without a hierarchy");
        ora_info info{};
        check(ora_solve(nullptr, nullptr, nullptr, &info) != 0, "solve without a hierarchy");
        Csr bad = A;
        std::swap(bad.col[1], bad.col[2]);
        check(ora_setup(&hb, n, bad.ptr.data(), bad.col.data(), bad.val.data(), &p) != 0, "unsorted columns");
        if (hb) ora_destroy(hb);  // kept on error for inspection; the caller frees it
    }

    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("oracle sanitizer run: all checks passed\n");
    return 0;
}
