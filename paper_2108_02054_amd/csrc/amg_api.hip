// amg_api.hip -- hierarchy manager, update strategies, V-cycle / PCG orchestration, and
// the exported C interface declared in include/amg.h.
//
// Strategies (Section 3 of the paper):
//   full rebuild   (Algorithm 1)  build_hierarchy(): aggregation, P, R, patterns, values
//   partial reuse  (Algorithm 4)  partial_rebuild(): numeric Galerkin chain on the cached
//                                 patterns, smoothers, coarse inverse; no host sync
//   full reuse     (Algorithm 3)  only the Krylov operator's values change
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <utility>
#include <vector>

#include "amg_internal.h"

using namespace amgmi;

namespace amgmi {

[[noreturn]] void throw_hip(hipError_t e, const char* expr, const char* file, int line) {
    (void)hipGetLastError();  // consume the error so later launch checks do not report it again
    const amg_status st = (e == hipErrorOutOfMemory) ? AMG_ERR_OOM : AMG_ERR_HIP;
    throw Fail{st, std::string(hipGetErrorString(e)) + " in " + expr + " (" + file + ":" + std::to_string(line) + ")"};
}

namespace {
thread_local DevMem* g_mem = nullptr;

// Contexts that own a private pool, so that an allocation that fails can have the kept
// blocks of every context handed back before it gives up.
std::mutex g_mems_mu;
std::vector<DevMem*> g_mems;

size_t block_class(size_t b) {
    if (b <= 4096) return (b + 255) & ~(size_t)255;
    const int e = 63 - __builtin_clzll((unsigned long long)b);  // 2^e <= b < 2^(e+1)
    const size_t step = (size_t)1 << (e - 3);
    return (b + step - 1) & ~(step - 1);
}

// Kept blocks of m back to its pool (caller holds m.mu).
void flush_kept(DevMem& m) {
    for (auto& kv : m.kept)
        for (void* p : kv.second) (void)hipFreeAsync(p, m.s);
    m.kept.clear();
    m.kept_bytes = 0;
}

hipError_t pool_alloc(DevMem& m, void** p, size_t bytes) {
    return m.pool ? hipMallocFromPoolAsync(p, bytes, m.pool, m.s) : hipMallocAsync(p, bytes, m.s);
}

// After a failed allocation: the kept blocks of this context, then of every context, go
// back to their pools and the pools release what no allocation uses.
bool reclaim(DevMem& m, int round) {
    if (round == 0) {
        {
            std::lock_guard<std::mutex> lk(m.mu);
            flush_kept(m);
        }
        (void)hipStreamSynchronize(m.s);
        if (m.pool) (void)hipMemPoolTrimTo(m.pool, 0);
        return true;
    }
    if (round == 1) {
        std::lock_guard<std::mutex> g(g_mems_mu);
        for (DevMem* o : g_mems) {
            if (o == &m) continue;
            std::lock_guard<std::mutex> lk(o->mu);
            flush_kept(*o);
        }
        (void)hipDeviceSynchronize();
        for (DevMem* o : g_mems)
            if (o->pool) (void)hipMemPoolTrimTo(o->pool, 0);
        return true;
    }
    return false;
}
}  // namespace

MemScope::MemScope(DevMem* m) : prev(g_mem) { g_mem = m; }
MemScope::~MemScope() { g_mem = prev; }

void mem_init(DevMem& m, hipStream_t s, void* (*a)(size_t, void*, void*), void (*f)(void*, size_t, void*, void*),
              void* user) {
    m.s = s;
    m.hook_alloc = a;
    m.hook_free = f;
    m.hook_user = user;
    if (a) return;
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    if (hipMemPoolCreate(&m.pool, &props) != hipSuccess) {  // the default pool then, as it is
        (void)hipGetLastError();
        m.pool = nullptr;
    } else {
        uint64_t keep = UINT64_MAX;
        HIP_CHECK(hipMemPoolSetAttribute(m.pool, hipMemPoolAttrReleaseThreshold, &keep));
    }
    std::lock_guard<std::mutex> g(g_mems_mu);
    g_mems.push_back(&m);
}

void mem_release(DevMem& m) {
    {
        std::lock_guard<std::mutex> g(g_mems_mu);
        g_mems.erase(std::remove(g_mems.begin(), g_mems.end(), &m), g_mems.end());
    }
    {
        std::lock_guard<std::mutex> lk(m.mu);
        flush_kept(m);
        if (!m.hook_free)
            for (auto& kv : m.live) (void)hipFreeAsync(kv.first, m.s);
        else
            for (auto& kv : m.live) m.hook_free(kv.first, kv.second, (void*)m.s, m.hook_user);
        m.live.clear();
        m.live_bytes = 0;
    }
    (void)hipStreamSynchronize(m.s);
    if (m.pool) {
        (void)hipMemPoolDestroy(m.pool);
        m.pool = nullptr;
    }
}

void* dalloc(size_t bytes, hipStream_t s) {
    DevMem* m = g_mem;
    if (bytes == 0) bytes = 8;
    if (!m) {
        void* p = nullptr;
        hipError_t e = hipMallocAsync(&p, bytes, s);
        if (e == hipErrorOutOfMemory) {
            (void)hipGetLastError();
            throw Fail{AMG_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
        }
        if (e != hipSuccess) throw_hip(e, "hipMallocAsync", __FILE__, __LINE__);
        return p;
    }
    if (m->hook_alloc) {
        void* p = m->hook_alloc(bytes, (void*)m->s, m->hook_user);
        if (!p) throw Fail{AMG_ERR_OOM, "the caller's allocator returned no block of " + std::to_string(bytes) + " bytes"};
        std::lock_guard<std::mutex> lk(m->mu);
        m->live.emplace(p, bytes);
        m->live_bytes += bytes;
        m->peak_bytes = std::max(m->peak_bytes, m->live_bytes);
        return p;
    }
    bytes = block_class(bytes);
    {
        std::lock_guard<std::mutex> lk(m->mu);
        auto it = m->kept.find(bytes);
        if (it != m->kept.end() && !it->second.empty()) {
            void* p = it->second.back();
            it->second.pop_back();
            m->kept_bytes -= bytes;
            m->live.emplace(p, bytes);
            m->live_bytes += bytes;
            m->peak_bytes = std::max(m->peak_bytes, m->live_bytes);
            return p;
        }
    }
    void* p = nullptr;
    hipError_t e = pool_alloc(*m, &p, bytes);
    for (int round = 0; e == hipErrorOutOfMemory && reclaim(*m, round); ++round) {
        (void)hipGetLastError();
        e = pool_alloc(*m, &p, bytes);
    }
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        throw Fail{AMG_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
    }
    if (e != hipSuccess) throw_hip(e, "hipMallocFromPoolAsync", __FILE__, __LINE__);
    std::lock_guard<std::mutex> lk(m->mu);
    m->live.emplace(p, bytes);
    m->live_bytes += bytes;
    m->peak_bytes = std::max(m->peak_bytes, m->live_bytes);
    return p;
}

void dfree(void* p, hipStream_t s) {
    if (!p) return;
    DevMem* m = g_mem;
    if (!m) {
        (void)hipFreeAsync(p, s);
        return;
    }
    std::lock_guard<std::mutex> lk(m->mu);
    auto it = m->live.find(p);
    if (it == m->live.end()) {  // not this context's block (not expected)
        (void)hipFreeAsync(p, s);
        return;
    }
    const size_t bytes = it->second;
    m->live.erase(it);
    m->live_bytes -= bytes;
    if (m->hook_free) {
        m->hook_free(p, bytes, (void*)m->s, m->hook_user);
        return;
    }
    // keep it for the next allocation of its class on this context's stream, within the
    // context's own peak working set
    if (m->live_bytes + m->kept_bytes + bytes > m->peak_bytes) flush_kept(*m);
    m->kept[bytes].push_back(p);
    m->kept_bytes += bytes;
}

// Temporaries of one setup step, released when the step ends or throws.
struct Temps {
    hipStream_t s;
    std::vector<void*> v;
    explicit Temps(hipStream_t st) : s(st) {}
    Temps(const Temps&) = delete;
    Temps& operator=(const Temps&) = delete;
    template <typename T>
    T* add(T* p) {
        v.push_back((void*)p);
        return p;
    }
    template <typename T>
    T* make(size_t n) {
        return add(dnew<T>(n, s));
    }
    ~Temps() {
        for (void* p : v) dfree(p, s);
    }
};

int lane_group(double avg) {
    int g = 2;
    while (g < 64 && g < avg) g <<= 1;
    return g;
}

// Largest power-of-two rows per block (<= RB_THREADS) whose blocks never hold more than
// RB_CAP nonzeros; 0 when a single row is longer than that.
int pick_rows_per_block(const int32_t* p, int32_t n) {
    for (int rpb = RB_THREADS; rpb >= 1; rpb >>= 1) {
        int64_t worst = 0;
        for (int64_t r0 = 0; r0 < n; r0 += rpb) {
            const int64_t r1 = r0 + rpb < n ? r0 + rpb : n;
            const int64_t w = (int64_t)p[r1] - p[r0];
            if (w > worst) worst = w;
        }
        if (worst <= RB_CAP) {
            // small matrices: fewer rows per workgroup, so that about RB_MIN_BLOCKS
            // workgroups (four per CU) share the latency of their dependent loads
            while (rpb > 1 && ((int64_t)n + rpb - 1) / rpb < RB_MIN_BLOCKS) rpb >>= 1;
            return rpb;
        }
    }
    return 0;
}

}  // namespace amgmi

namespace {

thread_local std::string g_setup_err;

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// ------------------------------------------------------------------ memory bookkeeping

template <typename T>
T* halloc(amg_ctx* c, size_t n) {
    T* p = dnew<T>(n, c->stream);
    c->hier_allocs.push_back(p);
    return p;
}

template <typename T>
T* oalloc(amg_ctx* c, size_t n) {
    T* p = dnew<T>(n, c->stream);
    c->own_allocs.push_back(p);
    return p;
}

void track(amg_ctx* c, const Csr& m) {
    for (void* p : {(void*)m.ptr, (void*)m.col, (void*)m.val, (void*)m.val32})
        if (p) c->hier_allocs.push_back(p);
}

void release(amg_ctx* c, void* p) {
    if (!p) return;
    for (auto& q : c->hier_allocs)
        if (q == p) {
            q = nullptr;
            dfree(p, c->stream);
            return;
        }
}

void release_csr(amg_ctx* c, Csr& m) {
    release(c, m.ptr);
    release(c, m.col);
    release(c, m.val);
    release(c, m.val32);
    release(c, m.c16);
    release(c, m.cblk);
    m = Csr{};
}

void d2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes) HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
}

bool mixed(const amg_ctx* c) { return c->prm.precision == 1; }

// Brackets the launches inside its scope with events when the class is traced.
struct Trace {
    amg_ctx* c;
    int cls, level;
    hipStream_t ts;  // the stream the bracketing events are recorded on
    hipEvent_t a = nullptr, b = nullptr;
    static hipEvent_t take(amg_ctx* c) {
        if (c->ev_pool.empty()) {
            hipEvent_t e;
            HIP_CHECK(hipEventCreate(&e));
            return e;
        }
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    // Classes whose scope is one kernel launch have the launch record its own events, which
    // time the kernel alone (not the dispatch gap before it, and with no extra commands in
    // the stream); the others (Galerkin products with their smoother, casts, the coarse
    // inverse, BiCGStab's products) are bracketed by events recorded on the stream.
    static bool single_launch(int k) {
        return k == AMG_K_CG_PQ || k == AMG_K_RESTRICT || k == AMG_K_PROLONG || k == AMG_K_JACOBI ||
               k == AMG_K_SMOOTH0_RES || k == AMG_K_CG_UPDATE || k == AMG_K_CG_RZ || k == AMG_K_CG_INIT ||
               k == AMG_K_COARSE_GEMV || k == AMG_K_TAIL;
    }
    bool own = false;
    Trace(amg_ctx* cc, int k, int lvl, hipStream_t st = nullptr) : c(cc), cls(k), level(lvl), ts(st ? st : cc->stream) {
        if (((c->trace_mask >> k) & 1u) && (c->trace_level < 0 || c->trace_level == lvl) && k >= 0 && k < 16 &&
            c->trace_seen[(size_t)k][(size_t)std::min(std::max(lvl, 0), 63)]++ % c->trace_every == 0) {
            a = take(c);
            b = take(c);
            if (single_launch(k)) {
                own = true;
                g_kernel_events = KernelEvents{a, b};
            } else {
                HIP_CHECK(hipEventRecord(a, ts));
            }
        }
    }
    ~Trace() {
        if (!a) return;
        if (!own) {
            (void)hipEventRecord(b, ts);
        } else if (g_kernel_events.start == a) {  // the scope launched nothing: not a launch
            g_kernel_events = KernelEvents{};
            c->ev_pool.push_back(a);
            c->ev_pool.push_back(b);
            return;
        }
        c->traced.push_back({cls, level, a, b});
    }
};

// One device-to-host copy of the scalar slots and the ||r||^2 and ||f||^2 partials.
void read_red(amg_ctx* c) {
    HIP_CHECK(hipMemcpyAsync(c->h_red, c->rs.scal(), RedScratch::host_doubles(c->rs.cap) * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    HIP_CHECK(hipStreamSynchronize(c->stream));
}

// The context's stream waits for the coarsest inverse of the last partial update (run on
// the side stream) before anything on it uses the inverse or its pivot flag.
void wait_coarse(amg_ctx* c) {
    if (!c->cinv_pending) return;
    HIP_CHECK(hipStreamWaitEvent(c->stream, c->ev_inv, 0));
    c->cinv_pending = false;
}

// Queue the copy of the scalar slots and the first nrr ||r||^2 partials (the CG loop's
// per-iteration read).
void queue_read_rr(amg_ctx* c, int nrr) {
    HIP_CHECK(hipMemcpyAsync(c->h_red, c->rs.scal(), (S_COUNT + (size_t)nrr) * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
}

double host_scal(const amg_ctx* c, int k) { return c->h_red[k]; }

// Sum of nb partials of P_RR or P_FF as last copied to the host, in block order.
double host_sum(const amg_ctx* c, int region, int nb) {
    const double* p = c->h_red + S_COUNT + (region == P_RR ? 0 : (size_t)c->rs.cap);
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += p[i];
    return s;
}

void read_flags(amg_ctx* c) {
    HIP_CHECK(hipMemcpyAsync(c->h_flags, c->d_flags, F_COUNT * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_CHECK(hipStreamSynchronize(c->stream));
}

void clear_flags(amg_ctx* c) { HIP_CHECK(hipMemsetAsync(c->d_flags, 0, F_COUNT * sizeof(int), c->stream)); }

// Pattern (and optionally values) checks of a CSR matrix on the device.
void validate(amg_ctx* c, const Csr& A, int32_t* diag_pos, const char* what) {
    clear_flags(c);
    launch_validate(A, diag_pos, c->d_flags, c->stream);
    read_flags(c);
    if (c->h_flags[F_ARG])
        throw Fail{AMG_ERR_ARG, std::string(what) + ": invalid CSR (pointers, unsorted/duplicate/out-of-range columns or non-finite values)"};
    if (c->h_flags[F_NOT_SPD])
        throw Fail{AMG_ERR_NOT_SPD, std::string(what) + ": missing or non-positive diagonal entry"};
}

// Systems with block_size unknowns per node: the pattern of L.A must consist of full blocks
// (AMG_ERR_PATTERN) and its row count be a multiple of the block size (AMG_ERR_ARG); its
// node pattern is kept for the node-group kernels.
void node_pattern(amg_ctx* c, Level& L) {
    release(c, L.nptr);
    release(c, L.ncol);
    L.nptr = L.ncol = nullptr;
    Csr pat = L.A, Nm;
    pat.val = nullptr;
    clear_flags(c);
    build_node_matrix(pat, c->prm.block_size, Nm, c->d_flags, c->h_flags, c->stream);
    L.nptr = Nm.ptr;
    L.ncol = Nm.col;
    L.node_pairs = std::getenv("AMGMI_NO_NODE_PAIRS") == nullptr;
    c->hier_allocs.push_back(L.nptr);
    c->hier_allocs.push_back(L.ncol);
}

// AMGMI_ROW_KERNELS=lanes selects the lane-group kernels everywhere (used by the tests
// to cover both kernel families); the default picks LDS-staged row blocks where they fit.
bool lanes_only() {
    const char* e = std::getenv("AMGMI_ROW_KERNELS");
    return e != nullptr && std::strcmp(e, "lanes") == 0;
}

// Galerkin form override (AMGMI_GALERKIN = pos | pos16 | lanes, optionally ":G" for the
// position-map form's lanes per row and ":G:T" also for its B terms per lane and entry;
// pos16 forces two-byte positions); used to exercise every form and launch shape.
// Default: the shape picker's choice.
struct GalForce {
    int lanes = 0;  // 1: lane-group kernels
    int wide = 0;   // 1: two-byte positions
    int g = 0;
    int t = 0;      // B terms per lane and entry (1 or 2)
};
GalForce galerkin_force() {
    GalForce f;
    const char* e = std::getenv("AMGMI_GALERKIN");
    if (e == nullptr) return f;
    if (std::strncmp(e, "lanes", 5) == 0) f.lanes = 1;
    if (std::strncmp(e, "pos16", 5) == 0) f.wide = 1;
    if (const char* c = std::strchr(e, ':')) {
        f.g = std::atoi(c + 1);
        if (const char* c2 = std::strchr(c + 1, ':')) f.t = std::atoi(c2 + 1);
    }
    return f;
}

// Launch shapes of a matrix's row kernels (reads its row pointers back once), and its
// two-byte column indices for the row-block kernels when every block's columns fit
// (matrices of at least C16_MIN_NNZ entries; AMGMI_NO_C16 keeps int32 everywhere).
constexpr int64_t C16_MIN_NNZ = 1 << 18;
void configure(amg_ctx* c, Csr& A, hipStream_t s) {
    A.g = lane_group(A.nrows > 0 ? (double)A.nnz / A.nrows : 1.0);
    std::vector<int32_t> hp((size_t)A.nrows + 1);
    HIP_CHECK(hipMemcpyAsync(hp.data(), A.ptr, hp.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    A.rpb = lanes_only() ? 0 : pick_rows_per_block(hp.data(), A.nrows);
    release(c, A.c16);
    release(c, A.cblk);
    A.c16 = nullptr;
    A.cblk = nullptr;
    if (A.rpb == 0 || A.nnz < C16_MIN_NNZ || std::getenv("AMGMI_NO_C16") != nullptr) return;
    const int nb = (A.nrows + A.rpb - 1) / A.rpb;
    int32_t* cblk = halloc<int32_t>(c, (size_t)nb);
    clear_flags(c);
    launch_c16_bases(A, cblk, c->d_flags + F_ARG, s);
    read_flags(c);
    if (c->h_flags[F_ARG]) {  // some block spans more than two bytes of columns
        release(c, cblk);
        return;
    }
    A.cblk = cblk;
    A.c16 = halloc<uint16_t>(c, (size_t)A.nnz);
    launch_c16_fill(A, cblk, A.c16, s);
}

template <typename T>
std::vector<T> to_host(const T* d, size_t n, hipStream_t s) {
    std::vector<T> h(n);
    if (n) HIP_CHECK(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    return h;
}

void release_posmap(amg_ctx* c, GalShape& gs) {
    for (void* p : {gs.pos, (void*)gs.off, (void*)gs.bst, (void*)gs.tof, (void*)gs.dpos}) release(c, p);
    gs = GalShape{};
}

void release_posmaps(amg_ctx* c, Level& L) {
    release_posmap(c, L.galAP);
    release_posmap(c, L.galRAP);
}

void release_node_gal(amg_ctx* c, NodeGal& g) {
    for (void* q : {(void*)g.tptr, (void*)g.toff, (void*)g.tlen, (void*)g.cout, (void*)g.clen}) release(c, q);
    g = NodeGal{};
}

// Node transfer maps of a block system, at setup: a level whose P is P_node (x) I_B with
// unit values keeps the aggregate of every node, and its V-cycle prolongation reads that
// map instead of P's row pointers, columns and values.  AMGMI_NO_NODE_TRANSFER keeps the
// CSR prolongation.
void configure_node_transfer(amg_ctx* c) {
    for (Level& L : c->lv) {
        release(c, L.nagg);
        L.nagg = nullptr;
    }
    const int B = c->prm.block_size;
    if (B < 2 || std::getenv("AMGMI_NO_NODE_TRANSFER") != nullptr) return;
    hipStream_t s = c->stream;
    for (size_t l = 0; l + 1 < c->lv.size(); ++l) {
        Level& L = c->lv[l];
        if (L.P.nrows == 0) continue;
        int32_t* nagg = halloc<int32_t>(c, (size_t)std::max(L.A.nrows / B, 1));
        clear_flags(c);
        launch_node_gal_agg(L.P, B, nagg, c->d_flags, s);
        read_flags(c);
        if (c->h_flags[F_NODEGAL]) {
            release(c, nagg);
            continue;
        }
        L.nagg = nagg;
    }
}

// Node Galerkin plans of a block system (every level's node pattern built), formed by the
// first partial update after a setup or a pattern change: a level whose P is
// P_node (x) I_B with unit values gets one, and its partial updates form A_{l+1} in one
// pass over A_l's blocks; other levels (user transfer operators of another form) keep the
// scalar position-map product.  AMGMI_NO_NODE_GAL keeps the scalar product everywhere.
void configure_node_gal(amg_ctx* c) {
    for (Level& L : c->lv) release_node_gal(c, L.ngal);
    const int B = c->prm.block_size;
    if (B < 2 || std::getenv("AMGMI_NO_NODE_GAL") != nullptr) return;
    hipStream_t s = c->stream;
    const int nlev = (int)c->lv.size();
    for (int l = 0; l + 1 < nlev; ++l) {
        Level& L = c->lv[(size_t)l];
        const Level& N = c->lv[(size_t)l + 1];
        if (L.P.nrows == 0 || L.nptr == nullptr || N.nptr == nullptr) continue;
        const int nn = L.A.nrows / B;
        const int64_t nb_fine = L.A.nnz / ((int64_t)B * B);
        const int64_t ncb = N.A.nnz / ((int64_t)B * B);
        Temps tmp(s);
        int32_t* nagg = tmp.make<int32_t>((size_t)std::max(nn, 1));
        int32_t* tpos = tmp.make<int32_t>((size_t)std::max<int64_t>(nb_fine, 1));
        int32_t* cnt = tmp.make<int32_t>((size_t)ncb + 1);
        HIP_CHECK(hipMemsetAsync(cnt, 0, ((size_t)ncb + 1) * sizeof(int32_t), s));
        clear_flags(c);
        launch_node_gal_agg(L.P, B, nagg, c->d_flags, s);
        launch_node_gal_count(L, N, B, nagg, tpos, cnt, c->d_flags, s);
        read_flags(c);
        if (c->h_flags[F_NODEGAL]) continue;
        NodeGal g;
        g.nblk = ncb;
        g.complete = c->h_flags[F_NODEPART] == 0;
        g.tptr = halloc<int32_t>(c, (size_t)ncb + 1);
        exclusive_scan_i32(cnt, g.tptr, ncb + 1, s);
        g.nterm = to_host(g.tptr + ncb, 1, s)[0];
        const size_t nt = (size_t)std::max<int64_t>(g.nterm, 1);
        g.toff = halloc<int32_t>(c, nt);
        g.tlen = halloc<int32_t>(c, nt);
        g.cout = halloc<int32_t>(c, (size_t)std::max<int64_t>(ncb, 1));
        g.clen = halloc<int32_t>(c, (size_t)std::max<int64_t>(ncb, 1));
        int32_t* cur = tmp.make<int32_t>((size_t)std::max<int64_t>(ncb, 1));
        int32_t* last = tmp.make<int32_t>((size_t)std::max<int64_t>(ncb, 1));
        launch_node_gal_fill(L, N, B, tpos, g, cur, last, s);
        HIP_CHECK(hipStreamSynchronize(s));
        L.ngal = g;
    }
}

// The launch shape and position map of C = L B (allocated with the hierarchy); with
// diag, also the diagonal index of every row of L (for the smoother).  Rows with more
// terms than the form takes, or C rows too long for it, leave the product to the
// lane-group kernels.
GalShape make_posmap(amg_ctx* c, const Csr& L, const Csr& B, const Csr& C, bool diag, const GalForce& f,
                     hipStream_t s) {
    if (lanes_only() || f.lanes || L.nrows == 0) return {};
    int64_t* off = halloc<int64_t>(c, (size_t)L.nrows + 1);
    int64_t max_row = 0;
    const int64_t terms = count_galerkin_terms(L, B, off, &max_row, s);
    const auto Cp = to_host(C.ptr, (size_t)C.nrows + 1, s);
    int maxlen = 0;
    for (int32_t i = 0; i < C.nrows; ++i) maxlen = std::max(maxlen, Cp[(size_t)i + 1] - Cp[(size_t)i]);
    GalShape gs = pick_galerkin_shape(L.nrows, L.nnz, terms, maxlen, f.g, f.t);
    if (gs.g == 0 || !galerkin_terms_fit(max_row)) {
        release(c, off);
        return {};
    }
    if (f.wide) gs.wide = 1;
    gs.off = off;
    gs.terms = terms;
    const size_t n = (size_t)std::max<int64_t>(terms, 1);
    gs.pos = gs.wide ? (void*)halloc<uint16_t>(c, n) : (void*)halloc<uint8_t>(c, n);
    gs.bst = halloc<int32_t>(c, (size_t)std::max<int64_t>(L.nnz, 1));
    gs.tof = halloc<uint16_t>(c, (size_t)std::max<int64_t>(L.nnz, 1));
    if (diag) gs.dpos = halloc<int32_t>(c, (size_t)L.nrows + 1);
    build_galerkin_posmap(L, B, C, gs, s);
    return gs;
}

// Launch shapes of a level's row kernels and Galerkin kernels (Ac: the next level's
// operator, whose pattern is the second Galerkin product's), with the position maps.
void set_groups(amg_ctx* c, Level& L, const Csr* Ac, hipStream_t s) {
    configure(c, L.A, s);
    if (L.P.nrows > 0 && Ac != nullptr) {
        configure(c, L.P, s);
        configure(c, L.R, s);
        L.gAP = lane_group((double)L.AP.nnz / (L.A.nrows > 0 ? (double)L.A.nrows : 1.0));
        const GalForce f = galerkin_force();
        L.galAP = make_posmap(c, L.A, L.P, L.AP, true, f, s);
        L.galRAP = make_posmap(c, L.R, L.AP, *Ac, false, f, s);
    }
}

// The fused coarse tail starts at the first level t >= 1 from which every level down to
// the coarsest fits the one-workgroup kernel: their rows together (LDS), their stored
// entries together with the restriction into level t (a single CU reads them all, so
// only the smallest levels gain from the fusion) and the level count.  A tail of the
// coarsest level alone replaces two launches (the restriction into it and the dense solve)
// by one on a single CU, whose dense solve reads the whole inverse: it is kept only for a
// coarsest level of at most TAIL_SOLO_ROWS rows.  0: no tail.
void configure_tail(amg_ctx* c) {
    const int nlev = (int)c->lv.size();
    c->tail = 0;
    if (nlev < 2 || std::getenv("AMGMI_NO_TAIL") != nullptr) return;
    int64_t max_nnz = TAIL_MAX_NNZ;
    if (const char* e = std::getenv("AMGMI_TAIL_NNZ")) max_nnz = std::atoll(e);
    int64_t solo = TAIL_SOLO_ROWS;
    if (const char* e = std::getenv("AMGMI_TAIL_SOLO")) solo = std::atoll(e);
    int64_t rows = 0, nnz = 0;
    for (int t = nlev - 1; t >= 1; --t) {
        const Level& L = c->lv[(size_t)t];
        rows += L.A.nrows;
        nnz += L.A.nnz + L.P.nnz + L.R.nnz;
        const int64_t in = c->lv[(size_t)t - 1].R.nnz;
        if (rows > TAIL_MAX_ROWS || nnz + in > max_nnz || nlev - t > TAIL_MAX_LEVELS) break;
        c->tail = t;
    }
    if (c->tail == nlev - 1 && c->lv.back().A.nrows > solo) c->tail = 0;
}

// Diagonal storage of A_0 when its pattern has at most DIA_MAX distinct column offsets
// and they are well filled (a stencil: 7 or 27 offsets, nearly every row full).  The
// hierarchy's CSR copy stays (the Galerkin product and the exports read it); the
// diagonal copy is refreshed from it after every rebuild.  AMGMI_NO_DIA disables it.
void release_dia(amg_ctx* c) {
    release(c, c->dia.val);
    release(c, c->dia.val32);
    release(c, c->dia.slot);
    c->dia = Dia{};
}

// The full set of diagonals is always written; when the offsets are symmetric the values
// are checked on the device, and the solve switches to the symmetric read (half the
// diagonals) once it has seen the result (c->dia.off.sym, set in the CG's first
// residual read-back).
// scatter = false: the values are already there (the level-0 A P kernel wrote them).
void refresh_dia(amg_ctx* c, bool scatter = true) {
    if (c->dia.ndiag == 0) return;
    const Level& L0 = c->lv[0];
    if (scatter) {
        launch_dia_scatter<double>(L0.A, c->dia, L0.A.val, c->dia.val, c->stream);
        if (c->dia.val32) launch_dia_scatter<float>(L0.A, c->dia, L0.A.val, c->dia.val32, c->stream);
    }
    c->dia.off.sym = 0;
    if (c->dia.symoff) launch_dia_symcheck(L0.A.nrows, c->dia, c->rs.scal(), c->stream);
}

// The CSR values of level 0 again equal to its diagonal storage (after partial updates
// that wrote only the latter).
void ensure_a0_csr(amg_ctx* c) {
    if (!c->a0_csr_stale) return;
    const Level& L0 = c->lv[0];
    launch_dia_gather<double>(L0.A, c->dia, c->dia.val, L0.A.val, c->stream);
    if (c->dia.val32 && L0.A.val32) launch_dia_gather<float>(L0.A, c->dia, c->dia.val32, L0.A.val32, c->stream);
    c->a0_csr_stale = false;
}

// After a read-back of the scalar slots: use the symmetric read when the last refresh
// found symmetric values.
void note_dia_symmetry(amg_ctx* c) {
    if (c->dia.ndiag > 0 && c->dia.symoff) c->dia.off.sym = host_scal(c, S_ASYM) == 0.0 ? 1 : 0;
}

void configure_dia(amg_ctx* c) {
    release_dia(c);
    // (the diagonal-storage kernels fuse scalar Jacobi sweeps; block smoothers use CSR)
    if (std::getenv("AMGMI_NO_DIA") != nullptr || c->prm.block_size > 1) return;
    hipStream_t s = c->stream;
    const Csr& A = c->lv[0].A;
    if (A.nrows == 0) return;
    const std::vector<int> offs = dia_offsets(A, s);
    const int nd = (int)offs.size();
    if (nd == 0 || (double)A.nnz < 0.75 * (double)nd * (double)A.nrows) return;  // not a well-filled stencil
    Dia D;
    D.ndiag = nd;
    for (int d = 0; d < nd; ++d) D.off.off[d] = offs[(size_t)d];
    D.symoff = (nd & 1) == 1 && offs[(size_t)nd / 2] == 0;
    for (int d = 0; d < nd / 2 && D.symoff; ++d) D.symoff = offs[(size_t)d] == -offs[(size_t)(nd - 1 - d)];
    // the 7-point marching kernels: offsets -a, -b, -1, 0, 1, b, a
    const bool seven = nd == 7 && offs[2] == -1 && offs[3] == 0 && offs[4] == 1 && offs[1] == -offs[5] &&
                       offs[0] == -offs[6];
    if (seven && std::getenv("AMGMI_NO_MARCH") == nullptr && march_blocks(A.nrows, offs[6]) <= c->rs.cap) {
        D.march_a = offs[6];
        D.march_b = offs[5];
    }
    // windowed kernels for other stencils (the kernels that read several FP64 vectors per
    // neighbour; every windowed kernel with AMGMI_WIN_ALL)
    if (D.march_a == 0 && std::getenv("AMGMI_NO_WIN") == nullptr) {
        D.win = win_plan(offs);
        D.win.all = std::getenv("AMGMI_WIN_ALL") != nullptr;
        if (std::getenv("AMGMI_NO_WIN2") != nullptr) D.win.two = false;
    }
    if (std::getenv("AMGMI_NO_DIA_SYM") != nullptr) D.symoff = false;
    c->rz32 = std::getenv("AMGMI_NO_RZ32") == nullptr;
    D.slot = halloc<uint8_t>(c, (size_t)A.nnz);
    launch_dia_slots(A, D, s);
    const size_t nv = (size_t)nd * (size_t)A.nrows;
    D.val = halloc<double>(c, nv);
    HIP_CHECK(hipMemsetAsync(D.val, 0, nv * sizeof(double), s));
    if (mixed(c)) {
        D.val32 = halloc<float>(c, nv);
        HIP_CHECK(hipMemsetAsync(D.val32, 0, nv * sizeof(float), s));
    }
    c->dia = D;
    refresh_dia(c);
}

// ------------------------------------------------------------------ Algorithm 4

// Keep P_l, R_l and every cached pattern; recompute A_{l+1} = R_l (A_l P_l) level by
// level, then the smoother diagonals, then the dense inverse of the coarsest operator.
// All sizes are known, so nothing here waits for the device.
template <typename T>
void partial_rebuild(amg_ctx* c, const double* val) {
    hipStream_t s = c->stream;
    Level& L0 = c->lv[0];
    wait_coarse(c);  // the last update's inverse reads A_L, which this update rewrites
    if (!c->ngal_ready) {
        configure_node_gal(c);
        c->ngal_ready = true;
    }
    HIP_CHECK(hipEventRecord(c->ev[0], s));
    c->outer_val = L0.A.val;
    const int nlev = (int)c->lv.size();
    std::vector<char> smoothed((size_t)nlev, 0);
    const bool blocked = c->prm.block_size > 1;
    // Ingest: the level-0 staged A P kernel takes the new values straight from the caller's
    // array and stores the hierarchy's copies (FP64, and FP32 in mixed precision) as it
    // reads them; otherwise they are copied first.
    bool ingested = false;
    const bool node0 = nlev > 1 && L0.ngal.nblk > 0;
    if (nlev == 1 || (node0 ? !L0.ngal.complete : L0.galAP.g == 0)) {
        if (val != L0.A.val) d2d(L0.A.val, val, (size_t)L0.A.nnz * sizeof(double), s);
        if constexpr (std::is_same<T, float>::value) launch_cast_d2f(L0.A.nnz, L0.A.val, L0.A.val32, s);
        ingested = true;
    }
    // with a diagonal storage of A_0 the A P kernel writes the new values there and not
    // into the CSR copy, which is formed again only when it is read (ensure_a0_csr)
    const bool direct = !ingested && c->dia.ndiag > 0;
    for (int l = 0; l + 1 < nlev; ++l) {
        const Level& L = c->lv[l];
        if (L.ngal.nblk > 0) {  // block system: R A P in one pass over A_l's blocks
            Trace tr(c, AMG_K_GALERKIN_AP, l);
            const bool in = l == 0 && !ingested;
            float* a32 = nullptr;
            if constexpr (std::is_same<T, float>::value) a32 = in ? L0.A.val32 : nullptr;
            launch_node_rap<T>(L.ngal, c->prm.block_size, L.A.v<T>(), in ? val : nullptr, in ? L0.A.val : nullptr,
                               a32, c->lv[l + 1].A.v<T>(), s);
            continue;
        }
        {
            // the staged A P kernel also forms this level's smoother diagonal
            Trace tr(c, AMG_K_GALERKIN_AP, l);
            const bool fused = launch_galerkin_ap<T>(L.A, L.P, L.AP, L.gAP, L.galAP, c->prm.smoother,
                                                     c->prm.jacobi_omega, blocked ? nullptr : L.mv<T>(),
                                                     (l == 0 && !ingested) ? val : nullptr, s,
                                                     (l == 0 && direct) ? &c->dia : nullptr);
            smoothed[(size_t)l] = fused && !blocked;
        }
        Trace tr(c, AMG_K_GALERKIN_RAP, l);
        launch_galerkin_rap<T>(L.R, L.AP, c->lv[l + 1].A, c->lv[l + 1].gRAP, L.galRAP, s);
    }
    {
        Trace tr(c, AMG_K_CAST, 0);
        refresh_dia(c, !direct);
    }
    if (direct && val != L0.A.val) c->a0_csr_stale = true;
    HIP_CHECK(hipEventRecord(c->ev[1], s));
    for (int l = 0; l + 1 < nlev; ++l) {
        if (smoothed[(size_t)l]) continue;
        const Level& L = c->lv[l];
        Trace tr(c, AMG_K_SMOOTHER, l);
        if (blocked)
            launch_block_inv<T>(L, c->prm.block_size, c->prm.jacobi_omega, L.mv<T>(), nullptr, s);
        else
            launch_smoother_diag<T>(L.A, c->prm.smoother, c->prm.jacobi_omega, L.mv<T>(), s);
    }
    HIP_CHECK(hipEventRecord(c->ev[2], s));
    // the blocked inverse (one workgroup per pivot block on its critical path) runs beside
    // the start of the next solve, which needs it only at the bottom of its first cycle
    const bool side = c->side != nullptr && c->nL > COARSE_LDS_MAX && c->tail == 0;
    hipStream_t cs = side ? c->side : s;
    if (side) {
        HIP_CHECK(hipEventRecord(c->ev_fork, s));
        HIP_CHECK(hipStreamWaitEvent(cs, c->ev_fork, 0));
    }
    {
        Trace tr(c, AMG_K_COARSE_INV, nlev - 1, cs);
        launch_densify<T>(c->lv.back().A, c->cinv, cs);
        launch_dense_inverse(c->nL, c->cinv, c->rs.scal(), c->cwork, cs);
    }
    HIP_CHECK(hipEventRecord(c->ev[3], cs));
    if (side) {
        HIP_CHECK(hipEventRecord(c->ev_inv, cs));
        c->cinv_pending = true;
    }
    c->phase_pending = true;
}

void partial_any(amg_ctx* c, const double* val) {
    if (mixed(c))
        partial_rebuild<float>(c, val);
    else
        partial_rebuild<double>(c, val);
}

template <typename T>
void alloc_vectors(amg_ctx* c) {
    for (Level& L : c->lv) {
        const size_t n = (size_t)L.A.nrows;
        L.u = halloc<T>(c, n);
        L.f = halloc<T>(c, n);
        L.r = halloc<T>(c, n);
        L.t = halloc<T>(c, n);
    }
}

// FP32 shadows of the hierarchy (mixed precision): every operator value array, and the
// transfer operators cast once.
void alloc_shadow(amg_ctx* c) {
    hipStream_t s = c->stream;
    for (Level& L : c->lv) {
        L.A.val32 = halloc<float>(c, (size_t)L.A.nnz);
        if (L.P.nrows > 0) {
            L.P.val32 = halloc<float>(c, (size_t)L.P.nnz);
            L.R.val32 = halloc<float>(c, (size_t)L.R.nnz);
            L.AP.val32 = halloc<float>(c, (size_t)L.AP.nnz);
            L.m32 = halloc<float>(c, (size_t)L.A.nrows * c->prm.block_size);
            launch_cast_d2f(L.P.nnz, L.P.val, L.P.val32, s);
            launch_cast_d2f(L.R.nnz, L.R.val, L.R.val32, s);
        }
    }
}

void alloc_cg(amg_ctx* c) {
    const size_t n = (size_t)c->lv[0].A.nrows;
    c->x = halloc<double>(c, n);
    c->r = halloc<double>(c, n);
    c->r2 = halloc<double>(c, n);
    c->z = halloc<double>(c, n);
    c->zold = halloc<double>(c, n);
    c->pa = halloc<double>(c, n);
    c->pb = halloc<double>(c, n);
    c->q = halloc<double>(c, n);
}

// Partial-sum scratch sized for the full grids of the level-0 kernels.
void alloc_reduction(amg_ctx* c) {
    const Csr& A = c->lv[0].A;
    int cap = full_grid_rows(A.nrows, A.rpb, A.g);
    if (c->prm.block_size > 1) cap = std::max(cap, node_grid(A.nrows / c->prm.block_size));
    if (cap < RED_BLOCKS) cap = RED_BLOCKS;
    c->rs.cap = cap;
    c->rs.part = halloc<double>(c, RedScratch::doubles(cap));
    HIP_CHECK(hipMemsetAsync(c->rs.part, 0, RedScratch::doubles(cap) * sizeof(double), c->stream));
    if (c->h_red) {
        HIP_CHECK(hipStreamSynchronize(c->stream));
        HIP_CHECK(hipHostFree(c->h_red));
        c->h_red = nullptr;
    }
    HIP_CHECK(hipHostMalloc((void**)&c->h_red, RedScratch::host_doubles(cap) * sizeof(double),
                            hipHostMallocMapped | hipHostMallocCoherent));
    c->rs.host = nullptr;
    if (std::getenv("AMGMI_NO_HOST_WRITE") == nullptr) {
        void* dptr = nullptr;
        HIP_CHECK(hipHostGetDevicePointer(&dptr, c->h_red, 0));
        c->rs.host = (double*)dptr;
    }
}

struct Transfer {
    int nlev;
    const int32_t* const* ptr;
    const int32_t* const* col;
    const double* const* val;
    const int32_t* nc;
    const int64_t* nnz;
};

// ------------------------------------------------------------------ Algorithm 1

void build_hierarchy(amg_ctx* c, int32_t n, int64_t nnz, const int32_t* ptr, const int32_t* col,
                     const double* val, const Transfer* tr) {
    wait_coarse(c);  // the old hierarchy's arrays are freed on the context's stream
    c->pol_updates = 0;
    c->pol_iters_ref = 0;
    c->pol_last_iters = 0;
    c->pol_last_conv = 0;
    c->bi_t = c->bi_w = c->bi_sc = c->bi_part = nullptr;  // hierarchy allocations: released with the old hierarchy
    hipStream_t s = c->stream;
    const amg_params& p = c->prm;
    const auto t_all = Clock::now();
    double ph[8] = {0, 0, 0, 0, 0, 0, 0, 0};

    // Copy the input first: it may be the current hierarchy's own level-0 arrays.
    std::vector<void*> old = std::move(c->hier_allocs);
    c->hier_allocs.clear();
    Csr A0;
    A0.nrows = A0.ncols = n;
    A0.nnz = nnz;
    A0.ptr = halloc<int32_t>(c, (size_t)n + 1);
    A0.col = halloc<int32_t>(c, (size_t)nnz);
    A0.val = halloc<double>(c, (size_t)nnz);
    d2d(A0.ptr, ptr, ((size_t)n + 1) * sizeof(int32_t), s);
    d2d(A0.col, col, (size_t)nnz * sizeof(int32_t), s);
    d2d(A0.val, val, (size_t)nnz * sizeof(double), s);
    for (void* q : old) dfree(q, s);
    c->lv.clear();
    c->outer_own = nullptr;
    c->cinv = nullptr;
    c->cwork = nullptr;
    c->dia = Dia{};  // its arrays were hierarchy allocations
    c->a0_csr_stale = false;
    c->tail = 0;
    c->lv.emplace_back();
    c->lv[0].A = A0;
    c->outer_val = A0.val;
    c->phase_pending = false;

    for (int l = 0;; ++l) {
        const Csr A = c->lv[(size_t)l].A;
        const int32_t nl = A.nrows;
        int32_t* diag_pos = dnew<int32_t>((size_t)nl, s);
        validate(c, A, diag_pos, l == 0 ? "input matrix" : "coarse operator");
        if (p.block_size > 1) node_pattern(c, c->lv[(size_t)l]);  // full blocks, node pattern
        const bool stop = tr ? (l >= tr->nlev) : (nl <= p.coarse_enough || l >= p.max_levels - 1);
        if (stop) {
            dfree(diag_pos, s);
            break;
        }
        Csr P;
        auto t0 = Clock::now();
        if (tr) {
            P.nrows = nl;
            P.ncols = tr->nc[l];
            P.nnz = tr->nnz[l];
            P.ptr = halloc<int32_t>(c, (size_t)nl + 1);
            P.col = halloc<int32_t>(c, (size_t)P.nnz);
            P.val = halloc<double>(c, (size_t)P.nnz);
            d2d(P.ptr, tr->ptr[l], ((size_t)nl + 1) * sizeof(int32_t), s);
            d2d(P.col, tr->col[l], (size_t)P.nnz * sizeof(int32_t), s);
            d2d(P.val, tr->val[l], (size_t)P.nnz * sizeof(double), s);
            validate(c, P, nullptr, "transfer operator");
        } else {
            uint8_t* strong = halloc<uint8_t>(c, (size_t)A.nnz);
            const double eps = std::ldexp(p.eps_strong, -l);
            int32_t* agg = halloc<int32_t>(c, (size_t)nl);
            int32_t nc = 0;
            if (p.block_size > 1) {
                // nodes of B unknowns: strength and MIS-2 on the node matrix of block norms
                const int B = p.block_size;
                Temps tmp(s);
                Csr Nm;
                clear_flags(c);
                build_node_matrix(A, B, Nm, c->d_flags, c->h_flags, s);
                tmp.add(Nm.ptr);
                tmp.add(Nm.col);
                tmp.add(Nm.val);
                const int32_t nn = Nm.nrows;
                int32_t* ndiag = tmp.make<int32_t>((size_t)nn);
                validate(c, Nm, ndiag, "node matrix");
                uint8_t* nstrong = tmp.make<uint8_t>((size_t)Nm.nnz);
                int32_t* ntpos = tmp.make<int32_t>((size_t)Nm.nnz);
                uint8_t* niso = tmp.make<uint8_t>((size_t)nn);
                uint8_t* nstate = tmp.make<uint8_t>((size_t)nn);
                int32_t* nagg = tmp.make<int32_t>((size_t)nn);
                clear_flags(c);
                launch_strength(Nm, ndiag, eps * eps, nstrong, ntpos, niso, c->d_flags, s);
                read_flags(c);
                if (c->h_flags[F_PATTERN]) throw Fail{AMG_ERR_PATTERN, "pattern is not structurally symmetric"};
                run_mis2(Nm, nstrong, niso, nstate, c->d_flags, c->h_flags, s);
                nc = run_aggregate(Nm, nstrong, ntpos, nstate, nagg, c->d_flags, c->h_flags, s) * B;
                launch_node_expand(A, B, Nm, nstrong, nagg, strong, agg, s);
            } else {
                Temps tmp(s);
                int32_t* tpos = tmp.make<int32_t>((size_t)A.nnz);
                uint8_t* iso = tmp.make<uint8_t>((size_t)nl);
                uint8_t* state = tmp.make<uint8_t>((size_t)nl);
                clear_flags(c);
                launch_strength(A, diag_pos, eps * eps, strong, tpos, iso, c->d_flags, s);
                read_flags(c);
                if (c->h_flags[F_PATTERN]) throw Fail{AMG_ERR_PATTERN, "pattern is not structurally symmetric"};
                run_mis2(A, strong, iso, state, c->d_flags, c->h_flags, s);
                nc = run_aggregate(A, strong, tpos, state, agg, c->d_flags, c->h_flags, s);
            }
            c->lv[(size_t)l].agg = agg;
            c->lv[(size_t)l].strong = strong;
            ph[0] += ms_since(t0);
            if (nc == 0 || nc >= nl) {
                dfree(diag_pos, s);
                break;
            }
            t0 = Clock::now();
            build_prolongator(A, strong, diag_pos, agg, nc, p.aggregation, P, s);
            track(c, P);
        }
        Csr R;
        build_transpose(P, R, s);
        track(c, R);
        HIP_CHECK(hipStreamSynchronize(s));
        ph[1] += ms_since(t0);
        t0 = Clock::now();
        Csr AP, Ac;
        symbolic_spgemm(A, P, AP, s);
        track(c, AP);
        symbolic_spgemm(R, AP, Ac, s);
        track(c, Ac);
        AP.val = halloc<double>(c, (size_t)AP.nnz);
        Ac.val = halloc<double>(c, (size_t)Ac.nnz);
        Ac.ncols = Ac.nrows;
        HIP_CHECK(hipStreamSynchronize(s));
        ph[2] += ms_since(t0);
        t0 = Clock::now();
        {
            Level& L = c->lv[(size_t)l];
            L.P = P;
            L.R = R;
            L.AP = AP;
            set_groups(c, L, &Ac, s);
        }
        Level next;
        next.A = Ac;
        set_groups(c, next, nullptr, s);
        next.gRAP = lane_group((double)Ac.nnz / (Ac.nrows > 0 ? (double)Ac.nrows : 1.0));
        launch_galerkin_ap<double>(A, P, AP, c->lv[(size_t)l].gAP, c->lv[(size_t)l].galAP, 0, 0.0,
                                   (double*)nullptr, nullptr, s);
        launch_galerkin_rap<double>(R, AP, Ac, next.gRAP, c->lv[(size_t)l].galRAP, s);
        HIP_CHECK(hipStreamSynchronize(s));
        ph[3] += ms_since(t0);
        dfree(diag_pos, s);
        c->lv.push_back(next);
    }
    set_groups(c, c->lv.back(), nullptr, s);

    alloc_reduction(c);
    auto t0 = Clock::now();
    const int nlev = (int)c->lv.size();
    clear_flags(c);
    for (int l = 0; l + 1 < nlev; ++l) {
        Level& L = c->lv[(size_t)l];
        L.m = halloc<double>(c, (size_t)L.A.nrows * p.block_size);
        if (p.block_size > 1)
            launch_block_inv<double>(L, p.block_size, p.jacobi_omega, L.m, c->d_flags, s);
        else
            launch_smoother_diag<double>(L.A, p.smoother, p.jacobi_omega, L.m, s);
    }
    read_flags(c);
    if (c->h_flags[F_NOT_SPD]) throw Fail{AMG_ERR_NOT_SPD, "singular diagonal block"};
    ph[4] += ms_since(t0);
    t0 = Clock::now();
    c->nL = c->lv.back().A.nrows;
    if (c->nL > COARSE_GLOBAL_MAX)
        throw Fail{AMG_ERR_ARG, "coarsest level has " + std::to_string(c->nL) + " rows; too many for a dense inverse"};
    c->cinv = halloc<double>(c, (size_t)c->nL * c->nL);
    c->cwork = c->nL > COARSE_LDS_MAX ? halloc<double>(c, COARSE_WORK_DOUBLES) : nullptr;
    launch_densify<double>(c->lv.back().A, c->cinv, s);
    launch_dense_inverse(c->nL, c->cinv, c->rs.scal(), c->cwork, s);
    read_red(c);
    if (host_scal(c, S_COARSE) != 0.0) throw Fail{AMG_ERR_NOT_SPD, "coarsest operator is not SPD"};
    ph[5] += ms_since(t0);
    c->ngal_ready = false;
    configure_node_transfer(c);

    if (mixed(c)) {
        alloc_shadow(c);
        partial_rebuild<float>(c, c->lv[0].A.val);
        wait_coarse(c);
        read_red(c);
        if (host_scal(c, S_COARSE) != 0.0) throw Fail{AMG_ERR_NOT_SPD, "coarsest FP32 operator is not SPD"};
        c->phase_pending = false;
        alloc_vectors<float>(c);
    } else {
        alloc_vectors<double>(c);
    }
    alloc_cg(c);
    configure_tail(c);
    configure_dia(c);
    HIP_CHECK(hipStreamSynchronize(s));
    ph[6] = ms_since(t_all);
    std::memcpy(c->phase_ms, ph, sizeof(ph));
}

// New pattern with the same number of rows: keep P_l and R_l, recompute the Galerkin
// patterns level by level (values follow in the partial update).
void repattern(amg_ctx* c) {
    wait_coarse(c);
    hipStream_t s = c->stream;
    Level& L0 = c->lv[0];
    Csr A;
    A.nrows = A.ncols = c->pend_n;
    A.nnz = c->pend_nnz;
    A.ptr = halloc<int32_t>(c, (size_t)A.nrows + 1);
    A.col = halloc<int32_t>(c, (size_t)A.nnz);
    A.val = halloc<double>(c, (size_t)A.nnz);
    d2d(A.ptr, c->pend_ptr, ((size_t)A.nrows + 1) * sizeof(int32_t), s);
    d2d(A.col, c->pend_col, (size_t)A.nnz * sizeof(int32_t), s);
    release_csr(c, L0.A);
    release(c, c->outer_own);
    c->outer_own = nullptr;
    L0.A = A;
    c->a0_csr_stale = false;
    c->outer_val = L0.A.val;
    dfree(c->pend_ptr, s);
    dfree(c->pend_col, s);
    c->pend_ptr = c->pend_col = nullptr;
    c->pend_n = 0;
    // structural checks only; the values are checked through the coarse factorisation
    Csr pat = A;
    pat.val = nullptr;
    int32_t* diag_pos = dnew<int32_t>((size_t)A.nrows, s);
    validate(c, pat, diag_pos, "new pattern");
    dfree(diag_pos, s);
    if (c->prm.block_size > 1) node_pattern(c, L0);  // the block kernels need full blocks
    const int nlev = (int)c->lv.size();
    for (int l = 0; l + 1 < nlev; ++l) {
        Level& L = c->lv[(size_t)l];
        Level& N = c->lv[(size_t)l + 1];
        release_csr(c, L.AP);
        Csr AP, Ac;
        symbolic_spgemm(L.A, L.P, AP, s);
        track(c, AP);
        AP.val = halloc<double>(c, (size_t)AP.nnz);
        if (mixed(c)) AP.val32 = halloc<float>(c, (size_t)AP.nnz);
        symbolic_spgemm(L.R, AP, Ac, s);
        track(c, Ac);
        Ac.ncols = Ac.nrows;
        Ac.val = halloc<double>(c, (size_t)Ac.nnz);
        if (mixed(c)) Ac.val32 = halloc<float>(c, (size_t)Ac.nnz);
        L.AP = AP;
        release_csr(c, N.A);
        N.A = Ac;
        release_posmaps(c, L);
        set_groups(c, L, &N.A, s);
        N.gRAP = lane_group((double)Ac.nnz / (Ac.nrows > 0 ? (double)Ac.nrows : 1.0));
    }
    if (mixed(c)) L0.A.val32 = halloc<float>(c, (size_t)L0.A.nnz);
    if (c->prm.block_size > 1)
        for (int l = 1; l < nlev; ++l) node_pattern(c, c->lv[(size_t)l]);
    for (Level& L : c->lv) release_node_gal(c, L.ngal);
    c->ngal_ready = false;
    set_groups(c, c->lv.back(), nullptr, s);
    release(c, c->rs.part);
    alloc_reduction(c);
    configure_tail(c);
    configure_dia(c);
    // The strength flags were per entry of the old patterns; the aggregates stay (they
    // still define the kept transfer operators).
    for (Level& L : c->lv) {
        release(c, L.strong);
        L.strong = nullptr;
    }
}

// ------------------------------------------------------------------ V-cycle

// CG dot products fused into the last step of the V-cycle (rho = r.z, beta).
struct RzEpilogue {
    int flexible;
    mutable int nb;  // partials written (set by the kernel that formed r.z)
    // mixed precision: the CG's FP64 r and z; the FP32 cycle's last level-0 sweep writes z
    // and forms r.z itself when it can (z_done), else the caller widens the cycle's output
    const double* r64 = nullptr;
    double* z64 = nullptr;
    mutable bool z_done = false;
};

// Algorithm 2 on level l from a zero initial guess; returns the buffer holding u_l.
// At level 0 the last post-smoothing sweep writes directly into `out` when given, and
// with an epilogue (FP64) it also forms the CG partial sums of r.z from f (= the CG
// residual) and z.  `ready` = 1: the first smoothing sweep u = m f is already in the
// level's u (the restriction forms it on coarser levels); 2: so is the residual f - A u
// in the level's r (the fused CG update forms both on level 0; one pre-sweep only).
// Restriction of level l's residual into the coarse tail and the tail levels down to the
// coarsest and back, in one workgroup; the tail's finest level gets its correction in u.
template <typename T>
void run_tail(amg_ctx* c, int l, const T* rres) {
    const Level& L = c->lv[(size_t)l];
    const Level& C = c->lv[(size_t)l + 1];
    const amg_params& p = c->prm;
    const int nlev = (int)c->lv.size();
    TailArgs<T> ta;
    ta.nlev = nlev - c->tail;
    ta.npre = p.npre;
    ta.npost = p.npost;
    ta.bs = p.block_size;
    ta.rin_ptr = L.R.ptr;
    ta.rin_col = L.R.col;
    ta.rin_val = L.R.v<T>();
    ta.rin = rres;
    ta.uout = (T*)C.u;
    ta.cinv = c->cinv;
    int soff = 0;
    for (int k = 0; k < ta.nlev; ++k) {
        const Level& Lk = c->lv[(size_t)(c->tail + k)];
        TailLevel<T>& tk = ta.lv[k];
        tk.n = Lk.A.nrows;
        tk.soff = soff;
        soff += 3 * tk.n;
        tk.Aptr = Lk.A.ptr;
        tk.Acol = Lk.A.col;
        tk.Aval = Lk.A.v<T>();
        tk.m = Lk.mv<T>();
        if (k + 1 < ta.nlev) {
            tk.Rptr = Lk.R.ptr;
            tk.Rcol = Lk.R.col;
            tk.Rval = Lk.R.v<T>();
            tk.Pptr = Lk.P.ptr;
            tk.Pcol = Lk.P.col;
            tk.Pval = Lk.P.v<T>();
        }
    }
    Trace tr(c, AMG_K_TAIL, l + 1);
    launch_vcycle_tail<T>(ta, c->stream);
}

template <typename T>
T* vcycle_level(amg_ctx* c, int l, const T* f, T* out, const RzEpilogue* ep = nullptr, int ready = 0);

// A non-coarsest level with damped block Jacobi (systems with B unknowns per node): each
// sweep u += M (f - A u) is one node-group pass (residual and block-diagonal product); the
// first sweep from zero is u = M f, the pre-smoothing residual a node-group pass on
// level 0 and a row-block pass below.
// Algorithm 2 with the scalar-diagonal fused forms left out; the coarse tail as for
// scalar systems.
template <typename T>
T* vcycle_level_block(amg_ctx* c, int l, const T* f, T* out, const RzEpilogue* ep) {
    hipStream_t s = c->stream;
    const Level& L = c->lv[(size_t)l];
    const amg_params& p = c->prm;
    const int B = p.block_size;
    const int n = L.A.nrows;
    T* cur = (T*)L.u;
    T* other = (T*)L.t;
    T* r = (T*)L.r;
    const T* m = L.mv<T>();
    const T* rres = f;
    auto sweep = [&](const T* uu, T* uout) { launch_node_sweep<T>(L, B, m, f, uu, uout, s); };
    if (p.npre == 0) {
        HIP_CHECK(hipMemsetAsync(cur, 0, (size_t)n * sizeof(T), s));
    } else {
        {
            Trace tr(c, AMG_K_SMOOTH0_RES, l);
            launch_block_apply<T>(n, B, m, f, (const T*)nullptr, cur, s);
        }
        for (int it = 1; it < p.npre; ++it) {
            Trace tr(c, AMG_K_JACOBI, l);
            sweep(cur, other);
            std::swap(cur, other);
        }
        Trace tr(c, AMG_K_SMOOTH0_RES, l);
        // (on the coarser levels the LDS-staged row-block residual is faster)
        if (l == 0)
            launch_node_residual<T>(L, B, f, cur, r, s);
        else
            launch_residual<T>(L.A, f, cur, r, s);
        rres = r;
    }
    const Level& C = c->lv[(size_t)l + 1];
    const T* uc;
    if (c->tail > 0 && l + 1 == c->tail) {
        run_tail<T>(c, l, rres);
        uc = (const T*)C.u;
    } else {
        {
            Trace tr(c, AMG_K_RESTRICT, l);
            launch_spmv<T>(L.R, rres, (T*)C.f, (const T*)nullptr, (T*)nullptr, s);
        }
        uc = vcycle_level<T>(c, l + 1, (const T*)C.f, nullptr, nullptr, 0);
    }
    {
        Trace tr(c, AMG_K_PROLONG, l);
        if (L.nagg != nullptr)
            launch_node_prolong<T>(L, B, uc, cur, s);
        else
            launch_prolong_add<T>(L.P, uc, cur, s);
    }
    bool fused = false;
    for (int it = 0; it < p.npost; ++it) {
        T* dst = (out && it == p.npost - 1) ? out : other;
        Trace tr(c, AMG_K_JACOBI, l);
        if constexpr (std::is_same<T, double>::value) {
            if (ep && dst == out) {  // the CG's r.z partials in the same pass
                ep->nb = launch_node_sweep_rz(L, B, m, f, cur, dst, c->rs, s);
                fused = true;
            } else {
                sweep(cur, dst);
            }
        } else {
            sweep(cur, dst);
        }
        if (dst == other)
            std::swap(cur, other);
        else
            cur = dst;
    }
    if (out && cur != out) {
        d2d(out, cur, (size_t)n * sizeof(T), s);
        cur = out;
    }
    if constexpr (std::is_same<T, double>::value) {  // (an FP32 cycle's r.z is formed by its caller)
        if (ep && !fused) {
            Trace tr(c, AMG_K_CG_RZ, 0);
            ep->nb = launch_cg_rz(n, (const double*)f, (const double*)cur, c->rs, s);
        }
    }
    return cur;
}

template <typename T>
T* vcycle_level(amg_ctx* c, int l, const T* f, T* out, const RzEpilogue* ep, int ready) {
    hipStream_t s = c->stream;
    const Level& L = c->lv[(size_t)l];
    const int nlev = (int)c->lv.size();
    if (l == nlev - 1) {
        T* u = out ? out : (T*)L.u;
        Trace tr(c, AMG_K_COARSE_GEMV, l);
        wait_coarse(c);
        launch_coarse_gemv<T>(c->nL, c->cinv, f, u, c->rs.scal() + S_COARSE, s);
        if (std::is_same<T, double>::value && ep) {  // (an FP32 cycle's r.z is formed by its caller)
            Trace tr2(c, AMG_K_CG_RZ, 0);
            if (ep->flexible) throw Fail{AMG_ERR_ARG, "flexible CG needs at least one post-smoothing sweep"};
            ep->nb = launch_cg_rz(L.A.nrows, (const double*)f, (const double*)u, c->rs, s);
        }
        return u;
    }
    const amg_params& p = c->prm;
    T* cur = (T*)L.u;
    T* other = (T*)L.t;
    T* r = (T*)L.r;
    const T* m = L.mv<T>();
    const T* rres = r;
    const int n = L.A.nrows;
    if (p.block_size > 1) return vcycle_level_block<T>(c, l, f, out, ep);
    const bool dia = l == 0 && c->dia.ndiag > 0;  // level 0 in diagonal storage
    auto residual = [&](const T* uu) {
        if (dia)
            launch_dia_residual<T>(n, c->dia, f, uu, r, s);
        else
            launch_residual<T>(L.A, f, uu, r, s);
    };
    auto sweep = [&](const T* uu, T* uout) {
        if (dia)
            launch_dia_jacobi<T>(n, c->dia, m, f, uu, uout, s);
        else
            launch_jacobi<T>(L.A, m, f, uu, uout, s);
    };
    if (p.npre == 0) {
        HIP_CHECK(hipMemsetAsync(cur, 0, (size_t)L.A.nrows * sizeof(T), s));
        rres = f;
    } else {
        if (ready == 2) {
            if (p.npre != 1) throw Fail{AMG_ERR_ARG, "a fused first sweep needs exactly one pre-sweep"};
        } else if (ready == 1) {
            Trace tr(c, AMG_K_SMOOTH0_RES, l);
            if (p.npre == 1) residual(cur);
        } else {
            Trace tr(c, AMG_K_SMOOTH0_RES, l);
            if (dia)
                launch_dia_smooth0_residual<T>(n, c->dia, m, f, cur, r, s);
            else
                launch_smooth0_residual<T>(L.A, m, f, cur, r, s);
        }
        for (int it = 1; it < p.npre; ++it) {
            Trace tr(c, AMG_K_JACOBI, l);
            sweep(cur, other);
            std::swap(cur, other);
        }
        if (p.npre > 1) residual(cur);
    }
    const Level& C = c->lv[(size_t)l + 1];
    const T* uc;
    if (c->tail > 0 && l + 1 == c->tail) {
        run_tail<T>(c, l, rres);
        uc = (const T*)C.u;
    } else {
        // the next level's first sweep from zero is formed by the restriction
        const bool c_smooths = (l + 2 < nlev) && p.npre > 0;
        {
            Trace tr(c, AMG_K_RESTRICT, l);
            launch_spmv<T>(L.R, rres, (T*)C.f, c_smooths ? C.mv<T>() : nullptr, c_smooths ? (T*)C.u : nullptr, s);
        }
        uc = vcycle_level<T>(c, l + 1, (const T*)C.f, nullptr, nullptr, c_smooths ? 1 : 0);
    }
    {
        Trace tr(c, AMG_K_PROLONG, l);
        launch_prolong_add<T>(L.P, uc, cur, s);
    }
    bool fused = false;
    for (int it = 0; it < p.npost; ++it) {
        const bool last = it == p.npost - 1;
        T* dst = (out && last) ? out : other;
        Trace tr(c, AMG_K_JACOBI, l);
        if constexpr (std::is_same<T, double>::value) {
            if (last && ep && dst == out) {
                ep->nb = dia ? launch_dia_jacobi_rz(n, c->dia, m, f, cur, dst, ep->flexible, c->rs, s)
                             : launch_jacobi_rz(L.A, m, f, cur, dst, ep->flexible, c->rs, s);
                fused = true;
            } else {
                sweep(cur, dst);
            }
        } else {
            if (last && ep && ep->z64 && dia && c->rz32) {
                const int nb = launch_dia_jacobi_rz32(n, c->dia, m, f, cur, ep->r64, ep->z64, ep->flexible, c->rs, s);
                if (nb > 0) {  // z is the FP64 result; the FP32 one is not written
                    ep->nb = nb;
                    ep->z_done = true;
                    break;
                }
            }
            sweep(cur, dst);
        }
        if (dst == other)
            std::swap(cur, other);
        else
            cur = dst;
    }
    if (out && cur != out) {
        d2d(out, cur, (size_t)L.A.nrows * sizeof(T), s);
        cur = out;
    }
    if constexpr (std::is_same<T, double>::value) {
        if (ep && !fused) {
            if (ep->flexible) throw Fail{AMG_ERR_ARG, "flexible CG needs at least one post-smoothing sweep"};
            Trace tr(c, AMG_K_CG_RZ, 0);
            ep->nb = launch_cg_rz(L.A.nrows, (const double*)f, (const double*)cur, c->rs, s);
        }
    }
    return cur;
}

// z = B r with r, z in FP64; in mixed precision the cycle itself runs in FP32.  With an
// epilogue, the CG scalars rho (= r.z) and beta are formed in the same pass.  `ready`:
// what the CG update already formed -- FP64: 2 = level 0's first sweep and residual;
// mixed: 1 = r in FP32 in level 0's f.
void vcycle_apply(amg_ctx* c, const double* r, double* z, const RzEpilogue* ep = nullptr, int ready = 0) {
    Level& L0 = c->lv[0];
    if (mixed(c)) {
        if (ready != 1) {
            Trace tr(c, AMG_K_CAST, 0);
            launch_cast_d2f(L0.A.nrows, r, (float*)L0.f, c->stream);
        }
        // the FP32 cycle forms z and r.z itself only in the level-0 diagonal-storage sweep;
        // every other FP32 path leaves them to the widening pass below
        const bool fuse = ep && c->rz32 && c->prm.block_size == 1 && c->dia.ndiag > 0 && c->lv.size() > 1;
        RzEpilogue e32{ep ? ep->flexible : 0, 0, r, z};
        const float* res = vcycle_level<float>(c, 0, (const float*)L0.f, nullptr, fuse ? &e32 : nullptr);
        if (e32.z_done) {
            ep->nb = e32.nb;
            return;
        }
        Trace tr(c, AMG_K_CAST, 0);
        if (ep)
            ep->nb = launch_cast_rz(L0.A.nrows, res, r, z, ep->flexible, c->rs, c->stream);
        else
            launch_cast_f2d(L0.A.nrows, res, z, c->stream);
    } else {
        vcycle_level<double>(c, 0, r, z, ep, ready);
    }
}

// ------------------------------------------------------------------ PCG

// CG preconditioned by one V-cycle; stops on the true relative residual.  Scalars stay on
// the device (each kernel adds the partials it needs); each iteration reads the ||r||^2
// partials and the breakdown flag back with one copy.
amg_status pcg(amg_ctx* c, const double* f, double* u, amg_solve_info* info) {
    hipStream_t s = c->stream;
    const Level& L0 = c->lv[0];
    const int n = L0.A.nrows;
    const amg_params& p = c->prm;
    amg_solve_info inf{0, 0, 0.0};
    // the CG residual; the fused update writes the new one to the other buffer
    double* rc = c->r;
    double* ra = c->r2;
    auto true_residual = [&]() {
        int nb;
        {
            Trace tr(c, AMG_K_CG_INIT, 0);
            nb = (c->dia.ndiag > 0 && c->outer_val == L0.A.val)
                     ? launch_dia_cg_init(n, c->dia, f, c->x, rc, c->rs, s)
                     : launch_cg_init(L0.A, c->outer_val, f, c->x, rc, c->rs, s);
        }
        read_red(c);
        note_dia_symmetry(c);
        return nb;
    };
    launch_copy(n, u, c->x, s);
    // with the inverse still running beside, its pivot flag is read after the first cycle
    // (a failed inverse makes that cycle's output NaN, hence a breakdown, checked below)
    const bool coarse_known = !c->cinv_pending;
    int nb = true_residual();
    auto coarse_failed = [&]() {
        if (!coarse_known) {
            wait_coarse(c);
            read_red(c);
        }
        return host_scal(c, S_COARSE) != 0.0;
    };
    if (coarse_known && coarse_failed())
        throw Fail{AMG_ERR_NOT_SPD, "coarsest operator of the last rebuild is not SPD"};
    const double ff = host_sum(c, P_FF, nb);
    if (ff == 0.0) {
        if (!coarse_known && coarse_failed())
            throw Fail{AMG_ERR_NOT_SPD, "coarsest operator of the last rebuild is not SPD"};
        HIP_CHECK(hipMemsetAsync(u, 0, (size_t)n * sizeof(double), s));
        HIP_CHECK(hipStreamSynchronize(s));
        inf.converged = 1;
        if (info) *info = inf;
        return AMG_OK;
    }
    const double nf = std::sqrt(ff);
    double res = std::sqrt(host_sum(c, P_RR, nb)) / nf;
    if (res <= p.rtol) {
        if (!coarse_known && coarse_failed())
            throw Fail{AMG_ERR_NOT_SPD, "coarsest operator of the last rebuild is not SPD"};
        inf.converged = 1;
        inf.rel_res_true = res;
        if (info) *info = inf;
        return AMG_OK;
    }
    RzEpilogue ep{p.flexible_cg, 0};
    auto precondition = [&](int first, int ready) {
        vcycle_apply(c, rc, c->z, &ep, ready);
        launch_fin_rz(ep.nb, p.flexible_cg, first, c->rs, s);
    };
    // The x, r update can start the next preconditioner application: on a level-0
    // diagonal storage (FP64) it also forms the first V-cycle sweep and its residual; in
    // mixed precision it stores r in FP32 for the V-cycle.
    const bool fuse_dia = !mixed(c) && c->dia.ndiag > 0 && p.npre == 1 && c->lv.size() > 1;
    const bool fuse_cast = mixed(c);
    precondition(1, 0);
    double* pold = c->pa;
    double* pnew = c->pb;
    int it = 0;
    bool converged = false;
    double rate = 1.0, rate_last = 1.0;  // recent per-iteration residual reduction
    while (it < p.maxiter) {
        ++it;
        int nb_pq;
        {
            Trace tr(c, AMG_K_CG_PQ, 0);
            // the diagonal storage holds the hierarchy's A_0, which is the Krylov operator
            // except after an operator-only update (full reuse)
            if (c->dia.ndiag > 0 && c->outer_val == L0.A.val)
                nb_pq = launch_dia_cg_pq(n, c->dia, c->z, pold, pnew, c->q, it == 1, c->rs, s);
            else if (p.block_size > 1)  // the Krylov operator has the pattern of A_0
                nb_pq = launch_node_cg_pq(L0, p.block_size, c->outer_val, c->z, pold, pnew, c->q, it == 1, c->rs, s);
            else
                nb_pq = launch_cg_pq(L0.A, c->outer_val, c->z, pold, pnew, c->q, it == 1, c->rs, s);
        }
        launch_fin_pq(nb_pq, c->rs, s);
        int ready = 0;
        {
            Trace tr(c, AMG_K_CG_UPDATE, 0);
            if (fuse_dia) {
                nb = launch_dia_update_smooth0(n, c->dia, pnew, c->q, c->x, rc, ra, L0.m, (double*)L0.u,
                                               (double*)L0.r, c->rs, s);
                std::swap(rc, ra);
                ready = 2;
            } else if (fuse_cast) {
                nb = launch_cg_update_cast(n, pnew, c->q, c->x, rc, (float*)L0.f, c->rs, s);
                ready = 1;
            } else {
                nb = launch_cg_update(n, pnew, c->q, c->x, rc, c->rs, s);
            }
        }
        // Read ||r||^2 back, but queue the next preconditioner application first so the
        // device keeps working while the host decides; it is discarded on convergence.
        // the update kernel wrote the ||r||^2 partials and the breakdown flag straight into
        // the host mirror; otherwise they are copied there
        if (c->rs.host == nullptr) queue_read_rr(c, nb);
        HIP_CHECK(hipEventRecord(c->ev_read, s));
        // (not with flexible CG: its r.z_old term reads the z a speculative sweep overwrites)
        // ... except when this update is likely the last one: the residual reduction of the
        // last two iterations predicts whether it reaches the tolerance, and a speculative
        // application after the final update would only delay the end of the solve.
        const double predicted = res * rate;
        const bool speculate = it < p.maxiter && !p.flexible_cg && !(it > 2 && predicted <= 3.0 * p.rtol);
        if (speculate) precondition(0, ready);
        HIP_CHECK(hipEventSynchronize(c->ev_read));
        if (host_scal(c, S_FLAG) != 0.0) {
            wait_coarse(c);
            read_red(c);  // a coarsest operator that is not SPD shows as a breakdown
            if (host_scal(c, S_COARSE) != 0.0)
                throw Fail{AMG_ERR_NOT_SPD, "coarsest operator of the last rebuild is not SPD"};
            c->err = "CG breakdown (p.Ap <= 0 or a non-finite scalar)";
            if (info) {
                inf.iters = it;
                *info = inf;
            }
            return AMG_ERR_BREAKDOWN;
        }
        const double res_prev = res;
        res = std::sqrt(host_sum(c, P_RR, nb)) / nf;
        const double ratio = res_prev > 0.0 ? res / res_prev : 1.0;
        rate = it == 1 ? ratio : std::sqrt(rate_last * ratio);  // geometric mean of the last two
        rate_last = ratio;
        if (res <= p.rtol) {
            nb = true_residual();
            res = std::sqrt(host_sum(c, P_RR, nb)) / nf;
            if (res <= p.rtol) {
                converged = true;
                break;
            }
            precondition(0, 0);  // continue from the true residual
        } else if (!speculate) {
            if (it >= p.maxiter) break;
            precondition(0, ready);
        }
        std::swap(pold, pnew);
    }
    if (!converged) {
        nb = true_residual();
        res = std::sqrt(host_sum(c, P_RR, nb)) / nf;
    }
    launch_copy(n, c->x, u, s);
    HIP_CHECK(hipStreamSynchronize(s));
    inf.iters = it;
    inf.converged = converged ? 1 : 0;
    inf.rel_res_true = res;
    if (info) *info = inf;
    return AMG_OK;
}

// ------------------------------------------------------------------ BiCGStab

// BiCGStab (van der Vorst) with one V-cycle applied on the right: the paper's Krylov
// method for its non-symmetric systems (Section 4), with the CG's stopping rule (true
// relative residual; when the recursive ||s|| or ||r|| reaches rtol the true residual is
// formed and, if it is not small enough, the method restarts from it with r^ = r).  Per
// iteration: two V-cycles, two products with the Krylov operator, and three host reads
// of dot-product partials (r^.v for alpha, ||s||, t.s and t.t for omega; r^.r and ||r||
// come with the update).  Scalars are formed on the host from partials added in
// workgroup order.
amg_status bicgstab(amg_ctx* c, const double* f, double* u, amg_solve_info* info) {
    hipStream_t s = c->stream;
    const Level& L0 = c->lv[0];
    const int n = L0.A.nrows;
    const amg_params& prm = c->prm;
    if (!c->bi_t) c->bi_t = halloc<double>(c, (size_t)n);
    if (!c->bi_sc) c->bi_sc = halloc<double>(c, (size_t)BS_COUNT);
    if (!c->bi_part) c->bi_part = halloc<double>(c, 6 * (size_t)RED_BLOCKS);
    if (!c->h_bi) {
        HIP_CHECK(hipHostMalloc((void**)&c->h_bi, (2 * (size_t)RED_BLOCKS + BS_COUNT) * sizeof(double),
                                hipHostMallocMapped | hipHostMallocCoherent));
        void* dptr = nullptr;
        HIP_CHECK(hipHostGetDevicePointer(&dptr, c->h_bi, 0));
        c->d_bi = (double*)dptr;
    }
    Csr Aout = L0.A;  // the Krylov operator: the hierarchy's pattern, the outer values
    Aout.val = c->outer_val;
    // y = A x: on the diagonal storage when it holds the Krylov operator (the Krylov SpMV
    // kernel with beta = 0 also copies x to bi_w and adds x.y partials, both unused)
    const bool on_dia = c->dia.ndiag > 0 && c->outer_val == L0.A.val;
    if (on_dia && !c->bi_w) c->bi_w = halloc<double>(c, (size_t)n);
    auto apply_A = [&](const double* xin, double* yout) {
        if (on_dia)
            launch_dia_cg_pq(n, c->dia, xin, xin, c->bi_w, yout, 1, c->rs, s);
        else
            launch_spmv<double>(Aout, xin, yout, nullptr, nullptr, s);
    };
    double *x = c->x, *r = c->r, *rh = c->r2, *p = c->pa, *v = c->q, *ph = c->z, *sv = c->zold, *sh = c->pb,
           *t = c->bi_t;
    const int nb = bi_grid(n);
    double* sc = c->bi_sc;
    // device partials, each region within its own RED_BLOCKS slots: r^.v (and the unused
    // second region the dot kernel writes), s.s, (t.s, t.t), r^.r
    double* p_rv = c->bi_part;
    double* p_ss = c->bi_part + 2 * RED_BLOCKS;
    double* p_tt = c->bi_part + 3 * RED_BLOCKS;
    double* p_rho = c->bi_part + 5 * RED_BLOCKS;
    const double* hp = c->h_bi;
    const double* hsc = c->h_bi + 2 * RED_BLOCKS;  // the scalars as the last update saw them
    auto sum = [&](int q) {
        double a = 0.0;
        for (int i = 0; i < nb; ++i) a += hp[(size_t)q * nb + i];
        return a;
    };
    auto wait = [&]() { HIP_CHECK(hipStreamSynchronize(s)); };
    auto true_residual = [&]() {  // r = f - A x; partials ||r||^2, ||f||^2 (host mirror)
        apply_A(x, t);
        launch_bi_residual(n, f, t, r, c->d_bi, nb, s);
        wait();
        return sum(0);
    };
    amg_solve_info inf{0, 0, 0.0};
    launch_copy(n, u, x, s);
    double rr = true_residual();
    const double ff = sum(1);
    if (ff == 0.0) {
        HIP_CHECK(hipMemsetAsync(u, 0, (size_t)n * sizeof(double), s));
        HIP_CHECK(hipStreamSynchronize(s));
        inf.converged = 1;
        if (info) *info = inf;
        return AMG_OK;
    }
    const double nf = std::sqrt(ff);
    double res = std::sqrt(rr) / nf;
    if (res <= prm.rtol) {
        inf.converged = 1;
        inf.rel_res_true = res;
        if (info) *info = inf;
        return AMG_OK;
    }
    // (re)start from the residual in r: r^ = r, rho = r.r, alpha = omega = 1
    auto restart = [&]() {
        d2d(rh, r, (size_t)n * sizeof(double), s);
        launch_bi_scal(BI_RESET, sc, nullptr, 0, rr, 0.0, s);
    };
    restart();
    bool fresh = true;
    int it = 0;
    bool converged = false;
    auto settle = [&]() {  // true residual; converged, or restart from it
        rr = true_residual();
        res = std::sqrt(rr) / nf;
        if (res <= prm.rtol) return true;
        restart();
        fresh = true;
        return false;
    };
    auto breakdown = [&](const char* what) {
        HIP_CHECK(hipStreamSynchronize(s));
        wait_coarse(c);
        read_red(c);  // a coarsest operator that is not SPD shows as a breakdown
        if (host_scal(c, S_COARSE) != 0.0)
            throw Fail{AMG_ERR_NOT_SPD, "coarsest operator of the last rebuild is not SPD"};
        c->err = std::string("BiCGStab breakdown: ") + what;
        if (info) {
            inf.iters = it;
            *info = inf;
        }
        return AMG_ERR_BREAKDOWN;
    };
    // One step (van der Vorst's BiCGStab, preconditioned on the right) is queued as a whole:
    // its scalars are formed on the device, and the host waits once, for the update's
    // ||r||^2 partials and flags.  (Queuing the next step's first half before that wait,
    // as the CG loop does, measured no gain here: 13.14 against 13.19 ms per 128^3 step.)
    while (it < prm.maxiter) {
        ++it;
        if (!fresh) launch_bi_scal(BI_BETA, sc, p_rho, nb, 0.0, 0.0, s);
        launch_bi_direction(n, r, v, sc, fresh ? 1 : 0, p, s);
        fresh = false;
        vcycle_apply(c, p, ph);
        {
            Trace tr(c, AMG_K_BICG_SPMV, 0);
            apply_A(ph, v);
        }
        launch_bi_dots(n, rh, v, nullptr, nullptr, p_rv, nb, s);
        launch_bi_scal(BI_ALPHA, sc, p_rv, nb, 0.0, 0.0, s);
        launch_bi_half(n, r, v, sc, sv, p_ss, nb, s);
        launch_bi_scal(BI_HALF, sc, p_ss, nb, 0.0, prm.rtol * nf, s);
        vcycle_apply(c, sv, sh);
        {
            Trace tr(c, AMG_K_BICG_SPMV, 0);
            apply_A(sh, t);
        }
        launch_bi_dots(n, t, sv, t, t, p_tt, nb, s);
        launch_bi_scal(BI_OMEGA, sc, p_tt, nb, 0.0, 0.0, s);
        launch_bi_update(n, ph, sh, sv, t, rh, sc, x, r, p_rho, c->d_bi, nb, s);
        wait();
        const int bad = (int)hsc[BS_BAD];
        if (bad & BI_BAD_RHO) return breakdown("r^.r = 0");
        if (bad & BI_BAD_RV) return breakdown("r^.v = 0");
        if (hsc[BS_HALF] != 0.0) {  // x += alpha p^ only: the half step reached the tolerance
            if (settle()) {
                converged = true;
                break;
            }
            continue;
        }
        if (bad & BI_BAD_TT) return breakdown("t.t = 0");
        if (std::sqrt(sum(0)) / nf <= prm.rtol) {
            if (settle()) {
                converged = true;
                break;
            }
            continue;
        }
        if (bad & BI_BAD_OMEGA) return breakdown("omega = 0");
    }
    if (!converged) {
        rr = true_residual();
        res = std::sqrt(rr) / nf;
    }
    launch_copy(n, x, u, s);
    HIP_CHECK(hipStreamSynchronize(s));
    inf.iters = it;
    inf.converged = converged ? 1 : 0;
    inf.rel_res_true = res;
    if (info) *info = inf;
    return AMG_OK;
}

// ------------------------------------------------------------------ context lifecycle

amg_status check_params(const amg_params& p) {
    if (p.smoother < 0 || p.smoother > 1 || p.aggregation < 0 || p.aggregation > 1 || p.precision < 0 ||
        p.precision > 1 || p.npre < 0 || p.npre > 16 || p.npost < 0 || p.npost > 16 || p.coarse_enough < 1 ||
        p.max_levels < 1 || p.max_levels > 64 || !(p.rtol > 0.0) || p.maxiter < 0 || !(p.eps_strong >= 0.0) ||
        !(p.jacobi_omega > 0.0) || p.block_size < 1 || p.block_size > 8 ||
        (p.block_size > 1 && (p.aggregation != 1 || p.smoother != 0 || p.flexible_cg != 0)) ||
        ((p.alloc == nullptr) != (p.dealloc == nullptr)))
        return AMG_ERR_ARG;
    return AMG_OK;
}

void destroy_ctx(amg_ctx* c) {
    if (!c) return;
    hipStream_t s = c->stream;
    if (c->side) (void)hipStreamSynchronize(c->side);
    (void)hipStreamSynchronize(s);
    {
        MemScope scope(&c->mem);
        for (void* p : c->hier_allocs) dfree(p, s);
        for (void* p : c->own_allocs) dfree(p, s);
        dfree(c->pend_ptr, s);
        dfree(c->pend_col, s);
    }
    mem_release(c->mem);
    if (c->h_red) (void)hipHostFree(c->h_red);
    if (c->h_bi) (void)hipHostFree(c->h_bi);
    if (c->h_flags) (void)hipHostFree(c->h_flags);
    for (hipEvent_t& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->ev_read) (void)hipEventDestroy(c->ev_read);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_inv) (void)hipEventDestroy(c->ev_inv);
    if (c->side) (void)hipStreamDestroy(c->side);
    for (auto& t : c->traced) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    delete c;
}

amg_ctx* create_ctx(const amg_params& p, void* stream) {
    amg_ctx* c = new amg_ctx();
    c->prm = p;
    c->stream = (hipStream_t)stream;
    try {
        HIP_CHECK(hipGetDevice(&c->device));
        mem_init(c->mem, c->stream, p.alloc, p.dealloc, p.alloc_user);
        MemScope scope(&c->mem);
        c->d_flags = oalloc<int>(c, F_COUNT);
        HIP_CHECK(hipHostMalloc((void**)&c->h_flags, F_COUNT * sizeof(int), hipHostMallocDefault));
        for (hipEvent_t& e : c->ev) HIP_CHECK(hipEventCreate(&e));
        HIP_CHECK(hipEventCreateWithFlags(&c->ev_read, hipEventDisableTiming));
        HIP_CHECK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        HIP_CHECK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        HIP_CHECK(hipEventCreateWithFlags(&c->ev_inv, hipEventDisableTiming));
    } catch (...) {
        destroy_ctx(c);
        throw;
    }
    return c;
}

// Runs f with c's device memory.  A HIP runtime error, or any failure while a full setup or
// a pattern change was replacing the hierarchy (its old arrays may already be freed, its
// new levels incomplete), leaves the context broken: later calls return AMG_ERR_STATE.
template <typename F>
amg_status guard(amg_ctx* c, F&& f) {
    if (c && c->broken) return AMG_ERR_STATE;
    MemScope scope(c ? &c->mem : nullptr);
    amg_status st = AMG_OK;
    try {
        return f();
    } catch (const Fail& e) {
        if (c) c->err = e.msg;
        else g_setup_err = e.msg;
        st = e.st;
    } catch (const std::bad_alloc&) {
        if (c) c->err = "host allocation failed";
        st = AMG_ERR_OOM;
    } catch (...) {
        if (c) c->err = "unexpected exception";
        st = AMG_ERR_HIP;
    }
    if (c && (st == AMG_ERR_HIP || c->replacing)) {
        c->broken = true;
        if (c->replacing) c->err += " (while replacing the hierarchy: the context must be destroyed)";
    }
    return st;
}

// Marks the scope of a full setup or pattern change on an existing context.
struct Replacing {
    amg_ctx* c;
    explicit Replacing(amg_ctx* cc) : c(cc) { c->replacing = true; }
    void done() { c->replacing = false; }
    Replacing(const Replacing&) = delete;
    Replacing& operator=(const Replacing&) = delete;
};

}  // namespace

// ======================================================================= C interface
extern "C" {

amg_status amg_params_default(amg_params* p) {
    if (!p) return AMG_ERR_ARG;
    p->smoother = 0;
    p->aggregation = 0;
    p->jacobi_omega = 0.72;
    p->eps_strong = 0.08;
    p->coarse_enough = 1024;
    p->max_levels = 12;
    p->npre = 1;
    p->npost = 1;
    p->precision = 0;
    p->rtol = 1e-8;
    p->maxiter = 100;
    p->flexible_cg = 0;
    p->block_size = 1;
    p->alloc = nullptr;
    p->dealloc = nullptr;
    p->alloc_user = nullptr;
    return AMG_OK;
}

static amg_status setup_common(amg_ctx** out, int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                               const double* val, const amg_params* p, void* stream, const Transfer* tr) {
    if (!out) return AMG_ERR_ARG;
    *out = nullptr;
    if (n <= 0 || nnz <= 0 || nnz >= ((int64_t)1 << 31) || !row_ptr || !col || !val) {
        g_setup_err = "amg_setup: invalid sizes or NULL arrays";
        return AMG_ERR_ARG;
    }
    amg_params prm;
    amg_params_default(&prm);
    if (p) prm = *p;
    if (check_params(prm) != AMG_OK) {
        g_setup_err = "amg_setup: invalid parameters";
        return AMG_ERR_ARG;
    }
    amg_ctx* c = nullptr;
    amg_status st = guard(nullptr, [&] {
        c = create_ctx(prm, stream);
        return AMG_OK;
    });
    if (st != AMG_OK) return st;
    c->transfer_given = tr != nullptr;
    st = guard(c, [&] {
        build_hierarchy(c, n, nnz, row_ptr, col, val, tr);
        return AMG_OK;
    });
    if (st != AMG_OK) {
        g_setup_err = c->err;
        destroy_ctx(c);
        return st;
    }
    *out = c;
    return AMG_OK;
}

amg_status amg_setup(amg_ctx** out, int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                     const double* val, const amg_params* p, void* hip_stream) {
    return setup_common(out, n, nnz, row_ptr, col, val, p, hip_stream, nullptr);
}

amg_status amg_setup_transfer(amg_ctx** out, int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                              const double* val, int nlev, const int32_t* const* P_ptr,
                              const int32_t* const* P_col, const double* const* P_val, const int32_t* nc,
                              const int64_t* nnzP, const amg_params* p, void* hip_stream) {
    if (nlev < 0 || (nlev > 0 && (!P_ptr || !P_col || !P_val || !nc || !nnzP))) {
        if (out) *out = nullptr;
        g_setup_err = "amg_setup_transfer: invalid transfer arrays";
        return AMG_ERR_ARG;
    }
    for (int l = 0; l < nlev; ++l)
        if (nc[l] <= 0 || nnzP[l] < 0 || !P_ptr[l] || (nnzP[l] > 0 && (!P_col[l] || !P_val[l]))) {
            if (out) *out = nullptr;
            g_setup_err = "amg_setup_transfer: invalid transfer operator";
            return AMG_ERR_ARG;
        }
    Transfer tr{nlev, P_ptr, P_col, P_val, nc, nnzP};
    return setup_common(out, n, nnz, row_ptr, col, val, p, hip_stream, &tr);
}

amg_status amg_rebuild_ex(amg_ctx* c, const double* val, amg_rebuild_mode m) {
    if (!c || !val) return AMG_ERR_ARG;
    return guard(c, [&] {
        switch (m) {
            case AMG_PARTIAL:
                partial_any(c, val);
                ++c->pol_updates;
                return AMG_OK;
            case AMG_FULL: {
                if (c->transfer_given) throw Fail{AMG_ERR_ARG, "full rebuild of a hierarchy with prescribed transfer operators"};
                const Csr A = c->lv[0].A;
                Replacing rp(c);
                build_hierarchy(c, A.nrows, A.nnz, A.ptr, A.col, val, nullptr);
                rp.done();
                return AMG_OK;
            }
            case AMG_OPERATOR_ONLY: {
                const Csr& A = c->lv[0].A;
                if (!c->outer_own) c->outer_own = halloc<double>(c, (size_t)A.nnz);
                d2d(c->outer_own, val, (size_t)A.nnz * sizeof(double), c->stream);
                c->outer_val = c->outer_own;
                ++c->pol_updates;
                return AMG_OK;
            }
        }
        throw Fail{AMG_ERR_ARG, "unknown rebuild mode"};
    });
}

amg_status amg_policy_pick(const amg_policy* p, int updates, int iters_ref, int last_iters, int last_converged,
                           amg_rebuild_mode* mode) {
    if (!p || !mode || (p->base != AMG_PARTIAL && p->base != AMG_OPERATOR_ONLY) || p->every < 0 ||
        !(p->growth >= 0.0))
        return AMG_ERR_ARG;
    bool full = p->every > 0 && updates + 1 >= p->every;
    if (p->growth > 0.0 && iters_ref > 0 && last_iters > 0 && (double)last_iters > p->growth * (double)iters_ref)
        full = true;
    if (p->base == AMG_OPERATOR_ONLY && last_iters > 0 && !last_converged) full = true;
    *mode = full ? AMG_FULL : p->base;
    return AMG_OK;
}

amg_status amg_rebuild_auto(amg_ctx* c, const double* val, const amg_policy* p, amg_rebuild_mode* taken) {
    if (!c || !val) return AMG_ERR_ARG;
    amg_rebuild_mode m;
    const amg_status st = amg_policy_pick(p, c->pol_updates, c->pol_iters_ref, c->pol_last_iters, c->pol_last_conv, &m);
    if (st != AMG_OK) return st;
    if (taken) *taken = m;
    return amg_rebuild_ex(c, val, m);
}

amg_status amg_rebuild(amg_ctx* c, const double* val, int pattern_changed) {
    if (!c || !val) return AMG_ERR_ARG;
    if (!pattern_changed) return amg_rebuild_ex(c, val, AMG_PARTIAL);
    return guard(c, [&] {
        if (!c->pend_ptr) throw Fail{AMG_ERR_ARG, "pattern_changed without a pending amg_set_pattern"};
        if (c->pend_n != c->lv[0].A.nrows || c->transfer_given) {
            if (c->transfer_given) throw Fail{AMG_ERR_ARG, "size change of a hierarchy with prescribed transfer operators"};
            const int32_t n = c->pend_n;
            const int64_t nnz = c->pend_nnz;
            int32_t* pp = c->pend_ptr;
            int32_t* pc = c->pend_col;
            c->pend_ptr = c->pend_col = nullptr;
            c->pend_n = 0;
            Replacing rp(c);
            try {
                build_hierarchy(c, n, nnz, pp, pc, val, nullptr);
            } catch (...) {
                dfree(pp, c->stream);
                dfree(pc, c->stream);
                throw;
            }
            dfree(pp, c->stream);
            dfree(pc, c->stream);
            rp.done();
            return AMG_OK;
        }
        Replacing rp(c);
        repattern(c);
        partial_any(c, val);
        rp.done();
        return AMG_OK;
    });
}

amg_status amg_set_pattern(amg_ctx* c, int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col) {
    if (!c || n <= 0 || nnz <= 0 || nnz >= ((int64_t)1 << 31) || !row_ptr || !col) return AMG_ERR_ARG;
    return guard(c, [&] {
        hipStream_t s = c->stream;
        dfree(c->pend_ptr, s);
        dfree(c->pend_col, s);
        c->pend_ptr = c->pend_col = nullptr;
        c->pend_ptr = dnew<int32_t>((size_t)n + 1, s);
        c->pend_col = dnew<int32_t>((size_t)nnz, s);
        d2d(c->pend_ptr, row_ptr, ((size_t)n + 1) * sizeof(int32_t), s);
        d2d(c->pend_col, col, (size_t)nnz * sizeof(int32_t), s);
        c->pend_n = n;
        c->pend_nnz = nnz;
        return AMG_OK;
    });
}

amg_status amg_solve(amg_ctx* c, const double* f, double* u, amg_solve_info* info) {
    if (!c || !f || !u) return AMG_ERR_ARG;
    amg_solve_info inf{0, 0, 0.0};
    const amg_status st = guard(c, [&] { return pcg(c, f, u, &inf); });
    c->pol_last_iters = st == AMG_OK ? (inf.iters > 0 ? inf.iters : 1) : (c->prm.maxiter > 0 ? c->prm.maxiter : 1);
    c->pol_last_conv = st == AMG_OK ? inf.converged : 0;
    if (c->pol_iters_ref == 0 && st == AMG_OK) c->pol_iters_ref = c->pol_last_iters;
    if (info) *info = inf;
    return st;
}

amg_status amg_solve_bicgstab(amg_ctx* c, const double* f, double* u, amg_solve_info* info) {
    if (!c || !f || !u) return AMG_ERR_ARG;
    amg_solve_info inf{0, 0, 0.0};
    const amg_status st = guard(c, [&] { return bicgstab(c, f, u, &inf); });
    c->pol_last_iters = st == AMG_OK ? (inf.iters > 0 ? inf.iters : 1) : (c->prm.maxiter > 0 ? c->prm.maxiter : 1);
    c->pol_last_conv = st == AMG_OK ? inf.converged : 0;
    if (c->pol_iters_ref == 0 && st == AMG_OK) c->pol_iters_ref = c->pol_last_iters;
    if (info) *info = inf;
    return st;
}

amg_status amg_apply_operator(amg_ctx* c, const double* x, double* y) {
    if (!c || !x || !y || x == y) return AMG_ERR_ARG;
    return guard(c, [&] {
        // the CG's Krylov SpMV in its first-iteration form (p = z = x, q = y); its p copy
        // goes to the CG's second direction vector, its p.q partials are not read
        const Level& L0 = c->lv[0];
        const int n = L0.A.nrows;
        double* w = c->pb;
        if (c->dia.ndiag > 0 && c->outer_val == L0.A.val)
            launch_dia_cg_pq(n, c->dia, x, x, w, y, 1, c->rs, c->stream);
        else if (c->prm.block_size > 1)
            launch_node_cg_pq(L0, c->prm.block_size, c->outer_val, x, x, w, y, 1, c->rs, c->stream);
        else
            launch_cg_pq(L0.A, c->outer_val, x, x, w, y, 1, c->rs, c->stream);
        return AMG_OK;
    });
}

// ------------------------------------------------------------------ allocation-free operator
//
// amg_apply_operator_noalloc runs the kernels of amg_apply_operator with their scratch (the
// copy of p the Krylov SpMV writes, and its p.q block partials) in this file-scope device
// array instead of the context's CG vectors.  Each device holds its own copy from the load
// of the library to the end of the process; its address on a device is taken once, with
// that device current, and only that address is handed to kernels.
namespace {
constexpr size_t NOALLOC_ROWS = (size_t)1 << 23;        // most rows (the p copy)
constexpr size_t NOALLOC_PART = (size_t)1 << 20;        // doubles for the reduction partials
static __device__ __align__(256) double scratch[NOALLOC_ROWS + NOALLOC_PART];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

double* scratch_on(int dev) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) throw Fail{AMG_ERR_ARG, "device index out of range"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* ptr = nullptr;
        HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = (double*)ptr;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

amg_status amg_vcycle(amg_ctx* c, const double* r, double* z) {
    if (!c || !r || !z) return AMG_ERR_ARG;
    return guard(c, [&] {
        vcycle_apply(c, r, z);
        return AMG_OK;
    });
}

amg_status amg_apply_operator_noalloc(amg_ctx* c, const double* x, double* y) {
    if (!c || !x || !y || x == y) return AMG_ERR_ARG;
    if (c->broken) return AMG_ERR_STATE;
    // no MemScope: nothing here allocates
    try {
        int dev = -1;
        HIP_CHECK(hipGetDevice(&dev));
        if (dev != c->device) throw Fail{AMG_ERR_ARG, "amg_apply_operator_noalloc: the context's device is not current"};
        const Level& L0 = c->lv[0];
        const int n = L0.A.nrows;
        if ((size_t)n > NOALLOC_ROWS)
            throw Fail{AMG_ERR_ARG, "amg_apply_operator_noalloc: " + std::to_string(n) + " rows exceed its " +
                                        std::to_string(NOALLOC_ROWS) + "-row scratch"};
        double* sp = scratch_on(dev);
        RedScratch rs;
        rs.cap = (int)((NOALLOC_PART - S_COUNT) / 5);
        rs.part = sp + NOALLOC_ROWS;
        rs.host = nullptr;
        double* w = sp;  // the p copy
        if (c->dia.ndiag > 0 && c->outer_val == L0.A.val)
            launch_dia_cg_pq(n, c->dia, x, x, w, y, 1, rs, c->stream);
        else if (c->prm.block_size > 1)
            launch_node_cg_pq(L0, c->prm.block_size, c->outer_val, x, x, w, y, 1, rs, c->stream);
        else
            launch_cg_pq(L0.A, c->outer_val, x, x, w, y, 1, rs, c->stream);
        return AMG_OK;
    } catch (const Fail& e) {
        c->err = e.msg;
        if (e.st == AMG_ERR_HIP) c->broken = true;
        return e.st;
    } catch (...) {
        c->err = "unexpected exception";
        return AMG_ERR_HIP;
    }
}

amg_status amg_destroy(amg_ctx* c) {
    if (!c) return AMG_ERR_ARG;
    destroy_ctx(c);
    return AMG_OK;
}

const char* amg_last_error(const amg_ctx* c) { return c ? c->err.c_str() : g_setup_err.c_str(); }

amg_status amg_num_levels(const amg_ctx* c, int* L) {
    if (!c || !L) return AMG_ERR_ARG;
    if (c->broken) return AMG_ERR_STATE;
    *L = (int)c->lv.size();
    return AMG_OK;
}

amg_status amg_level_dims(const amg_ctx* c, int l, int64_t* dims) {
    if (!c || !dims || l < 0 || l >= (int)c->lv.size()) return AMG_ERR_ARG;
    if (c->broken) return AMG_ERR_STATE;
    const Level& L = c->lv[(size_t)l];
    dims[0] = L.A.nrows;
    dims[1] = L.A.nnz;
    dims[2] = L.P.ncols;
    dims[3] = L.P.nnz;
    dims[4] = L.AP.nnz;
    return AMG_OK;
}

amg_status amg_level_format(const amg_ctx* c, int l, int* ndiag, int* nread, int* plane) {
    if (!c || !ndiag || l < 0 || l >= (int)c->lv.size()) return AMG_ERR_ARG;
    if (c->broken) return AMG_ERR_STATE;
    *ndiag = l == 0 ? c->dia.ndiag : 0;
    if (nread) *nread = (l == 0 && c->dia.off.sym) ? (c->dia.ndiag + 1) / 2 : *ndiag;
    if (plane) *plane = l == 0 ? c->dia.march_a : 0;
    return AMG_OK;
}

amg_status amg_export_level(const amg_ctx* cc, int l, int32_t* agg, uint8_t* strong, int32_t* A_ptr, int32_t* A_col,
                            double* A_val, int32_t* P_ptr, int32_t* P_col, double* P_val, double* m) {
    amg_ctx* c = const_cast<amg_ctx*>(cc);
    if (!c || l < 0 || l >= (int)c->lv.size()) return AMG_ERR_ARG;
    return guard(c, [&] {
        hipStream_t s = c->stream;
        const Level& L = c->lv[(size_t)l];
        const bool mx = mixed(c);
        auto d2h = [&](void* dst, const void* src, size_t bytes) {
            if (dst && src && bytes) HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
        };
        auto vals = [&](double* dst, const double* v64, const float* v32, int64_t n) {
            if (!dst || n == 0) return;
            if (mx && v32) {
                double* tmp = dnew<double>((size_t)n, s);
                launch_cast_f2d(n, v32, tmp, s);
                d2h(dst, tmp, (size_t)n * sizeof(double));
                HIP_CHECK(hipStreamSynchronize(s));
                dfree(tmp, s);
            } else {
                d2h(dst, v64, (size_t)n * sizeof(double));
            }
        };
        const int32_t n = L.A.nrows;
        if (l == 0) ensure_a0_csr(c);
        d2h(agg, L.agg, (size_t)n * sizeof(int32_t));
        d2h(strong, L.strong, (size_t)L.A.nnz);
        d2h(A_ptr, L.A.ptr, ((size_t)n + 1) * sizeof(int32_t));
        d2h(A_col, L.A.col, (size_t)L.A.nnz * sizeof(int32_t));
        vals(A_val, L.A.val, L.A.val32, L.A.nnz);
        if (L.P.nrows > 0) {
            d2h(P_ptr, L.P.ptr, ((size_t)n + 1) * sizeof(int32_t));
            d2h(P_col, L.P.col, (size_t)L.P.nnz * sizeof(int32_t));
            vals(P_val, L.P.val, L.P.val32, L.P.nnz);
            vals(m, L.m, L.m32, (int64_t)n * c->prm.block_size);
        }
        HIP_CHECK(hipStreamSynchronize(s));
        return AMG_OK;
    });
}

amg_status amg_export_coarse_inverse(const amg_ctx* cc, double* inv) {
    amg_ctx* c = const_cast<amg_ctx*>(cc);
    if (!c || !inv) return AMG_ERR_ARG;
    return guard(c, [&] {
        wait_coarse(c);
        HIP_CHECK(hipMemcpyAsync(inv, c->cinv, (size_t)c->nL * c->nL * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
        HIP_CHECK(hipStreamSynchronize(c->stream));
        return AMG_OK;
    });
}

amg_status amg_phase_times(const amg_ctx* cc, double* out) {
    amg_ctx* c = const_cast<amg_ctx*>(cc);
    if (!c || !out) return AMG_ERR_ARG;
    return guard(c, [&] {
        if (c->phase_pending) {
            HIP_CHECK(hipEventSynchronize(c->ev[3]));
            float a = 0, b = 0, d = 0, t = 0;
            HIP_CHECK(hipEventElapsedTime(&a, c->ev[0], c->ev[1]));
            HIP_CHECK(hipEventElapsedTime(&b, c->ev[1], c->ev[2]));
            HIP_CHECK(hipEventElapsedTime(&d, c->ev[2], c->ev[3]));
            HIP_CHECK(hipEventElapsedTime(&t, c->ev[0], c->ev[3]));
            double ph[8] = {0, 0, 0, a, b, d, t, 0};
            std::memcpy(c->phase_ms, ph, sizeof(ph));
            c->phase_pending = false;
        }
        std::memcpy(out, c->phase_ms, sizeof(c->phase_ms));
        return AMG_OK;
    });
}

amg_status amg_trace(amg_ctx* c, unsigned mask, int level) {
    if (!c) return AMG_ERR_ARG;
    c->trace_mask = mask;
    c->trace_level = level;
    for (auto& row : c->trace_seen) row.fill(0);
    return AMG_OK;
}

amg_status amg_trace_every(amg_ctx* c, int every) {
    if (!c || every < 1) return AMG_ERR_ARG;
    c->trace_every = every;
    for (auto& row : c->trace_seen) row.fill(0);
    return AMG_OK;
}

// Sums the traced intervals per class (nlev == 0) or per level and class into ms/launches.
static amg_status trace_collect(amg_ctx* c, int nlev, double* ms, int64_t* launches) {
    return guard(c, [&] {
        const int rows = nlev > 0 ? nlev : 1;
        for (int k = 0; k < rows * AMG_K_COUNT; ++k) {
            ms[k] = 0.0;
            launches[k] = 0;
        }
        HIP_CHECK(hipStreamSynchronize(c->stream));
        if (c->side) HIP_CHECK(hipStreamSynchronize(c->side));  // the coarsest inverse's events
        for (auto& t : c->traced) {
            float x = 0.f;
            HIP_CHECK(hipEventElapsedTime(&x, t.a, t.b));
            const int row = nlev > 0 ? std::min(std::max(t.level, 0), nlev - 1) : 0;
            if (t.cls >= 0 && t.cls < AMG_K_COUNT) {
                ms[row * AMG_K_COUNT + t.cls] += x;
                launches[row * AMG_K_COUNT + t.cls] += 1;
            }
            c->ev_pool.push_back(t.a);
            c->ev_pool.push_back(t.b);
        }
        c->traced.clear();
        return AMG_OK;
    });
}

amg_status amg_trace_read(amg_ctx* c, double* ms, int64_t* launches) {
    if (!c || !ms || !launches) return AMG_ERR_ARG;
    return trace_collect(c, 0, ms, launches);
}

amg_status amg_trace_read_levels(amg_ctx* c, int nlev, double* ms, int64_t* launches) {
    if (!c || !ms || !launches || nlev <= 0) return AMG_ERR_ARG;
    return trace_collect(c, nlev, ms, launches);
}

amg_status amg_level_storage(const amg_ctx* c, int l, int* out) {
    if (!c || !out || l < 0 || l >= (int)c->lv.size()) return AMG_ERR_ARG;
    if (c->broken) return AMG_ERR_STATE;
    const Level& L = c->lv[(size_t)l];
    out[0] = L.A.c16 != nullptr;
    out[1] = L.P.c16 != nullptr;
    out[2] = L.R.c16 != nullptr;
    out[3] = L.A.rpb;
    out[4] = L.P.rpb;
    out[5] = L.R.rpb;
    out[6] = (c->tail > 0 && l >= c->tail) ? 1 : 0;
    out[7] = mixed(c) ? 4 : 8;
    out[8] = L.ngal.nblk > 0 ? 1 : 0;
    out[9] = L.nagg != nullptr ? 1 : 0;
    return AMG_OK;
}

amg_status amg_logcoef7_assemble(int32_t nx, int32_t ny, int32_t nz, const double* theta, double* val,
                                 void* hip_stream) {
    if (nx <= 0 || ny <= 0 || nz <= 0 || !theta || !val) return AMG_ERR_ARG;
    return guard(nullptr, [&] {
        launch_logcoef7_assemble(nx, ny, nz, theta, val, (hipStream_t)hip_stream);
        return AMG_OK;
    });
}

amg_status amg_logcoef7_adjoint(int32_t nx, int32_t ny, int32_t nz, const double* theta, const double* u,
                                const double* lambda, double* grad, void* hip_stream) {
    if (nx <= 0 || ny <= 0 || nz <= 0 || !theta || !u || !lambda || !grad) return AMG_ERR_ARG;
    return guard(nullptr, [&] {
        launch_logcoef7_adjoint(nx, ny, nz, theta, u, lambda, grad, (hipStream_t)hip_stream);
        return AMG_OK;
    });
}

}  // extern "C"
