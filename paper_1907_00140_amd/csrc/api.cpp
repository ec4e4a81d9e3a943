// Host runtime behind the C-ABI of include/chl.h: argument checks, device
// validation and rank renumbering, the build schedule (rank-prefix pruning
// levels, grown by teams of workgroups or by the batched persistent kernel,
// then the main phase; or the plain one-root-per-launch form), growth of the
// label pool, label assembly, queries, statistics and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

using namespace chl;

namespace {

void* dflt_alloc(size_t b, void*) {
    void* p = nullptr;
    return hipMalloc(&p, b) == hipSuccess ? p : nullptr;
}
void dflt_free(void* p, void*) { (void)hipFree(p); }

const chl_allocator kDefaultAlloc = {dflt_alloc, dflt_free, nullptr};

// Allocations of one call; everything not released is freed on exit.
struct Arena {
    chl_allocator a;
    std::vector<void*> ptrs;
    bool oom = false;
    explicit Arena(const chl_allocator& al) : a(al) {}
    template <typename T>
    T* get(size_t count) {
        size_t bytes = std::max<size_t>(count * sizeof(T), 256);
        void* p = a.alloc(bytes, a.ctx);
        if (!p) { oom = true; return nullptr; }
        ptrs.push_back(p);
        return (T*)p;
    }
    void drop(void* p) {
        auto it = std::find(ptrs.begin(), ptrs.end(), p);
        if (it != ptrs.end()) { a.free(p, a.ctx); ptrs.erase(it); }
    }
    void release(void* p) {
        auto it = std::find(ptrs.begin(), ptrs.end(), p);
        if (it != ptrs.end()) ptrs.erase(it);
    }
    ~Arena() {
        for (void* p : ptrs) a.free(p, a.ctx);
    }
};

#define HIPCHK(x)                                  \
    do {                                           \
        if ((x) != hipSuccess) return CHL_ERR_HIP; \
    } while (0)
#define OOMCHK(p)                     \
    do {                              \
        if (!(p)) return CHL_ERR_OOM; \
    } while (0)

int check_device() {
    static int cached = 1;  // 1 = unknown
    if (cached != 1) return cached;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CHL_ERR_NO_DEVICE;
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return CHL_ERR_NO_DEVICE;
    cached = std::strncmp(pr.gcnArchName, "gfx950", 6) == 0 ? 0 : CHL_ERR_NO_DEVICE;
    return cached;
}

struct Timer {
    hipEvent_t a, b;
    hipStream_t s;
    explicit Timer(hipStream_t st) : s(st) {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        (void)hipEventRecord(a, s);
    }
    double stop() {
        record_end();
        (void)hipEventSynchronize(b);
        return elapsed();
    }
    void record_end() { (void)hipEventRecord(b, s); }
    double elapsed() {   // after the end event has completed
        float ms = 0;
        (void)hipEventElapsedTime(&ms, a, b);
        return ms;
    }
    ~Timer() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
};

// Small device-to-host readbacks (control words, error flags, samples) go
// through pinned host memory, so that several of them queue on the stream
// and complete with one synchronisation. Each host thread holds one block
// while it lives and hands it back to a process-wide free list when it ends,
// so that threads that come and go (the server's build workers) reuse blocks
// instead of allocating pinned memory, which can stall the device.
struct HostCtl {
    int32_t c32[16];
    unsigned long long c64[4];
    int64_t smp[64];
    int64_t sums[4];
};
std::mutex g_hc_mu;
std::vector<HostCtl*> g_hc_free;
struct HostCtlLease {
    HostCtl* h = nullptr;
    ~HostCtlLease() {
        if (!h) return;
        std::lock_guard<std::mutex> lk(g_hc_mu);
        g_hc_free.push_back(h);
    }
};
HostCtl* host_ctl() {
    static thread_local HostCtlLease lease;
    if (!lease.h) {
        {
            std::lock_guard<std::mutex> lk(g_hc_mu);
            if (!g_hc_free.empty()) {
                lease.h = g_hc_free.back();
                g_hc_free.pop_back();
            }
        }
        if (!lease.h && hipHostMalloc((void**)&lease.h, sizeof(HostCtl), hipHostMallocDefault) != hipSuccess)
            lease.h = nullptr;
    }
    return lease.h;
}

// ---------------------------------------------------------------- tuning
struct TuneKey {
    int32_t n;
    int64_t m;
    int32_t maxw;
    int mode;
    uint64_t sig;
    bool operator<(const TuneKey& o) const {
        return std::tie(n, m, maxw, mode, sig) < std::tie(o.n, o.m, o.maxw, o.mode, o.sig);
    }
};
struct TuneVal {
    int k, wg;          // trees in flight, workgroup size
    int64_t delta;      // bucket width
    bool small = false; // main phase by the small-tree kernel (LDS), the others as fallback
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;
std::map<TuneKey, bool> g_prune_keep;   // outcome of the pruning probe

// Device state shared by one build.
struct Build {
    int32_t n = 0;
    int64_t m = 0;
    int key_bits = 32;
    int32_t maxw = 1;
    RGraph g{};
    // control words
    int32_t* ctl32 = nullptr;          // [0] next_root [1] stop [2] nfailed [3] err
    unsigned long long* ctl64 = nullptr;  // [0] pool cursor [1] first failed base
    int32_t* failed = nullptr;         // [n]
    int32_t* roots = nullptr;          // [n] root list for resumed / probe runs
    int32_t* far2 = nullptr;           // [n] plain form
    int32_t* gstate = nullptr;         // plain form state words
    Pool pool{};
    int64_t* stats = nullptr;
    // rank-prefix pruning: labels found so far, grouped by rank position
    const int64_t* poff = nullptr;
    const uint64_t* plab = nullptr;
    uint32_t* pmin = nullptr;            // lower bound of each vertex's group distances
    int32_t dmaj = 0;                    // plab entries (dist << 32) | hub, groups by distance (TreeParams::dmaj)
    const uint64_t* plab_hub = nullptr;  // the same groups in hub order, (hub << 32) | dist
    int32_t hashdh = 0;                  // main phase: root distances hashed (TreeParams::hashdh)
    int32_t pbound = 0;                  // prune with the hubs [0, pbound)
    int32_t partner = 0;                 // combined graph of a directed build (TreeParams::partner)
    unsigned long long cursor_base = 0;  // pool entries kept before the main tree phase
    int32_t grown = 0;                   // roots [0, grown) done before the main phase
    double kernel_ms = 0;                // event-timed production tree launches
    int64_t kernel_launches = 0;
    uint64_t sig = 0;                    // graph and ranking signature (tuning caches)
    unsigned long long last_used = 0;    // pool cursor after the last tree launch
    // the rank-prefix levels as grown (chl_stats::levels ...)
    int nlev = 0;
    int64_t lv_end[CHL_MAX_LEVELS] = {};
    double lv_ms[CHL_MAX_LEVELS] = {};
    int64_t lv_team[CHL_MAX_LEVELS] = {};
    // pruned construction of the Hybrid (TreeParams::dhg / rlab)
    uint32_t* dhg = nullptr;
    int64_t* rlab = nullptr;
    void record_level(int32_t end, double ms, int team) {
        if (nlev < CHL_MAX_LEVELS) { lv_end[nlev] = end; lv_ms[nlev] = ms; lv_team[nlev] = team; nlev++; }
    }
};

// labels emitted by a pruning level above which the next level is only
// two or four times as large (else eight times)
constexpr unsigned long long LEVEL_LABELS_X2 = 1ull << 21;

size_t slot_bytes(int32_t n, int key_bits) {
    return (size_t)n * (key_bits / 8 + 4 + 12) + (size_t)((n + 7) / 8) * 4;
}

int alloc_slots(Arena& A, Build& B, int k, Slots& s, hipStream_t st) {
    s.k = k;
    s.stride = B.n;
    s.fstride = (B.n + 7) / 8;
    size_t kb = (size_t)B.key_bits / 8;
    s.key = A.get<uint8_t>((size_t)k * B.n * kb);
    s.flags = A.get<uint32_t>((size_t)k * s.fstride);
    s.touched = A.get<int32_t>((size_t)k * B.n);
    s.lists = A.get<int32_t>((size_t)k * 3 * B.n);
    if (!s.key || !s.flags || !s.touched || !s.lists) return CHL_ERR_OOM;
    HIPCHK(hipMemsetAsync(s.key, 0xFF, (size_t)k * B.n * kb, st));
    HIPCHK(hipMemsetAsync(s.flags, 0, (size_t)k * s.fstride * 4, st));
    return 0;
}

void free_slots(Arena& A, Slots& s) {
    A.drop(s.key);
    A.drop(s.flags);
    A.drop(s.touched);
    A.drop(s.lists);
    s = Slots{};
}

int grow_pool(Arena& A, Build& B, unsigned long long used, unsigned long long want, hipStream_t st) {
    unsigned long long cap = std::max<unsigned long long>(want, 2 * B.pool.cap);
    Pool np = B.pool;
    np.cap = cap;
    np.v = A.get<int32_t>(cap);
    np.hub = A.get<int32_t>(cap);
    np.dist = A.get<int32_t>(cap);
    if (!np.v || !np.hub || !np.dist) return CHL_ERR_OOM;
    if (used) {
        HIPCHK(hipMemcpyAsync(np.v, B.pool.v, used * 4, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(np.hub, B.pool.hub, used * 4, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(np.dist, B.pool.dist, used * 4, hipMemcpyDeviceToDevice, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    A.drop(B.pool.v);
    A.drop(B.pool.hub);
    A.drop(B.pool.dist);
    B.pool = np;
    return 0;
}

TreeParams params(Build& B, const Slots& s, int64_t delta, int early, const int32_t* roots,
                  int32_t nroots, int32_t root_base = 0) {
    TreeParams p{};
    p.g = B.g;
    p.s = s;
    p.pool = B.pool;
    p.delta = delta;
    p.early_term = early;
    p.next_root = B.ctl32 + 0;
    p.stop = B.ctl32 + 1;
    p.nfailed = B.ctl32 + 2;
    p.err = B.ctl32 + 3;
    p.failed = B.failed;
    p.far2 = B.far2;
    p.nroots = nroots;
    p.roots = roots;
    p.stats = B.stats;
    p.root_base = root_base;
    // many small trees per slot: take the roots several at a time so that
    // the queue counter is not contended (rank order is kept within 16)
    p.pop_batch = std::max(1, std::min(16, nroots / std::max(1, 8 * s.k)));
    p.poff = B.poff;
    p.plab = B.plab;
    p.pmin = B.pmin;
    p.dmaj = B.dmaj;
    p.hashdh = B.hashdh;
    p.ovf = B.far2;
    p.novf = B.ctl32 + 5;
    p.pbound = B.pbound;
    p.partner = B.partner;
    p.dhg = B.dhg;
    p.rlab = B.rlab;
    // teams and groups on one XCD each: the first levels' HBM-side fetches
    // fall 2.4x (R-MAT 20 level 0: 74.8 -> 30.8 GB), their time does not
    p.xcd_map = 1;
    return p;
}

// Teams of workgroups (one tree per team at a time) for a launch over few
// large trees; the team slots are the first nteams slots of the Slots passed.
struct TeamCfg {
    int size = 0;              // workgroups per team
    int nteams = 0;
    long long* tstate = nullptr;  // [nteams][TEAM_WORDS]
    int32_t* far2 = nullptr;      // [nteams][n]
};

// Groups of GROUP_TREES trees grown together by teams of workgroups (one
// group per team at a time), their keys vertex-major.
struct GroupCfg {
    int size = 0;                 // workgroups per team
    int ngroups = 0;              // teams
    Slots s{};                    // key: ngroups * n * GROUP_TREES keys; touched, lists as for teams
    long long* gstate = nullptr;  // [ngroups][GROUP_WORDS]
    int32_t* far2 = nullptr;      // [ngroups][n]
    uint32_t* gmask = nullptr;    // [ngroups][2n]
};

size_t group_bytes(int32_t n, int key_bits) {
    return (size_t)n * ((size_t)GROUP_TREES * key_bits / 8 + 8 + 16 + 4) + (size_t)GROUP_WORDS * 8;
}

int alloc_groups(Arena& A, Build& B, int ngroups, GroupCfg& gc, hipStream_t st) {
    const size_t n = (size_t)B.n;
    const size_t kb = (size_t)B.key_bits / 8;
    gc.s.k = ngroups;
    gc.s.stride = B.n;
    gc.s.fstride = 0;
    gc.s.flags = nullptr;
    gc.s.key = A.get<uint8_t>((size_t)ngroups * n * GROUP_TREES * kb);
    gc.s.touched = A.get<int32_t>((size_t)ngroups * n);
    gc.s.lists = A.get<int32_t>((size_t)ngroups * 3 * n);
    gc.far2 = A.get<int32_t>((size_t)ngroups * n);
    gc.gmask = A.get<uint32_t>((size_t)ngroups * 2 * n);
    gc.gstate = A.get<long long>((size_t)ngroups * GROUP_WORDS);
    if (!gc.s.key || !gc.s.touched || !gc.s.lists || !gc.far2 || !gc.gmask || !gc.gstate) return CHL_ERR_OOM;
    HIPCHK(hipMemsetAsync(gc.s.key, 0xFF, (size_t)ngroups * n * GROUP_TREES * kb, st));
    HIPCHK(hipMemsetAsync(gc.gmask, 0, (size_t)ngroups * 2 * n * 4, st));
    return 0;
}

void free_groups(Arena& A, GroupCfg& gc) {
    A.drop(gc.s.key);
    A.drop(gc.s.touched);
    A.drop(gc.s.lists);
    A.drop(gc.far2);
    A.drop(gc.gmask);
    A.drop(gc.gstate);
    gc = GroupCfg{};
}

// Run the batched kernel (or the team kernel when team is set, the group
// kernel when grp is set) over roots
// (NULL = all, in rank order; roots_in_place: the list is already in B.roots
// on the stream) until every root has emitted, growing the pool when it
// fills up.
int run_batched(Arena& A, Build& B, const Slots& s, int wg, int64_t delta, int early,
                const int32_t* roots_host, int32_t nroots, hipStream_t st, int* launches,
                int phase = 0, int32_t root_base = 0, const TeamCfg* team = nullptr,
                bool roots_in_place = false, const GroupCfg* grp = nullptr, int small_wgs = 0) {
    std::vector<int32_t> pending;
    std::vector<int32_t> overflow;      // roots the small or hashed kernel gave up (grown afterwards)
    // main phase and its probes with the root's prefix distances hashed
    const bool hs = B.hashdh && B.poff && B.pbound > 0 && (phase == 0 || phase == 1) && !team && !grp && !small_wgs;
    const int32_t* dev_roots = nullptr;
    if (roots_host) {
        HIPCHK(hipMemcpyAsync(B.roots, roots_host, (size_t)nroots * 4, hipMemcpyHostToDevice, st));
        dev_roots = B.roots;
    } else if (roots_in_place) {
        dev_roots = B.roots;
    }
    for (;;) {
        HIPCHK(hipMemsetAsync(B.ctl32, 0, 12, st));          // next_root, stop, nfailed
        HIPCHK(hipMemsetAsync(B.ctl32 + 5, 0, 4, st));       // overflow count of the small kernel
        HIPCHK(hipMemsetAsync(B.ctl64 + 1, 0xFF, 8, st));     // fail_base = none
        TreeParams p = params(B, grp ? grp->s : s, delta, early, dev_roots, nroots, root_base);
        if (small_wgs) p.pop_batch = std::max(1, std::min(16, nroots / std::max(1, 8 * small_wgs)));
        HostCtl* hc = host_ctl();
        if (!hc) return CHL_ERR_HIP;
        if (team) HIPCHK(hipMemsetAsync(team->tstate, 0, (size_t)team->nteams * TEAM_WORDS * 8, st));
        if (grp) HIPCHK(hipMemsetAsync(grp->gstate, 0, (size_t)grp->ngroups * GROUP_WORDS * 8, st));
        {
            // the launch is timed by events; the control words are read back
            // behind it, and one synchronisation completes both
            Timer tk(st);
            if (small_wgs) {
                if (launch_tree_small(p, B.key_bits, small_wgs, B.far2, B.ctl32 + 5, st)) return CHL_ERR_HIP;
            } else if (grp) {
                if (launch_tree_group(p, B.key_bits, 1024, grp->size, grp->ngroups, grp->gstate, grp->far2,
                                      grp->gmask, st))
                    return CHL_ERR_HIP;
            } else if (team) {
                if (launch_tree_team(p, B.key_bits, wg, team->size, team->nteams, team->tstate, team->far2, st))
                    return CHL_ERR_HIP;
            } else if (launch_tree_batched(p, B.key_bits, wg, phase, st)) {
                return CHL_ERR_HIP;
            }
            tk.record_end();
            HIPCHK(hipMemcpyAsync(hc->c32, B.ctl32, 24, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(hc->c64, B.ctl64, 16, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            const double ms = tk.elapsed();
            if (phase != 1) { B.kernel_ms += ms; B.kernel_launches++; }
        }
        (*launches)++;
        int32_t c32[6];
        unsigned long long c64[2];
        std::memcpy(c32, hc->c32, sizeof(c32));
        std::memcpy(c64, hc->c64, sizeof(c64));
        B.last_used = c64[0];
        if (c32[3] & ERR_BIT_INVALID) return CHL_ERR_INVALID_ARG;
        if (c32[3] & ERR_BIT_TEAM) return CHL_ERR_HIP;
        if ((small_wgs || hs) && c32[5] > 0) {
            const size_t no = overflow.size();
            overflow.resize(no + (size_t)std::min(c32[5], B.n));
            HIPCHK(hipMemcpy(overflow.data() + no, B.far2, (overflow.size() - no) * 4, hipMemcpyDeviceToHost));
        }
        if (!(c32[3] & ERR_BIT_POOL)) break;
        // pool full: keep what fitted, then resume with the failed roots and
        // the roots the queue had not handed out yet
        unsigned long long used = std::min(c64[0], c64[1]);
        int32_t nf = c32[2];
        std::vector<int32_t> failed(nf);
        if (nf) HIPCHK(hipMemcpy(failed.data(), B.failed, (size_t)nf * 4, hipMemcpyDeviceToHost));
        int32_t next = std::min(c32[0], nroots);
        std::vector<int32_t> rest;
        rest.reserve(nf + (nroots - next));
        rest.insert(rest.end(), failed.begin(), failed.end());
        if (roots_host) {
            rest.insert(rest.end(), roots_host + next, roots_host + nroots);
        } else if (dev_roots) {
            std::vector<int32_t> tail((size_t)(nroots - next));
            if (!tail.empty())
                HIPCHK(hipMemcpy(tail.data(), B.roots + next, tail.size() * 4, hipMemcpyDeviceToHost));
            rest.insert(rest.end(), tail.begin(), tail.end());
        } else {
            for (int32_t r = next; r < nroots; r++) rest.push_back(root_base + r);
        }
        // grow by doubling: label counts per root fall steeply with rank, so
        // the roots seen so far do not predict the rest
        unsigned long long est = used + 1024;
        if (int r = grow_pool(A, B, used, est, st)) return r;
        int32_t errclr = c32[3] & ~ERR_BIT_POOL;
        HIPCHK(hipMemcpyAsync(B.ctl64, &used, 8, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(B.ctl32 + 3, &errclr, 4, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        pending.swap(rest);
        nroots = (int32_t)pending.size();
        roots_host = pending.data();
        HIPCHK(hipMemcpyAsync(B.roots, roots_host, (size_t)nroots * 4, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        dev_roots = B.roots;
        if (nroots == 0) break;
    }
    if (!overflow.empty()) {
        std::sort(overflow.begin(), overflow.end());   // rank order
        const int32_t hsave = B.hashdh;
        B.hashdh = 0;                                  // the dense array for these roots
        const int r = run_batched(A, B, s, wg, delta, early, overflow.data(), (int32_t)overflow.size(), st, launches,
                                  phase);
        B.hashdh = hsave;
        return r;
    }
    return 0;
}

int run_plain(Arena& A, Build& B, const Slots& s, int wg, int64_t delta, int early,
              const std::vector<int32_t>& sel, hipStream_t st, int* launches) {
    int grid = plain_grid_size(B.key_bits, wg);
    if (grid <= 0) return CHL_ERR_HIP;
    grid = std::min(grid, std::max(1, (B.n + wg - 1) / wg) * 4);
    const int32_t CH = 1024;
    std::vector<int32_t> todo;
    const int32_t nr = sel.empty() ? B.n : (int32_t)sel.size();
    for (int32_t r0 = 0; r0 < nr; r0 += CH) {
        todo.clear();
        for (int32_t r = r0; r < std::min(nr, r0 + CH); r++) todo.push_back(sel.empty() ? r : sel[r]);
        while (!todo.empty()) {
            HIPCHK(hipMemsetAsync(B.ctl32, 0, 12, st));
            HIPCHK(hipMemsetAsync(B.ctl64 + 1, 0xFF, 8, st));
            for (int32_t r : todo) {
                TreeParams p = params(B, s, delta, early, nullptr, 0);
                if (launch_tree_plain(p, B.key_bits, wg, grid, r, B.gstate, st)) return CHL_ERR_HIP;
                (*launches)++;
            }
            int32_t c32[4];
            unsigned long long c64[2];
            HIPCHK(hipMemcpyAsync(c32, B.ctl32, 16, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(c64, B.ctl64, 16, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (!(c32[3] & ERR_BIT_POOL)) break;
            // the pool filled up: keep what fitted, grow, redo the roots that failed
            unsigned long long used = std::min(c64[0], c64[1]);
            int32_t nf = c32[2];
            std::vector<int32_t> failed(nf);
            if (nf) HIPCHK(hipMemcpy(failed.data(), B.failed, (size_t)nf * 4, hipMemcpyDeviceToHost));
            if (int r = grow_pool(A, B, used, used + 1024, st)) return r;
            int32_t errclr = c32[3] & ~ERR_BIT_POOL;
            HIPCHK(hipMemcpyAsync(B.ctl64, &used, 8, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(B.ctl32 + 3, &errclr, 4, hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
            std::sort(failed.begin(), failed.end());
            todo.swap(failed);
        }
    }
    return 0;
}

// A signature of the input: a few row offsets, arcs and ranking entries
// sampled at fixed positions. sample_graph queues the sample and its
// read-back on the stream; graph_signature mixes it once the stream has been
// synchronised.
int sample_graph(const chl_graph* g, const int32_t* order, int64_t* dev_tmp, hipStream_t st) {
    HostCtl* hc = host_ctl();
    if (!hc) return CHL_ERR_HIP;
    std::memset(hc->smp, 0, sizeof(hc->smp));
    if (launch_sample_input(g->n, g->n_arcs, g->row_ptr, g->col, g->w, order, dev_tmp, st) ||
        hipMemcpyAsync(hc->smp, dev_tmp, sizeof(hc->smp), hipMemcpyDeviceToHost, st) != hipSuccess)
        return CHL_ERR_HIP;
    return CHL_OK;
}

uint64_t graph_signature(const chl_graph* g) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t x) { h = (h ^ x) * 1099511628211ull; };
    mix((uint64_t)g->n);
    mix((uint64_t)g->n_arcs);
    HostCtl* hc = host_ctl();
    if (!hc) return h;
    for (int i = 0; i < 64; i++) mix((uint64_t)hc->smp[i]);
    return h;
}

}  // namespace

static int chl_build_impl(const chl_graph* g, const int32_t* order, const chl_build_opts* opts_in,
                          const chl_allocator* alloc_in, void* stream, chl_labels** out, bool directed);
static int chl_build_directed_impl(const chl_graph* g, const int32_t* order, const chl_build_opts* opts_in,
                                   const chl_allocator* alloc_in, void* stream, chl_labels** out);

// ====================================================================== ABI
extern "C" {

const char* chl_error_string(int code) {
    switch (code) {
        case CHL_OK: return "ok";
        case CHL_ERR_INVALID_ARG: return "invalid argument";
        case CHL_ERR_OOM: return "out of device memory";
        case CHL_ERR_HIP: return "HIP runtime error";
        case CHL_ERR_DIST_OVERFLOW: return "a label distance does not fit in int32";
        case CHL_ERR_NO_DEVICE: return "no gfx950 device";
        case CHL_ERR_BUSY: return "request rejected: over budget or queue full";
        default: return "unknown error";
    }
}

void chl_build_opts_default(chl_build_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->mode = CHL_MODE_BATCHED;
    o->early_term = 1;
    o->stats = 1;
    o->autotune = 1;
}

int chl_build(const chl_graph* g, const int32_t* order, const chl_build_opts* opts,
              const chl_allocator* alloc, void* stream, chl_labels** out) {
    // launches are checked with hipGetLastError: drop an error that an
    // earlier call on this thread left behind
    (void)hipGetLastError();
    try {
        return chl_build_impl(g, order, opts, alloc, stream, out, false);
    } catch (...) {
        return CHL_ERR_OOM;
    }
}

int chl_build_directed(const chl_graph* g, const int32_t* order, const chl_build_opts* opts,
                       const chl_allocator* alloc, void* stream, chl_labels** out) {
    (void)hipGetLastError();
    try {
        return chl_build_directed_impl(g, order, opts, alloc, stream, out);
    } catch (...) {
        return CHL_ERR_OOM;
    }
}

int chl_labels_directed(const chl_labels* h, int64_t* in_total) {
    if (!h) return CHL_ERR_INVALID_ARG;
    if (in_total) *in_total = h->directed ? h->in_total : h->total;
    return h->directed ? 1 : 0;
}

int chl_labels_export_in(const chl_labels* h, int64_t* offsets, int32_t* hub_pos, int32_t* dist, int to_host,
                         void* stream) {
    if (!h || !h->directed) return CHL_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    hipMemcpyKind k = to_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (offsets) HIPCHK(hipMemcpyAsync(offsets, h->in_offsets, (size_t)(h->n + 1) * 8, k, st));
    if (hub_pos && h->in_total) HIPCHK(hipMemcpyAsync(hub_pos, h->in_hub_pos, (size_t)h->in_total * 4, k, st));
    if (dist && h->in_total) HIPCHK(hipMemcpyAsync(dist, h->in_dist, (size_t)h->in_total * 4, k, st));
    if (to_host) HIPCHK(hipStreamSynchronize(st));
    return CHL_OK;
}

int chl_labels_info(const chl_labels* h, int32_t* n, int64_t* total) {
    if (!h) return CHL_ERR_INVALID_ARG;
    if (n) *n = h->n;
    if (total) *total = h->total;
    return CHL_OK;
}

int chl_labels_export(const chl_labels* h, int64_t* offsets, int32_t* hub_pos, int32_t* dist,
                      int to_host, void* stream) {
    if (!h) return CHL_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    hipMemcpyKind k = to_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (offsets) HIPCHK(hipMemcpyAsync(offsets, h->offsets, (size_t)(h->n + 1) * 8, k, st));
    if (hub_pos && h->total) HIPCHK(hipMemcpyAsync(hub_pos, h->hub_pos, (size_t)h->total * 4, k, st));
    if (dist && h->total) HIPCHK(hipMemcpyAsync(dist, h->dist, (size_t)h->total * 4, k, st));
    if (to_host) HIPCHK(hipStreamSynchronize(st));
    return CHL_OK;
}

int chl_labels_hub_vertex(const chl_labels* h, int32_t* hub_vertex, int to_host, void* stream) {
    if (!h || !hub_vertex) return CHL_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(hub_vertex, h->order, (size_t)h->n * 4,
                          to_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
    if (to_host) HIPCHK(hipStreamSynchronize(st));
    return CHL_OK;
}

int chl_query(const chl_labels* hc, const int32_t* pairs, int64_t q, int64_t* out, void* stream) {
    if (!hc || q < 0 || (q > 0 && (!pairs || !out))) return CHL_ERR_INVALID_ARG;
    if (q == 0) return CHL_OK;
    chl_labels* h = const_cast<chl_labels*>(hc);
    hipStream_t st = (hipStream_t)stream;
    (void)hipGetLastError();
    // the error word is per handle: concurrent queries on one handle serialise here
    std::lock_guard<std::mutex> lk(h->qmu);
    HIPCHK(hipMemsetAsync(h->qerr, 0, 4, st));
    double avg = h->n ? (double)h->total / h->n : 1.0;
    const bool dir = h->directed != 0;
    if (launch_query(h->n, h->offsets, h->hub_pos, h->dist, dir ? h->in_offsets : h->offsets,
                     dir ? h->in_hub_pos : h->hub_pos, dir ? h->in_dist : h->dist, pairs, q, out, h->qerr, avg, st))
        return CHL_ERR_HIP;
    int32_t e = 0;
    HIPCHK(hipMemcpyAsync(&e, h->qerr, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return e ? CHL_ERR_INVALID_ARG : CHL_OK;
}

int chl_build_stats(const chl_labels* h, chl_stats* totals, int64_t* per_root, int to_host, void* stream) {
    if (!h) return CHL_ERR_INVALID_ARG;
    if (per_root && !h->per_root) return CHL_ERR_INVALID_ARG;
    if (totals) *totals = h->st;
    if (per_root) {
        hipStream_t st = (hipStream_t)stream;
        HIPCHK(hipMemcpyAsync(per_root, h->per_root, (size_t)h->n * STAT_COLS * 8,
                              to_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
        if (to_host) HIPCHK(hipStreamSynchronize(st));
    }
    return CHL_OK;
}

void chl_labels_free(chl_labels* h) {
    if (!h) return;
    auto f = [&](void* p) { if (p) h->alloc.free(p, h->alloc.ctx); };
    f(h->offsets);
    f(h->hub_pos);
    f(h->dist);
    f(h->order);
    f(h->per_root);
    f(h->qerr);
    f(h->in_offsets);
    f(h->in_hub_pos);
    f(h->in_dist);
    delete h;
}

}  // extern "C"

// ====================================================================== build
static int pick_params(Arena& A, Build& B, const chl_graph* g, const chl_build_opts& o,
                       hipStream_t st, int& k, int& wg, int64_t& delta, bool& small, double& tune_ms);

// The rank-prefix levels of a batched build (see chl_build_impl): grows the
// trees of the roots [0, grown) and leaves their labels in the pool, the
// prefix groups in B.poff / B.plab and B.pbound = prefix size (0 when the
// probe drops pruning).
static int run_levels(Arena& A, Build& B, const chl_build_opts& o, void* scan_tmp, hipStream_t st,
                      int& launches, int32_t& grown) {
    const int32_t n = B.n;
    const double wm = 0.5 * (1.0 + B.maxw);
    // default prefix: n/64 hubs, at least 64, at most 8192: each level
    // adds latency, each prefix hub saves work in every later tree, and
    // there are more later trees on larger graphs (R-MAT 16: 1024 hubs
    // build 4% faster than 4096; R-MAT 20: 4096 run the main phase 2.8x
    // faster than 2048, and 8192 in 18.2 ms instead of 32.7, for a last
    // level [2048, 8192) of 9.4 ms instead of [2048, 4096) of 3.7)
    const int32_t gdef = std::min<int32_t>(MAX_PREFIX, std::max<int32_t>(64, n / 64));
    const int32_t gmax = std::min<int32_t>(o.prune_hubs > 0 ? o.prune_hubs : gdef, n / 2);
    // prefix labels grouped by vertex, double-buffered: each level's
    // labels extend the groups of the levels before it
    int32_t* pcount = A.get<int32_t>(n);
    int32_t* pfill = A.get<int32_t>(n);
    int64_t* poff[2] = {A.get<int64_t>((size_t)n + 1), A.get<int64_t>((size_t)n + 1)};
    B.pmin = A.get<uint32_t>(n);
    if (A.oom) return CHL_ERR_OOM;
    HIPCHK(hipMemsetAsync(B.pmin, 0xFF, (size_t)n * 4, st));
    uint64_t* plab[2] = {nullptr, nullptr};
    size_t plab_cap[2] = {0, 0};
    uint64_t* byd = nullptr;            // the groups ordered by distance
    size_t byd_cap = 0;
    int cur = -1;                       // buffer holding the groups so far
    unsigned long long grouped = 0;     // pool entries grouped so far
    // trees in flight and workgroup size of the levels: 512 and 1024
    // unless the caller fixed them (a caller that shares the device, such
    // as the server, caps both)
    const int kcap = o.roots_in_flight > 0 ? std::min(512, o.roots_in_flight) : 512;
    const int lwg = o.wg_size ? o.wg_size : 1024;
    const int kpre = std::min(kcap, std::max(1, (int)(std::min<size_t>(4096, (size_t)(1ull << 33) / std::max<size_t>(1, slot_bytes(n, B.key_bits))))));
    Slots s1{};
    if (int r = alloc_slots(A, B, kpre, s1, st)) return r;
    HIPCHK(hipMemsetAsync(B.ctl64, 0, 8, st));
    auto regroup = [&]() -> int {
        const unsigned long long used = B.last_used;
        const int nx = cur < 0 ? 0 : 1 - cur;
        if (used > plab_cap[nx]) {
            if (plab[nx]) A.drop(plab[nx]);
            plab_cap[nx] = std::max<size_t>(used, 2 * plab_cap[nx]);
            plab[nx] = A.get<uint64_t>(plab_cap[nx]);
            if (!plab[nx]) return CHL_ERR_OOM;
        }
        if (launch_prefix_extend(n, B.pool, grouped, used, pcount, cur < 0 ? nullptr : poff[cur],
                                 cur < 0 ? nullptr : plab[cur], poff[nx], plab[nx], pfill, scan_tmp, st) ||
            launch_group_min(B.pool, grouped, used, B.pmin, st))
            return CHL_ERR_HIP;
        cur = nx;
        grouped = used;
        B.poff = poff[cur];
        B.plab = plab[cur];
        B.plab_hub = plab[cur];
        B.dmaj = 0;
        B.cursor_base = used;
        // the kernels read the groups ordered by distance (a pruning test
        // stops at the first entry that cannot give a shorter walk); the
        // groups in hub order stay for the next extension
        if (used > byd_cap) {
            if (byd) A.drop(byd);
            byd_cap = std::max<size_t>(used, 2 * byd_cap);
            byd = A.get<uint64_t>(byd_cap);
            if (!byd) return CHL_ERR_OOM;
        }
        if (launch_swap_halves(plab[cur], byd, used, st) ||
            launch_segsort_u64(byd, poff[cur], n, (int64_t)used, nullptr, st))
            return CHL_ERR_HIP;
        B.plab = byd;
        B.dmaj = 1;
        return 0;
    };
    // level 0
    int32_t g = std::min<int32_t>(16, gmax);
    // the first levels hold the largest trees: 1024-thread workgroups,
    // teams of them for the narrow levels. Buckets of a quarter of the
    // mean weight for the unpruned trees of level 0 (wider ones cost
    // re-relaxation: R-MAT 20's level 0 relaxes 3.85x the oracle's arcs
    // at half the mean weight, 3.6x at a quarter; narrower ones cost more
    // team barriers than they save: an eighth relaxes 3.2x and takes as
    // long, a sixteenth 2.6x and takes longer), twice the mean weight for
    // the pruned levels, whose trees are smaller and latency bound
    // (measured on R-MAT scales 16 and 20)
    const int64_t dl = std::max<int64_t>(1, (int64_t)(wm / 4));
    const int64_t dl1 = std::max<int64_t>(1, (int64_t)(2 * wm));
    // levels with fewer trees than the device holds workgroups of that
    // size run as teams of workgroups, one tree per team
    const int tcap = o.team_wgs == 1 || lwg < 512 ? 0 : team_capacity(B.key_bits, lwg);
    auto team_shape = [&](int32_t nr, TeamCfg& tc) -> bool {
        if (tcap < 2 || nr <= 0 || 2 * nr > tcap) return false;
        tc.size = std::min(o.team_wgs ? o.team_wgs : 16, tcap / nr);
        tc.nteams = std::min<int>(std::min<int>(nr, tcap / std::max(1, tc.size)), s1.k);
        return tc.size >= 2;
    };
    // team buffers for the largest team launch of any level schedule
    int tmax = 0;
    for (int32_t f : {2, 4, 8})
        for (int32_t a = g, b = std::min<int32_t>(gmax, f * g); a < gmax; a = b, b = std::min<int32_t>(gmax, f * b)) {
            TeamCfg tc;
            if (team_shape(b - a, tc)) tmax = std::max(tmax, tc.nteams);
        }
    {
        TeamCfg tc;
        if (team_shape(g, tc)) tmax = std::max(tmax, tc.nteams);
    }
    int32_t* tfar2 = tmax ? A.get<int32_t>((size_t)tmax * n) : nullptr;
    long long* tstate = tmax ? A.get<long long>((size_t)tmax * TEAM_WORDS) : nullptr;
    // sort keys and segment bounds of a wide level's root order
    uint64_t* lkeys = A.get<uint64_t>((size_t)std::max<int32_t>(1, gmax));
    int64_t* loff = A.get<int64_t>(2);
    if (A.oom) return CHL_ERR_OOM;
    auto team_for = [&](int32_t nr, TeamCfg& tc) -> const TeamCfg* {
        if (!team_shape(nr, tc) || tc.nteams > tmax) return nullptr;
        tc.far2 = tfar2;
        tc.tstate = tstate;
        return &tc;
    };
    // Levels of 64 to 256 trees run as groups of GROUP_TREES trees with
    // vertex-major keys (the trees of a level reach largely the same
    // vertices), when the groups' state fits GROUP_MAX_BYTES. Measured on
    // R-MAT 20 against one tree per team: levels [64,128), [128,256) and
    // [256,512) take 26.8, 32.4 and 26.1 ms instead of 32.0, 44.6 and 38.6;
    // the levels of 16 and 32 trees, whose few groups span 128 to 256
    // workgroups each, are slower as groups (their hubs land on one workgroup
    // for all 16 trees, and every round's barrier has 128-256 members), and
    // so are levels of 512 trees, which share few vertices. The group
    // buffers are kept across levels and grown when a level needs more.
    GroupCfg gcfg;
    const bool groups_on = o.group_levels >= 0 && o.team_wgs != 1 && lwg == 1024;
    constexpr size_t GROUP_MAX_BYTES = (size_t)8 << 30;
    auto group_for = [&](int32_t nr, int32_t pbound, GroupCfg& gc) -> const GroupCfg* {
        if (!groups_on || nr < 4 * GROUP_TREES || nr > 256 || pbound > GROUP_MAX_PREFIX) return nullptr;
        const int ng = (nr + GROUP_TREES - 1) / GROUP_TREES;
        if ((size_t)ng * group_bytes(n, B.key_bits) > GROUP_MAX_BYTES) return nullptr;
        const int cap = group_capacity(B.key_bits, pbound);
        if (cap < ng) return nullptr;
        if (gcfg.ngroups < ng) {
            if (gcfg.ngroups) free_groups(A, gcfg);
            if (alloc_groups(A, B, ng, gcfg, st)) return nullptr;
        }
        gc = gcfg;
        gc.ngroups = ng;
        gc.s.k = ng;
        gc.size = std::max(1, std::min(256, cap / ng));
        return &gc;
    };
    TeamCfg tc0;
    GroupCfg gc0;
    const GroupCfg* gcp0 = group_for(g, 0, gc0);
    const TeamCfg* tcp0 = gcp0 ? nullptr : team_for(g, tc0);
    double ms0 = B.kernel_ms;
    if (int r = run_batched(A, B, s1, lwg, dl, o.early_term, nullptr, g, st, &launches, 2, 0, tcp0, false, gcp0))
        return r;
    B.record_level(g, B.kernel_ms - ms0, gcp0 ? -gcp0->size : tcp0 ? tcp0->size : 1);
    if (int r = regroup()) return r;
    unsigned long long level_labels = B.cursor_base;
    grown = g;
    bool probed = false;
    bool keep = o.prune_hubs > 0 || !o.autotune;
    const TuneKey pkey{n, B.m, B.maxw, -1, B.sig};
    if (!keep) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_prune_keep.find(pkey);
        if (it != g_prune_keep.end()) keep = it->second, probed = true;
    }
    if (!keep && !probed) {
        // keep pruning only if the 16-hub prefix cuts the work of a
        // rank-stratified sample of later trees at least in half (it does
        // not on graphs whose top-ranked vertices cover few shortest
        // paths, e.g. degree-ranked grids)
        const int32_t p0 = std::min<int32_t>(gmax, n - 1), nprobe = std::min<int32_t>(128, n - p0);
        std::vector<int32_t> probe;
        for (int32_t i = 0; i < nprobe; i++) probe.push_back(p0 + (int32_t)((int64_t)(n - p0) * i / nprobe));
        int64_t* sv = B.stats;
        int64_t* tmp_stats = sv ? nullptr : A.get<int64_t>((size_t)n * STAT_COLS);
        if (!sv && !tmp_stats) return CHL_ERR_OOM;
        B.stats = sv ? sv : tmp_stats;
        int64_t work[2] = {0, 0};
        std::vector<int64_t> rows((size_t)n * STAT_COLS);
        for (int on = 0; on < 2; on++) {
            B.pbound = on ? g : 0;
            HIPCHK(hipMemcpyAsync(B.ctl64, &B.cursor_base, 8, hipMemcpyHostToDevice, st));
            if (int r = run_batched(A, B, s1, lwg, dl, o.early_term, probe.data(), (int32_t)probe.size(), st,
                                    &launches, 1))
                return r;
            HIPCHK(hipMemcpy(rows.data(), B.stats, rows.size() * 8, hipMemcpyDeviceToHost));
            for (int32_t r : probe) work[on] += rows[(size_t)r * STAT_COLS + 1];
        }
        // the probe roots' statistics rows are written again by the main phase
        if (!sv) A.drop(tmp_stats);
        B.stats = sv;
        HIPCHK(hipMemcpyAsync(B.ctl64, &B.cursor_base, 8, hipMemcpyHostToDevice, st));
        keep = 2 * work[1] < work[0];
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_prune_keep[pkey] = keep;
    }
    B.pbound = 0;
    if (keep) {
        int32_t last_f = 0;
        while (g < gmax) {
            // a level whose trees emitted many labels did much work: grow
            // the prefix slowly, so that the next level is pruned by more
            // hubs, by 2 and 4 in turn (every level also costs a regrouping
            // of the table and a launch tail: on R-MAT 20, 2, 4, 2, 4, 2
            // built 3.5% faster than 2 throughout; 4 throughout, or 4 first,
            // was slower); after a small level, whose time is the latency of
            // its trees, grow by 8, to have fewer levels (the labels of a
            // root do not depend on the schedule, so neither does the
            // schedule itself). The first pruned level of a directed build
            // grows by 4: its combined graph's second level [16, 128) ends
            // with a few large trees on small teams, and [16, 64) on teams
            // of 5 builds the directed R-MAT 16 5% faster (the undirected
            // R-MAT 16 is 7% slower that way)
            const int32_t f = g == 16 && B.partner ? 4
                              : level_labels >= LEVEL_LABELS_X2 ? (last_f == 2 ? 4 : 2)
                                                                : 8;
            last_f = f;
            const int32_t g2 = std::min<int32_t>(gmax, f * g);
            B.pbound = g;
            TeamCfg tc;
            GroupCfg gc;
            const unsigned long long before = B.cursor_base;
            const GroupCfg* gcp = group_for(g2 - g, g, gc);
            const TeamCfg* tcp = gcp ? nullptr : team_for(g2 - g, tc);
            // a level of more trees than slots runs them in waves, and a large
            // tree that starts late sets the level's end: start the trees
            // whose roots carry the most prefix labels first (a directed
            // build counts those of the partner h ^ 1, whose labels prune
            // h's tree), a cheap predictor of a large pruned tree (R-MAT 16,
            // level [128, 1024): rank correlation 0.45 with the tree's
            // duration; builds 4.5% faster, the directed R-MAT 16 build 5%).
            // The order is computed and sorted on the stream, into B.roots.
            // (a group keeps rank order: roots close in rank reach the same
            // vertices)
            const bool ordered = !tcp && !gcp;
            if (ordered && launch_level_order(B.poff, g, g2, B.partner, lkeys, loff, B.roots, st))
                return CHL_ERR_HIP;
            const double ms1 = B.kernel_ms;
            if (int r = run_batched(A, B, s1, lwg, dl1, o.early_term, nullptr, g2 - g, st, &launches, 2, g, tcp,
                                    ordered, gcp))
                return r;
            B.record_level(g2, B.kernel_ms - ms1, gcp ? -gcp->size : tcp ? tcp->size : 1);
            if (int r = regroup()) return r;
            level_labels = B.cursor_base - before;
            g = g2;
        }
        grown = g;
        B.pbound = g;
    }
    free_slots(A, s1);
    if (gcfg.ngroups) free_groups(A, gcfg);
    if (tfar2) A.drop(tfar2);
    if (tstate) A.drop(tstate);
    B.grown = grown;
    if (o.root_count > 0) {
        // a root subset keeps only its own trees' labels
        B.cursor_base = 0;
        HIPCHK(hipMemsetAsync(B.ctl64, 0, 8, st));
        if (B.stats) HIPCHK(hipMemsetAsync(B.stats, 0, (size_t)n * STAT_COLS * 8, st));
    }
    return 0;
}

// The Hybrid construction (Section 4.2.1) on one device, for the roots
// [B.grown, n) that follow the rank-prefix levels. PLaNT trees grow in
// windows of consecutive roots; the first window whose vertex relaxations
// per label (Psi) exceed the threshold ends PLaNT. The remaining roots grow
// in supersteps as pruned Dijkstra trees with rank queries (Algorithm 1,
// batched kernel phase 3), pruned by the distance query over every label of
// the roots before the superstep, grouped by vertex; trees of one superstep
// run concurrently, so each superstep ends with the cleaning query DQ_Clean
// (Algorithm 2) over its labels, and the kept ones join the groups. The
// result is the CHL, the same labels as PLaNT trees for every root.
static int run_hybrid(Arena& A, Build& B, const chl_build_opts& o, const Slots& s, int wg, int64_t delta,
                      int small_wgs, void* scan_tmp, hipStream_t st, int* launches, chl_stats& S) {
    const int32_t n = B.n;
    int32_t lo = B.grown;
    // per-root statistics feed the Psi monitor
    int64_t* own_stats = nullptr;
    if (!B.stats) {
        own_stats = A.get<int64_t>((size_t)n * STAT_COLS);
        if (!own_stats) return CHL_ERR_OOM;
        HIPCHK(hipMemsetAsync(own_stats, 0, (size_t)n * STAT_COLS * 8, st));
        B.stats = own_stats;
    }
    std::vector<int64_t> rows;
    // Psi is taken over the last n/64 roots (at least 64) of a window, the
    // most recent trees; the first window holds that many roots and each
    // next one twice as many, up to 8 trees per slot, so that the switch
    // point is resolved finely early on and the slots stay busy later
    const int64_t recent = std::max<int64_t>(64, n / 64);
    const int64_t wmax = std::max<int64_t>(recent, 8 * (int64_t)s.k);
    int64_t win = recent;
    S.hybrid_switch = n;
    while (lo < n) {
        const int32_t hi = (int32_t)std::min<int64_t>(n, (int64_t)lo + win);
        if (int r = run_batched(A, B, s, wg, delta, o.early_term, nullptr, hi - lo, st, launches, 0, lo, nullptr,
                                false, nullptr, small_wgs))
            return r;
        rows.resize((size_t)(hi - lo) * STAT_COLS);
        HIPCHK(hipMemcpy(rows.data(), B.stats + (size_t)lo * STAT_COLS, rows.size() * 8, hipMemcpyDeviceToHost));
        int64_t relaxed = 0, labels = 0;
        for (int32_t i = (int32_t)std::max<int64_t>(0, (int64_t)(hi - lo) - recent); i < hi - lo; i++) {
            relaxed += rows[(size_t)i * STAT_COLS];
            labels += rows[(size_t)i * STAT_COLS + 2];
        }
        const double psi = (double)relaxed / (double)std::max<int64_t>(1, labels);
        lo = hi;
        if (psi > (double)o.hybrid_psi) {
            S.hybrid_switch = lo;
            S.hybrid_psi = psi;
            break;
        }
        win = std::min<int64_t>(wmax, 2 * win);
    }
    if (lo >= n) {
        if (own_stats) { A.drop(own_stats); B.stats = nullptr; }
        return 0;
    }

    // ---- pruned construction of the roots [lo, n)
    double clean_ms = 0;
    int32_t* count = A.get<int32_t>(n);
    int32_t* fill = A.get<int32_t>(n);
    int64_t* toff[2] = {A.get<int64_t>((size_t)n + 1), A.get<int64_t>((size_t)n + 1)};
    uint64_t* tlab[2] = {nullptr, nullptr};
    size_t tcap[2] = {0, 0};
    B.dhg = A.get<uint32_t>((size_t)s.k * n);
    B.rlab = A.get<int64_t>((size_t)2 * n);
    const int cwg = clean_workgroups(n, n);
    uint32_t* dc = A.get<uint32_t>((size_t)cwg * n);
    int64_t* kept_dev = A.get<int64_t>(1);
    if (A.oom) return CHL_ERR_OOM;
    HIPCHK(hipMemsetAsync(B.dhg, 0xFF, (size_t)s.k * n * 4, st));
    HIPCHK(hipMemsetAsync(dc, 0xFF, (size_t)cwg * n * 4, st));
    // groups of the pool entries [0, to) into buffer b, from the groups of
    // [0, from) in (off_old, lab_old) (NULL: none, from = 0)
    auto extend = [&](const int64_t* off_old, const uint64_t* lab_old, unsigned long long from,
                      unsigned long long to, int b) -> int {
        if (to > tcap[b]) {
            if (tlab[b]) A.drop(tlab[b]);
            tcap[b] = std::max<size_t>(to, 2 * tcap[b]);
            tlab[b] = A.get<uint64_t>(tcap[b]);
            if (!tlab[b]) return CHL_ERR_OOM;
        }
        if (launch_group_sizes(n, off_old, count, st)) return CHL_ERR_HIP;
        if (launch_prefix_extend(n, B.pool, off_old ? from : 0, to, count, off_old, lab_old, toff[b], tlab[b], fill,
                                 scan_tmp, st))
            return CHL_ERR_HIP;
        return 0;
    };
    // every label so far: the levels' groups (B.poff, the pool entries
    // [0, B.cursor_base)) and the PLaNT windows' entries after them
    unsigned long long grouped = B.last_used;
    const unsigned long long lev = B.poff ? B.cursor_base : 0;
    if (int r = extend(B.poff, B.dmaj ? B.plab_hub : B.plab, lev, grouped, 0)) return r;
    if (!B.pmin) {
        B.pmin = A.get<uint32_t>(n);
        if (!B.pmin) return CHL_ERR_OOM;
        HIPCHK(hipMemsetAsync(B.pmin, 0xFF, (size_t)n * 4, st));
        if (launch_group_min(B.pool, 0, grouped, B.pmin, st)) return CHL_ERR_HIP;
    } else if (launch_group_min(B.pool, lev, grouped, B.pmin, st)) {
        return CHL_ERR_HIP;
    }
    int cur = 0;
    int64_t x = std::max<int64_t>(64, 2 * (int64_t)s.k);
    HostCtl* hc = host_ctl();
    if (!hc) return CHL_ERR_HIP;
    // the pruned trees read the groups ordered by distance, as the other
    // trees do; the groups in hub order serve the extensions and the cleaning
    uint64_t* byd = nullptr;
    size_t byd_cap = 0;
    while (lo < n) {
        const int32_t hi = (int32_t)std::min<int64_t>(n, (int64_t)lo + x);
        if (grouped > byd_cap) {
            if (byd) A.drop(byd);
            byd_cap = std::max<size_t>(grouped, 2 * byd_cap);
            byd = A.get<uint64_t>(byd_cap);
            if (!byd) return CHL_ERR_OOM;
        }
        if (launch_swap_halves(tlab[cur], byd, grouped, st) ||
            launch_segsort_u64(byd, toff[cur], n, (int64_t)grouped, nullptr, st))
            return CHL_ERR_HIP;
        B.poff = toff[cur];
        B.plab = byd;
        B.dmaj = 1;
        B.pbound = lo;
        if (int r = run_batched(A, B, s, wg, delta, o.early_term, nullptr, hi - lo, st, launches, 3, lo)) return r;
        const unsigned long long used = B.last_used;
        const unsigned long long cnt = used - grouped;
        S.hybrid_emitted += (int64_t)cnt;
        S.hybrid_supersteps++;
        Timer tc(st);
        const int nx = 1 - cur;
        // the superstep's labels join the groups uncleaned: a redundant
        // label's witness may be a label of the same superstep
        if (int r = extend(toff[cur], tlab[cur], grouped, used, nx)) return r;
        int32_t* keep = A.get<int32_t>(std::max<unsigned long long>(1, cnt));
        int64_t* pos = A.get<int64_t>(cnt + 1);
        void* stmp = A.get<uint8_t>(scan_temp_bytes((int64_t)std::max<unsigned long long>(1, cnt)));
        int32_t* tv = A.get<int32_t>(std::max<unsigned long long>(1, cnt));
        int32_t* th = A.get<int32_t>(std::max<unsigned long long>(1, cnt));
        int32_t* td = A.get<int32_t>(std::max<unsigned long long>(1, cnt));
        if (A.oom) return CHL_ERR_OOM;
        if (launch_clean(lo, hi, n, B.rlab, B.pool, grouped, toff[nx], tlab[nx], dc, keep, B.stats, st))
            return CHL_ERR_HIP;
        if (launch_compact(B.pool, grouped, cnt, keep, pos, stmp, tv, th, td, st)) return CHL_ERR_HIP;
        HIPCHK(hipMemsetAsync(kept_dev, 0, 8, st));
        if (cnt) HIPCHK(hipMemcpyAsync(kept_dev, pos + cnt, 8, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(hc->c64, kept_dev, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        const unsigned long long kept = hc->c64[0];
        if (kept) {
            HIPCHK(hipMemcpyAsync(B.pool.v + grouped, tv, kept * 4, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(B.pool.hub + grouped, th, kept * 4, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(B.pool.dist + grouped, td, kept * 4, hipMemcpyDeviceToDevice, st));
        }
        const unsigned long long end = grouped + kept;
        HIPCHK(hipMemcpyAsync(B.ctl64, &end, 8, hipMemcpyHostToDevice, st));
        // the groups again, from the kept labels only
        if (int r = extend(toff[cur], tlab[cur], grouped, end, nx)) return r;
        if (launch_group_min(B.pool, grouped, end, B.pmin, st)) return CHL_ERR_HIP;
        clean_ms += tc.stop();
        A.drop(keep);
        A.drop(pos);
        A.drop(stmp);
        A.drop(tv);
        A.drop(th);
        A.drop(td);
        S.hybrid_removed += (int64_t)(cnt - kept);
        grouped = end;
        B.last_used = end;
        cur = nx;
        lo = hi;
        x *= 2;
    }
    S.hybrid_clean_ms = clean_ms;
    B.dhg = nullptr;
    B.rlab = nullptr;
    B.poff = toff[cur];
    B.plab = tlab[cur];
    B.dmaj = 0;
    if (own_stats) { A.drop(own_stats); B.stats = nullptr; }
    return 0;
}

static int chl_build_impl(const chl_graph* g, const int32_t* order, const chl_build_opts* opts_in,
                          const chl_allocator* alloc_in, void* stream, chl_labels** out, bool directed) {
    if (!g || !order || !out) return CHL_ERR_INVALID_ARG;
    if (g->n < 1 || g->n > 0x7FFFFFFE || g->n_arcs < 0 || g->n_arcs > 0xFFFFFFFFll) return CHL_ERR_INVALID_ARG;
    if (!g->row_ptr || (g->n_arcs > 0 && (!g->col || !g->w))) return CHL_ERR_INVALID_ARG;
    chl_build_opts o;
    chl_build_opts_default(&o);
    if (opts_in) o = *opts_in;
    if (o.mode != CHL_MODE_BATCHED && o.mode != CHL_MODE_PLAIN) return CHL_ERR_INVALID_ARG;
    if (o.wg_size != 0 && o.wg_size != 64 && o.wg_size != 128 && o.wg_size != 256 && o.wg_size != 512 &&
        o.wg_size != 1024)
        return CHL_ERR_INVALID_ARG;
    if (o.mode == CHL_MODE_PLAIN && o.wg_size != 0 && o.wg_size != 256 && o.wg_size != 512) return CHL_ERR_INVALID_ARG;
    if (o.mode == CHL_MODE_PLAIN && o.wg_size == 1024) return CHL_ERR_INVALID_ARG;
    if (o.roots_in_flight < 0 || o.delta < 0) return CHL_ERR_INVALID_ARG;
    if (o.root_count < 0) return CHL_ERR_INVALID_ARG;
    if (o.prune_hubs > MAX_PREFIX) return CHL_ERR_INVALID_ARG;
    if (o.team_wgs < 0 || o.team_wgs > 16) return CHL_ERR_INVALID_ARG;
    if (o.group_levels < -1 || o.group_levels > 0) return CHL_ERR_INVALID_ARG;
    if (o.small_trees < -1 || o.small_trees > 1) return CHL_ERR_INVALID_ARG;
    // the Hybrid construction: batched form, complete undirected builds
    if (o.hybrid_psi < 0) return CHL_ERR_INVALID_ARG;
    if (o.hybrid_psi > 0 && (o.mode != CHL_MODE_BATCHED || o.root_count > 0 || directed)) return CHL_ERR_INVALID_ARG;
    if (o.root_count > 0) {
        if (o.root_stride < 1 || o.root_begin < 0 || o.root_begin >= g->n) return CHL_ERR_INVALID_ARG;
        if ((int64_t)o.root_begin + (int64_t)(o.root_count - 1) * o.root_stride >= g->n) return CHL_ERR_INVALID_ARG;
    }
    if (int r = check_device()) return r;
    chl_allocator al = alloc_in ? *alloc_in : kDefaultAlloc;
    if (!al.alloc || !al.free) return CHL_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    Arena A(al);
    Build B;
    B.n = g->n;
    B.m = g->n_arcs;
    B.partner = directed ? 1 : 0;
    const int32_t n = g->n;
    chl_stats S{};
    S.n = n;

    // ---- validation and renumbering
    Timer tprep(st);
    B.ctl32 = A.get<int32_t>(16);
    B.ctl64 = A.get<unsigned long long>(4);
    int32_t* pos = A.get<int32_t>(n);
    int32_t* cnt = A.get<int32_t>(n);
    int64_t* rrow = A.get<int64_t>((size_t)n + 1);
    int64_t* rdeg = A.get<int64_t>(n);
    uint64_t* rarc = A.get<uint64_t>((size_t)std::max<int64_t>(1, B.m));
    void* scan_tmp = A.get<uint8_t>(scan_temp_bytes(std::max<int64_t>(n, 1)));
    int32_t* hub_order = A.get<int32_t>(n);
    if (A.oom) return CHL_ERR_OOM;
    HIPCHK(hipMemsetAsync(B.ctl32, 0, 64, st));
    HIPCHK(hipMemsetAsync(B.ctl64, 0, 32, st));
    HIPCHK(hipMemsetAsync(cnt, 0, (size_t)n * 4, st));
    int32_t* err = B.ctl32 + 3;
    int32_t* maxw = B.ctl32 + 4;
    if (launch_validate(n, B.m, g->row_ptr, g->col, g->w, order, pos, cnt, err, maxw, st)) return CHL_ERR_HIP;
    HostCtl* hc0 = host_ctl();
    if (!hc0) return CHL_ERR_HIP;
    HIPCHK(hipMemcpyAsync(hc0->c32, err, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hc0->c32[0]) return CHL_ERR_INVALID_ARG;
    B.maxw = std::max(1, hc0->c32[1]);
    if (launch_rank_degrees(n, g->row_ptr, order, rdeg, st)) return CHL_ERR_HIP;
    if (launch_scan_i64(rdeg, rrow, n, scan_tmp, st)) return CHL_ERR_HIP;
    if (launch_renumber(n, B.m, g->row_ptr, g->col, g->w, order, pos, rrow, rarc, st)) return CHL_ERR_HIP;
    if (launch_segsort_u64(rarc, rrow, n, B.m, nullptr, st)) return CHL_ERR_HIP;
    if (!directed && launch_check_symmetric(n, B.m, rrow, rarc, err, st)) return CHL_ERR_HIP;
    HIPCHK(hipMemcpyAsync(hub_order, order, (size_t)n * 4, hipMemcpyDeviceToDevice, st));
    // the tuner caches' input signature is sampled here (the input is valid),
    // so that its read-back completes with the symmetry check's
    int64_t* smp = A.get<int64_t>(64);
    if (!smp) return CHL_ERR_OOM;
    if (int r = sample_graph(g, order, smp, st)) return r;
    HIPCHK(hipMemcpyAsync(hc0->c32, err, 4, hipMemcpyDeviceToHost, st));
    tprep.record_end();
    // 32-bit keys are exact when no simple path can reach 2^31 - 1
    B.key_bits = ((double)(n - 1) * (double)B.maxw <= 2147483646.0) ? 32 : 64;
    S.key_bits = B.key_bits;

    // the build's buffers are taken while the renumbering runs
    B.failed = A.get<int32_t>(n);
    B.roots = A.get<int32_t>(n);
    B.far2 = A.get<int32_t>(n);
    B.gstate = (int32_t*)A.get<int64_t>(plain_gstate_words() + 8);
    if (o.stats) B.stats = A.get<int64_t>((size_t)n * STAT_COLS);
    // initial pool: 16 labels per vertex, grown on demand
    B.pool.cap = (unsigned long long)n * 64 + 4096;
    B.pool.v = A.get<int32_t>(B.pool.cap);
    B.pool.hub = A.get<int32_t>(B.pool.cap);
    B.pool.dist = A.get<int32_t>(B.pool.cap);
    B.pool.cursor = B.ctl64 + 0;
    B.pool.fail_base = B.ctl64 + 1;
    if (A.oom) return CHL_ERR_OOM;
    HIPCHK(hipStreamSynchronize(st));
    if (hc0->c32[0]) return CHL_ERR_INVALID_ARG;
    S.prep_ms = tprep.elapsed();
    B.sig = graph_signature(g);
    A.drop(smp);
    A.drop(rdeg);
    A.drop(cnt);
    B.g = RGraph{n, B.m, rrow, rarc};
    if (B.stats) HIPCHK(hipMemsetAsync(B.stats, 0, (size_t)n * STAT_COLS * 8, st));

    // ---- rank-prefix pruning (Section 4.3) in levels: the trees of roots
    //      [0, 16) grow unpruned; then every level [g, 8g) (or [g, 2g) and
    //      [g, 4g) in turn, see LEVEL_LABELS_X2) is pruned by the labels of
    //      the hubs [0, g), which are complete, and so on up to the prefix
    //      size; the main phase is pruned by the whole prefix. The labels of
    //      every level extend the per-vertex groups of the levels before it.
    int launches = 0;
    int prefix_launches = 0;
    double prune_ms = 0;
    int32_t grown = 0;
    // a graph on which the probe already found pruning not to pay skips the
    // levels: its first roots simply start the main phase
    bool known_unpruned = false;
    if (o.prune_hubs == 0 && o.autotune) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_prune_keep.find(TuneKey{n, B.m, B.maxw, -1, B.sig});
        known_unpruned = it != g_prune_keep.end() && !it->second;
    }
    // (the levels' end is only recorded: the main phase's set-up is queued
    // behind their last kernels, and the time is read after a later
    // synchronisation)
    std::unique_ptr<Timer> tp;
    if (o.mode == CHL_MODE_BATCHED && o.prune_hubs >= 0 && n >= 64 && !known_unpruned) {
        tp.reset(new Timer(st));
        if (int r = run_levels(A, B, o, scan_tmp, st, launches, grown)) return r;
        prefix_launches = launches;
        tp->record_end();
    }

    // ---- parameters
    int k = 0, wg = 0;
    int64_t delta = 0;
    double tune_ms = 0;
    bool small = false;
    // The pruning levels leave the groups ordered by distance (B.dmaj), as
    // the batched, team and group kernels read them: a candidate's pruning
    // test stops at the first entry whose distance, plus the root's nearest
    // prefix hub, exceeds the candidate (no later entry can give a shorter
    // walk). R-MAT 20: main phase 41.4 -> 32.7 ms. The small-tree kernel
    // reads the groups in hub order, and so does the tuner's probe of it.
    const uint64_t* plab_byd = B.dmaj ? B.plab : nullptr;
    if (B.dmaj) { B.plab = B.plab_hub; B.dmaj = 0; }
    // a large prefix: the main phase hashes each root's prefix distances in
    // LDS (more workgroups resident than with a dense prefix-size array)
    B.hashdh = B.pbound >= HASH_MIN_PREFIX ? 1 : 0;
    if (int r = pick_params(A, B, g, o, st, k, wg, delta, small, tune_ms)) return r;
    if (plab_byd && !small) { B.plab = plab_byd; B.dmaj = 1; }
    S.small_trees = small ? small_capacity(B.key_bits) : 0;
    S.tune_ms = tune_ms;
    S.roots_in_flight = k;
    S.wg_size = wg;
    S.delta = delta;
    S.prune_hubs = B.pbound;
    S.prefix_roots = B.grown;
    {
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess)
            S.clock_khz = khz;
    }

    // ---- trees
    Slots s{};
    if (int r = alloc_slots(A, B, o.mode == CHL_MODE_PLAIN ? 1 : k, s, st)) return r;
    HIPCHK(hipMemcpyAsync(B.ctl64, &B.cursor_base, 8, hipMemcpyHostToDevice, st));
    Timer ttree(st);
    std::vector<int32_t> sel;
    if (o.root_count > 0)
        for (int32_t i = 0; i < o.root_count; i++) sel.push_back(o.root_begin + i * o.root_stride);
    // The main phase of the batched form: a root without arcs, or one whose
    // neighbours all outrank it, has the root alone as its tree (every other
    // vertex is reached through an outranking neighbour), so its only label
    // (r, r, 0) is written directly; the tree kernels grow the other roots
    // from a list (R-MAT 20: 501,961 roots without arcs and 375,030 with
    // outranking neighbours of the 1,040,384 main-phase roots).
    int32_t nmain = n - grown;
    bool listed = false;
    if (o.mode != CHL_MODE_PLAIN && o.hybrid_psi <= 0 && sel.empty() && nmain > 0) {
        int32_t* flag = A.get<int32_t>((size_t)nmain);
        int32_t* one = A.get<int32_t>((size_t)nmain);
        int64_t* pos = A.get<int64_t>((size_t)nmain + 1);
        HostCtl* hc1 = host_ctl();
        if (!flag || !one || !pos) return CHL_ERR_OOM;
        if (!hc1) return CHL_ERR_HIP;
        if (launch_trivial_count(grown, nmain, B.g.row, B.g.arc, flag, one, pos, scan_tmp, st)) return CHL_ERR_HIP;
        HIPCHK(hipMemcpyAsync(hc1->c64, pos + nmain, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        const unsigned long long ntrivial = hc1->c64[0];
        if (ntrivial > 0) {
            const unsigned long long base = B.cursor_base;
            if (base + ntrivial > B.pool.cap)
                if (int r0 = grow_pool(A, B, base, base + ntrivial, st)) return r0;
            if (launch_trivial_split(grown, nmain, flag, pos, B.pool, base, B.roots, B.stats, st))
                return CHL_ERR_HIP;
            hc1->c64[1] = base + ntrivial;
            HIPCHK(hipMemcpyAsync(B.ctl64, &hc1->c64[1], 8, hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
            B.last_used = base + ntrivial;
            nmain -= (int32_t)ntrivial;
            listed = true;
        }
        A.drop(flag);
        A.drop(one);
        A.drop(pos);
    }
    int r = o.mode == CHL_MODE_PLAIN
                ? run_plain(A, B, s, wg, delta, o.early_term, sel, st, &launches)
            : o.hybrid_psi > 0
                ? run_hybrid(A, B, o, s, wg, delta, (int)S.small_trees, scan_tmp, st, &launches, S)
            : nmain == 0
                ? 0
                : run_batched(A, B, s, wg, delta, o.early_term, sel.empty() ? nullptr : sel.data(),
                              sel.empty() ? nmain : (int32_t)sel.size(), st, &launches, 0,
                              sel.empty() && !listed ? grown : 0, nullptr, listed, nullptr, (int)S.small_trees);
    if (r) return r;
    S.tree_ms = ttree.stop();
    if (tp) prune_ms = tp->elapsed();
    S.prefix_ms = prune_ms;
    S.kernel_ms = B.kernel_ms;
    S.kernel_launches = B.kernel_launches;
    // a root-subset build discards the levels' labels (run_levels)
    S.levels = o.root_count > 0 ? 0 : B.nlev;
    for (int i = 0; i < B.nlev; i++) {
        S.level_end[i] = B.lv_end[i];
        S.level_ms[i] = B.lv_ms[i];
        S.level_teams[i] = B.lv_team[i];
    }
    S.launches = launches - prefix_launches;
    free_slots(A, s);
    HostCtl* hc = host_ctl();
    if (!hc) return CHL_ERR_HIP;
    HIPCHK(hipMemcpyAsync(hc->c32, B.ctl32, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hc->c64, B.ctl64, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int32_t errw = hc->c32[3];
    const unsigned long long used = hc->c64[0];
    if (errw & ERR_BIT_OVERFLOW) return CHL_ERR_DIST_OVERFLOW;
    if (errw & ERR_BIT_INVALID) return CHL_ERR_INVALID_ARG;

    // ---- assembly
    Timer tasm(st);
    chl_labels* L = new chl_labels();
    L->n = n;
    L->total = (int64_t)used;
    L->alloc = al;
    Arena keep(al);  // buffers handed to the handle
    int32_t* count = A.get<int32_t>(n);
    int32_t* fill = A.get<int32_t>(n);
    uint64_t* tmp = A.get<uint64_t>(std::max<unsigned long long>(used, 1));
    L->offsets = keep.get<int64_t>((size_t)n + 1);
    L->hub_pos = keep.get<int32_t>(std::max<unsigned long long>(used, 1));
    L->dist = keep.get<int32_t>(std::max<unsigned long long>(used, 1));
    L->order = hub_order;
    L->qerr = keep.get<int32_t>(4);
    if (A.oom || keep.oom) { delete L; return CHL_ERR_OOM; }
    if (launch_assemble(n, order, B.pool, used, count, L->offsets, fill, tmp, L->hub_pos, L->dist, scan_tmp,
                        nullptr, st)) {
        delete L;
        return CHL_ERR_HIP;
    }
    S.assemble_ms = tasm.stop();
    // totals of the per-root statistics
    S.labels = (int64_t)used;
    if (B.stats) {
        int64_t* dsum = A.get<int64_t>(4);
        if (!dsum || hipMemsetAsync(dsum, 0, 32, st) != hipSuccess ||
            launch_stat_sums(n, B.stats, dsum, st) ||
            hipMemcpyAsync(hc->sums, dsum, 32, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            delete L;
            return CHL_ERR_HIP;
        }
        S.settled = hc->sums[0];
        S.arcs = hc->sums[1];
        S.early_trees = hc->sums[2];
        L->per_root = B.stats;
        A.release(B.stats);
    }
    A.release(hub_order);
    keep.ptrs.clear();   // now owned by the handle
    L->st = S;
    *out = L;
    return CHL_OK;
}

// ---------------------------------------------------------------- tuner
static int pick_params(Arena& A, Build& B, const chl_graph* g, const chl_build_opts& o, hipStream_t st,
                       int& k, int& wg, int64_t& delta, bool& small, double& tune_ms) {
    const int32_t n = B.n;
    const double wmean = 0.5 * (1.0 + B.maxw);
    size_t freeb = 0, totalb = 0;
    (void)hipMemGetInfo(&freeb, &totalb);
    size_t budget = freeb / 4;
    int kmax = (int)std::max<size_t>(1, std::min<size_t>(4096, budget / std::max<size_t>(1, slot_bytes(n, B.key_bits))));
    k = o.roots_in_flight ? std::min(o.roots_in_flight, kmax) : std::min(kmax, 1024);
    wg = o.wg_size ? o.wg_size : 256;
    delta = o.delta ? o.delta : std::max<int64_t>(1, (int64_t)(wmean));
    small = o.small_trees > 0;
    if (o.mode == CHL_MODE_PLAIN) {
        small = false;
        if (!o.wg_size) wg = 256;
        if (!o.delta) delta = std::max<int64_t>(1, (int64_t)(4 * wmean));
        return 0;
    }
    bool need = o.autotune && (!o.roots_in_flight || !o.wg_size || !o.delta || o.small_trees == 0);
    if (!need) return 0;
    // (unpruned builds share one entry whether or not their first roots ran
    // as a level)
    TuneKey key{n, B.m, B.maxw, (o.mode * 8192 + (B.pbound ? B.grown : 0)) * 8192 + B.pbound, B.sig};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            if (!o.roots_in_flight) k = std::min(it->second.k, kmax);
            if (!o.wg_size) wg = it->second.wg;
            if (!o.delta) delta = it->second.delta;
            if (!o.small_trees) small = it->second.small;
            return 0;
        }
    }
    // probe: a rank-stratified sample of the roots of the main phase (the
    // roots before it are done), large enough that a trial measures the
    // throughput of many trees per slot rather than the latency of a few
    // large ones or the launch: grown from 2048 roots by 4x until one run
    // takes 10 ms (at most 262144 roots, or all of them)
    std::vector<int32_t> probe;
    const int32_t r0 = B.grown;
    const int32_t rest = n - r0;
    auto make_probe = [&](int32_t strata) {
        probe.clear();
        for (int32_t i = 0; i < strata; i++) probe.push_back(r0 + (int32_t)((int64_t)rest * i / strata));
    };
    int32_t strata = std::min<int32_t>(rest, 2048);
    make_probe(strata);
    if (probe.empty()) return 0;
    int64_t* saved_stats = B.stats;
    B.stats = nullptr;              // probe runs leave no statistics
    auto t0 = std::chrono::steady_clock::now();
    double best = 1e30;
    TuneVal bv{k, wg, delta};
    int launches = 0;
    Slots s{};
    int kcur = 0;
    std::map<std::tuple<int, int, int64_t>, double> seen;
    // one timed run of the probe roots (kk, w, d already clamped)
    auto time_once = [&](int kk, int w, int64_t d, double& ms) -> int {
        if (kk != kcur) {
            free_slots(A, s);
            if (int r = alloc_slots(A, B, kk, s, st)) return r;
            kcur = kk;
        }
        HIPCHK(hipMemcpyAsync(B.ctl64, &B.cursor_base, 8, hipMemcpyHostToDevice, st));
        Timer t(st);
        if (int r = run_batched(A, B, s, w, d, o.early_term, probe.data(), (int32_t)probe.size(), st,
                                &launches, 1))
            return r;
        ms = t.stop();
        return 0;
    };
    auto trial = [&](int kk, int w, int64_t d) -> int {
        kk = std::max(1, std::min(kk, kmax));
        d = std::max<int64_t>(1, d);
        if (seen.count({kk, w, d})) return 0;
        double ms = 0;
        if (int r = time_once(kk, w, d, ms)) return r;
        seen[{kk, w, d}] = ms;
        if (ms < best) { best = ms; bv = TuneVal{kk, w, d}; }
        return 0;
    };
    // coordinate search: bucket width (coarse, then refined), workgroup
    // size at a fixed thread count, then trees in flight
    const int k0 = o.roots_in_flight ? k : std::min(kmax, 512);
    const int w0 = o.wg_size ? wg : 512;
    {
        const int64_t d0 = o.delta ? delta : std::max<int64_t>(1, (int64_t)wmean);
        for (;;) {
            double ms = 0;
            if (int r = time_once(std::max(1, std::min(k0, kmax)), w0, d0, ms)) return r;
            if (ms >= 10.0 || strata >= std::min<int32_t>(rest, 1 << 18)) break;
            strata = std::min<int32_t>(std::min<int32_t>(rest, 1 << 18), 4 * strata);
            make_probe(strata);
        }
    }
    if (!o.delta) {
        for (double f : {1.0 / 64, 1.0 / 16, 0.25, 1.0, 4.0})
            if (int r = trial(k0, w0, (int64_t)(f * wmean))) return r;
        int64_t d0 = bv.delta;
        for (double f : {0.5, 2.0})
            if (int r = trial(k0, w0, (int64_t)(f * d0))) return r;
    }
    // then workgroup size x threads in flight (trees in flight = threads /
    // workgroup size) at that bucket width
    {
        // (64 and 128 threads: one or two waves per tree, for graphs whose
        // main-phase trees are tiny)
        const int wgs[5] = {64, 128, 256, 512, 1024};
        for (int w : wgs) {
            if (o.wg_size && w != wg) continue;
            if (o.roots_in_flight) {
                if (int r = trial(k, w, bv.delta)) return r;
                continue;
            }
            for (int threads : {1 << 17, 1 << 18, 1 << 19, 1 << 20})
                if (int r = trial(threads / w, w, bv.delta)) return r;
        }
    }
    // time the two best settings once more and keep the faster in sum:
    // single trials of a few milliseconds are noisy
    if (seen.size() >= 2) {
        std::vector<std::pair<double, std::tuple<int, int, int64_t>>> rank;
        for (auto& kv : seen) rank.push_back({kv.second, kv.first});
        std::sort(rank.begin(), rank.end());
        double best2 = 1e30;
        for (int i = 0; i < 2; i++) {
            auto [kk, w, d] = rank[i].second;
            double ms = 0;
            if (int r = time_once(kk, w, d, ms)) return r;
            if (rank[i].first + ms < best2) { best2 = rank[i].first + ms; bv = TuneVal{kk, w, d}; }
        }
    }
    // then the small-tree kernel (trees in LDS, the batched kernel with the
    // setting found for the trees that do not fit), against the best setting
    if (!o.small_trees && small_capacity(B.key_bits) > 0) {
        const int kk = std::max(1, std::min(bv.k, kmax));
        double ms_b = 0, ms_s = 0;
        if (int r = time_once(kk, bv.wg, bv.delta, ms_b)) return r;
        if (kk != kcur) {
            free_slots(A, s);
            if (int r = alloc_slots(A, B, kk, s, st)) return r;
            kcur = kk;
        }
        HIPCHK(hipMemcpyAsync(B.ctl64, &B.cursor_base, 8, hipMemcpyHostToDevice, st));
        {
            Timer t(st);
            if (int r = run_batched(A, B, s, bv.wg, bv.delta, o.early_term, probe.data(), (int32_t)probe.size(), st,
                                    &launches, 1, 0, nullptr, false, nullptr, small_capacity(B.key_bits)))
                return r;
            ms_s = t.stop();
        }
        bv.small = ms_s < ms_b;
    }
    free_slots(A, s);
    B.stats = saved_stats;
    HIPCHK(hipMemcpyAsync(B.ctl64, &B.cursor_base, 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    k = bv.k;
    wg = bv.wg;
    delta = bv.delta;
    if (!o.small_trees) small = bv.small;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = bv;
    return 0;
}

// Directed graphs (footnote of Section 1): the trees grown along the arcs
// give, at every vertex they reach clean, the in-label (h, d(h, v)); the
// trees grown on the reversed graph give the out-label (h, d(v, h)). Both
// kinds are the trees of one build over a combined graph of 2n vertices: the
// graph (ids [0, n)) and its reversal (ids [n, 2n)), two components, with the
// ranking interleaved (v at rank position 2 pos(v), its reversed copy at
// 2 pos(v) + 1), so that "u outranks h" keeps its meaning inside each
// component, and every level of the rank-prefix pruning holds both trees of
// its vertices. The pruning test needs d(h, x) + d(x, u) for a tree along the
// arcs: d(x, u) is u's in-label from x, and d(h, x) the out-label of h from
// x, i.e. the label of h's reversed copy from x's reversed copy, the partner
// positions (TreeParams::partner).
static int chl_build_directed_impl(const chl_graph* g, const int32_t* order, const chl_build_opts* opts_in,
                                   const chl_allocator* alloc_in, void* stream, chl_labels** out) {
    if (!g || !order || !out) return CHL_ERR_INVALID_ARG;
    if (g->n < 1 || g->n > 0x3FFFFFFE || g->n_arcs < 0 || g->n_arcs > 0x7FFFFFFFll) return CHL_ERR_INVALID_ARG;
    if (!g->row_ptr || (g->n_arcs > 0 && (!g->col || !g->w))) return CHL_ERR_INVALID_ARG;
    if (int r = check_device()) return r;
    chl_allocator al = alloc_in ? *alloc_in : kDefaultAlloc;
    if (!al.alloc || !al.free) return CHL_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int32_t n = g->n;
    const int64_t m = g->n_arcs;
    chl_labels* L = nullptr;
    {
        Arena A(al);
        // validate the graph and the ranking before any kernel indexes with them
        int32_t* ctl = A.get<int32_t>(16);
        int32_t* pos = A.get<int32_t>(n);
        int32_t* cnt = A.get<int32_t>(n);
        if (A.oom) return CHL_ERR_OOM;
        HIPCHK(hipMemsetAsync(ctl, 0, 64, st));
        HIPCHK(hipMemsetAsync(cnt, 0, (size_t)n * 4, st));
        if (launch_validate(n, m, g->row_ptr, g->col, g->w, order, pos, cnt, ctl, ctl + 1, st)) return CHL_ERR_HIP;
        HostCtl* hc = host_ctl();
        if (!hc) return CHL_ERR_HIP;
        HIPCHK(hipMemcpyAsync(hc->c32, ctl, 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (hc->c32[0]) return CHL_ERR_INVALID_ARG;
        A.drop(pos);
        // the reversed graph, then the combined graph
        int64_t* trow = A.get<int64_t>((size_t)n + 1);
        auto* cursor = A.get<unsigned long long>(n);
        uint64_t* tkey = A.get<uint64_t>((size_t)std::max<int64_t>(m, 1));
        int32_t* tcol = A.get<int32_t>((size_t)std::max<int64_t>(m, 1));
        int32_t* tw = A.get<int32_t>((size_t)std::max<int64_t>(m, 1));
        void* tmp = A.get<uint8_t>(scan_temp_bytes(std::max<int64_t>(n, 1)));
        int64_t* row2 = A.get<int64_t>(2 * (size_t)n + 1);
        int32_t* col2 = A.get<int32_t>((size_t)std::max<int64_t>(2 * m, 1));
        int32_t* w2 = A.get<int32_t>((size_t)std::max<int64_t>(2 * m, 1));
        int32_t* order2 = A.get<int32_t>(2 * (size_t)n);
        if (A.oom) return CHL_ERR_OOM;
        if (launch_transpose(n, m, g->row_ptr, g->col, g->w, cnt, trow, cursor, tkey, tcol, tw, tmp, st) ||
            launch_directed_union(n, m, g->row_ptr, g->col, g->w, order, trow, tcol, tw, row2, col2, w2, order2, st))
            return CHL_ERR_HIP;
        chl_graph g2{2 * n, 2 * m, row2, col2, w2};
        int r = chl_build_impl(&g2, order2, opts_in, alloc_in, stream, &L, true);
        HIPCHK(hipStreamSynchronize(st));   // the arena's buffers are released next
        if (r) return r;
    }
    // split the combined labeling: in-labels in place, out-labels copied out
    Arena keep(al);
    int64_t tin = 0;
    int64_t* out_off = nullptr;
    int32_t *out_hub = nullptr, *out_dist = nullptr, *ord = nullptr;
    int r = CHL_OK;
    HostCtl* hc = host_ctl();
    if (!hc || hipMemcpyAsync(hc->c64, L->offsets + n, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        r = CHL_ERR_HIP;
    } else {
        tin = (int64_t)hc->c64[0];
        const int64_t tout = L->total - tin;
        out_off = keep.get<int64_t>((size_t)n + 1);
        out_hub = keep.get<int32_t>((size_t)std::max<int64_t>(tout, 1));
        out_dist = keep.get<int32_t>((size_t)std::max<int64_t>(tout, 1));
        ord = keep.get<int32_t>(n);
        if (keep.oom) r = CHL_ERR_OOM;
        else if (launch_directed_split(n, L->total, L->offsets, L->hub_pos, L->dist, out_off, out_hub, out_dist, st) ||
                 hipMemcpyAsync(ord, order, (size_t)n * 4, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                 hipStreamSynchronize(st) != hipSuccess)
            r = CHL_ERR_HIP;
    }
    if (r) {
        chl_labels_free(L);
        return r;
    }
    auto f = [&](void* p) { if (p) L->alloc.free(p, L->alloc.ctx); };
    L->directed = 1;
    L->in_total = tin;
    L->in_offsets = L->offsets;     // the first n + 1 of the 2n + 1 offsets
    L->in_hub_pos = L->hub_pos;
    L->in_dist = L->dist;
    L->offsets = out_off;
    L->hub_pos = out_hub;
    L->dist = out_dist;
    L->total -= tin;
    f(L->order);
    L->order = ord;
    f(L->per_root);                 // per-root statistics are not kept for a directed labeling
    L->per_root = nullptr;
    L->n = n;
    L->st.n = n;
    keep.release(out_off);
    keep.release(out_hub);
    keep.release(out_dist);
    keep.release(ord);
    *out = L;
    return CHL_OK;
}
