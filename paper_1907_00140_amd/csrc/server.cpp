// Continuous-batching server: labelings stay resident on the device; a
// dispatcher thread batches the distance queries that have arrived (every
// query is due at its scheduled arrival time) onto a query stream, with up to
// two batches in flight, and admits build requests by their device-memory
// footprint onto build streams, where they run concurrently with the queries.
// Latency of a request = time its result is observed - its scheduled arrival.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"

namespace {

using clk = std::chrono::steady_clock;

struct QBlock {
    int32_t gid;
    const int32_t* pairs;
    const double* t;
    int64_t q;
    int64_t* out;
    double* lat;
    int64_t next = 0;  // first query not yet dispatched
};

struct BuildReq {
    int32_t n;
    int64_t m;
    std::vector<int64_t> row;
    std::vector<int32_t> col, w, order;
    double t;
    int32_t* gid_out;
    double* lat;
    int32_t* status;
    size_t footprint;
    int attempts = 0;
    bool started = false, done = false;
};

void bump_peak(std::atomic<int64_t>& peak, int64_t v) {
    int64_t p = peak.load();
    while (v > p && !peak.compare_exchange_weak(p, v)) {
    }
}

// Device allocator of one build stream, with byte accounting against the
// server's budget. A build is admitted with an estimate of its footprint
// (charged); an allocation that takes its live bytes past the charge first
// charges the difference to the shared budget and fails (the build then
// returns CHL_ERR_OOM and is queued again with a larger estimate) when that
// would overrun mem_budget. Memory comes from the stream-ordered pool of the
// build stream, or from the caller's allocator when the server was created
// with one.
struct StreamAlloc {
    hipStream_t s;
    std::atomic<int64_t>* budget_used = nullptr;   // the server's charged bytes
    std::atomic<int64_t>* budget_peak = nullptr;
    int64_t budget = 0;                            // mem_budget
    const chl_allocator* user = nullptr;           // the caller's allocator or NULL
    std::mutex mu;
    int64_t bytes = 0;      // live bytes of the current build
    int64_t charged = 0;    // bytes charged to the budget for the current build
    int64_t peak = 0;       // largest live bytes of the current build
    bool refused = false;   // an allocation was refused for the budget
    std::vector<std::pair<void*, size_t>> live;
    void start(int64_t reserve) {
        std::lock_guard<std::mutex> lk(mu);
        bytes = 0; charged = reserve; peak = 0; refused = false;
    }
    static void* alloc(size_t b, void* ctx) {
        auto* a = (StreamAlloc*)ctx;
        {
            std::lock_guard<std::mutex> lk(a->mu);
            const int64_t need = a->bytes + (int64_t)b - a->charged;
            if (need > 0) {
                int64_t cur = a->budget_used->load();
                do {
                    if (cur + need > a->budget) { a->refused = true; return nullptr; }
                } while (!a->budget_used->compare_exchange_weak(cur, cur + need));
                a->charged += need;
                bump_peak(*a->budget_peak, cur + need);
            }
            a->bytes += (int64_t)b;
            a->peak = std::max(a->peak, a->bytes);
        }
        void* p = nullptr;
        if (a->user) p = a->user->alloc(b, a->user->ctx);
        else if (hipMallocAsync(&p, b, a->s) != hipSuccess) p = nullptr;
        std::lock_guard<std::mutex> lk(a->mu);
        if (!p) { a->bytes -= (int64_t)b; return nullptr; }
        a->live.push_back({p, b});
        return p;
    }
    static void release(void* p, void* ctx) {
        auto* a = (StreamAlloc*)ctx;
        if (a->user) {
            // a caller's allocator is not ordered with the build stream: the
            // work queued there may still use the memory
            (void)hipStreamSynchronize(a->s);
            a->user->free(p, a->user->ctx);
        } else {
            (void)hipFreeAsync(p, a->s);
        }
        std::lock_guard<std::mutex> lk(a->mu);
        for (size_t i = 0; i < a->live.size(); i++)
            if (a->live[i].first == p) {
                a->bytes -= (int64_t)a->live[i].second;
                a->live.erase(a->live.begin() + i);
                break;
            }
        // (memory of finished builds' labelings is not in `live`: it no
        // longer counts against the current build)
    }
    // the build is over: its charge returns to the budget (the budget covers
    // builds in flight; a finished labeling is resident like the ones added
    // with chl_server_add_labels)
    int64_t finish() {
        std::lock_guard<std::mutex> lk(mu);
        const int64_t ret = charged;
        charged = 0;
        live.clear();
        bytes = 0;
        return ret;
    }
};

struct Batch {
    int32_t cap = 0;
    int32_t* h_pairs = nullptr;   // pinned
    int64_t* h_out = nullptr;     // pinned
    int32_t* d_pairs = nullptr;
    int64_t* d_out = nullptr;
    hipEvent_t ev{};
    bool busy = false;
    std::vector<std::pair<int32_t, int64_t>> who;  // (block, query index)
    double t_launch = 0;     // server time the batch was queued on the device
    double t_oldest = 0;     // earliest scheduled arrival among its queries
};

// One row of the server's trace (chl_server_trace).
struct TraceRow {
    double kind, t0, t1, t2, size;
};

}  // namespace

struct chl_server {
    chl_server_opts o{};
    chl_allocator user{};        // the caller's allocator (user.alloc == NULL: stream-ordered pools)
    hipStream_t qs{};
    std::vector<hipStream_t> bs;
    std::vector<std::unique_ptr<StreamAlloc>> ba;
    std::vector<bool> bs_busy;
    std::vector<const chl_labels*> graphs;
    std::vector<chl_labels*> owned;
    std::deque<QBlock> qblocks;
    std::deque<BuildReq> builds;
    Batch batch[2];
    int32_t* d_err = nullptr;
    std::mutex mu;
    std::thread disp;
    std::vector<std::thread> workers;
    std::atomic<bool> running{false};
    std::atomic<int64_t> budget_used{0};
    std::atomic<int64_t> budget_peak{0};     // largest budget_used seen
    std::atomic<int32_t> builds_left{0};
    int64_t queries_left = 0;
    clk::time_point t0;
    std::condition_variable done_cv;
    bool all_done = false;
    std::vector<TraceRow> trace;   // batches and builds of the last run (under mu for builds)

    double now() const { return std::chrono::duration<double>(clk::now() - t0).count(); }
    void dispatch_loop();
    void run_build(size_t idx, int stream_slot);
};

namespace {

size_t build_footprint(int32_t n, int64_t m, int k) {
    // CSR copy + renumbered CSR + per-tree slots + a label pool of 64 per
    // vertex. An estimate: a build that needs more charges the rest while it
    // runs (StreamAlloc), or is queued again with a larger estimate.
    size_t slots = (size_t)k * ((size_t)n * 24 + (size_t)n / 2);
    return (size_t)m * 24 + (size_t)n * 64 + slots + (size_t)n * 64 * 28;
}

}  // namespace

void chl_server::run_build(size_t idx, int slot) {
    BuildReq& b = builds[idx];
    hipStream_t s = bs[slot];
    StreamAlloc* a = ba[slot].get();
    a->start((int64_t)b.footprint);
    const double t_admit = now();
    chl_allocator al{StreamAlloc::alloc, StreamAlloc::release, a};
    int code = CHL_OK;
    int64_t* d_row = nullptr;
    int32_t *d_col = nullptr, *d_w = nullptr, *d_order = nullptr;
    d_row = (int64_t*)StreamAlloc::alloc((size_t)(b.n + 1) * 8, a);
    d_col = (int32_t*)StreamAlloc::alloc(std::max<size_t>(4, (size_t)b.m * 4), a);
    d_w = (int32_t*)StreamAlloc::alloc(std::max<size_t>(4, (size_t)b.m * 4), a);
    d_order = (int32_t*)StreamAlloc::alloc((size_t)b.n * 4, a);
    chl_labels* L = nullptr;
    if (!d_row || !d_col || !d_w || !d_order) {
        code = CHL_ERR_OOM;
    } else {
        (void)hipMemcpyAsync(d_row, b.row.data(), (size_t)(b.n + 1) * 8, hipMemcpyHostToDevice, s);
        if (b.m) {
            (void)hipMemcpyAsync(d_col, b.col.data(), (size_t)b.m * 4, hipMemcpyHostToDevice, s);
            (void)hipMemcpyAsync(d_w, b.w.data(), (size_t)b.m * 4, hipMemcpyHostToDevice, s);
        }
        (void)hipMemcpyAsync(d_order, b.order.data(), (size_t)b.n * 4, hipMemcpyHostToDevice, s);
        chl_graph g{b.n, b.m, d_row, d_col, d_w};
        chl_build_opts bo;
        chl_build_opts_default(&bo);
        bo.roots_in_flight = o.build_wg;
        bo.wg_size = 256;
        bo.autotune = 0;
        bo.stats = 0;
        // builds share the device with queries and other builds: no
        // cooperative (whole-team resident) launches
        bo.team_wgs = 1;
        code = chl_build(&g, d_order, &bo, &al, (void*)s, &L);
    }
    for (void* p : {(void*)d_row, (void*)d_col, (void*)d_w, (void*)d_order})
        if (p) StreamAlloc::release(p, a);
    (void)hipStreamSynchronize(s);
    double tc = now();
    {
        std::lock_guard<std::mutex> lk(mu);
        trace.push_back({1.0, b.t, t_admit, tc, (double)b.n});
    }
    const bool refused = code == CHL_ERR_OOM && a->refused;
    const int64_t peak = a->peak;
    budget_used -= a->finish();
    std::lock_guard<std::mutex> lk(mu);
    bs_busy[slot] = false;
    if (refused && b.attempts < 4 && b.footprint < o.mem_budget) {
        // the estimate was too small and other builds held the rest of the
        // budget: queue the request again with a larger estimate (at most
        // the whole budget: then it runs alone)
        b.footprint = std::min<size_t>(o.mem_budget, std::max<size_t>(2 * b.footprint, (size_t)peak * 5 / 4));
        b.started = false;
        return;
    }
    *b.status = code;
    *b.lat = tc - b.t;
    if (code == CHL_OK) {
        *b.gid_out = (int32_t)graphs.size();
        graphs.push_back(L);
        owned.push_back(L);
    } else {
        *b.gid_out = -1;
    }
    b.done = true;
    builds_left--;
}

void chl_server::dispatch_loop() {
    for (;;) {
        bool idle = true;
        double tnow = now();
        // ---- completed query batches
        for (Batch& B : batch) {
            if (!B.busy || hipEventQuery(B.ev) != hipSuccess) continue;
            double tc = now();
            {
                std::lock_guard<std::mutex> lk(mu);
                trace.push_back({0.0, B.t_oldest, B.t_launch, tc, (double)B.who.size()});
            }
            for (size_t j = 0; j < B.who.size(); j++) {
                QBlock& qb = qblocks[B.who[j].first];
                int64_t i = B.who[j].second;
                qb.out[i] = B.h_out[j];
                qb.lat[i] = tc - qb.t[i];
            }
            queries_left -= (int64_t)B.who.size();
            B.who.clear();
            B.busy = false;
            idle = false;
        }
        // ---- admit builds that have arrived, in arrival order
        {
            std::lock_guard<std::mutex> lk(mu);
            for (size_t i = 0; i < builds.size(); i++) {
                BuildReq& b = builds[i];
                if (b.started || b.t > tnow) continue;
                if (b.footprint > o.mem_budget) {  // can never fit
                    b.started = b.done = true;
                    *b.status = CHL_ERR_BUSY;
                    *b.gid_out = -1;
                    *b.lat = tnow - b.t;
                    builds_left--;
                    continue;
                }
                if (budget_used + (int64_t)b.footprint > (int64_t)o.mem_budget) break;  // wait for memory
                int slot = -1;
                for (size_t k = 0; k < bs_busy.size(); k++)
                    if (!bs_busy[k]) { slot = (int)k; break; }
                if (slot < 0) break;                                                  // wait for a stream
                bs_busy[slot] = true;
                b.started = true;
                b.attempts++;
                bump_peak(budget_peak, budget_used += (int64_t)b.footprint);
                workers.emplace_back(&chl_server::run_build, this, i, slot);
                idle = false;
            }
        }
        // ---- launch a batch of the queries that have arrived
        for (Batch& B : batch) {
            if (B.busy) continue;
            int32_t fill = 0;
            std::vector<std::pair<int32_t, int32_t>> seg;  // (block, count) in buffer order
            for (size_t bi = 0; bi < qblocks.size() && fill < B.cap; bi++) {
                QBlock& qb = qblocks[bi];
                int32_t c0 = fill;
                while (qb.next < qb.q && qb.t[qb.next] <= tnow && fill < B.cap) {
                    B.h_pairs[2 * fill] = qb.pairs[2 * qb.next];
                    B.h_pairs[2 * fill + 1] = qb.pairs[2 * qb.next + 1];
                    B.who.push_back({(int32_t)bi, qb.next});
                    qb.next++;
                    fill++;
                }
                if (fill > c0) seg.push_back({(int32_t)bi, fill - c0});
            }
            if (fill == 0) break;
            (void)hipMemcpyAsync(B.d_pairs, B.h_pairs, (size_t)fill * 8, hipMemcpyHostToDevice, qs);
            int32_t off = 0;
            for (auto& sg : seg) {
                const chl_labels* L;
                {
                    std::lock_guard<std::mutex> lk(mu);
                    L = graphs[qblocks[sg.first].gid];
                }
                double avg = L->n ? (double)L->total / L->n : 1.0;
                const bool dir = L->directed != 0;
                chl::launch_query(L->n, L->offsets, L->hub_pos, L->dist, dir ? L->in_offsets : L->offsets,
                                  dir ? L->in_hub_pos : L->hub_pos, dir ? L->in_dist : L->dist,
                                  B.d_pairs + 2 * off, sg.second, B.d_out + off, d_err, avg, qs);
                off += sg.second;
            }
            (void)hipMemcpyAsync(B.h_out, B.d_out, (size_t)fill * 8, hipMemcpyDeviceToHost, qs);
            (void)hipEventRecord(B.ev, qs);
            B.t_launch = now();
            B.t_oldest = qblocks[B.who[0].first].t[B.who[0].second];
            for (auto& w : B.who) B.t_oldest = std::min(B.t_oldest, qblocks[w.first].t[w.second]);
            B.busy = true;
            idle = false;
        }
        // ---- finished?
        bool qdone = queries_left == 0 && !batch[0].busy && !batch[1].busy;
        if (qdone && builds_left.load() == 0) break;
        if (idle) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    for (auto& t : workers) t.join();
    workers.clear();
    std::lock_guard<std::mutex> lk(mu);
    all_done = true;
    done_cv.notify_all();
}

extern "C" {

void chl_server_opts_default(chl_server_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->mem_budget = (size_t)16 << 30;
    o->max_batch = 1 << 16;
    o->build_streams = 2;
    o->build_wg = 128;
}

int chl_server_create(const chl_server_opts* o, const chl_allocator* alloc, chl_server** out) {
    if (!out) return CHL_ERR_INVALID_ARG;
    if (alloc && (!alloc->alloc || !alloc->free)) return CHL_ERR_INVALID_ARG;
    chl_server_opts so;
    chl_server_opts_default(&so);
    if (o) so = *o;
    if (so.max_batch < 1 || so.build_streams < 1 || so.build_streams > 8 || so.build_wg < 1)
        return CHL_ERR_INVALID_ARG;
    auto* s = new chl_server();
    s->o = so;
    if (alloc) s->user = *alloc;
    // Builds allocate from the device's default stream-ordered pool, which
    // serves a build's temporaries from memory freed by earlier builds. No
    // memory is reserved up front: the pool was measured to keep at most
    // about 0.75 GB of freed memory whatever its release threshold, so
    // allocating the budget here and freeing it into the pool only mapped
    // device memory and handed it straight back to the system.
    bool ok = hipStreamCreateWithFlags(&s->qs, hipStreamNonBlocking) == hipSuccess;
    for (int i = 0; i < so.build_streams && ok; i++) {
        hipStream_t st;
        ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (!ok) break;
        s->bs.push_back(st);
        auto a = std::make_unique<StreamAlloc>();
        a->s = st;
        a->budget_used = &s->budget_used;
        a->budget_peak = &s->budget_peak;
        a->budget = (int64_t)so.mem_budget;
        a->user = s->user.alloc ? &s->user : nullptr;
        s->ba.push_back(std::move(a));
        s->bs_busy.push_back(false);
    }
    for (Batch& B : s->batch) {
        if (!ok) break;
        B.cap = so.max_batch;
        ok = hipHostMalloc((void**)&B.h_pairs, (size_t)B.cap * 8, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void**)&B.h_out, (size_t)B.cap * 8, hipHostMallocDefault) == hipSuccess &&
             hipMalloc((void**)&B.d_pairs, (size_t)B.cap * 8) == hipSuccess &&
             hipMalloc((void**)&B.d_out, (size_t)B.cap * 8) == hipSuccess &&
             hipEventCreateWithFlags(&B.ev, hipEventDisableTiming) == hipSuccess;
    }
    ok = ok && hipMalloc((void**)&s->d_err, 4) == hipSuccess;
    if (!ok) {
        chl_server_destroy(s);
        return CHL_ERR_HIP;
    }
    *out = s;
    return CHL_OK;
}

int chl_server_add_labels(chl_server* s, const chl_labels* h, int32_t* graph_id) {
    if (!s || !h || !graph_id) return CHL_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *graph_id = (int32_t)s->graphs.size();
    s->graphs.push_back(h);
    return CHL_OK;
}

int chl_server_submit_queries(chl_server* s, int32_t graph_id, const int32_t* pairs, const double* t_arrival,
                              int64_t q, int64_t* out, double* lat) {
    if (!s || q < 0 || (q && (!pairs || !t_arrival || !out || !lat))) return CHL_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->running) return CHL_ERR_BUSY;   // the dispatcher reads the request lists without the lock
    if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size()) return CHL_ERR_INVALID_ARG;
    for (int64_t i = 1; i < q; i++)
        if (t_arrival[i] < t_arrival[i - 1]) return CHL_ERR_INVALID_ARG;
    if (q == 0) return CHL_OK;
    QBlock b;
    b.gid = graph_id; b.pairs = pairs; b.t = t_arrival; b.q = q; b.out = out; b.lat = lat;
    s->qblocks.push_back(b);
    s->queries_left += q;
    return CHL_OK;
}

int chl_server_submit_build(chl_server* s, int32_t n, int64_t n_arcs, const int64_t* row_ptr,
                            const int32_t* col, const int32_t* w, const int32_t* order, double t_arrival,
                            int32_t* graph_id, double* lat, int32_t* status) {
    if (!s || n < 1 || n_arcs < 0 || !row_ptr || !order || !graph_id || !lat || !status) return CHL_ERR_INVALID_ARG;
    if (n_arcs && (!col || !w)) return CHL_ERR_INVALID_ARG;
    BuildReq b;
    b.n = n; b.m = n_arcs;
    b.row.assign(row_ptr, row_ptr + n + 1);
    b.col.assign(col, col + n_arcs);
    b.w.assign(w, w + n_arcs);
    b.order.assign(order, order + n);
    b.t = t_arrival; b.gid_out = graph_id; b.lat = lat; b.status = status;
    b.footprint = build_footprint(n, n_arcs, s->o.build_wg);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->running) return CHL_ERR_BUSY;
    // keep builds in arrival order
    auto it = std::upper_bound(s->builds.begin(), s->builds.end(), t_arrival,
                               [](double t, const BuildReq& r) { return t < r.t; });
    s->builds.insert(it, std::move(b));
    s->builds_left++;
    return CHL_OK;
}

int chl_server_trace(chl_server* s, double* rows, int64_t cap, int64_t* count) {
    if (!s || !count || cap < 0 || (cap > 0 && !rows)) return CHL_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *count = (int64_t)s->trace.size();
    const int64_t k = std::min<int64_t>(cap, (int64_t)s->trace.size());
    for (int64_t i = 0; i < k; i++) {
        const TraceRow& r = s->trace[i];
        rows[5 * i + 0] = r.kind;
        rows[5 * i + 1] = r.t0;
        rows[5 * i + 2] = r.t1;
        rows[5 * i + 3] = r.t2;
        rows[5 * i + 4] = r.size;
    }
    return CHL_OK;
}

size_t chl_server_budget_peak(const chl_server* s) {
    return s ? (size_t)s->budget_peak.load() : 0;
}

size_t chl_server_build_footprint(const chl_server* s, int32_t n, int64_t n_arcs) {
    if (!s || n < 1 || n_arcs < 0) return 0;
    return build_footprint(n, n_arcs, s->o.build_wg);
}

int chl_server_start(chl_server* s) {
    if (!s) return CHL_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->running) return CHL_ERR_INVALID_ARG;
    s->running = true;
    s->all_done = false;
    s->trace.clear();
    s->t0 = clk::now();
    s->disp = std::thread(&chl_server::dispatch_loop, s);
    return CHL_OK;
}

int chl_server_wait(chl_server* s) {
    if (!s) return CHL_ERR_INVALID_ARG;
    if (s->disp.joinable()) s->disp.join();
    s->running = false;
    return CHL_OK;
}

const chl_labels* chl_server_labels(chl_server* s, int32_t graph_id) {
    if (!s) return nullptr;
    std::lock_guard<std::mutex> lk(s->mu);
    if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size()) return nullptr;
    return s->graphs[graph_id];
}

void chl_server_destroy(chl_server* s) {
    if (!s) return;
    if (s->disp.joinable()) s->disp.join();
    for (auto& t : s->workers) t.join();
    for (chl_labels* L : s->owned) chl_labels_free(L);
    for (hipStream_t st : s->bs) { (void)hipStreamSynchronize(st); (void)hipStreamDestroy(st); }
    if (s->qs) { (void)hipStreamSynchronize(s->qs); (void)hipStreamDestroy(s->qs); }
    for (Batch& B : s->batch) {
        if (B.h_pairs) (void)hipHostFree(B.h_pairs);
        if (B.h_out) (void)hipHostFree(B.h_out);
        if (B.d_pairs) (void)hipFree(B.d_pairs);
        if (B.d_out) (void)hipFree(B.d_out);
        if (B.ev) (void)hipEventDestroy(B.ev);
    }
    if (s->d_err) (void)hipFree(s->d_err);
    delete s;
}

}  // extern "C"
