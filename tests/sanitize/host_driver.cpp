// Drives the C-ABI of libchl on every path that runs without a device --
// argument checks, error strings, option defaults, the server's creation and
// destruction when no device is usable -- for a build whose host code is
// compiled with AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/test_sanitize.py). The device code is built as usual.
#include <cstdio>
#include <cstring>

#include "chl.h"

static int fails = 0;
#define EXPECT(cond)                                                         \
    do {                                                                     \
        if (!(cond)) { std::fprintf(stderr, "failed: %s (line %d)\n", #cond, __LINE__); fails++; } \
    } while (0)

static void* no_alloc(size_t, void*) { return nullptr; }
static void no_free(void*, void*) {}

int main() {
    for (int c = -8; c <= 1; c++) EXPECT(chl_error_string(c) != nullptr);
    chl_build_opts_default(nullptr);
    chl_build_opts o;
    chl_build_opts_default(&o);
    EXPECT(o.mode == CHL_MODE_BATCHED && o.early_term == 1 && o.autotune == 1);

    // a valid 3-vertex path 0 - 1 - 2 on host memory (never read: no device)
    int64_t row[4] = {0, 1, 3, 4};
    int32_t col[4] = {1, 0, 2, 1};
    int32_t w[4] = {1, 1, 2, 2};
    int32_t order[3] = {1, 0, 2};
    chl_graph g{3, 4, row, col, w};
    chl_labels* L = nullptr;
    EXPECT(chl_build(nullptr, order, &o, nullptr, nullptr, &L) == CHL_ERR_INVALID_ARG);
    EXPECT(chl_build(&g, nullptr, &o, nullptr, nullptr, &L) == CHL_ERR_INVALID_ARG);
    EXPECT(chl_build(&g, order, &o, nullptr, nullptr, nullptr) == CHL_ERR_INVALID_ARG);
    chl_graph bad = g;
    bad.n = 0;
    EXPECT(chl_build(&bad, order, &o, nullptr, nullptr, &L) == CHL_ERR_INVALID_ARG);
    bad = g;
    bad.n_arcs = -1;
    EXPECT(chl_build(&bad, order, &o, nullptr, nullptr, &L) == CHL_ERR_INVALID_ARG);
    bad = g;
    bad.col = nullptr;
    EXPECT(chl_build(&bad, order, &o, nullptr, nullptr, &L) == CHL_ERR_INVALID_ARG);
    struct { const char* what; void (*set)(chl_build_opts&); } bad_opts[] = {
        {"mode", [](chl_build_opts& x) { x.mode = 7; }},
        {"wg", [](chl_build_opts& x) { x.wg_size = 96; }},
        {"plain wg", [](chl_build_opts& x) { x.mode = CHL_MODE_PLAIN; x.wg_size = 1024; }},
        {"delta", [](chl_build_opts& x) { x.delta = -1; }},
        {"k", [](chl_build_opts& x) { x.roots_in_flight = -2; }},
        {"stride", [](chl_build_opts& x) { x.root_count = 2; x.root_stride = 0; }},
        {"range", [](chl_build_opts& x) { x.root_count = 2; x.root_stride = 5; }},
        {"prefix", [](chl_build_opts& x) { x.prune_hubs = 8193; }},
        {"hybrid", [](chl_build_opts& x) { x.hybrid_psi = -1; }},
        {"team", [](chl_build_opts& x) { x.team_wgs = 17; }},
    };
    for (auto& b : bad_opts) {
        chl_build_opts x = o;
        b.set(x);
        const int r = chl_build(&g, order, &x, nullptr, nullptr, &L);
        if (r != CHL_ERR_INVALID_ARG) std::fprintf(stderr, "option %s: %d\n", b.what, r);
        EXPECT(r == CHL_ERR_INVALID_ARG);
    }
    chl_allocator half{no_alloc, nullptr, nullptr};
    EXPECT(chl_build(&g, order, &o, &half, nullptr, &L) == CHL_ERR_INVALID_ARG ||
           chl_build(&g, order, &o, &half, nullptr, &L) == CHL_ERR_NO_DEVICE);
    // valid arguments: no usable device here
    const int r = chl_build(&g, order, &o, nullptr, nullptr, &L);
    EXPECT(r == CHL_ERR_NO_DEVICE || r == CHL_ERR_HIP);
    EXPECT(L == nullptr);
    EXPECT(chl_build_directed(nullptr, order, &o, nullptr, nullptr, &L) == CHL_ERR_INVALID_ARG);
    EXPECT(chl_build_directed(&g, order, &o, nullptr, nullptr, &L) != CHL_OK);

    // calls on a NULL handle
    int32_t n = 0;
    int64_t total = 0;
    EXPECT(chl_labels_info(nullptr, &n, &total) == CHL_ERR_INVALID_ARG);
    EXPECT(chl_labels_export(nullptr, nullptr, nullptr, nullptr, 1, nullptr) == CHL_ERR_INVALID_ARG);
    EXPECT(chl_labels_export_in(nullptr, nullptr, nullptr, nullptr, 1, nullptr) == CHL_ERR_INVALID_ARG);
    EXPECT(chl_labels_directed(nullptr, nullptr) == CHL_ERR_INVALID_ARG);
    EXPECT(chl_labels_hub_vertex(nullptr, nullptr, 1, nullptr) == CHL_ERR_INVALID_ARG);
    EXPECT(chl_query(nullptr, nullptr, 1, nullptr, nullptr) == CHL_ERR_INVALID_ARG);
    EXPECT(chl_build_stats(nullptr, nullptr, nullptr, 1, nullptr) == CHL_ERR_INVALID_ARG);
    EXPECT(chl_labels_parents(nullptr, &g, nullptr, nullptr, nullptr) == CHL_ERR_INVALID_ARG);
    EXPECT(chl_query_path_hops(nullptr, nullptr, nullptr, nullptr, 1, nullptr, nullptr, nullptr) ==
           CHL_ERR_INVALID_ARG);
    EXPECT(chl_query_paths(nullptr, nullptr, nullptr, nullptr, 1, nullptr, nullptr, nullptr) == CHL_ERR_INVALID_ARG);
    chl_labels_free(nullptr);

    // server: options, creation without a device, destruction of a partial server
    chl_server_opts so;
    chl_server_opts_default(nullptr);
    chl_server_opts_default(&so);
    EXPECT(so.max_batch > 0 && so.build_streams > 0);
    chl_server* s = nullptr;
    EXPECT(chl_server_create(&so, nullptr, nullptr) == CHL_ERR_INVALID_ARG);
    chl_server_opts sb = so;
    sb.max_batch = 0;
    EXPECT(chl_server_create(&sb, nullptr, &s) == CHL_ERR_INVALID_ARG);
    sb = so;
    sb.build_streams = 9;
    EXPECT(chl_server_create(&sb, nullptr, &s) == CHL_ERR_INVALID_ARG);
    chl_allocator nofree{no_alloc, nullptr, nullptr};
    EXPECT(chl_server_create(&so, &nofree, &s) == CHL_ERR_INVALID_ARG);
    chl_allocator al{no_alloc, no_free, nullptr};
    const int rs = chl_server_create(&so, &al, &s);
    if (rs == CHL_OK) chl_server_destroy(s);
    else EXPECT(rs == CHL_ERR_HIP);
    EXPECT(chl_server_build_footprint(nullptr, 10, 10) == 0);
    EXPECT(chl_server_budget_peak(nullptr) == 0);
    EXPECT(chl_server_start(nullptr) == CHL_ERR_INVALID_ARG);
    EXPECT(chl_server_wait(nullptr) == CHL_ERR_INVALID_ARG);
    EXPECT(chl_server_labels(nullptr, 0) == nullptr);
    chl_server_destroy(nullptr);
    int64_t done = 0;
    double ms = 0;
    EXPECT(chl_microbench_atomic_min(nullptr, 10, 32, 10, &done, &ms, nullptr) != CHL_OK);
    if (fails) return 1;
    std::printf("host driver: ok\n");
    return 0;
}
