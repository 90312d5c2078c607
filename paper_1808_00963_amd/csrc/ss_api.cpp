// Host side of libss: contexts, workspace, the recursion-level loop and the
// C ABI declared in include/ss.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/ss.h"
#include "ss_device.h"
#include "ss_internal.h"

using namespace ss;

namespace {
enum KernelId {
    K_INIT, K_ROOTS, K_BASE_W1, K_BASE_W4, K_BASE, K_SAMPLE, K_CLASSIFY, K_SCAN, K_SCATTER, K_CHILDREN,
    K_LCP_FILL, K_PERSIST, K_COUNT
};
const char* const KNAME[K_COUNT] = {"k_init", "k_roots", "k_base_wave1", "k_base_wave4", "k_base", "k_sample",
                                    "k_classify", "k_scan", "k_scatter", "k_children", "k_lcp_fill", "k_persist"};
const char* const KUNIT[K_COUNT] = {"strings", "sets", "strings", "strings", "strings", "segments", "strings",
                                    "counters", "strings", "segments", "boundaries", "strings"};

// Event pairs around kernel launches, resolved at the next host sync.
struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> ev;  // pairs (start, stop)
    std::vector<int> kid;
    std::vector<double> units;
    size_t used = 0;
    double ms[K_COUNT] = {};
    double unit_sum[K_COUNT] = {};
    uint32_t launches[K_COUNT] = {};
};
}  // namespace

struct ss_ctx {
    int device = 0;
    size_t scratch_limit = 0;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    uint32_t ws_n = 0;  // largest n the workspace was laid out for
    Work work{};
    Ctl* host_ctl = nullptr;  // pinned copy of the device control block
    ss_config cfg{10, 64, 1024, 0};
    ss_status sticky = SS_OK;
    ss_stats stats{};
    Profiler prof;
    uint32_t persist_blocks = 0;  // co-resident work groups of the persistent kernel
};

struct ss_graph {
    ss_ctx* ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

constexpr uint32_t MAX_LEVELS = 1u << 17;

void clamp_config(ss_config* c) {
    c->max_log_splitters = std::min<uint32_t>(std::max<uint32_t>(c->max_log_splitters, 1), MAX_LOGV);
    c->bucket_target = std::min<uint32_t>(std::max<uint32_t>(c->bucket_target, 16), 1u << 20);
    c->base_max = std::min<uint32_t>(std::max<uint32_t>(c->base_max, 64), BASE_CAP);
    c->persistent = c->persistent ? 1u : 0u;
}

// Worst-case pool sizes of one recursion level for n strings (the segments
// of a level are disjoint, so their sizes sum to at most n).
Caps caps_for(uint32_t n, const ss_config& c) {
    uint64_t N = n;
    Caps k{};
    uint64_t dist = N / (c.base_max + 1) + 2;
    k.dist = (uint32_t)dist;
    k.tiles = (uint32_t)(N / TILE + dist + 2);
    k.base[0] = (uint32_t)(N / 2 + 2);
    k.base[1] = (uint32_t)(N / (CLS_MAX[0] + 1) + 2);
    k.base[2] = (uint32_t)(N / (CLS_MAX[1] + 1) + 2);
    // sum of (2v+1) * tiles: at most MAX_BUCKETS per tile of a multi-tile
    // segment, at most max(3, 2 size / bucket_target) for one-tile segments
    k.cnt = (uint32_t)std::min<uint64_t>(
        (uint64_t)MAX_BUCKETS * (N / TILE + dist) + 2 * N / c.bucket_target + 3 * dist + 4096, 0xFFFFFFF0ull);
    k.tree = (uint32_t)(2 * dist + N / c.bucket_target + 2 * (1u << MAX_LOGV));
    k.pend = (uint32_t)(N + 1);
    return k;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Lays out the workspace; with base == nullptr only computes the size.
size_t layout(uint32_t n, const Caps& k, char* base, Work* w) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    size_t N = std::max<uint32_t>(n, 1);
    Work t{};
    for (int i = 0; i < 2; ++i) t.buf[i] = (Elem*)take(sizeof(Elem) * N);
    t.bkt = (uint16_t*)take(sizeof(uint16_t) * N);
    for (int i = 0; i < 2; ++i) t.cnt[i] = (uint32_t*)take(sizeof(uint32_t) * k.cnt);
    t.partial = (uint32_t*)take(sizeof(uint32_t) * (k.cnt / 4096 + 4));
    for (int i = 0; i < 2; ++i) t.dist[i] = (Seg*)take(sizeof(Seg) * k.dist);
    for (int c = 0; c < NCLS; ++c)
        for (int i = 0; i < 2; ++i) t.base[c][i] = (BaseSeg*)take(sizeof(BaseSeg) * k.base[c]);
    for (int i = 0; i < 2; ++i) t.tile_seg[i] = (uint32_t*)take(sizeof(uint32_t) * k.tiles);
    for (int i = 0; i < 2; ++i) t.tree_key[i] = (uint64_t*)take(sizeof(uint64_t) * k.tree);
    for (int i = 0; i < 2; ++i) t.tree_r[i] = (uint8_t*)take(k.tree);
    t.pend = (uint2*)take(sizeof(uint2) * k.pend);
    t.ctl = (Ctl*)take(sizeof(Ctl));
    t.bar = (GridBar*)take(sizeof(GridBar));
    t.caps = k;
    if (w) *w = t;
    return off;
}

ss_status hip_status(hipError_t e) { return e == hipSuccess ? SS_OK : SS_HIP_ERROR; }

#define SS_TRY(expr)                                  \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return SS_HIP_ERROR;    \
    } while (0)

ss_status ensure_workspace(ss_ctx* ctx, uint32_t n) {
    if (ctx->ws && n <= ctx->ws_n) return SS_OK;
    uint32_t want = std::max<uint32_t>(n, std::min<uint32_t>(ctx->ws_n ? ctx->ws_n * 2u : n, 0xFFFFFFFEu));
    want = std::max(want, n);
    Caps k = caps_for(want, ctx->cfg);
    size_t bytes = layout(want, k, nullptr, nullptr);
    if (ctx->scratch_limit && bytes > ctx->scratch_limit) {
        want = n;
        k = caps_for(want, ctx->cfg);
        bytes = layout(want, k, nullptr, nullptr);
        if (bytes > ctx->scratch_limit) return SS_OUT_OF_MEMORY;
    }
    if (ctx->ws) {
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_n = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return SS_OUT_OF_MEMORY;
    }
    ctx->ws = p;
    ctx->ws_bytes = bytes;
    ctx->ws_n = want;
    layout(want, k, (char*)p, &ctx->work);
    return SS_OK;
}

ss_status device_error_status(uint32_t err) {
    if (err & ERR_OFFSETS) return SS_LIMIT;
    if (err & ERR_SETS) return SS_INVALID_ARG;
    return SS_INTERNAL;
}

// Launches `fn` and, when profiling, brackets it with an event pair.
template <typename F>
hipError_t timed(ss_ctx* ctx, hipStream_t s, int id, double units, F&& fn) {
    Profiler& P = ctx->prof;
    if (!P.on) return fn();
    if (P.used * 2 + 2 > P.ev.size()) {
        for (int i = 0; i < 64; ++i) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            P.ev.push_back(e);
        }
    }
    hipEvent_t a = P.ev[2 * P.used], b = P.ev[2 * P.used + 1];
    hipError_t r = hipEventRecord(a, s);
    if (r != hipSuccess) return r;
    r = fn();
    if (r != hipSuccess) return r;
    r = hipEventRecord(b, s);
    if (r != hipSuccess) return r;
    if (P.kid.size() <= P.used) { P.kid.resize(P.used + 1); P.units.resize(P.used + 1); }
    P.kid[P.used] = id;
    P.units[P.used] = units;
    ++P.used;
    return hipSuccess;
}

// Accumulates the durations of all recorded pairs (stream already synced).
void resolve_timings(ss_ctx* ctx) {
    Profiler& P = ctx->prof;
    for (size_t i = 0; i < P.used; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, P.ev[2 * i], P.ev[2 * i + 1]) == hipSuccess) {
            P.ms[P.kid[i]] += ms;
            P.unit_sum[P.kid[i]] += P.units[i];
            P.launches[P.kid[i]] += 1;
        }
    }
    P.used = 0;
}

// Reads the control block into the pinned host copy (synchronous).
ss_status read_ctl(ss_ctx* ctx, hipStream_t s) {
    SS_TRY(hipMemcpyAsync(ctx->host_ctl, ctx->work.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    SS_TRY(hipStreamSynchronize(s));
    if (ctx->prof.used) resolve_timings(ctx);
    return SS_OK;
}

// Reset + the persistent kernel (no host synchronisation; capturable).
ss_status enqueue_persistent(ss_ctx* ctx, const Params& p, const uint32_t* set_begin, uint32_t nroots,
                             hipStream_t s) {
    if (ctx->persist_blocks == 0) {
        uint32_t b = 0;
        SS_TRY(persistent_capacity(ctx->device, &b));
        if (b == 0) return SS_HIP_ERROR;
        ctx->persist_blocks = b;
    }
    const Work& w = ctx->work;
    SS_TRY(launch_reset(w, s));
    SS_TRY(timed(ctx, s, K_PERSIST, p.n, [&] {
        return launch_persistent(w, p, set_begin, nroots, ctx->persist_blocks, s);
    }));
    return SS_OK;
}

// The sort: initial key gather, roots, then one iteration per recursion
// level over all live segments, then the boundary LCPs.
ss_status run_sort(ss_ctx* ctx, const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                   const uint32_t* set_begin, uint32_t num_sets, uint32_t* perm, uint32_t* lcp,
                   hipStream_t s) {
    ctx->stats = ss_stats{};
    if (n == 0) return SS_OK;
    int cur_dev = -1;
    SS_TRY(hipGetDevice(&cur_dev));
    if (cur_dev != ctx->device) SS_TRY(hipSetDevice(ctx->device));
    ss_status st = ensure_workspace(ctx, n);
    if (st != SS_OK) return st;
    const Work& w = ctx->work;
    Params p{chars, offsets, n, perm, lcp, ctx->cfg.max_log_splitters, ctx->cfg.bucket_target, ctx->cfg.base_max};

    const uint32_t nroots = set_begin ? num_sets : 1;
    if (ctx->cfg.persistent) {
        if ((st = enqueue_persistent(ctx, p, set_begin, nroots, s)) != SS_OK) return st;
        if ((st = read_ctl(ctx, s)) != SS_OK) return st;
        ctx->stats.pending_lcps = ctx->host_ctl->n_pend;
        ctx->stats.base_rounds = ctx->host_ctl->base_rounds;
        if (ctx->host_ctl->err) return device_error_status(ctx->host_ctl->err);
        return SS_OK;
    }
    SS_TRY(launch_reset(w, s));
    SS_TRY(timed(ctx, s, K_INIT, n, [&] { return launch_init(w, p, s); }));
    SS_TRY(timed(ctx, s, K_ROOTS, nroots, [&] { return launch_roots(w, p, set_begin, nroots, s); }));
    int cur = 0;
    uint32_t level = 0;
    for (;;) {
        if ((st = read_ctl(ctx, s)) != SS_OK) return st;
        if (ctx->host_ctl->err) return device_error_status(ctx->host_ctl->err);
        const Counts c = ctx->host_ctl->c[cur];
        ctx->stats.levels = level + 1;
        ctx->stats.dist_segments += c.n_dist;
        ctx->stats.dist_tiles += c.n_tiles;
        ctx->stats.base_segments += c.n_base[0] + c.n_base[1] + c.n_base[2];
        ctx->stats.max_depth = std::max(ctx->stats.max_depth, c.max_depth);
        for (int cls = 0; cls < NCLS; ++cls) {
            if (!c.n_base[cls]) continue;
            const uint32_t nb = c.n_base[cls];
            SS_TRY(timed(ctx, s, K_BASE_W1 + cls, c.base_strings[cls],
                         [&] { return launch_base(w, p, cur, cls, nb, s); }));
        }
        if (c.n_dist == 0) break;
        SS_TRY(launch_zero_counts(w, cur ^ 1, s));
        SS_TRY(timed(ctx, s, K_SAMPLE, c.n_dist, [&] { return launch_sample(w, p, cur, c.n_dist, s); }));
        SS_TRY(timed(ctx, s, K_CLASSIFY, c.dist_strings,
                     [&] { return launch_classify(w, p, cur, c.n_tiles, c.n_dist, s); }));
        SS_TRY(timed(ctx, s, K_SCAN, c.n_cnt, [&] { return launch_scan(w, cur, c.n_cnt, s); }));
        SS_TRY(timed(ctx, s, K_SCATTER, c.dist_strings,
                     [&] { return launch_scatter(w, p, cur, c.n_tiles, c.n_dist, s); }));
        SS_TRY(timed(ctx, s, K_CHILDREN, c.n_dist, [&] { return launch_children(w, p, cur, c.n_dist, s); }));
        cur ^= 1;
        if (++level >= MAX_LEVELS) return SS_INTERNAL;
    }
    // the pending count is known on the device only; units are added below
    SS_TRY(timed(ctx, s, K_LCP_FILL, 0.0, [&] { return launch_lcp_fill(w, p, s); }));
    if ((st = read_ctl(ctx, s)) != SS_OK) return st;
    if (ctx->prof.on) ctx->prof.unit_sum[K_LCP_FILL] += ctx->host_ctl->n_pend;
    ctx->stats.pending_lcps = ctx->host_ctl->n_pend;
    ctx->stats.base_rounds = ctx->host_ctl->base_rounds;
    if (ctx->host_ctl->err) return device_error_status(ctx->host_ctl->err);
    return SS_OK;
}

ss_status sort_checked(ss_ctx* ctx, const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                       const uint32_t* set_begin, uint32_t num_sets, uint32_t* perm, uint32_t* lcp,
                       void* stream) {
    if (!ctx) return SS_INVALID_ARG;
    if (n == 0) return SS_OK;
    if (n > 0xFFFFFFFEu) return SS_LIMIT;
    if (!offsets || !perm || !lcp) return SS_INVALID_ARG;  // chars may be NULL when all strings are empty
    if ((void*)perm == (void*)lcp) return SS_INVALID_ARG;
    ss_status st = run_sort(ctx, chars, offsets, n, set_begin, num_sets, perm, lcp, (hipStream_t)stream);
    if (st != SS_OK && st != SS_INVALID_ARG) ctx->sticky = st;
    return st;
}

std::mutex g_mu;
std::map<int, std::unique_ptr<ss_ctx, void (*)(ss_ctx*)>>* g_ctx = nullptr;

}  // namespace

extern "C" {

const char* ss_status_string(ss_status s) {
    switch (s) {
    case SS_OK: return "ok";
    case SS_INVALID_ARG: return "invalid argument";
    case SS_OUT_OF_MEMORY: return "out of device memory";
    case SS_HIP_ERROR: return "HIP runtime error";
    case SS_LIMIT: return "input beyond limits (n, string length or offsets)";
    case SS_REJECTED: return "request rejected";
    case SS_TIMEOUT: return "timeout";
    case SS_INTERNAL: return "internal error";
    default: return "unknown status";
    }
}

const char* ss_version(void) { return "libss 0.1 (gfx950)"; }

ss_status ss_ctx_create(ss_ctx** out, int device, size_t scratch_limit) {
    if (!out) return SS_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SS_INVALID_ARG;
    auto* c = new ss_ctx();
    c->device = device;
    c->scratch_limit = scratch_limit;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(device);
    hipError_t e = hipHostMalloc((void**)&c->host_ctl, sizeof(Ctl), hipHostMallocDefault);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        delete c;
        return SS_HIP_ERROR;
    }
    *out = c;
    return SS_OK;
}

void ss_ctx_destroy(ss_ctx* ctx) {
    if (!ctx) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    for (hipEvent_t e : ctx->prof.ev) (void)hipEventDestroy(e);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->host_ctl) (void)hipHostFree(ctx->host_ctl);
    (void)hipSetDevice(prev);
    delete ctx;
}

ss_status ss_get_config(const ss_ctx* ctx, ss_config* cfg) {
    if (!ctx || !cfg) return SS_INVALID_ARG;
    *cfg = ctx->cfg;
    return SS_OK;
}

ss_status ss_set_config(ss_ctx* ctx, const ss_config* cfg) {
    if (!ctx || !cfg) return SS_INVALID_ARG;
    ss_config c = *cfg;
    clamp_config(&c);
    bool relayout = c.base_max != ctx->cfg.base_max || c.bucket_target != ctx->cfg.bucket_target;
    ctx->cfg = c;
    if (relayout && ctx->ws) {
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_n = 0;
    }
    return SS_OK;
}

ss_status ss_workspace_query(const ss_ctx* ctx, uint32_t n, size_t* bytes) {
    if (!bytes) return SS_INVALID_ARG;
    ss_config c = ctx ? ctx->cfg : ss_config{10, 64, 1024, 0};
    *bytes = layout(n, caps_for(n, c), nullptr, nullptr);
    return SS_OK;
}

ss_status ss_sort_ex(ss_ctx* ctx, const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                     uint32_t* perm_out, uint32_t* lcp_out, void* stream) {
    return sort_checked(ctx, chars, offsets, n, nullptr, 1, perm_out, lcp_out, stream);
}

ss_status ss_sort(const uint8_t* chars, const uint64_t* offsets, uint32_t n, uint32_t* perm_out,
                  uint32_t* lcp_out, void* stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SS_HIP_ERROR;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ctx) g_ctx = new std::map<int, std::unique_ptr<ss_ctx, void (*)(ss_ctx*)>>();
    auto it = g_ctx->find(dev);
    if (it == g_ctx->end()) {
        ss_ctx* c = nullptr;
        ss_status st = ss_ctx_create(&c, dev, 0);
        if (st != SS_OK) return st;
        it = g_ctx->emplace(dev, std::unique_ptr<ss_ctx, void (*)(ss_ctx*)>(c, ss_ctx_destroy)).first;
    }
    return sort_checked(it->second.get(), chars, offsets, n, nullptr, 1, perm_out, lcp_out, stream);
}

ss_status ss_sort_batch(ss_ctx* ctx, const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                        const uint32_t* set_begin, uint32_t num_sets, uint32_t* perm_out,
                        uint32_t* lcp_out, void* stream) {
    if (!ctx) return SS_INVALID_ARG;
    if (num_sets == 0) return n == 0 ? SS_OK : SS_INVALID_ARG;
    if (!set_begin) return SS_INVALID_ARG;
    return sort_checked(ctx, chars, offsets, n, set_begin, num_sets, perm_out, lcp_out, stream);
}

ss_status ss_graph_create_batch(ss_ctx* ctx, const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                                const uint32_t* set_begin, uint32_t num_sets, uint32_t* perm_out,
                                uint32_t* lcp_out, ss_graph** graph_out) {
    if (!ctx || !graph_out || !offsets || !perm_out || !lcp_out || !set_begin || num_sets == 0 || n == 0)
        return SS_INVALID_ARG;
    if (n > 0xFFFFFFFEu) return SS_LIMIT;
    *graph_out = nullptr;
    int cur_dev = -1;
    SS_TRY(hipGetDevice(&cur_dev));
    if (cur_dev != ctx->device) SS_TRY(hipSetDevice(ctx->device));
    ss_status st = ensure_workspace(ctx, n);  // no allocation may happen during capture
    if (st != SS_OK) return st;
    hipStream_t cs = nullptr;
    SS_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    const bool prof = ctx->prof.on;
    ctx->prof.on = false;  // no event records inside the graph
    Params p{chars, offsets, n, perm_out, lcp_out, ctx->cfg.max_log_splitters, ctx->cfg.bucket_target,
             ctx->cfg.base_max};
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = enqueue_persistent(ctx, p, set_begin, num_sets, cs);
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (st == SS_OK && e2 != hipSuccess) st = SS_HIP_ERROR;
    } else {
        st = SS_HIP_ERROR;
    }
    ctx->prof.on = prof;
    (void)hipStreamDestroy(cs);
    if (st != SS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return SS_HIP_ERROR;
    }
    auto* gr = new ss_graph();
    gr->ctx = ctx;
    gr->graph = g;
    gr->exec = ex;
    *graph_out = gr;
    return SS_OK;
}

ss_status ss_graph_launch(ss_graph* graph, void* stream) {
    if (!graph || !graph->exec) return SS_INVALID_ARG;
    return hipGraphLaunch(graph->exec, (hipStream_t)stream) == hipSuccess ? SS_OK : SS_HIP_ERROR;
}

void ss_graph_destroy(ss_graph* graph) {
    if (!graph) return;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
}

ss_status ss_ctx_sync(ss_ctx* ctx, void* stream) {
    if (!ctx) return SS_INVALID_ARG;
    ss_status st = read_ctl(ctx, (hipStream_t)stream);
    if (st != SS_OK) return st;
    if (ctx->host_ctl->err) {
        st = device_error_status(ctx->host_ctl->err);
        ctx->sticky = st;
        return st;
    }
    return SS_OK;
}

ss_status ss_get_last_error(const ss_ctx* ctx) { return ctx ? ctx->sticky : SS_INVALID_ARG; }

void ss_clear_error(ss_ctx* ctx) {
    if (ctx) ctx->sticky = SS_OK;
}

ss_status ss_get_stats(const ss_ctx* ctx, ss_stats* st) {
    if (!ctx || !st) return SS_INVALID_ARG;
    *st = ctx->stats;
    return SS_OK;
}

ss_status ss_set_profiling(ss_ctx* ctx, int enable) {
    if (!ctx) return SS_INVALID_ARG;
    ctx->prof.on = enable != 0;
    return SS_OK;
}

ss_status ss_get_kernel_times(const ss_ctx* ctx, ss_kernel_time* out, uint32_t max_entries, uint32_t* n_entries) {
    if (!ctx || !n_entries || (max_entries && !out)) return SS_INVALID_ARG;
    uint32_t k = 0;
    for (int i = 0; i < K_COUNT && k < max_entries; ++i, ++k)
        out[k] = ss_kernel_time{KNAME[i], KUNIT[i], ctx->prof.launches[i], ctx->prof.ms[i], ctx->prof.unit_sum[i]};
    *n_entries = K_COUNT;
    return SS_OK;
}

void ss_reset_kernel_times(ss_ctx* ctx) {
    if (!ctx) return;
    Profiler& P = ctx->prof;
    P.used = 0;
    for (int i = 0; i < K_COUNT; ++i) P.ms[i] = P.unit_sum[i] = 0, P.launches[i] = 0;
}

// ---- host-side test entry points ----

uint64_t ss_host_key(const uint8_t* s, uint64_t len, uint64_t h, uint32_t* r_out) {
    uint32_t rem = len > h ? (uint32_t)std::min<uint64_t>(len - h, 8) : 0;
    if (r_out) *r_out = rem;
    if (rem == 0) return 0;
    // the same aligned-word assembly as the kernels
    uintptr_t a = (uintptr_t)(s + h);
    uint32_t sh = (uint32_t)(a & 7);
    const uint8_t* base = (const uint8_t*)(a & ~(uintptr_t)7);
    uint64_t w0 = 0, w1 = 0;
    // only bytes that belong to the string are read; the rest stay zero
    for (uint32_t b = 0; b < 8; ++b)
        if (b >= sh && b - sh < rem) w0 |= (uint64_t)base[b] << (8 * b);
    for (uint32_t b = 0; b < 8; ++b)
        if (8 + b - sh < rem) w1 |= (uint64_t)base[8 + b] << (8 * b);
    return key_from_words(w0, w1, sh, rem);
}

uint32_t ss_host_level_index(uint32_t j, uint32_t d) { return level_index(j, d); }
uint32_t ss_host_inorder_index(uint32_t l, uint32_t d) { return inorder_index(l, d); }

int ss_host_classify(const uint64_t* xk, const uint32_t* xr, uint32_t d, const uint64_t* ck,
                     const uint32_t* cr, uint32_t m, uint32_t* buckets) {
    if (d < 1 || d > 16) return 1;
    uint32_t v = (1u << d) - 1;
    std::unique_ptr<uint64_t[]> tk(new uint64_t[v + 1]);
    std::unique_ptr<uint32_t[]> tr(new uint32_t[v + 1]);
    for (uint32_t j = 0; j < v; ++j) {
        uint32_t l = level_index(j, d);
        tk[l] = xk[j];
        tr[l] = xr[j];
    }
    const uint64_t* tkp = tk.get();
    const uint32_t* trp = tr.get();
    for (uint32_t i = 0; i < m; ++i) buckets[i] = classify(ck[i], cr[i], tkp, trp, d);
    return 0;
}

int ss_host_select_splitters(const uint64_t* sk, const uint32_t* sr, uint32_t a, uint32_t d, uint64_t* xk,
                             uint32_t* xr) {
    if (d < 1 || d > 16 || a == 0) return 1;
    uint32_t v = (1u << d) - 1;
    std::unique_ptr<uint64_t[]> TK(new uint64_t[v + 1]);
    std::unique_ptr<uint32_t[]> TR(new uint32_t[v + 1]);
    std::unique_ptr<uint32_t[]> NL(new uint32_t[v + 1]);
    std::unique_ptr<uint32_t[]> NH(new uint32_t[v + 1]);
    NL[1] = 0;
    NH[1] = a;
    for (uint32_t L = 0; L < d; ++L) {
        for (uint32_t q = 1u << L; q < (2u << L); ++q) {
            uint32_t lo = NL[q], hi = NH[q], llo = 0, lhi = 0, rlo = 0, rhi = 0;
            if (lo < hi) {
                uint32_t mid, lh, rl;
                select_node(sk, sr, lo, hi, &mid, &lh, &rl);
                TK[q] = sk[mid];
                TR[q] = sr[mid];
                llo = lo; lhi = lh; rlo = rl; rhi = hi;
            } else {
                TK[q] = TK[q >> 1];
                TR[q] = TR[q >> 1];
            }
            if (L + 1 < d) {
                NL[2 * q] = llo; NH[2 * q] = lhi;
                NL[2 * q + 1] = rlo; NH[2 * q + 1] = rhi;
            }
        }
    }
    for (uint32_t j = 0; j < v; ++j) {
        uint32_t l = level_index(j, d);
        xk[j] = TK[l];
        xr[j] = TR[l];
    }
    return 0;
}

}  // extern "C"
