// Host side of libss: contexts, workspace, the recursion-level loop and the
// C ABI declared in include/ss.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/ss.h"
#include "ss_device.h"
#include "ss_internal.h"

using namespace ss;

namespace {
enum KernelId {
    K_INIT, K_ROOTS, K_BASE_W1, K_BASE_W2, K_BASE_W4, K_BASE, K_SAMPLE, K_CLASSIFY, K_SCAN, K_SCATTER, K_CHILDREN,
    K_LCP_FILL, K_PERSIST, K_LEVEL_BEGIN, K_MERGE_SPLIT, K_MERGE, K_SA_STRINGS, K_SA_RENAME, K_ALPHABET, K_COUNT
};
const char* const KNAME[K_COUNT] = {"k_init", "k_roots", "k_base_wave1", "k_base_wave2", "k_base_wave4", "k_base",
                                    "k_sample", "k_classify", "k_scan", "k_scatter", "k_children", "k_lcp_fill",
                                    "k_persist", "k_level_begin", "k_merge_split", "k_merge_tile", "k_sa_strings",
                                    "k_sa_rename", "k_alphabet"};
const char* const KUNIT[K_COUNT] = {"strings", "sets", "strings", "strings", "strings", "strings", "segments",
                                    "strings", "counters", "strings", "segments", "boundaries", "strings", "levels",
                                    "tiles", "strings", "suffixes", "suffixes", "strings"};

// What a timed launch counts (resolved once the sort's control block is on
// the host): a constant, or a field of the work counts of its level.
enum UnitField { U_CONST = -1, U_BASE0 = 0, U_DIST = NCLS, U_DIST_STRINGS, U_CNT, U_PEND };
struct UnitSpec {
    double units = 0.0;
    int field = U_CONST;
    uint32_t level = 0;
};
UnitSpec units_const(double u) { return UnitSpec{u, U_CONST, 0}; }
UnitSpec units_level(int field, uint32_t level) { return UnitSpec{0.0, field, level}; }

// Event pairs around kernel launches, resolved after the sort completes.
struct Profiler {
    bool on = false;
    uint32_t mask = ~0u;  // kernels (bit per KernelId) that get event pairs
    std::vector<hipEvent_t> ev;  // pairs (start, stop)
    std::vector<int> kid;
    std::vector<UnitSpec> spec;
    size_t used = 0;
    double ms[K_COUNT] = {};
    double unit_sum[K_COUNT] = {};
    uint32_t launches[K_COUNT] = {};
};

// A sort workspace: one device allocation laid out as a Work, with the
// string count and the configuration its pools were sized for.
struct Ws {
    void* mem = nullptr;
    size_t bytes = 0;
    uint32_t n = 0;
    uint32_t bucket_target = 0, base_max = 0;
    Work work{};
};
}  // namespace

struct ss_graph;

struct ss_ctx {
    int device = 0;
    size_t scratch_limit = 0;
    Ws ws;                    // workspace of the context's own sorts
    Ctl* host_ctl = nullptr;  // pinned: the control block after the last sort
    ss_config cfg{10, 64, 1024, SS_MODE_LEVELS, SS_ALPHABET_BYTES};
    uint32_t alphabet_retries = 0;  // of the last sort: compressed keys met a byte outside the probed set
    ss_status sticky = SS_OK;
    ss_stats stats{};
    bool pending = false;     // host_ctl of the last sort not yet absorbed
    uint32_t level_hint = 0;  // levels the last completed sort needed
    Profiler prof;
    KernelCaps kc{};          // resident work groups of each level kernel
    bool kc_ok = false;
    // merge workspace (grow-only): device part and pinned staging of the
    // task tables and the error word
    void* mws = nullptr;
    size_t mws_bytes = 0;
    void* mhost = nullptr;
    size_t mhost_bytes = 0;
    // suffix-array workspace (grow-only) and a pinned word for the group count
    void* saws = nullptr;
    size_t saws_bytes = 0;
    uint32_t* sa_host = nullptr;
    // two library streams (default priority) for the steps of a sort that
    // overlap others: the first level's sampling beside the key gather, the
    // base cases of a level beside its distribution steps; fork/join events;
    // `done` marks the end of the last sort (the workspace is free again)
    hipStream_t side[2] = {nullptr, nullptr};
    hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr}, done = nullptr;
    bool done_recorded = false;
    std::vector<ss_graph*> graphs;  // live graphs (their errors are read by ss_ctx_sync)
};

struct ss_graph {
    ss_ctx* ctx = nullptr;
    Ws ws;  // the graph's own workspace, bound into its kernels
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t levels = 0;  // levels enqueued as separate launches before the persistent tail
};

namespace {

constexpr uint32_t MAX_LEVELS = 1u << 17;
constexpr uint32_t DEFAULT_LEVELS = 4;   // level launches of a context's first sort
constexpr uint32_t MAX_LEVEL_LAUNCHES = 32;
// Smallest sort whose first-level sampling runs beside the key gather (the
// gather of 2^21 strings takes about as long as one sampling step).
constexpr uint32_t FORK_MIN = 1u << 21;
static_assert(NCLS == 4, "ss_stats reports four base-case classes");

static_assert(SS_ALPHABET_AUTO == ALPHABET_AUTO && SS_ALPHABET_BYTES == ALPHABET_BYTES &&
                  SS_ALPHABET_COMPRESS == ALPHABET_COMPRESS,
              "alphabet setting passed to the kernels");

void clamp_config(ss_config* c) {
    c->max_log_splitters = std::min<uint32_t>(std::max<uint32_t>(c->max_log_splitters, 1), MAX_LOGV);
    c->bucket_target = std::min<uint32_t>(std::max<uint32_t>(c->bucket_target, 16), 1u << 20);
    c->base_max = std::min<uint32_t>(std::max<uint32_t>(c->base_max, 64), BASE_CAP);
    if (c->mode > SS_MODE_HOST_LEVELS) c->mode = SS_MODE_LEVELS;
    if (c->alphabet > SS_ALPHABET_COMPRESS) c->alphabet = SS_ALPHABET_BYTES;
}

// Worst-case pool sizes of one recursion level for n strings (the segments
// of a level are disjoint, so their sizes sum to at most n).
//   counters: a distribution segment of s strings has T = ceil(s / TILE)
//   tiles and k = 2v+1 <= min(MAX_BUCKETS, max(3, 2 s / bucket_target))
//   buckets; with several tiles k T < MAX_BUCKETS * 2 s / TILE < s / 2, with
//   one tile k T <= 3 + 2 s / bucket_target.  Summed: n/2 + 2n/bt + 3 dist.
//   tree slots: v + 1 <= max(2, s / bucket_target) per segment.
Caps caps_for(uint32_t n, uint32_t bucket_target, uint32_t base_max) {
    uint64_t N = n;
    Caps k{};
    uint64_t dist = N / (base_max + 1) + 2;
    k.dist = (uint32_t)dist;
    k.tiles = (uint32_t)(N / TILE + dist + 2);
    k.base[0] = (uint32_t)(N / 2 + 2);
    for (int c = 1; c < NCLS; ++c) k.base[c] = (uint32_t)(N / (CLS_MAX[c - 1] + 1) + 2);
    static_assert(4 * MAX_BUCKETS <= TILE, "multi-tile counter bound");
    k.cnt = (uint32_t)std::min<uint64_t>(N / 2 + 2 * N / bucket_target + 3 * dist + 4096, 0xFFFFFFF0ull);
    k.tree = (uint32_t)(2 * dist + N / bucket_target + 2 * (1u << MAX_LOGV));
    k.pend = (uint32_t)(N + 1);
    return k;
}
Caps caps_for(uint32_t n, const ss_config& c) { return caps_for(n, c.bucket_target, c.base_max); }

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
    t.wide = N >= NARROW_MAX_N ? 1u : 0u;
    for (int i = 0; i < 2; ++i) {
        t.rec[i] = (Rec*)take(sizeof(Rec) * N);
        t.rw[i] = t.wide ? (uint8_t*)take(N) : nullptr;
    }
    t.bkt = (uint16_t*)take(sizeof(uint16_t) * N);
    for (int i = 0; i < 2; ++i) t.cnt[i] = (uint32_t*)take(sizeof(uint32_t) * k.cnt);
    t.partial = (uint32_t*)take(sizeof(uint32_t) * (k.cnt / 4096 + 4));
    for (int i = 0; i < 2; ++i) t.dist[i] = (Seg*)take(sizeof(Seg) * k.dist);
    for (int c = 0; c < NCLS; ++c)
        for (int i = 0; i < 2; ++i) t.base[c][i] = (BaseSeg*)take(sizeof(BaseSeg) * k.base[c]);
    for (int i = 0; i < 2; ++i) t.tile_seg[i] = (uint32_t*)take(sizeof(uint32_t) * k.tiles);
    for (int i = 0; i < 2; ++i) t.tree_key[i] = (uint64_t*)take(sizeof(uint64_t) * k.tree);
    for (int i = 0; i < 2; ++i) t.tree_r[i] = (uint8_t*)take(k.tree);
    for (int i = 0; i < 2; ++i) t.tree_next[i] = (uint64_t*)take(sizeof(uint64_t) * k.tree);
    for (int i = 0; i < 2; ++i) t.tree_diff[i] = (uint32_t*)take(sizeof(uint32_t) * k.tree);
    t.pend = (Pend*)take(sizeof(Pend) * k.pend);
    t.pend2 = nullptr;
    t.ctl = (Ctl*)take(sizeof(Ctl));
    t.feed = (FeedLine*)take(sizeof(FeedLine) * FEED_LINES);
    t.bar = (GridBar*)take(sizeof(GridBar));
    t.zero_base = (uint32_t*)take(256);
    t.set_base = t.zero_base;  // a plain sort is one set starting at 0
    t.remaining = nullptr;
    t.done = nullptr;
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

void ws_free(Ws& ws) {
    if (ws.mem) (void)hipFree(ws.mem);
    ws = Ws{};
}

// Makes `ws` hold a sort of n strings under configuration `c`: a new layout
// when n is larger than the current one or when c's pools are larger
// (smaller bucket target or base-case size).  The caller must make sure no
// sort still uses the old allocation.
ss_status ws_ensure(Ws& ws, uint32_t n, const ss_config& c, size_t limit, bool* moved = nullptr) {
    if (moved) *moved = false;
    const bool fits = ws.mem && n <= ws.n && c.bucket_target >= ws.bucket_target && c.base_max >= ws.base_max;
    if (fits) return SS_OK;
    uint32_t want = std::max<uint32_t>(n, std::min<uint32_t>(ws.n ? ws.n * 2u : n, 0xFFFFFFFEu));
    want = std::max(want, n);
    // pools for the smaller of the old and new parameters, so switching back
    // does not lay out again
    const uint32_t bt = ws.mem ? std::min(c.bucket_target, ws.bucket_target) : c.bucket_target;
    const uint32_t bm = ws.mem ? std::min(c.base_max, ws.base_max) : c.base_max;
    Caps k = caps_for(want, bt, bm);
    size_t bytes = layout(want, k, nullptr, nullptr);
    if (limit && bytes > limit) {
        want = n;
        k = caps_for(want, c);
        bytes = layout(want, k, nullptr, nullptr);
        if (bytes > limit) return SS_OUT_OF_MEMORY;
    }
    ws_free(ws);
    if (moved) *moved = true;
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return SS_OUT_OF_MEMORY;
    }
    ws.mem = p;
    ws.bytes = bytes;
    ws.n = want;
    ws.bucket_target = bt;
    ws.base_max = bm;
    layout(want, k, (char*)p, &ws.work);
    // a fresh allocation holds whatever the memory held before; the sticky
    // error word is kept across resets, so it starts at zero here
    // (synchronous, before any sort can use the workspace)
    const Ctl zero{};
    if (hipMemcpy(ws.work.ctl, &zero, sizeof(Ctl), hipMemcpyHostToDevice) != hipSuccess) {
        ws_free(ws);
        return SS_HIP_ERROR;
    }
    return SS_OK;
}

ss_status device_error_status(uint32_t err) {
    if (err & ERR_OFFSETS) return SS_LIMIT;
    if (err & ERR_SETS) return SS_INVALID_ARG;
    return SS_INTERNAL;
}

// Launches `fn` and, when profiling, brackets it with an event pair.
template <typename F>
hipError_t timed(Profiler* prof, hipStream_t s, int id, UnitSpec u, F&& fn) {
    if (!prof || !prof->on || !((prof->mask >> id) & 1u)) return fn();
    Profiler& P = *prof;
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
    if (P.kid.size() <= P.used) { P.kid.resize(P.used + 1); P.spec.resize(P.used + 1); }
    P.kid[P.used] = id;
    P.spec[P.used] = u;
    ++P.used;
    return hipSuccess;
}

double spec_units(const UnitSpec& u, const Ctl& c) {
    if (u.field == U_CONST) return u.units;
    if (u.field == U_PEND) return c.n_pend;
    if (u.level >= LEVEL_RECS || u.level >= c.stats.levels) return 0.0;
    const LevelRec& r = c.lv[u.level];
    if (u.field >= U_BASE0 && u.field < U_BASE0 + NCLS) return r.base_strings[u.field - U_BASE0];
    if (u.field == U_DIST) return r.n_dist;
    if (u.field == U_DIST_STRINGS) return r.dist_strings;
    if (u.field == U_CNT) return r.n_cnt;
    return 0.0;
}

// Accumulates the durations of all recorded pairs (the sort has completed and
// host_ctl holds its control block).
void resolve_timings(ss_ctx* ctx) {
    Profiler& P = ctx->prof;
    for (size_t i = 0; i < P.used; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, P.ev[2 * i], P.ev[2 * i + 1]) == hipSuccess) {
            P.ms[P.kid[i]] += ms;
            P.unit_sum[P.kid[i]] += spec_units(P.spec[i], *ctx->host_ctl);
            P.launches[P.kid[i]] += 1;
        }
    }
    P.used = 0;
}

// Takes over the control block of the last sort (its copy in host_ctl is
// complete): statistics, level hint, device-side errors.
void absorb(ss_ctx* ctx) {
    const Ctl& c = *ctx->host_ctl;
    ss_stats st{};
    st.levels = c.stats.levels;
    st.dist_segments = c.stats.dist_segments;
    st.dist_tiles = c.stats.dist_tiles;
    st.max_depth = c.stats.max_depth;
    for (int q = 0; q < NCLS; ++q) {
        st.base_segments += c.stats.base_segments[q];
        st.base_segments_by_class[q] = c.stats.base_segments[q];
        st.base_strings_by_class[q] = c.stats.base_strings[q];
    }
    st.pending_lcps = c.n_pend;
    st.base_rounds = base_rounds_of(c);
    st.key_chars = c.alpha.bpc ? c.alpha.cpw : W;
    if (c.alpha.bpc)
        for (int q = 0; q < 4; ++q) st.alphabet_size += (uint32_t)__builtin_popcountll(c.alpha.seen[q]);
    st.alphabet_retries = ctx->alphabet_retries;
    ctx->stats = st;
    if (c.stats.levels) ctx->level_hint = c.stats.levels;
    // the device keeps the errors of every sort since the last clear, so an
    // error of a sort whose control block was never taken over here (a later
    // sort was enqueued first) is still seen
    if (c.err_sticky && ctx->sticky == SS_OK) ctx->sticky = device_error_status(c.err_sticky);
    ctx->pending = false;
}

// Waits for the last sort of the context and takes over its control block.
ss_status finish_pending(ss_ctx* ctx) {
    if (!ctx->pending) return SS_OK;
    SS_TRY(hipEventSynchronize(ctx->done));
    if (ctx->prof.used) resolve_timings(ctx);
    absorb(ctx);
    return SS_OK;
}

// Reads the control block into the pinned host copy (synchronous; the
// host-driven level loop and the serving worker).
ss_status read_ctl(ss_ctx* ctx, const Work& w, hipStream_t s) {
    SS_TRY(hipMemcpyAsync(ctx->host_ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    SS_TRY(hipStreamSynchronize(s));
    return SS_OK;
}

ss_status ensure_streams(ss_ctx* ctx) {
    if (ctx->done) return SS_OK;
    for (int i = 0; i < 2; ++i) {
        SS_TRY(hipStreamCreateWithFlags(&ctx->side[i], hipStreamNonBlocking));
        SS_TRY(hipEventCreateWithFlags(&ctx->join[i], hipEventDisableTiming));
    }
    SS_TRY(hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
    SS_TRY(hipEventCreateWithFlags(&ctx->done, hipEventDisableTiming));
    return SS_OK;
}

ss_status ensure_caps(ss_ctx* ctx) {
    if (ctx->kc_ok) return SS_OK;
    SS_TRY(kernel_caps(ctx->device, &ctx->kc));
    ctx->kc_ok = true;
    return SS_OK;
}

// What a sort's launches run with: the kernels' resident capacities, the
// profiler (null: no timing) and the library streams for the steps that
// overlap others (null: everything on the sort's stream).
struct Engine {
    const KernelCaps* kc = nullptr;
    Profiler* prof = nullptr;
    hipStream_t side[2] = {nullptr, nullptr};
    hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};
};
Engine engine_of(ss_ctx* ctx) {
    Engine e;
    e.kc = &ctx->kc;
    e.prof = &ctx->prof;
    for (int i = 0; i < 2; ++i) {
        e.side[i] = ctx->side[i];
        e.join[i] = ctx->join[i];
    }
    e.fork = ctx->fork;
    return e;
}

// What the host knows about a level when it enqueues it: exact counts (the
// host-driven loop and serving) or nothing (pool capacities bound the work).
struct LevelPlan {
    bool exact = false;
    Counts c{};
    bool maybe_dist = true;
    uint32_t maybe_base = (1u << NCLS) - 1;  // classes that may have segments
    bool sampled = false;                    // sampling already enqueued (first level)
};

uint32_t clamp_grid(uint32_t resident, uint32_t need) { return std::max<uint32_t>(1, std::min(resident, need)); }
// Rounds of resident work groups launched for the item kernels: the items
// of the launched groups are static (the hardware starts a group when
// another leaves), the rest is taken from the feed.
constexpr uint32_t ROUNDS_BASE = 16, ROUNDS_TILES = 8;
// The scatter takes one half tile per work group (see k_scatter); its grid
// covers up to this many rounds of resident groups.
constexpr uint32_t ROUNDS_SCATTER = 16;

// Enqueues recursion level `level` on slot `cur` (its counts read on the
// device): level start, then the distribution steps (sample, classify, scan,
// scatter, children) on `s` and the base cases on the two library streams
// (classes 0 and 3 on one, 1 and 2 on the other), forked from `s` after the
// level start and joined into `s` at the end.  Without library streams
// everything runs on `s`.  Kernels that the plan shows to have no work are
// left out.
ss_status enqueue_level(const Engine& e, const Work& w, const Params& p, int cur, uint32_t level, const LevelPlan& L,
                        hipStream_t s) {
    const KernelCaps& kc = *e.kc;
    const Caps& cap = w.caps;
    uint32_t bases = 0;
    for (int q = 0; q < NCLS; ++q)
        if ((L.maybe_base >> q) & 1u && (!L.exact || L.c.n_base[q])) bases |= 1u << q;
    const bool dist = L.maybe_dist && (!L.exact || L.c.n_dist);
    SS_TRY(timed(e.prof, s, K_LEVEL_BEGIN, units_const(1.0), [&] { return launch_level_begin(w, cur, level, s); }));
    const uint32_t on[2] = {bases & (1u | 1u << 3), bases & (1u << 1 | 1u << 2)};
    const bool sides = e.side[0] && e.side[1];
    bool forked[2] = {false, false};
    if (bases && sides) SS_TRY(hipEventRecord(e.fork, s));
    // the distribution steps are enqueued first, so the host's calls for the
    // library streams do not hold them back
    if (dist) {
        const Counts& c = L.c;
        const uint32_t n_dist = L.exact ? c.n_dist : cap.dist, n_tiles = L.exact ? c.n_tiles : cap.tiles;
        const uint32_t n_cnt = L.exact ? c.n_cnt : cap.cnt;
        if (!L.sampled)
            SS_TRY(timed(e.prof, s, K_SAMPLE, units_level(U_DIST, level),
                         [&] { return launch_sample(w, p, cur, clamp_grid(kc.sample, n_dist), false, s); }));
        SS_TRY(timed(e.prof, s, K_CLASSIFY, units_level(U_DIST_STRINGS, level), [&] {
            return launch_classify(w, p, cur, clamp_grid(ROUNDS_TILES * kc.classify, grid_classify(n_tiles)), s);
        }));
        SS_TRY(timed(e.prof, s, K_SCAN, units_level(U_CNT, level),
                     [&] { return launch_scan(w, cur, clamp_grid(kc.scan, grid_scan(n_cnt)), s); }));
        SS_TRY(timed(e.prof, s, K_SCATTER, units_level(U_DIST_STRINGS, level), [&] {
            const uint32_t need = grid_scatter(n_tiles), g = clamp_grid(ROUNDS_SCATTER * kc.scatter, need);
            return launch_scatter(w, p, cur, g, need > g ? kc.scatter : 0u, s);
        }));
        SS_TRY(timed(e.prof, s, K_CHILDREN, units_level(U_DIST, level), [&] {
            return launch_children(w, p, cur, clamp_grid(kc.children, grid_children(n_dist)), s);
        }));
    }
    for (int k = 0; k < 2; ++k) {
        if (!on[k]) continue;
        // without distribution steps, `s` takes one share
        hipStream_t bs = sides && (dist || k == 1) ? e.side[k] : s;
        if (bs != s) {
            SS_TRY(hipStreamWaitEvent(bs, e.fork, 0));
            forked[k] = true;
        }
        for (int q = 0; q < NCLS; ++q) {
            if (!((on[k] >> q) & 1u)) continue;
            const uint32_t need = grid_base(q, L.exact ? L.c.n_base[q] : cap.base[q]);
            SS_TRY(timed(e.prof, bs, K_BASE_W1 + q, units_level(U_BASE0 + q, level),
                         [&] { return launch_base(w, p, cur, q, clamp_grid(ROUNDS_BASE * kc.base[q], need), bs); }));
        }
    }
    for (int k = 0; k < 2; ++k) {
        if (!forked[k]) continue;
        SS_TRY(hipEventRecord(e.join[k], e.side[k]));
        SS_TRY(hipStreamWaitEvent(s, e.join[k], 0));
    }
    return SS_OK;
}

// Start of every sort: reset, roots and key gather.  For 2^21 strings or
// more (and with library streams) the roots are emitted before the gather
// and the first level's sampling reads its keys from the strings on a
// library stream while the gather fills the buffer (joined before the first
// classification); its grid covers every root that can be a distribution
// segment.  Returns whether the first level's sampling was enqueued.
ss_status enqueue_start(const Engine& e, const Work& w, const Params& p, const uint32_t* set_begin, uint32_t nroots,
                        hipStream_t s, bool* sampled, bool started) {
    const uint32_t n = p.n;
    if (!started) SS_TRY(launch_reset(w, s));  // else: reset and alphabet already enqueued (decide_alphabet)
    *sampled = n >= FORK_MIN && e.side[0];
    if (*sampled) {
        SS_TRY(timed(e.prof, s, K_ROOTS, units_const(nroots), [&] { return launch_roots(w, p, set_begin, nroots, s); }));
        const uint32_t root_grid = clamp_grid(e.kc->sample, std::min<uint32_t>(nroots, n / (p.base_max + 1) + 1));
        SS_TRY(hipEventRecord(e.fork, s));
        SS_TRY(timed(e.prof, s, K_INIT, units_const(n), [&] { return launch_init(w, p, s); }));
        SS_TRY(hipStreamWaitEvent(e.side[0], e.fork, 0));
        SS_TRY(timed(e.prof, e.side[0], K_SAMPLE, units_level(U_DIST, 0),
                     [&] { return launch_sample(w, p, 0, root_grid, true, e.side[0]); }));
        SS_TRY(hipEventRecord(e.join[0], e.side[0]));
        SS_TRY(hipStreamWaitEvent(s, e.join[0], 0));
    } else {
        SS_TRY(timed(e.prof, s, K_INIT, units_const(n), [&] { return launch_init(w, p, s); }));
        SS_TRY(timed(e.prof, s, K_ROOTS, units_const(nroots), [&] { return launch_roots(w, p, set_begin, nroots, s); }));
    }
    return SS_OK;
}

// The device-driven sort: start, `levels` levels enqueued without knowing
// their counts, then one persistent launch that runs whatever is left and
// the boundary LCPs.  The last enqueued level gets its base cases only: the
// last level of a sort has no distribution segments, so when `levels` is
// what the sort needs, that level is complete and the persistent launch
// finds nothing to do; otherwise it continues with that level's
// distribution segments.  No host synchronisation; capturable.
ss_status enqueue_sort_levels(const Engine& e, const Work& w, const Params& p, const uint32_t* set_begin,
                              uint32_t nroots, uint32_t levels, hipStream_t s, bool started = false) {
    bool sampled = false;
    ss_status st = enqueue_start(e, w, p, set_begin, nroots, s, &sampled, started);
    if (st != SS_OK) return st;
    bool one_root_base = false;
    if (!set_begin) {  // one root: a distribution segment (two levels at least), a base case or nothing
        if (p.n > p.base_max) levels = std::max<uint32_t>(levels, 2);
        else levels = 1, one_root_base = true;
    }
    int cur = 0;
    for (uint32_t level = 0; level < levels; ++level) {
        LevelPlan L;
        L.sampled = level == 0 && sampled;
        L.maybe_dist = level + 1 < levels;
        if (level == 0 && !set_begin) {
            L.maybe_base = one_root_base && p.n >= 2 ? 1u << size_class(p.n) : 0u;
            L.maybe_dist = L.maybe_dist && !one_root_base;
        }
        if ((st = enqueue_level(e, w, p, cur, level, L, s)) != SS_OK) return st;
        if (level + 1 < levels) cur ^= 1;
    }
    SS_TRY(timed(e.prof, s, K_PERSIST, units_const(0.0), [&] {
        return launch_persistent(w, p, set_begin, nroots, e.kc->persist, false, levels - 1, cur, true, s);
    }));
    return SS_OK;
}

// The host-driven sort: the host reads each level's counts and enqueues the
// level with exact grids (synchronises once per level).
ss_status run_sort_host_levels(ss_ctx* ctx, const Work& w, const Params& p, const uint32_t* set_begin,
                               uint32_t nroots, hipStream_t s, bool started) {
    const Engine e = engine_of(ctx);
    bool sampled = false;
    ss_status st = enqueue_start(e, w, p, set_begin, nroots, s, &sampled, started);
    if (st != SS_OK) return st;
    int cur = 0;
    for (uint32_t level = 0;; ++level) {
        if ((st = read_ctl(ctx, w, s)) != SS_OK) return st;
        if (ctx->host_ctl->err) break;
        LevelPlan L;
        L.exact = true;
        L.c = counts_of(ctx->host_ctl->cl[cur]);
        L.sampled = level == 0 && sampled;
        bool work = L.c.n_dist != 0;
        for (int q = 0; q < NCLS; ++q) work |= L.c.n_base[q] != 0;
        if (!work) break;
        if ((st = enqueue_level(e, w, p, cur, level, L, s)) != SS_OK) return st;
        if (L.c.n_dist == 0) break;
        cur ^= 1;
        if (level + 1 >= MAX_LEVELS) return SS_INTERNAL;
    }
    SS_TRY(timed(&ctx->prof, s, K_LCP_FILL, units_level(U_PEND, 0), [&] { return launch_lcp_fill(w, p, s); }));
    return SS_OK;
}

// Levels to enqueue as separate launches: what the context's last completed
// sort needed (the persistent tail covers any more).
uint32_t level_budget(ss_ctx* ctx) {
    if (ctx->pending && hipEventQuery(ctx->done) == hipSuccess) absorb(ctx);
    const uint32_t h = ctx->level_hint ? ctx->level_hint : DEFAULT_LEVELS;
    return std::min<uint32_t>(std::max<uint32_t>(h, 1), MAX_LEVEL_LAUNCHES);
}

// One sort on the context's workspace, enqueued on `s`.  The previous sort
// of the context (on any stream) is waited for on the device; the device-
// driven form returns without waiting for the sort.
ss_status run_sort(ss_ctx* ctx, const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                   const uint32_t* set_begin, uint32_t num_sets, uint32_t* perm, uint32_t* lcp,
                   hipStream_t s) {
    if (n == 0) return SS_OK;
    int cur_dev = -1;
    SS_TRY(hipGetDevice(&cur_dev));
    if (cur_dev != ctx->device) SS_TRY(hipSetDevice(ctx->device));
    ss_status st = ensure_streams(ctx);
    if (st == SS_OK) st = ensure_caps(ctx);
    if (st != SS_OK) return st;
    const uint32_t levels = level_budget(ctx);
    {
        const bool fits = ctx->ws.mem && n <= ctx->ws.n && ctx->cfg.bucket_target >= ctx->ws.bucket_target &&
                          ctx->cfg.base_max >= ctx->ws.base_max;
        if (!fits && ctx->done_recorded) SS_TRY(hipEventSynchronize(ctx->done));  // the old workspace is free
        if ((st = ws_ensure(ctx->ws, n, ctx->cfg, ctx->scratch_limit)) != SS_OK) return st;
    }
    // the workspace is free once the context's previous sort (on any stream)
    // is done; its control block copy may still land in host_ctl before this
    // sort's, which only drops statistics of an intermediate sort
    if (ctx->done_recorded) SS_TRY(hipStreamWaitEvent(s, ctx->done, 0));
    Work w = ctx->ws.work;
    if (set_begin) w.set_base = set_begin;  // perm entries are set-local
    Params p{chars,
             offsets,
             n,
             perm,
             lcp,
             ctx->cfg.max_log_splitters,
             ctx->cfg.bucket_target,
             ctx->cfg.base_max,
             ctx->cfg.alphabet};
    const uint32_t nroots = set_begin ? num_sets : 1;
    ctx->alphabet_retries = 0;
    if (ctx->cfg.mode == SS_MODE_PERSISTENT) {  // the persistent kernel reads the key format on the device
        SS_TRY(launch_reset(w, s));
        SS_TRY(timed(&ctx->prof, s, K_ALPHABET, units_const(n),
                     [&] { return launch_alphabet(w, p, ctx->kc.classify, true, s); }));
        SS_TRY(timed(&ctx->prof, s, K_PERSIST, units_const(n), [&] {
            return launch_persistent(w, p, set_begin, nroots, ctx->kc.persist, true, 0, 0, false, s);
        }));
    } else {
        // the level kernels come in a byte-key and a compressed-key form; the
        // host picks one, so a sort that may compress its keys first waits
        // for the alphabet probe.  The first attempt trusts the probe's byte
        // set (no pass over every character); a compressed gather that meets
        // another byte flags it, and the sort is run again with the set
        // checked in full (the results depend only on gathered bytes, so an
        // unflagged attempt equals the byte-key sort).
        for (bool checked = false;; checked = true) {
            bool started = false;
            if (p.alphabet != SS_ALPHABET_BYTES) {
                SS_TRY(launch_reset(w, s));
                SS_TRY(timed(&ctx->prof, s, K_ALPHABET, units_const(n),
                             [&] { return launch_alphabet(w, p, ctx->kc.classify, checked, s); }));
                decltype(Ctl::alpha) a;
                SS_TRY(hipMemcpyAsync(&a, &w.ctl->alpha, sizeof(a), hipMemcpyDeviceToHost, s));
                SS_TRY(hipStreamSynchronize(s));
                uint64_t m[4] = {0, 0, 0, 0};
                if (a.cand && !a.over)
                    for (int q = 0; q < 4; ++q) m[q] = a.seen[q];
                p.ac = key_fmt_of(m).bpc != 0 ? 1u : 0u;
                started = true;
            }
            if (ctx->cfg.mode == SS_MODE_HOST_LEVELS) {
                if ((st = run_sort_host_levels(ctx, w, p, set_begin, nroots, s, started)) != SS_OK) return st;
            } else if ((st = enqueue_sort_levels(engine_of(ctx), w, p, set_begin, nroots, levels, s, started)) !=
                       SS_OK) {
                return st;
            }
            if (!p.ac || checked) break;
            uint32_t miss = 0;
            SS_TRY(hipMemcpyAsync(&miss, &w.ctl->alpha.miss, sizeof(miss), hipMemcpyDeviceToHost, s));
            SS_TRY(hipStreamSynchronize(s));
            if (!miss) break;
            ++ctx->alphabet_retries;
        }
    }
    SS_TRY(hipMemcpyAsync(ctx->host_ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    SS_TRY(hipEventRecord(ctx->done, s));
    ctx->done_recorded = true;
    ctx->pending = true;
    if (ctx->prof.on) return finish_pending(ctx);  // timings need the sort to have run
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

// ---- LCP-aware merge of sorted runs ----

// Grows the merge workspace to at least `dev_bytes` device / `host_bytes`
// pinned host bytes.
ss_status ensure_merge_ws(ss_ctx* ctx, size_t dev_bytes, size_t host_bytes) {
    if (ctx->scratch_limit && dev_bytes > ctx->scratch_limit) return SS_OUT_OF_MEMORY;
    if (dev_bytes > ctx->mws_bytes) {
        if (ctx->mws) (void)hipFree(ctx->mws);
        ctx->mws = nullptr;
        ctx->mws_bytes = 0;
        if (hipMalloc(&ctx->mws, dev_bytes) != hipSuccess) {
            (void)hipGetLastError();
            ctx->mws = nullptr;
            return SS_OUT_OF_MEMORY;
        }
        ctx->mws_bytes = dev_bytes;
    }
    if (host_bytes > ctx->mhost_bytes) {
        if (ctx->mhost) (void)hipHostFree(ctx->mhost);
        ctx->mhost = nullptr;
        ctx->mhost_bytes = 0;
        if (hipHostMalloc(&ctx->mhost, host_bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            ctx->mhost = nullptr;
            return SS_OUT_OF_MEMORY;
        }
        ctx->mhost_bytes = host_bytes;
    }
    return SS_OK;
}

ss_status merge_error_status(uint32_t err) {
    if (err & MERR_INDEX) return SS_INVALID_ARG;
    if (err & MERR_OFFSETS) return SS_LIMIT;
    return SS_INTERNAL;
}

// Pairwise rounds: runs 2t and 2t+1 of a round become run t of the next
// (an odd last run is carried by a task with an empty B).  Empty runs are
// dropped first; a single run is one task that copies it.
ss_status run_merge(ss_ctx* ctx, const uint8_t* chars, const uint64_t* offsets, uint32_t n_strings,
                    const uint32_t* perm, const uint32_t* lcp, const uint64_t* run_begin, uint32_t num_runs,
                    uint32_t* perm_out, uint32_t* lcp_out, hipStream_t s) {
    const uint64_t m = run_begin[num_runs];
    std::vector<uint32_t> size;
    for (uint32_t r = 0; r < num_runs; ++r)
        if (run_begin[r + 1] > run_begin[r]) size.push_back((uint32_t)(run_begin[r + 1] - run_begin[r]));
    std::vector<std::vector<MergeTask>> rounds;
    std::vector<uint32_t> tiles;  // per round
    do {
        std::vector<MergeTask> tasks;
        std::vector<uint32_t> next;
        uint32_t a = 0, c0 = 0;
        for (size_t r = 0; r < size.size(); r += 2) {
            const uint32_t na = size[r], nb = r + 1 < size.size() ? size[r + 1] : 0u;
            tasks.push_back(MergeTask{a, na, nb, c0});
            c0 += (uint32_t)(((uint64_t)na + nb + MERGE_TILE - 1) / MERGE_TILE);
            a += na + nb;
            next.push_back(na + nb);
        }
        rounds.push_back(std::move(tasks));
        tiles.push_back(c0);
        size.swap(next);
    } while (size.size() > 1);
    const size_t R = rounds.size();

    size_t n_tasks = 0, max_tiles = 0;
    for (size_t r = 0; r < R; ++r) n_tasks += rounds[r].size(), max_tiles = std::max<size_t>(max_tiles, tiles[r]);
    const size_t tmp_bufs = R >= 3 ? 2 : R - 1;  // ping-pong (perm, lcp) pairs between rounds
    const size_t arr = align_up(m * sizeof(uint32_t));
    const size_t off_split = tmp_bufs * 2 * arr;
    const size_t off_cross = off_split + align_up(max_tiles * sizeof(uint32_t));
    const size_t off_tasks = off_cross + align_up(max_tiles * sizeof(uint32_t));
    const size_t off_err = off_tasks + align_up(n_tasks * sizeof(MergeTask));
    const size_t dev_bytes = off_err + 256;
    const size_t host_tasks = align_up(n_tasks * sizeof(MergeTask));
    ss_status st = ensure_merge_ws(ctx, dev_bytes, host_tasks + 256);
    if (st != SS_OK) return st;

    char* dws = (char*)ctx->mws;
    MergeTask* htask = (MergeTask*)ctx->mhost;
    uint32_t* herr = (uint32_t*)((char*)ctx->mhost + host_tasks);
    size_t t0 = 0;
    for (size_t r = 0; r < R; ++r) {
        std::copy(rounds[r].begin(), rounds[r].end(), htask + t0);
        t0 += rounds[r].size();
    }
    MergeTask* dtask = (MergeTask*)(dws + off_tasks);
    uint32_t* derr = (uint32_t*)(dws + off_err);
    SS_TRY(hipMemcpyAsync(dtask, htask, n_tasks * sizeof(MergeTask), hipMemcpyHostToDevice, s));
    SS_TRY(hipMemsetAsync(derr, 0, sizeof(uint32_t), s));

    uint32_t* tmp_perm[2] = {(uint32_t*)dws, (uint32_t*)(dws + 2 * arr)};
    uint32_t* tmp_lcp[2] = {(uint32_t*)(dws + arr), (uint32_t*)(dws + 3 * arr)};
    t0 = 0;
    for (size_t r = 0; r < R; ++r) {
        MergeArgs a{};
        a.chars = chars;
        a.offsets = offsets;
        a.n_strings = n_strings;
        a.src_perm = r == 0 ? perm : tmp_perm[(r - 1) & 1];
        a.src_lcp = r == 0 ? lcp : tmp_lcp[(r - 1) & 1];
        a.dst_perm = r + 1 == R ? perm_out : tmp_perm[r & 1];
        a.dst_lcp = r + 1 == R ? lcp_out : tmp_lcp[r & 1];
        a.tasks = dtask + t0;
        a.n_tasks = (uint32_t)rounds[r].size();
        a.n_tiles = tiles[r];
        a.split = (uint32_t*)(dws + off_split);
        a.cross = (uint32_t*)(dws + off_cross);
        a.err = derr;
        SS_TRY(timed(&ctx->prof, s, K_MERGE_SPLIT, units_const(a.n_tiles), [&] { return launch_merge_split(a, s); }));
        SS_TRY(timed(&ctx->prof, s, K_MERGE, units_const((double)m), [&] { return launch_merge_tiles(a, s); }));
        t0 += rounds[r].size();
    }
    SS_TRY(hipMemcpyAsync(herr, derr, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SS_TRY(hipStreamSynchronize(s));
    if (ctx->prof.used) resolve_timings(ctx);
    if (*herr) return merge_error_status(*herr);
    return SS_OK;
}

// ---- suffix array by prefix doubling ----

ss_status run_suffix_array(ss_ctx* ctx, const uint8_t* text, uint32_t n, uint32_t* sa, uint32_t* isa_out,
                           uint32_t* rounds_out, hipStream_t s) {
    const size_t a4 = align_up((size_t)n * 4);
    const size_t b_chars = align_up((size_t)n * std::max<uint32_t>(std::max(SA_W0, SA_PACKED_LEN), 8));
    static_assert(SA_PACKED_LEN % 8 == 0, "packed windows are whole words");
    const size_t b_offs = align_up(((size_t)n + 1) * 8);
    const size_t b_part = align_up(((size_t)sa_tiles(n) + 1) * 4);
    // chars, offsets, lcp, perm, idx, two position lists, names, two counter arrays
    const size_t bytes = b_chars + b_offs + 5 * a4 + (isa_out ? 0 : a4) + 2 * b_part + 512;
    if (ctx->scratch_limit && bytes > ctx->scratch_limit) return SS_OUT_OF_MEMORY;
    if (bytes > ctx->saws_bytes) {
        if (ctx->saws) (void)hipFree(ctx->saws);
        ctx->saws = nullptr;
        ctx->saws_bytes = 0;
        if (hipMalloc(&ctx->saws, bytes) != hipSuccess) {
            (void)hipGetLastError();
            ctx->saws = nullptr;
            return SS_OUT_OF_MEMORY;
        }
        ctx->saws_bytes = bytes;
    }
    if (!ctx->sa_host) {
        // [0]: group count; [8..16): byte mask; bytes 64..320: rank table
        if (hipHostMalloc((void**)&ctx->sa_host, 512, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            ctx->sa_host = nullptr;
            return SS_OUT_OF_MEMORY;
        }
    }
    char* p = (char*)ctx->saws;
    auto take = [&](size_t b) { char* q = p; p += b; return q; };
    uint8_t* chars = (uint8_t*)take(b_chars);
    uint64_t* offsets = (uint64_t*)take(b_offs);
    uint32_t* lcp = (uint32_t*)take(a4);
    uint32_t* perm = (uint32_t*)take(a4);
    uint32_t* idx = (uint32_t*)take(a4);
    uint32_t* pos[2] = {(uint32_t*)take(a4), (uint32_t*)take(a4)};
    uint32_t* names = isa_out ? isa_out : (uint32_t*)take(a4);
    uint32_t* part_max = (uint32_t*)take(b_part);
    uint32_t* part_cnt = (uint32_t*)take(b_part);
    uint32_t* mask = (uint32_t*)take(256);  // 8 words of byte presence
    uint8_t* rank = (uint8_t*)take(256);    // byte -> rank among the bytes present

    // the suffix windows and name pairs split into many small buckets; the
    // sorts run with a bucket target of at least 256 strings
    struct CfgGuard {
        ss_ctx* c;
        ss_config saved;
        ~CfgGuard() { c->cfg = saved; }
    } guard{ctx, ctx->cfg};
    ctx->cfg.bucket_target = std::max<uint32_t>(ctx->cfg.bucket_target, 256u);
    ctx->cfg.alphabet = SS_ALPHABET_BYTES;  // windows and name pairs are binary already
    // the rounds' sorts need different numbers of levels (the first sorts
    // every suffix, later ones the unfinished few), so a level count
    // carried over from the previous round would send deeper rounds to the
    // persistent tail; the host reads each level's counts instead (every
    // round synchronises anyway)
    ctx->cfg.mode = SS_MODE_HOST_LEVELS;

    SaArgs a{};
    a.n = n;
    a.sa = sa;
    a.names = names;
    a.part_max = part_max;
    a.part_cnt = part_cnt;
    // the text's alphabet: at most 16 distinct bytes are packed in round 0
    SS_TRY(hipMemsetAsync(mask, 0, 8 * sizeof(uint32_t), s));
    SS_TRY(launch_sa_alphabet(text, n, mask, s));
    uint32_t* hmask = ctx->sa_host + 8;
    uint8_t* hrank = (uint8_t*)ctx->sa_host + 64;
    SS_TRY(hipMemcpyAsync(hmask, mask, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SS_TRY(hipStreamSynchronize(s));
    uint32_t sigma = 0;
    for (uint32_t v = 0; v < 256; ++v) {
        hrank[v] = (uint8_t)sigma;
        if ((hmask[v >> 5] >> (v & 31)) & 1u) ++sigma;
    }
    uint32_t bits = 1;  // 1, 2 or 4 bits per character (ranks fit; 64 / bits whole characters per word)
    while ((1u << bits) < sigma) bits *= 2;
    const bool packed = bits <= 4;
    const uint32_t w0 = packed ? 128 / bits : SA_W0;  // characters resolved by round 0
    // round 0: every suffix by its first w0 characters, sorted into sa
    SS_TRY(timed(&ctx->prof, s, K_SA_STRINGS, units_const(n), [&] {
        if (!packed) return launch_sa_windows(text, n, chars, offsets, s);
        hipError_t e = hipMemcpyAsync(rank, hrank, 256, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
        // the packed blocks live in the LCP buffer until round 0's sort
        return launch_sa_windows_packed(text, n, rank, bits, (uint64_t*)lcp, chars, offsets, s);
    }));
    ss_status st = run_sort(ctx, chars, offsets, n, nullptr, 1, sa, lcp, s);
    if (st != SS_OK) return st;
    a.perm = sa;
    a.lcp = lcp;
    a.m = n;
    a.round0 = 1;
    a.round0_len = packed ? SA_PACKED_LEN : 0u;
    a.idx = nullptr;
    a.pos = nullptr;
    a.next_pos = pos[0];
    uint32_t rounds = 1, cur = 0;
    uint64_t h = w0;  // depth the names resolve
    for (;;) {
        SS_TRY(timed(&ctx->prof, s, K_SA_RENAME, units_const(a.m), [&] { return launch_sa_rename(a, s); }));
        SS_TRY(hipMemcpyAsync(ctx->sa_host, part_cnt + sa_tiles(a.m), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        SS_TRY(hipStreamSynchronize(s));
        // the round's sort has completed: its device-side errors
        if ((st = finish_pending(ctx)) != SS_OK) return st;
        if (ctx->host_ctl->err) return device_error_status(ctx->host_ctl->err);
        if (ctx->prof.used) resolve_timings(ctx);
        const uint32_t m = *ctx->sa_host;  // suffixes still sharing their group
        if (m == 0) break;
        if (h >= n || m > n) return SS_INTERNAL;  // suffixes differ within n characters
        // next round: the m unfinished suffixes by (name, name at +h)
        a.round0 = 0;
        a.m = m;
        a.pos = pos[cur];
        a.idx = idx;
        a.next_pos = pos[cur ^ 1];
        SS_TRY(timed(&ctx->prof, s, K_SA_STRINGS, units_const(m), [&] { return launch_sa_pairs(a, (uint32_t)h, chars, offsets, s); }));
        st = run_sort(ctx, chars, offsets, m, nullptr, 1, perm, lcp, s);
        if (st != SS_OK) return st;
        a.perm = perm;
        cur ^= 1;
        h *= 2;
        ++rounds;
    }
    if (rounds_out) *rounds_out = rounds;
    return SS_OK;
}

std::mutex g_mu;
std::map<int, std::unique_ptr<ss_ctx, void (*)(ss_ctx*)>>* g_ctx = nullptr;

// ---- sorting without allocation ----
//
// The workspace of ss_sort_noalloc is this array: one copy per device,
// allocated when the library's code object is loaded there and held until
// the process ends.  Host code never uses the array's name as an address:
// set-up takes each device's address with hipGetSymbolAddress (with that
// device current) and the kernels get that address.
constexpr uint32_t NOALLOC_MAX_N = SS_NOALLOC_MAX_STRINGS;
constexpr size_t NOALLOC_BYTES = (size_t)72 << 20;
constexpr uint32_t NOALLOC_LEVELS = 4;  // level launches before the persistent tail
static __device__ __align__(256) uint8_t scratch[NOALLOC_BYTES];

constexpr int NOALLOC_DEVICES = 64;
struct NoAllocDevice {
    bool ready = false;
    ss_status status = SS_OK;  // of the set-up
    Work work{};
    KernelCaps kc{};
};
std::mutex g_na_mu;
NoAllocDevice g_na[NOALLOC_DEVICES];

// Set-up on device `dev` (current): the array's address on this device, the
// workspace laid out in it for NOALLOC_MAX_N strings, the kernels' resident
// capacities.  Runs once per device.
const NoAllocDevice* noalloc_device(int dev) {
    if (dev < 0 || dev >= NOALLOC_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_na_mu);
    NoAllocDevice& d = g_na[dev];
    if (d.ready) return &d;
    d.ready = true;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        d.status = SS_HIP_ERROR;
        return &d;
    }
    const ss_config c{10, 64, 1024, SS_MODE_LEVELS};
    const Caps k = caps_for(NOALLOC_MAX_N, c);
    if (layout(NOALLOC_MAX_N, k, nullptr, nullptr) > NOALLOC_BYTES) {
        d.status = SS_INTERNAL;
        return &d;
    }
    layout(NOALLOC_MAX_N, k, (char*)ptr, &d.work);
    if (kernel_caps(dev, &d.kc) != hipSuccess) {
        (void)hipGetLastError();
        d.status = SS_HIP_ERROR;
    }
    return &d;
}

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
    if (ctx->done_recorded) (void)hipEventSynchronize(ctx->done);
    for (ss_graph* g : ctx->graphs) g->ctx = nullptr;  // graphs own their workspaces
    for (hipEvent_t e : ctx->prof.ev) (void)hipEventDestroy(e);
    ws_free(ctx->ws);
    if (ctx->host_ctl) (void)hipHostFree(ctx->host_ctl);
    if (ctx->mws) (void)hipFree(ctx->mws);
    if (ctx->mhost) (void)hipHostFree(ctx->mhost);
    if (ctx->saws) (void)hipFree(ctx->saws);
    if (ctx->sa_host) (void)hipHostFree(ctx->sa_host);
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    if (ctx->done) (void)hipEventDestroy(ctx->done);
    for (int i = 0; i < 2; ++i) {
        if (ctx->join[i]) (void)hipEventDestroy(ctx->join[i]);
        if (ctx->side[i]) (void)hipStreamDestroy(ctx->side[i]);
    }
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
    ctx->cfg = c;  // the next sort lays the workspace out again if its pools are too small
    return SS_OK;
}

ss_status ss_workspace_query(const ss_ctx* ctx, uint32_t n, size_t* bytes) {
    if (!bytes) return SS_INVALID_ARG;
    ss_config c = ctx ? ctx->cfg : ss_config{10, 64, 1024, SS_MODE_LEVELS, SS_ALPHABET_BYTES};
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

ss_status ss_sort_noalloc(const uint8_t* chars, const uint64_t* offsets, uint32_t n, uint32_t* perm_out,
                          uint32_t* lcp_out, uint32_t* err_out, void* stream) {
    if (n == 0) return SS_OK;
    if (n > NOALLOC_MAX_N) return SS_LIMIT;
    if (!offsets || !perm_out || !lcp_out || (void*)perm_out == (void*)lcp_out) return SS_INVALID_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SS_HIP_ERROR;
    const NoAllocDevice* d = noalloc_device(dev);
    if (!d) return SS_INVALID_ARG;
    if (d->status != SS_OK) return d->status;
    hipStream_t s = (hipStream_t)stream;
    Engine e;
    e.kc = &d->kc;  // no profiler, no library streams: every launch goes to `stream`
    const Params p{chars, offsets, n, perm_out, lcp_out, 10, 64, 1024, SS_ALPHABET_BYTES};
    ss_status st = enqueue_sort_levels(e, d->work, p, nullptr, 1, NOALLOC_LEVELS, s);
    if (st == SS_OK && err_out) st = hip_status(launch_report(d->work, err_out, s));
    return st;
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
    ss_status st = ensure_streams(ctx);
    if (st == SS_OK) st = ensure_caps(ctx);
    if (st == SS_OK) st = finish_pending(ctx);  // host_ctl is used by the sizing run below
    if (st != SS_OK) return st;
    std::unique_ptr<ss_graph> gr(new ss_graph());
    gr->ctx = ctx;
    if ((st = ws_ensure(gr->ws, n, ctx->cfg, ctx->scratch_limit)) != SS_OK) return st;
    Params p{chars, offsets, n, perm_out, lcp_out, ctx->cfg.max_log_splitters, ctx->cfg.bucket_target,
             ctx->cfg.base_max, ctx->cfg.alphabet};
    Work w = gr->ws.work;
    w.set_base = set_begin;
    hipStream_t cs = nullptr;
    SS_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    const bool prof = ctx->prof.on;
    ctx->prof.on = false;  // no event records inside the graph
    // sizing run: the batched sort once, level by level from the host, on
    // the graph's workspace; the graph enqueues as many level launches as it
    // needed (a persistent tail runs any further levels of later contents)
    st = run_sort_host_levels(ctx, w, p, set_begin, num_sets, cs, false);
    if (st == SS_OK) st = read_ctl(ctx, w, cs);
    if (st == SS_OK && ctx->host_ctl->err) st = device_error_status(ctx->host_ctl->err);
    hipGraph_t g = nullptr;
    if (st == SS_OK) {
        gr->levels = std::min<uint32_t>(std::max<uint32_t>(ctx->host_ctl->stats.levels, 1), MAX_LEVEL_LAUNCHES);
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            st = enqueue_sort_levels(engine_of(ctx), w, p, set_begin, num_sets, gr->levels, cs);
            hipError_t e2 = hipStreamEndCapture(cs, &g);
            if (st == SS_OK && e2 != hipSuccess) st = SS_HIP_ERROR;
        } else {
            st = SS_HIP_ERROR;
        }
    }
    ctx->prof.on = prof;
    (void)hipStreamDestroy(cs);
    if (st != SS_OK) {
        if (g) (void)hipGraphDestroy(g);
        ws_free(gr->ws);
        return st;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        ws_free(gr->ws);
        return SS_HIP_ERROR;
    }
    gr->graph = g;
    gr->exec = ex;
    ctx->graphs.push_back(gr.get());
    *graph_out = gr.release();
    return SS_OK;
}

ss_status ss_graph_launch(ss_graph* graph, void* stream) {
    if (!graph || !graph->exec) return SS_INVALID_ARG;
    return hipGraphLaunch(graph->exec, (hipStream_t)stream) == hipSuccess ? SS_OK : SS_HIP_ERROR;
}

void ss_graph_destroy(ss_graph* graph) {
    if (!graph) return;
    if (graph->ctx) {
        auto& v = graph->ctx->graphs;
        v.erase(std::remove(v.begin(), v.end(), graph), v.end());
    }
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    ws_free(graph->ws);
    delete graph;
}

uint32_t ss_graph_levels(const ss_graph* graph) { return graph ? graph->levels : 0u; }

ss_status ss_ctx_sync(ss_ctx* ctx, void* stream) {
    if (!ctx) return SS_INVALID_ARG;
    int cur_dev = -1;
    SS_TRY(hipGetDevice(&cur_dev));
    if (cur_dev != ctx->device) SS_TRY(hipSetDevice(ctx->device));
    SS_TRY(hipStreamSynchronize((hipStream_t)stream));
    ss_status st = finish_pending(ctx);
    if (st != SS_OK) return st;
    for (ss_graph* g : ctx->graphs) {
        uint32_t err = 0;
        SS_TRY(hipMemcpy(&err, &g->ws.work.ctl->err_sticky, sizeof(err), hipMemcpyDeviceToHost));
        if (err && ctx->sticky == SS_OK) ctx->sticky = device_error_status(err);
    }
    return ctx->sticky;
}

namespace {

// Autotuner state: the best configuration found per (device, workload
// signature).  The signature buckets n, the character count and the set
// count by powers of two, so workloads of about the same shape share an
// entry.
struct TuneKey {
    int device;
    uint32_t log_n, log_chars, log_sets;
    bool operator<(const TuneKey& o) const {
        return std::tie(device, log_n, log_chars, log_sets) < std::tie(o.device, o.log_n, o.log_chars, o.log_sets);
    }
};
struct TuneEntry {
    ss_config cfg;
    double ms;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;

uint32_t ilog2_u64(uint64_t x) { return x ? 63u - (uint32_t)__builtin_clzll(x) : 0u; }

// Median wall time of `reps` sorts under `c` on `s` (after one warm-up);
// negative on failure.
double time_config(ss_ctx* ctx, const ss_config& c, const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                   const uint32_t* set_begin, uint32_t num_sets, uint32_t* perm, uint32_t* lcp, hipStream_t s,
                   uint32_t reps, hipEvent_t e0, hipEvent_t e1) {
    if (ss_set_config(ctx, &c) != SS_OK) return -1.0;
    if (sort_checked(ctx, chars, offsets, n, set_begin, num_sets, perm, lcp, s) != SS_OK) return -1.0;
    if (ss_ctx_sync(ctx, s) != SS_OK) return -1.0;
    std::vector<double> t;
    for (uint32_t r = 0; r < reps; ++r) {
        if (hipEventRecord(e0, s) != hipSuccess) return -1.0;
        if (sort_checked(ctx, chars, offsets, n, set_begin, num_sets, perm, lcp, s) != SS_OK) return -1.0;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.0;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
        t.push_back(ms);
    }
    if (ss_ctx_sync(ctx, s) != SS_OK) return -1.0;
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

}  // namespace

ss_status ss_autotune(ss_ctx* ctx, const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                      const uint32_t* set_begin, uint32_t num_sets, uint32_t* perm_out, uint32_t* lcp_out,
                      void* stream, uint32_t reps, int use_cache, ss_config* best, double* best_ms) {
    if (!ctx || !offsets || !perm_out || !lcp_out || n == 0) return SS_INVALID_ARG;
    if (set_begin ? num_sets == 0 : num_sets != 1) return SS_INVALID_ARG;
    if (n > 0xFFFFFFFEu) return SS_LIMIT;
    reps = std::max<uint32_t>(1, std::min<uint32_t>(reps, 50));
    hipStream_t s = (hipStream_t)stream;
    int cur_dev = -1;
    SS_TRY(hipGetDevice(&cur_dev));
    if (cur_dev != ctx->device) SS_TRY(hipSetDevice(ctx->device));
    uint64_t total_chars = 0;
    SS_TRY(hipMemcpyAsync(&total_chars, offsets + n, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    SS_TRY(hipStreamSynchronize(s));
    const TuneKey key{ctx->device, ilog2_u64(n), ilog2_u64(total_chars), ilog2_u64(num_sets)};
    if (use_cache) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            ss_set_config(ctx, &it->second.cfg);
            if (best) *best = it->second.cfg;
            if (best_ms) *best_ms = it->second.ms;
            return sort_checked(ctx, chars, offsets, n, set_begin, num_sets, perm_out, lcp_out, stream);
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SS_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SS_HIP_ERROR;
    }
    const ss_config start = ctx->cfg;
    ss_config top = start;
    double top_ms = -1.0;
    auto consider = [&](const ss_config& c) {
        double ms = time_config(ctx, c, chars, offsets, n, set_begin, num_sets, perm_out, lcp_out, s, reps, e0, e1);
        if (ms < 0) {
            ss_clear_error(ctx);  // a failed candidate (e.g. workspace cap) is skipped
            return;
        }
        if (top_ms < 0 || ms < top_ms) {
            top_ms = ms;
            top = c;
        }
    };
    // stage 1: the level-by-level form over splitter count, bucket target
    // and base-case size; stage 2: the persistent form with the winner's
    // parameters
    for (uint32_t d : {8u, 9u, 10u})
        for (uint32_t bt : {32u, 64u, 128u})
            for (uint32_t bm : {512u, 1024u}) consider(ss_config{d, bt, bm, SS_MODE_LEVELS, start.alphabet});
    if (top_ms >= 0) {
        for (uint32_t m : {SS_MODE_HOST_LEVELS, SS_MODE_PERSISTENT}) {
            ss_config pc = top;
            pc.mode = m;
            consider(pc);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (top_ms < 0) {
        ss_set_config(ctx, &start);
        return SS_INTERNAL;
    }
    ss_set_config(ctx, &top);
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune[key] = TuneEntry{top, top_ms};
    }
    if (best) *best = top;
    if (best_ms) *best_ms = top_ms;
    // the outputs hold the result of the chosen configuration
    return sort_checked(ctx, chars, offsets, n, set_begin, num_sets, perm_out, lcp_out, stream);
}

void ss_autotune_clear_cache(void) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.clear();
}

ss_status ss_get_last_error(ss_ctx* ctx) {
    if (!ctx) return SS_INVALID_ARG;
    if (ctx->pending && hipEventQuery(ctx->done) == hipSuccess) {
        if (ctx->prof.used) resolve_timings(ctx);
        absorb(ctx);
    }
    return ctx->sticky;
}

void ss_clear_error(ss_ctx* ctx) {
    if (!ctx) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    if (ctx->done_recorded) (void)hipEventSynchronize(ctx->done);
    ctx->pending = false;
    const uint32_t zero = 0;
    if (ctx->ws.mem) (void)hipMemcpy(&ctx->ws.work.ctl->err_sticky, &zero, sizeof(zero), hipMemcpyHostToDevice);
    for (ss_graph* g : ctx->graphs)
        (void)hipMemcpy(&g->ws.work.ctl->err_sticky, &zero, sizeof(zero), hipMemcpyHostToDevice);
    ctx->sticky = SS_OK;
    (void)hipSetDevice(prev);
}

ss_status ss_get_stats(ss_ctx* ctx, ss_stats* st) {
    if (!ctx || !st) return SS_INVALID_ARG;
    ss_status r = finish_pending(ctx);
    if (r != SS_OK) return r;
    *st = ctx->stats;
    return SS_OK;
}

ss_status ss_set_profiling(ss_ctx* ctx, int enable) {
    if (!ctx) return SS_INVALID_ARG;
    ctx->prof.on = enable != 0;
    ctx->prof.mask = ~0u;
    return SS_OK;
}

ss_status ss_set_profiling_only(ss_ctx* ctx, const char* kernel) {
    if (!ctx || !kernel) return SS_INVALID_ARG;
    for (int i = 0; i < K_COUNT; ++i) {
        if (std::strcmp(kernel, KNAME[i]) == 0) {
            ctx->prof.on = true;
            ctx->prof.mask = 1u << i;
            return SS_OK;
        }
    }
    return SS_INVALID_ARG;
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
    (void)finish_pending(ctx);
    Profiler& P = ctx->prof;
    P.used = 0;
    for (int i = 0; i < K_COUNT; ++i) P.ms[i] = P.unit_sum[i] = 0, P.launches[i] = 0;
}

ss_status ss_merge_runs(ss_ctx* ctx, const uint8_t* chars, const uint64_t* offsets, uint32_t n_strings,
                        const uint32_t* perm, const uint32_t* lcp, const uint64_t* run_begin, uint32_t num_runs,
                        uint32_t* perm_out, uint32_t* lcp_out, void* stream) {
    if (!ctx || !run_begin || num_runs == 0) return SS_INVALID_ARG;
    if (run_begin[0] != 0) return SS_INVALID_ARG;
    for (uint32_t r = 0; r < num_runs; ++r)
        if (run_begin[r + 1] < run_begin[r]) return SS_INVALID_ARG;
    const uint64_t m = run_begin[num_runs];
    if (m == 0) return SS_OK;
    if (m > 0xFFFFFFFEull) return SS_LIMIT;
    if (!offsets || !perm || !lcp || !perm_out || !lcp_out || n_strings == 0) return SS_INVALID_ARG;
    if ((const void*)perm_out == (const void*)lcp_out || (const void*)perm_out == (const void*)perm ||
        (const void*)perm_out == (const void*)lcp || (const void*)lcp_out == (const void*)perm ||
        (const void*)lcp_out == (const void*)lcp)
        return SS_INVALID_ARG;
    int cur_dev = -1;
    SS_TRY(hipGetDevice(&cur_dev));
    if (cur_dev != ctx->device) SS_TRY(hipSetDevice(ctx->device));
    ss_status st = run_merge(ctx, chars, offsets, n_strings, perm, lcp, run_begin, num_runs, perm_out, lcp_out,
                             (hipStream_t)stream);
    if (st != SS_OK && st != SS_INVALID_ARG) ctx->sticky = st;
    return st;
}

ss_status ss_suffix_array(ss_ctx* ctx, const uint8_t* text, uint32_t n, uint32_t* sa_out, uint32_t* isa_out,
                          uint32_t* rounds_out, void* stream) {
    if (rounds_out) *rounds_out = 0;
    if (!ctx) return SS_INVALID_ARG;
    if (n == 0) return SS_OK;
    if (n > 0xFFFFFFFEu) return SS_LIMIT;
    if (!text || !sa_out || (void*)sa_out == (void*)isa_out) return SS_INVALID_ARG;
    int cur_dev = -1;
    SS_TRY(hipGetDevice(&cur_dev));
    if (cur_dev != ctx->device) SS_TRY(hipSetDevice(ctx->device));
    ss_status st = run_suffix_array(ctx, text, n, sa_out, isa_out, rounds_out, (hipStream_t)stream);
    if (st != SS_OK && st != SS_INVALID_ARG) ctx->sticky = st;
    return st;
}

ss_status ss_hbm_copy(void* dst, const void* src, size_t bytes, void* stream) {
    if (!dst || !src || (bytes & 15) || (((uintptr_t)dst | (uintptr_t)src) & 15)) return SS_INVALID_ARG;
    SS_TRY(launch_copy(dst, src, bytes / 16, (hipStream_t)stream));
    return SS_OK;
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

uint64_t ss_host_gather_key(const uint8_t* chars, uint64_t off, uint32_t h, uint32_t len) {
    return gather_key_with(chars, off, h, len, [](const uint64_t* q) {
        uint64_t w;
        std::memcpy(&w, q, sizeof(w));
        return w;
    });
}

uint32_t ss_host_lcp_stream(const uint8_t* chars, uint64_t oa, uint32_t la, uint64_t ob, uint32_t lb, uint32_t from,
                            uint32_t cap, uint32_t ahead) {
    auto load = [](const uint64_t* q) {
        uint64_t w;
        std::memcpy(&w, q, sizeof(w));
        return w;
    };
    if (ahead <= 1) return lcp_stream_with<1>(chars, oa, la, ob, lb, from, cap, load);
    if (ahead <= 2) return lcp_stream_with<2>(chars, oa, la, ob, lb, from, cap, load);
    return lcp_stream_with<4>(chars, oa, la, ob, lb, from, cap, load);
}

uint64_t ss_host_gather_packed(const uint8_t* chars, uint64_t off, uint32_t h, uint32_t len, const uint64_t* byte_set,
                               uint32_t* chars_per_key, int* miss) {
    uint64_t m[4] = {0, 0, 0, 0};
    if (byte_set)
        for (int i = 0; i < 4; ++i) m[i] = byte_set[i];
    const KeyFmt f = key_fmt_of(m);
    if (chars_per_key) *chars_per_key = f.bpc ? f.cpw : W;
    bool mi = false;
    const uint64_t k = f.bpc ? gather_packed_with(chars, off, h, len, f,
                                                  [](const uint64_t* q) {
                                                      uint64_t w;
                                                      std::memcpy(&w, q, sizeof(w));
                                                      return w;
                                                  },
                                                  &mi)
                             : ss_host_gather_key(chars, off, h, len);
    if (miss) *miss = mi ? 1 : 0;
    return k;
}

uint32_t ss_host_key_lcp(const uint64_t* byte_set, uint64_t a, uint32_t len_a, uint64_t b, uint32_t len_b, uint32_t h) {
    uint64_t m[4] = {0, 0, 0, 0};
    if (byte_set)
        for (int i = 0; i < 4; ++i) m[i] = byte_set[i];
    const KeyFmt f = key_fmt_of(m);
    return kf_lcp_word(f, a, kf_r(f, len_a, h), b, kf_r(f, len_b, h));
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

// ===========================================================================
// serving
// ===========================================================================

namespace {

// First-fit allocator of ranges of [0, cap).
class RangeAlloc {
  public:
    void init(uint64_t cap) {
        free_.clear();
        if (cap) free_[0] = cap;
    }
    bool alloc(uint64_t size, uint64_t* out) {
        if (size == 0) { *out = 0; return true; }
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= size) {
                *out = it->first;
                const uint64_t b = it->first + size, rest = it->second - size;
                free_.erase(it);
                if (rest) free_[b] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t begin, uint64_t size) {
        if (size == 0) return;
        auto next = free_.lower_bound(begin);
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == begin) {
                begin = prev->first;
                size += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && begin + size == next->first) {
            size += next->second;
            free_.erase(next);
        }
        free_[begin] = size;
    }

  private:
    std::map<uint64_t, uint64_t> free_;
};

enum ReqState { RQ_QUEUED, RQ_RUNNING, RQ_DONE };

struct Req {
    uint64_t ticket = 0;
    ss_request r{};
    uint64_t nchars = 0;
    int state = RQ_QUEUED;
    ss_status status = SS_OK;
    uint32_t rid = 0;
    uint64_t pos = 0, cbase = 0;
    std::chrono::steady_clock::time_point t_submit, t_done;
};

using Clock = std::chrono::steady_clock;

}  // namespace

struct ss_server {
    ss_ctx* ctx = nullptr;
    int device = 0;
    uint32_t max_inflight = 0;
    uint32_t cap_n = 0;        // index slots
    uint64_t cap_c = 0;        // characters
    size_t slot_bytes = 0;     // arena bytes per index slot
    void* mem = nullptr;
    Work w{};
    Params p{};
    uint32_t* d_set_base = nullptr;
    uint32_t* d_remaining = nullptr;
    uint8_t* d_done = nullptr;
    uint32_t* h_remaining = nullptr;  // pinned
    uint32_t* h_slot = nullptr;       // pinned staging: set_base, remaining per rid
    uint8_t* h_done = nullptr;        // pinned
    RangeAlloc idx_alloc, chr_alloc;
    std::vector<uint32_t> free_rids;
    std::vector<Req*> running;        // by rid
    std::deque<Req*> queue;
    std::unordered_map<uint64_t, Req*> reqs;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    uint64_t next_ticket = 1;
    hipStream_t stream = nullptr;
    int cur = 0;
    uint32_t level = 0;  // levels run (numbers the level records)
    // statistics
    ss_server_stats st{};
    std::vector<double> lat_us;
    double busy_s = 0;
    uint64_t footprint_now = 0;
    size_t arena_bytes = 0;
};

namespace {

size_t server_footprint(const ss_server* s, uint32_t n, uint64_t nchars) {
    return (size_t)(n + 1) * s->slot_bytes + (size_t)nchars;
}

void finish_locked(ss_server* S, Req* r, ss_status status) {
    r->state = RQ_DONE;
    r->status = status;
    r->t_done = Clock::now();
    if (status == SS_OK) {
        const double us = std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count();
        S->lat_us.push_back(us);
        S->st.completed++;
        S->st.strings_completed += r->r.n;
        S->st.chars_completed += r->nchars;
    }
}

// Admits queued requests (FIFO) while their footprint fits.
void admit_locked(ss_server* S, std::vector<Req*>& admitted) {
    while (!S->queue.empty() && !S->free_rids.empty()) {
        Req* r = S->queue.front();
        uint64_t pos = 0, cb = 0;
        if (!S->idx_alloc.alloc((uint64_t)r->r.n + 1, &pos)) break;
        if (!S->chr_alloc.alloc(r->nchars, &cb)) {
            S->idx_alloc.release(pos, (uint64_t)r->r.n + 1);
            break;
        }
        S->queue.pop_front();
        S->footprint_now += server_footprint(S, r->r.n, r->nchars);
        S->st.footprint_max = std::max<uint64_t>(S->st.footprint_max, S->footprint_now);
        r->pos = pos;
        r->cbase = cb;
        r->rid = S->free_rids.back();
        S->free_rids.pop_back();
        r->state = RQ_RUNNING;
        S->running[r->rid] = r;
        admitted.push_back(r);
    }
}

void release_locked(ss_server* S, Req* r) {
    S->footprint_now -= server_footprint(S, r->r.n, r->nchars);
    S->idx_alloc.release(r->pos, (uint64_t)r->r.n + 1);
    S->chr_alloc.release(r->cbase, r->nchars);
    S->running[r->rid] = nullptr;
    S->free_rids.push_back(r->rid);
}

// Copies a request to the device and adds it as a root of list slot `cur`.
ss_status stage_request(ss_server* S, Req* r) {
    hipStream_t s = S->stream;
    const uint64_t o0 = r->r.offsets[0];
    if (r->nchars)
        SS_TRY(hipMemcpyAsync(const_cast<uint8_t*>(S->p.chars) + r->cbase, r->r.chars + o0, r->nchars,
                              hipMemcpyHostToDevice, s));
    uint64_t* off = const_cast<uint64_t*>(S->p.offsets) + r->pos;
    SS_TRY(hipMemcpyAsync(off, r->r.offsets, sizeof(uint64_t) * ((size_t)r->r.n + 1), hipMemcpyHostToDevice, s));
    SS_TRY(launch_rebase(off, off, r->r.n, r->cbase - o0, s));
    S->h_slot[2 * r->rid] = (uint32_t)r->pos;
    S->h_slot[2 * r->rid + 1] = r->r.n;
    SS_TRY(hipMemcpyAsync(S->d_set_base + r->rid, &S->h_slot[2 * r->rid], 4, hipMemcpyHostToDevice, s));
    SS_TRY(hipMemcpyAsync(S->d_remaining + r->rid, &S->h_slot[2 * r->rid + 1], 4, hipMemcpyHostToDevice, s));
    SS_TRY(launch_admit(S->w, S->p, S->cur, (uint32_t)r->pos, r->r.n, r->rid, s));
    return SS_OK;
}

void fail_all_locked(ss_server* S, ss_status st) {
    for (auto& r : S->running)
        if (r) {
            finish_locked(S, r, st);
            release_locked(S, r);
        }
}

// One iteration of the engine: admit, run one level for every live request,
// complete finished requests.
void server_loop(ss_server* S) {
    (void)hipSetDevice(S->device);
    ss_ctx* ctx = S->ctx;
    for (;;) {
        std::vector<Req*> admitted;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                size_t live = 0;
                for (auto* r : S->running) live += r != nullptr;
                admit_locked(S, admitted);
                live += admitted.size();
                if (live) {
                    S->st.inflight_max = std::max<uint32_t>(S->st.inflight_max, (uint32_t)live);
                    break;
                }
                if (S->stop && S->queue.empty()) return;
                S->cv_work.wait(lk);
            }
        }
        const auto t_begin = Clock::now();
        double wait_us = 0;  // time spent waiting for the device in this iteration
        auto waited = [&](auto&& f) {
            const auto a = Clock::now();
            auto v = f();
            wait_us += std::chrono::duration<double, std::micro>(Clock::now() - a).count();
            return v;
        };
        ss_status st = SS_OK;
        for (Req* r : admitted)
            if ((st = stage_request(S, r)) != SS_OK) break;
        const double stage_us = std::chrono::duration<double, std::micro>(Clock::now() - t_begin).count();
        if (st == SS_OK) st = waited([&] { return read_ctl(ctx, S->w, S->stream); });
        if (st == SS_OK && ctx->host_ctl->err) st = device_error_status(ctx->host_ctl->err);
        if (st == SS_OK) {
            LevelPlan L;
            L.exact = true;
            L.c = counts_of(ctx->host_ctl->cl[S->cur]);
            st = enqueue_level(engine_of(ctx), S->w, S->p, S->cur, S->level, L, S->stream);
            S->cur ^= 1;
            ++S->level;
        }
        // which requests are finished?
        std::vector<Req*> finished;
        if (st == SS_OK) {
            hipError_t e = hipMemcpyAsync(S->h_remaining, S->d_remaining, sizeof(uint32_t) * S->max_inflight,
                                          hipMemcpyDeviceToHost, S->stream);
            if (e == hipSuccess) e = waited([&] { return hipStreamSynchronize(S->stream); });
            if (e != hipSuccess) st = SS_HIP_ERROR;
        }
        if (st == SS_OK) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->st.levels++;
            for (auto* r : S->running)
                if (r && S->h_remaining[r->rid] == 0) finished.push_back(r);
        }
        if (st == SS_OK && !finished.empty()) {
            for (Req* r : finished) S->h_done[r->rid] = 1;
            hipError_t e = hipMemcpyAsync(S->d_done, S->h_done, S->max_inflight, hipMemcpyHostToDevice, S->stream);
            if (e == hipSuccess) e = launch_pend_filter(S->w, S->p, S->stream);
            if (e == hipSuccess) e = launch_pend_swap(S->w, S->stream);
            std::swap(S->w.pend, S->w.pend2);
            for (Req* r : finished) {
                if (e != hipSuccess) break;
                if (r->r.n) {
                    e = hipMemcpyAsync(r->r.perm_out, S->p.perm + r->pos, sizeof(uint32_t) * r->r.n,
                                       hipMemcpyDeviceToHost, S->stream);
                    if (e == hipSuccess)
                        e = hipMemcpyAsync(r->r.lcp_out, S->p.lcp + r->pos, sizeof(uint32_t) * r->r.n,
                                           hipMemcpyDeviceToHost, S->stream);
                }
            }
            if (e == hipSuccess) e = waited([&] { return hipStreamSynchronize(S->stream); });
            for (Req* r : finished) S->h_done[r->rid] = 0;
            if (e == hipSuccess) e = hipMemcpyAsync(S->d_done, S->h_done, S->max_inflight, hipMemcpyHostToDevice, S->stream);
            if (e != hipSuccess) st = SS_HIP_ERROR;
            if (st == SS_OK && ctx->host_ctl->err == 0) {
                if (waited([&] { return read_ctl(ctx, S->w, S->stream); }) != SS_OK) st = SS_HIP_ERROR;
                else if (ctx->host_ctl->err) st = device_error_status(ctx->host_ctl->err);
            }
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            const double it_us = std::chrono::duration<double, std::micro>(Clock::now() - t_begin).count();
            S->busy_s += it_us * 1e-6;
            if (it_us > S->st.iter_max_us) {
                S->st.iter_max_us = it_us;
                S->st.iter_max_wait_us = wait_us;
                S->st.iter_max_stage_us = stage_us;
            }
            if (st != SS_OK) {
                fail_all_locked(S, st);
                // start over with an empty device state
                (void)launch_reset(S->w, S->stream);
                (void)hipStreamSynchronize(S->stream);
                S->cur = 0;
                S->level = 0;
            } else {
                for (Req* r : finished) {
                    finish_locked(S, r, SS_OK);
                    release_locked(S, r);
                }
            }
        }
        S->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

size_t ss_server_footprint(const ss_server* srv, uint32_t n, uint64_t n_chars) {
    return srv ? server_footprint(srv, n, n_chars) : 0;
}

ss_status ss_server_create(ss_server** out, int device, size_t hbm_budget, uint32_t max_inflight,
                           uint32_t mean_len_hint, const ss_config* cfg) {
    if (!out || max_inflight == 0 || max_inflight > 65536) return SS_INVALID_ARG;
    *out = nullptr;
    auto* S = new ss_server();
    ss_status st = ss_ctx_create(&S->ctx, device, 0);
    if (st != SS_OK) {
        delete S;
        return st;
    }
    if (cfg) {
        ss_config c = *cfg;
        c.mode = SS_MODE_HOST_LEVELS;  // the worker reads every level's counts
        clamp_config(&c);
        S->ctx->cfg = c;
    }
    S->device = device;
    S->max_inflight = max_inflight;
    const uint64_t L = mean_len_hint ? mean_len_hint : 48;
    // arena bytes per index slot: workspace + offsets + perm + lcp + second pending list
    const uint32_t probe = 1u << 20;
    const size_t ws = layout(probe, caps_for(probe, S->ctx->cfg), nullptr, nullptr);
    if (ensure_streams(S->ctx) != SS_OK || ensure_caps(S->ctx) != SS_OK) {
        ss_ctx_destroy(S->ctx);
        delete S;
        return SS_HIP_ERROR;
    }
    S->slot_bytes = ws / probe + 1 + sizeof(uint64_t) + 2 * sizeof(uint32_t) + sizeof(Pend);
    // 1% of the budget is left for the fixed tables and alignment
    const uint64_t cap_n = std::min<uint64_t>((hbm_budget - hbm_budget / 100) / (S->slot_bytes + L), 0xFFFFFFF0ull);
    if (cap_n < 1024) {
        ss_ctx_destroy(S->ctx);
        delete S;
        return SS_INVALID_ARG;
    }
    S->cap_n = (uint32_t)cap_n;
    S->cap_c = cap_n * L;
    (void)hipSetDevice(device);
    // one allocation: workspace | offsets | perm | lcp | pend2 | chars | slot tables
    const Caps k = caps_for(S->cap_n, S->ctx->cfg);
    const size_t ws_bytes = layout(S->cap_n, k, nullptr, nullptr);
    size_t off = ws_bytes;
    auto take = [&](size_t b) { size_t o = off; off += align_up(b); return o; };
    const size_t o_off = take(sizeof(uint64_t) * ((size_t)S->cap_n + 1));
    const size_t o_perm = take(sizeof(uint32_t) * (size_t)S->cap_n);
    const size_t o_lcp = take(sizeof(uint32_t) * (size_t)S->cap_n);
    const size_t o_pend2 = take(sizeof(Pend) * k.pend);
    const size_t o_chars = take(S->cap_c + 16);
    const size_t o_base = take(sizeof(uint32_t) * max_inflight);
    const size_t o_rem = take(sizeof(uint32_t) * max_inflight);
    const size_t o_done = take(max_inflight);
    if (off > hbm_budget) {  // the fixed part does not fit the budget
        ss_ctx_destroy(S->ctx);
        delete S;
        return SS_INVALID_ARG;
    }
    S->arena_bytes = off;
    if (hipMalloc(&S->mem, off) != hipSuccess) {
        (void)hipGetLastError();
        ss_ctx_destroy(S->ctx);
        delete S;
        return SS_OUT_OF_MEMORY;
    }
    char* base = (char*)S->mem;
    layout(S->cap_n, k, base, &S->w);
    S->w.pend2 = (Pend*)(base + o_pend2);
    S->d_set_base = (uint32_t*)(base + o_base);
    S->d_remaining = (uint32_t*)(base + o_rem);
    S->d_done = (uint8_t*)(base + o_done);
    S->w.set_base = S->d_set_base;
    S->w.remaining = S->d_remaining;
    S->w.done = S->d_done;
    const ss_config& c = S->ctx->cfg;
    S->p = Params{(const uint8_t*)(base + o_chars), (const uint64_t*)(base + o_off), S->cap_n,
                  (uint32_t*)(base + o_perm), (uint32_t*)(base + o_lcp), c.max_log_splitters, c.bucket_target,
                  c.base_max};
    bool ok = hipHostMalloc((void**)&S->h_remaining, sizeof(uint32_t) * max_inflight, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void**)&S->h_slot, 2 * sizeof(uint32_t) * max_inflight, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void**)&S->h_done, max_inflight, hipHostMallocDefault) == hipSuccess &&
              hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) == hipSuccess;
    if (ok) {
        std::memset(S->h_done, 0, max_inflight);
        std::memset(S->h_remaining, 0, sizeof(uint32_t) * max_inflight);
        ok = hipMemcpyAsync(S->d_done, S->h_done, max_inflight, hipMemcpyHostToDevice, S->stream) == hipSuccess &&
             hipMemcpyAsync(S->d_remaining, S->h_remaining, sizeof(uint32_t) * max_inflight, hipMemcpyHostToDevice,
                            S->stream) == hipSuccess &&
             launch_reset(S->w, S->stream) == hipSuccess && hipStreamSynchronize(S->stream) == hipSuccess;
    }
    if (!ok) {
        ss_server_destroy(S);
        return SS_HIP_ERROR;
    }
    S->idx_alloc.init(S->cap_n);
    S->chr_alloc.init(S->cap_c);
    S->running.assign(max_inflight, nullptr);
    for (uint32_t r = max_inflight; r-- > 0;) S->free_rids.push_back(r);
    S->worker = std::thread(server_loop, S);
    *out = S;
    return SS_OK;
}

ss_status ss_server_submit(ss_server* S, const ss_request* req, uint64_t* ticket) {
    if (!S || !req || !ticket || !req->offsets) return SS_INVALID_ARG;
    if (req->n && (!req->perm_out || !req->lcp_out)) return SS_INVALID_ARG;
    const uint64_t* o = req->offsets;
    for (uint32_t i = 0; i < req->n; ++i)
        if (o[i + 1] < o[i] || o[i + 1] - o[i] > MAX_LEN) return SS_LIMIT;
    const uint64_t nchars = o[req->n] - o[0];
    if (nchars && !req->chars) return SS_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    S->st.submitted++;
    if ((uint64_t)req->n + 1 > S->cap_n || nchars > S->cap_c) {
        S->st.rejected++;
        return SS_REJECTED;
    }
    auto* r = new Req();
    r->ticket = S->next_ticket++;
    r->r = *req;
    r->nchars = nchars;
    r->t_submit = Clock::now();
    S->reqs[r->ticket] = r;
    S->queue.push_back(r);
    *ticket = r->ticket;
    S->cv_work.notify_one();
    return SS_OK;
}

ss_status ss_server_wait(ss_server* S, uint64_t ticket, int timeout_ms, double* latency_us) {
    if (!S) return SS_INVALID_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return SS_INVALID_ARG;
    Req* r = it->second;
    auto pred = [&] { return r->state == RQ_DONE; };
    if (timeout_ms < 0) S->cv_done.wait(lk, pred);
    else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred)) return SS_TIMEOUT;
    const ss_status st = r->status;
    if (latency_us) *latency_us = std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count();
    S->reqs.erase(it);
    delete r;
    return st;
}

ss_status ss_server_cancel(ss_server* S, uint64_t ticket) {
    if (!S) return SS_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end() || it->second->state != RQ_QUEUED) return SS_INVALID_ARG;
    Req* r = it->second;
    for (auto q = S->queue.begin(); q != S->queue.end(); ++q)
        if (*q == r) {
            S->queue.erase(q);
            break;
        }
    S->st.cancelled++;
    S->reqs.erase(it);
    delete r;
    return SS_OK;
}

ss_status ss_server_get_stats(ss_server* S, ss_server_stats* out) {
    if (!S || !out) return SS_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    ss_server_stats st = S->st;
    std::vector<double> v = S->lat_us;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) { return v[std::min(v.size() - 1, (size_t)(q * (double)(v.size() - 1) + 0.5))]; };
        st.p50_us = pct(0.50);
        st.p99_us = pct(0.99);
        double sum = 0;
        for (double x : v) sum += x;
        st.mean_us = sum / (double)v.size();
        st.max_us = v.back();
    }
    st.busy_s = S->busy_s;
    st.arena_bytes = S->arena_bytes;
    *out = st;
    return SS_OK;
}

void ss_server_reset_stats(ss_server* S) {
    if (!S) return;
    std::lock_guard<std::mutex> lk(S->mu);
    S->st = ss_server_stats{};
    S->st.footprint_max = S->footprint_now;
    S->lat_us.clear();
    S->busy_s = 0;
}

void ss_server_destroy(ss_server* S) {
    if (!S) return;
    if (S->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
        }
        S->cv_work.notify_all();
        S->worker.join();
    }
    (void)hipSetDevice(S->device);
    if (S->stream) (void)hipStreamDestroy(S->stream);
    if (S->mem) (void)hipFree(S->mem);
    if (S->h_remaining) (void)hipHostFree(S->h_remaining);
    if (S->h_slot) (void)hipHostFree(S->h_slot);
    if (S->h_done) (void)hipHostFree(S->h_done);
    for (auto& kv : S->reqs) delete kv.second;
    if (S->ctx) ss_ctx_destroy(S->ctx);
    delete S;
}

}  // extern "C"
