// gfx950 kernels of the string sample sort.
//
// One recursion level of the sort processes every live segment at once:
//   k_base      segments of <= base_max strings: sorted in LDS, LCPs inside
//   k_sample    per large segment: regular sample, sort, splitter tree
//   k_classify  per tile: tree descent -> bucket ids, tile histogram
//   k_scan_*    exclusive scan over all (bucket-major, tile-minor) counters
//   k_scatter   per tile: stable scatter into the other ping-pong buffer
//   k_children  per large segment: buckets -> next-level segments
// and k_lcp_fill resolves the LCPs at bucket boundaries at the end.
#include <algorithm>

#include "ss_device.h"
#include "ss_gather.h"
#include "ss_internal.h"

namespace ss {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ void raise_err(const Work& w, uint32_t bits) {
    atomicOr(&w.ctl->err, bits);
    atomicOr(&w.ctl->err_sticky, bits);
}
// Record fields (Rec: narrow records keep r in the top bits of the index
// word, wide ones in the side array rw).
__device__ __forceinline__ uint64_t rec_key(const Rec& x) { return (uint64_t)x.klo | (uint64_t)x.khi << 32; }
__device__ __forceinline__ uint32_t rec_idx(const Work& w, const Rec& x) { return w.wide ? x.ix : x.ix & IX_MASK; }
__device__ __forceinline__ uint32_t rec_r(const Work& w, const Rec& x, int buf, uint32_t i) {
    return w.wide ? (uint32_t)w.rw[buf][i] : x.ix >> IX_BITS;
}
__device__ __forceinline__ Rec rec_make(const Work& w, uint64_t key, uint32_t idx, uint32_t r) {
    Rec x;
    x.klo = (uint32_t)key;
    x.khi = (uint32_t)(key >> 32);
    x.ix = w.wide ? idx : idx | r << IX_BITS;
    return x;
}
__device__ __forceinline__ void rec_put(const Work& w, int buf, uint32_t i, uint64_t key, uint32_t idx, uint32_t r) {
    w.rec[buf][i] = rec_make(w, key, idx, r);
    if (w.wide) w.rw[buf][i] = (uint8_t)r;
}

// Two counters in one 64-bit atomic word (low, high); neither half of a
// level's counters reaches 2^32, so no carry crosses.
__device__ __forceinline__ unsigned long long pack2(uint32_t lo, uint32_t hi) {
    return (unsigned long long)lo | ((unsigned long long)hi << 32);
}

// A level's work counter, written by earlier launches (or, in the
// persistent kernel, before the last grid barrier).
__device__ __forceinline__ unsigned long long load_count(const CLine& l) {
    return __hip_atomic_load(&l.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Counts clamped to the pool capacities: after a capacity error (raised by
// whoever overflowed a pool) the entries past the capacity were never
// written, so no kernel may index them.
__device__ __forceinline__ void clamp_counts(Counts& c, const Caps& k) {
    c.n_dist = min_u32(c.n_dist, k.dist);
    c.n_tiles = min_u32(c.n_tiles, k.tiles);
    c.n_cnt = min_u32(c.n_cnt, k.cnt);
    c.n_tree = min_u32(c.n_tree, k.tree);
    for (int q = 0; q < NCLS; ++q) c.n_base[q] = min_u32(c.n_base[q], k.base[q]);
}
__device__ __forceinline__ uint32_t n_dist_of(const Work& w, int cur) {
    return min_u32((uint32_t)load_count(w.ctl->cl[cur].dist), w.caps.dist);
}
__device__ __forceinline__ uint32_t n_tiles_of(const Work& w, int cur) {
    return min_u32((uint32_t)(load_count(w.ctl->cl[cur].tree_tiles) >> 32), w.caps.tiles);
}
__device__ __forceinline__ uint32_t n_cnt_of(const Work& w, int cur) {
    return min_u32((uint32_t)load_count(w.ctl->cl[cur].cnt), w.caps.cnt);
}
__device__ __forceinline__ uint32_t n_base_of(const Work& w, int cur, int cls) {
    return min_u32((uint32_t)load_count(w.ctl->cl[cur].base[cls]), w.caps.base[cls]);
}
__device__ __forceinline__ Counts load_counts(const Work& w, int cur) {
    unsigned long long v[COUNT_LINES];
    const CLine* L = &w.ctl->cl[cur].dist;
    for (uint32_t i = 0; i < COUNT_LINES; ++i) v[i] = load_count(L[i]);
    return counts_of(v);
}

__device__ __forceinline__ FeedLine* feed_of(const Work& w, int cur, uint32_t kind) {
    return w.feed + ((uint32_t)cur * FEED_KINDS + kind) * FEED_PARTS;
}

// Next chunk [*lo, *hi) of part `part` of the items [first, n) (see
// FeedLine); false once the part is used up.  The parts are contiguous, so
// a part's items are neighbours (for tiles: adjacent parts of the same
// buckets, written through the same L2).
__device__ __forceinline__ bool feed_take(FeedLine* f, uint32_t first, uint32_t n, uint32_t part, uint32_t chunk,
                                          uint32_t* lo, uint32_t* hi) {
    if (first >= n) return false;
    const uint32_t len = (n - first + FEED_PARTS - 1) / FEED_PARTS;
    const uint32_t b = first + part * len;
    const uint32_t e = min_u32(b + len, n);
    if (b >= e) return false;
    const uint32_t i = atomicAdd(&f[part].next, chunk);
    if (i >= e - b) return false;
    *lo = b + i;
    *hi = min_u32(b + i + chunk, e);
    return true;
}

// Static first items of a launch's work groups, keeping consecutive items on
// the same XCD (work groups are dispatched to the 8 XCDs round robin): the
// items of XCD x are a contiguous range, so concurrently running
// neighbouring tiles write adjacent parts of the same buckets through the
// same L2.  A bijection on [0, nt).
__device__ __forceinline__ uint32_t xcd_item(uint32_t b, uint32_t nt) {
    constexpr uint32_t X = FEED_PARTS;
    const uint32_t x = b % X, i = b / X, q = nt / X, r = nt % X;
    return x * q + (x < r ? x : r) + i;
}

// A value every lane of the wave holds alike (read back from an LDS
// mailbox), marked uniform so that what is derived from it (segment fields,
// addresses) stays in scalar registers.
__device__ __forceinline__ uint32_t uniform(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }

// The sort's key format (KeyFmt; chosen by the alphabet kernels below and
// kept in the control block).  fmt_full derives it from the byte set (the
// key gather and the first sampling, and every compressed gather);
// fmt_head reads the code width and characters per word that the key
// gather stored, enough for everything but a gather (kernels that only
// compare keys do not hold the set).
__device__ __forceinline__ bool fmt_compressed(const Work& w) {
    return uniform(w.ctl->alpha.cand) != 0u && uniform(w.ctl->alpha.over) == 0u;
}
__device__ __forceinline__ KeyFmt fmt_full(const Work& w) {
    uint64_t m[4] = {0, 0, 0, 0};
    if (fmt_compressed(w)) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint64_t v = w.ctl->alpha.seen[i];
            m[i] = (uint64_t)uniform((uint32_t)v) | (uint64_t)uniform((uint32_t)(v >> 32)) << 32;
        }
    }
    return key_fmt_of(m);  // byte keys for an empty set
}
__device__ __forceinline__ KeyFmt fmt_head(const Work& w) {
    KeyFmt h{};
    h.bpc = uniform(w.ctl->alpha.bpc);
    h.cpw = uniform(w.ctl->alpha.cpw);
    return h;
}
// The key format as a compile-time choice: kernels instantiate their
// bodies for byte keys and for compressed keys and pick one per sort, so
// the byte-key body carries none of the compressed code.
template <bool AC>
__device__ __forceinline__ KeyFmt fmt_of(const Work& w) {
    if constexpr (AC) {
        return fmt_head(w);
    } else {
        KeyFmt f{};
        f.bpc = 0;
        f.cpw = W;
        return f;
    }
}
// Stores the code width and characters per word for fmt_head (one thread
// of the key gather).
__device__ __forceinline__ void fmt_publish(const Work& w, const KeyFmt& f) {
    w.ctl->alpha.bpc = f.bpc;
    w.ctl->alpha.cpw = f.cpw;
}
// chars_h in the sort's key format.
__device__ __forceinline__ uint64_t key_at_packed(const Work& w, const uint8_t* chars, uint64_t off, uint32_t h,
                                                  uint32_t len) {
    const KeyFmt f = fmt_full(w);
    bool miss = false;
    const uint64_t key = gather_packed_with(
        chars, off, h, len, f, [](const uint64_t* q) { return __builtin_nontemporal_load(q); }, &miss);
    // a byte outside the set (possible when the input was not checked in
    // full): the key is not to be trusted, the host sorts again
    if (miss) w.ctl->alpha.miss = 1;
    return key;
}
__device__ __forceinline__ uint64_t key_at(const Work& w, const KeyFmt& fh, const uint8_t* chars, uint64_t off,
                                           uint32_t h, uint32_t len) {
    if (fh.bpc == 0) return gather_key(chars, off, h, len);
    return key_at_packed(w, chars, off, h, len);
}
// The same as a call: the scatter's write loop and the base cases'
// refinement, at their register budgets, keep the compressed gather out of
// line.
__device__ __attribute__((noinline)) uint64_t key_at_packed_call(const Work& w, const uint8_t* chars, uint64_t off,
                                                                 uint32_t h, uint32_t len) {
    return key_at_packed(w, chars, off, h, len);
}

// A string of an equality bucket moves on to depth h: its key there and the
// code of its characters inside that key, from its offsets (the length is
// not carried with the record).
__device__ __forceinline__ void regather(const Work& w, const KeyFmt& fh, const Params& p, uint32_t idx, uint32_t h,
                                         uint64_t& key, uint32_t& r) {
    const uint64_t o0 = p.offsets[idx], o1 = p.offsets[idx + 1];
    const uint32_t len = (uint32_t)(o1 - o0);
    key = fh.bpc == 0 ? gather_key(p.chars, o0, h, len) : key_at_packed_call(w, p.chars, o0, h, len);
    r = kf_r(fh, len, h);
}

// A member of an equality bucket, with its key one word beyond the
// splitter's: when that key differs from the splitter's sample string's
// key there (or the member ends inside the word), the bucket cannot skip
// the word (k_children).  The flag only ever goes from 0 to 1, so plain
// stores suffice, and reading it first skips most of them.
__device__ __forceinline__ void note_next(const Work& w, int cur, uint32_t t, uint64_t key, uint32_t r) {
    uint32_t* const df = &w.tree_diff[cur][t];
    if (*df == 0 && (key != w.tree_next[cur][t] || r != W)) *df = 1;
}

// One item of the dynamic part [first, n) for a work group (n when none is
// left).
__device__ __forceinline__ uint32_t feed_one(FeedLine* f, uint32_t first, uint32_t n, uint32_t part) {
    uint32_t lo = 0, hi = 0;
    return feed_take(f, first, n, part, 1, &lo, &hi) ? lo : n;
}

// Records a level's work counts when it starts (statistics; the profiler's
// per-launch units).  One thread.
__device__ void note_level(const Work& w, const Counts& c, uint32_t level) {
    bool work = c.n_dist != 0;
    for (int q = 0; q < NCLS; ++q) work |= c.n_base[q] != 0;
    if (!work) return;
    DevStats& st = w.ctl->stats;
    st.levels = level + 1;
    st.dist_segments += c.n_dist;
    st.dist_tiles += c.n_tiles;
    st.dist_strings += c.dist_strings;
    if (c.max_depth > st.max_depth) st.max_depth = c.max_depth;
    for (int q = 0; q < NCLS; ++q) {
        st.base_segments[q] += c.n_base[q];
        st.base_strings[q] += c.base_strings[q];
    }
    if (level < LEVEL_RECS) {
        LevelRec r;
        r.n_dist = c.n_dist;
        r.n_tiles = c.n_tiles;
        r.n_cnt = c.n_cnt;
        r.dist_strings = c.dist_strings;
        for (int q = 0; q < NCLS; ++q) {
            r.n_base[q] = c.n_base[q];
            r.base_strings[q] = c.base_strings[q];
        }
        w.ctl->lv[level] = r;
    }
}


// Appends a segment of the next level (positions [begin, begin+size) of
// buffer `buf`, common prefix `depth`) to the work lists of counts slot
// `nxt`: a single string is final at once, small segments go to the base
// case, larger ones get a distribution step with its tree, counters and
// tiles reserved here.
__device__ void emit_segment(const Work& w, const Params& p, int nxt, int buf, uint32_t begin,
                             uint32_t size, uint32_t depth, uint32_t rid) {
    if (size == 0) return;
    if (size == 1) {
        p.perm[begin] = rec_idx(w, w.rec[buf][begin]) - w.set_base[rid];
        if (w.remaining) atomicSub(&w.remaining[rid], 1u);
        return;
    }
    CountLines* c = &w.ctl->cl[nxt];
    atomicMax(&c->depth.v, (unsigned long long)depth);
    if (size <= p.base_max) {
        const int cls = size_class(size);
        const uint32_t slot = (uint32_t)atomicAdd(&c->base[cls].v, pack2(1u, size));
        if (slot >= w.caps.base[cls]) { raise_err(w, ERR_CAPACITY); return; }
        w.base[cls][nxt][slot] = BaseSeg{begin, size, depth, rid};
        return;
    }
    uint32_t logv = choose_logv(size, p.bucket_target, p.max_logv);
    uint32_t v = (1u << logv) - 1, k = 2 * v + 1;
    uint32_t T = (size + TILE - 1) / TILE;
    const uint32_t slot = (uint32_t)atomicAdd(&c->dist.v, pack2(1u, size));
    const unsigned long long tt = atomicAdd(&c->tree_tiles.v, pack2(v + 1, T));
    const uint32_t toff = (uint32_t)tt, tioff = (uint32_t)(tt >> 32);
    const uint32_t coff = (uint32_t)atomicAdd(&c->cnt.v, (unsigned long long)(k * T));
    if (slot >= w.caps.dist || toff + v + 1 > w.caps.tree || coff + k * T > w.caps.cnt ||
        tioff + T > w.caps.tiles) {
        raise_err(w, ERR_CAPACITY);
        return;
    }
    // the tile list entries are written by k_sample (one work group per segment)
    w.dist[nxt][slot] = Seg{begin, size, depth, logv, toff, coff, tioff, rid, 0u};
}

// wave-level inclusive scans over 64 lanes
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
    const uint32_t lane = threadIdx.x & 63;
#pragma unroll
    for (uint32_t o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}
__device__ __forceinline__ uint32_t wave_max(uint32_t x) {
#pragma unroll
    for (uint32_t o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_xor(x, o, 64);
        x = x > y ? x : y;
    }
    return x;
}
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t x) {
    const uint32_t lane = threadIdx.x & 63;
#pragma unroll
    for (uint32_t o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x = x > y ? x : y;
    }
    return x;
}


// Shared-memory layouts of the per-item device functions.  Standalone
// kernels declare the one they need; the persistent kernel declares their
// union, so its LDS footprint is the largest of them.
struct SmBase {
    uint64_t K[BASE_CAP];  // packed sort records: hi words
    uint64_t A[BASE_CAP];  // lo words
    uint32_t dep[BASE_CAP];
    uint32_t lv[BASE_CAP];
    uint32_t aux[BASE_CAP];   // bit 31: tie with the left neighbour; low bits: run start
    uint32_t rmin[BASE_CAP];  // per run start: common prefix of the run
    uint32_t wtot[WAVES];
    uint32_t any;
};
struct SmWave {
    uint32_t LIDX[WAVES][256];  // per run start: index of the run's first string
    uint32_t RMIN[WAVES][256];  // per run start: common prefix of the run
};
struct SmSample {
    uint64_t SK[2 << MAX_LOGV];
    uint32_t SR[2 << MAX_LOGV];
    union {
        uint64_t SA[2 << MAX_LOGV];  // sort records' second words (while sorting)
        struct {
            uint64_t TK[1 << MAX_LOGV];
            uint32_t TR[1 << MAX_LOGV];
            uint16_t NL[1 << MAX_LOGV];
            uint16_t NH[1 << MAX_LOGV];
        };
    };
};
struct SmClassify {
    uint64_t TK[1 << MAX_LOGV];
    uint32_t TR[1 << MAX_LOGV];
    uint32_t H[MAX_BUCKETS + 1];
};
struct SmScatter {
    uint32_t WC[WAVES][MAX_BUCKETS + 1];  // per-wave counts, then per-wave write bases
};
struct SmChildren {
    uint32_t ST[MAX_BUCKETS + 1];  // bucket starts relative to the segment
    uint32_t n_cls[NCLS], s_cls[NCLS], slot_cls[NCLS], cur_cls[NCLS];
    uint32_t n_pend_l, slot_pend, cur_pend, max_d;
    // distribution children: counts / sums, reserved bases, running offsets
    uint32_t nd, sd, ntree, ncnt, ntile;
    uint32_t bd, btree, bcnt, btile;
    uint32_t cd, ctree, ccnt, ctile;
};
constexpr uint32_t SCAN_PER_THREAD = 16;
constexpr uint32_t SCAN_CHUNK = BLOCK * SCAN_PER_THREAD;
struct SmScan {
    uint32_t wt[16];
    uint32_t carry;
    uint32_t t[SCAN_CHUNK + SCAN_CHUNK / 32];  // a chunk, one pad word per 32 (conflict-free columns)
};
union SmAll {
    SmBase base;
    SmWave wave;
    SmSample sample;
    SmClassify classify;
    SmScatter scatter;
    SmChildren children;
    SmScan scan;
};

// ---------------------------------------------------------------------------
// reset / init / roots
// ---------------------------------------------------------------------------

__global__ void k_reset(Work w) {
    uint32_t* p = (uint32_t*)w.ctl;
    constexpr uint32_t keep = offsetof(Ctl, err_sticky) / 4;  // survives the reset
    for (uint32_t i = threadIdx.x; i < sizeof(Ctl) / 4; i += blockDim.x)
        if (i != keep) p[i] = 0;
    if (threadIdx.x == 0) w.zero_base[0] = 0;
    uint32_t* b = (uint32_t*)w.bar;
    for (uint32_t i = threadIdx.x; i < sizeof(GridBar) / 4; i += blockDim.x) b[i] = 0;
    for (uint32_t i = threadIdx.x; i < FEED_LINES; i += blockDim.x) w.feed[i].next = 0;
}

__global__ void k_level_begin(Work w, int cur, uint32_t level) {
    // A sort with an error stops here: the level's counts are dropped, so no
    // kernel of this or a later level finds work (malformed offsets are
    // found by the key gather, before any string is read past its first
    // word).
    if (__hip_atomic_load(&w.ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        CLine* C = &w.ctl->cl[cur].dist;
        for (uint32_t i = threadIdx.x; i < COUNT_LINES; i += blockDim.x) C[i].v = 0;
    } else if (threadIdx.x == 0) {
        note_level(w, load_counts(w, cur), level);
    }
    CLine* L = &w.ctl->cl[cur ^ 1].dist;
    for (uint32_t i = threadIdx.x; i < COUNT_LINES; i += blockDim.x) L[i].v = 0;
    FeedLine* f = feed_of(w, cur, 0);
    for (uint32_t i = threadIdx.x; i < FEED_KINDS * FEED_PARTS; i += blockDim.x) f[i].next = 0;
}

// Key gather at depth 0 for every string (Algorithm 4.1's chars_h with
// h = 0), plus offset validation.
__device__ __forceinline__ void dev_init_one(const Work& w, const KeyFmt& fh, const Params& p, uint32_t i) {
    uint64_t o0 = p.offsets[i], o1 = p.offsets[i + 1];
    uint32_t len = 0;
    if (o1 < o0 || o1 - o0 > MAX_LEN || (o1 > o0 && p.chars == nullptr)) raise_err(w, ERR_OFFSETS);
    else len = (uint32_t)(o1 - o0);
    rec_put(w, 0, i, key_at(w, fh, p.chars, o0, 0, len), i, kf_r(fh, len, 0));
}

// The key gather with compressed keys codes every string's first word.  It
// reads each byte's code from a table in LDS (tab[c]: the code of c, or
// TAB_MISS for a byte outside the set) instead of ranking the byte in the
// set as key_at_packed does, loads the (at most five) aligned words that
// hold the first CPW = 64 / BPC characters at once, aligns them into 8-byte
// groups and codes every character position unrolled (positions past the
// string's end code 0), so the loads and the table reads are all in flight
// together.
constexpr uint32_t TAB_MISS = 0x80;
template <uint32_t BPC>
__device__ __forceinline__ uint64_t gather_packed_tab(const uint8_t* chars, uint64_t off, uint32_t len,
                                                      const uint8_t* tab, uint32_t& bad) {
    constexpr uint32_t CPW = 64 / BPC, NG = (CPW + 7) / 8;
    const uint32_t rem = len < CPW ? len : CPW;
    if (rem == 0) return 0;
    const uintptr_t a = (uintptr_t)(chars + off);
    const uint64_t* q = (const uint64_t*)(a & ~(uintptr_t)7);
    const uint32_t sh = (uint32_t)(a & 7), nw = (sh + rem + 7) >> 3;  // words that hold the characters
    uint64_t wd[NG + 1];
#pragma unroll
    for (uint32_t u = 0; u <= NG; ++u) wd[u] = u < nw ? __builtin_nontemporal_load(q + u) : 0ull;
    uint64_t key = 0;
#pragma unroll
    for (uint32_t g = 0; g < NG; ++g) {
        // characters 8g .. 8g+7 of the string
        const uint64_t grp = sh ? (wd[g] >> (8 * sh)) | (wd[g + 1] << (64 - 8 * sh)) : wd[g];
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) {
            const uint32_t k = 8 * g + j;
            if (k >= CPW) break;
            const uint32_t t = k < rem ? (uint32_t)tab[(uint32_t)(grp >> (8 * j)) & 0xFFu] : 0u;
            bad |= t;
            key |= (uint64_t)(t & 0x0Fu) << (64 - BPC * (k + 1));
        }
    }
    return key;
}

template <bool AC>
__global__ __launch_bounds__(BLOCK) void k_init(Work w, Params p) {
    uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if constexpr (AC) {
        __shared__ uint8_t tab[256];
        const KeyFmt f = fmt_full(w);
        if (i == 0) fmt_publish(w, f);
        for (uint32_t c = threadIdx.x; c < 256; c += BLOCK)
            tab[c] = (uint8_t)(kf_has(f, c) ? kf_code(f, c) : TAB_MISS);
        __syncthreads();
        if (i < p.n) {
            uint64_t o0 = p.offsets[i], o1 = p.offsets[i + 1];
            uint32_t len = 0;
            if (o1 < o0 || o1 - o0 > MAX_LEN || (o1 > o0 && p.chars == nullptr)) raise_err(w, ERR_OFFSETS);
            else len = (uint32_t)(o1 - o0);
            uint32_t bad = 0;
            const uint64_t key = f.bpc == 2   ? gather_packed_tab<2>(p.chars, o0, len, tab, bad)
                                 : f.bpc == 3 ? gather_packed_tab<3>(p.chars, o0, len, tab, bad)
                                              : gather_packed_tab<4>(p.chars, o0, len, tab, bad);
            // a byte outside the set (the input was not checked in full): the
            // host sorts again
            if (bad & TAB_MISS) w.ctl->alpha.miss = 1;
            rec_put(w, 0, i, key, i, kf_r(f, len, 0));
        }
    } else {
        if (i < p.n) dev_init_one(w, fmt_of<false>(w), p, i);
    }
}

// One root segment per set (one set = the whole input for a plain sort).
__device__ __forceinline__ void dev_root_one(const Work& w, const Params& p, const uint32_t* set_begin,
                                             uint32_t num_sets, uint32_t j) {
    uint32_t b = 0, e = p.n;
    if (set_begin) {
        b = set_begin[j];
        e = set_begin[j + 1];
        if (e < b || e > p.n || (j == 0 && b != 0) || (j + 1 == num_sets && e != p.n)) {
            raise_err(w, ERR_SETS);
            return;
        }
    }
    if (e > b) p.lcp[b] = 0;
    if (e - b == 1) {  // final at once; string b (the key gather may not have run yet)
        p.perm[b] = b - w.set_base[set_begin ? j : 0u];
        if (w.remaining) atomicSub(&w.remaining[set_begin ? j : 0u], 1u);
        return;
    }
    emit_segment(w, p, 0, 0, b, e - b, 0, set_begin ? j : 0u);
}

__global__ void k_roots(Work w, Params p, const uint32_t* set_begin, uint32_t num_sets) {
    uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < num_sets) dev_root_one(w, p, set_begin, num_sets, j);
}

// ---------------------------------------------------------------------------
// base case for small segments: one wave per segment, data in registers
// ---------------------------------------------------------------------------

// Sort record of the register networks (wave base case, sample sort): two
// words compared as one unsigned 128-bit number, so a single comparison
// orders by (group, key, r, idx):
//   hi = group(16) | key bits 63..16,   lo = key bits 15..0 | 0(12) | r(4) | idx(32).
__device__ __forceinline__ void pr_pack(uint32_t grp, uint64_t key, uint32_t r, uint32_t idx, uint64_t& hi,
                                        uint64_t& lo) {
    hi = ((uint64_t)grp << 48) | (key >> 16);
    lo = (key << 48) | ((uint64_t)r << 32) | (uint64_t)idx;
}
__device__ __forceinline__ uint64_t pr_key(uint64_t hi, uint64_t lo) { return (hi << 16) | (lo >> 48); }
__device__ __forceinline__ uint32_t pr_grp(uint64_t hi) { return (uint32_t)(hi >> 48); }
__device__ __forceinline__ uint32_t pr_r(uint64_t lo) { return (uint32_t)(lo >> 32) & 0xFu; }
__device__ __forceinline__ uint32_t pr_idx(uint64_t lo) { return (uint32_t)lo; }
__device__ __forceinline__ uint64_t pr_regroup(uint64_t hi, uint32_t grp) {
    return (hi & 0x0000FFFFFFFFFFFFull) | ((uint64_t)grp << 48);
}
__device__ __forceinline__ bool pr_gt(uint64_t ah, uint64_t al, uint64_t bh, uint64_t bl) {
    return ah > bh || (ah == bh && al > bl);
}

// Value of lane (lane ^ J) of a wave: DPP quad permutations for 1 and 2, an
// LDS-crossbar swizzle for 4, 8 and 16, and the gfx950 row-swap permute for
// 32 (after the swap the two results hold the even and the odd halves; each
// lane picks the one of its partner).
template <uint32_t J>
__device__ __forceinline__ uint32_t xlane32(uint32_t x) {
    static_assert(J == 1 || J == 2 || J == 4 || J == 8 || J == 16 || J == 32, "lane distance");
    const int v = (int)x;
    // every lane's source lies inside its row, so no lane keeps an old value
    if constexpr (J == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
    } else if constexpr (J == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
    } else if constexpr (J == 4 || J == 8 || J == 16) {
        // LDS crossbar swizzle in bit-mask mode (lane ^ J inside 32 lanes):
        // one instruction off the vector ALU, which the networks saturate
        return (uint32_t)__builtin_amdgcn_ds_swizzle(v, (int)((J << 10) | 0x1F));
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        return (__lane_id() & 32) ? r[0] : r[1];
    }
}
template <uint32_t J>
__device__ __forceinline__ uint64_t xlane64(uint64_t x) {
    return (uint64_t)xlane32<J>((uint32_t)x) | ((uint64_t)xlane32<J>((uint32_t)(x >> 32)) << 32);
}
__device__ __forceinline__ uint64_t xlane(uint64_t x, uint32_t lj) {
    switch (lj) {  // lj is a compile-time constant at every call site after unrolling
    case 1: return xlane64<1>(x);
    case 2: return xlane64<2>(x);
    case 4: return xlane64<4>(x);
    case 8: return xlane64<8>(x);
    case 16: return xlane64<16>(x);
    default: return xlane64<32>(x);
    }
}

// Lanes of a wave whose record (global index base + lane*E + r of a
// blocked layout) has the bit `bit` (a power of two) set: a constant lane
// pattern when the bit falls on the lane number, all or none otherwise.
// Used through inverse ballots, the compare-exchange directions cost no
// vector instructions.
template <int E>
__device__ __forceinline__ uint64_t lanes_with_bit(uint32_t bit, uint32_t r, uint32_t base) {
    if (bit < (uint32_t)E) return (r & bit) ? ~0ull : 0ull;
    if (bit >= 64u * E) return (base & bit) ? ~0ull : 0ull;
    switch (bit / E) {
    case 1: return 0xAAAAAAAAAAAAAAAAull;
    case 2: return 0xCCCCCCCCCCCCCCCCull;
    case 4: return 0xF0F0F0F0F0F0F0F0ull;
    case 8: return 0xFF00FF00FF00FF00ull;
    case 16: return 0xFFFF0000FFFF0000ull;
    default: return 0xFFFFFFFF00000000ull;
    }
}
__device__ __forceinline__ bool lane_in(uint64_t lanes) { return __builtin_amdgcn_inverse_ballot_w64(lanes); }

// One compare-exchange stage (k, j) of a bitonic network over records in
// blocked layout (lane holds records lane*E .. lane*E+E-1 of a block whose
// first record has global index `base`): partners inside a lane are
// exchanged in registers, partners in other lanes (j >= E) through
// cross-lane shuffles.  Directions follow the global index, so blocks of
// several waves can form one network.
template <int E>
__device__ __forceinline__ void wave_stage(uint64_t (&K)[E], uint64_t (&A)[E], uint32_t lane, uint32_t base,
                                           uint32_t k, uint32_t j) {
    if (j < (uint32_t)E) {
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)E; ++r) {
            if ((r & j) == 0) {
                const uint32_t r2 = r | j;
                const bool up = lane_in(~lanes_with_bit<E>(k, r, base));
                if (pr_gt(K[r], A[r], K[r2], A[r2]) == up) {
                    uint64_t tk = K[r]; K[r] = K[r2]; K[r2] = tk;
                    uint64_t ta = A[r]; A[r] = A[r2]; A[r2] = ta;
                }
            }
        }
    } else {
        const uint32_t lj = j / E;
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)E; ++r) {
            const uint64_t pk = xlane(K[r], lj);
            const uint64_t pa = xlane(A[r], lj);
            // keep the smaller when the bits j and k of the index agree
            const bool keep_min = lane_in(~(lanes_with_bit<E>(j, r, base) ^ lanes_with_bit<E>(k, r, base)));
            const bool self_gt = pr_gt(K[r], A[r], pk, pa);
            if (self_gt == keep_min) { K[r] = pk; A[r] = pa; }
        }
    }
}

// Bitonic sorting network over the 64*E records of one wave (merge sizes
// k = 2 .. 64E).  No LDS, no barriers.  With base = 0 the block ends up
// ascending; as part of a larger network (base = wave * 64E) blocks
// alternate in direction.
template <int E>
__device__ __forceinline__ void wave_bitonic(uint64_t (&K)[E], uint64_t (&A)[E], uint32_t lane, uint32_t base = 0) {
#pragma unroll
    for (uint32_t k = 2; k <= 64u * E; k <<= 1) {
#pragma unroll
        for (uint32_t j = k >> 1; j > 0; j >>= 1) wave_stage<E>(K, A, lane, base, k, j);
    }
}

// The stages j = 32E .. 1 of merge size k (> 64E) of a larger bitonic
// network, on one wave's block.
template <int E>
__device__ __forceinline__ void wave_merge_tail(uint64_t (&K)[E], uint64_t (&A)[E], uint32_t lane, uint32_t base,
                                                uint32_t k) {
#pragma unroll
    for (uint32_t j = 32u * E; j > 0; j >>= 1) wave_stage<E>(K, A, lane, base, k, j);
}

// The same network on records packed into one 64-bit word: one compare and
// half the exchanges of the two-word form.
template <int E>
__device__ __forceinline__ void wave_stage1(uint64_t (&K)[E], uint32_t lane, uint32_t base, uint32_t k, uint32_t j) {
    if (j < (uint32_t)E) {
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)E; ++r) {
            if ((r & j) == 0) {
                const uint32_t r2 = r | j;
                const bool up = lane_in(~lanes_with_bit<E>(k, r, base));
                const uint64_t a = K[r], b = K[r2];
                if ((a > b) == up) { K[r] = b; K[r2] = a; }
            }
        }
    } else {
        const uint32_t lj = j / E;
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)E; ++r) {
            const uint64_t pk = xlane(K[r], lj);
            // keep the smaller when the bits j and k of the index agree
            const bool keep_min = lane_in(~(lanes_with_bit<E>(j, r, base) ^ lanes_with_bit<E>(k, r, base)));
            if ((K[r] > pk) == keep_min) K[r] = pk;
        }
    }
}
template <int E>
__device__ __forceinline__ void wave_bitonic1(uint64_t (&K)[E], uint32_t lane, uint32_t base = 0) {
#pragma unroll
    for (uint32_t k = 2; k <= 64u * E; k <<= 1) {
#pragma unroll
        for (uint32_t j = k >> 1; j > 0; j >>= 1) wave_stage1<E>(K, lane, base, k, j);
    }
}
template <int E>
__device__ __forceinline__ void wave_merge_tail1(uint64_t (&K)[E], uint32_t lane, uint32_t base, uint32_t k) {
#pragma unroll
    for (uint32_t j = 32u * E; j > 0; j >>= 1) wave_stage1<E>(K, lane, base, k, j);
}

// Bitwise OR over the 64 lanes of a wave (every lane gets the result).
__device__ __forceinline__ uint64_t wave_or64(uint64_t x) {
    x |= xlane64<1>(x);
    x |= xlane64<2>(x);
    x |= xlane64<4>(x);
    x |= xlane64<8>(x);
    x |= xlane64<16>(x);
    x |= xlane64<32>(x);
    return x;
}
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
    return (uint64_t)uniform((uint32_t)x) | (uint64_t)uniform((uint32_t)(x >> 32)) << 32;
}

// One-word sort records of a base case whose keys share their first c >= 2
// bytes: the key bits below the shared bytes, then r (4 bits), then the
// record's position in the segment (PB bits).  Keys that are equal with
// equal r are identical strings (r < 8) or a tie to refine (r = 8); either
// way the position orders them as the index does, because every
// distribution pass keeps the input order inside a bucket, and the input
// order of a segment's records is ascending in index.
__device__ __forceinline__ uint64_t shl_key(uint64_t x, uint32_t s) { return s < 64 ? x << s : 0ull; }
__device__ __forceinline__ uint64_t shr_key(uint64_t x, uint32_t s) { return s < 64 ? x >> s : 0ull; }
__device__ __forceinline__ uint64_t p1_pack(uint64_t key, uint32_t r, uint32_t pos, uint32_t sh, uint32_t pb) {
    return shl_key(key, sh) | (uint64_t)r << pb | pos;
}
// key (with the shared bytes `pre` restored), r and position of a record
__device__ __forceinline__ uint64_t p1_key(uint64_t x, uint64_t pre, uint32_t sh) {
    return pre | shr_key(x & ~0xFFFFull, sh);  // sh >= 16: the low 16 bits hold r and position
}
__device__ __forceinline__ uint32_t p1_r(uint64_t x, uint32_t pb) { return (uint32_t)(x >> pb) & 0xFu; }
// LCP contribution of the words of two one-word records (their r codes
// r1, r0) whose keys share their first c bytes (sh = 8c bits), as
// kf_lcp_word gives it for the full keys (`pre` holds the shared bytes)
__device__ __forceinline__ uint32_t p1_lcp(const KeyFmt& fh, uint64_t x1, uint32_t r1, uint64_t x0, uint32_t r0,
                                           uint32_t c, uint64_t pre, uint32_t sh) {
    if (fh.bpc) {
        const uint64_t d = (x1 ^ x0) & ~0xFFFFull;
        return d ? (sh + (uint32_t)__builtin_clzll(d)) / fh.bpc : kf_chars(fh, p1_key(x1, pre, sh));
    }
    uint32_t cb = c + common_bytes(x1 & ~0xFFFFull, x0 & ~0xFFFFull);
    cb = cb < W ? cb : W;
    cb = cb < r0 ? cb : r0;
    return cb < r1 ? cb : r1;
}
__device__ __forceinline__ uint32_t p1_pos(uint64_t x, uint32_t pb) { return (uint32_t)x & ((1u << pb) - 1); }

// One step of odd-even transposition sort over the blocked 64*E records:
// pairs (2i, 2i+1) on even steps, (2i+1, 2i+2) on odd steps, each put in
// order.  Records of different groups are already in order (groups are
// contiguous and numbered by position), so L steps sort every run of at
// most L records without disturbing anything else.
template <int E>
__device__ __forceinline__ void wave_oddeven_step(uint64_t (&K)[E], uint64_t (&A)[E], uint32_t lane, bool odd) {
    if (E == 1) {
        const uint64_t xk = __shfl_xor(K[0], 1, 64), xa = __shfl_xor(A[0], 1, 64);
        const uint64_t dk = __shfl_down(K[0], 1, 64), da = __shfl_down(A[0], 1, 64);
        const uint64_t uk = __shfl_up(K[0], 1, 64), ua = __shfl_up(A[0], 1, 64);
        bool lower, has;
        uint64_t pk, pa;
        if (!odd) {
            lower = (lane & 1) == 0; has = true; pk = xk; pa = xa;
        } else {
            lower = (lane & 1) == 1;
            has = lower ? lane < 63 : lane > 0;
            pk = lower ? dk : uk;
            pa = lower ? da : ua;
        }
        if (has) {
            const bool take = lower ? pr_gt(K[0], A[0], pk, pa) : pr_gt(pk, pa, K[0], A[0]);
            if (take) { K[0] = pk; A[0] = pa; }
        }
        return;
    }
    // neighbours across the lane boundary (old values, before any exchange)
    const uint64_t nk = __shfl_down(K[0], 1, 64), na = __shfl_down(A[0], 1, 64);
    const uint64_t pk = __shfl_up(K[E - 1], 1, 64), pa = __shfl_up(A[E - 1], 1, 64);
    if (!odd) {
#pragma unroll
        for (uint32_t r = 0; r + 1 < (uint32_t)E; r += 2) {
            if (pr_gt(K[r], A[r], K[r + 1], A[r + 1])) {
                uint64_t t = K[r]; K[r] = K[r + 1]; K[r + 1] = t;
                t = A[r]; A[r] = A[r + 1]; A[r + 1] = t;
            }
        }
    } else {
        uint64_t k0 = K[0], a0 = A[0], kl = K[E - 1], al = A[E - 1];
#pragma unroll
        for (uint32_t r = 1; r + 1 < (uint32_t)E; r += 2) {
            if (pr_gt(K[r], A[r], K[r + 1], A[r + 1])) {
                uint64_t t = K[r]; K[r] = K[r + 1]; K[r + 1] = t;
                t = A[r]; A[r] = A[r + 1]; A[r + 1] = t;
            }
        }
        if (lane < 63 && pr_gt(kl, al, nk, na)) { K[E - 1] = nk; A[E - 1] = na; }
        if (lane > 0 && pr_gt(pk, pa, k0, a0)) { K[0] = pk; A[0] = pa; }
    }
}

// A base segment's descriptor and its set's first index, in scalar
// registers, loaded before the segment is sorted (so a wave loads the next
// segment's descriptor while it sorts one).
struct BaseDesc {
    BaseSeg sg;
    uint32_t obase;
    bool ok;
};
template <int E>
__device__ __forceinline__ BaseDesc base_wave_desc(const Work& w, const Params& p, int cur, int cls, uint32_t si,
                                                   uint32_t nseg) {
    const uint32_t lane = threadIdx.x & 63;
    BaseDesc d{};
    if (si >= nseg) return d;  // uniform per wave
    const BaseSeg sg = w.base[cls][cur][si];
    d.sg = BaseSeg{uniform(sg.begin), uniform(sg.size), uniform(sg.depth), uniform(sg.rid)};
    const uint32_t m = d.sg.size;
    if (m < 2 || m > 64u * E || d.sg.begin > p.n || m > p.n - d.sg.begin) {
        if (lane == 0) raise_err(w, ERR_BOUNDS);
        return d;
    }
    d.ok = true;
    d.obase = uniform(w.set_base[d.sg.rid]);
    return d;
}
template <int E>
__device__ __forceinline__ void base_wave_recs(const Work& w, int cur, const BaseDesc& d, Rec (&x)[E]) {
    const uint32_t lane = threadIdx.x & 63;
    const Rec* src = w.rec[cur] + d.sg.begin;
#pragma unroll
    for (uint32_t r = 0; r < (uint32_t)E; ++r) {
        const uint32_t e = lane * E + r;
        x[r] = d.ok && e < d.sg.size ? src[e] : Rec{0, 0, 0};
    }
}

// Same job as k_base for a segment of at most 64*E strings: sort by
// (key, r, index), refine runs of equal full words at depth + 8 (keys
// re-gathered only for those strings), LCP of neighbours from the word at
// the depth where they separate.  Depth and LCP are kept per position
// (a run never moves), keys and records move.
template <int E, bool AC>
__device__ void dev_base_wave_run(const Work& w, const Params& p, int cur, const BaseDesc& in, const Rec (&X)[E],
                                  uint32_t si, SmWave& sm) {
    auto& LIDX = sm.LIDX;
    auto& RMIN = sm.RMIN;
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (!in.ok) return;  // uniform per wave
    const BaseSeg& sg = in.sg;
    const uint32_t m = sg.size, h = sg.depth;
    const KeyFmt fh = fmt_of<AC>(w);
    uint32_t rounds = 0;
    uint64_t K[E], A[E];
    uint32_t D[E], LV[E];
#pragma unroll
    for (uint32_t r = 0; r < (uint32_t)E; ++r) {
        const uint32_t e = lane * E + r;
        if (e < m) {
            const Rec& x = X[r];
            K[r] = rec_key(x);
            A[r] = (uint64_t)rec_r(w, x, cur, sg.begin + e) << 32 | rec_idx(w, x);
        } else {
            K[r] = ~0ull;
            A[r] = ~0ull;
        }
        D[r] = h;
        LV[r] = 0;
    }
    // bytes shared by all keys of the segment
    const uint64_t k0 = uniform64(K[0]);
    uint64_t dx = 0;
#pragma unroll
    for (uint32_t r = 0; r < (uint32_t)E; ++r)
        if (lane * E + r < m) dx |= K[r] ^ k0;
    const uint32_t c = uniform(common_bytes(wave_or64(dx), 0));
    bool presorted = false;
    if (c >= 2) {
        // one-word records; the indices wait in LDS, found by position
        constexpr uint32_t PB = E == 1 ? 6 : E == 2 ? 7 : 8;
        const uint32_t sh = 8 * c;
        uint64_t P[E];
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)E; ++r) {
            const uint32_t e = lane * E + r;
            P[r] = ~0ull;
            if (e < m) {
                LIDX[wv][e] = (uint32_t)A[r];
                P[r] = p1_pack(K[r], (uint32_t)(A[r] >> 32), e, sh, PB);
            }
        }
        wave_bitonic1<E>(P, lane);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // neighbours: equal words with r = 8 tie, else the LCP is final
        const uint64_t pre = k0 & ~shr_key(~0ull, sh);
        const uint64_t pl = __shfl_up(P[E - 1], 1, 64);
        uint32_t tb = 0;
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)E; ++r) {
            const uint32_t e = lane * E + r;
            const uint64_t q = r == 0 ? pl : P[r - 1];
            if (e > 0 && e < m) {
                const uint32_t r1 = p1_r(P[r], PB), r0 = p1_r(q, PB);
                if (((P[r] ^ q) >> PB) == 0 && r1 == W) tb |= 1u << r;
                else LV[r] = h + p1_lcp(fh, P[r], r1, q, r0, c, pre, sh);
            }
        }
        if (__ballot(tb != 0) == 0) {  // no ties: order and LCPs are final
            const uint32_t obase = in.obase;
#pragma unroll
            for (uint32_t r = 0; r < (uint32_t)E; ++r) {
                const uint32_t e = lane * E + r;
                if (e < m) {
                    p.perm[sg.begin + e] = LIDX[wv][p1_pos(P[r], PB)] - obase;
                    if (e > 0) p.lcp[sg.begin + e] = LV[r];
                }
            }
            if (lane == 0 && w.remaining) atomicSub(&w.remaining[sg.rid], m);
            return;
        }
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)E; ++r) {
            const uint32_t e = lane * E + r;
            if (e < m) {
                pr_pack(0, p1_key(P[r], pre, sh), p1_r(P[r], PB), LIDX[wv][p1_pos(P[r], PB)], K[r], A[r]);
            } else {
                K[r] = ~0ull;
                A[r] = ~0ull;
            }
        }
        // LIDX is rewritten by the refinement below
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        presorted = true;
    } else {
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)E; ++r)
            if (lane * E + r < m) pr_pack(0, K[r], (uint32_t)(A[r] >> 32), (uint32_t)A[r], K[r], A[r]);
    }
    uint32_t span = ~0u;
    for (;;) {
        if (presorted) {
            presorted = false;
        } else if (span <= (E == 1 ? 12u : 32u)) {
            for (uint32_t st = 0; st < span; ++st) wave_oddeven_step<E>(K, A, lane, (st & 1u) != 0);
        } else {
            wave_bitonic<E>(K, A, lane);
        }
        uint64_t pk0 = __shfl_up(K[E - 1], 1, 64);
        uint64_t pa0 = __shfl_up(A[E - 1], 1, 64);
        uint32_t tb = 0;
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)E; ++r) {
            const uint32_t e = lane * E + r;
            const uint64_t pk = r == 0 ? pk0 : K[r - 1];
            const uint64_t pa = r == 0 ? pa0 : A[r - 1];
            if (e > 0 && e < m && pr_grp(pk) == pr_grp(K[r])) {
                // same group: equal words with r = 8 tie, else the LCP is final
                const uint32_t r1 = pr_r(A[r]), r0 = pr_r(pa);
                if (K[r] == pk && (A[r] >> 32) == (pa >> 32) && r1 == 8) tb |= 1u << r;
                else LV[r] = D[r] + kf_lcp_word(fh, pr_key(pk, pa), r0, pr_key(K[r], A[r]), r1);
            }
        }
        if (__ballot(tb != 0) == 0) break;
        ++rounds;
        // run starts (inclusive max-scan of "tie ? 0 : position")
        uint32_t loc[E];
        uint32_t run = 0;
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)E; ++r) {
            const uint32_t e = lane * E + r;
            const uint32_t x = ((tb >> r) & 1u) ? 0u : e;
            run = run > x ? run : x;
            loc[r] = run;
        }
        uint32_t incl = wave_incl_max(run);
        uint32_t excl = __shfl_up(incl, 1, 64);
        if (lane == 0) excl = 0;
        const uint32_t tb_next_lane = __shfl_down(tb, 1, 64);
        const uint32_t next_tie = lane < 63 ? (tb_next_lane & 1u) : 0u;
        uint32_t RS[E];
        uint32_t act = 0;
        span = 0;
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)E; ++r) {
            const uint32_t e = lane * E + r;
            RS[r] = excl > loc[r] ? excl : loc[r];
            const bool t_here = (tb >> r) & 1u;
            const bool t_next = r + 1 < (uint32_t)E ? ((tb >> (r + 1)) & 1u) : next_tie;
            if (e < m && (t_here || t_next)) {
                act |= 1u << r;
                span = span > e - RS[r] + 1 ? span : e - RS[r] + 1;
            }
            if (e < m && RS[r] == e && (act >> r) & 1u) {  // run leader publishes its string
                LIDX[wv][e] = pr_idx(A[r]);
                RMIN[wv][e] = ~0u;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // common prefix of each run: members' LCP with the leader's string,
        // starting past the shared word; every string of a run
        // keeps its offset and length for the re-gather below
        uint64_t OA[E];
        uint32_t LA[E];
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)E; ++r) {
            const uint32_t e = lane * E + r;
            OA[r] = 0;
            LA[r] = 0;
            if (!((act >> r) & 1u)) continue;
            const uint32_t a = pr_idx(A[r]);
            const uint64_t oa = p.offsets[a];
            const uint32_t la = (uint32_t)(p.offsets[a + 1] - oa);
            OA[r] = oa;
            LA[r] = la;
            if (RS[r] == e) continue;
            const uint32_t b = LIDX[wv][RS[r]];
            const uint64_t ob = p.offsets[b];
            const uint32_t lb = (uint32_t)(p.offsets[b + 1] - ob);
            // (a lookahead only where the registers allow it at the kernel's occupancy)
            uint32_t l;
            if constexpr (E == 4) l = lcp_stream<4>(p.chars, oa, la, ob, lb, D[r] + kf_step(fh));
            else l = lcp_from<1>(p.chars, oa, la, ob, lb, D[r] + kf_step(fh));
            atomicMin(&RMIN[wv][RS[r]], l);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)E; ++r) {
            const uint32_t e = lane * E + r;
            if (e >= m) continue;
            const uint32_t idx = pr_idx(A[r]);
            if ((act >> r) & 1u) {
                const uint32_t d2 = RMIN[wv][RS[r]];
                D[r] = d2;
                const uint64_t key2 = fh.bpc == 0 ? gather_key(p.chars, OA[r], d2, LA[r])
                                                  : key_at_packed_call(w, p.chars, OA[r], d2, LA[r]);
                pr_pack(RS[r], key2, kf_r(fh, LA[r], d2), idx, K[r], A[r]);
            } else {
                K[r] = pr_regroup(K[r], e);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        span = wave_max(span);
    }
#pragma unroll
    for (uint32_t r = 0; r < (uint32_t)E; ++r) {
        const uint32_t e = lane * E + r;
        if (e < m) {
            p.perm[sg.begin + e] = pr_idx(A[r]) - in.obase;
            if (e > 0) p.lcp[sg.begin + e] = LV[r];
        }
    }
    if (lane == 0 && w.remaining) atomicSub(&w.remaining[sg.rid], m);
    if (lane == 0 && rounds) atomicAdd(&w.ctl->base_rounds[si % ROUND_LINES].v, rounds);
}
template <int E>
__device__ void dev_base_wave(const Work& w, const Params& p, int cur, int cls, uint32_t si, uint32_t nseg,
                              SmWave& sm) {
    const BaseDesc d = base_wave_desc<E>(w, p, cur, cls, si, nseg);
    Rec x[E];
    base_wave_recs<E>(w, cur, d, x);
    if (fmt_head(w).bpc) dev_base_wave_run<E, true>(w, p, cur, d, x, si, sm);
    else dev_base_wave_run<E, false>(w, p, cur, d, x, si, sm);
}

// Waves take segments: wave g of the launch takes segment g, then chunks
// of its XCD's part of the rest.
constexpr uint32_t BASE_WAVE_CHUNK = 4;
// The item loops of the level kernels keep values of the loop around that a
// one-item kernel would recompute; each kernel's register budget is pinned
// to the occupancy its one-item body reaches (the waves that hide the
// latency of its global loads matter more than the recomputation).
template <int E>
constexpr int base_wave_occupancy() { return E == 1 ? 7 : E == 2 ? 6 : 4; }
template <int E, bool AC>
__device__ __forceinline__ void base_wave_loop(const Work& w, const Params& p, int cur, int cls, SmWave& sm) {
    const uint32_t n = n_base_of(w, cur, cls);
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t G = gridDim.x * WAVES, g = blockIdx.x * WAVES + wv;
    const uint32_t s0 = min_u32(G, n);
    if (g >= s0) return;  // no static segment: nothing is left for this wave either
    FeedLine* f = feed_of(w, cur, FEED_BASE + cls);
    const uint32_t part = blockIdx.x % FEED_PARTS;
    uint32_t lo = g, hi = g + 1;
    for (;;) {
        // the next chunk's atomic is issued before this chunk is sorted, so
        // its round trip overlaps the work
        uint32_t nlo = 0, nhi = 0, ok = 0;
        if (lane == 0) ok = feed_take(f, s0, n, part, BASE_WAVE_CHUNK, &nlo, &nhi) ? 1u : 0u;
        BaseDesc d = base_wave_desc<E>(w, p, cur, cls, lo, n);
        for (uint32_t si = lo; si < hi; ++si) {
            Rec x[E];
            base_wave_recs<E>(w, cur, d, x);
            const BaseDesc nd = base_wave_desc<E>(w, p, cur, cls, si + 1 < hi ? si + 1 : n, n);
            dev_base_wave_run<E, AC>(w, p, cur, d, x, si, sm);
            d = nd;
        }
        ok = (uint32_t)__builtin_amdgcn_readfirstlane((int)ok);
        if (!ok) break;
        lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)nlo);
        hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)nhi);
    }
}
template <int E, bool AC>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(base_wave_occupancy<E>())))
void k_base_wave(Work w, Params p, int cur, int cls) {
    __shared__ SmWave sm;
    base_wave_loop<E, AC>(w, p, cur, cls, sm);
}

// ---------------------------------------------------------------------------
// base case: one work group per segment, records in LDS, depth refinement
// ---------------------------------------------------------------------------

// Sorts NB * 256 packed records held in LDS (hi words H, lo words L): the
// waves sort blocks of 256 in registers, then a bitonic network merges the
// blocks, its cross-block stages in LDS, its in-block stages in registers.
__device__ void lds_block_sort(uint64_t* H, uint64_t* L, uint32_t NB) {
    constexpr uint32_t E = 4, R = 64 * E;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint64_t K[E], A[E];
    for (uint32_t b = wv; b < NB; b += WAVES) {  // uniform per wave
#pragma unroll
        for (uint32_t r = 0; r < E; ++r) {
            K[r] = H[b * R + lane * E + r];
            A[r] = L[b * R + lane * E + r];
        }
        wave_bitonic<E>(K, A, lane, NB > 1 ? b * R : 0u);
#pragma unroll
        for (uint32_t r = 0; r < E; ++r) {
            H[b * R + lane * E + r] = K[r];
            L[b * R + lane * E + r] = A[r];
        }
    }
    __syncthreads();
    for (uint32_t k = 2 * R; k <= NB * R; k <<= 1) {
        for (uint32_t j = k >> 1; j >= R; j >>= 1) {
            for (uint32_t t = tid; t < NB * R / 2; t += BLOCK) {
                const uint32_t i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                const uint32_t l = i | j;
                const bool up = (i & k) == 0;
                const uint64_t hi = H[i], hl = H[l], li = L[i], ll = L[l];
                if (pr_gt(hi, li, hl, ll) == up) {
                    H[i] = hl; H[l] = hi; L[i] = ll; L[l] = li;
                }
            }
            __syncthreads();
        }
        for (uint32_t b = wv; b < NB; b += WAVES) {
#pragma unroll
            for (uint32_t r = 0; r < E; ++r) {
                K[r] = H[b * R + lane * E + r];
                A[r] = L[b * R + lane * E + r];
            }
            wave_merge_tail<E>(K, A, lane, b * R, k);
#pragma unroll
            for (uint32_t r = 0; r < E; ++r) {
                H[b * R + lane * E + r] = K[r];
                L[b * R + lane * E + r] = A[r];
            }
        }
        __syncthreads();
    }
}

// lds_block_sort on one-word records.
__device__ void lds_block_sort1(uint64_t* H, uint32_t NB) {
    constexpr uint32_t E = 4, R = 64 * E;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint64_t K[E];
    for (uint32_t b = wv; b < NB; b += WAVES) {  // uniform per wave
#pragma unroll
        for (uint32_t r = 0; r < E; ++r) K[r] = H[b * R + lane * E + r];
        wave_bitonic1<E>(K, lane, NB > 1 ? b * R : 0u);
#pragma unroll
        for (uint32_t r = 0; r < E; ++r) H[b * R + lane * E + r] = K[r];
    }
    __syncthreads();
    for (uint32_t k = 2 * R; k <= NB * R; k <<= 1) {
        for (uint32_t j = k >> 1; j >= R; j >>= 1) {
            for (uint32_t t = tid; t < NB * R / 2; t += BLOCK) {
                const uint32_t i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                const uint32_t l = i | j;
                const bool up = (i & k) == 0;
                const uint64_t a = H[i], b = H[l];
                if ((a > b) == up) { H[i] = b; H[l] = a; }
            }
            __syncthreads();
        }
        for (uint32_t b = wv; b < NB; b += WAVES) {
#pragma unroll
            for (uint32_t r = 0; r < E; ++r) K[r] = H[b * R + lane * E + r];
            wave_merge_tail1<E>(K, lane, b * R, k);
#pragma unroll
            for (uint32_t r = 0; r < E; ++r) H[b * R + lane * E + r] = K[r];
        }
        __syncthreads();
    }
}

// Sorts a segment of m <= BASE_CAP strings with common prefix h by
// (key, r, index).  Runs of equal full words are then refined at depth
// h+8, h+16, ... inside LDS (keys re-gathered for those strings only).
// LCPs of neighbours separated at depth d are d plus the common bytes of
// their words at d (the "last compared word"); the role of LCP-insertion
// sort (Algorithm 4.6) as the paper's base case.
template <bool AC>
__device__ void dev_base_wg(const Work& w, const Params& p, int cur, uint32_t item, uint32_t nseg, SmBase& sm) {
    uint64_t* K = sm.K;
    uint64_t* A = sm.A;
    uint32_t* dep = sm.dep;
    uint32_t* lv = sm.lv;
    uint32_t* aux = sm.aux;
    uint32_t* rmin = sm.rmin;
    uint32_t* wtot = sm.wtot;
    uint32_t& any = sm.any;
    constexpr uint32_t PER = BASE_CAP / BLOCK;

    if (item >= nseg) return;  // uniform
    const BaseSeg sg = w.base[CLS_WG][cur][item];
    const uint32_t tid = threadIdx.x, m = sg.size, h = sg.depth;
    const KeyFmt fh = fmt_of<AC>(w);
    uint32_t rounds = 0;
    if (m < 2 || m > BASE_CAP || m > p.base_max || sg.begin > p.n || m > p.n - sg.begin) {  // uniform
        if (tid == 0) raise_err(w, ERR_BOUNDS);
        return;
    }
    uint32_t P = 256;  // whole blocks of the block sort
    while (P < m) P <<= 1;
    const Rec* in = w.rec[cur] + sg.begin;
    // keys and (r, index) first; the bytes all keys share decide the record form
    const uint64_t k0 = rec_key(in[0]);
    uint64_t dx = 0;
    for (uint32_t i = tid; i < P; i += BLOCK) {
        if (i < m) {
            const Rec x = in[i];
            K[i] = rec_key(x);
            A[i] = (uint64_t)rec_r(w, x, cur, sg.begin + i) << 32 | rec_idx(w, x);
            dx |= K[i] ^ k0;
        } else {
            K[i] = ~0ull;
            A[i] = ~0ull;
        }
        dep[i] = h;
        lv[i] = 0;
    }
    dx = wave_or64(dx);
    if ((tid & 63) == 0) {  // rmin is free until the refinement
        rmin[2 * (tid >> 6)] = (uint32_t)dx;
        rmin[2 * (tid >> 6) + 1] = (uint32_t)(dx >> 32);
    }
    __syncthreads();
    dx = 0;
#pragma unroll
    for (uint32_t q = 0; q < WAVES; ++q) dx |= (uint64_t)rmin[2 * q] | (uint64_t)rmin[2 * q + 1] << 32;
    const uint32_t c = common_bytes(dx, 0);
    bool presorted = false;
    if (c >= 2) {
        // one-word records; the indices wait in aux, found by position
        constexpr uint32_t PB = 10;
        static_assert(BASE_CAP <= (1u << PB) && PB + 4 <= 16, "one-word base records");
        const uint32_t sh = 8 * c;
        for (uint32_t i = tid; i < m; i += BLOCK) {
            aux[i] = (uint32_t)A[i];
            K[i] = p1_pack(K[i], (uint32_t)(A[i] >> 32), i, sh, PB);
        }
        if (tid == 0) any = 0;
        __syncthreads();
        lds_block_sort1(K, P / 256);
        const uint64_t pre = k0 & ~shr_key(~0ull, sh);
        for (uint32_t i = tid + 1; i < m; i += BLOCK) {
            const uint64_t x = K[i], q = K[i - 1];
            const uint32_t r1 = p1_r(x, PB), r0 = p1_r(q, PB);
            if (((x ^ q) >> PB) == 0 && r1 == W) any = 1;
            else lv[i] = h + p1_lcp(fh, x, r1, q, r0, c, pre, sh);
        }
        __syncthreads();
        if (!any) {  // no ties: order and LCPs are final
            const uint32_t obase = w.set_base[sg.rid];
            for (uint32_t i = tid; i < m; i += BLOCK) {
                p.perm[sg.begin + i] = aux[p1_pos(K[i], PB)] - obase;
                if (i > 0) p.lcp[sg.begin + i] = lv[i];
            }
            if (tid == 0 && w.remaining) atomicSub(&w.remaining[sg.rid], m);
            return;
        }
        for (uint32_t i = tid; i < m; i += BLOCK) {
            const uint64_t x = K[i];
            pr_pack(0, p1_key(x, pre, sh), p1_r(x, PB), aux[p1_pos(x, PB)], K[i], A[i]);
        }
        presorted = true;
    } else {
        for (uint32_t i = tid; i < m; i += BLOCK)
            pr_pack(0, K[i], (uint32_t)(A[i] >> 32), (uint32_t)A[i], K[i], A[i]);
    }
    __syncthreads();

    for (;;) {
        if (tid == 0) any = 0;
        if (presorted) presorted = false;
        else lds_block_sort(K, A, P / 256);
        // neighbours inside a group: tie (equal full word, refine) or split
        for (uint32_t i = tid; i < m; i += BLOCK) {
            uint32_t t = 0;
            if (i > 0) {
                const uint64_t a1 = A[i], a0 = A[i - 1], k1 = K[i], k0 = K[i - 1];
                if (pr_grp(k1) == pr_grp(k0)) {
                    const uint32_t r1 = pr_r(a1), r0 = pr_r(a0);
                    if (k1 == k0 && (a1 >> 32) == (a0 >> 32) && r1 == 8) t = 1;
                    else lv[i] = dep[i] + kf_lcp_word(fh, pr_key(k0, a0), r0, pr_key(k1, a1), r1);
                }
            }
            aux[i] = t << 31;
            if (t) any = 1;
        }
        __syncthreads();
        if (!any) break;
        ++rounds;
        // run starts: inclusive max-scan of (tie ? 0 : position)
        {
            const uint32_t base = tid * PER;
            uint32_t loc[PER];
            uint32_t run = 0;
#pragma unroll
            for (uint32_t e = 0; e < PER; ++e) {
                uint32_t i = base + e;
                uint32_t x = (i < m && !(aux[i] >> 31)) ? i : 0u;
                run = run > x ? run : x;
                loc[e] = run;
            }
            uint32_t incl = wave_incl_max(run);
            uint32_t excl = __shfl_up(incl, 1, 64);
            if ((tid & 63) == 0) excl = 0;
            if ((tid & 63) == 63) wtot[tid >> 6] = incl;
            __syncthreads();
            for (uint32_t q = 0; q < (tid >> 6); ++q) excl = excl > wtot[q] ? excl : wtot[q];
#pragma unroll
            for (uint32_t e = 0; e < PER; ++e) {
                uint32_t i = base + e;
                if (i < m) {
                    aux[i] = (aux[i] & 0x80000000u) | (excl > loc[e] ? excl : loc[e]);
                    rmin[i] = ~0u;
                }
            }
        }
        __syncthreads();
        // common prefix of each run: every member's LCP with the run's first
        // string (all members agree on the word at their depth, so the
        // comparison starts 8 characters further)
        for (uint32_t i = tid; i < m; i += BLOCK) {
            const uint32_t ai = aux[i];
            const bool act = (ai >> 31) || (i + 1 < m && (aux[i + 1] >> 31));
            const uint32_t rs = ai & 0x7FFFFFFFu;
            if (act && rs != i) {
                const uint32_t a = pr_idx(A[i]), b = pr_idx(A[rs]);
                const uint64_t oa = p.offsets[a], ob = p.offsets[b];
                const uint32_t la = (uint32_t)(p.offsets[a + 1] - oa), lb = (uint32_t)(p.offsets[b + 1] - ob);
                atomicMin(&rmin[rs], lcp_stream<8>(p.chars, oa, la, ob, lb, dep[i] + kf_step(fh)));
            }
        }
        __syncthreads();
        // strings of a run move on to the run's common prefix
        for (uint32_t i = tid; i < m; i += BLOCK) {
            const uint32_t ai = aux[i];
            const bool act = (ai >> 31) || (i + 1 < m && (aux[i + 1] >> 31));
            const uint32_t idx = pr_idx(A[i]);
            if (act) {
                const uint32_t rs = ai & 0x7FFFFFFFu;
                const uint32_t d2 = rmin[rs];
                dep[i] = d2;
                const uint64_t o0 = p.offsets[idx], o1 = p.offsets[idx + 1];
                const uint32_t len = (uint32_t)(o1 - o0);
                const uint64_t key2 = fh.bpc == 0 ? gather_key(p.chars, o0, d2, len)
                                                  : key_at_packed_call(w, p.chars, o0, d2, len);
                pr_pack(rs, key2, kf_r(fh, len, d2), idx, K[i], A[i]);
            } else {
                K[i] = pr_regroup(K[i], i);
            }
        }
        __syncthreads();
    }
    const uint32_t obase = w.set_base[sg.rid];
    for (uint32_t i = tid; i < m; i += BLOCK) {
        p.perm[sg.begin + i] = pr_idx(A[i]) - obase;
        if (i > 0) p.lcp[sg.begin + i] = lv[i];
    }
    if (tid == 0 && w.remaining) atomicSub(&w.remaining[sg.rid], m);
    if (tid == 0 && rounds) atomicAdd(&w.ctl->base_rounds[item % ROUND_LINES].v, rounds);
}

// Work groups take segments: group b takes segment b, then segments of its
// XCD's part of the rest.
template <bool AC>
__device__ __forceinline__ void base_wg_loop(const Work& w, const Params& p, int cur, SmBase& sm) {
    uint32_t& s_item = sm.wtot[0];  // item mailbox: wtot is first written after the body's first barrier
    const uint32_t n = n_base_of(w, cur, CLS_WG);
    const uint32_t s0 = min_u32(gridDim.x, n);
    FeedLine* f = feed_of(w, cur, FEED_BASE + CLS_WG);
    uint32_t item = blockIdx.x < s0 ? blockIdx.x : n;
    while (item < n) {
        uint32_t nxt = n;
        if (threadIdx.x == 0) nxt = feed_one(f, s0, n, blockIdx.x % FEED_PARTS);  // overlaps the work
        dev_base_wg<AC>(w, p, cur, item, n, sm);
        __syncthreads();
        if (threadIdx.x == 0) s_item = nxt;
        __syncthreads();
        item = uniform(s_item);
    }
}
template <bool AC>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_base(Work w, Params p, int cur) {
    __shared__ SmBase sm;
    base_wg_loop<AC>(w, p, cur, sm);
}


// ---------------------------------------------------------------------------
// distribution step: sample + splitter tree
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool kr_gt(uint64_t ka, uint32_t ra, uint64_t kb, uint32_t rb) {
    return ka > kb || (ka == kb && ra > rb);
}

// A sorted sample's r code (bits 0..7) and sample number (bits 8..18;
// a < 2^11); padding is all ones.  Comparisons see the r code only
// (SampleR).  A chosen splitter adds the number of samples equal to it
// (bits 19..31).
static_assert((2u << MAX_LOGV) <= (1u << 11), "sample numbers fit 11 bits");
__device__ __forceinline__ uint32_t sr_word(uint64_t lo) {
    return lo == ~0ull ? 0xFFFFFFFFu : pr_r(lo) | pr_idx(lo) << 8;
}
struct SampleR {
    const uint32_t* s;
    __device__ uint32_t operator[](uint32_t i) const { return s[i] & 0xFFu; }
};

// The regular sample of a segment (a = 2v+1 keys at evenly spaced
// positions) sorted by (key, r) into SK / SR, padded with maxima to a power
// of two.  The NB blocks of 64E records are sorted in registers by the
// waves (block b by wave b mod WAVES); with several blocks they are merged
// by a bitonic network whose cross-block stages go through LDS and whose
// in-block stages run in registers again.
template <int E>
__device__ __forceinline__ void sample_sort(const Work& w, const Params& p, int cur, const Seg& sg, uint32_t a,
                                            uint32_t NB, bool root_keys, SmSample& sm) {
    constexpr uint32_t R = 64u * E;  // records per block
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const Rec* in = w.rec[cur];
    uint64_t K[E], A[E];
    for (uint32_t b = wv; b < NB; b += WAVES) {  // uniform per wave
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)E; ++r) {
            const uint32_t j = b * R + lane * E + r;
            K[r] = ~0ull;
            A[r] = ~0ull;
            if (j < a) {
                const uint32_t pos = sg.begin + (uint32_t)(((2ull * j + 1) * sg.size) / (2ull * a));
                uint64_t key;
                uint32_t rr;
                if (root_keys) {  // a root segment: position = string, depth 0, key read as k_init does
                    const uint64_t o0 = p.offsets[pos], o1 = p.offsets[pos + 1];
                    const bool bad = o1 < o0 || o1 - o0 > MAX_LEN || (o1 > o0 && p.chars == nullptr);
                    const uint32_t len = bad ? 0u : (uint32_t)(o1 - o0);
                    const KeyFmt fh = fmt_full(w);  // beside the key gather, which publishes the format
                    key = key_at(w, fh, p.chars, o0, 0, len);
                    rr = kf_r(fh, len, 0);
                } else if (sg.regather) {  // records of an earlier depth: read the key at sg.depth
                    const KeyFmt fh = fmt_full(w);
                    const uint32_t idx = rec_idx(w, in[pos]);
                    const uint64_t o0 = p.offsets[idx], o1 = p.offsets[idx + 1];
                    const uint32_t len = (uint32_t)(o1 - o0);
                    key = key_at(w, fh, p.chars, o0, sg.depth, len);
                    rr = kf_r(fh, len, sg.depth);
                } else {
                    const Rec x = in[pos];
                    key = rec_key(x);
                    rr = rec_r(w, x, cur, pos);
                }
                pr_pack(0, key, rr, j, K[r], A[r]);
            }
        }
        wave_bitonic<E>(K, A, lane, NB > 1 ? b * R : 0u);
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)E; ++r) {
            const uint32_t j = b * R + lane * E + r;
            if (NB == 1) {
                sm.SK[j] = pr_key(K[r], A[r]);
                sm.SR[j] = sr_word(A[r]);
            } else {
                sm.SK[j] = K[r];
                sm.SA[j] = A[r];
            }
        }
    }
    __syncthreads();
    if (NB == 1) return;
    for (uint32_t k = 2 * R; k <= NB * R; k <<= 1) {
        // cross-block stages (k, j >= R) over all NB*R records in LDS
        for (uint32_t j = k >> 1; j >= R; j >>= 1) {
            for (uint32_t t = tid; t < NB * R / 2; t += BLOCK) {
                const uint32_t i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                const uint32_t l = i | j;
                const bool up = (i & k) == 0;
                const uint64_t ki = sm.SK[i], kl = sm.SK[l], ai = sm.SA[i], al = sm.SA[l];
                if (pr_gt(ki, ai, kl, al) == up) {
                    sm.SK[i] = kl; sm.SK[l] = ki; sm.SA[i] = al; sm.SA[l] = ai;
                }
            }
            __syncthreads();
        }
        // in-block stages: each wave on its own blocks
        const bool last = k == NB * R;
        for (uint32_t b = wv; b < NB; b += WAVES) {
#pragma unroll
            for (uint32_t r = 0; r < (uint32_t)E; ++r) {
                const uint32_t j = b * R + lane * E + r;
                K[r] = sm.SK[j];
                A[r] = sm.SA[j];
            }
            wave_merge_tail<E>(K, A, lane, b * R, k);
#pragma unroll
            for (uint32_t r = 0; r < (uint32_t)E; ++r) {
                const uint32_t j = b * R + lane * E + r;
                if (last) {
                    sm.SK[j] = pr_key(K[r], A[r]);
                    sm.SR[j] = sr_word(A[r]);
                } else {
                    sm.SK[j] = K[r];
                    sm.SA[j] = A[r];
                }
            }
        }
        __syncthreads();
    }
}

// The sampling step of Algorithm 4.1: a regular sample of alpha(v+1)-1 keys (alpha =
// 2) is sorted (sample_sort); splitters are chosen by recursive middle selection
// skipping duplicates (section 4.2.2, "Sampling"), level by level, directly
// into the level-order tree; an empty sub-range repeats its parent's
// splitter so the in-order splitter sequence stays sorted.  With
// root_keys the segments are roots and their sample keys are read from the
// strings themselves, so the step need not wait for the key gather.
__device__ void dev_sample(const Work& w, const Params& p, int cur, uint32_t item, bool root_keys, SmSample& sm) {
    uint64_t* SK = sm.SK;
    uint32_t* SR = sm.SR;
    uint64_t* TK = sm.TK;
    uint32_t* TR = sm.TR;
    uint16_t* NL = sm.NL;
    uint16_t* NH = sm.NH;
    const Seg sg = w.dist[cur][item];
    const uint32_t tid = threadIdx.x, d = sg.logv;
    if (d < 1 || d > MAX_LOGV || sg.begin > p.n || sg.size > p.n - sg.begin || sg.size < (4u << d)) {
        if (tid == 0) raise_err(w, ERR_BOUNDS);
        return;
    }
    const uint32_t v = (1u << d) - 1, a = 2 * v + 1, P = 2u << d;
    {
        const uint32_t T = (sg.size + TILE - 1) / TILE;
        uint32_t* ts = w.tile_seg[cur] + sg.tile_off;
        for (uint32_t t = tid; t < T; t += BLOCK) ts[t] = item;
    }
    // blocks of 256 records (the last padded); P <= 2^(MAX_LOGV+1) = 8 blocks
    sample_sort<4>(w, p, cur, sg, a, P > 256 ? P / 256 : 1u, root_keys && sg.depth == 0, sm);
    if (tid == 0) { NL[1] = 0; NH[1] = (uint16_t)a; }
    __syncthreads();
    for (uint32_t L = 0; L < d; ++L) {
        for (uint32_t q = (1u << L) + tid; q < (2u << L); q += BLOCK) {
            uint32_t lo = NL[q], hi = NH[q];
            uint32_t llo = 0, lhi = 0, rlo = 0, rhi = 0;
            if (lo < hi) {
                uint32_t mid, lh, rl;
                select_node(SK, SampleR{SR}, lo, hi, &mid, &lh, &rl);
                TK[q] = SK[mid];
                TR[q] = (SR[mid] & 0x7FFFFu) | min_u32(rl - lh, 0x1FFFu) << 19;  // + samples equal to it
                llo = lo; lhi = lh; rlo = rl; rhi = hi;
            } else {
                TK[q] = TK[q >> 1];
                TR[q] = TR[q >> 1];
            }
            if (L + 1 < d) {
                NL[2 * q] = (uint16_t)llo; NH[2 * q] = (uint16_t)lhi;
                NL[2 * q + 1] = (uint16_t)rlo; NH[2 * q + 1] = (uint16_t)rhi;
            }
        }
        __syncthreads();
    }
    uint64_t* tk = w.tree_key[cur] + sg.tree_off;
    uint8_t* tr = w.tree_r[cur] + sg.tree_off;
    uint64_t* tn = w.tree_next[cur] + sg.tree_off;
    uint32_t* tdf = w.tree_diff[cur] + sg.tree_off;
    const bool roots = root_keys && sg.depth == 0;
    const KeyFmt fh = fmt_full(w);
    const uint32_t h1 = sg.depth + kf_step(fh);
    for (uint32_t q = 1 + tid; q <= v; q += BLOCK) {
        tk[q - 1] = TK[q];
        // The splitter's sample string is a member of its equality bucket
        // (same key and r code); its key one word deeper is what the
        // scatter compares the members' next keys with.  Only for buckets
        // the sample suggests are large (a bucket of more than base_max
        // strings holds about 16 or more of the samples) and a sample
        // string that goes on for a whole word there; the others are not
        // candidates for the skip (TR_SKIP clear) and cost the scatter
        // nothing.
        uint32_t code = TR[q] & 0xFFu;
        if (code == W && (TR[q] >> 19) >= SKIP_MIN_SAMPLES) {
            const uint32_t j = (TR[q] >> 8) & 0x7FFu;
            const uint32_t pos = sg.begin + (uint32_t)(((2ull * j + 1) * sg.size) / (2ull * a));
            const uint32_t idx = roots ? pos : rec_idx(w, w.rec[cur][pos]);
            const uint64_t o0 = p.offsets[idx], o1 = p.offsets[idx + 1];
            const uint32_t len = (uint32_t)(o1 - o0);
            if (kf_r(fh, len, h1) == W) {
                tn[q - 1] = key_at(w, fh, p.chars, o0, h1, len);
                tdf[q - 1] = 0;
                code |= TR_SKIP;
            }
        }
        tr[q - 1] = (uint8_t)code;
    }
}

__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_sample(Work w, Params p, int cur, int root_keys) {
    __shared__ SmSample sm;
    const uint32_t n = n_dist_of(w, cur);
    for (uint32_t item = blockIdx.x; item < n; item += gridDim.x) {
        __syncthreads();
        dev_sample(w, p, cur, item, root_keys != 0, sm);
    }
}

// ---------------------------------------------------------------------------
// distribution step: classification and tile histograms
// ---------------------------------------------------------------------------

struct TreeView {
    const uint64_t* k;
    const uint32_t* r;
};

// The classification and counting steps of Algorithm 4.1 for one tile (Theorem 4.4: every tile keeps its
// own bucket counters): each string's bucket is stored in the oracle array
// `bkt`, the tile's 2v+1 counts go to the counter pool in bucket-major
// order (bucket b of tile t of segment s at cnt_off + b*T + t).
__device__ void dev_classify(const Work& w, const Params& p, int cur, uint32_t t, uint32_t n_dist,
                             SmClassify& sm) {
    uint64_t* TK = sm.TK;
    uint32_t* TR = sm.TR;
    uint32_t* H = sm.H;
    const uint32_t tid = threadIdx.x;
    const uint32_t si = w.tile_seg[cur][t];
    if (si >= n_dist) {
        if (tid == 0) raise_err(w, ERR_BOUNDS);
        return;
    }
    const Seg sg = w.dist[cur][si];
    const uint32_t d = sg.logv, v = (1u << d) - 1, k = 2 * v + 1;
    const uint32_t T = (sg.size + TILE - 1) / TILE;
    const uint32_t ti = t - sg.tile_off;
    if (d < 1 || d > MAX_LOGV || ti >= T || sg.begin > p.n || sg.size > p.n - sg.begin) {
        if (tid == 0) raise_err(w, ERR_BOUNDS);
        return;
    }
    const uint32_t start = sg.begin + ti * TILE;
    const uint32_t end = min_u32(start + TILE, sg.begin + sg.size);
    const uint64_t* gk = w.tree_key[cur] + sg.tree_off;
    const uint8_t* gr = w.tree_r[cur] + sg.tree_off;
    for (uint32_t q = 1 + tid; q <= v; q += BLOCK) { TK[q] = gk[q - 1]; TR[q] = gr[q - 1] & TR_CODE; }
    for (uint32_t b = tid; b < k; b += BLOCK) H[b] = 0;
    __syncthreads();
    const Rec* in = w.rec[cur];
    if (sg.regather) {  // an equality bucket that skipped a word: its keys at sg.depth, read
                        // back below by the same thread (the scatter moves the new keys)
        const KeyFmt fh = fmt_head(w);
        if (fh.bpc == 0) {
            constexpr uint32_t G = 4;  // gathers in flight per thread
            for (uint32_t i0 = start + tid; i0 < end; i0 += G * BLOCK) {
                uint32_t idx[G], len[G];
                uint64_t o0[G];
#pragma unroll
                for (uint32_t u = 0; u < G; ++u) idx[u] = i0 + u * BLOCK < end ? rec_idx(w, in[i0 + u * BLOCK]) : 0u;
#pragma unroll
                for (uint32_t u = 0; u < G; ++u) {
                    o0[u] = p.offsets[idx[u]];
                    len[u] = (uint32_t)(p.offsets[idx[u] + 1] - o0[u]);
                }
#pragma unroll
                for (uint32_t u = 0; u < G; ++u) {
                    const uint32_t i = i0 + u * BLOCK;
                    const uint64_t key = gather_key(p.chars, o0[u], sg.depth, len[u]);
                    if (i < end) rec_put(w, cur, i, key, idx[u], kf_r(fh, len[u], sg.depth));
                }
            }
        } else {
            for (uint32_t i = start + tid; i < end; i += BLOCK) {
                const uint32_t idx = rec_idx(w, in[i]);
                uint64_t key;
                uint32_t r;
                regather(w, fh, p, idx, sg.depth, key, r);
                rec_put(w, cur, i, key, idx, r);
            }
        }
    }
    constexpr uint32_t U = 4;  // strings per thread and step, descents interleaved
    for (uint32_t i0 = start + tid; i0 < end; i0 += U * BLOCK) {
        uint64_t c[U];
        uint32_t cr[U], b[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t i = i0 + u * BLOCK;
            c[u] = 0;
            cr[u] = 0;
            if (i < end) {
                const Rec x = in[i];
                c[u] = rec_key(x);
                cr[u] = rec_r(w, x, cur, i);
            }
        }
        classify_n<U>(c, cr, TK, TR, d, b);
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t i = i0 + u * BLOCK;
            if (i < end) {
                w.bkt[i] = (uint16_t)b[u];
                atomicAdd(&H[b[u]], 1u);
            }
        }
    }
    __syncthreads();
    uint32_t* c = w.cnt[cur] + sg.cnt_off + ti;
    for (uint32_t b = tid; b < k; b += BLOCK) c[(size_t)b * T] = H[b];
}

// Work groups take tiles from their XCD's part of the level's tiles.
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8))) void k_classify(Work w, Params p, int cur) {
    __shared__ SmClassify sm;
    uint32_t& s_t = sm.TR[0];  // tile mailbox: the tree is one-based, TR[0] is never used
    const uint32_t n_dist = n_dist_of(w, cur);
    const uint32_t n_tiles = n_tiles_of(w, cur);
    FeedLine* f = feed_of(w, cur, FEED_CLASSIFY);
    const uint32_t s0 = min_u32(gridDim.x, n_tiles);
    uint32_t t = blockIdx.x < s0 ? xcd_item(blockIdx.x, s0) : n_tiles;
    while (t < n_tiles) {
        uint32_t nxt = n_tiles;
        if (threadIdx.x == 0) nxt = feed_one(f, s0, n_tiles, blockIdx.x % FEED_PARTS);  // overlaps the work
        dev_classify(w, p, cur, t, n_dist, sm);
        __syncthreads();
        if (threadIdx.x == 0) s_t = nxt;
        __syncthreads();
        t = uniform(s_t);
    }
}

// ---------------------------------------------------------------------------
// exclusive scan over the counter pool ("interleaved global prefix sum",
// Theorem 4.4)
// ---------------------------------------------------------------------------

__device__ void dev_scan_reduce(const uint32_t* x, uint32_t n, uint32_t* partial, uint32_t blk, SmScan& sm) {
    const uint32_t base = blk * SCAN_CHUNK;
    uint32_t s = 0;
    for (uint32_t i = base + threadIdx.x; i < n && i < base + SCAN_CHUNK; i += BLOCK) s += x[i];
    s = wave_incl_sum(s);
    if ((threadIdx.x & 63) == 63) sm.wt[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (uint32_t q = 0; q < WAVES; ++q) t += sm.wt[q];
        partial[blk] = t;
    }
}

// exclusive scan of the per-chunk sums by one work group of any size
__device__ void dev_scan_partials(uint32_t* partial, uint32_t nb, SmScan& sm) {
    const uint32_t nt = blockDim.x, nw = nt >> 6;
    if (threadIdx.x == 0) sm.carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < nb; base += nt) {
        uint32_t i = base + threadIdx.x;
        uint32_t x = i < nb ? partial[i] : 0u;
        uint32_t incl = wave_incl_sum(x);
        if ((threadIdx.x & 63) == 63) sm.wt[threadIdx.x >> 6] = incl;
        __syncthreads();
        uint32_t off = sm.carry;
        for (uint32_t q = 0; q < (threadIdx.x >> 6); ++q) off += sm.wt[q];
        if (i < nb) partial[i] = off + incl - x;
        __syncthreads();
        if (threadIdx.x == nt - 1) sm.carry = off + incl;
        __syncthreads();
    }
    (void)nw;
}

// The chunk moves between HBM and LDS in coalesced rows (thread t holds
// elements t, t + BLOCK, ...); each thread scans 16 consecutive elements
// out of LDS.
__device__ void dev_scan_down(uint32_t* x, uint32_t n, const uint32_t* partial, uint32_t blk, SmScan& sm) {
    const uint32_t tid = threadIdx.x, b0 = blk * SCAN_CHUNK;
    auto at = [](uint32_t i) { return i + (i >> 5); };
#pragma unroll
    for (uint32_t e = 0; e < SCAN_PER_THREAD; ++e) {
        const uint32_t i = e * BLOCK + tid;
        sm.t[at(i)] = b0 + i < n ? x[b0 + i] : 0u;
    }
    __syncthreads();
    uint32_t v[SCAN_PER_THREAD];
    uint32_t s = 0;
#pragma unroll
    for (uint32_t e = 0; e < SCAN_PER_THREAD; ++e) {
        v[e] = sm.t[at(tid * SCAN_PER_THREAD + e)];
        s += v[e];
    }
    const uint32_t incl = wave_incl_sum(s);
    if ((tid & 63) == 63) sm.wt[tid >> 6] = incl;
    __syncthreads();
    uint32_t off = partial[blk] + incl - s;
    for (uint32_t q = 0; q < (tid >> 6); ++q) off += sm.wt[q];
#pragma unroll
    for (uint32_t e = 0; e < SCAN_PER_THREAD; ++e) {
        sm.t[at(tid * SCAN_PER_THREAD + e)] = off;
        off += v[e];
    }
    __syncthreads();
#pragma unroll
    for (uint32_t e = 0; e < SCAN_PER_THREAD; ++e) {
        const uint32_t i = e * BLOCK + tid;
        if (b0 + i < n) x[b0 + i] = sm.t[at(i)];
    }
}

__global__ __launch_bounds__(BLOCK) void k_scan_reduce(Work w, int cur) {
    __shared__ SmScan sm;
    const uint32_t n = n_cnt_of(w, cur), nb = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    for (uint32_t b = blockIdx.x; b < nb; b += gridDim.x) {
        __syncthreads();
        dev_scan_reduce(w.cnt[cur], n, w.partial, b, sm);
    }
}
__global__ __launch_bounds__(1024) void k_scan_partials(Work w, int cur) {
    __shared__ SmScan sm;
    const uint32_t n = n_cnt_of(w, cur);
    if (n) dev_scan_partials(w.partial, (n + SCAN_CHUNK - 1) / SCAN_CHUNK, sm);
}
__global__ __launch_bounds__(BLOCK) void k_scan_down(Work w, int cur) {
    __shared__ SmScan sm;
    const uint32_t n = n_cnt_of(w, cur), nb = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    for (uint32_t b = blockIdx.x; b < nb; b += gridDim.x) {
        __syncthreads();
        dev_scan_down(w.cnt[cur], n, w.partial, b, sm);
    }
}

// ---------------------------------------------------------------------------
// distribution step: stable scatter
// ---------------------------------------------------------------------------

// The distribution step of Algorithm 4.1 for one tile, out of place into the other buffer
// (section 4.2.8, "Out-of-place Redistribution").  Each wave owns a
// contiguous quarter of the tile; within a wave, strings with the same
// bucket are ranked by lane order through a ballot-built peer mask, so the
// scatter keeps input order inside every bucket (stable).  Strings of an
// equality bucket whose splitter ends inside the word are identical and
// final: they are written to perm/lcp directly.  Strings of the other
// equality buckets get their next key (depth + 8) on the way.
__device__ void dev_scatter(const Work& w, const Params& p, int cur, uint32_t t, uint32_t n_dist,
                            SmScatter& sm) {
    auto& WC = sm.WC;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint32_t si = w.tile_seg[cur][t];
    if (si >= n_dist) {
        if (tid == 0) raise_err(w, ERR_BOUNDS);
        return;
    }
    const Seg sg = w.dist[cur][si];
    const uint32_t d = sg.logv, v = (1u << d) - 1, k = 2 * v + 1;
    const uint32_t T = (sg.size + TILE - 1) / TILE;
    const uint32_t ti = t - sg.tile_off;
    if (d < 1 || d > MAX_LOGV || ti >= T || sg.begin > p.n || sg.size > p.n - sg.begin) {
        if (tid == 0) raise_err(w, ERR_BOUNDS);
        return;
    }
    const uint32_t start = sg.begin + ti * TILE;
    const uint32_t end = min_u32(start + TILE, sg.begin + sg.size);
    for (uint32_t b = tid; b < k; b += BLOCK) {
#pragma unroll
        for (uint32_t q = 0; q < WAVES; ++q) WC[q][b] = 0;
    }
    const uint8_t* gr = w.tree_r[cur] + sg.tree_off;
    __syncthreads();

    // phase 1: ranks within the wave's chunk
    constexpr uint32_t CH = TILE / WAVES;
    const uint32_t cbeg = start + wv * CH;
    uint32_t rank2[IPT / 2];  // two 16-bit ranks per register (bucket ids are re-read in phase 3)
#pragma unroll
    for (uint32_t it = 0; it < IPT; ++it) {
        uint32_t i = cbeg + it * 64 + lane;
        bool valid = i < end;
        uint32_t b = valid ? (uint32_t)w.bkt[i] : 0u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (uint32_t bit = 0; bit < MAX_LOGV + 1; ++bit) {
            uint64_t m = __ballot((b >> bit) & 1u);
            peers &= ((b >> bit) & 1u) ? m : ~m;
        }
        uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(peers >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
        uint32_t leader = valid ? (uint32_t)__builtin_ctzll(peers) : 0u;
        uint32_t old = 0;
        if (valid && lane == leader) old = atomicAdd(&WC[wv][b], (uint32_t)__builtin_popcountll(peers));
        old = __shfl(old, (int)leader, 64);
        const uint32_t rk = old + below;
        if (it & 1) rank2[it >> 1] |= rk << 16;
        else rank2[it >> 1] = rk;
    }
    __syncthreads();
    // phase 2: absolute write base of every (wave, bucket) of the tile
    const uint32_t* sc = w.cnt[cur] + sg.cnt_off;
    const uint32_t s0 = sc[0];
    for (uint32_t b = tid; b < k; b += BLOCK) {
        uint32_t run = sg.begin + sc[(size_t)b * T + ti] - s0;
#pragma unroll
        for (uint32_t q = 0; q < WAVES; ++q) {
            const uint32_t c = WC[q][b];
            WC[q][b] = run;
            run += c;
        }
    }
    __syncthreads();
    // phase 3: move
    const Rec* in = w.rec[cur];
    const uint32_t seg_end = sg.begin + sg.size;
    const uint32_t obase = w.set_base[sg.rid];
#pragma unroll 4
    for (uint32_t it = 0; it < IPT; ++it) {
        const uint32_t i = cbeg + it * 64 + lane;
        if (i >= end) continue;
        const Rec x = in[i];
        uint64_t key = rec_key(x);
        const uint32_t idx = rec_idx(w, x);
        uint32_t rr = rec_r(w, x, cur, i);
        const uint32_t b = w.bkt[i], rank = (rank2[it >> 1] >> (16 * (it & 1))) & 0xFFFFu;
        const uint32_t pos = WC[wv][b] + rank;
        if (pos < sg.begin || pos >= seg_end) { raise_err(w, ERR_BOUNDS); continue; }
        if (b & 1u) {
            const uint32_t lx = level_index(b >> 1, d) - 1;
            const uint32_t rx = gr[lx] & TR_CODE;
            const KeyFmt fh = fmt_head(w);
            if (rx < W) {  // identical strings ending inside this word: final
                p.perm[pos] = idx - obase;
                if (pos != sg.begin + sc[(size_t)b * T] - s0)
                    p.lcp[pos] = sg.depth + kf_tail(fh, fh.bpc ? w.tree_key[cur][sg.tree_off + lx] : 0ull, rx);
                continue;
            }
            regather(w, fh, p, idx, sg.depth + kf_step(fh), key, rr);
            if (gr[lx] & TR_SKIP) note_next(w, cur, sg.tree_off + lx, key, rr);
        }
        rec_put(w, cur ^ 1, pos, key, idx, rr);
    }
}

// Level-by-level form of the scatter: one work group of 1024 threads per
// half of a classification tile (SC_TILE records) stages its records in LDS
// in bucket order before writing, so each bucket's part leaves as one
// contiguous run (whole lines instead of scattered 16-byte pieces).  Half
// tiles let two groups share a compute unit, so one group's loads overlap
// the other's stores.  Same output as dev_scatter.
//   1. every wave loads its 256-record chunk (4 per lane) and bucket ids;
//      the second half also counts the first half's buckets from the
//      stored bucket ids;
//   2. ranks inside the wave per bucket (ballot peer masks; order = chunk
//      order, so the result is stable);
//   3. per bucket: prefix over the waves and the half's total, block scan of
//      the totals = the bucket's first slot in the half;
//   4. records go to their slots in LDS, then slot j is written to
//      delta[b] + j where delta[b] = global start of (b, tile) + the first
//      half's count of b (second half only) - first slot.
constexpr uint32_t SC_TILE = TILE / 2;
constexpr uint32_t SB_R = 12;  // r sits above the 11 bits of a bucket id in a staged slot
static_assert(2 * MAX_BUCKETS < (1u << SB_R) && (W << SB_R) < (1u << 16), "slot word layout");
constexpr uint32_t SC_THREADS = 1024, SC_WAVES = SC_THREADS / 64, SC_PER = SC_TILE / SC_THREADS;
static_assert(SC_PER * SC_THREADS == SC_TILE && MAX_BUCKETS < 2 * SC_THREADS, "scatter tile shape");
static_assert(SC_TILE >= 2 * (MAX_BUCKETS + 1) && SC_WAVES * 4 <= (MAX_BUCKETS + 1),
              "first-half counts and wave sums share the slot-bucket array");
struct SmScatterTile {
    union {
        uint16_t WC[SC_WAVES][MAX_BUCKETS + 1];  // per-wave counts, then per-wave first slots
        Rec stage[SC_TILE];                      // the half tile's records in bucket order
    };
    // bucket | r << SB_R of each slot (staging; r is needed there by wide
    // records only); before staging, its first 64 bytes hold the wave sums
    // and its second half the first half's bucket counts (two 16-bit counts
    // per word)
    uint16_t sb[SC_TILE];
    uint32_t delta[MAX_BUCKETS + 1];    // tile totals, then global position - slot
};

template <bool AC>
__device__ void dev_scatter_half(const Work& w, const Params& p, int cur, uint32_t ht, uint32_t n_dist,
                                 SmScatterTile& sm) {
    const uint32_t t = ht >> 1, half = ht & 1u;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint32_t* const wsum = (uint32_t*)sm.sb;
    uint32_t* const first_half = (uint32_t*)(sm.sb + (MAX_BUCKETS + 1));
    const uint32_t si = w.tile_seg[cur][t];
    if (si >= n_dist) {
        if (tid == 0) raise_err(w, ERR_BOUNDS);
        return;
    }
    const Seg sg = w.dist[cur][si];
    const uint32_t d = sg.logv, v = (1u << d) - 1, k = 2 * v + 1;
    const uint32_t T = (sg.size + TILE - 1) / TILE;
    const uint32_t ti = t - sg.tile_off;
    if (d < 1 || d > MAX_LOGV || ti >= T || sg.begin > p.n || sg.size > p.n - sg.begin) {
        if (tid == 0) raise_err(w, ERR_BOUNDS);
        return;
    }
    const uint32_t tile_start = sg.begin + ti * TILE;
    const uint32_t tile_end = min_u32(tile_start + TILE, sg.begin + sg.size);
    const uint32_t start = min_u32(tile_start + half * SC_TILE, tile_end);
    const uint32_t end = min_u32(start + SC_TILE, tile_end);
    const uint32_t m = end - start;
    if (m == 0) return;  // the second half of a tile of at most SC_TILE strings (uniform)
    // 1. loads (all issued before any use)
    const Rec* in = w.rec[cur] + start;
    const uint32_t c0 = wv * (SC_TILE / SC_WAVES);  // the wave's chunk in the half tile
    Rec e[SC_PER];
    uint32_t bk[SC_PER];  // bucket id in bits 0..15 (0xFFFF: no record), r above
#pragma unroll
    for (uint32_t r = 0; r < SC_PER; ++r) {
        const uint32_t q = c0 + r * 64 + lane;
        bk[r] = 0xFFFFu;
        e[r] = Rec{0, 0, 0};
        if (q < m) {
            e[r] = in[q];
            bk[r] = (uint32_t)w.bkt[start + q];
            if (w.wide) bk[r] |= (uint32_t)w.rw[cur][start + q] << 16;
        }
    }
    // the per-wave counts are handled two buckets per 32-bit word (16-bit
    // halves that never carry: every count and sum is at most SC_TILE)
    static_assert(SC_TILE < 65536 && (MAX_BUCKETS + 1) % 8 == 0, "packed bucket counts");
    constexpr uint32_t ROW_WORDS = (MAX_BUCKETS + 1) / 2;
    uint32_t* const WC32 = (uint32_t*)&sm.WC[0][0];
    for (uint32_t i = tid; i < SC_WAVES * ROW_WORDS / 4; i += SC_THREADS) ((uint4*)WC32)[i] = make_uint4(0, 0, 0, 0);
    for (uint32_t b = tid; b < (MAX_BUCKETS + 1) / 2; b += SC_THREADS) first_half[b] = 0;
    __syncthreads();
    if (half) {  // buckets of the first half, two 16-bit counts per word
        for (uint32_t q = tid; q < SC_TILE && tile_start + q < tile_end; q += SC_THREADS) {
            const uint32_t b = w.bkt[tile_start + q];
            if (b < k) atomicAdd(&first_half[b >> 1], 1u << (16 * (b & 1u)));
        }
    }
    // 2. ranks inside the wave
    const uint32_t nbits = 32u - (uint32_t)__builtin_clz(k);  // bits of a bucket id (k = 2v + 1 buckets)
    uint32_t rank[SC_PER];
#pragma unroll
    for (uint32_t r = 0; r < SC_PER; ++r) {
        const uint32_t b = bk[r] & 0xFFFFu;
        const bool valid = b != 0xFFFFu;
        uint64_t peers = __ballot(valid);
        // peers: the lanes whose bucket id agrees with this lane's in each of
        // the id's `nbits` bits (a lane with bit 0 keeps the complement)
        for (uint32_t bit = 0; bit < nbits; ++bit) {
            const uint32_t x = (b >> bit) & 1u;
            const uint64_t mk = __ballot(x);
            peers &= mk ^ ((uint64_t)x - 1u);
        }
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(peers >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
        const uint32_t leader = valid ? (uint32_t)__builtin_ctzll(peers) : 0u;
        uint32_t old = 0;
        if (valid && lane == leader) {  // one writer per bucket and wave
            old = sm.WC[wv][b];
            sm.WC[wv][b] = (uint16_t)(old + (uint32_t)__builtin_popcountll(peers));
        }
        old = __shfl(old, (int)leader, 64);
        rank[r] = old + below;
    }
    __syncthreads();
    // 3. prefix over the waves, tile totals, block scan of the totals
    for (uint32_t pw = tid; 2 * pw < k; pw += SC_THREADS) {  // buckets 2pw, 2pw + 1
        uint32_t run = 0;
#pragma unroll
        for (uint32_t q = 0; q < SC_WAVES; ++q) {
            const uint32_t c = WC32[q * ROW_WORDS + pw];
            WC32[q * ROW_WORDS + pw] = run;
            run += c;
        }
        sm.delta[2 * pw] = run & 0xFFFFu;
        if (2 * pw + 1 < k) sm.delta[2 * pw + 1] = run >> 16;
    }
    __syncthreads();
    const uint32_t b0 = 2 * tid, b1 = 2 * tid + 1;
    const uint32_t n0 = b0 < k ? sm.delta[b0] : 0u, n1 = b1 < k ? sm.delta[b1] : 0u;
    const uint32_t incl = wave_incl_sum(n0 + n1);
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    uint32_t first0 = incl - n0 - n1;
    for (uint32_t q = 0; q < wv; ++q) first0 += wsum[q];
    const uint32_t* sc = w.cnt[cur] + sg.cnt_off;
    const uint32_t s0 = sc[0];
    // b0 and b1 share a word of first-half counts (b0 even)
    const uint32_t fh = first_half[b0 >> 1];
    const uint32_t first1 = first0 + n0;
    if (b0 < k) {
        sm.delta[b0] = sg.begin + sc[(size_t)b0 * T + ti] + (fh & 0xFFFFu) - s0 - first0;
        if (b1 < k) sm.delta[b1] = sg.begin + sc[(size_t)b1 * T + ti] + (fh >> 16) - s0 - first1;
        // both buckets' first slots at once (bucket k, when b1 == k, has no records)
        const uint32_t add = first0 | first1 << 16;
#pragma unroll
        for (uint32_t q = 0; q < SC_WAVES; ++q) atomicAdd(&WC32[q * ROW_WORDS + tid], add);  // no return: one LDS op
    }
    __syncthreads();
    // 4. records to their slots, then out in slot order
    uint32_t slot[SC_PER];
#pragma unroll
    for (uint32_t r = 0; r < SC_PER; ++r)
        slot[r] = (bk[r] & 0xFFFFu) != 0xFFFFu ? sm.WC[wv][bk[r] & 0xFFFFu] + rank[r] : 0u;
    __syncthreads();  // WC is overwritten by the staged records
#pragma unroll
    for (uint32_t r = 0; r < SC_PER; ++r) {
        if ((bk[r] & 0xFFFFu) == 0xFFFFu) continue;
        if (slot[r] >= m) { raise_err(w, ERR_BOUNDS); continue; }
        sm.stage[slot[r]] = e[r];
        sm.sb[slot[r]] = (uint16_t)((bk[r] & 0xFFFFu) | (bk[r] >> 16) << SB_R);
    }
    __syncthreads();
    Rec* out = w.rec[cur ^ 1];
    const uint32_t seg_end = sg.begin + sg.size;
    const uint32_t obase = w.set_base[sg.rid];
    const uint8_t* gr = w.tree_r[cur] + sg.tree_off;
#pragma unroll
    for (uint32_t r = 0; r < SC_PER; ++r) {
        const uint32_t j = r * SC_THREADS + tid;
        if (j >= m) break;
        const uint32_t sbw = sm.sb[j];
        const uint32_t b = sbw & ((1u << SB_R) - 1);
        Rec x = sm.stage[j];
        const uint32_t pos = sm.delta[b] + j;
        if (pos < sg.begin || pos >= seg_end) { raise_err(w, ERR_BOUNDS); continue; }
        if (b & 1u) {
            const uint32_t lx = level_index(b >> 1, d) - 1;
            const uint32_t rx = gr[lx] & TR_CODE;
            const uint32_t idx = rec_idx(w, x);
            const KeyFmt fh = fmt_of<AC>(w);
            if (rx < W) {  // identical strings ending inside this word: final
                p.perm[pos] = idx - obase;
                if (pos != sg.begin + sc[(size_t)b * T] - s0)
                    p.lcp[pos] = sg.depth + kf_tail(fh, fh.bpc ? w.tree_key[cur][sg.tree_off + lx] : 0ull, rx);
                continue;
            }
            uint64_t key;
            uint32_t rr;
            regather(w, fh, p, idx, sg.depth + kf_step(fh), key, rr);  // byte keys: inline gather
            if (gr[lx] & TR_SKIP) note_next(w, cur, sg.tree_off + lx, key, rr);
            x = rec_make(w, key, idx, rr);
            if (w.wide) w.rw[cur ^ 1][pos] = (uint8_t)rr;
        } else if (w.wide) {
            w.rw[cur ^ 1][pos] = (uint8_t)(sbw >> SB_R);
        }
        out[pos] = x;
    }
}

// One half tile per work group: group b takes half tile xcd_item(b, m) of the
// first m = min(groups, half tiles) half tiles, so neighbouring tiles, whose
// runs of a bucket are adjacent in the output, are written through the same
// L2.  A loop over several items here would cost the body two of its four
// waves per SIMD (values of the loop would be held in registers), so the
// half tiles beyond the grid are left to k_scatter_more.
template <bool AC>
__global__ __launch_bounds__(SC_THREADS) __attribute__((amdgpu_waves_per_eu(8))) void k_scatter(Work w, Params p, int cur) {
    __shared__ SmScatterTile sm;
    const uint32_t n_half = 2 * n_tiles_of(w, cur);
    const uint32_t m = min_u32(gridDim.x, n_half);
    if (blockIdx.x >= m) return;
    dev_scatter_half<AC>(w, p, cur, xcd_item(blockIdx.x, m), n_dist_of(w, cur), sm);
}

// The half tiles from `first` on (first = k_scatter's grid), taken from the
// feed by the work groups of its XCD; nothing to do in the common case of a
// level with at most `first` half tiles.
template <bool AC>
__global__ __launch_bounds__(SC_THREADS) __attribute__((amdgpu_waves_per_eu(8)))
void k_scatter_more(Work w, Params p, int cur, uint32_t first) {
    __shared__ SmScatterTile sm;
    // half-tile mailbox (a separate word would take the LDS past 80 KB, and
    // two groups would no longer fit a compute unit): delta is first written
    // after the body's first barrier
    uint32_t& s_ht = sm.delta[0];
    const uint32_t n_half = 2 * n_tiles_of(w, cur);
    if (first >= n_half) return;
    const uint32_t n_dist = n_dist_of(w, cur);
    FeedLine* f = feed_of(w, cur, FEED_SCATTER);
    const uint32_t part = blockIdx.x % FEED_PARTS;
    if (threadIdx.x == 0) s_ht = feed_one(f, first, n_half, part);
    __syncthreads();
    uint32_t ht = uniform(s_ht);
    while (ht < n_half) {
        uint32_t nxt = n_half;
        if (threadIdx.x == 0) nxt = feed_one(f, first, n_half, part);  // overlaps the work
        dev_scatter_half<AC>(w, p, cur, ht, n_dist, sm);
        __syncthreads();
        if (threadIdx.x == 0) s_ht = nxt;
        __syncthreads();
        ht = uniform(s_ht);
    }
}

// ---------------------------------------------------------------------------
// distribution step: children
// ---------------------------------------------------------------------------

// Output description of Algorithm 4.1: bucket i of a segment with common
// prefix h holds strings with common prefix h (even i; the keys at h stay
// valid) or h + 8 (odd i, the full splitter word; section 4.2.2), or
// h + 16 for a large equality bucket whose members all share the next word
// too (note_next: any depth all members share is as valid a start for the
// recursive sort).  Every bucket
// start inside the segment gets a pending LCP (its neighbours differ within
// the word at depth h); the value is filled in once the final order is
// known (figure 4.7).  List slots for the children of the whole segment are
// reserved with one global atomic per list (two passes over the buckets).
__device__ void dev_children(const Work& w, const Params& p, int cur, uint32_t item, uint32_t chunk,
                             uint32_t chunk_buckets, SmChildren& sm) {
    const Seg sg = w.dist[cur][item];
    const uint32_t tid = threadIdx.x, d = sg.logv, v = (1u << d) - 1, k = 2 * v + 1;
    const uint32_t T = (sg.size + TILE - 1) / TILE;
    const int nxt = cur ^ 1;
    if (d < 1 || d > MAX_LOGV || sg.begin > p.n || sg.size > p.n - sg.begin) {
        if (tid == 0) raise_err(w, ERR_BOUNDS);
        return;
    }
    // this work group's buckets: [lo, hi)
    const uint32_t lo = chunk * chunk_buckets;
    if (lo >= k) return;  // uniform
    const uint32_t hi = min_u32(k, lo + chunk_buckets);
    if (tid < NCLS) { sm.n_cls[tid] = 0; sm.s_cls[tid] = 0; sm.cur_cls[tid] = 0; }
    if (tid == 0) {
        sm.n_pend_l = 0; sm.cur_pend = 0; sm.max_d = 0;
        sm.nd = 0; sm.sd = 0; sm.ntree = 0; sm.ncnt = 0; sm.ntile = 0;
        sm.cd = 0; sm.ctree = 0; sm.ccnt = 0; sm.ctile = 0;
    }
    // bucket starts: the first tile's scanned counter of every bucket
    const uint32_t* sc = w.cnt[cur] + sg.cnt_off;
    const uint32_t s0 = sc[0];
    for (uint32_t b = lo + tid; b <= hi; b += BLOCK) sm.ST[b - lo] = b < k ? sc[(size_t)b * T] - s0 : sg.size;
    __syncthreads();
    const uint8_t* gr = w.tree_r[cur] + sg.tree_off;
    const uint32_t* tdf = w.tree_diff[cur] + sg.tree_off;
    const Rec* out = w.rec[nxt];
    const uint32_t obase = w.set_base[sg.rid];
    const uint32_t step = kf_step(fmt_head(w));
    // bucket b -> (start, count, child depth); depth == ~0u: no child
    // segment.  An equality bucket that becomes a distribution segment and
    // whose members all share the word after the splitter's (note_next)
    // starts one more word deeper; its records hold keys of the word after
    // the splitter's and are read again by the next level (`again`).
    auto bucket = [&](uint32_t b, uint32_t& st, uint32_t& cnt, uint32_t& depth, uint32_t& again) {
        st = sm.ST[b - lo];
        const uint32_t en = sm.ST[b - lo + 1];
        cnt = en > st ? en - st : 0u;
        if (en > sg.size) { raise_err(w, ERR_BOUNDS); cnt = 0; }
        depth = sg.depth;
        again = 0;
        if (b & 1u) {
            const uint32_t lx = level_index(b >> 1, d) - 1;
            if ((gr[lx] & TR_CODE) < W) {
                depth = ~0u;  // identical strings, written by the scatter
            } else {
                depth += step;
                // every member has the sample string's next key: skip that word too
                if ((gr[lx] & TR_SKIP) && cnt > p.base_max && tdf[lx] == 0) { depth += step; again = 1; }
            }
        }
    };
    // shape of a distribution child of `cnt` strings
    auto dist_shape = [&](uint32_t cnt, uint32_t& logv, uint32_t& nv, uint32_t& nk, uint32_t& nt) {
        logv = choose_logv(cnt, p.bucket_target, p.max_logv);
        nv = 1u << logv;  // v + 1 tree slots
        nk = 2 * nv - 1;  // 2v + 1 buckets
        nt = (cnt + TILE - 1) / TILE;
    };
    // pass 1: count per list, finish singletons
    for (uint32_t b = lo + tid; b < hi; b += BLOCK) {
        uint32_t st, cnt, depth, again;
        bucket(b, st, cnt, depth, again);
        if (cnt == 0) continue;
        const uint32_t pos = sg.begin + st;
        if (st > 0) atomicAdd(&sm.n_pend_l, 1u);
        if (depth == ~0u) {  // identical strings: final (written by the scatter)
            if (w.remaining) atomicSub(&w.remaining[sg.rid], cnt);
            continue;
        }
        if (cnt == 1) {
            p.perm[pos] = rec_idx(w, out[pos]) - obase;
            if (w.remaining) atomicSub(&w.remaining[sg.rid], 1u);
            continue;
        }
        atomicMax(&sm.max_d, depth);
        if (cnt <= p.base_max) {
            const int cls = size_class(cnt);
            atomicAdd(&sm.n_cls[cls], 1u);
            atomicAdd(&sm.s_cls[cls], cnt);
        } else {
            uint32_t logv, nv, nk, nt;
            dist_shape(cnt, logv, nv, nk, nt);
            atomicAdd(&sm.nd, 1u);
            atomicAdd(&sm.sd, cnt);
            atomicAdd(&sm.ntree, nv);
            atomicAdd(&sm.ncnt, nk * nt);
            atomicAdd(&sm.ntile, nt);
        }
    }
    __syncthreads();
    // one reservation per list for the whole segment, the lists' atomics
    // issued by different threads so their round trips overlap
    CountLines* const cl = &w.ctl->cl[nxt];
    if (tid < NCLS) {
        const uint32_t q = tid;
        sm.slot_cls[q] = sm.n_cls[q] ? (uint32_t)atomicAdd(&cl->base[q].v, pack2(sm.n_cls[q], sm.s_cls[q])) : 0u;
    } else if (tid == NCLS) {
        if (sm.max_d) atomicMax(&cl->depth.v, (unsigned long long)sm.max_d);
    } else if (tid == NCLS + 1) {
        sm.slot_pend = sm.n_pend_l ? atomicAdd(&w.ctl->n_pend, sm.n_pend_l) : 0u;
    } else if (tid == NCLS + 2) {
        sm.bd = sm.nd ? (uint32_t)atomicAdd(&cl->dist.v, pack2(sm.nd, sm.sd)) : 0u;
    } else if (tid == NCLS + 3) {
        const unsigned long long tt = sm.nd ? atomicAdd(&cl->tree_tiles.v, pack2(sm.ntree, sm.ntile)) : 0ull;
        sm.btree = (uint32_t)tt;
        sm.btile = (uint32_t)(tt >> 32);
    } else if (tid == NCLS + 4) {
        sm.bcnt = sm.nd ? (uint32_t)atomicAdd(&cl->cnt.v, (unsigned long long)sm.ncnt) : 0u;
    }
    __syncthreads();
    if (tid == 0) {
        for (int q = 0; q < NCLS; ++q)
            if (sm.slot_cls[q] + sm.n_cls[q] > w.caps.base[q]) raise_err(w, ERR_CAPACITY);
        if (sm.slot_pend + sm.n_pend_l > w.caps.pend) raise_err(w, ERR_CAPACITY);
        if (sm.nd && (sm.bd + sm.nd > w.caps.dist || sm.btree + sm.ntree > w.caps.tree ||
                      sm.bcnt + sm.ncnt > w.caps.cnt || sm.btile + sm.ntile > w.caps.tiles)) {
            raise_err(w, ERR_CAPACITY);
            sm.nd = 0;  // write no distribution child
        }
    }
    __syncthreads();
    // pass 2: write the reserved entries
    for (uint32_t b = lo + tid; b < hi; b += BLOCK) {
        uint32_t st, cnt, depth, again;
        bucket(b, st, cnt, depth, again);
        if (cnt == 0) continue;
        const uint32_t pos = sg.begin + st;
        if (st > 0) {
            const uint32_t q = sm.slot_pend + atomicAdd(&sm.cur_pend, 1u);
            if (q < w.caps.pend) w.pend[q] = Pend{pos, sg.rid, sg.depth, 0u};
        }
        if (depth == ~0u || cnt == 1) continue;
        if (cnt <= p.base_max) {
            const int cls = size_class(cnt);
            const uint32_t q = sm.slot_cls[cls] + atomicAdd(&sm.cur_cls[cls], 1u);
            if (q < w.caps.base[cls]) w.base[cls][nxt][q] = BaseSeg{pos, cnt, depth, sg.rid};
        } else if (sm.nd) {
            uint32_t logv, nv, nk, nt;
            dist_shape(cnt, logv, nv, nk, nt);
            const uint32_t slot = sm.bd + atomicAdd(&sm.cd, 1u);
            const uint32_t toff = sm.btree + atomicAdd(&sm.ctree, nv);
            const uint32_t coff = sm.bcnt + atomicAdd(&sm.ccnt, nk * nt);
            const uint32_t tioff = sm.btile + atomicAdd(&sm.ctile, nt);
            // the tile list entries are written by k_sample (one work group per segment)
            w.dist[nxt][slot] = Seg{pos, cnt, depth, logv, toff, coff, tioff, sg.rid, again};
        }
    }
}

// At most CHILD_CHUNKS work groups per segment, BLOCK buckets each; with
// many segments fewer, larger chunks, so that the launch stays near one
// round of resident groups (each group's steps are a chain of dependent
// global accesses, and a second round would repeat the chain).
constexpr uint32_t CHILD_CHUNKS = (MAX_BUCKETS + BLOCK - 1) / BLOCK;
constexpr uint32_t CHILD_GROUPS = 2048;  // about one round: 256 CUs x 8 groups
__host__ __device__ inline uint32_t child_chunks(uint32_t n_dist) {
    const uint32_t c = n_dist ? CHILD_GROUPS / n_dist : CHILD_CHUNKS;
    return c < 1 ? 1u : c > CHILD_CHUNKS ? CHILD_CHUNKS : c;
}
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8))) void k_children(Work w, Params p, int cur) {
    __shared__ SmChildren sm;
    const uint32_t n_dist = n_dist_of(w, cur);
    const uint32_t chunks = child_chunks(n_dist), items = n_dist * chunks;
    for (uint32_t q = blockIdx.x; q < items; q += gridDim.x) {
        __syncthreads();
        dev_children(w, p, cur, q / chunks, q % chunks, (MAX_BUCKETS + chunks - 1) / chunks, sm);
    }
}

// ---------------------------------------------------------------------------
// boundary LCPs
// ---------------------------------------------------------------------------

// A pending entry at position q separates two buckets of a segment with
// common prefix h: the strings now at q-1 and q differ within the word at
// depth h, so their LCP is h plus the common bytes of those two words.
__device__ __forceinline__ void resolve_pending(const Work& w, const Params& p, const Pend& pe) {
    const uint32_t q = pe.pos, h = pe.depth;
    if (q == 0 || q >= p.n) { raise_err(w, ERR_BOUNDS); return; }
    const uint32_t ob = w.set_base[pe.rid];
    const uint32_t a = p.perm[q - 1] + ob, b = p.perm[q] + ob;
    if (a >= p.n || b >= p.n) { raise_err(w, ERR_BOUNDS); return; }
    const uint64_t oa = p.offsets[a], ob0 = p.offsets[b];
    const uint32_t la = (uint32_t)(p.offsets[a + 1] - oa), lb = (uint32_t)(p.offsets[b + 1] - ob0);
    if (la < h || lb < h) { raise_err(w, ERR_BOUNDS); return; }
    const KeyFmt fh = fmt_head(w);
    const uint64_t ka = key_at(w, fh, p.chars, oa, h, la), kb = key_at(w, fh, p.chars, ob0, h, lb);
    p.lcp[q] = h + kf_lcp_word(fh, ka, kf_r(fh, la, h), kb, kf_r(fh, lb, h));
}

__device__ void dev_lcp_fill(const Work& w, const Params& p, uint32_t first, uint32_t stride) {
    const uint32_t np = min_u32(__hip_atomic_load(&w.ctl->n_pend, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                                w.caps.pend);
    for (uint32_t s = first; s < np; s += stride) resolve_pending(w, p, w.pend[s]);
}

__global__ __launch_bounds__(BLOCK) void k_lcp_fill(Work w, Params p) {
    dev_lcp_fill(w, p, blockIdx.x * BLOCK + threadIdx.x, gridDim.x * BLOCK);
}


// ---------------------------------------------------------------------------
// persistent form: the whole level loop in one launch
// ---------------------------------------------------------------------------

constexpr uint32_t MAX_LEVELS_DEV = 1u << 16;
constexpr uint64_t BARRIER_TIMEOUT_TICKS = 300000000ull;  // 3 s of the 100 MHz wall clock

// Grid-wide barrier among `nblocks` resident work groups.  The last block to
// arrive resets the counter and publishes the next generation; the others
// wait for it with a wall-clock bound: on timeout the block records
// ERR_BARRIER and returns false, and the caller leaves the kernel (every
// other block then times out too, so the grid always drains).  Agent-scope
// release/acquire fences make each phase's global writes visible to all
// blocks of the next phase.
__device__ bool grid_sync(const Work& w, uint32_t nblocks, uint32_t& gen, uint32_t* s_ok) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t target = gen + 1;
        uint32_t good = 1;
        __threadfence();
        const uint32_t prev = atomicAdd(&w.bar->count, 1u);
        if (prev + 1 == nblocks) {
            atomicExch(&w.bar->count, 0u);
            __threadfence();
            __hip_atomic_store(&w.bar->gen, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const uint64_t t0 = wall_clock64();
            while (__hip_atomic_load(&w.bar->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != target) {
                __builtin_amdgcn_s_sleep(2);
                if (wall_clock64() - t0 > BARRIER_TIMEOUT_TICKS) {
                    good = 0;
                    raise_err(w, ERR_BARRIER);
                    break;
                }
            }
        }
        __threadfence();
        gen = target;
        *s_ok = good;
    }
    __syncthreads();
    return *s_ok != 0;
}

__global__ __launch_bounds__(BLOCK) void k_persist(Work w, Params p, const uint32_t* set_begin, uint32_t num_sets,
                                                   int full, uint32_t level0, int cur0, int bases_done) {
    __shared__ SmAll sm;
    __shared__ uint32_t s_ok, s_err;
    __shared__ unsigned long long sc[COUNT_LINES];
    const uint32_t G = gridDim.x, bid = blockIdx.x, tid = threadIdx.x, wv = tid >> 6;
    uint32_t gen = 0;

    if (full) {
        const KeyFmt f = fmt_full(w);
        if (bid == 0 && tid == 0) fmt_publish(w, f);
        for (uint32_t i = bid * BLOCK + tid; i < p.n; i += G * BLOCK) dev_init_one(w, f, p, i);
        if (!grid_sync(w, G, gen, &s_ok)) return;
        const uint32_t nroots = set_begin ? num_sets : 1u;
        for (uint32_t j = bid * BLOCK + tid; j < nroots; j += G * BLOCK) dev_root_one(w, p, set_begin, nroots, j);
        if (!grid_sync(w, G, gen, &s_ok)) return;
    }

    int cur = cur0;
    uint32_t level = level0;
    for (;; ++level) {
        if (tid < COUNT_LINES) sc[tid] = load_count((&w.ctl->cl[cur].dist)[tid]);
        if (tid == 0) s_err = __hip_atomic_load(&w.ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // Every block reads the counts (and error bits) before any block
        // changes them.  The first level of a continuation needs no barrier:
        // no block of this launch has written anything yet, so all read the
        // same counts; its error bits are not consulted (errors of earlier
        // launches are reported at the end all the same, and every loop here
        // is bounded by the counts).
        const bool first_cont = !full && level == level0;
        if (first_cont) {
            __syncthreads();
        } else if (!grid_sync(w, G, gen, &s_ok)) {
            return;
        }
        Counts c = counts_of(sc);
        clamp_counts(c, w.caps);
        if (!first_cont && s_err) break;
        if (level - level0 >= MAX_LEVELS_DEV) {
            if (bid == 0 && tid == 0) raise_err(w, ERR_LEVELS);
            break;
        }
        // a continuation whose first level's base cases ran as separate
        // launches (that level was enqueued without its distribution steps)
        // takes only that level's distribution segments
        const bool skip = first_cont && bases_done;
        const uint32_t nb0 = skip ? 0u : (c.n_base[0] + WAVES - 1) / WAVES;
        const uint32_t nb1 = skip ? 0u : (c.n_base[1] + WAVES - 1) / WAVES;
        const uint32_t nb2 = skip ? 0u : (c.n_base[2] + WAVES - 1) / WAVES, nb3 = skip ? 0u : c.n_base[3];
        const uint32_t nitems = nb0 + nb1 + nb2 + nb3 + c.n_dist;
        if (nitems == 0) break;
        if (bid == 0 && tid == 0 && !skip) note_level(w, c, level);
        if (bid == 0 && tid < COUNT_LINES)
            __hip_atomic_store(&(&w.ctl->cl[cur ^ 1].dist)[tid].v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // base cases of every class and the splitter trees of the level
        for (uint32_t it = bid; it < nitems; it += G) {
            __syncthreads();
            if (it < nb0) dev_base_wave<1>(w, p, cur, 0, it * WAVES + wv, c.n_base[0], sm.wave);
            else if (it < nb0 + nb1) dev_base_wave<2>(w, p, cur, 1, (it - nb0) * WAVES + wv, c.n_base[1], sm.wave);
            else if (it < nb0 + nb1 + nb2)
                dev_base_wave<4>(w, p, cur, 2, (it - nb0 - nb1) * WAVES + wv, c.n_base[2], sm.wave);
            else if (it < nb0 + nb1 + nb2 + nb3) {
                if (fmt_head(w).bpc) dev_base_wg<true>(w, p, cur, it - nb0 - nb1 - nb2, c.n_base[3], sm.base);
                else dev_base_wg<false>(w, p, cur, it - nb0 - nb1 - nb2, c.n_base[3], sm.base);
            }
            else dev_sample(w, p, cur, it - nb0 - nb1 - nb2 - nb3, false, sm.sample);
        }
        if (c.n_dist == 0) {
            ++level;
            break;
        }
        if (!grid_sync(w, G, gen, &s_ok)) return;
        for (uint32_t t = bid; t < c.n_tiles; t += G) {
            __syncthreads();
            dev_classify(w, p, cur, t, c.n_dist, sm.classify);
        }
        if (!grid_sync(w, G, gen, &s_ok)) return;
        const uint32_t nsb = (c.n_cnt + SCAN_CHUNK - 1) / SCAN_CHUNK;
        for (uint32_t b = bid; b < nsb; b += G) {
            __syncthreads();
            dev_scan_reduce(w.cnt[cur], c.n_cnt, w.partial, b, sm.scan);
        }
        if (!grid_sync(w, G, gen, &s_ok)) return;
        if (bid == 0) dev_scan_partials(w.partial, nsb, sm.scan);
        if (!grid_sync(w, G, gen, &s_ok)) return;
        for (uint32_t b = bid; b < nsb; b += G) {
            __syncthreads();
            dev_scan_down(w.cnt[cur], c.n_cnt, w.partial, b, sm.scan);
        }
        if (!grid_sync(w, G, gen, &s_ok)) return;
        for (uint32_t t = bid; t < c.n_tiles; t += G) {
            __syncthreads();
            dev_scatter(w, p, cur, t, c.n_dist, sm.scatter);
        }
        if (!grid_sync(w, G, gen, &s_ok)) return;
        for (uint32_t q = bid; q < c.n_dist * CHILD_CHUNKS; q += G) {
            __syncthreads();
            dev_children(w, p, cur, q / CHILD_CHUNKS, q % CHILD_CHUNKS, BLOCK, sm.children);
        }
        if (!grid_sync(w, G, gen, &s_ok)) return;  // the next level's counts are complete
        cur ^= 1;
    }
    // the boundary LCPs need every level's output; nothing to wait for when
    // a continuation found no level left
    if ((full || level > level0) && !grid_sync(w, G, gen, &s_ok)) return;
    dev_lcp_fill(w, p, bid * BLOCK + tid, G * BLOCK);
}


// ---------------------------------------------------------------------------
// serving helpers
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(BLOCK) void k_rebase(uint64_t* out, const uint64_t* in, uint32_t m, uint64_t add) {
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i <= m) out[i] = in[i] + add;
}

__global__ __launch_bounds__(BLOCK) void k_admit_init(Work w, Params p, int cur, uint32_t pos, uint32_t m) {
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= m) return;
    const uint32_t g = pos + i;
    const uint64_t o0 = p.offsets[g], o1 = p.offsets[g + 1];
    uint32_t len = 0;
    if (o1 < o0 || o1 - o0 > MAX_LEN) raise_err(w, ERR_OFFSETS);
    else len = (uint32_t)(o1 - o0);
    const KeyFmt fh = fmt_head(w);  // byte keys: serving runs no alphabet check
    rec_put(w, cur, g, key_at(w, fh, p.chars, o0, 0, len), g, kf_r(fh, len, 0));
}

__global__ void k_admit_root(Work w, Params p, int cur, uint32_t pos, uint32_t m, uint32_t rid) {
    if (threadIdx.x != 0) return;
    if (m) p.lcp[pos] = 0;
    emit_segment(w, p, cur, cur, pos, m, 0, rid);
}

__global__ __launch_bounds__(BLOCK) void k_pend_filter(Work w, Params p) {
    const uint32_t np = min_u32(w.ctl->n_pend, w.caps.pend);
    for (uint32_t s = blockIdx.x * BLOCK + threadIdx.x; s < np; s += gridDim.x * BLOCK) {
        const Pend pe = w.pend[s];
        if (w.done[pe.rid]) {
            resolve_pending(w, p, pe);
        } else {
            const uint32_t q = atomicAdd(&w.ctl->n_pend2, 1u);
            if (q < w.caps.pend) w.pend2[q] = pe;
            else raise_err(w, ERR_CAPACITY);
        }
    }
}

__global__ void k_pend_swap(Work w) {
    if (threadIdx.x == 0) {
        w.ctl->n_pend = min_u32(w.ctl->n_pend2, w.caps.pend);
        w.ctl->n_pend2 = 0;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline uint32_t blocks_for(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }

hipError_t launch_reset(const Work& w, hipStream_t s) {
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(BLOCK), 0, s, w);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// alphabet of a sort (alphabet compression, §4.6.1): probe, then check
// ---------------------------------------------------------------------------

// Sets the bit of byte c in a 256-bit set held as four words.
__device__ __forceinline__ void set_add(uint64_t (&m)[4], uint32_t c) {
    const uint64_t bit = 1ull << (c & 63);
    const uint32_t q = c >> 6;
    m[0] |= q == 0 ? bit : 0ull;
    m[1] |= q == 1 ? bit : 0ull;
    m[2] |= q == 2 ? bit : 0ull;
    m[3] |= q == 3 ? bit : 0ull;
}

// The first 16 bytes of up to 1024 strings spread over the input: when they
// hold few enough distinct values, they become the candidate set (cand).
// ALPHABET_AUTO asks for at most 3 (2-bit codes, 32 characters per key
// instead of 8) and at most COMPRESS_MAX_AVG characters per string on
// average (a retry's check below reads every character once, the sort moves
// about 26 bytes per string and level); ALPHABET_COMPRESS asks for at most 15 and
// any length.  Otherwise nothing is set and the sort uses byte keys (the
// reset cleared the state).
constexpr uint32_t PROBE_STRINGS = 1024, COMPRESS_MAX_AVG = 64, AUTO_MAX_SYMBOLS = 3;
__global__ __launch_bounds__(PROBE_STRINGS) void k_alpha_probe(Work w, Params p) {
    __shared__ unsigned long long acc[4];
    const uint32_t t = threadIdx.x, lane = t & 63;
    if (p.alphabet == ALPHABET_BYTES || p.n == 0 || p.chars == nullptr) return;  // uniform
    const uint64_t b0 = p.offsets[0], b1 = p.offsets[p.n];
    if (b1 < b0) return;  // malformed offsets are the key gather's to report
    if (p.alphabet == ALPHABET_AUTO && b1 - b0 > (uint64_t)COMPRESS_MAX_AVG * p.n) return;  // uniform
    const uint32_t max_symbols = p.alphabet == ALPHABET_AUTO ? AUTO_MAX_SYMBOLS : 15u;
    if (t < 4) acc[t] = 0;
    __syncthreads();
    uint64_t m[4] = {0, 0, 0, 0};
    const uint32_t S = min_u32(p.n, PROBE_STRINGS);
    if (t < S) {
        const uint32_t i = (uint32_t)(((2ull * t + 1) * p.n) / (2ull * S));
        const uint64_t o0 = p.offsets[i], o1 = p.offsets[i + 1];
        if (o1 > o0 && o1 - o0 <= MAX_LEN) {
            const uint32_t len = (uint32_t)(o1 - o0);
            const uint64_t k0 = gather_key(p.chars, o0, 0, len), k1 = gather_key(p.chars, o0, W, len);
            const uint32_t lim = len < 2 * W ? len : 2 * W;
            for (uint32_t k = 0; k < lim; ++k) set_add(m, (uint32_t)((k < W ? k0 : k1) >> (56 - 8 * (k & 7))) & 0xFFu);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint64_t v = wave_or64(m[q]);
        if (lane == 0 && v) atomicOr(&acc[q], (unsigned long long)v);
    }
    __syncthreads();
    if (t == 0) {
        uint32_t s = 0;
        for (int q = 0; q < 4; ++q) s += (uint32_t)__popcll(acc[q]);
        if (s <= max_symbols) {
            for (int q = 0; q < 4; ++q) w.ctl->alpha.seen[q] = acc[q];
            w.ctl->alpha.limit = max_symbols;
            w.ctl->alpha.cand = 1;
        }
    }
}

// Every byte of chars[offsets[0], offsets[n]) against the set (before a
// persistent sort, or when a sort with the probed set met another byte): a byte
// outside it is added (each work group keeps a byte table in LDS, so a new
// byte costs one global atomic per group), and once the set holds more than
// the probe's limit `over` is set and every group stops.  Reads whole aligned
// 16-byte blocks (inside the pages that hold the range); only the range's
// bytes count.
__global__ __launch_bounds__(BLOCK) void k_alpha_check(Work w, Params p) {
    __shared__ uint8_t tab[256];
    const uint32_t tid = threadIdx.x;
    if (uniform(w.ctl->alpha.cand) == 0u) return;
    const uint64_t b0 = p.offsets[0], b1 = p.offsets[p.n];
    if (b1 <= b0) return;  // no characters (malformed offsets are reported by the key gather)
    for (uint32_t c = tid; c < 256; c += BLOCK) tab[c] = (uint8_t)((w.ctl->alpha.seen[c >> 6] >> (c & 63)) & 1u);
    __syncthreads();
    const uintptr_t lo = (uintptr_t)(p.chars + b0), hi = (uintptr_t)(p.chars + b1);
    const uintptr_t first = lo & ~(uintptr_t)15;
    const uint64_t blocks = (uint64_t)((hi - first + 15) >> 4);
    const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    // four 16-byte blocks per thread and iteration, loaded before any is used
    for (uint64_t k0 = (uint64_t)blockIdx.x * BLOCK + tid; k0 < blocks; k0 += 4 * stride) {
        if (__builtin_nontemporal_load(&w.ctl->alpha.over) != 0u) break;  // the set is too large: byte keys
        u32x4 v[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            const uint64_t k = k0 + u * stride;
            v[u] = k < blocks ? __builtin_nontemporal_load((const u32x4*)(first + 16 * k)) : u32x4{0, 0, 0, 0};
        }
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            const uint64_t k = k0 + u * stride;
            if (k >= blocks) break;
            const uintptr_t a = first + 16 * k;
            const uint32_t wd[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
            for (uint32_t j = 0; j < 16; ++j) {
                const uintptr_t at = a + j;
                const uint32_t c = (wd[j >> 2] >> (8 * (j & 3))) & 0xFFu;
                if (at < lo || at >= hi || tab[c]) continue;
                tab[c] = 1;
                const unsigned long long bit = 1ull << (c & 63);
                const unsigned long long old = atomicOr((unsigned long long*)&w.ctl->alpha.seen[c >> 6], bit);
                if (old & bit) continue;
                uint32_t s = 0;
                for (int q = 0; q < 4; ++q)
                    s += (uint32_t)__popcll(atomicOr((unsigned long long*)&w.ctl->alpha.seen[q], 0ull));
                if (s > w.ctl->alpha.limit) atomicOr(&w.ctl->alpha.over, 1u);
            }
        }
    }
}

hipError_t launch_alphabet(const Work& w, const Params& p, uint32_t check_grid, bool check, hipStream_t s) {
    if (p.alphabet == ALPHABET_BYTES) return hipSuccess;  // byte keys: the reset left the state empty
    hipLaunchKernelGGL(k_alpha_probe, dim3(1), dim3(PROBE_STRINGS), 0, s, w, p);
    if (check) hipLaunchKernelGGL(k_alpha_check, dim3(check_grid > 0 ? check_grid : 1), dim3(BLOCK), 0, s, w, p);
    return hipGetLastError();
}
__global__ void k_report(Work w, uint32_t* out) {
    if (threadIdx.x == 0) out[0] = w.ctl->err;
}
hipError_t launch_report(const Work& w, uint32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_report, dim3(1), dim3(64), 0, s, w, out);
    return hipGetLastError();
}
hipError_t launch_level_begin(const Work& w, int cur, uint32_t level, hipStream_t s) {
    hipLaunchKernelGGL(k_level_begin, dim3(1), dim3(BLOCK), 0, s, w, cur, level);
    return hipGetLastError();
}
hipError_t launch_init(const Work& w, const Params& p, hipStream_t s) {
    if (p.n == 0) return hipSuccess;
    if (p.ac) hipLaunchKernelGGL(k_init<true>, dim3(blocks_for(p.n, BLOCK)), dim3(BLOCK), 0, s, w, p);
    else hipLaunchKernelGGL(k_init<false>, dim3(blocks_for(p.n, BLOCK)), dim3(BLOCK), 0, s, w, p);
    return hipGetLastError();
}
hipError_t launch_roots(const Work& w, const Params& p, const uint32_t* set_begin, uint32_t num_sets,
                        hipStream_t s) {
    if (num_sets == 0) return hipSuccess;
    hipLaunchKernelGGL(k_roots, dim3(blocks_for(num_sets, 64)), dim3(64), 0, s, w, p, set_begin, num_sets);
    return hipGetLastError();
}
static inline dim3 grid_of(uint32_t g) { return dim3(g ? g : 1u); }
template <bool AC>
static void launch_base_as(const Work& w, const Params& p, int cur, int cls, uint32_t grid, hipStream_t s) {
    if (cls == 0)
        hipLaunchKernelGGL((k_base_wave<1, AC>), grid_of(grid), dim3(BLOCK), 0, s, w, p, cur, 0);
    else if (cls == 1)
        hipLaunchKernelGGL((k_base_wave<2, AC>), grid_of(grid), dim3(BLOCK), 0, s, w, p, cur, 1);
    else if (cls == 2)
        hipLaunchKernelGGL((k_base_wave<4, AC>), grid_of(grid), dim3(BLOCK), 0, s, w, p, cur, 2);
    else
        hipLaunchKernelGGL(k_base<AC>, grid_of(grid), dim3(BLOCK), 0, s, w, p, cur);
}
hipError_t launch_base(const Work& w, const Params& p, int cur, int cls, uint32_t grid, hipStream_t s) {
    if (p.ac) launch_base_as<true>(w, p, cur, cls, grid, s);
    else launch_base_as<false>(w, p, cur, cls, grid, s);
    return hipGetLastError();
}
hipError_t launch_sample(const Work& w, const Params& p, int cur, uint32_t grid, bool root_keys, hipStream_t s) {
    hipLaunchKernelGGL(k_sample, grid_of(grid), dim3(BLOCK), 0, s, w, p, cur, root_keys ? 1 : 0);
    return hipGetLastError();
}
hipError_t launch_classify(const Work& w, const Params& p, int cur, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(k_classify, grid_of(grid), dim3(BLOCK), 0, s, w, p, cur);
    return hipGetLastError();
}
hipError_t launch_scan(const Work& w, int cur, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_reduce, grid_of(grid), dim3(BLOCK), 0, s, w, cur);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, w, cur);
    hipLaunchKernelGGL(k_scan_down, grid_of(grid), dim3(BLOCK), 0, s, w, cur);
    return hipGetLastError();
}
hipError_t launch_scatter(const Work& w, const Params& p, int cur, uint32_t grid, uint32_t more_grid,
                          hipStream_t s) {
    if (p.ac) {
        hipLaunchKernelGGL(k_scatter<true>, grid_of(grid), dim3(SC_THREADS), 0, s, w, p, cur);
        if (more_grid)
            hipLaunchKernelGGL(k_scatter_more<true>, grid_of(more_grid), dim3(SC_THREADS), 0, s, w, p, cur,
                               grid_of(grid).x);
    } else {
        hipLaunchKernelGGL(k_scatter<false>, grid_of(grid), dim3(SC_THREADS), 0, s, w, p, cur);
        if (more_grid)
            hipLaunchKernelGGL(k_scatter_more<false>, grid_of(more_grid), dim3(SC_THREADS), 0, s, w, p, cur,
                               grid_of(grid).x);
    }
    return hipGetLastError();
}
hipError_t launch_children(const Work& w, const Params& p, int cur, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(k_children, grid_of(grid), dim3(BLOCK), 0, s, w, p, cur);
    return hipGetLastError();
}
hipError_t launch_lcp_fill(const Work& w, const Params& p, hipStream_t s) {
    uint32_t nb = blocks_for(p.n, BLOCK);
    if (nb > 2048) nb = 2048;
    if (nb == 0) nb = 1;
    hipLaunchKernelGGL(k_lcp_fill, dim3(nb), dim3(BLOCK), 0, s, w, p);
    return hipGetLastError();
}

uint32_t grid_base(int cls, uint32_t n_base) { return cls == CLS_WG ? n_base : blocks_for(n_base, WAVES); }
uint32_t grid_classify(uint32_t n_tiles) { return n_tiles; }
uint32_t grid_scan(uint32_t n_cnt) { return blocks_for(n_cnt, SCAN_CHUNK); }
uint32_t grid_scatter(uint32_t n_tiles) { return 2 * n_tiles; }
uint32_t grid_children(uint32_t n_dist) { return n_dist * child_chunks(n_dist); }

hipError_t launch_persistent(const Work& w, const Params& p, const uint32_t* set_begin, uint32_t num_sets,
                             uint32_t blocks, bool full, uint32_t level, int cur, bool bases_done, hipStream_t s) {
    hipLaunchKernelGGL(k_persist, dim3(blocks), dim3(BLOCK), 0, s, w, p, set_begin, num_sets, full ? 1 : 0, level,
                       cur, bases_done ? 1 : 0);
    return hipGetLastError();
}

template <typename K>
static hipError_t resident(K kernel, int threads, int cus, uint32_t* out) {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0);
    if (e != hipSuccess) return e;
    *out = (uint32_t)std::max(1, per_cu * cus);
    return hipSuccess;
}

hipError_t kernel_caps(int device, KernelCaps* k) {
    int cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e == hipSuccess) e = resident(k_base_wave<1, false>, BLOCK, cus, &k->base[0]);
    if (e == hipSuccess) e = resident(k_base_wave<2, false>, BLOCK, cus, &k->base[1]);
    if (e == hipSuccess) e = resident(k_base_wave<4, false>, BLOCK, cus, &k->base[2]);
    if (e == hipSuccess) e = resident(k_base<false>, BLOCK, cus, &k->base[3]);
    if (e == hipSuccess) e = resident(k_sample, BLOCK, cus, &k->sample);
    if (e == hipSuccess) e = resident(k_classify, BLOCK, cus, &k->classify);
    if (e == hipSuccess) e = resident(k_scan_reduce, BLOCK, cus, &k->scan);
    if (e == hipSuccess) e = resident(k_scatter<false>, SC_THREADS, cus, &k->scatter);
    if (e == hipSuccess) e = resident(k_children, BLOCK, cus, &k->children);
    if (e == hipSuccess) e = resident(k_persist, BLOCK, cus, &k->persist);
    return e;
}

hipError_t launch_admit(const Work& w, const Params& p, int cur, uint32_t pos, uint32_t m, uint32_t rid,
                        hipStream_t s) {
    if (m) hipLaunchKernelGGL(k_admit_init, dim3(blocks_for(m, BLOCK)), dim3(BLOCK), 0, s, w, p, cur, pos, m);
    hipLaunchKernelGGL(k_admit_root, dim3(1), dim3(64), 0, s, w, p, cur, pos, m, rid);
    return hipGetLastError();
}
hipError_t launch_rebase(uint64_t* out, const uint64_t* in, uint32_t m, uint64_t add, hipStream_t s) {
    hipLaunchKernelGGL(k_rebase, dim3(blocks_for((uint64_t)m + 1, BLOCK)), dim3(BLOCK), 0, s, out, in, m, add);
    return hipGetLastError();
}
hipError_t launch_pend_filter(const Work& w, const Params& p, hipStream_t s) {
    hipLaunchKernelGGL(k_pend_filter, dim3(512), dim3(BLOCK), 0, s, w, p);
    return hipGetLastError();
}
hipError_t launch_pend_swap(const Work& w, hipStream_t s) {
    hipLaunchKernelGGL(k_pend_swap, dim3(1), dim3(64), 0, s, w);
    return hipGetLastError();
}

// Plain streaming copy: every lane moves COPY_U 16-byte words per
// iteration (all loads issued before the stores), grid-stride over the
// buffer; the reference for the achievable HBM bandwidth and the kernel of
// known traffic for counter calibration.
constexpr uint32_t COPY_U = 4;
__global__ __launch_bounds__(BLOCK) void k_copy(uint4* __restrict__ dst, const uint4* __restrict__ src, size_t n16) {
    const size_t stride = (size_t)gridDim.x * BLOCK * COPY_U;
    for (size_t i0 = (size_t)blockIdx.x * BLOCK * COPY_U + threadIdx.x; i0 < n16; i0 += stride) {
        uint4 v[COPY_U];
#pragma unroll
        for (uint32_t u = 0; u < COPY_U; ++u) {
            const size_t i = i0 + (size_t)u * BLOCK;
            if (i < n16) v[u] = src[i];
        }
#pragma unroll
        for (uint32_t u = 0; u < COPY_U; ++u) {
            const size_t i = i0 + (size_t)u * BLOCK;
            if (i < n16) dst[i] = v[u];
        }
    }
}

hipError_t launch_copy(void* dst, const void* src, size_t n16, hipStream_t s) {
    if (n16 == 0) return hipSuccess;
    // 16 groups of 256 lanes per compute unit at most: every lane then keeps
    // four 16-byte loads in flight
    const uint32_t nb = (uint32_t)std::min<size_t>((n16 + BLOCK * COPY_U - 1) / (BLOCK * COPY_U), 256u * 16u);
    hipLaunchKernelGGL(k_copy, dim3(nb), dim3(BLOCK), 0, s, (uint4*)dst, (const uint4*)src, n16);
    return hipGetLastError();
}

}  // namespace ss
