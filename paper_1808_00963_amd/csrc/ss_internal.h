// Internal data structures and kernel launchers of libss.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace ss {

// A string in flight, one ping-pong buffer per recursion level parity
// (section 4.2.8, "Out-of-place Redistribution"): its 8-byte key at the
// segment's depth h (big-endian, zero padded), its index in the input
// (global over a batch) and r = min(len - h, 8), the characters of the
// string inside the key (0 is a character, so r tells a string that ends
// inside the word from one with zero bytes there).  12 bytes, moved as one
// 3-dword access: with fewer than 2^28 strings r sits in the top 4 bits of
// the index word; wider sorts keep the whole index there and r in a side
// byte array.  The length itself is re-read from the offsets where a key is
// gathered again deeper.
struct Rec {
    uint32_t klo, khi;  // key
    uint32_t ix;        // index | r << IX_BITS (narrow), index (wide)
};
static_assert(sizeof(Rec) == 12, "12-byte records");
constexpr uint32_t IX_BITS = 28;
constexpr uint32_t IX_MASK = (1u << IX_BITS) - 1;
constexpr uint32_t NARROW_MAX_N = 1u << IX_BITS;  // sorts of fewer strings are narrow

// A segment of the ping-pong element array that still needs a distribution
// step (sample, classify, scatter; Algorithm 4.1).  All its strings share a
// common prefix of `depth` characters.
struct Seg {
    uint32_t begin;     // first position
    uint32_t size;      // number of strings
    uint32_t depth;     // common prefix length h
    uint32_t logv;      // d: v = 2^d - 1 splitters, 2v+1 buckets
    uint32_t tree_off;  // first splitter in the tree pool
    uint32_t cnt_off;   // first counter in the counter pool
    uint32_t tile_off;  // first tile in the tile list
    uint32_t rid;       // set (batch) or request (serving) the segment belongs to
    uint32_t regather;  // 1: the records hold keys of a smaller depth (an equality
                        // bucket that skipped its common prefix); read them again at `depth`
};

// A boundary whose LCP is filled in once the final order is known: the
// strings at pos-1 and pos differ within the word at `depth`.
struct Pend {
    uint32_t pos, rid, depth, pad;
};

// A segment small enough for the in-LDS base case.
struct BaseSeg {
    uint32_t begin, size, depth, rid;
};

// Base-case size classes: one wave per segment with 1, 2 or 4 strings per
// lane (<= 64, <= 128, <= 256), one work group with the segment in LDS
// (<= base_max).
constexpr int NCLS = 4;
constexpr int CLS_WG = NCLS - 1;
constexpr uint32_t CLS_MAX[NCLS] = {64, 128, 256, 1024};
__host__ __device__ constexpr int size_class(uint32_t size) {
    return size <= CLS_MAX[0] ? 0 : size <= CLS_MAX[1] ? 1 : size <= CLS_MAX[2] ? 2 : 3;
}

// Work-list sizes of one recursion level.
struct Counts {
    uint32_t n_dist;
    uint32_t n_tiles;
    uint32_t n_cnt;
    uint32_t n_tree;
    uint32_t n_base[NCLS];
    uint32_t max_depth;
    uint32_t base_strings[NCLS];  // strings in the base-case segments of each class
    uint32_t dist_strings;        // strings in the distribution segments of the level
};

// Device-side form of a level's counts: every counter word on its own
// 128-byte line (atomics on different lines proceed in parallel), and
// counters that are always advanced together share one 64-bit word, so one
// atomic reserves both.
struct alignas(128) CLine {
    unsigned long long v;
    uint32_t pad[30];
};
struct CountLines {
    CLine dist;        // n_dist | dist_strings << 32
    CLine tree_tiles;  // n_tree | n_tiles << 32
    CLine cnt;         // n_cnt
    CLine depth;       // max_depth
    CLine base[NCLS];  // n_base[q] | base_strings[q] << 32
};
constexpr uint32_t COUNT_LINES = sizeof(CountLines) / sizeof(CLine);

__host__ __device__ inline Counts counts_of(const unsigned long long* v) {
    Counts c{};
    c.n_dist = (uint32_t)v[0];
    c.dist_strings = (uint32_t)(v[0] >> 32);
    c.n_tree = (uint32_t)v[1];
    c.n_tiles = (uint32_t)(v[1] >> 32);
    c.n_cnt = (uint32_t)v[2];
    c.max_depth = (uint32_t)v[3];
    for (int q = 0; q < NCLS; ++q) {
        c.n_base[q] = (uint32_t)v[4 + q];
        c.base_strings[q] = (uint32_t)(v[4 + q] >> 32);
    }
    return c;
}
inline Counts counts_of(const CountLines& l) {
    unsigned long long v[COUNT_LINES];
    const CLine* L = &l.dist;
    for (uint32_t i = 0; i < COUNT_LINES; ++i) v[i] = L[i].v;
    return counts_of(v);
}

constexpr uint32_t ROUND_LINES = 32;  // lines of the base_rounds statistic
constexpr uint32_t LEVEL_RECS = 64;    // levels whose work counts are kept for the profiler

// Work counts of one recursion level as recorded when the level starts
// (statistics and per-launch units of the profiler).
struct LevelRec {
    uint32_t n_dist, n_tiles, n_cnt, dist_strings;
    uint32_t n_base[NCLS], base_strings[NCLS];
};

// Statistics of one sort, accumulated on the device level by level.
struct DevStats {
    uint32_t levels;          // levels that had work
    uint32_t dist_segments;
    uint32_t dist_tiles;
    uint32_t max_depth;
    uint32_t base_segments[NCLS];
    uint64_t base_strings[NCLS];
    uint64_t dist_strings;
};

// Device-side control block.  Every group of fields that kernels update
// with atomics sits on its own 128-byte line, so the atomics never share a
// line with data other waves read.
struct Ctl {
    CountLines cl[2];
    uint32_t n_pend;
    uint32_t n_pend2;      // survivors of a pending-list filter (serving)
    uint32_t pad0[30];
    uint32_t err;          // errors of this sort (zeroed when a sort starts)
    uint32_t err_sticky;   // errors of every sort on this workspace until cleared by the host
    uint32_t pad1[30];
    // refinement rounds run by base cases (statistics), spread over lines so
    // the waves that report them do not queue on one address
    struct {
        uint32_t v;
        uint32_t pad[31];
    } base_rounds[ROUND_LINES];
    DevStats stats;
    LevelRec lv[LEVEL_RECS];
    // Alphabet of the sort (the key format follows from it, see KeyFmt):
    // the probe sets `cand` when a sample of the strings shows at most
    // `limit` distinct bytes and records them in `seen`; the check (when
    // run) adds every other byte of the input to `seen` and sets `over` once
    // more than `limit` are known.  Compressed keys exactly when
    // cand && !over.  Without the check, every compressed gather sets
    // `miss` when it meets a byte outside `seen`, and the host sorts again.
    // The key gather (k_init) also writes the resulting code width and
    // characters per word for the kernels after it (bpc = 0: byte keys).
    struct alignas(128) {
        uint32_t cand;
        uint32_t over;
        uint32_t bpc;
        uint32_t cpw;
        uint64_t seen[4];
        uint32_t limit;  // most bytes the set may hold for compressed keys
        uint32_t miss;   // a compressed gather met a byte outside the set
    } alpha;
};
inline uint32_t base_rounds_of(const Ctl& c) {
    uint32_t t = 0;
    for (uint32_t i = 0; i < ROUND_LINES; ++i) t += c.base_rounds[i].v;
    return t;
}

// Dynamic distribution of a launch's items over its workers (work groups or
// waves): the items are cut into FEED_PARTS contiguous parts, one per XCD
// (work groups are dispatched to the XCDs round robin), and a worker takes
// chunks of its part through an atomic counter on the part's own line, so
// workers that finish early take more and neighbouring items stay on one
// XCD.  Each kernel kind of a level has its own FEED_PARTS lines; the
// counters of the two level slots alternate and are zeroed when a level
// starts.
constexpr uint32_t FEED_PARTS = 8;
enum FeedKind : uint32_t { FEED_BASE = 0, FEED_CLASSIFY = NCLS, FEED_SCATTER, FEED_KINDS };
struct alignas(128) FeedLine {
    uint32_t next;
    uint32_t pad[31];
};
constexpr uint32_t FEED_LINES = 2 * FEED_KINDS * FEED_PARTS;

// Error bits raised on the device.
enum : uint32_t {
    ERR_OFFSETS = 1u,      // non-monotone offsets or string too long
    ERR_CAPACITY = 2u,     // an internal pool overflowed
    ERR_BOUNDS = 4u,       // a computed position fell outside its segment
    ERR_SETS = 8u,         // batch set boundaries invalid
    ERR_BARRIER = 16u,     // a grid barrier of the persistent kernel timed out
    ERR_LEVELS = 32u,      // the level limit of the persistent kernel was reached
};

// Grid barrier of the persistent kernel: arrival counter and generation on
// separate 128-byte lines.
struct GridBar {
    uint32_t count;
    uint32_t pad0[31];
    uint32_t gen;
    uint32_t pad1[31];
};

constexpr uint32_t MAX_LEN = 0x7FFFFF00u;   // longest accepted string
constexpr uint32_t BLOCK = 256;             // threads per work group
constexpr uint32_t WAVES = BLOCK / 64;
constexpr uint32_t IPT = 32;                // tile elements per thread
constexpr uint32_t TILE = BLOCK * IPT;      // strings per classify/scatter tile
constexpr uint32_t MAX_LOGV = 10;           // at most 1023 splitters
constexpr uint32_t MAX_BUCKETS = (2u << MAX_LOGV) - 1;
constexpr uint32_t BASE_CAP = 1024;         // largest base-case segment
constexpr uint32_t SKIP_MIN_SAMPLES = 4;    // equal samples before an equality bucket may skip a word
constexpr uint32_t TR_CODE = 0x7F;          // a splitter's r code in its tree_r byte
constexpr uint32_t TR_SKIP = 0x80;          // ... and whether its equality bucket may skip a word

// Pool capacities of one level, derived from n (see ss_api.cpp).
struct Caps {
    uint32_t dist, tiles, base[NCLS], cnt, tree, pend;
};

// Pointers to the workspace of one sort.
struct Work {
    Rec* rec[2];
    uint8_t* rw[2];      // wide layout: r of each position (else null)
    uint32_t wide;       // 1: the index word holds the whole index
    uint16_t* bkt;
    uint32_t* cnt[2];
    uint32_t* partial;
    Seg* dist[2];
    BaseSeg* base[NCLS][2];
    uint32_t* tile_seg[2];
    uint64_t* tree_key[2];
    uint8_t* tree_r[2];      // r code | TR_SKIP
    uint64_t* tree_next[2];  // per TR_SKIP splitter: its sample string's key one word deeper
    uint32_t* tree_diff[2];  // per TR_SKIP splitter: 0 while every member of its equality
                             // bucket has that next key (and a full word there), else 1
    Pend* pend;               // pending boundary LCPs
    Pend* pend2;              // filter target (serving)
    Ctl* ctl;
    FeedLine* feed;           // FEED_LINES work-distribution counters
    GridBar* bar;
    const uint32_t* set_base; // per set/request id: its first position (subtracted from perm entries)
    uint32_t* zero_base;      // one zero word on its own line: set base of a plain sort
    uint32_t* remaining;      // per request id: strings not yet final (serving; else null)
    const uint8_t* done;      // per request id: 1 once finished (serving; else null)
    Caps caps;
};

// Parameters of one sort.
struct Params {
    const uint8_t* chars;
    const uint64_t* offsets;
    uint32_t n;
    uint32_t* perm;
    uint32_t* lcp;
    uint32_t max_logv;
    uint32_t bucket_target;
    uint32_t base_max;
    uint32_t alphabet;  // ALPHABET_*: which inputs get alphabet-compressed keys
    uint32_t ac;        // the sort's keys are compressed (known to the host before the key gather)
};
// The C ABI's SS_ALPHABET_AUTO, _BYTES and _COMPRESS.
constexpr uint32_t ALPHABET_AUTO = 0, ALPHABET_BYTES = 1, ALPHABET_COMPRESS = 2;

// ---- launchers (ss_kernels.hip) ----
// Every kernel of a recursion level reads its work counts from the control
// block (slot `cur`), so a level can be enqueued before the previous one has
// run.  `grid` is the number of work groups to launch: any value >= 1 gives
// the same result (workers take items until none are left); the host picks
// it from what it knows (exact counts, or the pool capacities and the
// device's resident capacity).
hipError_t launch_reset(const Work& w, hipStream_t s);
// The sort's alphabet (after launch_reset, before launch_init): a probe of
// a sample of the strings, then, when it found at most 15 distinct bytes, a
// check of every byte of the input.
hipError_t launch_alphabet(const Work& w, const Params& p, uint32_t check_grid, bool check, hipStream_t s);
hipError_t launch_init(const Work& w, const Params& p, hipStream_t s);
hipError_t launch_roots(const Work& w, const Params& p, const uint32_t* set_begin, uint32_t num_sets,
                        hipStream_t s);
// Starts level `level` on slot `cur`: records its counts (statistics),
// zeroes the next slot's counts and this slot's feed counters (no memset:
// stays capturable).
hipError_t launch_level_begin(const Work& w, int cur, uint32_t level, hipStream_t s);
// out[0] = the sort's error bits (a device word of the caller).
hipError_t launch_report(const Work& w, uint32_t* out, hipStream_t s);
hipError_t launch_base(const Work& w, const Params& p, int cur, int cls, uint32_t grid, hipStream_t s);
// root_keys: the first level's sampling, reading keys from the strings.
hipError_t launch_sample(const Work& w, const Params& p, int cur, uint32_t grid, bool root_keys, hipStream_t s);
hipError_t launch_classify(const Work& w, const Params& p, int cur, uint32_t grid, hipStream_t s);
hipError_t launch_scan(const Work& w, int cur, uint32_t grid, hipStream_t s);
// One half tile per work group of `grid`; with more_grid != 0 a second
// launch of more_grid groups takes the half tiles beyond `grid` (none when
// the level has at most `grid` of them).
hipError_t launch_scatter(const Work& w, const Params& p, int cur, uint32_t grid, uint32_t more_grid,
                          hipStream_t s);
hipError_t launch_children(const Work& w, const Params& p, int cur, uint32_t grid, hipStream_t s);
hipError_t launch_lcp_fill(const Work& w, const Params& p, hipStream_t s);
// Resident capacity (work groups) of each level kernel on `device`.
struct KernelCaps {
    uint32_t base[NCLS], sample, classify, scan, scatter, children, persist;
};
hipError_t kernel_caps(int device, KernelCaps* k);
// Work groups of a level kernel that suffice for the given work counts.
uint32_t grid_base(int cls, uint32_t n_base);
uint32_t grid_classify(uint32_t n_tiles);
uint32_t grid_scan(uint32_t n_cnt);
uint32_t grid_scatter(uint32_t n_tiles);
uint32_t grid_children(uint32_t n_dist);
// The sort's levels in ONE persistent launch of `blocks` work groups that
// must all be resident, separated by grid barriers.  full: starts with the
// key gather and the roots (after launch_reset); otherwise continues from
// slot `cur` at level `level` (the levels before were enqueued as separate
// launches; with bases_done, so were the base cases of `level` itself, and
// only its distribution segments are left).  Ends with the boundary LCPs
// either way.
hipError_t launch_persistent(const Work& w, const Params& p, const uint32_t* set_begin, uint32_t num_sets,
                             uint32_t blocks, bool full, uint32_t level, int cur, bool bases_done, hipStream_t s);
// Serving: gathers keys at depth 0 for positions [pos, pos+m) into buffer
// `cur` and makes them one root segment of request `rid` in the lists of
// `cur`.
hipError_t launch_admit(const Work& w, const Params& p, int cur, uint32_t pos, uint32_t m, uint32_t rid,
                        hipStream_t s);
// Serving: offsets_out[i] = offsets_in[i] + add for i <= m.
hipError_t launch_rebase(uint64_t* out, const uint64_t* in, uint32_t m, uint64_t add, hipStream_t s);
// Serving: resolves the pending LCPs of finished requests and keeps the
// others (moved to pend2; the caller swaps the lists).
hipError_t launch_pend_filter(const Work& w, const Params& p, hipStream_t s);
hipError_t launch_pend_swap(const Work& w, hipStream_t s);
// Streaming copy (bandwidth calibration).
hipError_t launch_copy(void* dst, const void* src, size_t n16, hipStream_t s);


// ---- LCP-aware merging of sorted runs (ss_merge.hip) ----
constexpr uint32_t MERGE_BLOCK = 256;
constexpr uint32_t MERGE_PER = 8;                          // outputs per thread of k_merge_tile
constexpr uint32_t MERGE_TILE = MERGE_BLOCK * MERGE_PER;   // outputs per work group

enum : uint32_t {
    MERR_INDEX = 1u,     // a perm entry is not below the number of strings
    MERR_OFFSETS = 2u,   // non-monotone offsets or a string too long
    MERR_INTERNAL = 4u,  // a split point fell outside its pair of runs
};

// One pair of adjacent runs A = [a, a+na), B = [a+na, a+na+nb) of the source
// arrays, merged into [a, a+na+nb) of the destination arrays; its tiles of
// MERGE_TILE outputs are tile0, tile0+1, ... (ceil((na+nb)/MERGE_TILE)).
struct MergeTask {
    uint32_t a, na, nb, tile0;
};

struct MergeArgs {
    const uint8_t* chars;
    const uint64_t* offsets;
    uint32_t n_strings;
    const uint32_t* src_perm;
    const uint32_t* src_lcp;
    uint32_t* dst_perm;
    uint32_t* dst_lcp;
    const MergeTask* tasks;  // ordered by tile0
    uint32_t n_tasks;
    uint32_t n_tiles;
    uint32_t* split;  // per tile: outputs taken from A before it
    uint32_t* cross;  // per tile: LCP of the first strings of its A and B windows
    uint32_t* err;
};

hipError_t launch_merge_split(const MergeArgs& m, hipStream_t s);
hipError_t launch_merge_tiles(const MergeArgs& m, hipStream_t s);

// ---- suffix array by prefix doubling (ss_sa.hip) ----
constexpr uint32_t SA_BLOCK = 256;
constexpr uint32_t SA_PER = 16;                     // sorted positions per thread when renaming
constexpr uint32_t SA_TILE = SA_BLOCK * SA_PER;
constexpr uint32_t SA_W0 = 32;                      // characters per suffix in the first round
constexpr uint32_t SA_PACKED_LEN = 24;              // bytes of an alphabet-compressed first-round window
static_assert(SA_BLOCK == 256, "the packing kernel stages one rank per thread");
// Words of packed ranks for a text of n characters at b bits (two extra
// words of zeros so every window can read three).
inline uint32_t sa_pack_blocks(uint32_t n, uint32_t b) { return (uint32_t)(((uint64_t)n + 64 / b - 1) / (64 / b) + 2); }
inline uint32_t sa_tiles(uint32_t n) { return (uint32_t)(((uint64_t)n + SA_TILE - 1) / SA_TILE); }

struct SaArgs {
    const uint32_t* perm;  // the round's sort: permutation of its m strings
    const uint32_t* lcp;   // and their LCP array
    uint32_t n;            // text length
    uint32_t m;            // strings sorted in this round
    uint32_t round0;       // 1: all suffixes as first-round windows, sorted straight into sa
    uint32_t round0_len;   // round 0: string length of a packed window, 0 for plain SA_W0-character windows
    uint32_t* idx;         // rounds > 0: suffix of string e
    const uint32_t* pos;   // rounds > 0: suffix-array position of string e (increasing)
    uint32_t* next_pos;    // positions that stay unfinished, in order
    uint32_t* sa;          // suffix array (final entries stay in place)
    uint32_t* names;       // n: name of every suffix (first position of its group)
    uint32_t* part_max;    // sa_tiles(m) scratch counters
    uint32_t* part_cnt;    // sa_tiles(m) + 1; [sa_tiles(m)] receives the count of next_pos
};

// Round-0 strings: window i = text[i .. i + min(SA_W0, n - i)), packed, with
// their n+1 offsets (chars needs SA_W0 * n bytes at most).
hipError_t launch_sa_windows(const uint8_t* text, uint32_t n, uint8_t* chars, uint64_t* offsets, hipStream_t s);
// Byte values present in the text: atomically ORed into mask[8] (zeroed by
// the caller).
hipError_t launch_sa_alphabet(const uint8_t* text, uint32_t n, uint32_t* mask, hipStream_t s);
// Round-0 strings of a text of at most 16 distinct bytes: the ranks
// (rank[256]) of the 128 / b characters from i on, b in {1, 2, 4} bits
// each, in 16 bytes, then a word holding the count min(128 / b, n - i)
// (SA_PACKED_LEN bytes per suffix).  blocks: sa_pack_blocks(n, b) words of
// scratch.
hipError_t launch_sa_windows_packed(const uint8_t* text, uint32_t n, const uint8_t* rank, uint32_t b,
                                    uint64_t* blocks, uint8_t* chars, uint64_t* offsets, hipStream_t s);
// Name-pair strings of depth h for the m unfinished suffixes at a.pos (also
// fills a.idx): 8 bytes per string, offsets 8e.
hipError_t launch_sa_pairs(const SaArgs& a, uint32_t h, uint8_t* chars, uint64_t* offsets, hipStream_t s);
// After the round's sort: places the suffixes, renames them and lists the
// unfinished positions (their count goes to part_cnt[sa_tiles(m)]).
hipError_t launch_sa_rename(const SaArgs& a, hipStream_t s);

}  // namespace ss
