// LCP-aware merging of sorted runs (section 4.3.1: binary LCP-merge,
// Algorithms 4.2-4.4 and Lemma 4.5), re-shaped for a GPU.
//
// The paper merges K runs with an LCP-aware tournament tree walked by one
// thread.  Here the K runs are merged pairwise in ceil(log2 K) rounds; each
// round is two launches over all pairs at once:
//   k_merge_split  a group of 16 lanes per tile of MERGE_TILE outputs finds,
//                  by a 16-ary search along the merge path, how many of the
//                  outputs before the tile come from run A;
//   k_merge_tile   one work group per tile stages the tile's two input
//                  windows in LDS with, per string, its location and the 8
//                  characters from the depth all strings of the tile share
//                  (known from the LCP arrays);
//                  it splits the tile among its threads by binary searches
//                  in LDS, and every thread runs the LCP-merge over
//                  MERGE_PER outputs; the outputs leave through LDS in
//                  coalesced stores.  Characters are read from HBM again
//                  only when two strings agree on all 8 cached ones.
// In the LCP-merge the heads a, b of the two runs carry h_a = LCP(p, a) and
// h_b = LCP(p, b), p being the string output last.  By Lemma 4.5, h_a > h_b
// means a < b and LCP(a, b) = h_b, so a is output with LCP h_a and h_b stays
// valid for the new p; only h_a == h_b needs characters, compared from depth
// h_a on (the cached 8 characters first).  The loser's LCP becomes the LCP of
// a and b; the winner's successor takes the LCP its run stores.  Equal
// strings are ordered by string index (the sort's order), run A first for
// the very same index.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ss_device.h"
#include "ss_gather.h"
#include "ss_internal.h"

namespace ss {

namespace {

// A string as the merge compares it: index, location, the 8 characters
// from depth kdep on (big-endian, zero padded) and how many of them the
// string has.
struct El {
    uint64_t off;
    uint64_t key;
    uint32_t x;
    uint32_t len;
    uint32_t rem;
    uint32_t kdep;
};

struct StrRef {
    uint64_t off;
    uint32_t len;
};

// Location of string `x`; an index out of range or malformed offsets raise
// an error bit and read as the empty string.
__device__ __forceinline__ StrRef load_str(const MergeArgs& m, uint32_t x) {
    if (x >= m.n_strings) {
        atomicOr(m.err, MERR_INDEX);
        return {0, 0};
    }
    const uint64_t o0 = m.offsets[x], o1 = m.offsets[x + 1];
    if (o1 < o0 || o1 - o0 > MAX_LEN || (o1 > o0 && m.chars == nullptr)) {
        atomicOr(m.err, MERR_OFFSETS);
        return {0, 0};
    }
    return {o0, (uint32_t)(o1 - o0)};
}

__device__ __forceinline__ El make_el(const uint8_t* chars, StrRef s, uint32_t x, uint32_t d) {
    return El{s.off, gather_key(chars, s.off, d, s.len), x, s.len, s.len > d ? min_u32(s.len - d, W) : 0u, d};
}

__device__ __forceinline__ El load_el(const MergeArgs& m, uint32_t x) { return make_el(m.chars, load_str(m, x), x, 0); }

struct Cmp {
    uint32_t lcp;
    bool after;  // a is ordered after b
};

// Compares two strings from the character array, knowing they share their
// first h characters.  Equal strings go by index, a first for equal indices.
__device__ __forceinline__ Cmp compare_global(const uint8_t* chars, const El& a, const El& b, uint32_t h) {
    const uint32_t l = lcp_from(chars, a.off, a.len, b.off, b.len, h);
    bool after;
    if (l == a.len && l == b.len) after = a.x > b.x;
    else if (l == a.len) after = false;
    else if (l == b.len) after = true;
    else after = chars[a.off + l] > chars[b.off + l];
    return Cmp{l, after};
}

// LCP and order of two strings known to share their first h characters.
// When both carry their words from the same depth d (two strings of one
// tile, which share at least d characters), the words decide unless they
// agree on all 8 characters; the character array is read from there on.
__device__ __forceinline__ Cmp compare_el(const MergeArgs& m, const El& a, const El& b, uint32_t h) {
    const uint32_t d = a.kdep;
    if (d == b.kdep && h < d + W) {
        const uint32_t c = common_bytes(a.key, b.key);
        const uint32_t r = min_u32(a.rem, b.rem);
        if (c < r) return Cmp{d + c, (a.key >> (56 - 8 * c) & 0xFFu) > (b.key >> (56 - 8 * c) & 0xFFu)};
        // the real characters of the shorter word all match
        if (a.rem < W || b.rem < W) {
            if (a.rem == b.rem) return Cmp{d + r, a.x > b.x};  // equal strings
            return Cmp{d + r, a.rem > b.rem};                   // the one ending first is smaller
        }
        h = d + W;
    }
    return compare_global(m.chars, a, b, h);
}

__device__ __forceinline__ uint32_t find_task(const MergeArgs& m, uint32_t t) {
    uint32_t lo = 0, hi = m.n_tasks;  // last task with tile0 <= t
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (m.tasks[mid].tile0 <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

struct SmMerge {
    uint64_t off[MERGE_TILE];
    uint64_t key[MERGE_TILE];  // 8 characters from the tile's common depth
    uint32_t len[MERGE_TILE];
    uint32_t x[MERGE_TILE];    // string index; the output's after the merge
    uint32_t lcp[MERGE_TILE];  // LCP with the run predecessor; the output's after the merge
    uint8_t rem[MERGE_TILE];   // characters of the string inside its key
    uint32_t depth;            // characters shared by all strings of the tile
};

__device__ __forceinline__ El sm_el(const SmMerge& sm, uint32_t e, uint32_t d) {
    return El{sm.off[e], sm.key[e], sm.x[e], sm.len[e], sm.rem[e], d};
}

}  // namespace

// Merge-path split at the start of every tile: the first i in [lo, hi] with
// A[i] after B[k-1-i] (A[0..i) and B[0..k-i) are the first k outputs).  The
// predicate is monotone in i; a group of SPLIT_LANES lanes searches one
// boundary, each step probing SPLIT_LANES evenly spaced candidates at once
// and keeping the gap before the first true one.
constexpr uint32_t SPLIT_LANES = 16;

__global__ __launch_bounds__(MERGE_BLOCK) void k_merge_split(MergeArgs m) {
    const uint32_t lane = threadIdx.x & (SPLIT_LANES - 1);
    const uint32_t group_shift = (threadIdx.x & 63u) & ~(SPLIT_LANES - 1);  // first lane of the group in the wave
    const uint32_t t = blockIdx.x * (MERGE_BLOCK / SPLIT_LANES) + threadIdx.x / SPLIT_LANES;
    const bool live = t < m.n_tiles;  // groups past the end idle through the ballots
    MergeTask T{0, 0, 0, 0};
    if (live) T = m.tasks[find_task(m, t)];
    const uint32_t k = live ? (t - T.tile0) * MERGE_TILE : 0u;
    const uint32_t* pa = m.src_perm + T.a;
    const uint32_t* pb = pa + T.na;
    uint32_t lo = k > T.nb ? k - T.nb : 0u, hi = min_u32(k, T.na);
    // every lane of the wave stays in the loop until all its groups are done
    for (;;) {
        const bool active = lo < hi;
        if (__ballot(active) == 0) break;
        bool pred = false;
        uint32_t step = 1;
        if (active) {
            step = (hi - lo + SPLIT_LANES - 1) / SPLIT_LANES;
            const uint32_t q = lo + lane * step;
            if (q < hi) pred = compare_el(m, load_el(m, pa[q]), load_el(m, pb[k - 1 - q]), 0).after;
        }
        const uint32_t mask = (uint32_t)(__ballot(pred) >> group_shift) & ((1u << SPLIT_LANES) - 1);
        if (active) {
            if (mask == 0) {
                const uint32_t nv = (hi - lo + step - 1) / step;  // probes below hi
                lo += (nv - 1) * step + 1;
            } else {
                const uint32_t f = (uint32_t)__builtin_ctz(mask);
                if (f == 0) {
                    hi = lo;
                } else {
                    hi = lo + f * step;
                    lo += (f - 1) * step + 1;
                }
            }
        }
    }
    if (live && lane == 0) {
        m.split[t] = lo;
        // LCP of the first strings of the tile's two windows, A[lo] and
        // B[k-lo] (0 when a window is empty past the run's end)
        uint32_t c = 0;
        if (lo < T.na && k - lo < T.nb) c = compare_el(m, load_el(m, pa[lo]), load_el(m, pb[k - lo]), 0).lcp;
        m.cross[t] = c;
    }
}

__global__ __launch_bounds__(MERGE_BLOCK) void k_merge_tile(MergeArgs m) {
    __shared__ SmMerge sm;
    const uint32_t t = blockIdx.x;
    const MergeTask T = m.tasks[find_task(m, t)];
    const uint32_t total = T.na + T.nb;
    const uint32_t last = T.tile0 + (total + MERGE_TILE - 1) / MERGE_TILE - 1;
    const uint32_t k0 = (t - T.tile0) * MERGE_TILE;
    const uint32_t k1 = min_u32(k0 + MERGE_TILE, total);
    const uint32_t i0 = m.split[t];
    const uint32_t i1 = t < last ? m.split[t + 1] : T.na;
    if (!(i0 <= k0 && i1 <= k1 && i0 <= i1 && i1 <= T.na && k0 - i0 <= k1 - i1 && k1 - i1 <= T.nb)) {
        if (threadIdx.x == 0) atomicOr(m.err, MERR_INTERNAL);
        return;  // uniform over the work group
    }
    const uint32_t j0 = k0 - i0;
    const uint32_t nA = i1 - i0, n = k1 - k0, nB = n - nA;
    const uint32_t* pa = m.src_perm + T.a;
    const uint32_t* la = m.src_lcp + T.a;
    const uint32_t* pb = pa + T.na;
    const uint32_t* lb = la + T.na;

    // The two windows, A at [0, nA) and B at [nA, n).  Each step is issued
    // for all of a thread's elements before the next (dependent) one.
    static_assert(MERGE_TILE == MERGE_PER * MERGE_BLOCK, "one element per thread and step");
    uint32_t xs[MERGE_PER];
    StrRef str[MERGE_PER];
#pragma unroll
    for (uint32_t r = 0; r < MERGE_PER; ++r) {
        const uint32_t e = threadIdx.x + r * MERGE_BLOCK;
        xs[r] = 0;
        if (e < n) {
            const bool in_a = e < nA;
            xs[r] = in_a ? pa[i0 + e] : pb[j0 + e - nA];
            sm.lcp[e] = in_a ? la[i0 + e] : lb[j0 + e - nA];
        }
    }
    if (threadIdx.x == 0) sm.depth = ~0u;
    uint32_t lmin = ~0u;  // LCPs inside the windows (not at a window's first string)
#pragma unroll
    for (uint32_t r = 0; r < MERGE_PER; ++r) {
        const uint32_t e = threadIdx.x + r * MERGE_BLOCK;
        str[r] = StrRef{0, 0};
        if (e < n) {
            str[r] = load_str(m, xs[r]);
            sm.x[e] = xs[r];
            sm.off[e] = str[r].off;
            sm.len[e] = str[r].len;
            if (e != 0 && e != nA) lmin = min_u32(lmin, sm.lcp[e]);
        }
    }
    __syncthreads();
    atomicMin(&sm.depth, lmin);
    __syncthreads();
    // Every string of the tile shares `depth` characters: within a window
    // the minimum of its LCPs, across the windows via their first strings.
    uint32_t depth = sm.depth;
    if (nA > 0 && nB > 0) depth = min_u32(depth, m.cross[t]);
    if (depth == ~0u) depth = 0;  // a single string
#pragma unroll
    for (uint32_t r = 0; r < MERGE_PER; ++r) {
        const uint32_t e = threadIdx.x + r * MERGE_BLOCK;
        if (e < n) {
            const El el = make_el(m.chars, str[r], xs[r], depth);
            sm.key[e] = el.key;
            sm.rem[e] = (uint8_t)el.rem;
        }
    }
    __syncthreads();

    // this thread's outputs [s0, s0 + MERGE_PER) of the tile, kept in
    // registers until every thread is done reading the windows
    const uint32_t s0 = threadIdx.x * MERGE_PER;
    uint32_t ox[MERGE_PER], ol[MERGE_PER];
    if (s0 < n) {
        // this thread's split inside the tile
        uint32_t i = s0 > nB ? s0 - nB : 0u, hi = min_u32(s0, nA);
        while (i < hi) {
            const uint32_t mid = (i + hi) >> 1;
            if (compare_el(m, sm_el(sm, mid, depth), sm_el(sm, nA + s0 - 1 - mid, depth), 0).after) hi = mid;
            else i = mid + 1;
        }
        uint32_t j = s0 - i;
        // LCPs of the heads with the string output last (p), which may lie
        // before the tile
        uint32_t ha = 0, hb = 0;
        const uint32_t gi = i0 + i, gj = j0 + j;
        if (gi > 0 || gj > 0) {
            const El pa_el = gi == 0 ? El{0, 0, 0, 0, 0, 0} : (i > 0 ? sm_el(sm, i - 1, depth) : load_el(m, pa[gi - 1]));
            const El pb_el = gj == 0 ? El{0, 0, 0, 0, 0, 0} : (j > 0 ? sm_el(sm, nA + j - 1, depth) : load_el(m, pb[gj - 1]));
            const bool p_is_a = gj == 0 || (gi > 0 && compare_el(m, pa_el, pb_el, 0).after);
            if (p_is_a) {
                if (i < nA) ha = sm.lcp[i];
                if (j < nB) hb = compare_el(m, pa_el, sm_el(sm, nA + j, depth), 0).lcp;
            } else {
                if (j < nB) hb = sm.lcp[nA + j];
                if (i < nA) ha = compare_el(m, pb_el, sm_el(sm, i, depth), 0).lcp;
            }
        }
#pragma unroll
        for (uint32_t r = 0; r < MERGE_PER; ++r) {
            if (s0 + r < n) {
                bool take_a;
                uint32_t h;
                if (j >= nB) {
                    take_a = true;
                    h = ha;
                } else if (i >= nA) {
                    take_a = false;
                    h = hb;
                } else if (ha != hb) {
                    // Lemma 4.5: the head with the longer LCP to p is the smaller
                    take_a = ha > hb;
                    h = take_a ? ha : hb;
                } else {
                    const Cmp c = compare_el(m, sm_el(sm, i, depth), sm_el(sm, nA + j, depth), ha);
                    take_a = !c.after;
                    h = ha;
                    if (take_a) hb = c.lcp;
                    else ha = c.lcp;
                }
                ox[r] = take_a ? sm.x[i] : sm.x[nA + j];
                ol[r] = k0 + s0 + r == 0 ? 0u : h;
                if (take_a) {
                    ++i;
                    if (i < nA) ha = sm.lcp[i];
                } else {
                    ++j;
                    if (j < nB) hb = sm.lcp[nA + j];
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < MERGE_PER; ++r) {
        if (s0 + r < n) {
            sm.x[s0 + r] = ox[r];
            sm.lcp[s0 + r] = ol[r];
        }
    }
    __syncthreads();
    uint32_t* op = m.dst_perm + T.a + k0;
    uint32_t* olp = m.dst_lcp + T.a + k0;
    for (uint32_t e = threadIdx.x; e < n; e += MERGE_BLOCK) {
        op[e] = sm.x[e];
        olp[e] = sm.lcp[e];
    }
}

hipError_t launch_merge_split(const MergeArgs& m, hipStream_t s) {
    if (m.n_tiles == 0) return hipSuccess;
    constexpr uint32_t groups = MERGE_BLOCK / SPLIT_LANES;
    hipLaunchKernelGGL(k_merge_split, dim3((m.n_tiles + groups - 1) / groups), dim3(MERGE_BLOCK), 0, s, m);
    return hipGetLastError();
}

hipError_t launch_merge_tiles(const MergeArgs& m, hipStream_t s) {
    if (m.n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge_tile, dim3(m.n_tiles), dim3(MERGE_BLOCK), 0, s, m);
    return hipGetLastError();
}

}  // namespace ss
