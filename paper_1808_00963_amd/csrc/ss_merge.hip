// LCP-aware merging of sorted runs (section 4.3.1: binary LCP-merge,
// Algorithms 4.2-4.4 and Lemma 4.5), re-shaped for a GPU.
//
// The paper merges K runs with an LCP-aware tournament tree walked by one
// thread.  Here the K runs are merged pairwise in ceil(log2 K) rounds; each
// round is two launches over all pairs at once:
//   k_merge_split  one wave per tile of MERGE_TILE outputs finds, by a
//                  64-ary search along the merge path, how many of the
//                  outputs before the tile come from run A;
//   k_merge_tile   one work group per tile stages the tile's two input
//                  windows in LDS with each string's offset, length and first
//                  8 characters (one parallel gather), splits the tile among
//                  its threads by binary searches in LDS, and every thread
//                  runs the LCP-merge over MERGE_PER outputs; the outputs
//                  leave through LDS in coalesced stores.
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

// A string as the merge sees it: index, location and its first 8
// characters (big-endian, zero padded).
struct El {
    uint64_t off;
    uint64_t k0;
    uint32_t x;
    uint32_t len;
};

// Element of string `x`; an index out of range or malformed offsets raise an
// error bit and read as the empty string.
__device__ __forceinline__ El load_el(const MergeArgs& m, uint32_t x) {
    if (x >= m.n_strings) {
        atomicOr(m.err, MERR_INDEX);
        return El{0, 0, x, 0};
    }
    const uint64_t o0 = m.offsets[x], o1 = m.offsets[x + 1];
    if (o1 < o0 || o1 - o0 > MAX_LEN || (o1 > o0 && m.chars == nullptr)) {
        atomicOr(m.err, MERR_OFFSETS);
        return El{0, 0, x, 0};
    }
    const uint32_t len = (uint32_t)(o1 - o0);
    return El{o0, gather_key(m.chars, o0, 0, len), x, len};
}

// LCP of two strings known to share their first h characters: the cached
// first 8 characters decide it when it is below 8, the character array is
// read from depth max(h, 8) otherwise.
__device__ __forceinline__ uint32_t lcp_el(const uint8_t* chars, const El& a, const El& b, uint32_t h) {
    const uint32_t lim = min_u32(a.len, b.len);
    if (h < W) {
        const uint32_t c = common_bytes(a.k0, b.k0);  // padding may match: capped by lim
        if (c < W || lim <= W) return min_u32(c, lim);
        h = W;
    }
    return lcp_from(chars, a.off, a.len, b.off, b.len, h);
}

__device__ __forceinline__ uint32_t char_at(const uint8_t* chars, const El& e, uint32_t d) {
    return d < W ? (uint32_t)(e.k0 >> (56 - 8 * d)) & 0xFFu : (uint32_t)chars[e.off + d];
}

// Order of two strings with LCP l: true when a goes after b.  Equal strings
// go by index, a first when the indices are equal.
__device__ __forceinline__ bool after_el(const uint8_t* chars, const El& a, const El& b, uint32_t l) {
    if (l == a.len && l == b.len) return a.x > b.x;
    if (l == a.len) return false;
    if (l == b.len) return true;
    return char_at(chars, a, l) > char_at(chars, b, l);
}

__device__ __forceinline__ bool after_full(const uint8_t* chars, const El& a, const El& b) {
    return after_el(chars, a, b, lcp_el(chars, a, b, 0));
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
    uint64_t k0[MERGE_TILE];
    uint32_t x[MERGE_TILE];
    uint32_t lcp[MERGE_TILE];
    uint32_t len[MERGE_TILE];
    uint32_t ox[MERGE_TILE];
    uint32_t ol[MERGE_TILE];
};

__device__ __forceinline__ El sm_el(const SmMerge& sm, uint32_t e) {
    return El{sm.off[e], sm.k0[e], sm.x[e], sm.len[e]};
}

}  // namespace

// Merge-path split at the start of every tile: the first i in [lo, hi] with
// A[i] after B[k-1-i] (A[0..i) and B[0..k-i) are the first k outputs).  The
// predicate is monotone in i; each step probes 64 evenly spaced candidates
// at once, one per lane, and keeps the gap before the first true one.
__global__ __launch_bounds__(MERGE_BLOCK) void k_merge_split(MergeArgs m) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t t = blockIdx.x * (MERGE_BLOCK / 64) + (threadIdx.x >> 6);
    if (t >= m.n_tiles) return;  // uniform per wave
    const MergeTask T = m.tasks[find_task(m, t)];
    const uint32_t k = (t - T.tile0) * MERGE_TILE;
    const uint32_t* pa = m.src_perm + T.a;
    const uint32_t* pb = pa + T.na;
    uint32_t lo = k > T.nb ? k - T.nb : 0u, hi = min_u32(k, T.na);
    while (lo < hi) {
        const uint32_t step = (hi - lo + 63) / 64;
        const uint32_t q = lo + lane * step;
        bool pred = false;
        if (q < hi) pred = after_full(m.chars, load_el(m, pa[q]), load_el(m, pb[k - 1 - q]));
        const uint64_t mask = __ballot(pred);
        if (mask == 0) {
            const uint32_t nv = (hi - lo + step - 1) / step;  // probes below hi
            lo += (nv - 1) * step + 1;
        } else {
            const uint32_t f = (uint32_t)__builtin_ctzll(mask);
            if (f == 0) {
                hi = lo;
            } else {
                hi = lo + f * step;
                lo += (f - 1) * step + 1;
            }
        }
    }
    if (lane == 0) m.split[t] = lo;
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

    // the two windows, A at [0, nA) and B at [nA, n), with string data
    for (uint32_t e = threadIdx.x; e < n; e += MERGE_BLOCK) {
        const bool in_a = e < nA;
        const uint32_t x = in_a ? pa[i0 + e] : pb[j0 + e - nA];
        const uint32_t l = in_a ? la[i0 + e] : lb[j0 + e - nA];
        const El el = load_el(m, x);
        sm.x[e] = x;
        sm.lcp[e] = l;
        sm.off[e] = el.off;
        sm.len[e] = el.len;
        sm.k0[e] = el.k0;
    }
    __syncthreads();

    const uint32_t s0 = threadIdx.x * MERGE_PER;
    if (s0 < n) {
        const uint32_t s1 = min_u32(s0 + MERGE_PER, n);
        // this thread's split inside the tile
        uint32_t i = s0 > nB ? s0 - nB : 0u, hi = min_u32(s0, nA);
        while (i < hi) {
            const uint32_t mid = (i + hi) >> 1;
            if (after_full(m.chars, sm_el(sm, mid), sm_el(sm, nA + s0 - 1 - mid))) hi = mid;
            else i = mid + 1;
        }
        uint32_t j = s0 - i;
        // LCPs of the heads with the string output last (p), which may lie
        // before the tile
        uint32_t ha = 0, hb = 0;
        const uint32_t gi = i0 + i, gj = j0 + j;
        if (gi > 0 || gj > 0) {
            const El pa_el = gi == 0 ? El{} : (i > 0 ? sm_el(sm, i - 1) : load_el(m, pa[gi - 1]));
            const El pb_el = gj == 0 ? El{} : (j > 0 ? sm_el(sm, nA + j - 1) : load_el(m, pb[gj - 1]));
            const bool p_is_a = gj == 0 || (gi > 0 && after_full(m.chars, pa_el, pb_el));
            if (p_is_a) {
                if (i < nA) ha = sm.lcp[i];
                if (j < nB) hb = lcp_el(m.chars, pa_el, sm_el(sm, nA + j), 0);
            } else {
                if (j < nB) hb = sm.lcp[nA + j];
                if (i < nA) ha = lcp_el(m.chars, pb_el, sm_el(sm, i), 0);
            }
        }
        for (uint32_t s = s0; s < s1; ++s) {
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
                const El a = sm_el(sm, i), b = sm_el(sm, nA + j);
                const uint32_t hab = lcp_el(m.chars, a, b, ha);
                take_a = !after_el(m.chars, a, b, hab);
                h = ha;
                if (take_a) hb = hab;
                else ha = hab;
            }
            sm.ox[s] = take_a ? sm.x[i] : sm.x[nA + j];
            sm.ol[s] = k0 + s == 0 ? 0u : h;
            if (take_a) {
                ++i;
                if (i < nA) ha = sm.lcp[i];
            } else {
                ++j;
                if (j < nB) hb = sm.lcp[nA + j];
            }
        }
    }
    __syncthreads();
    uint32_t* op = m.dst_perm + T.a + k0;
    uint32_t* ol = m.dst_lcp + T.a + k0;
    for (uint32_t e = threadIdx.x; e < n; e += MERGE_BLOCK) {
        op[e] = sm.ox[e];
        ol[e] = sm.ol[e];
    }
}

hipError_t launch_merge_split(const MergeArgs& m, hipStream_t s) {
    if (m.n_tiles == 0) return hipSuccess;
    constexpr uint32_t waves = MERGE_BLOCK / 64;
    hipLaunchKernelGGL(k_merge_split, dim3((m.n_tiles + waves - 1) / waves), dim3(MERGE_BLOCK), 0, s, m);
    return hipGetLastError();
}

hipError_t launch_merge_tiles(const MergeArgs& m, hipStream_t s) {
    if (m.n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge_tile, dim3(m.n_tiles), dim3(MERGE_BLOCK), 0, s, m);
    return hipGetLastError();
}

}  // namespace ss
