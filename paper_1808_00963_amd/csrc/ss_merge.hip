// LCP-aware merging of sorted runs (section 4.3.1: binary LCP-merge,
// Algorithms 4.2-4.4 and Lemma 4.5), re-shaped for a GPU.
//
// The paper merges K runs with an LCP-aware tournament tree walked by one
// thread.  Here the K runs are merged pairwise in ceil(log2 K) rounds; each
// round is two launches over all pairs at once:
//   k_merge_split   one thread per chunk of MERGE_CHUNK outputs finds, by a
//                   binary search along the merge path, how many of the
//                   first k outputs come from run A;
//   k_merge_chunks  one thread per chunk runs the LCP-merge from that point
//                   for MERGE_CHUNK steps.
// In the LCP-merge the heads a, b of the two runs carry h_a = LCP(p, a) and
// h_b = LCP(p, b), p being the string output last.  By Lemma 4.5, h_a > h_b
// means a < b and LCP(a, b) = h_b, so a is output with LCP h_a and h_b stays
// valid for the new p; only h_a == h_b needs characters, compared from depth
// h_a on.  The loser's LCP becomes the LCP of a and b; the winner's successor
// takes the LCP its run stores.  Equal strings are ordered by string index
// (the sort's order), run A first for the very same index.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ss_device.h"
#include "ss_gather.h"
#include "ss_internal.h"

namespace ss {

namespace {

struct StrRef {
    uint64_t off;
    uint32_t len;
};

// (offset, length) of string `idx`; an index out of range or malformed
// offsets raise an error bit and read as the empty string.
__device__ __forceinline__ StrRef load_str(const MergeArgs& m, uint32_t idx) {
    if (idx >= m.n_strings) {
        atomicOr(m.err, MERR_INDEX);
        return {0, 0};
    }
    const uint64_t o0 = m.offsets[idx], o1 = m.offsets[idx + 1];
    if (o1 < o0 || o1 - o0 > MAX_LEN || (o1 > o0 && m.chars == nullptr)) {
        atomicOr(m.err, MERR_OFFSETS);
        return {0, 0};
    }
    return {o0, (uint32_t)(o1 - o0)};
}

// Decides the order of two strings that share their first h characters
// (h = their LCP): true when x is ordered after y.  Equal strings go by
// index, x first when the indices are equal.
__device__ __forceinline__ bool after_at(const uint8_t* chars, StrRef x, uint32_t xi, StrRef y, uint32_t yi,
                                         uint32_t h) {
    if (h == x.len && h == y.len) return xi > yi;
    if (h == x.len) return false;
    if (h == y.len) return true;
    return chars[x.off + h] > chars[y.off + h];
}

__device__ __forceinline__ uint32_t find_task(const MergeArgs& m, uint32_t c) {
    uint32_t lo = 0, hi = m.n_tasks;  // last task with chunk0 <= c
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (m.tasks[mid].chunk0 <= c) lo = mid;
        else hi = mid;
    }
    return lo;
}

}  // namespace

__global__ __launch_bounds__(MERGE_BLOCK) void k_merge_split(MergeArgs m) {
    const uint32_t c = blockIdx.x * MERGE_BLOCK + threadIdx.x;
    if (c >= m.n_chunks) return;
    const MergeTask T = m.tasks[find_task(m, c)];
    const uint32_t k = (c - T.chunk0) * MERGE_CHUNK;
    const uint32_t* pa = m.src_perm + T.a;
    const uint32_t* pb = pa + T.na;
    // smallest i with A[i] after B[k-1-i]: A[0..i) and B[0..k-i) are the
    // first k outputs
    uint32_t lo = k > T.nb ? k - T.nb : 0u, hi = min_u32(k, T.na);
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        const uint32_t xa = pa[mid], xb = pb[k - 1 - mid];
        const StrRef sa = load_str(m, xa), sb = load_str(m, xb);
        const uint32_t h = lcp_from(m.chars, sa.off, sa.len, sb.off, sb.len, 0);
        if (after_at(m.chars, sa, xa, sb, xb, h)) hi = mid;
        else lo = mid + 1;
    }
    m.split[c] = lo;
}

__global__ __launch_bounds__(MERGE_BLOCK) void k_merge_chunks(MergeArgs m) {
    const uint32_t c = blockIdx.x * MERGE_BLOCK + threadIdx.x;
    if (c >= m.n_chunks) return;
    const MergeTask T = m.tasks[find_task(m, c)];
    const uint32_t total = T.na + T.nb;
    uint32_t k = (c - T.chunk0) * MERGE_CHUNK;
    const uint32_t kend = min_u32(k + MERGE_CHUNK, total);
    const uint32_t na = T.na, nb = T.nb;
    uint32_t i = m.split[c];
    if (i > na || k - i > nb || i > k) {
        atomicOr(m.err, MERR_INTERNAL);
        return;
    }
    uint32_t j = k - i;
    const uint32_t* pa = m.src_perm + T.a;
    const uint32_t* la = m.src_lcp + T.a;
    const uint32_t* pb = pa + na;
    const uint32_t* lb = la + na;
    uint32_t* op = m.dst_perm + T.a;
    uint32_t* ol = m.dst_lcp + T.a;

    // heads and their LCPs with the string output last (p)
    uint32_t xa = i < na ? pa[i] : 0u, xb = j < nb ? pb[j] : 0u;
    uint32_t ha = 0, hb = 0;
    StrRef sa{0, 0}, sb{0, 0};
    bool have_a = false, have_b = false;
    if (k > 0) {
        bool p_is_a;
        StrRef sp{0, 0};
        uint32_t xp;
        if (i == 0 || j == 0) {
            p_is_a = j == 0;
            xp = p_is_a ? pa[i - 1] : pb[j - 1];
            sp = load_str(m, xp);
        } else {
            const uint32_t x1 = pa[i - 1], x2 = pb[j - 1];
            const StrRef s1 = load_str(m, x1), s2 = load_str(m, x2);
            const uint32_t h = lcp_from(m.chars, s1.off, s1.len, s2.off, s2.len, 0);
            p_is_a = after_at(m.chars, s1, x1, s2, x2, h);
            xp = p_is_a ? x1 : x2;
            sp = p_is_a ? s1 : s2;
        }
        if (p_is_a) {
            if (i < na) ha = la[i];
            if (j < nb) {
                sb = load_str(m, xb);
                have_b = true;
                hb = lcp_from(m.chars, sp.off, sp.len, sb.off, sb.len, 0);
            }
        } else {
            if (j < nb) hb = lb[j];
            if (i < na) {
                sa = load_str(m, xa);
                have_a = true;
                ha = lcp_from(m.chars, sp.off, sp.len, sa.off, sa.len, 0);
            }
        }
    }

    for (; k < kend; ++k) {
        bool take_a;
        uint32_t h;
        if (j >= nb) {
            take_a = true;
            h = ha;
        } else if (i >= na) {
            take_a = false;
            h = hb;
        } else if (ha != hb) {
            // Lemma 4.5: the head with the longer LCP to p is the smaller
            take_a = ha > hb;
            h = take_a ? ha : hb;
        } else {
            if (!have_a) sa = load_str(m, xa), have_a = true;
            if (!have_b) sb = load_str(m, xb), have_b = true;
            const uint32_t hab = lcp_from(m.chars, sa.off, sa.len, sb.off, sb.len, ha);
            take_a = !after_at(m.chars, sa, xa, sb, xb, hab);
            h = ha;
            if (take_a) hb = hab;
            else ha = hab;
        }
        const uint32_t x = take_a ? xa : xb;
        if (x >= m.n_strings) atomicOr(m.err, MERR_INDEX);  // every output is checked, compared or not
        op[k] = x;
        ol[k] = k == 0 ? 0u : h;
        if (take_a) {
            ++i;
            if (i < na) xa = pa[i], ha = la[i];
            have_a = false;
        } else {
            ++j;
            if (j < nb) xb = pb[j], hb = lb[j];
            have_b = false;
        }
    }
}

hipError_t launch_merge_split(const MergeArgs& m, hipStream_t s) {
    if (m.n_chunks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge_split, dim3((m.n_chunks + MERGE_BLOCK - 1) / MERGE_BLOCK), dim3(MERGE_BLOCK), 0, s, m);
    return hipGetLastError();
}

hipError_t launch_merge_chunks(const MergeArgs& m, hipStream_t s) {
    if (m.n_chunks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge_chunks, dim3((m.n_chunks + MERGE_BLOCK - 1) / MERGE_BLOCK), dim3(MERGE_BLOCK), 0, s,
                       m);
    return hipGetLastError();
}

}  // namespace ss
