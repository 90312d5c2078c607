// Device helpers shared by the sort and merge kernels: reading 8-byte keys
// from the character array and comparing strings word by word.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "ss_device.h"
#include "ss_internal.h"

namespace ss {

__device__ __forceinline__ uint32_t min_u32(uint32_t a, uint32_t b) { return a < b ? a : b; }

// chars_h(s) on the device (gather_key_with in ss_device.h), read with
// non-temporal loads: string characters are touched once per level.
__device__ __forceinline__ uint64_t gather_key(const uint8_t* chars, uint64_t off, uint32_t h, uint32_t len) {
    return gather_key_with(chars, off, h, len, [](const uint64_t* q) { return __builtin_nontemporal_load(q); });
}

__device__ __forceinline__ uint32_t rem8(uint32_t len, uint32_t h) { return min_u32(len - h, 8u); }

// Length of the common prefix of two strings known to agree on their first
// `from` characters, by comparing 8-byte words (at most `limit` = the
// shorter length, or `cap` when that is smaller).  The first step compares
// one word (it usually decides); later steps load AHEAD words of each
// string at once, so a long common prefix costs one memory round trip per
// AHEAD words (callers with registers to spare take more).
template <uint32_t AHEAD = 1>
__device__ __forceinline__ uint32_t lcp_from(const uint8_t* chars, uint64_t oa, uint32_t la, uint64_t ob, uint32_t lb,
                                             uint32_t from, uint32_t cap = ~0u) {
    const uint32_t limit = min_u32(la < lb ? la : lb, cap);
    uint32_t d = from;
    if (d < limit) {
        const uint64_t ka = gather_key(chars, oa, d, la), kb = gather_key(chars, ob, d, lb);
        if (ka != kb) {
            const uint32_t c = d + common_bytes(ka, kb);
            return c < limit ? c : limit;
        }
        d += W;
    }
    while (d < limit) {
        uint64_t ka[AHEAD], kb[AHEAD];
#pragma unroll
        for (uint32_t u = 0; u < AHEAD; ++u) {  // past an end a key is 0 and reads nothing
            ka[u] = gather_key(chars, oa, d + u * W, la);
            kb[u] = gather_key(chars, ob, d + u * W, lb);
        }
#pragma unroll
        for (uint32_t u = 0; u < AHEAD; ++u) {
            if (ka[u] != kb[u]) {
                const uint32_t c = d + u * W + common_bytes(ka[u], kb[u]);
                return c < limit ? c : limit;
            }
        }
        d += AHEAD * W;
    }
    return limit;
}

// lcp_from with each string's words read once (lcp_stream_with in
// ss_device.h): AHEAD words per string per memory round trip at the
// registers lcp_from needs for half as many.
template <uint32_t AHEAD = 2>
__device__ __forceinline__ uint32_t lcp_stream(const uint8_t* chars, uint64_t oa, uint32_t la, uint64_t ob, uint32_t lb,
                                               uint32_t from, uint32_t cap = ~0u) {
    return lcp_stream_with<AHEAD>(chars, oa, la, ob, lb, from, cap,
                                  [](const uint64_t* q) { return __builtin_nontemporal_load(q); });
}

}  // namespace ss
