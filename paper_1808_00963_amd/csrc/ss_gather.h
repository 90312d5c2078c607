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
// shorter length).
__device__ __forceinline__ uint32_t lcp_from(const uint8_t* chars, uint64_t oa, uint32_t la, uint64_t ob, uint32_t lb,
                                             uint32_t from) {
    const uint32_t limit = la < lb ? la : lb;
    uint32_t d = from;
    while (d < limit) {
        const uint64_t ka = gather_key(chars, oa, d, la), kb = gather_key(chars, ob, d, lb);
        if (ka != kb) {
            const uint32_t c = d + common_bytes(ka, kb);
            return c < limit ? c : limit;
        }
        d += W;
    }
    return limit;
}

}  // namespace ss
