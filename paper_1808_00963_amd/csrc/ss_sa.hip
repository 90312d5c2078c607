// Suffix array construction by prefix doubling with discarding (section
// 8.2: Observation 8.1, Algorithm 8.1; the discarding of finished suffixes
// of section 8.2.5) with the string sorter as the sorting step.
//
// Names are the paper's h-names (section 8.2.1): the smallest rank, i.e. the
// first suffix-array position, of the group of suffixes equal to depth h.
// Round 0 sorts all suffixes by their first SA_W0 characters: suffix i
// becomes the string T[i .. i + min(SA_W0, n - i)), so a suffix ending inside
// the window keeps its proper-prefix order (a longer first window costs only
// its copy when suffixes differ early and saves doubling rounds when they do
// not).  For a text of at most 16 distinct bytes the window is alphabet
// compressed instead (one of the refinements the paper proposes for string
// sample sort, §4.6.1): each byte becomes its rank among the bytes present,
// b = 1, 2 or 4 bits (the smallest power of two that holds sigma ranks), and
// 128 / b characters are packed big-endian into 16 bytes, followed by a word
// holding the window's character count; the packed codes order the windows
// as the characters do, zero padding makes a shorter window sort first
// unless its continuation is all rank-0 characters, and the count settles
// that case.  Each later round, resolving depth 2h from
// depth h, sorts only the suffixes whose group still holds more than one
// suffix (the others are final and drop out), as the 8-byte strings
//     BE32(name(i)) . BE32(i + h < n ? name(i + h) + 1 : 0)
// (Observation 8.1; 0 stands for the empty suffix past the end, smaller than
// every name).  The sorted strings of the round refill the positions of the
// unfinished groups in order: the first name keeps the groups apart and in
// place, the second orders each group.  A string starts a new group unless
// its LCP with the previous one covers its whole length; every suffix then
// takes the position of its group's first string as its name, and groups of
// one suffix are discarded.  The rounds stop when no group is left: the
// positions hold the suffix array and the names are its inverse.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ss_internal.h"

namespace ss {

namespace {

__device__ __forceinline__ uint32_t min_u32(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint32_t max_u32(uint32_t a, uint32_t b) { return a > b ? a : b; }

// Offset of suffix window i in the round-0 string array: sum over j < i of
// min(SA_W0, n - j).
__device__ __forceinline__ uint64_t window_offset(uint64_t i, uint64_t n) {
    const uint64_t a = n > SA_W0 ? n - SA_W0 : 0;  // windows before a are SA_W0 long
    if (i <= a) return SA_W0 * i;
    const uint64_t k = i - a;  // windows a .. i-1 have lengths n-a, n-a-1, ...
    return SA_W0 * a + k * (n - a) - k * (k - 1) / 2;
}

// One tile's permutation and LCP entries (and the next tile's first),
// staged in LDS with coalesced loads.
struct SmSaTile {
    uint32_t perm[SA_TILE + 1];
    uint32_t lcp[SA_TILE + 1];
};

__device__ __forceinline__ void stage_tile(const SaArgs& a, SmSaTile& t) {
    const uint64_t tile0 = (uint64_t)blockIdx.x * SA_TILE;
    const uint32_t cnt = (uint32_t)min((uint64_t)SA_TILE + 1, (uint64_t)a.m - tile0);
    for (uint32_t j = threadIdx.x; j < cnt; j += SA_BLOCK) {
        t.perm[j] = a.perm[tile0 + j];
        t.lcp[j] = a.lcp[tile0 + j];
    }
    __syncthreads();
}

// Sorted element k (j inside the tile) starts a group: the first one, or its
// LCP with the previous string is shorter than its own length.
__device__ __forceinline__ bool starts_group(const SaArgs& a, const SmSaTile& t, uint64_t k, uint32_t j) {
    if (k == 0) return true;
    const uint32_t len = !a.round0 ? 8u : a.round0_len ? a.round0_len : min_u32(SA_W0, a.n - t.perm[j]);
    return t.lcp[j] < len;
}

// Element k stays for the next round: its group has another element.
__device__ __forceinline__ bool keeps(const SaArgs& a, const SmSaTile& t, uint64_t k, uint32_t j) {
    return !(starts_group(a, t, k, j) && (k + 1 == a.m || starts_group(a, t, k + 1, j + 1)));
}

struct Scan2 {
    uint32_t mx;   // largest group-start element index so far
    uint32_t cnt;  // kept elements so far
};

// Inclusive (max, sum) scan of one pair per thread over the work group.
__device__ __forceinline__ Scan2 block_scan2(Scan2 v, Scan2* buf) {
    buf[threadIdx.x] = v;
    __syncthreads();
    for (uint32_t d = 1; d < SA_BLOCK; d <<= 1) {
        Scan2 add{0, 0};
        if (threadIdx.x >= d) add = buf[threadIdx.x - d];
        __syncthreads();
        buf[threadIdx.x].mx = max_u32(buf[threadIdx.x].mx, add.mx);
        buf[threadIdx.x].cnt += add.cnt;
        __syncthreads();
    }
    const Scan2 r = buf[threadIdx.x];
    __syncthreads();
    return r;
}

// This thread's elements and their (max group start, kept count).
__device__ __forceinline__ Scan2 thread_part(const SaArgs& a, const SmSaTile& t, uint32_t* starts, uint32_t* kept) {
    Scan2 v{0, 0};
    uint32_t s = 0, kb = 0;
    const uint32_t j0 = threadIdx.x * SA_PER;
    const uint64_t base = (uint64_t)blockIdx.x * SA_TILE + j0;
    for (uint32_t r = 0; r < SA_PER; ++r) {
        const uint64_t k = base + r;
        if (k >= a.m) break;
        if (starts_group(a, t, k, j0 + r)) {
            s |= 1u << r;
            v.mx = (uint32_t)k;
        }
        if (keeps(a, t, k, j0 + r)) {
            kb |= 1u << r;
            ++v.cnt;
        }
    }
    *starts = s;
    *kept = kb;
    return v;
}

}  // namespace

__global__ __launch_bounds__(SA_BLOCK) void k_sa_windows(const uint8_t* __restrict__ text, uint32_t n,
                                                        uint8_t* __restrict__ chars, uint64_t* __restrict__ offsets) {
    const uint32_t i = blockIdx.x * SA_BLOCK + threadIdx.x;
    if (i > n) return;
    const uint64_t off = window_offset(i, n);
    offsets[i] = off;
    if (i == n) return;
    const uint32_t len = min_u32(SA_W0, n - i);
    if (len < SA_W0) {
        for (uint32_t b = 0; b < len; ++b) chars[off + b] = text[i + b];
        return;
    }
    // a full window starts at a multiple of 8 (off = SA_W0 * i): funnel the
    // aligned words that hold its characters into aligned stores; every
    // word read holds at least one character of the window
    static_assert(SA_W0 % 8 == 0, "window stores are whole words");
    const uint64_t* src = (const uint64_t*)((uintptr_t)(text + i) & ~(uintptr_t)7);
    const uint32_t sh = (uint32_t)((uintptr_t)(text + i) & 7);
    uint64_t* dst = (uint64_t*)(chars + off);
    uint64_t w = src[0];
#pragma unroll
    for (uint32_t q = 0; q < SA_W0 / 8; ++q) {
        const uint64_t nx = (sh != 0) ? src[q + 1] : 0ull;  // holds window byte 8q + 8 - sh
        dst[q] = sh ? (w >> (8 * sh)) | (nx << (64 - 8 * sh)) : w;
        w = sh ? nx : src[q + 1 < SA_W0 / 8 ? q + 1 : q];
    }
}

// Which byte values occur in the text (bit v of mask[v / 32]).
__global__ __launch_bounds__(SA_BLOCK) void k_sa_alphabet(const uint8_t* __restrict__ text, uint32_t n,
                                                         uint32_t* __restrict__ mask) {
    __shared__ uint32_t seen[8];
    if (threadIdx.x < 8) seen[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t stride = gridDim.x * SA_BLOCK;
    for (uint32_t i = blockIdx.x * SA_BLOCK + threadIdx.x; i < n; i += stride) {
        const uint32_t v = text[i];
        atomicOr(&seen[v >> 5], 1u << (v & 31));
    }
    __syncthreads();
    if (threadIdx.x < 8 && seen[threadIdx.x]) atomicOr(&mask[threadIdx.x], seen[threadIdx.x]);
}

// Packed ranks of 64 / b consecutive characters per word: block q holds
// the characters from q * 64 / b on, the first at the top; positions past
// the text are rank 0.
__global__ __launch_bounds__(SA_BLOCK) void k_sa_pack_blocks(const uint8_t* __restrict__ text, uint32_t n,
                                                            const uint8_t* __restrict__ rank, uint32_t b,
                                                            uint32_t n_blocks, uint64_t* __restrict__ blocks) {
    __shared__ uint8_t rk[256];
    rk[threadIdx.x] = rank[threadIdx.x];  // SA_BLOCK == 256
    __syncthreads();
    const uint32_t q = blockIdx.x * SA_BLOCK + threadIdx.x;
    if (q >= n_blocks) return;
    const uint32_t per = 64 / b;
    const uint64_t i0 = (uint64_t)q * per;
    uint64_t w = 0;
    for (uint32_t c = 0; c < per; ++c) {
        const uint64_t i = i0 + c;
        w = (w << b) | (i < n ? rk[text[i]] : 0u);
    }
    blocks[q] = w;
}

// Round-0 strings of a small alphabet: window i = ranks of the 128 / b
// characters from i on (rank 0 past the end) as 16 big-endian bytes, then
// the count min(128 / b, n - i) in the top byte of a third word;
// SA_PACKED_LEN bytes per suffix, every word aligned.
__global__ __launch_bounds__(SA_BLOCK) void k_sa_windows_packed(const uint64_t* __restrict__ blocks, uint32_t n,
                                                               uint32_t b, uint64_t* __restrict__ out,
                                                               uint64_t* __restrict__ offsets) {
    const uint32_t i = blockIdx.x * SA_BLOCK + threadIdx.x;
    if (i > n) return;
    offsets[i] = (uint64_t)SA_PACKED_LEN * i;
    if (i == n) return;
    const uint32_t per = 64 / b;
    const uint32_t q = i / per, sh = (i % per) * b;
    const uint64_t w0 = blocks[q], w1 = blocks[q + 1], w2 = blocks[q + 2];
    const uint64_t hi = sh ? (w0 << sh) | (w1 >> (64 - sh)) : w0;
    const uint64_t lo = sh ? (w1 << sh) | (w2 >> (64 - sh)) : w1;
    const uint64_t k = min_u32(2 * per, n - i);
    uint64_t* p = out + (uint64_t)(SA_PACKED_LEN / 8) * i;
    p[0] = __builtin_bswap64(hi);
    p[1] = __builtin_bswap64(lo);
    p[2] = __builtin_bswap64(k << 56);
}

// Name pairs of the unfinished suffixes: element e is the suffix at
// suffix-array position pos[e].
__global__ __launch_bounds__(SA_BLOCK) void k_sa_pairs(SaArgs a, uint32_t h, uint64_t* __restrict__ chars,
                                                      uint64_t* __restrict__ offsets) {
    const uint32_t e = blockIdx.x * SA_BLOCK + threadIdx.x;
    if (e > a.m) return;
    offsets[e] = 8ull * e;
    if (e == a.m) return;
    const uint32_t i = a.sa[a.pos[e]];
    a.idx[e] = i;
    const uint64_t first = a.names[i];
    const uint64_t second = (uint64_t)h < (uint64_t)(a.n - i) ? (uint64_t)a.names[i + h] + 1u : 0u;
    chars[e] = __builtin_bswap64((first << 32) | second);  // big-endian: the first name leads
}

// Per tile of SA_TILE sorted elements: the last group start and the number
// of kept elements.
__global__ __launch_bounds__(SA_BLOCK) void k_sa_tiles(SaArgs a) {
    __shared__ Scan2 buf[SA_BLOCK];
    __shared__ SmSaTile t;
    stage_tile(a, t);
    uint32_t s, kb;
    const Scan2 v = thread_part(a, t, &s, &kb);
    const Scan2 tot = block_scan2(v, buf);
    if (threadIdx.x == SA_BLOCK - 1) {
        a.part_max[blockIdx.x] = tot.mx;
        a.part_cnt[blockIdx.x] = tot.cnt;
    }
}

// Exclusive scans of the tiles' pairs (one work group); the total kept count
// goes to part_cnt[n_tiles].
__global__ __launch_bounds__(SA_BLOCK) void k_sa_scan(uint32_t* part_max, uint32_t* part_cnt, uint32_t n_tiles) {
    __shared__ Scan2 buf[SA_BLOCK];
    Scan2 carry{0, 0};
    for (uint32_t b0 = 0; b0 < n_tiles; b0 += SA_BLOCK) {
        const uint32_t b = b0 + threadIdx.x;
        const Scan2 v = b < n_tiles ? Scan2{part_max[b], part_cnt[b]} : Scan2{0, 0};
        (void)block_scan2(v, buf);  // leaves the inclusive scan in buf
        if (b < n_tiles) {
            // exclusive: the prefix before this tile
            const Scan2 prev = threadIdx.x > 0 ? buf[threadIdx.x - 1] : Scan2{0, 0};
            part_max[b] = max_u32(carry.mx, prev.mx);
            part_cnt[b] = carry.cnt + prev.cnt;
        }
        const Scan2 last = buf[SA_BLOCK - 1];  // block_scan2 leaves the inclusive scan in buf
        carry.mx = max_u32(carry.mx, last.mx);
        carry.cnt += last.cnt;
        __syncthreads();
    }
    if (threadIdx.x == 0) part_cnt[n_tiles] = carry.cnt;
}

// Places the sorted suffixes, names them by their group's first position and
// lists the positions of the suffixes that stay unfinished.
__global__ __launch_bounds__(SA_BLOCK) void k_sa_apply(SaArgs a) {
    __shared__ Scan2 buf[SA_BLOCK];
    __shared__ SmSaTile t;
    stage_tile(a, t);
    const uint32_t j0 = threadIdx.x * SA_PER;
    const uint64_t base = (uint64_t)blockIdx.x * SA_TILE + j0;
    uint32_t s, kb;
    const Scan2 v = thread_part(a, t, &s, &kb);
    (void)block_scan2(v, buf);  // leaves the inclusive scan in buf
    // exclusive prefix of this thread inside the tile
    const Scan2 prev = threadIdx.x > 0 ? buf[threadIdx.x - 1] : Scan2{0, 0};
    uint32_t start = max_u32(a.part_max[blockIdx.x], prev.mx);
    uint32_t out = a.part_cnt[blockIdx.x] + prev.cnt;
    for (uint32_t r = 0; r < SA_PER; ++r) {
        const uint64_t k = base + r;
        if (k >= a.m) break;
        if ((s >> r) & 1u) start = (uint32_t)k;
        const uint32_t i = a.idx ? a.idx[t.perm[j0 + r]] : t.perm[j0 + r];
        const uint32_t p = a.pos ? a.pos[k] : (uint32_t)k;
        if (a.idx) a.sa[p] = i;  // round 0 sorted straight into the suffix array
        a.names[i] = a.pos ? a.pos[start] : start;
        if ((kb >> r) & 1u) a.next_pos[out++] = p;
    }
}

hipError_t launch_sa_windows(const uint8_t* text, uint32_t n, uint8_t* chars, uint64_t* offsets, hipStream_t s) {
    const uint32_t nb = (uint32_t)(((uint64_t)n + 1 + SA_BLOCK - 1) / SA_BLOCK);
    hipLaunchKernelGGL(k_sa_windows, dim3(nb), dim3(SA_BLOCK), 0, s, text, n, chars, offsets);
    return hipGetLastError();
}

hipError_t launch_sa_alphabet(const uint8_t* text, uint32_t n, uint32_t* mask, hipStream_t s) {
    const uint32_t nb = (uint32_t)std::min<uint64_t>(((uint64_t)n + SA_BLOCK - 1) / SA_BLOCK, 2048u);
    hipLaunchKernelGGL(k_sa_alphabet, dim3(nb ? nb : 1), dim3(SA_BLOCK), 0, s, text, n, mask);
    return hipGetLastError();
}

hipError_t launch_sa_windows_packed(const uint8_t* text, uint32_t n, const uint8_t* rank, uint32_t b,
                                    uint64_t* blocks, uint8_t* chars, uint64_t* offsets, hipStream_t s) {
    const uint32_t n_blocks = sa_pack_blocks(n, b);
    hipLaunchKernelGGL(k_sa_pack_blocks, dim3((n_blocks + SA_BLOCK - 1) / SA_BLOCK), dim3(SA_BLOCK), 0, s, text, n,
                       rank, b, n_blocks, blocks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint32_t nb = (uint32_t)(((uint64_t)n + 1 + SA_BLOCK - 1) / SA_BLOCK);
    hipLaunchKernelGGL(k_sa_windows_packed, dim3(nb), dim3(SA_BLOCK), 0, s, blocks, n, b, (uint64_t*)chars, offsets);
    return hipGetLastError();
}

hipError_t launch_sa_pairs(const SaArgs& a, uint32_t h, uint8_t* chars, uint64_t* offsets, hipStream_t s) {
    const uint32_t nb = (uint32_t)(((uint64_t)a.m + 1 + SA_BLOCK - 1) / SA_BLOCK);
    hipLaunchKernelGGL(k_sa_pairs, dim3(nb), dim3(SA_BLOCK), 0, s, a, h, (uint64_t*)chars, offsets);
    return hipGetLastError();
}

hipError_t launch_sa_rename(const SaArgs& a, hipStream_t s) {
    const uint32_t tiles = sa_tiles(a.m);
    hipLaunchKernelGGL(k_sa_tiles, dim3(tiles), dim3(SA_BLOCK), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sa_scan, dim3(1), dim3(SA_BLOCK), 0, s, a.part_max, a.part_cnt, tiles);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sa_apply, dim3(tiles), dim3(SA_BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace ss
