// Primitive operations of the string sample sort, shared by the gfx950
// kernels and by host-side test entry points (so their logic can be checked
// on the CPU).  Nothing here allocates or launches.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

#define SS_HD __host__ __device__ __forceinline__

namespace ss {

// Characters per machine word: keys hold w = 8 bytes of a string at the
// current depth, most significant byte first ("chars_h", section 4.2.2,
// paragraph "Character Reordering").
constexpr uint32_t W = 8;

// Assembles the 8-byte big-endian key of the bytes starting at byte `sh`
// (0..7) of the little-endian aligned word `w0`, continuing into `w1`, and
// keeps only the first `rem` bytes (rem = characters left in the string,
// clamped to 8); bytes past the string end are zero.
SS_HD uint64_t key_from_words(uint64_t w0, uint64_t w1, uint32_t sh, uint32_t rem) {
    if (rem == 0) return 0;
    uint64_t le = sh ? ((w0 >> (8 * sh)) | (w1 << (64 - 8 * sh))) : w0;
    uint64_t be = __builtin_bswap64(le);
    if (rem >= 8) return be;
    return be & ~(~0ull >> (8 * rem));
}

// chars_h(s): the 8 characters of a string starting at depth h, big-endian,
// zero padded past the end (section 4.2.2, "Character Reordering").  Reads,
// through `load`, the aligned 8-byte word holding the first character and,
// only when the key straddles a word boundary, the next one (it then holds a
// character of the string), so no read touches a word without string data.
// The address arithmetic is the same on the device (non-temporal loads) and
// on the host (plain loads, for the exhaustive CPU test).
template <typename Load>
SS_HD uint64_t gather_key_with(const uint8_t* chars, uint64_t off, uint32_t h, uint32_t len, Load load) {
    uint32_t rem = len > h ? len - h : 0u;
    rem = rem < 8u ? rem : 8u;
    if (rem == 0) return 0;
    const uintptr_t a = (uintptr_t)(chars + off + h);
    const uint64_t* p = (const uint64_t*)(a & ~(uintptr_t)7);
    const uint32_t sh = (uint32_t)(a & 7);
    const uint64_t w0 = load(p);
    const uint64_t w1 = (sh + rem > 8) ? load(p + 1) : 0ull;
    return key_from_words(w0, w1, sh, rem);
}

// Number of leading equal bytes of two big-endian keys (8 when equal).
SS_HD uint32_t common_bytes(uint64_t a, uint64_t b) {
    uint64_t x = a ^ b;
    return x ? (uint32_t)(__builtin_clzll(x) >> 3) : 8u;
}

// Length of the common prefix of two strings a = chars[oa, oa + la) and
// b = chars[ob, ob + lb) that agree on their first `from` characters, at
// most limit = min(la, lb, cap).  The first 8 characters past `from` are
// compared as keys (they usually decide); after that each string's aligned
// words are read once, in steps of AHEAD words per string loaded together,
// and every 8 characters are compared as a little-endian group formed from
// two neighbouring words (the first difference is the lowest differing
// byte).  Like gather_key_with, it reads only words that hold characters
// of the string.
template <uint32_t AHEAD, typename Load>
SS_HD uint32_t lcp_stream_with(const uint8_t* chars, uint64_t oa, uint32_t la, uint64_t ob, uint32_t lb,
                               uint32_t from, uint32_t cap, Load load) {
    uint32_t limit = la < lb ? la : lb;
    limit = limit < cap ? limit : cap;
    uint32_t d = from;
    if (d >= limit) return limit;
    {
        const uint64_t ka = gather_key_with(chars, oa, d, la, load), kb = gather_key_with(chars, ob, d, lb, load);
        if (ka != kb) {
            const uint32_t c = d + common_bytes(ka, kb);
            return c < limit ? c : limit;
        }
        d += 8;
        if (d >= limit) return limit;
    }
    const uintptr_t xa = (uintptr_t)(chars + oa + d), xb = (uintptr_t)(chars + ob + d);
    const uint64_t* pa = (const uint64_t*)(xa & ~(uintptr_t)7);
    const uint64_t* pb = (const uint64_t*)(xb & ~(uintptr_t)7);
    const uint32_t sa = 8 * (uint32_t)(xa & 7), sb = 8 * (uint32_t)(xb & 7);
    // words from pa (pb) on that hold a character of the string
    const uint32_t na = (uint32_t)(((xa & 7) + (la - d) + 7) >> 3), nb = (uint32_t)(((xb & 7) + (lb - d) + 7) >> 3);
    uint64_t ca = load(pa), cb = load(pb);  // they hold character d
    for (uint32_t u = 1;; u += AHEAD) {
        uint64_t wa[AHEAD], wb[AHEAD];
        for (uint32_t v = 0; v < AHEAD; ++v) {
            wa[v] = u + v < na ? load(pa + u + v) : 0ull;
            wb[v] = u + v < nb ? load(pb + u + v) : 0ull;
        }
        for (uint32_t v = 0; v < AHEAD; ++v) {
            const uint64_t ga = sa ? (ca >> sa) | (wa[v] << (64 - sa)) : ca;
            const uint64_t gb = sb ? (cb >> sb) | (wb[v] << (64 - sb)) : cb;
            uint64_t x = ga ^ gb;
            const uint32_t m = limit - d;  // > 0
            if (m < 8) x &= (1ull << (8 * m)) - 1;
            if (x) return d + ((uint32_t)__builtin_ctzll(x) >> 3);
            d += 8;
            if (d >= limit) return limit;
            ca = wa[v];
            cb = wb[v];
        }
    }
}

// Key format of a sort.  Byte keys (bpc = 0): 8 characters per word, as
// above.  Alphabet-compressed keys (alphabet compression, §4.6.1): when the
// strings use at most 15 distinct bytes, a character is coded as 1 + its
// rank among the bytes present, in bpc = 2, 3 or 4 bits, 0 marking the end
// of the string, and a key word holds cpw = 64 / bpc characters (32, 21 or
// 16), most significant first.  The codes keep the byte order and the end
// code is below every character, so keys compare like the strings' next
// cpw characters; equal keys mean equal characters and an equal end.
struct KeyFmt {
    uint32_t bpc;       // 0: byte keys
    uint32_t cpw;       // characters per key word
    uint64_t m[4];      // bytes present (bit c of the 256-bit set)
    uint32_t pre[4];    // bytes present below 64 * i
};
// Builds the compressed format of the byte set `m` (at most 15 members);
// byte keys when the set has fewer than 1 or more than 15 members.
SS_HD KeyFmt key_fmt_of(const uint64_t (&m)[4]) {
    KeyFmt f{};
    uint32_t s = 0;
    for (int i = 0; i < 4; ++i) {
        f.m[i] = m[i];
        f.pre[i] = s;
        s += (uint32_t)__builtin_popcountll(m[i]);
    }
    if (s < 1 || s > 15) {
        f.bpc = 0;
        f.cpw = W;
    } else {
        f.bpc = s <= 3 ? 2u : s <= 7 ? 3u : 4u;
        f.cpw = 64u / f.bpc;
    }
    return f;
}
// Word i (0..3) of the set and the members below it, chosen by selects (a
// per-lane index into the arrays would place them in scratch memory).
SS_HD uint64_t kf_word(const KeyFmt& f, uint32_t i) {
    const uint64_t m0 = f.m[0], m1 = f.m[1], m2 = f.m[2], m3 = f.m[3];
    const uint64_t lo = (i & 1u) ? m1 : m0, hi = (i & 1u) ? m3 : m2;
    return (i & 2u) ? hi : lo;
}
SS_HD uint32_t kf_pre(const KeyFmt& f, uint32_t i) {
    const uint32_t p0 = f.pre[0], p1 = f.pre[1], p2 = f.pre[2], p3 = f.pre[3];
    const uint32_t lo = (i & 1u) ? p1 : p0, hi = (i & 1u) ? p3 : p2;
    return (i & 2u) ? hi : lo;
}
// Code of byte c (1 + rank among the bytes present).
SS_HD uint32_t kf_code(const KeyFmt& f, uint32_t c) {
    const uint32_t i = c >> 6;
    const uint64_t below = kf_word(f, i) & ((1ull << (c & 63)) - 1);  // c & 63 < 64
    return 1u + kf_pre(f, i) + (uint32_t)__builtin_popcountll(below);
}
// Whether byte c is in the set.
SS_HD bool kf_has(const KeyFmt& f, uint32_t c) { return (kf_word(f, c >> 6) >> (c & 63)) & 1u; }
// Characters of a string inside its word at depth h, as kept in a record:
// r = min(len - h, cpw) for byte keys; for compressed keys 8 when the
// string fills the word (r = cpw), else min(r, 7) — the exact count is read
// off the key (kf_chars) where it is needed.  Either way a record's code is
// 8 exactly when the string continues past the word, and equal keys have
// equal codes.
SS_HD uint32_t kf_r(const KeyFmt& f, uint32_t len, uint32_t h) {
    const uint32_t cpw = f.bpc ? f.cpw : W;
    const uint32_t r = len > h ? (len - h < cpw ? len - h : cpw) : 0u;
    if (f.bpc == 0) return r;
    return r == cpw ? W : (r < 7u ? r : 7u);
}
// Characters per key word: the depth step of an equality bucket or a tied run.
SS_HD uint32_t kf_step(const KeyFmt& f) { return f.bpc ? f.cpw : W; }
// Characters of the string inside a compressed key (codes before the first 0).
SS_HD uint32_t kf_chars(const KeyFmt& f, uint64_t key) {
    return key ? (63u - (uint32_t)__builtin_ctzll(key)) / f.bpc + 1u : 0u;
}
// Characters of the word past depth h that a string shares with the key of
// an identical string (equal keys, code rc < 8): rc for byte keys.
SS_HD uint32_t kf_tail(const KeyFmt& f, uint64_t key, uint32_t rc) { return f.bpc ? kf_chars(f, key) : rc; }
// The compressed key of the string [off, off + len) at depth h: its next
// min(len - h, cpw) bytes coded, most significant first, 0 past the end.
// Reads, through `load`, only the aligned words that hold those bytes, all
// of them at once (at most five), aligns them into 8-byte groups and codes
// every character position unrolled for the code width BPC.  *miss is set
// when one of the bytes is not in the set.
template <uint32_t BPC, typename Load>
SS_HD uint64_t gather_packed_fixed(const uint8_t* chars, uint64_t off, uint32_t h, uint32_t len, const KeyFmt& f,
                                   Load load, bool* miss) {
    constexpr uint32_t CPW = 64 / BPC, NG = (CPW + 7) / 8;
    uint32_t rem = len > h ? len - h : 0u;
    rem = rem < CPW ? rem : CPW;
    if (rem == 0) return 0;
    const uintptr_t a = (uintptr_t)(chars + off + h);
    const uint64_t* q = (const uint64_t*)(a & ~(uintptr_t)7);
    const uint32_t sh = (uint32_t)(a & 7), nw = (sh + rem + 7) >> 3;  // words that hold the characters
    uint64_t wd[NG + 1];
    for (uint32_t u = 0; u <= NG; ++u) wd[u] = u < nw ? load(q + u) : 0ull;
    uint64_t key = 0;
    bool bad = false;
    for (uint32_t g = 0; g < NG; ++g) {
        const uint64_t grp = sh ? (wd[g] >> (8 * sh)) | (wd[g + 1] << (64 - 8 * sh)) : wd[g];
        for (uint32_t j = 0; j < 8; ++j) {
            const uint32_t k = 8 * g + j;
            if (k >= CPW) break;
            if (k < rem) {
                const uint32_t c = (uint32_t)(grp >> (8 * j)) & 0xFFu;
                if (!kf_has(f, c)) bad = true;
                key |= (uint64_t)kf_code(f, c) << (64 - BPC * (k + 1));
            }
        }
    }
    if (bad) *miss = true;
    return key;
}
// The same for the code width of f (2, 3 or 4 bits).
template <typename Load>
SS_HD uint64_t gather_packed_with(const uint8_t* chars, uint64_t off, uint32_t h, uint32_t len, const KeyFmt& f,
                                  Load load, bool* miss) {
    if (f.bpc == 2) return gather_packed_fixed<2>(chars, off, h, len, f, load, miss);
    if (f.bpc == 3) return gather_packed_fixed<3>(chars, off, h, len, f, load, miss);
    return gather_packed_fixed<4>(chars, off, h, len, f, load, miss);
}

// LCP contribution of one word: the strings agree on the first
// common_bytes(a, b) characters of the word, but not beyond the end of the
// shorter string (ra, rb = characters of each string inside the word).
SS_HD uint32_t lcp_word(uint64_t a, uint32_t ra, uint64_t b, uint32_t rb) {
    uint32_t c = common_bytes(a, b);
    c = c < ra ? c : ra;
    return c < rb ? c : rb;
}
// Characters a string inside its word shares with the next: lcp_word for
// byte keys; for compressed keys the equal leading codes, or the string's
// characters when the keys are equal.
SS_HD uint32_t kf_lcp_word(const KeyFmt& f, uint64_t a, uint32_t ra, uint64_t b, uint32_t rb) {
    if (f.bpc == 0) return lcp_word(a, ra, b, rb);
    const uint64_t x = a ^ b;
    return x ? (uint32_t)__builtin_clzll(x) / f.bpc : kf_chars(f, a);
}

// Total order on (key, r) pairs: the 8 characters first, then the number
// of characters inside the word, so a string ending inside the word sorts
// before a longer one with the same (zero-padded) bytes.
SS_HD bool kr_greater(uint64_t ka, uint32_t ra, uint64_t kb, uint32_t rb) {
    return ka > kb || (ka == kb && ra > rb);
}

// Lemma 4.1 (section 4.2.2): one-based level-order index of the splitter at
// zero-based in-order ("pre-order" in the paper) position j of a perfect
// binary search tree with d levels (v = 2^d - 1 splitters).  In-order
// position j+1 = rank * 2^(t+1) + 2^t where t = trailing zeros; the vertex
// sits on level d-1-t at position `rank` of that level.
SS_HD uint32_t level_index(uint32_t j, uint32_t d) {
    uint32_t q = j + 1;
    uint32_t t = (uint32_t)__builtin_ctz(q);
    return (1u << (d - 1 - t)) + (q >> (t + 1));
}

// Inverse mapping: zero-based in-order position of level-order vertex l.
SS_HD uint32_t inorder_index(uint32_t l, uint32_t d) {
    uint32_t level = 31u - (uint32_t)__builtin_clz(l);  // floor(log2 l)
    uint32_t rank = l - (1u << level);
    uint32_t t = d - 1 - level;
    return (rank << (t + 1)) + (1u << t) - 1;
}

// Classification (Algorithm 4.1, with the comparison of its descent step
// taken as "go right when c is greater than the splitter"): descend the
// level-order tree tk/tr (one-based, v = 2^d - 1 vertices) using only
// comparisons, giving j = number of splitters smaller than c, then test c
// for equality with the in-order splitter x_j found through level_index.
// Returns the bucket 2j (strictly between x_{j-1} and x_j) or 2j+1 (equal
// to x_j); 2v+1 buckets in total.
// classify_n does the same for N strings at once, their descents
// interleaved so their tree reads overlap.
template <uint32_t N, typename KeyArr, typename RArr>
SS_HD void classify_n(const uint64_t (&c)[N], const uint32_t (&cr)[N], const KeyArr& tk, const RArr& tr, uint32_t d,
                      uint32_t (&b)[N]) {
    uint32_t q[N];
    for (uint32_t u = 0; u < N; ++u) q[u] = 1;
    for (uint32_t l = 0; l < d; ++l) {
        // the splitters' length codes decide only between equal keys, so
        // they are read only by a string whose key equals its splitter's
        uint64_t t[N];
        uint32_t gt[N];
        bool any_eq = false;
        for (uint32_t u = 0; u < N; ++u) t[u] = tk[q[u]];
        for (uint32_t u = 0; u < N; ++u) {
            gt[u] = c[u] > t[u] ? 1u : 0u;
            any_eq |= c[u] == t[u];
        }
        if (any_eq) {
            for (uint32_t u = 0; u < N; ++u)
                if (c[u] == t[u]) gt[u] = cr[u] > (uint32_t)tr[q[u]] ? 1u : 0u;
        }
        for (uint32_t u = 0; u < N; ++u) q[u] = 2 * q[u] + gt[u];
    }
    const uint32_t v = (1u << d) - 1;
    for (uint32_t u = 0; u < N; ++u) {
        const uint32_t j = q[u] - (v + 1);
        b[u] = 2 * j;
        if (j < v) {
            const uint32_t lq = level_index(j, d);
            if (tk[lq] == c[u] && (uint32_t)tr[lq] == cr[u]) b[u] += 1;
        }
    }
}
template <typename KeyArr, typename RArr>
SS_HD uint32_t classify(uint64_t c, uint32_t cr, const KeyArr& tk, const RArr& tr, uint32_t d) {
    const uint64_t cc[1] = {c};
    const uint32_t rr[1] = {cr};
    uint32_t b[1];
    classify_n<1>(cc, rr, tk, tr, d, b);
    return b[0];
}

// One step of the splitter selection heuristic (section 4.2.2, paragraph
// "Sampling"): for a non-empty range [lo, hi) of the sorted sample (sk, sr)
// take the middle sample as the splitter and find the boundaries of the run
// of samples equal to it, so the two sub-ranges exclude it:
//   *mid      = (lo + hi) / 2
//   *left_hi  = first index in [lo, mid] whose sample is not smaller
//   *right_lo = first index in [mid, hi) whose sample is greater (or hi)
// Binary searches replace the paper's linear scans; the result is the same.
template <typename KeyArr, typename RArr>
SS_HD void select_node(const KeyArr& sk, const RArr& sr, uint32_t lo, uint32_t hi, uint32_t* mid,
                       uint32_t* left_hi, uint32_t* right_lo) {
    uint32_t m = (lo + hi) >> 1;
    uint64_t xk = sk[m];
    uint32_t xr = sr[m];
    uint32_t a = lo, b = m;  // lower bound in [lo, m]
    while (a < b) {
        uint32_t c = (a + b) >> 1;
        if (kr_greater(xk, xr, sk[c], sr[c])) a = c + 1; else b = c;
    }
    *left_hi = a;
    a = m + 1; b = hi;       // upper bound in [m+1, hi)
    while (a < b) {
        uint32_t c = (a + b) >> 1;
        if (kr_greater(sk[c], sr[c], xk, xr)) b = c; else a = c + 1;
    }
    *right_lo = a;
    *mid = m;
}

// Number of splitter levels d for a segment of `size` strings: about
// size / bucket_target splitters, as a power of two minus one, within
// [1, max_logv].
SS_HD uint32_t choose_logv(uint32_t size, uint32_t bucket_target, uint32_t max_logv) {
    uint32_t q = size / (bucket_target ? bucket_target : 1);
    uint32_t d = q >= 2 ? 31u - (uint32_t)__builtin_clz(q) : 1u;
    if (d < 1) d = 1;
    if (d > max_logv) d = max_logv;
    return d;
}

}  // namespace ss
