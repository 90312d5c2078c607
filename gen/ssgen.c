/*
 * Seeded synthetic string-set generators.
 *
 * This module is shared by the GPU sorter's tests/benchmarks and by the CPU
 * oracle's tests.  It only produces inputs (an offsets array and a character
 * array); it contains none of the sorting or LCP arithmetic.
 *
 * Every string is generated from its own counter-based random stream
 * (SplitMix64 seeded with a hash of (seed, stream, index)), so the output is
 * independent of the number of threads.
 *
 * Models (synthetic stand-ins for the paper's inputs, sections 2.3.2 and 6.4):
 *   0  "random":  lengths uniform in [1,32], bytes uniform over 'a'..'z'
 *   1  "markov":  lengths round(LogNormal(ln 40, 0.6)) clamped to [1,512],
 *                 bytes from an order-2 Markov chain over the 64 base64url
 *                 symbols, Zipf(1.1) transitions over a seeded permutation
 *                 per context; the first two symbols are Zipf(1.1) over a
 *                 seeded permutation
 *   2  "urls":    one of 2000 seeded 20..40-byte host prefixes followed by
 *                 1..6 '/'-separated path tokens from a seeded 10^4-token
 *                 vocabulary (3..12 bytes of [a-z0-9]) drawn Zipf(1.1)
 *   3  "suffixes": all n suffixes of a seeded ACGT text of length n, with
 *                 ceil(0.05 n / 1024) planted copies of random 1 KiB windows
 *                 at non-overlapping destinations, each suffix truncated to
 *                 512 bytes
 *   4  "binary":  lengths uniform in [1,64], bytes uniform over {'0','1'}
 *   5  "bytes":   lengths uniform in [0,12], bytes uniform over 0..255 with
 *                 extra weight on 0x00 and 0xFF
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SSGEN_RANDOM 0
#define SSGEN_MARKOV 1
#define SSGEN_URLS 2
#define SSGEN_SUFFIXES 3
#define SSGEN_BINARY 4
#define SSGEN_BYTES 5

/* ---- SplitMix64 (Steele, Lea, Flood 2014) ---------------------------- */
typedef struct { uint64_t s; } rng_t;

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline uint64_t rng_next(rng_t* r) {
    r->s += 0x9E3779B97F4A7C15ULL;
    return mix64(r->s);
}
static inline rng_t rng_for(uint64_t seed, uint64_t stream, uint64_t i) {
    rng_t r;
    r.s = mix64(mix64(seed ^ 0x6A09E667F3BCC908ULL) + stream * 0xD1B54A32D192ED03ULL) + i * 0x9E3779B97F4A7C15ULL;
    r.s = mix64(r.s);
    return r;
}
/* uniform integer in [0, k) (multiply-high reduction) */
static inline uint32_t rng_below(rng_t* r, uint32_t k) {
    return (uint32_t)(((unsigned __int128)rng_next(r) * k) >> 64);
}
/* uniform double in [0, 1) */
static inline double rng_unit(rng_t* r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* ---- Zipf(s) over ranks 0..K-1 via a cumulative table ----------------- */
typedef struct { int K; double* cdf; } zipf_t;

static zipf_t zipf_make(int K, double s) {
    zipf_t z; z.K = K; z.cdf = (double*)malloc(sizeof(double) * (size_t)K);
    double acc = 0.0;
    for (int r = 0; r < K; ++r) { acc += pow((double)(r + 1), -s); z.cdf[r] = acc; }
    for (int r = 0; r < K; ++r) z.cdf[r] /= acc;
    z.cdf[K - 1] = 1.0;
    return z;
}
static inline int zipf_draw(const zipf_t* z, rng_t* r) {
    double u = rng_unit(r);
    int lo = 0, hi = z->K - 1;           /* first rank with cdf > u */
    while (lo < hi) { int m = (lo + hi) >> 1; if (z->cdf[m] > u) hi = m; else lo = m + 1; }
    return lo;
}

static void shuffle_u8(uint8_t* a, int k, rng_t* r) {
    for (int i = k - 1; i > 0; --i) { int j = (int)rng_below(r, (uint32_t)i + 1); uint8_t t = a[i]; a[i] = a[j]; a[j] = t; }
}

/* ---- model 1 tables --------------------------------------------------- */
static const char B64URL[65] = "-0123456789ABCDEFGHIJKLMNOPQRSTUVWXYZ_abcdefghijklmnopqrstuvwxyz";

typedef struct { uint8_t first[64]; uint8_t* perm; zipf_t z; } markov_t;

static markov_t markov_make(uint64_t seed) {
    markov_t m; rng_t r = rng_for(seed, 101, 0);
    for (int i = 0; i < 64; ++i) m.first[i] = (uint8_t)i;
    shuffle_u8(m.first, 64, &r);
    m.perm = (uint8_t*)malloc(64 * 64 * 64);
    for (int c = 0; c < 64 * 64; ++c) {
        uint8_t* p = m.perm + 64 * c;
        for (int i = 0; i < 64; ++i) p[i] = (uint8_t)i;
        shuffle_u8(p, 64, &r);
    }
    m.z = zipf_make(64, 1.1);
    return m;
}
static void markov_free(markov_t* m) { free(m->perm); free(m->z.cdf); }

static uint32_t markov_len(uint64_t seed, uint32_t i) {
    rng_t r = rng_for(seed, 1, i);
    double u1 = 1.0 - rng_unit(&r), u2 = rng_unit(&r);  /* u1 in (0,1] */
    double g = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    double L = exp(log(40.0) + 0.6 * g);
    long l = lround(L);
    if (l < 1) l = 1;
    if (l > 512) l = 512;
    return (uint32_t)l;
}

/* ---- model 2 tables --------------------------------------------------- */
#define URL_HOSTS 2000
#define URL_VOCAB 10000
static const char* TLDS[8] = {"com", "org", "net", "de", "io", "edu", "info", "fr"};
static const char ALNUM[37] = "abcdefghijklmnopqrstuvwxyz0123456789";

typedef struct {
    char host[URL_HOSTS][48]; uint8_t host_len[URL_HOSTS];
    char tok[URL_VOCAB][16]; uint8_t tok_len[URL_VOCAB];
    zipf_t z;
} urls_t;

static urls_t* urls_make(uint64_t seed) {
    urls_t* u = (urls_t*)calloc(1, sizeof(urls_t));
    rng_t r = rng_for(seed, 201, 0);
    for (int h = 0; h < URL_HOSTS; ++h) {
        int L = 20 + (int)rng_below(&r, 21);            /* total 20..40 bytes */
        const char* scheme = rng_below(&r, 2) ? "https://" : "http://";
        const char* tld = TLDS[rng_below(&r, 8)];
        int ls = (int)strlen(scheme), lt = (int)strlen(tld);
        int label = L - ls - lt - 1;                     /* >= 6 */
        char* p = u->host[h];
        memcpy(p, scheme, (size_t)ls); p += ls;
        int www = label > 12 && rng_below(&r, 2);
        if (www) { memcpy(p, "www.", 4); p += 4; label -= 4; }
        for (int k = 0; k < label; ++k) *p++ = ALNUM[rng_below(&r, k == 0 ? 26 : 36)];
        *p++ = '.';
        memcpy(p, tld, (size_t)lt); p += lt;
        u->host_len[h] = (uint8_t)(p - u->host[h]);
    }
    for (int t = 0; t < URL_VOCAB; ++t) {
        int L = 3 + (int)rng_below(&r, 10);
        for (int k = 0; k < L; ++k) u->tok[t][k] = ALNUM[rng_below(&r, 36)];
        u->tok_len[t] = (uint8_t)L;
    }
    u->z = zipf_make(URL_VOCAB, 1.1);
    return u;
}
static void urls_free(urls_t* u) { free(u->z.cdf); free(u); }

/* one URL: host id, number of tokens, token ids; returns length */
static uint32_t url_shape(const urls_t* u, uint64_t seed, uint32_t i, int* host, int* ntok, int toks[6]) {
    rng_t r = rng_for(seed, 2, i);
    *host = (int)rng_below(&r, URL_HOSTS);
    *ntok = 1 + (int)rng_below(&r, 6);
    uint32_t len = u->host_len[*host];
    for (int k = 0; k < *ntok; ++k) { toks[k] = zipf_draw(&u->z, &r); len += 1u + u->tok_len[toks[k]]; }
    return len;
}

/* ---- model 3 text ----------------------------------------------------- */
static uint8_t* suffix_text(uint64_t seed, uint32_t n) {
    uint8_t* T = (uint8_t*)malloc((size_t)n + 1);
    rng_t r = rng_for(seed, 301, 0);
    static const char ACGT[4] = {'A', 'C', 'G', 'T'};
    for (uint32_t i = 0; i < n; ++i) T[i] = (uint8_t)ACGT[rng_below(&r, 4)];
    const uint32_t W = 1024;
    uint32_t copies = (uint32_t)((0.05 * (double)n + W - 1) / W);
    if (n >= 4 * W && copies > 0) {
        uint32_t* dst = (uint32_t*)malloc(sizeof(uint32_t) * copies);
        uint32_t placed = 0, tries = 0;
        while (placed < copies && tries < 1000u * copies) {
            ++tries;
            uint32_t d = rng_below(&r, n - W + 1);
            int ok = 1;
            for (uint32_t k = 0; k < placed; ++k)
                if (d < dst[k] + W && dst[k] < d + W) { ok = 0; break; }
            if (!ok) continue;
            uint32_t s = rng_below(&r, n - W + 1);
            memmove(T + d, T + s, W);
            dst[placed++] = d;
        }
        free(dst);
    }
    return T;
}

/* ---- public API ------------------------------------------------------- */

/* Fills offsets[0..n] (offsets[0] = 0) and returns the total character count,
 * or UINT64_MAX for an unknown model. */
uint64_t ssgen_lengths(int model, uint64_t seed, uint32_t n, uint64_t* offsets) {
    uint32_t* len = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)n + 1));
    if (!len) return UINT64_MAX;
    urls_t* u = NULL;
    if (model == SSGEN_URLS) u = urls_make(seed);
    int bad = 0;
    #pragma omp parallel for schedule(static)
    for (long long ii = 0; ii < (long long)n; ++ii) {
        uint32_t i = (uint32_t)ii;
        rng_t r = rng_for(seed, 1, i);
        switch (model) {
        case SSGEN_RANDOM: len[i] = 1 + rng_below(&r, 32); break;
        case SSGEN_MARKOV: len[i] = markov_len(seed, i); break;
        case SSGEN_URLS: { int h, nt, tk[6]; len[i] = url_shape(u, seed, i, &h, &nt, tk); } break;
        case SSGEN_SUFFIXES: len[i] = (n - i) < 512u ? (n - i) : 512u; break;
        case SSGEN_BINARY: len[i] = 1 + rng_below(&r, 64); break;
        case SSGEN_BYTES: len[i] = rng_below(&r, 13); break;
        default: bad = 1; len[i] = 0;
        }
    }
    if (u) urls_free(u);
    if (bad) { free(len); return UINT64_MAX; }
    uint64_t acc = 0;
    offsets[0] = 0;
    for (uint32_t i = 0; i < n; ++i) { acc += len[i]; offsets[i + 1] = acc; }
    free(len);
    return acc;
}

/* Fills chars[offsets[0] .. offsets[n]) for the lengths made by
 * ssgen_lengths with the same (model, seed, n).  Returns 0 on success. */
int ssgen_chars(int model, uint64_t seed, uint32_t n, const uint64_t* offsets, uint8_t* chars) {
    markov_t mk; urls_t* u = NULL; uint8_t* T = NULL;
    if (model < 0 || model > SSGEN_BYTES) return 1;
    if (model == SSGEN_MARKOV) mk = markov_make(seed);
    if (model == SSGEN_URLS) u = urls_make(seed);
    if (model == SSGEN_SUFFIXES) T = suffix_text(seed, n);
    #pragma omp parallel for schedule(dynamic, 4096)
    for (long long ii = 0; ii < (long long)n; ++ii) {
        uint32_t i = (uint32_t)ii;
        uint8_t* p = chars + offsets[i];
        uint32_t L = (uint32_t)(offsets[i + 1] - offsets[i]);
        rng_t r = rng_for(seed, 3, i);
        switch (model) {
        case SSGEN_RANDOM:
            for (uint32_t k = 0; k < L; ++k) p[k] = (uint8_t)('a' + rng_below(&r, 26));
            break;
        case SSGEN_MARKOV: {
            uint8_t a = 0, b = 0;
            for (uint32_t k = 0; k < L; ++k) {
                uint8_t s;
                if (k < 2) s = mk.first[zipf_draw(&mk.z, &r)];
                else s = mk.perm[64 * (64 * a + b) + zipf_draw(&mk.z, &r)];
                p[k] = (uint8_t)B64URL[s];
                a = b; b = s;
            }
        } break;
        case SSGEN_URLS: {
            int h, nt, tk[6];
            url_shape(u, seed, i, &h, &nt, tk);
            memcpy(p, u->host[h], u->host_len[h]); p += u->host_len[h];
            for (int k = 0; k < nt; ++k) { *p++ = '/'; memcpy(p, u->tok[tk[k]], u->tok_len[tk[k]]); p += u->tok_len[tk[k]]; }
        } break;
        case SSGEN_SUFFIXES:
            memcpy(p, T + i, L);
            break;
        case SSGEN_BINARY:
            for (uint32_t k = 0; k < L; ++k) p[k] = (uint8_t)('0' + rng_below(&r, 2));
            break;
        case SSGEN_BYTES:
            for (uint32_t k = 0; k < L; ++k) {
                uint32_t x = rng_below(&r, 320);
                p[k] = x < 256 ? (uint8_t)x : (x < 288 ? 0x00 : 0xFF);
            }
            break;
        }
    }
    if (model == SSGEN_MARKOV) markov_free(&mk);
    if (u) urls_free(u);
    free(T);
    return 0;
}

/* Texts for suffix sorting.  Kinds: 0 the ACGT text of the "suffixes" model
 * (with its planted 1 KiB repeats); 1 bytes uniform over 0..255; 2 a
 * period of 1..16 random lowercase letters repeated, with one random byte
 * changed per 4096; 3 lowercase letters with Zipf(1.1) frequencies.
 * Returns 0 on success. */
int ssgen_text(int kind, uint64_t seed, uint32_t n, uint8_t* out) {
    if (kind == 0) {
        uint8_t* T = suffix_text(seed, n);
        if (!T) return 1;
        memcpy(out, T, n);
        free(T);
        return 0;
    }
    rng_t r = rng_for(seed, 401, (uint64_t)kind);
    if (kind == 1) {
        for (uint32_t i = 0; i < n; ++i) out[i] = (uint8_t)rng_below(&r, 256);
        return 0;
    }
    if (kind == 2) {
        uint8_t per[16];
        uint32_t p = 1 + rng_below(&r, 16);
        for (uint32_t k = 0; k < p; ++k) per[k] = (uint8_t)('a' + rng_below(&r, 26));
        for (uint32_t i = 0; i < n; ++i) out[i] = per[i % p];
        for (uint32_t i = 0; i + 4096 <= n; i += 4096) out[i + rng_below(&r, 4096)] = (uint8_t)rng_below(&r, 256);
        return 0;
    }
    if (kind == 3) {
        zipf_t z = zipf_make(26, 1.1);
        for (uint32_t i = 0; i < n; ++i) out[i] = (uint8_t)('a' + zipf_draw(&z, &r));
        free(z.cdf);
        return 0;
    }
    return 1;
}

/* Helper for batched/serving workloads: a value log-uniform in [lo, hi]
 * drawn from stream (seed, 7, j). */
uint64_t ssgen_log_uniform(uint64_t seed, uint64_t j, double lo, double hi) {
    rng_t r = rng_for(seed, 7, j);
    double u = rng_unit(&r);
    return (uint64_t)llround(exp(log(lo) + u * (log(hi) - log(lo))));
}

/* Helper: uniform integer in [0, k) from stream (seed, 8, j). */
uint32_t ssgen_uniform(uint64_t seed, uint64_t j, uint32_t k) {
    rng_t r = rng_for(seed, 8, j);
    return rng_below(&r, k);
}

/* Helper: exponential variate with mean 1 from stream (seed, 9, j). */
double ssgen_exponential(uint64_t seed, uint64_t j) {
    rng_t r = rng_for(seed, 9, j);
    return -log(1.0 - rng_unit(&r));
}

/* Mixes two 64-bit values (per-set seeds of batched workloads). */
uint64_t ssgen_hash(uint64_t a, uint64_t b) { return mix64(mix64(a) ^ (b * 0x9E3779B97F4A7C15ULL + 0x632BE59BD9B4E019ULL)); }
