/*
 * ORACLE for the string sorter -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this file.  The product (the HIP library and its Python binding)
 * never calls it, and it shares no code with the GPU path.
 *
 * What it computes (the definition of the result, section 2.1 "Notation and
 * Preliminaries"):
 *   - string i is chars[offsets[i] .. offsets[i+1]); every byte 0..255 is a
 *     character, compared as an unsigned value;
 *   - a < b lexicographically: at the first differing position the smaller
 *     byte wins; if one string is a proper prefix of the other, the shorter
 *     one is smaller (the empty string is smallest), which is what the
 *     zero-terminator convention of section 2.1 gives;
 *   - equal strings are ordered by their original index, so the output
 *     permutation is unique;
 *   - lcp[0] = 0 (the undefined first entry of the LCP array H, read as the
 *     LCP with the empty string), lcp[k] = length of the longest common
 *     prefix of the strings at sorted positions k-1 and k (section 2.1).
 *
 * ss_oracle_sort: the definition written out -- a library comparison sort
 *   (qsort) of the indices with a memcmp comparator, then a brute-force
 *   character loop for each adjacent LCP.  Single-threaded, unoptimised.
 * ss_oracle_sort_mt: the same result on several threads, for the CPU
 *   baseline on all host cores: each thread sorts one contiguous chunk of
 *   the indices with the same comparator, sorted chunks are merged in
 *   pairwise rounds (a plain two-way merge per pair, pairs on separate
 *   threads), and the adjacent LCPs are computed by the same character loop
 *   over disjoint ranges.  The comparator orders by (string, index), a total
 *   order, so the merged result is the single correct answer.
 * ss_oracle_check: verifies a claimed (perm, lcp) against the same
 *   definition without sorting: perm is a permutation, each adjacent pair is
 *   strictly increasing in (string, index) order, and each lcp entry equals
 *   the brute-force common prefix.  Because the correct output is unique,
 *   passing this check is equivalent to equality with ss_oracle_sort.
 *
 * Suffix sorting (section 5.1 definitions; section 8.2 h-order and h-names):
 * ss_oracle_suffix_array: the suffix array of a text T[0..n) written out --
 *   qsort of the start positions, comparing the suffixes T[i..n) as strings
 *   (memcmp, then the shorter one first; suffixes are distinct, so no tie
 *   rule is needed).  No sentinel is appended.
 * ss_oracle_h_names: the lexicographic h-name of every suffix, defined as
 *   the smallest rank among the suffixes equal to it in h-order (the order
 *   of the suffixes truncated to h characters): a qsort by truncated suffix,
 *   then the first sorted position of each run of equal truncations.
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    const uint8_t* chars;
    const uint64_t* offsets;
} strset_t;

/* three-way comparison of strings a and b by (bytes, length, index) */
static int cmp_idx(const strset_t* S, uint32_t a, uint32_t b) {
    const uint8_t* sa = S->chars + S->offsets[a];
    const uint8_t* sb = S->chars + S->offsets[b];
    uint64_t la = S->offsets[a + 1] - S->offsets[a];
    uint64_t lb = S->offsets[b + 1] - S->offsets[b];
    uint64_t m = la < lb ? la : lb;
    int c = m ? memcmp(sa, sb, (size_t)m) : 0;   /* memcmp compares unsigned bytes */
    if (c) return c < 0 ? -1 : 1;
    if (la != lb) return la < lb ? -1 : 1;      /* proper prefix is smaller */
    if (a != b) return a < b ? -1 : 1;          /* ties by original index */
    return 0;
}

static int qsort_cmp(const void* pa, const void* pb, void* ctx) {
    return cmp_idx((const strset_t*)ctx, *(const uint32_t*)pa, *(const uint32_t*)pb);
}

/* longest common prefix of strings a and b by a character loop */
static uint32_t lcp_brute(const strset_t* S, uint32_t a, uint32_t b) {
    const uint8_t* sa = S->chars + S->offsets[a];
    const uint8_t* sb = S->chars + S->offsets[b];
    uint64_t la = S->offsets[a + 1] - S->offsets[a];
    uint64_t lb = S->offsets[b + 1] - S->offsets[b];
    uint64_t m = la < lb ? la : lb, k = 0;
    while (k < m && sa[k] == sb[k]) ++k;
    return (uint32_t)k;
}

/* Sorts indices 0..n-1 and fills perm[0..n) and lcp[0..n).  Returns 0. */
int ss_oracle_sort(const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                   uint32_t* perm, uint32_t* lcp) {
    strset_t S = {chars, offsets};
    for (uint32_t i = 0; i < n; ++i) perm[i] = i;
    qsort_r(perm, n, sizeof(uint32_t), qsort_cmp, &S);
    if (n) lcp[0] = 0;
    for (uint32_t k = 1; k < n; ++k) lcp[k] = lcp_brute(&S, perm[k - 1], perm[k]);
    return 0;
}

/* Returns -1 when (perm, lcp) is the correct output, otherwise a code
 *   k               first sorted position k whose lcp entry is wrong,
 *   n + k           first position k >= 1 where (perm[k-1], perm[k]) is not
 *                   strictly increasing in (string, index) order,
 *   2n + i          perm is not a permutation (i = first bad entry),
 *   3n              lcp[0] != 0.                                           */
long long ss_oracle_check(const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                          const uint32_t* perm, const uint32_t* lcp) {
    strset_t S = {chars, offsets};
    uint8_t* seen = (uint8_t*)calloc((size_t)n + 1, 1);
    if (!seen) return -2;
    for (uint32_t i = 0; i < n; ++i) {
        if (perm[i] >= n || seen[perm[i]]) { free(seen); return 2LL * n + i; }
        seen[perm[i]] = 1;
    }
    free(seen);
    if (n && lcp[0] != 0) return 3LL * n;
    for (uint32_t k = 1; k < n; ++k)
        if (cmp_idx(&S, perm[k - 1], perm[k]) >= 0) return (long long)n + k;
    for (uint32_t k = 1; k < n; ++k)
        if (lcp[k] != lcp_brute(&S, perm[k - 1], perm[k])) return k;
    return -1;
}

/* Brute-force LCP of two strings (used by sampled checks of outputs too
 * large for a full oracle run). */
uint32_t ss_oracle_lcp(const uint8_t* chars, const uint64_t* offsets, uint32_t a, uint32_t b) {
    strset_t S = {chars, offsets};
    return lcp_brute(&S, a, b);
}

/* Three-way comparison of two strings by (bytes, length, index) (used by
 * sampled checks). */
int ss_oracle_compare(const uint8_t* chars, const uint64_t* offsets, uint32_t a, uint32_t b) {
    strset_t S = {chars, offsets};
    return cmp_idx(&S, a, b);
}

/* ---- the same sort on several threads ---------------------------------- */

typedef struct {
    const strset_t* S;
    uint32_t* src;
    uint32_t* dst;
    uint32_t* lcp;
    uint32_t lo, mid, hi; /* chunk sort: [lo, hi); merge: [lo, mid) + [mid, hi) */
} job_t;

static void* job_sort(void* arg) {
    job_t* j = (job_t*)arg;
    for (uint32_t i = j->lo; i < j->hi; ++i) j->src[i] = i;
    qsort_r(j->src + j->lo, j->hi - j->lo, sizeof(uint32_t), qsort_cmp, (void*)j->S);
    return NULL;
}

static void* job_merge(void* arg) {
    job_t* j = (job_t*)arg;
    uint32_t a = j->lo, b = j->mid, o = j->lo;
    while (a < j->mid && b < j->hi)
        j->dst[o++] = cmp_idx(j->S, j->src[a], j->src[b]) < 0 ? j->src[a++] : j->src[b++];
    while (a < j->mid) j->dst[o++] = j->src[a++];
    while (b < j->hi) j->dst[o++] = j->src[b++];
    return NULL;
}

static void* job_lcp(void* arg) {
    job_t* j = (job_t*)arg;
    for (uint32_t k = j->lo; k < j->hi; ++k)
        j->lcp[k] = k ? lcp_brute(j->S, j->src[k - 1], j->src[k]) : 0;
    return NULL;
}

/* runs jobs[0..m) on their own threads (the calling thread takes the last) */
static int run_jobs(void* (*fn)(void*), job_t* jobs, uint32_t m) {
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (m ? m : 1));
    if (!th) return -1;
    uint32_t started = 0;
    int rc = 0;
    for (uint32_t t = 0; t + 1 < m; ++t) {
        if (pthread_create(&th[t], NULL, fn, &jobs[t]) != 0) { rc = -1; break; }
        ++started;
    }
    if (rc == 0 && m) fn(&jobs[m - 1]);
    for (uint32_t t = 0; t < started; ++t) pthread_join(th[t], NULL);
    free(th);
    return rc;
}

/* Same output as ss_oracle_sort, computed by `threads` threads.  Returns 0,
 * or -1 if memory or threads are not available. */
int ss_oracle_sort_mt(const uint8_t* chars, const uint64_t* offsets, uint32_t n, uint32_t* perm, uint32_t* lcp,
                      uint32_t threads) {
    strset_t S = {chars, offsets};
    if (threads < 1) threads = 1;
    if (threads > n) threads = n ? n : 1;
    uint32_t* tmp = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)n + 1));
    uint32_t* bound = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)threads + 1));
    job_t* jobs = (job_t*)calloc(threads, sizeof(job_t));
    if (!tmp || !bound || !jobs) { free(tmp); free(bound); free(jobs); return -1; }
    for (uint32_t t = 0; t <= threads; ++t) bound[t] = (uint32_t)((uint64_t)n * t / threads);
    for (uint32_t t = 0; t < threads; ++t) jobs[t] = (job_t){&S, perm, NULL, NULL, bound[t], 0, bound[t + 1]};
    int rc = run_jobs(job_sort, jobs, threads);
    uint32_t *src = perm, *dst = tmp;
    for (uint32_t w = 1; rc == 0 && w < threads; w *= 2) {
        uint32_t m = 0;
        for (uint32_t c = 0; c < threads; c += 2 * w) {
            uint32_t mid = c + w < threads ? c + w : threads, hi = c + 2 * w < threads ? c + 2 * w : threads;
            jobs[m++] = (job_t){&S, src, dst, NULL, bound[c], bound[mid], bound[hi]};
        }
        rc = run_jobs(job_merge, jobs, m);
        uint32_t* x = src; src = dst; dst = x;
    }
    if (rc == 0 && src != perm) memcpy(perm, src, sizeof(uint32_t) * (size_t)n);
    for (uint32_t t = 0; rc == 0 && t < threads; ++t) jobs[t] = (job_t){&S, perm, NULL, lcp, bound[t], 0, bound[t + 1]};
    if (rc == 0) rc = run_jobs(job_lcp, jobs, threads);
    free(tmp); free(bound); free(jobs);
    return rc;
}

/* ---- suffix sorting --------------------------------------------------- */

typedef struct {
    const uint8_t* text;
    uint64_t n;
    uint64_t h; /* compare at most h characters (UINT64_MAX: whole suffixes) */
} suftext_t;

/* three-way comparison of the suffixes a and b truncated to h characters */
static int cmp_suffix(const suftext_t* S, uint32_t a, uint32_t b) {
    uint64_t la = S->n - a, lb = S->n - b;
    if (la > S->h) la = S->h;
    if (lb > S->h) lb = S->h;
    uint64_t m = la < lb ? la : lb;
    int c = m ? memcmp(S->text + a, S->text + b, (size_t)m) : 0;
    if (c) return c < 0 ? -1 : 1;
    if (la != lb) return la < lb ? -1 : 1; /* proper prefix is smaller */
    return 0;
}

static int qsort_suffix(const void* pa, const void* pb, void* ctx) {
    return cmp_suffix((const suftext_t*)ctx, *(const uint32_t*)pa, *(const uint32_t*)pb);
}

int ss_oracle_suffix_array(const uint8_t* text, uint32_t n, uint32_t* sa) {
    suftext_t S = {text, n, UINT64_MAX};
    for (uint32_t i = 0; i < n; ++i) sa[i] = i;
    qsort_r(sa, n, sizeof(uint32_t), qsort_suffix, &S);
    return 0;
}

int ss_oracle_h_names(const uint8_t* text, uint32_t n, uint64_t h, uint32_t* names) {
    suftext_t S = {text, n, h};
    uint32_t* order = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!order) return -1;
    for (uint32_t i = 0; i < n; ++i) order[i] = i;
    qsort_r(order, n, sizeof(uint32_t), qsort_suffix, &S);
    uint32_t first = 0;
    for (uint32_t k = 0; k < n; ++k) {
        if (k > 0 && cmp_suffix(&S, order[k - 1], order[k]) != 0) first = k;
        names[order[k]] = first;
    }
    free(order);
    return 0;
}
