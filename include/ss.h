/*
 * libss -- string sample sort on one AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Sorts a set of n byte strings lexicographically and returns the
 * sorted permutation and the LCP array, the problem of section 2.1 of
 * Bingmann, "Scalable String and Suffix Sorting" (arXiv:1808.00963): the
 * array S = [s_0 .. s_{n-1}] of n strings with N characters in total is
 * sorted lexicographically, and the LCP array H holds for each sorted
 * position k >= 1 the length of the longest common prefix of the strings at
 * positions k-1 and k.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * Input layout.  `chars` holds the characters of all strings back to back;
 * `offsets` holds n+1 non-decreasing 64-bit byte offsets into `chars`:
 * string i is chars[offsets[i] .. offsets[i+1]).  Every byte value 0..255 is
 * a character (compared unsigned); strings carry explicit lengths instead of
 * the paper's zero terminator, so a proper prefix sorts before the longer
 * string, as with a terminator smaller than every character (section 2.1).
 *
 * Output.  perm_out[k] = index of the string at sorted position k; equal
 * strings keep their input order (ties by original index), which makes the
 * result unique.  lcp_out[0] = 0 (the paper's undefined first entry),
 * lcp_out[k] = LCP(s_{perm[k-1]}, s_{perm[k]}).
 *
 * Memory.  Unless stated otherwise every pointer is a DEVICE pointer on the
 * current HIP device, allocated and owned by the caller; the library never
 * frees it.  Inputs are read only.  perm_out and lcp_out must not alias each
 * other or the inputs.  The chars buffer must be readable up to
 * offsets[n]; the library also reads the aligned 8-byte words that contain
 * the first and last character of each string (never past a page that
 * holds a character).
 *
 * Streams and errors.  `stream` is a hipStream_t (NULL = default stream).
 * Sort calls are asynchronous and stream-ordered: they enqueue the whole
 * sort on `stream` and return without waiting for it; the outputs are
 * complete once `stream` has reached the point where the call was made
 * (synchronise it, or order later work after it).  The sort starts after
 * the work enqueued on `stream` before the call and after the context's
 * previous sort (on whichever stream that ran).  Inside a sort, independent
 * steps also run on two streams that the context owns (default priority),
 * forked from and joined back into `stream` by events, so the caller sees
 * only `stream`; the device-driven form is capturable into a hipGraph.
 * Host-detectable errors (null pointers, aliased outputs, sizes beyond the
 * limits) are returned by the call without enqueueing anything.  Errors
 * detected on the device (non-monotone offsets, a string of 2^31 or more
 * bytes, bad set boundaries, an internal limit) are recorded on the device
 * and are sticky: ss_ctx_sync, ss_get_last_error (once the sort has
 * completed) and ss_get_stats report them until ss_clear_error.  The
 * outputs of a sort with a device-side error are unspecified.
 *
 * Limits.  n <= 2^32 - 2 strings; each string shorter than 2^31 bytes.
 * n = 0 is a no-op.
 */
#ifndef SS_H
#define SS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int ss_status;
#define SS_OK 0
#define SS_INVALID_ARG 1      /* null pointer, bad size, bad set boundaries */
#define SS_OUT_OF_MEMORY 2    /* workspace allocation failed */
#define SS_HIP_ERROR 3        /* a HIP runtime call failed */
#define SS_LIMIT 4            /* n or a string length beyond the limits above,
                                 or non-monotone offsets (detected on device) */
#define SS_REJECTED 5         /* serving: request does not fit the budget */
#define SS_TIMEOUT 6          /* serving: wait timed out */
#define SS_INTERNAL 7         /* an internal capacity check failed */

typedef struct ss_ctx ss_ctx;

#define SS_MODE_LEVELS 0
#define SS_MODE_PERSISTENT 1
#define SS_MODE_HOST_LEVELS 2

#define SS_ALPHABET_AUTO 0
#define SS_ALPHABET_BYTES 1
#define SS_ALPHABET_COMPRESS 2

/* Tunable parameters (performance only; results never depend on them). */
typedef struct {
    uint32_t max_log_splitters; /* d_max: at most v = 2^d_max - 1 splitters
                                   per distribution step (section 4.2.2),
                                   1..10, default 10 */
    uint32_t bucket_target;     /* expected strings per bucket used to pick
                                   v for a segment, 16..2^20, default 64 */
    uint32_t base_max;          /* segments with at most this many strings go
                                   to the base case, 64..1024, default 1024 */
    uint32_t mode;              /* how the recursion levels are driven:
                                   SS_MODE_LEVELS (default): every level is
                                   enqueued as separate launches whose kernels
                                   read the level's work counts on the device,
                                   as many levels as the context's last sort
                                   needed, then one persistent launch runs any
                                   levels left; no host synchronisation.  The
                                   persistent launch is the slow form: a
                                   context that alternates between inputs of
                                   different depth (or a first sort deeper
                                   than 4 levels) pays for it once per deeper
                                   sort; HOST_LEVELS avoids it.
                                   SS_MODE_PERSISTENT: the whole sort in ONE
                                   persistent launch that walks the levels on
                                   the device.  SS_MODE_HOST_LEVELS: the host
                                   reads each level's counts and enqueues it
                                   with exact grids (synchronises once per
                                   level; kept for comparison). */
    uint32_t alphabet;          /* key format (alphabet compression, section
                                   4.6.1).  A compressed key holds each
                                   character as 1 + its rank among the bytes
                                   the input uses, in 2, 3 or 4 bits (1..3,
                                   4..7 or 8..15 distinct bytes; 32, 21 or 16
                                   characters per 64-bit key instead of 8).
                                   SS_ALPHABET_BYTES (default): always 8 bytes
                                   per key; the call does not wait for the
                                   device.  SS_ALPHABET_AUTO: the sort first
                                   probes the first 16 bytes of 1024 strings;
                                   for inputs of at most 3 distinct bytes and
                                   at most 64 characters per string on average
                                   the keys are compressed with the probed
                                   byte set.  Every compressed key gather
                                   checks its bytes against the set; if one
                                   lies outside, the sort runs again after a
                                   pass over chars[offsets[0], offsets[n])
                                   that finds every byte (compressed if the
                                   whole input qualifies, else byte keys;
                                   ss_stats.alphabet_retries counts it).
                                   SS_ALPHABET_COMPRESS: the same for inputs
                                   of at most 15 distinct bytes and any
                                   length.  With AUTO or COMPRESS the call
                                   waits for the probe and, when the keys are
                                   compressed, for the sort (the level kernels
                                   come in a byte-key and a compressed form;
                                   the host launches one); SS_MODE_PERSISTENT
                                   checks every byte before its single
                                   launch and does not wait.  Graphs,
                                   ss_sort_noalloc and serving use byte keys.
                                   Results never depend on this setting. */
} ss_config;

/* Returns a short description of a status code (static storage). */
const char* ss_status_string(ss_status s);

/* Library version string (static storage). */
const char* ss_version(void);

/* Creates a context bound to HIP device `device`.  The context owns the
 * sort's working memory: the two ping-pong element arrays of the
 * out-of-place redistribution (section 4.2.8), the bucket ("oracle") array
 * and the per-tile bucket counters of the distribution steps (Algorithm
 * 4.1), the splitter trees (section 4.2.2) and the lists of segments and
 * pending boundary LCPs (Figure 4.7).  The workspace is grow-only (freed by
 * ss_ctx_destroy); `scratch_limit` bytes caps it (0 = no cap; a call needing
 * more returns SS_OUT_OF_MEMORY).  One context must not be used by two host
 * threads at once; sorts on one context run one after the other on the
 * device even when issued on different streams. */
ss_status ss_ctx_create(ss_ctx** ctx, int device, size_t scratch_limit);
void ss_ctx_destroy(ss_ctx* ctx);

/* Reads / replaces the tuning parameters of a context.  Out-of-range fields
 * are clamped. */
ss_status ss_get_config(const ss_ctx* ctx, ss_config* cfg);
ss_status ss_set_config(ss_ctx* ctx, const ss_config* cfg);

/* Bytes of workspace a sort of n strings needs under the context's current
 * configuration (host function, no device access): the arrays listed at
 * ss_ctx_create, sized for the worst case of one recursion level -- at most
 * n strings in flight, n/2 + 2n/bucket_target + 3 n/(base_max+1) bucket
 * counters (Algorithm 4.1 keeps 2v+1 counters per tile, Theorem 4.4) and
 * n pending boundary LCPs (Figure 4.7). */
ss_status ss_workspace_query(const ss_ctx* ctx, uint32_t n, size_t* bytes);

/* Sorts one string set (section 2.1 problem, method of section 4.2:
 * string sample sort with 8-byte keys, equality buckets and an LCP array).
 * chars: device, offsets[n] bytes; offsets: device, n+1 uint64;
 * perm_out, lcp_out: device, n uint32 each. */
ss_status ss_sort_ex(ss_ctx* ctx, const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                     uint32_t* perm_out, uint32_t* lcp_out, void* stream);

/* Same as ss_sort_ex with an implicit per-device context (created on first
 * use on the current device, kept until process exit, internally locked). */
ss_status ss_sort(const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                  uint32_t* perm_out, uint32_t* lcp_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the sort
 * of ss_sort, with its workspace in a fixed array of the library instead of
 * a context's allocation.  It calls no allocating routine; every launch goes
 * to `stream` (asynchronous, stream-ordered, capturable).  The array (72 MiB,
 * workspace for SS_NOALLOC_MAX_STRINGS strings) is allocated on each device
 * when the library is loaded there and held until the process ends; all
 * calls on one device share it, so calls on one device must not overlap
 * (order them on one stream, or synchronise between them): overlapping calls
 * race on the shared workspace.  Each call starts by clearing the control
 * data it relies on.  chars, offsets, perm_out, lcp_out: as for ss_sort_ex.
 * err_out: device pointer to one uint32 (or NULL) that receives the sort's
 * device-side error bits when it has run (0 = success; nonzero = offsets not
 * monotone, a string too long, or an internal limit; the outputs are then
 * unspecified).  Returns SS_LIMIT for n > SS_NOALLOC_MAX_STRINGS,
 * SS_INVALID_ARG for null or aliased pointers; n = 0 is a no-op. */
#define SS_NOALLOC_MAX_STRINGS (1u << 20)
ss_status ss_sort_noalloc(const uint8_t* chars, const uint64_t* offsets, uint32_t n, uint32_t* perm_out,
                          uint32_t* lcp_out, uint32_t* err_out, void* stream);

/* Batched form: sorts num_sets independent string sets in one pass of the
 * pipeline (all sets' segments are processed by the same kernel launches):
 * each set is the section 2.1 problem on its own, and the sets are the
 * independent jobs that section 4.2.8 runs side by side (every job of any
 * size shares the processors with the others).
 * The strings of all sets are given as one string array (chars, offsets
 * with offsets[set_begin[num_sets]] characters); set j consists of strings
 * set_begin[j] .. set_begin[j+1]-1.  set_begin: device, num_sets+1
 * non-decreasing uint32 with set_begin[0] = 0; n = set_begin[num_sets] is
 * passed as `n` and checked on the device.  Output position p of set j
 * (set_begin[j] <= p < set_begin[j+1]) receives a SET-LOCAL index:
 * perm_out[p] = i - set_begin[j] for the string i sorted there, and
 * lcp_out[set_begin[j]] = 0. */
ss_status ss_sort_batch(ss_ctx* ctx, const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                        const uint32_t* set_begin, uint32_t num_sets,
                        uint32_t* perm_out, uint32_t* lcp_out, void* stream);

/* Graph form of the batched sort (section 4.2.8, the batched sets as
 * independent jobs): captures the complete batched sort of the given
 * buffers as a hipGraph, so repeated launches cost one graph launch each.
 * Creating the graph runs the batched sort once (synchronously; the outputs
 * then hold its result) to learn how many recursion levels it needs; the
 * graph holds that many levels of separate launches whose kernels read the
 * level's work counts on the device, then ONE persistent launch that runs
 * any levels left (later contents may need more) and the boundary LCPs.
 * The graph owns its workspace (allocated here, freed by ss_graph_destroy),
 * so it is independent of the context's own sorts.  The buffers must stay
 * valid and keep their shapes while the graph exists; the contents may
 * change between launches.  Launches of one graph must not overlap each
 * other.  ss_graph_launch enqueues and returns; device-side errors of a
 * launch are reported by ss_ctx_sync of the context the graph was created
 * on.  ss_graph_levels returns the number of level launches in the graph. */
typedef struct ss_graph ss_graph;
ss_status ss_graph_create_batch(ss_ctx* ctx, const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                                const uint32_t* set_begin, uint32_t num_sets, uint32_t* perm_out,
                                uint32_t* lcp_out, ss_graph** graph_out);
ss_status ss_graph_launch(ss_graph* graph, void* stream);
void ss_graph_destroy(ss_graph* graph);
uint32_t ss_graph_levels(const ss_graph* graph);

/* Waits for `stream` and for the context's last sort, and returns the
 * context's sticky device-side status: SS_OK, or the error of any sort or
 * graph launch of the context since the last ss_clear_error. */
ss_status ss_ctx_sync(ss_ctx* ctx, void* stream);

/* Autotuner (variant tuning of section 4.4 / the evaluation's tuned
 * variants; results never depend on the configuration).  Times candidate
 * configurations on the given input -- a grid over max_log_splitters
 * {8,9,10} x bucket_target {32,64,128} x base_max {512,1024} in the
 * level-by-level form, then the persistent form with the winner's
 * parameters -- as the median of `reps` sorts after one warm-up each, and
 * keeps the fastest: it becomes the context's configuration and is cached
 * per process under (device, floor(log2) of n, of the character count and
 * of the set count).  With use_cache != 0 a cached entry for the signature
 * is applied without timing.  Afterwards perm_out / lcp_out hold the sort's
 * result (identical under every configuration).  set_begin == NULL with
 * num_sets == 1 tunes the single-set sort; otherwise the arguments are those
 * of ss_sort_batch.  Candidates that fail (e.g. beyond the workspace cap)
 * are skipped; SS_INTERNAL if all fail (the configuration is then left as
 * it was).  best / best_ms (may be NULL) receive the chosen configuration
 * and its median milliseconds.  Synchronizes `stream`. */
ss_status ss_autotune(ss_ctx* ctx, const uint8_t* chars, const uint64_t* offsets, uint32_t n,
                      const uint32_t* set_begin, uint32_t num_sets, uint32_t* perm_out, uint32_t* lcp_out,
                      void* stream, uint32_t reps, int use_cache, ss_config* best, double* best_ms);
/* Forgets every cached autotuning result of the process. */
void ss_autotune_clear_cache(void);

/* LCP-aware merge of sorted runs (section 4.3.1: binary LCP-merge,
 * Algorithms 4.2-4.4, Lemma 4.5), done as pairwise GPU rounds.
 * perm[run_begin[r] .. run_begin[r+1]) is run r: string indices (each below
 * n_strings) sorted by string, equal strings by index, as ss_sort_ex leaves
 * them, and lcp[p] is the LCP of the strings at p-1 and p within the run
 * (the entry at a run's first position is ignored).  The output is the
 * union of the runs in the same order with its LCP array (lcp_out[0] = 0):
 * for runs that sort disjoint parts of one set it equals ss_sort_ex of the
 * whole set.  The same index may appear in several runs (copies stay
 * adjacent).
 * chars, offsets: device, as for ss_sort_ex with n_strings strings;
 * perm, lcp: device, run_begin[num_runs] uint32 each (inputs, unchanged);
 * run_begin: HOST, num_runs+1 non-decreasing uint64 with run_begin[0] = 0;
 * perm_out, lcp_out: device, run_begin[num_runs] uint32 each, not
 * overlapping the inputs or each other.
 * Errors: SS_INVALID_ARG for bad run boundaries, aliased buffers or a perm
 * entry >= n_strings (detected on device), SS_LIMIT for more than
 * 2^32-2 elements or malformed offsets.  Empty runs are allowed.  The merge
 * workspace (up to four run_begin[num_runs]-entry arrays) is kept by the
 * context.  Synchronizes `stream` before returning. */
ss_status ss_merge_runs(ss_ctx* ctx, const uint8_t* chars, const uint64_t* offsets, uint32_t n_strings,
                        const uint32_t* perm, const uint32_t* lcp, const uint64_t* run_begin, uint32_t num_runs,
                        uint32_t* perm_out, uint32_t* lcp_out, void* stream);

/* Suffix array of a byte text by prefix doubling (section 8.2: Observation
 * 8.1, Algorithm 8.1, with the discarding of section 8.2.5), every round
 * being one sort of the context's string sorter.  Round 0 sorts the suffixes
 * by their first 32 characters (64 or 128 for texts of at most 4 or 2
 * distinct bytes, whose windows are alphabet compressed); each later round
 * sorts, for every suffix
 * whose group (suffixes equal to depth h) has other members, the 8-byte
 * string of its name and the name of suffix i + h (names: first suffix-array
 * position of the group), doubling h, until every suffix has its own
 * group.  Suffix i is text[i .. n); a proper prefix sorts first, every byte
 * value is an ordinary character and no sentinel is needed.
 * text: device, n bytes; sa_out: device, n uint32 (the suffix array);
 * isa_out: device, n uint32 (its inverse) or NULL; rounds_out: host, the
 * number of sorts run (may be NULL).  The workspace (about 64 n bytes plus
 * the sort's) is kept by the context; the sorts use the context's
 * configuration with a bucket target of at least 256.  SS_LIMIT for
 * n > 2^32 - 2.
 * Synchronizes `stream` once per round and before returning. */
ss_status ss_suffix_array(ss_ctx* ctx, const uint8_t* text, uint32_t n, uint32_t* sa_out, uint32_t* isa_out,
                          uint32_t* rounds_out, void* stream);

/* ---- serving: continuous batching under an HBM budget ------------------
 * A server owns one device (its own stream and worker thread) and a fixed
 * device arena sized by `hbm_budget` bytes: character storage plus index
 * slots (keys, ping-pong elements, offsets, outputs).  Requests are host
 * buffers; the worker copies a request to the device when its footprint
 * (ss_server_footprint) fits into the free arena, and adds it as a new root
 * segment to the recursion level that is running, so requests that arrive
 * while others are on the GPU share every later kernel launch with them.
 * A request completes when all its strings are final; its pending boundary
 * LCPs are resolved and its outputs copied back.  Results are identical to
 * ss_sort of the request alone (perm set-local, lcp[0] = 0).
 *
 * ss_request: chars, offsets (n+1, non-decreasing, string i =
 * chars[offsets[i] .. offsets[i+1])), perm_out and lcp_out (n entries) are
 * HOST pointers owned by the caller and must stay valid until
 * ss_server_wait reports completion (or ss_server_cancel succeeds).
 * Malformed offsets or a request larger than the whole arena are rejected at
 * submission (SS_LIMIT / SS_REJECTED). */
typedef struct ss_server ss_server;
typedef struct {
    const uint8_t* chars;
    const uint64_t* offsets;
    uint32_t n;
    uint32_t* perm_out;
    uint32_t* lcp_out;
} ss_request;
typedef struct {
    uint64_t submitted, completed, rejected, cancelled;
    uint64_t levels;              /* recursion levels run by the worker */
    uint64_t strings_completed, chars_completed;
    uint32_t inflight_max;        /* most requests on the device at once */
    uint32_t pad;
    uint64_t footprint_max;       /* largest sum of admitted footprints (bytes) */
    uint64_t arena_bytes;         /* size of the device arena (<= hbm_budget) */
    double p50_us, p99_us, mean_us, max_us;  /* latency submit -> outputs on host */
    double busy_s;                /* wall time with requests in flight */
    double iter_max_us;           /* longest engine iteration (admit, one level, completions) */
    double iter_max_wait_us;      /* of it: time the worker waited for the device */
    double iter_max_stage_us;     /* of it: time enqueueing the admitted requests' copies */
} ss_server_stats;
/* max_inflight: request slots on the device (1..65536); mean_len_hint:
 * expected characters per string used to split the budget between
 * characters and index slots (0 = 48); cfg may be NULL (defaults). */
ss_status ss_server_create(ss_server** out, int device, size_t hbm_budget, uint32_t max_inflight,
                           uint32_t mean_len_hint, const ss_config* cfg);
ss_status ss_server_submit(ss_server* srv, const ss_request* req, uint64_t* ticket);
/* Waits up to timeout_ms (< 0: forever).  Returns SS_OK when the outputs
 * are on the host (latency_us may be NULL), SS_TIMEOUT, or the request's
 * failure status.  A completed ticket can be waited for once. */
ss_status ss_server_wait(ss_server* srv, uint64_t ticket, int timeout_ms, double* latency_us);
/* Cancels a request that has not been admitted yet (SS_INVALID_ARG if it
 * already runs or is unknown). */
ss_status ss_server_cancel(ss_server* srv, uint64_t ticket);
/* Bytes of the arena a request of n strings and n_chars characters takes. */
size_t ss_server_footprint(const ss_server* srv, uint32_t n, uint64_t n_chars);
ss_status ss_server_get_stats(ss_server* srv, ss_server_stats* st);
void ss_server_reset_stats(ss_server* srv);
/* Stops the worker after the in-flight and queued requests finish. */
void ss_server_destroy(ss_server* srv);

/* Sticky error of a context (SS_OK if none): host-side failures, and the
 * device-side errors of sorts that have completed (it does not wait).
 * ss_clear_error waits for the context's last sort and clears both. */
ss_status ss_get_last_error(ss_ctx* ctx);
void ss_clear_error(ss_ctx* ctx);

/* Statistics of the last sort on a context, counted on the device level by
 * level: recursion levels, distribution steps (Algorithm 4.1), base-case
 * segments, pending boundary LCPs (Figure 4.7).  Waits for the last sort. */
typedef struct {
    uint32_t levels;
    uint32_t dist_segments;
    uint32_t dist_tiles;
    uint32_t base_segments;
    uint32_t pending_lcps;
    uint32_t max_depth;
    uint32_t base_rounds;   /* refinement rounds (depth + 8) run inside base cases */
    uint32_t base_segments_by_class[4]; /* base-case segments of <= 64, <= 128,
                                           <= 256 and <= base_max strings */
    uint64_t base_strings_by_class[4];  /* strings in those segments */
    uint32_t key_chars;     /* characters per 64-bit key: 8 (byte keys) or 16,
                               21 or 32 (alphabet-compressed keys) */
    uint32_t alphabet_size; /* distinct bytes of the key format's byte set
                               when the keys were compressed, else 0 */
    uint32_t alphabet_retries; /* 1 when compressed keys met a byte outside the
                                  probed set and the sort ran again */
} ss_stats;
ss_status ss_get_stats(ss_ctx* ctx, ss_stats* st);

/* Per-kernel timing (tracing).  When enabled on a context, every kernel
 * launch of a sort is bracketed by a pair of HIP events on the stream it is
 * launched on, and the sort call waits for the sort to finish (tracing makes
 * sorts synchronous); durations are accumulated per kernel until
 * ss_reset_kernel_times.  `units` counts the work items the launches
 * processed (strings, segments, counters or boundary entries, see `unit`),
 * taken from the level's work counts recorded on the device.  Launches of
 * a level that turned out to have no work for a kernel count as launches
 * with zero units. */
typedef struct {
    const char* name;      /* kernel name (static storage) */
    const char* unit;      /* what `units` counts (static storage) */
    uint32_t launches;
    double total_ms;
    double units;
} ss_kernel_time;
ss_status ss_set_profiling(ss_ctx* ctx, int enable);
/* Enables tracing for the one kernel named `kernel` (a name reported by
 * ss_get_kernel_times); the other launches get no events, so the sort runs
 * at full speed while that kernel is timed.  SS_INVALID_ARG for an unknown
 * name. */
ss_status ss_set_profiling_only(ss_ctx* ctx, const char* kernel);
ss_status ss_get_kernel_times(const ss_ctx* ctx, ss_kernel_time* out, uint32_t max_entries, uint32_t* n_entries);
void ss_reset_kernel_times(ss_ctx* ctx);

/* Streaming copy of `bytes` bytes (device pointers, 16-byte aligned, bytes a
 * multiple of 16) on `stream`.  Used to measure the achievable HBM
 * bandwidth and to calibrate hardware byte counters against a kernel whose
 * traffic is known (2 * bytes). */
ss_status ss_hbm_copy(void* dst, const void* src, size_t bytes, void* stream);

/* ---- host-side test entry points (no device access) -------------------
 * These run the same primitive functions the kernels use, on the host, so
 * the test suite can check them on a machine without a GPU. */

/* Key of string bytes s[h .. h+8) (host pointers), big-endian, zero padded;
 * *r_out = min(len - h, 8). */
uint64_t ss_host_key(const uint8_t* s, uint64_t len, uint64_t h, uint32_t* r_out);

/* The kernels' key gather (chars_h of section 4.2.2) run on the host with
 * plain loads: the key of string chars[off .. off+len) at depth h, reading
 * only the aligned 8-byte word(s) that hold characters of the key.  The
 * caller must make those words readable (the test places strings next to
 * unreadable pages to show that nothing else is read). */
uint64_t ss_host_gather_key(const uint8_t* chars, uint64_t off, uint32_t h, uint32_t len);

/* The base cases' common-prefix scan (the LCP of two strings known to
 * agree on their first `from` characters, at most min(la, lb, cap): the
 * LCPs of neighbours inside a base case, section 4.2.8, a role LCP-insertion
 * sort, Algorithm 4.6, plays in the paper) on the host:
 * strings chars[oa, oa + la) and chars[ob, ob + lb), each string's aligned
 * words read once, `ahead` (1, 2 or 4) words per string per step.  Reads
 * only aligned words that hold characters of the strings; the caller
 * guarantees the first `from` characters agree. */
uint32_t ss_host_lcp_stream(const uint8_t* chars, uint64_t oa, uint32_t la, uint64_t ob, uint32_t lb,
                            uint32_t from, uint32_t cap, uint32_t ahead);

/* The kernels' alphabet-compressed key gather (alphabet compression,
 * section 4.6.1) on the host: byte_set = the 256-bit set of bytes present
 * (four words, bit c of word c/64); with 1..15 members each character is
 * coded as 1 + its rank in the set in 2, 3 or 4 bits, 0 past the string's
 * end, most significant first (*chars_per_key = 32, 21 or 16); otherwise
 * the byte key of ss_host_gather_key (*chars_per_key = 8).  Reads only the
 * aligned words that hold the key's bytes; *miss = 1 if one of them is not
 * in the set.  Either output pointer may be NULL. */
uint64_t ss_host_gather_packed(const uint8_t* chars, uint64_t off, uint32_t h, uint32_t len,
                               const uint64_t* byte_set, uint32_t* chars_per_key, int* miss);
/* Characters two strings of lengths len_a, len_b share inside their keys a,
 * b at depth h, in the key format of byte_set (as above). */
uint32_t ss_host_key_lcp(const uint64_t* byte_set, uint64_t a, uint32_t len_a, uint64_t b, uint32_t len_b,
                         uint32_t h);

/* Lemma 4.1 mapping: level-order index of in-order position j (d levels),
 * and its inverse. */
uint32_t ss_host_level_index(uint32_t j, uint32_t d);
uint32_t ss_host_inorder_index(uint32_t l, uint32_t d);

/* Builds the level-order tree of v = 2^d - 1 sorted splitters (host arrays
 * xk[v], xr[v], in-order) and classifies m keys (ck[m], cr[m]) into
 * buckets[m] (0..2v).  Returns 0. */
int ss_host_classify(const uint64_t* xk, const uint32_t* xr, uint32_t d,
                     const uint64_t* ck, const uint32_t* cr, uint32_t m, uint32_t* buckets);

/* Splitter selection of section 4.2.2 ("Sampling"): from a sorted sample
 * (host arrays sk[a], sr[a]) picks v = 2^d - 1 in-order splitters
 * (xk[v], xr[v]) by recursive middle selection skipping duplicates. */
int ss_host_select_splitters(const uint64_t* sk, const uint32_t* sr, uint32_t a, uint32_t d,
                             uint64_t* xk, uint32_t* xr);

#ifdef __cplusplus
}
#endif
#endif /* SS_H */
