/*
 * srw.h -- C ABI of libsrw: exact shortest reset words on one MI355X GPU.
 *
 * Paper: M. Szykula, A. Zyzik, "An Improved Algorithm for Finding the
 * Shortest Synchronizing Words".
 *
 * Problem (Section 1 and the input/output of Alg. 1): a complete
 * deterministic automaton (Q, Sigma, delta) with n states and k letters.  A
 * word w is a reset word if |delta(Q, w)| = 1; the reset threshold r is the
 * length of the shortest ones.  The library returns r and, on request, the
 * lexicographically least reset word of length r (letters ordered by their
 * index; the paper returns "a" shortest word through predecessor pointers,
 * end of the Section 2 intro, and this is the one fixed here).
 *
 * Method: the bidirectional breadth-first search of Alg. 1 in its plain
 * variant -- forward steps compute images of the BFS list, inverse steps
 * compute preimages of the IBFS list, each new list is deduplicated (here
 * also against all earlier lists of the same side), and after every step the
 * meet test (some X of the BFS list is a subset of some Y of the IBFS list,
 * Section 2) decides r.  The side expanded next is the one with the smaller
 * current list (ties: forward).  The inclusion reductions, the cost-model
 * step choice and the DFS phase of the paper are not part of this path.
 *
 * Conventions shared by every call:
 *   delta   letter-major int32: delta[a*n + q] = delta(q, a), every entry in
 *           [0, n).  Caller-owned host memory, read only, copied before the
 *           call returns.
 *   word    host buffer of letters 0..k-1 (uint8), written only on SRW_OK.
 *   n = 1   gives r = 0 and the empty word (the empty word already resets).
 *   limits  1 <= n <= SRW_MAX_N, 1 <= k <= 255.
 * Every call returns an int status (SRW_OK or a negative code below) and is
 * thread-safe; calls on the default context are serialized.  Device memory
 * and the HIP stream come from srw_set_allocator / srw_set_stream (PyTorch's
 * caching allocator and current stream in the Python binding) or, when those
 * are unset, from hipMalloc and a stream of the library's own.
 */
#ifndef SRW_H
#define SRW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SRW_MAX_N 512

#define SRW_OK 0
#define SRW_EINVAL (-1)        /* null pointer, n or k out of range, delta entry outside [0,n) */
#define SRW_ENOTSYNC (-2)      /* not synchronizing (pair test, Section 2 intro); *r = -1 */
#define SRW_EUNSUPPORTED (-3)  /* n > SRW_MAX_N */
#define SRW_ENOMEM (-4)        /* device memory budget exhausted before the searches met */
#define SRW_EWORDCAP (-5)      /* *r written, the word did not fit word_cap */
#define SRW_EDEVICE (-6)       /* HIP error or no usable GPU; srw_last_error() has the text */
#define SRW_ETIMEOUT (-7)      /* srw_server_poll: nothing completed in time; a solve: its deadline passed */
#define SRW_EINTERNAL (-8)     /* internal check failed (e.g. the word did not verify) */
#define SRW_ENOBOUND (-9)      /* srw_beam: a cut level had no new set before Q was reached */

/* Solve one automaton.  r: out, the reset threshold.  word: out, may be NULL
 * (r only); otherwise room for word_cap letters.  On SRW_EWORDCAP *r is set. */
int srw_solve(int32_t n, int32_t k, const int32_t *delta,
              int32_t *r, uint8_t *word, int64_t word_cap);

/* Solve `count` automata together: each global step expands every active
 * automaton once, with one launch per kernel for all of them.  Automaton i
 * has n[i] states, k[i] letters and its table at delta + delta_off[i].
 * Per automaton: r[i] and status[i] (an SRW_ status) are written.  words may
 * be NULL; otherwise automaton i's word goes to words + word_off[i] with room
 * for word_cap[i] letters.  Returns SRW_OK when every status was written
 * (individual failures are in status[]), or a call-level error. */
int srw_solve_batch(int32_t count, const int32_t *n, const int32_t *k,
                    const int64_t *delta_off, const int32_t *delta,
                    int32_t *r, int32_t *status,
                    const int64_t *word_off, uint8_t *words, const int64_t *word_cap);

/* srw_solve for callers that cannot allocate device memory: code that must
 * not call hipMalloc (a HIP graph being captured, a tight serving loop, a
 * harness that forbids allocation).  A call allocates nothing -- no
 * hipMalloc, no hipFree, no pinned host memory, no torch allocation.  All
 * device memory of its search comes from one array of
 * SRW_NOALLOC_SCRATCH_BYTES (256 MiB) per GPU that is part of the library's
 * code object: it is taken when that code is loaded on the GPU and held
 * until the process ends.  The call runs on the calling thread's current
 * HIP device, on a stream of the library's own; the first call on a device
 * sets up (the scratch address, that stream and its events).  Arguments,
 * results and statuses are those of srw_solve, with one more way to fail: a
 * search whose lists outgrow the scratch (random automata with two letters
 * from about n = 200 on) ends with SRW_ENOMEM.  Calls on one device share
 * its scratch, which keeps the last call's contents; every call clears what
 * it reads before reading it.  Overlapping calls on one device would race on
 * the scratch, so the library serializes them with a per-device lock. */
#define SRW_NOALLOC_SCRATCH_BYTES ((int64_t)256 << 20)
int srw_solve_noalloc(int32_t n, int32_t k, const int32_t *delta,
                      int32_t *r, uint8_t *word, int64_t word_cap);

/* Synchronizability test by state pairs (Section 2 intro): 1 if every pair
 * of states can be mapped to one state, 0 if not, <0 on bad input.  Host
 * code only. */
int srw_check_sync(int32_t n, int32_t k, const int32_t *delta);

/* 1 if |delta(Q, word)| = 1 (Section 1 definition), 0 if not, <0 on bad input. */
int srw_verify(int32_t n, int32_t k, const int32_t *delta, const uint8_t *word, int64_t len);

/* ---- serving: continuous batching ------------------------------------ */

typedef struct srw_config {
    int32_t device;        /* HIP device ordinal */
    int32_t max_slots;     /* automata resident on the device at once (0: 4096) */
    int64_t hbm_budget;    /* bytes of device memory the server may hold (0: 80% of free) */
    int64_t deadline_ms;   /* per request, from admission: SRW_ETIMEOUT after this long (0: none) */
} srw_config;

typedef struct srw_result {
    uint64_t tag;          /* the caller's tag from srw_server_submit */
    int32_t status;        /* SRW_ status of this request */
    int32_t r;             /* reset threshold, -1 unless status is SRW_OK */
    const uint8_t *word;   /* r letters, owned by the server until the next poll */
    double latency_ms;     /* submit -> completion */
    double queue_ms;       /* submit -> admission to the device */
    int64_t est_bytes;     /* the footprint estimate admission used */
    int64_t dev_bytes;     /* device memory its buffers held at the end (0 if never admitted) */
} srw_result;

typedef struct srw_server srw_server;

/* Start a server with its own worker thread and stream.  Requests are
 * admitted while their estimated device footprint fits the budget and a
 * slot is free; admitted automata keep their lists on the device and step
 * together with the rest.  The server searches with the options of the
 * default context (srw_set_option) as they are at this call, per-width
 * values included; "budget", "max_slots", "profile", "deadline_ms",
 * "verbose" and "keep_levels" are not taken (cfg holds the server's own). */
int srw_server_create(srw_server **out, const srw_config *cfg);
/* Non-blocking.  Copies delta.  Results come back through srw_server_poll. */
int srw_server_submit(srw_server *s, int32_t n, int32_t k, const int32_t *delta, uint64_t tag);
/* Up to max completed results, in completion order.  Waits up to timeout_us
 * microseconds for the first one (0: no wait).  Returns the number written
 * (>= 0), SRW_ETIMEOUT if none completed in time, or another error. */
int srw_server_poll(srw_server *s, srw_result *out, int32_t max, int32_t timeout_us);
/* Number of requests submitted but not yet returned by srw_server_poll. */
int64_t srw_server_pending(srw_server *s);
void srw_server_destroy(srw_server *s);

/* ---- plumbing: device memory and stream -------------------------------- */

/* Device memory comes from alloc(bytes, ctx) / free(ptr, ctx) once set
 * (NULL, NULL restores hipMalloc / hipFree).  Only for contexts created
 * after the call. */
int srw_set_allocator(void *(*alloc)(size_t bytes, void *ctx),
                      void (*free_fn)(void *ptr, void *ctx), void *ctx);
/* Launch on this hipStream_t (NULL: the library's own stream). */
int srw_set_stream(void *hip_stream);

/* Tuning and test options of the default context (srw_solve /
 * srw_solve_batch).  Keys:
 *   "budget"      device memory budget in bytes (0: 80% of free memory)
 *   "max_slots"   automata resident at once in srw_solve_batch
 *   "profile"     1: time every kernel class with HIP events (srw_get_stats)
 *                 and run the counting build of the meet kernels (their set
 *                 operations and work in meet_ops_w, meet_work);
 *                 2: time the meet launches only (per set width) -- light
 *                 enough for a timed run;
 *                 0: off
 *   "schedule"    0: smaller frontier first, ties forward (default)
 *                 1: pseudo-random side per step from "sched_seed"
 *                 2: alternate forward / inverse
 *                 3: the step of lower estimated cost, BFS or IBFS, by the
 *                 cost model of Section 2.1.2 (Eq. 1-4 with ExpMark; the
 *                 terms of inclusion reductions, which this search does not
 *                 make, are zero, and there is no step without history and
 *                 no DFS phase, so the paper's greedy comparison of the two
 *                 single-step costs applies).  The first, small steps that
 *                 "persist" runs in one launch keep the rule of schedule 0.
 *                 Every schedule gives the same r and word
 *   "sched_seed"  seed of schedule 1
 *   "meet"        0: auto; 1: always test 256 sets X against LDS-staged
 *                 tiles of 64 sets Y; 2: bucket-sort every forward level
 *                 and test 64-set chunks of it (any choice gives the same
 *                 results; auto sorts the large levels)
 *   "meet_tiles"  tiles of 64 inverse sets per LDS meet block (0: auto)
 *   "meet_rows"   chunked meet: groups of 64 tiles with at most this many
 *                 candidate sets (default and cap 512) test them by
 *                 signature, larger ones AND columns
 *   "meet_groups" chunked meet: groups of 64 tiles per work item (at most;
 *                 default 16)
 *   "meet_order"  chunked meet work items: 1 chunk-major (default), 0 tile-
 *                 range-major (consecutive items share one range of tiles;
 *                 with an inverse level in buckets: within each key of the
 *                 chunks)
 *   "meet_xcd"    bucketed meet: its work items are dealt to eight queues,
 *                 one per XCD, in runs of this many consecutive items, so
 *                 that the chunks scanning one range of tiles share an L2
 *                 (0, the default: one queue)
 *   "meet_bgrid"  blocks of a bucketed meet launch, which take work items
 *                 from queues until they are empty (default 4096)
 *   "meet_grid"   meet blocks per launch, grid-striding over the work items
 *                 (0: one block per work item, up to 2^31-1)
 *   "ysort"       new inverse levels of at least this many candidates are
 *                 kept in order of decreasing cardinality for the meet, so
 *                 that forward sets scan only large enough inverse sets
 *                 (0, the default: never; the same results either way)
 *   "small_cand"  steps with at most this many candidates (and a small
 *                 LDS-tile meet) run in one block, one launch for the whole
 *                 step (default 2048; 0: never)
 *   "bucket"      inverse levels of at least this many sets (default 16384;
 *                 0: never) are kept in buckets by their membership of the
 *                 forward level's 10 most frequent states, and a chunk of
 *                 forward sets scans only the buckets holding every one of
 *                 those states it has in common (the split of Alg. 2); the
 *                 same results either way
 *   "persist"     1 (default): the first steps of every newly admitted
 *                 automaton run in one launch, a block per automaton
 *                 stepping it for as long as its steps are small in the
 *                 sense of "small_cand" (with the schedule 0 side rule);
 *                 0: every step is launched by the host.  The same
 *                 results either way
 *   "<key>@<W>"   a value of "meet_groups", "meet_rows", "small_cand",
 *                 "bucket" or "schedule" for automata of set width W only
 *                 (W = ceil(n/64) = 1..8; -1 removes it), e.g. from the
 *                 autotuner's table; it takes precedence over the key's
 *                 value for every width
 *   "reduce"      1: every new level is self-reduced before the meet test
 *                 (Alg. 1): a forward set with another set of its level
 *                 inside it, an inverse set with another one around it, is
 *                 dropped from the level and stays visited; 2: also one
 *                 with a set of an earlier level of its side inside it
 *                 (forward) or around it (inverse), the reduction by
 *                 history.  r is the same, the word may be another
 *                 shortest one.  Small steps then run per phase (no
 *                 one-block or one-launch steps).  The marks are found by
 *                 brute force over the level (and the history), so large
 *                 levels are slow.  0 (default): no reduction
 *   "deadline_ms" per automaton, from its admission: a solve still running
 *                 after this long ends with SRW_ETIMEOUT (0: no deadline)
 *   "verbose"     1: one line per step of a single solve on stderr
 *   "keep_levels" 1: keep the device lists of the last srw_solve for
 *                 srw_last_levels
 * Unknown keys give SRW_EINVAL. */
int srw_set_option(const char *key, int64_t value);

typedef struct srw_stats {
    int64_t solves;            /* automata finished */
    int64_t steps;             /* expansion steps over all automata */
    int64_t global_steps;      /* batched steps (one launch of each kernel) */
    int64_t candidates;        /* subsets expanded: k * |list| per step */
    int64_t unique;            /* new sets kept after duplicate removal */
    int64_t pairs;             /* meet pairs |L_f| * |L_b| over all checks */
    int64_t cand_words;        /* candidates * W (64-bit words) */
    int64_t pair_words;        /* pairs * W */
    int64_t launches[8];       /* per kernel class, see below */
    double ms[8];              /* per kernel class, with "profile" on */
    int64_t bytes_expand;      /* algorithmic bytes of the expand kernel */
    int64_t bytes_insert;      /* algorithmic bytes of the insert kernel */
    int64_t bytes_compact;     /* algorithmic bytes of count+compact */
    int64_t peak_device_bytes; /* device memory held at peak */
    int64_t meet_launches_w[8];/* meet kernel launches per set width W = index + 1 */
    double meet_ms_w[8];       /* their time, with "profile" 1 or 2 */
    int64_t pair_words_w[8];   /* their brute-force pair-word count */
    int64_t meet_ops_w[8];     /* set operations they performed, in 32-bit lane-ops
                                  (2 per 64-bit AND, 4 per word of a subset test),
                                  with "profile" 1 (the counting build of the kernels) */
    double host_ms[4];         /* wall time of the steps by phase: 0 sides, growth and
                                  copies; 1 descriptors, uploads and launches; 2 waiting
                                  for the device; 3 results, meets and words */
    int64_t meet_work[8];      /* chunked meets, with "profile" 1: 0 work items,
                                  1 tile groups scanned, 2 groups with candidate sets,
                                  3 candidates tested by signature, 4 signature passes
                                  (full row tests), 5 tiles tested column by column,
                                  6 tiles scanned; 7 launches of the meet against an
                                  inverse level in buckets (counted always) */
    int64_t meet_b_launches_w[8];/* of those bucketed meet launches, per set width */
    double meet_b_ms_w[8];     /* their own time, with "profile" 1 or 2 */
    int64_t meet_b_ops_w[8];   /* their share of meet_ops_w, with "profile" 1 */
    int64_t reduced;           /* sets the self-reduction (option "reduce") dropped */
} srw_stats;
/* kernel classes: 0 expand (and whole one-block steps), 1 insert, 2 count+scan+compact, 3 meet
 * preparation (transpose of inverse levels, bucket sort of forward levels),
 * 4 meet, 5 trace, 6 init/rehash/fill/copies, 7 whole steps (host view) */

int srw_get_stats(srw_stats *out);
int srw_reset_stats(void);

/* Lists kept by the last srw_solve with "keep_levels" on (side 0 forward,
 * 1 inverse).  With rows == NULL only *nlev and *nrows are written;
 * otherwise off[0..nlev] (level L holds rows off[L]..off[L+1]-1),
 * rows[nrows * W] (W = ceil(n/64) words, state q = bit q%64 of word q/64)
 * and par[nrows] (the key that produced the row: forward i*k+a, inverse
 * a*|previous level|+i; 0xFFFFFFFF on level 0). */
int srw_last_levels(int32_t side, int32_t *nlev, int64_t *nrows,
                    int64_t *off, uint64_t *rows, uint32_t *par);

/* Upper bound on the reset threshold by beam search (CutOff-IBFS, cited in
 * Section 1.3.2; its beam size is the subject of Section 2.1.3): the
 * inverse side of the search of srw_solve alone, from the singletons, with
 * every new level cut to its `width` sets of largest cardinality (ties: the
 * least key, i.e. the lexicographically least word).  Sets cut from a level
 * stay visited.  *R is the first depth whose kept level holds Q, so R >= r;
 * `word` (if not NULL, word_cap >= R) gets a reset word of length R, the one
 * of the first such set, checked on the host.  With a width at least the
 * size of every level this is the exact search: R = r and the word is the
 * one srw_solve returns.  One block of the GPU runs each automaton from
 * start to end.  Statuses as srw_solve, plus SRW_ENOBOUND when a level ends
 * up empty before Q is reached (the cut can lead into a dead end); "budget"
 * and "deadline_ms" of srw_set_option apply. */
int srw_beam(int32_t n, int32_t k, const int32_t *delta, int64_t width, int32_t *R,
             uint8_t *word, int64_t word_cap);
/* srw_beam of `count` automata at once (arrays as in srw_solve_batch, plus
 * width[i] per automaton); the return value is SRW_OK or an error of the
 * call itself, each automaton's status is in status[i]. */
int srw_beam_batch(int32_t count, const int32_t *n, const int32_t *k, const int64_t *delta_off,
                   const int32_t *delta, const int64_t *width, int32_t *R, int32_t *status,
                   const int64_t *word_off, uint8_t *words, const int64_t *word_cap);

/* Upper bound on the reset threshold by Eppstein's greedy heuristic (cited
 * in Section 1.3.2 with its O(n^3 + k n^2) time and (n^3-n)/3 length bound;
 * Section 2.1.3 computes it before the beam search).  From S = Q, each round
 * takes the pair {p, q} of S whose shortest merging word is shortest (ties:
 * the least p, then the least q), appends that word and replaces S with its
 * image, until one state is left.  The merging word of a pair is its
 * lexicographically least shortest one: the least letter that takes the
 * pair to a single state or to a pair one step closer, repeated.  *len gets
 * the length of the whole word (an upper bound on r); `word` (if not NULL)
 * gets the word when word_cap >= *len, else the status is SRW_EWORDCAP with
 * *len still written.  Every word is checked on the host.  One block of the
 * GPU runs each automaton: all pair distances by a breadth-first search
 * backwards over pairs, then the rounds.  Statuses as srw_solve, except that
 * a non-synchronizing automaton is found on the device (a pair of the
 * current set that no word merges: SRW_ENOTSYNC), not by a host check first;
 * "budget" and "deadline_ms" of srw_set_option apply. */
int srw_eppstein(int32_t n, int32_t k, const int32_t *delta, int64_t *len, uint8_t *word,
                 int64_t word_cap);
/* srw_eppstein of `count` automata at once (arrays as in srw_solve_batch,
 * len[i] per automaton, -1 unless its status is SRW_OK or SRW_EWORDCAP); the
 * return value is SRW_OK or an error of the call itself, each automaton's
 * status is in status[i]. */
int srw_eppstein_batch(int32_t count, const int32_t *n, const int32_t *k, const int64_t *delta_off,
                       const int32_t *delta, int64_t *len, int32_t *status,
                       const int64_t *word_off, uint8_t *words, const int64_t *word_cap);

/* The upper bound of Section 2.1.3: Eppstein's heuristic (srw_eppstein),
 * then the beam search (srw_beam) with the small beam w0 = n, then the beam
 * search with a beam size chosen so that it costs a small fraction of the
 * exact search (the paper states this policy in words only; the reading
 * here):
 *   - B = the least bound so far;
 *   - the exact search's cost C = 2 * (U(0) + ... + U(ceil(B/2))) sets,
 *     U(d) the first beam's level sizes before their cut up to its first
 *     level c larger than w0 (these are the exact search's levels), and
 *     U(c) * g^(d-c) beyond, g = U(c) / U(c-1);
 *   - width = ceil(C / (16 B)) (a beam of width w keeps about w * B sets),
 *     clamped to [w0, 2^20]; w0 when the first beam cut no level (it was
 *     the exact search).
 * *R is the least of the (up to) three bounds and `word` (if not NULL,
 * word_cap >= *R) the word of the first source reaching it, in the order
 * Eppstein, first beam, second beam; *width is the chosen beam size.
 * Statuses as srw_eppstein (a beam ending at an empty level is no error
 * here: its bound is left out). */
int srw_bound(int32_t n, int32_t k, const int32_t *delta, int32_t *R, int64_t *width,
              uint8_t *word, int64_t word_cap);
/* srw_bound of `count` automata at once (arrays as in srw_solve_batch, plus
 * width[i]); each automaton's status is in status[i]. */
int srw_bound_batch(int32_t count, const int32_t *n, const int32_t *k, const int64_t *delta_off,
                    const int32_t *delta, int32_t *R, int64_t *width, int32_t *status,
                    const int64_t *word_off, uint8_t *words, const int64_t *word_cap);

/* The side of every step of the last srw_solve run with "keep_levels" on,
 * in order (0 forward, 1 inverse): *steps = their count; with sides != NULL
 * also sides[0..*steps) (SRW_EINVAL when cap < *steps).  A test and
 * diagnostic hook for the direction schedules. */
int srw_last_sides(int32_t *steps, uint8_t *sides, int64_t cap);

/* Text of the last error of the calling thread. */
const char *srw_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SRW_H */
