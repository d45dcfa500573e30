/*
 * srw_oracle.c -- plain, slow, single-threaded CPU oracle for shortest reset
 * words.  TEST INFRASTRUCTURE ONLY: the library never links, loads or calls
 * anything in this file; only the test suite, the smoke check and the CPU
 * baseline of the benchmark do.  It shares no code with the GPU path.
 *
 * What it computes (paper: Szykula & Zyzik, "An Improved Algorithm for
 * Finding the Shortest Synchronizing Words"):
 *   - the reset threshold r = min |w| with |delta(Q,w)| = 1   (Section 1)
 *   - the lexicographically least reset word of length r (letters ordered by
 *     index); the paper returns "a" shortest word via predecessor pointers
 *     (end of Section 2 intro) without fixing which one, so the lex-least one
 *     is the reading taken here.
 *
 * Functions and the passage each follows:
 *   orc_is_synchronizing  pair-merging test, Section 2 intro (every pair of
 *                         states can be mapped to one state)
 *   orc_image/preimage    the two definitions at the start of Section 2
 *   orc_bruteforce        trivial algorithm of Section 1.3: all words of
 *                         length 0,1,2,... in lex order
 *   orc_exhaustive        standard power-automaton BFS over all 2^n subsets
 *                         (Section 1.3.1), n <= 24
 *   orc_forward           forward BFS over subsets from Q (one side of
 *                         Alg. 1), stops at the first singleton
 *   orc_bidir_reduced     the same with every new level self-reduced
 *                         (non-minimal forward / non-maximal inverse sets
 *                         dropped, Alg. 1); parity unpinned beyond r and
 *                         the invariants its tests check
 *   orc_bidir_history     self-reduction and reduction by history (sets
 *                         dominated by a set of an earlier level dropped);
 *                         pinned the same way
 *   orc_bidir_reduce      either reduction by flags, with the drops found
 *                         by all pairs or by Alg. 2; pinned by equality of
 *                         the two and the invariants above
 *   orc_beam              beam search (CutOff-IBFS, cited in Section 1.3.2
 *                         and tuned in Section 2.1.3): the inverse side of
 *                         the plain search with every level cut to its
 *                         largest sets; an upper bound R >= r and a reset
 *                         word of length R
 *   orc_pair_dist         shortest merging word length of every pair of
 *                         states, from its recursive definition (the pair
 *                         test of the Section 2 intro, with lengths)
 *   orc_eppstein          Eppstein's greedy heuristic (cited in Section
 *                         1.3.2, the first bound of Section 2.1.3): merge
 *                         the pair of the current set with the shortest
 *                         merging word, until one state is left
 *   orc_bidir             plain bidirectional BFS (Alg. 1 with only the
 *                         duplicate removal kept): forward images from Q,
 *                         inverse preimages from the singletons, meet test
 *                         X subset-of Y after every step.  The meet is either
 *                         brute force over all pairs (the definition) or
 *                         Alg. 2 MarkSupersets followed by a scan of the
 *                         marked sets for the least pair.
 *
 * Ordering conventions (these make the returned word the lex-least one):
 *   forward level: candidate key g = i*k + a (parent index i, letter a)
 *   inverse level: candidate key g = a*|L| + i (letter-major; the letter
 *                  applied last is the FIRST letter of the inverse half)
 *   duplicates: the smallest key wins; sets already seen on an earlier level
 *   of the same side are dropped; empty preimages are dropped.
 *
 * Dedup here is by lexicographic sort, the paper's own method (Alg. 1).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOTSYNC (-2)
#define ORC_ELIMIT (-3)
#define ORC_ENOMEM (-4)
#define ORC_EWORDCAP (-5)

#define ORC_MAX_N 512

static int nwords(int n) { return (n + 63) / 64; }

static int check_input(int n, int k, const int32_t *delta) {
    if (n < 1 || n > ORC_MAX_N || k < 1 || k > 255 || !delta) return ORC_EINVAL;
    for (int64_t i = 0; i < (int64_t)n * k; i++)
        if (delta[i] < 0 || delta[i] >= n) return ORC_EINVAL;
    return ORC_OK;
}

static int getbit(const u64 *S, int q) { return (int)((S[q >> 6] >> (q & 63)) & 1u); }
static void setbit(u64 *S, int q) { S[q >> 6] |= (u64)1 << (q & 63); }

static int popcount_set(const u64 *S, int W) {
    int c = 0;
    for (int w = 0; w < W; w++) c += __builtin_popcountll(S[w]);
    return c;
}

/* delta(S, a) = { delta(q, a) | q in S }  (Section 2) */
void orc_image(int n, int k, const int32_t *delta, int a, const u64 *S, u64 *X) {
    int W = nwords(n);
    (void)k;
    memset(X, 0, sizeof(u64) * W);
    for (int q = 0; q < n; q++)
        if (getbit(S, q)) setbit(X, delta[(int64_t)a * n + q]);
}

/* delta^-1(S, a) = { q | delta(q, a) in S }  (Section 2) */
void orc_preimage(int n, int k, const int32_t *delta, int a, const u64 *S, u64 *Y) {
    int W = nwords(n);
    (void)k;
    memset(Y, 0, sizeof(u64) * W);
    for (int q = 0; q < n; q++)
        if (getbit(S, delta[(int64_t)a * n + q])) setbit(Y, q);
}

/* The automaton is synchronizing iff every pair {p,q} can be mapped to a
 * single state.  Mergeable pairs are the least fixpoint of: {p,p} is
 * mergeable; {p,q} is mergeable if some letter maps it to a mergeable pair. */
int orc_is_synchronizing(int n, int k, const int32_t *delta) {
    int rc = check_input(n, k, delta);
    if (rc) return rc;
    unsigned char *m = calloc((size_t)n * n, 1);
    if (!m) return ORC_ENOMEM;
    for (int p = 0; p < n; p++) m[(size_t)p * n + p] = 1;
    int changed = 1;
    while (changed) {
        changed = 0;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) {
                if (m[(size_t)p * n + q]) continue;
                for (int a = 0; a < k; a++) {
                    int pp = delta[(int64_t)a * n + p], qq = delta[(int64_t)a * n + q];
                    if (m[(size_t)pp * n + qq]) {
                        m[(size_t)p * n + q] = m[(size_t)q * n + p] = 1;
                        changed = 1;
                        break;
                    }
                }
            }
    }
    int all = 1;
    for (int p = 0; p < n && all; p++)
        for (int q = p + 1; q < n; q++)
            if (!m[(size_t)p * n + q]) { all = 0; break; }
    free(m);
    return all;
}

/* 1 if |delta(Q, word)| = 1, 0 if not, <0 on bad input (Section 1). */
int orc_verify(int n, int k, const int32_t *delta, const uint8_t *word, int64_t len) {
    int rc = check_input(n, k, delta);
    if (rc) return rc;
    int W = nwords(n);
    u64 S[8], X[8];
    memset(S, 0, sizeof S);
    for (int q = 0; q < n; q++) setbit(S, q);
    for (int64_t i = 0; i < len; i++) {
        if (word[i] >= k) return ORC_EINVAL;
        orc_image(n, k, delta, word[i], S, X);
        memcpy(S, X, sizeof(u64) * W);
    }
    return popcount_set(S, W) == 1;
}

/* ---------------- trivial algorithm: all words in lex order ------------- */

static int bf_search(int n, int k, const int32_t *delta, int W, int depth, int len,
                     const u64 *S, uint8_t *word) {
    if (depth == len) return popcount_set(S, W) == 1;
    u64 X[8];
    for (int a = 0; a < k; a++) {
        orc_image(n, k, delta, a, S, X);
        word[depth] = (uint8_t)a;
        if (bf_search(n, k, delta, W, depth + 1, len, X, word)) return 1;
    }
    return 0;
}

/* Checks every word of length 0,1,...,max_len in lexicographic order and
 * returns the first reset word (Section 1.3, the trivial O(n k^r) method). */
int orc_bruteforce(int n, int k, const int32_t *delta, int max_len,
                   int32_t *r, uint8_t *word, int64_t word_cap) {
    int rc = check_input(n, k, delta);
    if (rc) return rc;
    int W = nwords(n);
    u64 Q[8];
    memset(Q, 0, sizeof Q);
    for (int q = 0; q < n; q++) setbit(Q, q);
    uint8_t *buf = malloc((size_t)max_len + 1);
    if (!buf) return ORC_ENOMEM;
    for (int len = 0; len <= max_len; len++) {
        if (bf_search(n, k, delta, W, 0, len, Q, buf)) {
            *r = len;
            if (word) {
                if (word_cap < len) { free(buf); return ORC_EWORDCAP; }
                memcpy(word, buf, (size_t)len);
            }
            free(buf);
            return ORC_OK;
        }
    }
    free(buf);
    return ORC_ELIMIT;
}

/* ------------- standard power-automaton BFS over all 2^n subsets ------- */

/* Breadth-first search in the power automaton from Q (Section 1.3.1).  The
 * queue is processed first-in first-out and letters in increasing order, so
 * the first visit of a subset is by its lex-least shortest word.  r is the
 * least distance of a singleton; among singletons at that distance the one
 * discovered first carries the lex-least word.  n <= 24. */
int orc_exhaustive(int n, int k, const int32_t *delta, int32_t *r,
                   uint8_t *word, int64_t word_cap) {
    int rc = check_input(n, k, delta);
    if (rc) return rc;
    if (n > 24) return ORC_EINVAL;
    size_t N = (size_t)1 << n;
    int32_t *dist = malloc(N * sizeof(int32_t));
    uint32_t *from = malloc(N * sizeof(uint32_t));
    uint8_t *via = malloc(N);
    uint32_t *queue = malloc(N * sizeof(uint32_t));
    if (!dist || !from || !via || !queue) {
        free(dist); free(from); free(via); free(queue);
        return ORC_ENOMEM;
    }
    for (size_t i = 0; i < N; i++) dist[i] = -1;
    uint32_t full = (uint32_t)(N - 1);
    size_t head = 0, tail = 0;
    dist[full] = 0;
    queue[tail++] = full;
    while (head < tail) {
        uint32_t S = queue[head++];
        for (int a = 0; a < k; a++) {
            uint32_t X = 0;
            for (int q = 0; q < n; q++)
                if (S >> q & 1u) X |= 1u << delta[(int64_t)a * n + q];
            if (dist[X] < 0) {
                dist[X] = dist[S] + 1;
                from[X] = S;
                via[X] = (uint8_t)a;
                queue[tail++] = X;
            }
        }
    }
    /* singletons in discovery order */
    int best = -1;
    uint32_t best_set = 0;
    for (size_t i = 0; i < tail; i++) {
        uint32_t X = queue[i];
        if (__builtin_popcount(X) == 1) {
            if (best < 0 || dist[X] < best) { best = dist[X]; best_set = X; }
            break; /* BFS order is nondecreasing in distance: first is least */
        }
    }
    int out = ORC_OK;
    if (best < 0) {
        out = ORC_ENOTSYNC;
    } else {
        *r = best;
        if (word) {
            if (word_cap < best) out = ORC_EWORDCAP;
            else {
                uint32_t X = best_set;
                for (int i = best - 1; i >= 0; i--) { word[i] = via[X]; X = from[X]; }
            }
        }
    }
    free(dist); free(from); free(via); free(queue);
    return out;
}

/* ---------------------- level lists with sorted dedup ------------------- */

typedef struct {
    int W;
    u64 *rows;          /* all visited sets of this side, level after level */
    int64_t *par;       /* candidate key g that produced the row (-1 at level 0) */
    int64_t nrows, cap;
    int64_t *off;       /* level L holds rows off[L] .. off[L+1]-1 */
    int nlev, levcap;
    int64_t *sorted;    /* row ids of all visited rows in row order */
    u64 *ghost;         /* sets dropped by a reduction that still count as
                           visited (reduce flag 8), sorted in row order */
    int64_t nghost, ghost_cap;
} Side;

static const u64 *g_rows;
static int g_W;

static int rowcmp(const u64 *a, const u64 *b, int W) {
    for (int w = 0; w < W; w++) {
        if (a[w] < b[w]) return -1;
        if (a[w] > b[w]) return 1;
    }
    return 0;
}

/* order candidates by (set, key) */
static int cmp_cand(const void *pa, const void *pb) {
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    int c = rowcmp(g_rows + a * g_W, g_rows + b * g_W, g_W);
    if (c) return c;
    return (a > b) - (a < b);
}

static int side_reserve(Side *s, int64_t more) {
    if (s->nrows + more > s->cap) {
        int64_t nc = s->cap ? s->cap : 1024;
        while (nc < s->nrows + more) nc *= 2;
        u64 *r = realloc(s->rows, (size_t)nc * s->W * sizeof(u64));
        if (!r) return ORC_ENOMEM;
        s->rows = r;
        int64_t *p = realloc(s->par, (size_t)nc * sizeof(int64_t));
        if (!p) return ORC_ENOMEM;
        s->par = p;
        int64_t *so = realloc(s->sorted, (size_t)nc * sizeof(int64_t));
        if (!so) return ORC_ENOMEM;
        s->sorted = so;
        s->cap = nc;
    }
    if (s->nlev + 2 > s->levcap) {
        int nl = s->levcap ? s->levcap * 2 : 64;
        int64_t *o = realloc(s->off, (size_t)nl * sizeof(int64_t));
        if (!o) return ORC_ENOMEM;
        s->off = o;
        s->levcap = nl;
    }
    return ORC_OK;
}

static void side_free(Side *s) {
    free(s->rows); free(s->par); free(s->off); free(s->sorted); free(s->ghost);
    memset(s, 0, sizeof *s);
}

static int64_t level_size(const Side *s, int L) { return s->off[L + 1] - s->off[L]; }
static const u64 *level_row(const Side *s, int L, int64_t i) {
    return s->rows + (s->off[L] + i) * s->W;
}

/* binary search of a set among the visited rows, then among the ghosts */
static int visited(const Side *s, const u64 *x) {
    int64_t lo = 0, hi = s->nrows;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        int c = rowcmp(s->rows + s->sorted[mid] * s->W, x, s->W);
        if (c == 0) return 1;
        if (c < 0) lo = mid + 1; else hi = mid;
    }
    lo = 0, hi = s->nghost;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        int c = rowcmp(s->ghost + mid * s->W, x, s->W);
        if (c == 0) return 1;
        if (c < 0) lo = mid + 1; else hi = mid;
    }
    return 0;
}

static int cmp_ghost(const void *a, const void *b) {
    return rowcmp((const u64 *)a, (const u64 *)b, g_W);
}

/* Appends a new level made of the candidates cand[0..C-1] (key = index):
 * empty sets dropped, the least key of each set kept, sets already visited
 * dropped, survivors stored in key order. */
static int side_push_level(Side *s, const u64 *cand, int64_t C) {
    int W = s->W;
    int64_t *idx = malloc((size_t)(C ? C : 1) * sizeof(int64_t));
    unsigned char *keep = calloc((size_t)(C ? C : 1), 1);
    if (!idx || !keep) { free(idx); free(keep); return ORC_ENOMEM; }
    for (int64_t g = 0; g < C; g++) idx[g] = g;
    g_rows = cand; g_W = W;
    qsort(idx, (size_t)C, sizeof(int64_t), cmp_cand);
    int64_t U = 0;
    for (int64_t t = 0; t < C; t++) {
        int64_t g = idx[t];
        if (t > 0 && rowcmp(cand + idx[t - 1] * W, cand + g * W, W) == 0) continue;
        if (popcount_set(cand + g * W, W) == 0) continue;
        if (visited(s, cand + g * W)) continue;
        keep[g] = 1;
        U++;
    }
    int rc = side_reserve(s, U);
    if (rc) { free(idx); free(keep); return rc; }
    int64_t base = s->nrows;
    int64_t pos = base;
    for (int64_t g = 0; g < C; g++) {
        if (!keep[g]) continue;
        memcpy(s->rows + pos * W, cand + g * W, sizeof(u64) * W);
        s->par[pos] = g;
        pos++;
    }
    /* merge the new rows into the sorted visited index */
    int64_t *newsorted = malloc((size_t)(U ? U : 1) * sizeof(int64_t));
    int64_t *merged = malloc((size_t)(s->nrows + U ? s->nrows + U : 1) * sizeof(int64_t));
    if (!newsorted || !merged) { free(idx); free(keep); free(newsorted); free(merged); return ORC_ENOMEM; }
    for (int64_t i = 0; i < U; i++) newsorted[i] = base + i;
    g_rows = s->rows; g_W = W;
    qsort(newsorted, (size_t)U, sizeof(int64_t), cmp_cand);
    int64_t a = 0, b = 0, m = 0;
    while (a < s->nrows || b < U) {
        if (b >= U || (a < s->nrows &&
                       rowcmp(s->rows + s->sorted[a] * W, s->rows + newsorted[b] * W, W) < 0))
            merged[m++] = s->sorted[a++];
        else
            merged[m++] = newsorted[b++];
    }
    memcpy(s->sorted, merged, (size_t)m * sizeof(int64_t));
    free(newsorted); free(merged);
    s->nrows += U;
    s->off[s->nlev + 1] = s->nrows;
    s->nlev++;
    free(idx); free(keep);
    return ORC_OK;
}

static int side_init(Side *s, int W, const u64 *rows, int64_t count) {
    memset(s, 0, sizeof *s);
    s->W = W;
    int rc = side_reserve(s, count);
    if (rc) return rc;
    s->off[0] = 0;
    s->nlev = 0;
    /* level 0: keep the given order; its "keys" are the positions */
    rc = side_push_level(s, rows, count);
    if (rc) return rc;
    for (int64_t i = 0; i < s->nrows; i++) s->par[i] = -1;
    return ORC_OK;
}

/* forward step: L <- { delta(S, a) }, key g = i*k + a */
static int step_forward(Side *s, int n, int k, const int32_t *delta) {
    int W = s->W;
    int L = s->nlev - 1;
    int64_t m = level_size(s, L);
    u64 *cand = malloc((size_t)((m * k) > 0 ? m * k : 1) * W * sizeof(u64));
    if (!cand) return ORC_ENOMEM;
    for (int64_t i = 0; i < m; i++)
        for (int a = 0; a < k; a++)
            orc_image(n, k, delta, a, level_row(s, L, i), cand + (i * k + a) * W);
    int rc = side_push_level(s, cand, m * k);
    free(cand);
    return rc;
}

/* inverse step: L <- { delta^-1(S, a) }, key g = a*|L| + i */
static int step_inverse(Side *s, int n, int k, const int32_t *delta) {
    int W = s->W;
    int L = s->nlev - 1;
    int64_t m = level_size(s, L);
    u64 *cand = malloc((size_t)((m * k) > 0 ? m * k : 1) * W * sizeof(u64));
    if (!cand) return ORC_ENOMEM;
    for (int a = 0; a < k; a++)
        for (int64_t i = 0; i < m; i++)
            orc_preimage(n, k, delta, a, level_row(s, L, i), cand + ((int64_t)a * m + i) * W);
    int rc = side_push_level(s, cand, m * k);
    free(cand);
    return rc;
}

static int is_subset(const u64 *X, const u64 *Y, int W) {
    for (int w = 0; w < W; w++)
        if (X[w] & ~Y[w]) return 0;
    return 1;
}

/* Self-reduction of the newest level of a side (Alg. 1: deleting the
 * non-minimal sets of the BFS list, and on the IBFS side the analogous
 * deletion of the non-maximal sets).  Forward (dir 0): a set is dropped when
 * another set of its level is a proper subset of it.  Inverse (dir 1): a
 * set is dropped when another set of its level is a proper superset of it.
 * The sets of a level are distinct, so "another set contained in it" is
 * already a proper subset.  Survivors keep key order (and so the ranks that
 * the next level's keys refer to are ranks among survivors).  Dropped sets
 * leave the visited index as well: they never enter the history, and may be
 * generated again later.  Brute force over all pairs of the level, or, with
 * alg2, the marks of Alg. 2 (alg2_drops). */
static int alg2_drops(const Side *s, int dir, int history, int n, unsigned char *drop,
                      int64_t *tests);

static int side_reduce(Side *s, int dir, int history, int alg2, int keep_dropped, int n,
                       int64_t *tests) {
    const int W = s->W, L = s->nlev - 1;
    const int64_t m = level_size(s, L), base = s->off[L];
    unsigned char *drop = calloc((size_t)(m ? m : 1), 1);
    if (!drop) return ORC_ENOMEM;
    if (alg2) {
        int rc = alg2_drops(s, dir, history, n, drop, tests);
        if (rc) { free(drop); return rc; }
    }
    for (int64_t i = 0; i < m && !alg2; i++) {
        const u64 *A = level_row(s, L, i);
        for (int64_t j = 0; j < m && !drop[i]; j++) {
            if (j == i) continue;
            const u64 *B = level_row(s, L, j);
            (*tests)++;
            if (dir == 0 ? is_subset(B, A, W) : is_subset(A, B, W)) drop[i] = 1;
        }
        /* reduction by history: a set stored on an earlier level of the side
         * that lies inside A (forward) or contains A (inverse) reaches the
         * same singletons with a shorter word */
        for (int64_t h = 0; history && h < base && !drop[i]; h++) {
            const u64 *H = s->rows + h * W;
            (*tests)++;
            if (dir == 0 ? is_subset(H, A, W) : is_subset(A, H, W)) drop[i] = 1;
        }
    }
    if (keep_dropped) {
        /* the dropped sets stay visited: they join the sorted ghost rows */
        int64_t nd = 0;
        for (int64_t i = 0; i < m; i++) nd += drop[i];
        if (s->nghost + nd > s->ghost_cap) {
            int64_t cap = 2 * (s->nghost + nd) + 16;
            u64 *g = realloc(s->ghost, (size_t)cap * W * sizeof(u64));
            if (!g) { free(drop); return ORC_ENOMEM; }
            s->ghost = g;
            s->ghost_cap = cap;
        }
        for (int64_t i = 0; i < m; i++)
            if (drop[i]) memcpy(s->ghost + (s->nghost++) * W, level_row(s, L, i), sizeof(u64) * W);
        g_W = W;
        qsort(s->ghost, (size_t)s->nghost, sizeof(u64) * W, cmp_ghost);
    }
    int64_t pos = base;
    for (int64_t i = 0; i < m; i++) {
        if (drop[i]) continue;
        if (pos != base + i) {
            memmove(s->rows + pos * W, s->rows + (base + i) * W, sizeof(u64) * W);
            s->par[pos] = s->par[base + i];
        }
        pos++;
    }
    free(drop);
    s->nrows = pos;
    s->off[L + 1] = pos;
    /* the visited index again, over the remaining rows */
    for (int64_t t = 0; t < s->nrows; t++) s->sorted[t] = t;
    g_rows = s->rows; g_W = W;
    qsort(s->sorted, (size_t)s->nrows, sizeof(int64_t), cmp_cand);
    return ORC_OK;
}

/* ---------------- Alg. 2: MarkSupersets(A, B, d) ---------------------- */

typedef struct {
    const Side *A_side; int A_lev;   /* A: forward level, via lex-sorted ids */
    const Side *B_side; int B_lev;   /* B: inverse level */
    const int64_t *A;                /* indices into the A level, lex sorted */
    int64_t *B;                      /* indices into the B level (permuted) */
    int n, W, minsize;
    int64_t tests;
    int proper;                      /* A and B are one list: skip a set against itself */
} MarkCtx;

static const u64 *A_row(const MarkCtx *c, int64_t t) { return level_row(c->A_side, c->A_lev, c->A[t]); }
static const u64 *B_row(const MarkCtx *c, int64_t t) { return level_row(c->B_side, c->B_lev, c->B[t]); }

/* Returns the new end of the active part of B: the sets of B[blo..bhi) that
 * are supersets of some set of A[alo..ahi) are moved behind it. */
static int64_t mark_supersets(MarkCtx *c, int64_t alo, int64_t ahi,
                              int64_t blo, int64_t bhi, int d) {
    if (alo >= ahi || blo >= bhi) return bhi;
    if (ahi - alo < c->minsize || d >= c->n) {
        int64_t b = blo;
        while (b < bhi) {
            int hit = 0;
            for (int64_t a = alo; a < ahi && !hit; a++) {
                if (c->proper && c->A[a] == c->B[b]) continue;
                c->tests++;
                hit = is_subset(A_row(c, a), B_row(c, b), c->W);
            }
            if (hit) {
                int64_t t = c->B[b]; c->B[b] = c->B[bhi - 1]; c->B[bhi - 1] = t;
                bhi--;
            } else {
                b++;
            }
        }
        return bhi;
    }
    /* A is lex sorted and all its sets agree on states 0..d-1, so the sets
     * without state d form a prefix: find its end by binary search. */
    int64_t lo = alo, hi = ahi;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (getbit(A_row(c, mid), d)) hi = mid; else lo = mid + 1;
    }
    int64_t split = lo;
    bhi = mark_supersets(c, alo, split, blo, bhi, d + 1);
    /* partition the still active part of B: sets containing d go last */
    int64_t i = blo, j = bhi;
    while (i < j) {
        if (getbit(B_row(c, i), d)) {
            j--;
            int64_t t = c->B[i]; c->B[i] = c->B[j]; c->B[j] = t;
        } else {
            i++;
        }
    }
    return mark_supersets(c, split, ahi, j, bhi, d + 1);
}

/* lexicographic order of characteristic vectors, state 0 first */
static const Side *g_lex_side;
static int g_lex_lev;
static int g_lex_n;
static int cmp_lex(const void *pa, const void *pb) {
    const u64 *x = level_row(g_lex_side, g_lex_lev, *(const int64_t *)pa);
    const u64 *y = level_row(g_lex_side, g_lex_lev, *(const int64_t *)pb);
    for (int q = 0; q < g_lex_n; q++) {
        int bx = getbit(x, q), by = getbit(y, q);
        if (bx != by) return bx - by;
    }
    return 0;
}

/* least (i, j) with X_i subset of Y_j, or found = 0 */
static int meet(const Side *F, const Side *B, int n, int mode, int64_t *bi, int64_t *bj,
                int *found, int64_t *tests) {
    int W = F->W;
    int lf = F->nlev - 1, lb = B->nlev - 1;
    int64_t nx = level_size(F, lf), ny = level_size(B, lb);
    *found = 0;
    if (mode == 0) {
        /* the definition: scan pairs in lexicographic (i, j) order */
        for (int64_t i = 0; i < nx; i++)
            for (int64_t j = 0; j < ny; j++) {
                (*tests)++;
                if (is_subset(level_row(F, lf, i), level_row(B, lb, j), W)) {
                    *bi = i; *bj = j; *found = 1;
                    return ORC_OK;
                }
            }
        return ORC_OK;
    }
    /* Alg. 2: mark every Y that is a superset of some X, then the least
     * pair is found among the marked Y only (every meeting pair's Y is
     * marked). */
    int64_t *A = malloc((size_t)(nx ? nx : 1) * sizeof(int64_t));
    int64_t *Bi = malloc((size_t)(ny ? ny : 1) * sizeof(int64_t));
    if (!A || !Bi) { free(A); free(Bi); return ORC_ENOMEM; }
    for (int64_t i = 0; i < nx; i++) A[i] = i;
    for (int64_t j = 0; j < ny; j++) Bi[j] = j;
    g_lex_side = F; g_lex_lev = lf; g_lex_n = n;
    qsort(A, (size_t)nx, sizeof(int64_t), cmp_lex);
    MarkCtx c = {F, lf, B, lb, A, Bi, n, W, 16, 0, 0};
    int64_t active = mark_supersets(&c, 0, nx, 0, ny, 0);
    *tests += c.tests;
    int64_t nm = ny - active;
    if (nm > 0) {
        int64_t *marked = Bi + active;
        /* ascending j */
        for (int64_t a = 1; a < nm; a++) {
            int64_t v = marked[a], b = a - 1;
            while (b >= 0 && marked[b] > v) { marked[b + 1] = marked[b]; b--; }
            marked[b + 1] = v;
        }
        for (int64_t i = 0; i < nx && !*found; i++)
            for (int64_t t = 0; t < nm; t++) {
                (*tests)++;
                if (is_subset(level_row(F, lf, i), level_row(B, lb, marked[t]), W)) {
                    *bi = i; *bj = marked[t]; *found = 1;
                    break;
                }
            }
    }
    free(A); free(Bi);
    return ORC_OK;
}

/* Self-reduction and reduction by history with Alg. 2 instead of all pairs.
 * Forward: MarkProperSupersets(L, L) marks the sets of L that properly
 * contain another set of L; MarkSupersets(H, L) those that contain a set of
 * the history H (the rows of the side's earlier levels).  Inverse: X lies
 * inside Y exactly when the complement of Y lies inside the complement of X,
 * so the same two calls run on complemented rows (padding bits cleared).
 * Every marked set of L is dropped; the result is the same set of drops as
 * the all-pairs rule. */
static int alg2_mark(const u64 *arows, int64_t na, const u64 *brows, int64_t nb, int n, int W,
                     int proper, unsigned char *drop, int64_t *tests) {
    if (na == 0 || nb == 0) return ORC_OK;
    int64_t aoff[2] = {0, na}, boff[2] = {0, nb};
    Side av = {0}, bv = {0};
    av.W = bv.W = W;
    av.rows = (u64 *)arows; av.off = aoff; av.nlev = 1;
    bv.rows = (u64 *)brows; bv.off = boff; bv.nlev = 1;
    int64_t *A = malloc((size_t)na * sizeof(int64_t));
    int64_t *B = malloc((size_t)nb * sizeof(int64_t));
    if (!A || !B) { free(A); free(B); return ORC_ENOMEM; }
    for (int64_t i = 0; i < na; i++) A[i] = i;
    for (int64_t j = 0; j < nb; j++) B[j] = j;
    g_lex_side = &av; g_lex_lev = 0; g_lex_n = n;
    qsort(A, (size_t)na, sizeof(int64_t), cmp_lex);
    MarkCtx c = {&av, 0, &bv, 0, A, B, n, W, 16, 0, proper};
    int64_t active = mark_supersets(&c, 0, na, 0, nb, 0);
    for (int64_t t = active; t < nb; t++) drop[B[t]] = 1;
    *tests += c.tests;
    free(A); free(B);
    return ORC_OK;
}

static int alg2_drops(const Side *s, int dir, int history, int n, unsigned char *drop,
                      int64_t *tests) {
    const int W = s->W, L = s->nlev - 1;
    const int64_t m = level_size(s, L), base = s->off[L];
    const int64_t nh = history ? base : 0;
    const u64 *lev = level_row(s, L, 0), *hist = s->rows;
    u64 *comp = NULL;
    if (dir == 1) {
        /* complements of the history rows, then of the level rows */
        comp = malloc((size_t)((nh + m) ? (nh + m) : 1) * W * sizeof(u64));
        if (!comp) return ORC_ENOMEM;
        for (int64_t t = 0; t < nh + m; t++) {
            const u64 *src = t < nh ? s->rows + t * W : lev + (t - nh) * W;
            for (int w = 0; w < W; w++) {
                int lo = w * 64;
                u64 mask = n - lo >= 64 ? ~(u64)0 : (((u64)1 << (n - lo)) - 1);
                comp[t * W + w] = ~src[w] & mask;
            }
        }
        hist = comp;
        lev = comp + nh * W;
    }
    int rc = alg2_mark(lev, m, lev, m, n, W, 1, drop, tests);
    if (!rc && nh) rc = alg2_mark(hist, nh, lev, m, n, W, 0, drop, tests);
    free(comp);
    return rc;
}

/* ------------------------------ O-F ------------------------------------ */

typedef struct {
    int n, k;
    Side F, B;
    int64_t pair_tests;     /* subset tests actually made */
    int64_t reduce_tests;   /* subset tests made by the list reductions */
    int64_t pairs;          /* sum of |L_f| * |L_b| over all meet checks */
    int64_t candidates;     /* sets generated by expansion steps */
    int steps;
} OrcRun;

static void trace_forward(const Side *s, int k, int L, int64_t i, uint8_t *out) {
    for (int d = L; d > 0; d--) {
        int64_t g = s->par[s->off[d] + i];
        out[d - 1] = (uint8_t)(g % k);
        i = g / k;
    }
}

static void trace_inverse(const Side *s, int L, int64_t j, uint8_t *out) {
    for (int d = L, pos = 0; d > 0; d--, pos++) {
        int64_t g = s->par[s->off[d] + j];
        int64_t prev = level_size(s, d - 1);
        out[pos] = (uint8_t)(g / prev);
        j = g % prev;
    }
}

/* Forward BFS from Q; the first singleton generated at the first level that
 * has one is reached by the lex-least shortest reset word. */
int orc_forward(int n, int k, const int32_t *delta, int64_t max_sets,
                int32_t *r, uint8_t *word, int64_t word_cap) {
    int rc = check_input(n, k, delta);
    if (rc) return rc;
    rc = orc_is_synchronizing(n, k, delta);
    if (rc < 0) return rc;
    if (rc == 0) return ORC_ENOTSYNC;
    int W = nwords(n);
    u64 Q[8];
    memset(Q, 0, sizeof Q);
    for (int q = 0; q < n; q++) setbit(Q, q);
    Side F;
    rc = side_init(&F, W, Q, 1);
    if (rc) { side_free(&F); return rc; }
    int out = ORC_OK;
    for (;;) {
        int L = F.nlev - 1;
        int64_t m = level_size(&F, L);
        int64_t hit = -1;
        for (int64_t i = 0; i < m; i++)
            if (popcount_set(level_row(&F, L, i), W) == 1) { hit = i; break; }
        if (hit >= 0) {
            *r = L;
            if (word) {
                if (word_cap < L) out = ORC_EWORDCAP;
                else trace_forward(&F, k, L, hit, word);
            }
            break;
        }
        if (m == 0) { out = ORC_ENOTSYNC; break; }
        if (F.nrows + m * k > max_sets) { out = ORC_ELIMIT; break; }
        rc = step_forward(&F, n, k, delta);
        if (rc) { out = rc; break; }
    }
    side_free(&F);
    return out;
}

/* ------------------------------ O-B ------------------------------------ */

/* sides_out[s] = 0 for a forward step, 1 for an inverse step; reduce: 1 to
 * self-reduce every new level (side_reduce) before the meet test, 2 also by
 * history, 4 with Alg. 2, 8 dropped sets kept as visited.  stats_out (nine entries, or NULL): steps, forward
 * depth, inverse depth, forward and inverse sets kept, candidates generated,
 * meet subset tests made, sum of |L_f|*|L_b| over the meet checks, subset
 * tests made by the reductions */
static int bidir_impl(int n, int k, const int32_t *delta, int meet_mode,
                      const uint8_t *sched, int sched_len, int max_steps,
                      int32_t *r, uint8_t *word, int64_t word_cap,
                      uint8_t *sides_out, int64_t *stats_out, void **handle_out, int reduce) {
    int rc = check_input(n, k, delta);
    if (rc) return rc;
    if (handle_out) *handle_out = NULL;
    rc = orc_is_synchronizing(n, k, delta);
    if (rc < 0) return rc;
    if (rc == 0) return ORC_ENOTSYNC;
    int W = nwords(n);
    OrcRun *run = calloc(1, sizeof(OrcRun));
    if (!run) return ORC_ENOMEM;
    run->n = n; run->k = k;
    u64 *init = calloc((size_t)n * W, sizeof(u64));
    if (!init) { free(run); return ORC_ENOMEM; }
    for (int q = 0; q < n; q++) setbit(init + (int64_t)q * W, q);
    u64 Q[8];
    memset(Q, 0, sizeof Q);
    for (int q = 0; q < n; q++) setbit(Q, q);
    rc = side_init(&run->F, W, Q, 1);
    if (!rc) rc = side_init(&run->B, W, init, n);
    free(init);
    int out = rc;
    if (!rc) {
        int step = 0;
        for (;;) {
            int64_t bi = 0, bj = 0;
            int found = 0;
            run->pairs += level_size(&run->F, run->F.nlev - 1) * level_size(&run->B, run->B.nlev - 1);
            rc = meet(&run->F, &run->B, n, meet_mode, &bi, &bj, &found, &run->pair_tests);
            if (rc) { out = rc; break; }
            if (found) {
                int f = run->F.nlev - 1, b = run->B.nlev - 1;
                *r = f + b;
                if (word) {
                    if (word_cap < f + b) out = ORC_EWORDCAP;
                    else {
                        trace_forward(&run->F, k, f, bi, word);
                        trace_inverse(&run->B, b, bj, word + f);
                    }
                }
                break;
            }
            if (step >= max_steps) { out = ORC_ELIMIT; break; }
            int64_t lf = level_size(&run->F, run->F.nlev - 1);
            int64_t lb = level_size(&run->B, run->B.nlev - 1);
            int side;
            if (sched && step < sched_len) side = sched[step] ? 1 : 0;
            else side = (lb < lf) ? 1 : 0;   /* smaller frontier; tie: forward */
            if (sides_out) sides_out[step] = (uint8_t)side;
            run->candidates += (side ? lb : lf) * k;
            rc = side ? step_inverse(&run->B, n, k, delta) : step_forward(&run->F, n, k, delta);
            if (!rc && reduce)
                rc = side_reduce(side ? &run->B : &run->F, side, reduce & 2, reduce & 4,
                                 reduce & 8, n, &run->reduce_tests);
            if (rc) { out = rc; break; }
            step++;
            int64_t nl = side ? level_size(&run->B, run->B.nlev - 1)
                              : level_size(&run->F, run->F.nlev - 1);
            if (nl == 0) { out = ORC_ENOTSYNC; break; }
        }
        run->steps = step;
    }
    if (stats_out) {
        stats_out[0] = run->steps;
        stats_out[1] = run->F.nlev ? run->F.nlev - 1 : 0;
        stats_out[2] = run->B.nlev ? run->B.nlev - 1 : 0;
        stats_out[3] = run->F.nrows;
        stats_out[4] = run->B.nrows;
        stats_out[5] = run->candidates;
        stats_out[6] = run->pair_tests;
        stats_out[7] = run->pairs;
        stats_out[8] = run->reduce_tests;
    }
    if (handle_out && (out == ORC_OK || out == ORC_ELIMIT)) {
        /* also the lists of a search stopped at its step limit */
        *handle_out = run;
    } else {
        side_free(&run->F); side_free(&run->B); free(run);
    }
    return out;
}

int orc_bidir(int n, int k, const int32_t *delta, int meet_mode,
              const uint8_t *sched, int sched_len, int max_steps,
              int32_t *r, uint8_t *word, int64_t word_cap,
              uint8_t *sides_out, int64_t *stats_out, void **handle_out) {
    return bidir_impl(n, k, delta, meet_mode, sched, sched_len, max_steps, r, word, word_cap,
                      sides_out, stats_out, handle_out, 0);
}

/* ------------- beam search: CutOff-IBFS (Section 1.3.2, 2.1.3) ---------- */

/* Keeps the `beam` sets of largest cardinality of the newest level (ties:
 * the earlier place in the level, i.e. the least key); the sets cut stay
 * visited (ghost rows) and leave the level, whose kept sets keep key
 * order.  Returns how many sets were cut, or a negative ORC_ code. */
static int64_t side_cut(Side *s, int64_t beam, int n) {
    const int W = s->W, L = s->nlev - 1;
    const int64_t m = level_size(s, L), base = s->off[L];
    if (m <= beam) return 0;
    int64_t *count = calloc((size_t)n + 1, sizeof(int64_t));
    unsigned char *drop = malloc((size_t)m);
    if (!count || !drop) { free(count); free(drop); return ORC_ENOMEM; }
    for (int64_t i = 0; i < m; i++) count[popcount_set(level_row(s, L, i), W)]++;
    /* the least cardinality that is kept, and how many of it */
    int cstar = n;
    int64_t above = 0;
    while (above + count[cstar] < beam) above += count[cstar--];
    int64_t quota = beam - above, cut = 0;
    for (int64_t i = 0; i < m; i++) {
        const int c = popcount_set(level_row(s, L, i), W);
        drop[i] = !(c > cstar || (c == cstar && quota > 0));
        if (c == cstar && !drop[i]) quota--;
        cut += drop[i];
    }
    free(count);
    if (s->nghost + cut > s->ghost_cap) {
        int64_t cap = 2 * (s->nghost + cut) + 16;
        u64 *g = realloc(s->ghost, (size_t)cap * W * sizeof(u64));
        if (!g) { free(drop); return ORC_ENOMEM; }
        s->ghost = g;
        s->ghost_cap = cap;
    }
    int64_t pos = base;
    for (int64_t i = 0; i < m; i++) {
        if (drop[i]) {
            memcpy(s->ghost + (s->nghost++) * W, level_row(s, L, i), sizeof(u64) * W);
            continue;
        }
        if (pos != base + i) {
            memmove(s->rows + pos * W, s->rows + (base + i) * W, sizeof(u64) * W);
            s->par[pos] = s->par[base + i];
        }
        pos++;
    }
    free(drop);
    g_W = W;
    qsort(s->ghost, (size_t)s->nghost, sizeof(u64) * W, cmp_ghost);
    s->nrows = pos;
    s->off[L + 1] = pos;
    for (int64_t t = 0; t < s->nrows; t++) s->sorted[t] = t;
    g_rows = s->rows;
    qsort(s->sorted, (size_t)s->nrows, sizeof(int64_t), cmp_cand);
    return cut;
}

/* Beam search for an upper bound R >= r: the inverse BFS of Alg. 1 from the
 * singletons (preimages, letter-major keys, duplicates as in the plain
 * search), every new level cut to its `beam` largest sets (side_cut), until
 * a level holds Q.  R is that depth and the word traced from the first such
 * set (least key) is a reset word of length R.  Which sets the cut keeps is
 * not fixed by the paper (it cites the method): the largest, as a set
 * closer to Q in size.  With a beam at least as large as every level, this
 * is the plain search run on the inverse side only, so R = r and the word
 * is the lex-least one.  stats_out (4 entries, may be NULL): steps, sets
 * kept, sets cut, largest level after the cut.  ORC_ELIMIT: a level became
 * empty (the cut can lead into a dead end) or max_steps passed. */
static int beam_run(int n, int k, const int32_t *delta, int64_t beam, int max_steps,
                    int32_t *R, uint8_t *word, int64_t word_cap, int64_t *stats_out,
                    int64_t *sizes, int sizes_cap, int *nsizes) {
    int rc = check_input(n, k, delta);
    if (rc) return rc;
    if (beam < 1 || !R) return ORC_EINVAL;
    rc = orc_is_synchronizing(n, k, delta);
    if (rc < 0) return rc;
    if (rc == 0) return ORC_ENOTSYNC;
    int64_t st[4] = {0, 0, 0, 0};
    if (n == 1) {
        *R = 0;
        if (stats_out) memcpy(stats_out, st, sizeof st);
        return ORC_OK;
    }
    const int W = nwords(n);
    u64 *init = calloc((size_t)n * W, sizeof(u64));
    if (!init) return ORC_ENOMEM;
    for (int q = 0; q < n; q++) setbit(init + (int64_t)q * W, q);
    Side B;
    rc = side_init(&B, W, init, n);
    free(init);
    int out = ORC_ELIMIT;
    int ns = 0;
    if (sizes && sizes_cap > 0) sizes[ns++] = n;
    if (!rc) {
        const int64_t cut0 = side_cut(&B, beam, n);   /* level 0 too, if n > beam */
        if (cut0 < 0) out = (int)cut0;
        else st[2] += cut0;
    } else {
        out = rc;
    }
    for (int step = 1; !rc && out == ORC_ELIMIT && step <= max_steps; step++) {
        rc = step_inverse(&B, n, k, delta);
        if (rc) { out = rc; break; }
        const int L = B.nlev - 1;
        if (level_size(&B, L) == 0) break;          /* dead end */
        const int64_t U = level_size(&B, L);
        const int64_t cut = side_cut(&B, beam, n);
        if (cut < 0) { out = (int)cut; break; }
        if (sizes && ns < sizes_cap) sizes[ns++] = U;
        st[0] = step;
        st[1] += level_size(&B, L);
        st[2] += cut;
        if (level_size(&B, L) > st[3]) st[3] = level_size(&B, L);
        for (int64_t j = 0; j < level_size(&B, L); j++) {
            if (popcount_set(level_row(&B, L, j), W) != n) continue;
            *R = step;
            out = ORC_OK;
            if (word) {
                if (word_cap < step) out = ORC_EWORDCAP;
                else trace_inverse(&B, L, j, word);
            }
            break;
        }
    }
    side_free(&B);
    if (stats_out) memcpy(stats_out, st, sizeof st);
    if (nsizes) *nsizes = ns;
    return out;
}

int orc_beam(int n, int k, const int32_t *delta, int64_t beam, int max_steps,
             int32_t *R, uint8_t *word, int64_t word_cap, int64_t *stats_out) {
    return beam_run(n, k, delta, beam, max_steps, R, word, word_cap, stats_out, NULL, 0, NULL);
}

/* orc_beam that also writes the size of every level before its cut:
 * sizes[0] = n (the singletons), sizes[L] = the new sets of depth L, for
 * the levels made (at most sizes_cap), *nsizes of them. */
int orc_beam_sizes(int n, int k, const int32_t *delta, int64_t beam, int max_steps,
                   int32_t *R, uint8_t *word, int64_t word_cap, int64_t *sizes, int sizes_cap,
                   int *nsizes) {
    return beam_run(n, k, delta, beam, max_steps, R, word, word_cap, NULL, sizes, sizes_cap, nsizes);
}

/* ---------------- Eppstein's greedy heuristic -------------------------- */

/* Shortest merging words of pairs of states: dist[p*n+q] is the least |w|
 * with delta(p,w) = delta(q,w) (0 when p = q, -1 when no word merges them:
 * the pair test of the Section 2 intro, with lengths).  Filled from its
 * recursive definition, dist{p,q} = 1 + min over letters a of
 * dist{delta(p,a), delta(q,a)}, in rounds d = 1, 2, ...: a pair gets d in
 * round d when some letter takes it to a pair (or a single state) of
 * distance d - 1.  next[p*n+q] is the least such letter (255 where
 * dist <= 0).  Both arrays are n*n and symmetric. */
int orc_pair_dist(int n, int k, const int32_t *delta, int32_t *dist, uint8_t *next) {
    int rc = check_input(n, k, delta);
    if (rc) return rc;
    if (!dist || !next) return ORC_EINVAL;
    for (int p = 0; p < n; p++)
        for (int q = 0; q < n; q++) {
            dist[(size_t)p * n + q] = p == q ? 0 : -1;
            next[(size_t)p * n + q] = 255;
        }
    for (int d = 1;; d++) {
        int any = 0;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) {
                if (dist[(size_t)p * n + q] != -1) continue;
                for (int a = 0; a < k; a++) {
                    int pp = delta[(int64_t)a * n + p], qq = delta[(int64_t)a * n + q];
                    if (dist[(size_t)pp * n + qq] == d - 1) {
                        dist[(size_t)p * n + q] = dist[(size_t)q * n + p] = d;
                        next[(size_t)p * n + q] = next[(size_t)q * n + p] = (uint8_t)a;
                        any = 1;
                        break;
                    }
                }
            }
        if (!any) break;
    }
    return ORC_OK;
}

/* Eppstein's greedy heuristic (cited in Section 1.3.2, the first upper
 * bound of Section 2.1.3).  From S = Q, each round picks the pair {p, q}
 * of S whose merging word is shortest (ties: least p, then least q),
 * appends that word (next{p,q}, then next of the image pair, and so on,
 * dist{p,q} letters) and replaces S with its image under it, until S is a
 * single state.  The result is a reset word, so its length bounds r from
 * above.  rounds (3 ints per round: p, q, dist{p,q}; at most n - 1 rounds;
 * may be NULL) and *nrounds describe the rounds for the tests.  *len is the
 * whole length even when it exceeds word_cap (then ORC_EWORDCAP and only
 * the first word_cap letters are written). */
int orc_eppstein(int n, int k, const int32_t *delta, uint8_t *word, int64_t word_cap,
                 int64_t *len, int32_t *rounds, int32_t *nrounds) {
    int rc = check_input(n, k, delta);
    if (rc) return rc;
    if (!len) return ORC_EINVAL;
    rc = orc_is_synchronizing(n, k, delta);
    if (rc < 0) return rc;
    if (rc == 0) return ORC_ENOTSYNC;
    int32_t *dist = malloc(sizeof(int32_t) * (size_t)n * n);
    uint8_t *next = malloc((size_t)n * n);
    unsigned char *in = calloc((size_t)n, 1), *img = calloc((size_t)n, 1);
    if (!dist || !next || !in || !img) {
        free(dist); free(next); free(in); free(img);
        return ORC_ENOMEM;
    }
    rc = orc_pair_dist(n, k, delta, dist, next);
    int64_t total = 0;
    int32_t nr = 0;
    int size = n;
    for (int q = 0; q < n; q++) in[q] = 1;
    while (!rc && size > 1) {
        if (nr == n - 1) {          /* every round merges a pair: cannot happen */
            rc = ORC_ELIMIT;
            break;
        }
        int bp = -1, bq = -1, bd = 0;
        for (int p = 0; p < n; p++) {
            if (!in[p]) continue;
            for (int q = p + 1; q < n; q++) {
                if (!in[q]) continue;
                const int d = dist[(size_t)p * n + q];
                if (bp < 0 || d < bd) { bp = p; bq = q; bd = d; }
            }
        }
        if (rounds) {
            rounds[3 * nr] = bp;
            rounds[3 * nr + 1] = bq;
            rounds[3 * nr + 2] = bd;
        }
        nr++;
        int p = bp, q = bq;
        for (int t = 0; t < bd; t++) {
            const int a = next[(size_t)p * n + q];
            if (word && total < word_cap) word[total] = (uint8_t)a;
            total++;
            memset(img, 0, (size_t)n);
            size = 0;
            for (int s = 0; s < n; s++)
                if (in[s] && !img[delta[(int64_t)a * n + s]]) {
                    img[delta[(int64_t)a * n + s]] = 1;
                    size++;
                }
            memcpy(in, img, (size_t)n);
            p = delta[(int64_t)a * n + p];
            q = delta[(int64_t)a * n + q];
        }
    }
    free(dist); free(next); free(in); free(img);
    if (rc) return rc;
    *len = total;
    if (nrounds) *nrounds = nr;
    return total > word_cap && word ? ORC_EWORDCAP : ORC_OK;
}

/* orc_bidir with every new level self-reduced (side_reduce) */
int orc_bidir_reduced(int n, int k, const int32_t *delta, int meet_mode,
                      const uint8_t *sched, int sched_len, int max_steps,
                      int32_t *r, uint8_t *word, int64_t word_cap,
                      uint8_t *sides_out, int64_t *stats_out, void **handle_out) {
    return bidir_impl(n, k, delta, meet_mode, sched, sched_len, max_steps, r, word, word_cap,
                      sides_out, stats_out, handle_out, 1);
}

/* orc_bidir_reduced, and every new level also reduced by history: a new
 * forward set containing a set stored on an earlier forward level, a new
 * inverse set contained in one stored on an earlier inverse level, is
 * dropped (Alg. 1, deleting the supersets of the BFS history list) */
int orc_bidir_history(int n, int k, const int32_t *delta, int meet_mode,
                      const uint8_t *sched, int sched_len, int max_steps,
                      int32_t *r, uint8_t *word, int64_t word_cap,
                      uint8_t *sides_out, int64_t *stats_out, void **handle_out) {
    return bidir_impl(n, k, delta, meet_mode, sched, sched_len, max_steps, r, word, word_cap,
                      sides_out, stats_out, handle_out, 1 | 2);
}

/* orc_bidir with the reductions chosen by flags: 1 self-reduction, 2 also
 * reduction by history, 4 drops found with Alg. 2 instead of all pairs (the
 * same drops), 8 dropped sets stay in the visited index instead of being
 * forgotten */
int orc_bidir_reduce(int n, int k, const int32_t *delta, int meet_mode,
                     const uint8_t *sched, int sched_len, int max_steps,
                     int32_t *r, uint8_t *word, int64_t word_cap,
                     uint8_t *sides_out, int64_t *stats_out, void **handle_out, int flags) {
    if (flags & ~15 || ((flags & 14) && !(flags & 1))) return ORC_EINVAL;
    return bidir_impl(n, k, delta, meet_mode, sched, sched_len, max_steps, r, word, word_cap,
                      sides_out, stats_out, handle_out, flags);
}

/* Level data of a finished orc_bidir run (side 0 forward, 1 inverse).
 * With rows == NULL only the counts are returned: *nlev levels and
 * *nrows rows in total.  Otherwise off[0..nlev], rows[nrows*W] and
 * par[nrows] are filled. */
int orc_levels(void *handle, int side, int32_t *nlev, int64_t *nrows,
               int64_t *off, u64 *rows, int64_t *par) {
    OrcRun *run = handle;
    if (!run) return ORC_EINVAL;
    const Side *s = side ? &run->B : &run->F;
    *nlev = s->nlev;
    *nrows = s->nrows;
    if (!rows) return ORC_OK;
    memcpy(off, s->off, sizeof(int64_t) * (s->nlev + 1));
    memcpy(rows, s->rows, sizeof(u64) * s->nrows * s->W);
    memcpy(par, s->par, sizeof(int64_t) * s->nrows);
    return ORC_OK;
}

void orc_free(void *handle) {
    OrcRun *run = handle;
    if (!run) return;
    side_free(&run->F); side_free(&run->B); free(run);
}
