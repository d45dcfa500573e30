// srw_device.h -- data shared between the host engine and the HIP kernels.
//
// One "segment" is one automaton taking one step of the bidirectional
// breadth-first search (Alg. 1 of the paper with only duplicate removal).
// Every kernel of a step is launched once for all segments of the step; a
// block finds its segment by binary search in a per-kernel block prefix.
#pragma once
#include <stdint.h>

namespace srw {

typedef unsigned long long u64;
typedef uint32_t u32;

constexpr int kMaxW = 8;                 // subsets of up to 512 states
constexpr u64 kEmpty = ~0ull;            // free hash slot
constexpr u32 kCandBit = 0x80000000u;    // slot ref names a candidate of this step
constexpr u32 kDrop = 0xFFFFFFFFu;       // candidate dropped (empty or seen before)
constexpr u32 kGhostBit = 0x40000000u;   // slot ref names a set dropped by a reduction
                                         // (with StepDesc::ghost set; rows then stay below 2^30)
constexpr int kBS = 256;                 // threads per block (4 wave64)
constexpr int kCB = 1024;                // candidates per compaction block
constexpr int kMeetTileWords = 32;       // LDS budget of the meet: tiles*W <= this
constexpr int64_t kMeetMaxGrid = 0x7fffffff;  // meet blocks per launch (grid-stride beyond)
constexpr int kCommonMax = 8;            // chunked meet: common states used per chunk
constexpr int kCommonRound = 4;          // common columns loaded per round
// meet operation counters: per set width, kOpsSlots counters kOpsStride words
// apart (one 128-byte line each), so that the blocks of a launch spread their
// atomic adds over many addresses
constexpr int kOpsSlots = 64;
constexpr int kOpsStride = 16;
constexpr int kOpsWords = kMaxW * kOpsSlots * kOpsStride;
constexpr int kMstatCounters = 8;
constexpr int kMstatSlots = 64;
constexpr int kMstatWords = kMstatSlots * kOpsStride;
constexpr int64_t kSmallMeetBlocks = 64;  // small steps: at most this many LDS-tile meet blocks
constexpr int kRowBatchMax = 512;        // chunked meet: most candidates per group tested by signature
// LDS words per wave of the chunked meet: kRowBatchMax candidate indices (u32)
// and their signatures; also holds one tile of columns (64 * W words)
constexpr int kSliceWords = kRowBatchMax / 2 + kRowBatchMax;
constexpr int kMeetLdsWords = kMeetTileWords * 64 > (kBS / 64) * kSliceWords ? kMeetTileWords * 64
                                                                               : (kBS / 64) * kSliceWords;

// A hash-slot is 64 bits: high 32 = fingerprint of the set, low 32 = ref.
// ref < 2^31: id of a stored (visited) row of this side;
// ref >= 2^31: candidate (ref - 2^31) of the current step.

// ---- an inverse level kept in buckets (the bucketed meet) -------------
//
// A set that holds state s can only lie in sets that hold s too (the split
// of Alg. 2).  A large inverse level is kept in 2^kYBits buckets by its
// membership of kYBits split states (the most frequent states of the
// forward level), each bucket padded with empty sets to whole tiles of 64
// sets.  For each key a, the tiles of every bucket whose key contains a are
// listed, so that a chunk of forward sets whose common states include the
// split states of a scans those tiles only.
constexpr int kYBits = 10;
constexpr int kYBins = 1 << kYBits;
constexpr int64_t kYMin = 16384;          // default: inverse levels at least this large are bucketed
constexpr int64_t kYListPerTile = 32;     // room for list entries per tile of the level
// A bucketed meet's plan orders its work items by an order key per chunk:
// first by kIndexBins bins of the chunk's least index in the forward level
// (the least meeting pair is sought, so a pair found early lets the chunks
// of larger index stop), then by the chunk's bucket key, then tile range by
// tile range of that key's list, and within a range chunk by chunk (the
// waves in flight read the same tiles, which then come from the cache).
constexpr int kIndexBins = 16;
constexpr int kOrderKeys = kIndexBins * kYBins;
constexpr int kKCount = 0, kKStart = kOrderKeys, kKRanges = 2 * kOrderKeys, kKPre = 3 * kOrderKeys,
              kKCur = 4 * kOrderKeys + 1, kKInfoWords = 5 * kOrderKeys + 1;

struct YbMeta {
    int32_t nt;                 // tiles of the padded level
    int32_t ok;                 // 1: the tile lists fit their room (0: every chunk scans every tile)
    int64_t entries;            // list entries of the keys other than 0
    int32_t split[kYBits];      // split state i is key bit kYBits-1-i (-1: none)
};

struct YbDesc {                 // bucketing of one inverse level
    int32_t n, W;
    const u64 *rows;            // the level, in level order
    const u64 *cnt;             // its size is *cnt when set (a new level), else `count`
    int64_t count;
    int64_t count_ub;           // upper bound of the size
    int64_t nt_ub;              // tiles of room: ceil(count_ub / 64) + kYBins
    const int32_t *top;         // split states: top[0 .. kYBits-1]
    YbMeta *meta;
    uint16_t *key;              // count_ub keys
    u32 *bins;                  // kYBins set counts, then kYBins insertion cursors
    u32 *tb;                    // kYBins + 1 first tiles of the buckets
    u32 *lsize;                 // kYBins list lengths (tiles)
    u32 *loff;                  // kYBins + 1 list offsets
    u32 *lcur;                  // kYBins list cursors
    u32 *list;                  // list_cap entries
    int64_t list_cap;
    u32 *idx;                   // nt_ub * 64: padded position -> index in the level (~0: padding)
    u64 *YT, *YTt, *Ysig;       // the padded level transposed (state-major with nt tiles)
};

struct StepDesc {
    // automaton
    int32_t n, k, W, dir;      // dir 0: forward (images), 1: inverse (preimages)
    const uint16_t *delta;     // delta[a*n + q], k*n entries
    // expansion input: the current level of the expanded side
    const u64 *par_rows;       // m rows of W words
    int64_t m;                 // parent count
    int64_t C;                 // candidates = k*m
    u64 *cand;                 // C rows
    u32 *cslot;                // C slot positions (or kDrop)
    // dedup (visited hash set of the expanded side)
    u64 *tab;
    u64 tab_mask;              // capacity - 1 (capacity is a power of two)
    const u64 *vis_rows;       // all stored rows of the side (ids < 2^31)
    // self-reduction of the new level (Alg. 1), when `ghost` is set: its
    // dropped sets go to ghost rows ghost_base.. and stay visited; mark[i]
    // flags new set i, red_par holds the kept sets' keys while they move;
    // res[3] = sets dropped
    u64 *ghost;
    int64_t ghost_base;
    u32 *mark;
    u32 *red_par;
    int64_t red_hist;          // 1: also reduce by the side's earlier levels (history)
    // compaction
    u64 *out_rows;             // where the new level starts (vis_rows + base*W)
    u32 *out_par;              // parent key per new row
    int64_t out_base;          // store id of the first new row
    int64_t cblk_base;         // first compaction block of this segment
    int64_t ncblk;             // compaction blocks of this segment
    // meet (X: forward level, Y: inverse level, transposed in tiles of 64
    // sets; column q of tile t -- bit j says whether state q is in set
    // 64t+j -- is YT[q * nt + t] (state-major, nt = ceil(|Y| / 64)) and
    // YTt[t * 64W + q] (tile-major))
    const u64 *X;              // mode 1: the level sorted by key
    int64_t nX;                // -1: the new level (count in res[0])
    u64 *YT;
    u64 *YTt;
    const u64 *Yrows;          // the inverse level's rows
    u64 *Ysig;                 // signature of each inverse set: the OR of its W words
    int64_t nY;                // -1: the new level (count in res[0])
    int64_t nXb, nYc;          // mode 0 grid of this segment (upper bounds)
    int32_t tpb;               // mode 0: tiles per meet block
    int32_t meet_mode;         // 0: LDS tiles, 1: sorted 64-set chunks, 2: chunks against buckets
    int32_t small;             // 1: the whole step runs in one block (k_step_small)
    int32_t ysort;             // 1: sort the new inverse level by cardinality (dir 1)
    // the inverse level in cardinality order, largest first (null: level order)
    const u32 *Yidx;           // sorted position -> index in the level
    const u32 *Ycnt;           // Ycnt[c] = sets of the level with at least c states, c = 0..n+1
    // the sort of a new inverse level
    u32 *ys_hist;              // n + 1 counters
    u32 *ys_cnt;               // n + 2 entries
    u32 *ys_idx;               // position -> index
    const u32 *Xidx;           // mode 1: rank of each sorted X in its level
    const u64 *Xcom;           // mode 1: AND of the 64 sets of each chunk
    int64_t gitems_ub;         // mode 1: work items per chunk (upper bound)
    int64_t ngi;               // mode 1: tile groups (of 64 tiles) per item
    int64_t row_batch_max;     // mode 1: more candidates per group than this: column chains
    int64_t nch_ub;            // mode 1: chunks (upper bound)
    int64_t item_order;        // mode 1: 0 tile-range-major items, 1 chunk-major
    int64_t xcd_granule;       // mode 2: runs of this many consecutive work items go to
                               // one XCD's queue, round robin (0: one queue for all)
    // mode 2 (bucketed meet): the inverse level in buckets, and the plan of
    // the work items (one chunk, a range of its tiles) taken from a queue
    const YbMeta *yb;
    const u32 *yb_lsize, *yb_loff, *yb_list;
    u32 *ckey;                 // per chunk: its order key (see kOrderKeys)
    u32 *korder;               // the chunks in order of their order keys
    u32 *kinfo;                // per order key: chunks, first place in korder, tile
                               // ranges, first work item (kOrderKeys + 1), cursor
    u32 *queue;                // [0] next work item, [1] work items, [2 + x] next
                               // item of XCD x's queue (with xcd_granule)
    // transpose of a new inverse level into YT
    int64_t ntr_waves;         // upper bound of (tile, word) waves
    // results: res[0] = new level size, res[1] = least (i << 32 | j) meeting
    // pair, res[2] = sum of the cardinalities of the new level's sets (its
    // density times n times its size); kResWords words per segment
    u64 *res;
    // chunked meets, when profiling: kMstatSlots slots of kMstatCounters
    // counters (kOpsStride words apart), see srw_stats.meet_work
    u64 *mstat;
};

// A block that runs every step of one automaton by itself for as long as
// the steps stay small (k_run_small): the search's buffers, as the host set
// them up, and the limits within which the block may go on.
struct RunState;
struct RunDesc {
    int32_t n, k, W, max_lev;  // max_lev: entries of each side's level offset array
    const uint16_t *delta;     // delta[a*n + q]
    u64 *rows[2];              // per side (0 forward, 1 inverse): stored rows
    u32 *par[2];               // parent keys
    u64 *tab[2];               // visited hash sets
    u64 tab_mask[2];           // capacity - 1
    int64_t rows_cap[2];       // rows of capacity
    int64_t *off[2];           // level L of side s: rows off[s][L] .. off[s][L+1]-1
    u64 *cand;                 // candidates of a step
    u32 *cslot;
    int64_t cand_cap;
    u64 *colT;                 // the current inverse level transposed: colT_cap words
    int64_t colT_cap;          // state-major, then colT_cap words tile-major
    u64 *ysig;                 // signature of each set of the current inverse level
    int64_t ysig_cap;
    int64_t small_cand;        // most candidates of a step run here
    int64_t max_ticks;         // stop after this many wall_clock64 ticks (0: no limit)
    RunState *st;
};
constexpr int kResWords = 4;             // step result words per segment
constexpr int kRunSideWords = 128;       // step sides a runner records (bits)
struct RunState {
    int64_t nrows[2];          // in/out: rows stored per side
    int32_t nlev[2];           // in/out: levels per side (level 0 included)
    int32_t status;            // out: 0 the next step is not small, 1 met, 2 a list became empty
    int32_t steps;             // out: steps run here
    u64 best;                  // out: the least meeting pair (i << 32 | j), when met
    u64 res[kResWords];        // step results (as StepDesc::res)
    int64_t candidates, unique, pairs;   // out: over the steps run here
    u64 popsum[2];             // in/out: sum of the cardinalities of each side's current level
    u64 sides[kRunSideWords];  // out: bit t = side of step t (steps beyond 64 * kRunSideWords unrecorded)
};

constexpr int kKeyBits = 16;             // sort key: the 16 most frequent states
constexpr int kSortBins = 1 << kKeyBits;

// Bucket sort of a new forward level by the membership of its most frequent
// states, so that 64 consecutive sets share as many states as possible.
struct SortDesc {
    int32_t n, W;
    const u64 *X;              // the new level (unsorted)
    const u64 *cnt;            // &res[0]: its size
    int64_t nub;               // upper bound of its size
    u32 *hist;                 // n state counts
    int32_t *top;              // kKeyBits states, most frequent first
    u32 *keys;                 // nub
    u32 *bins;                 // kSortBins counters, then offsets
    u64 *xs_rows;              // nub rows, sorted
    u32 *xs_idx;               // nub ranks
    u64 *xs_common;            // ceil(nub/64) rows
};

struct InitDesc {
    int32_t n, W;
    u64 *rows_f;               // forward level 0: Q
    u64 *rows_b;               // inverse level 0: the n singletons
    u32 *par_f, *par_b;
    const uint16_t *delta_src; // the table as uploaded (all automata of the call in one copy)
    uint16_t *delta;           // the automaton's own k*n table
    int32_t k, pad;
};

// device-to-device copy of `count` 32-bit words (grown buffers keep their
// contents); one launch copies every buffer grown in a step
struct CopyDesc {
    const u32 *src;
    u32 *dst;
    int64_t count;
};
constexpr int kCopyPerBlock = 4096;      // words per block of k_copy

struct RehashDesc {
    int32_t W;
    int32_t ref_or;            // or-ed into every ref (kGhostBit: ghost rows)
    const u64 *rows;           // rows 0..count-1 to insert
    int64_t count;
    u64 *tab;
    u64 tab_mask;
};

struct TransposeDesc {
    int32_t W, pad;
    const u64 *rows;
    int64_t count;
    u64 *YT, *YTt, *Ysig;
};

// Beam search (CutOff-IBFS) of one automaton, run by one block from start
// to end (k_beam): inverse steps from the singletons, every new level cut to
// its `beam` largest sets.  Every distinct set generated is stored (it stays
// visited); level L holds rows lev[3L] .. lev[3L]+lev[3L+1]-1 (the kept sets,
// in key order), then its cut sets up to lev[3L+2].
struct BeamState;
struct BeamDesc {
    int32_t n, k, W, max_lev;  // max_lev: levels the lev array holds (the step limit + 1)
    const uint16_t *delta;     // delta[a*n + q]
    int64_t beam;              // sets kept per level
    u64 *rows;                 // stored sets, rows_cap of them
    u32 *par;                  // key of each stored set (0xFFFFFFFF on level 0)
    int64_t rows_cap;
    u64 *tab;                  // visited hash set, at least 2 * rows_cap slots, cleared
    u64 tab_mask;
    u64 *cand;                 // candidates of a step, cand_cap >= k * beam (and >= n)
    u32 *cslot;
    int64_t cand_cap;
    int64_t *lev;              // 3 * max_lev entries
    uint8_t *word;             // max_lev - 1 letters
    int64_t max_ticks;         // stop after this many wall_clock64 ticks (0: no limit)
    BeamState *st;
};
struct BeamState {
    int32_t status;            // 1 Q reached, 2 a level became empty, 3 rows or levels ran out, 4 deadline
    int32_t R;                 // with status 1: the depth of Q (the word is in BeamDesc::word)
    int32_t nlev;              // levels stored (level 0 included)
    int32_t pad;
    int64_t nrows;             // sets stored
    int64_t candidates, kept, cut;   // over the steps run
};

// Eppstein's greedy heuristic, one block per automaton (k_eppstein).  Pairs
// {p, q}, p < q, are numbered q(q-1)/2 + p.
struct EppState {
    int32_t status;            // 1 done, 4 deadline, 5 a pair of the set cannot be merged
    int32_t rounds;            // pairs merged
    int64_t len;               // letters of the whole word (also those beyond word_cap)
};
struct EppDesc {
    int32_t n, k;
    const uint16_t *delta;     // delta[a*n + q]
    u32 *dist;                 // n(n-1)/2 shortest merging lengths (0: not reached)
    uint8_t *next;             // n(n-1)/2 first letters of the lex-least shortest merging words
    u32 *queue;                // 2 * n(n-1)/2: two BFS frontiers of pair numbers
    uint16_t *inv;             // k*n: states of each inverse list, letter by letter
    u32 *inv_off;              // k*(n+1): list a, t is inv[inv_off[a*(n+1)+t] .. inv_off[a*(n+1)+t+1])
    u32 *inv_cur;              // k*n fill cursors
    uint8_t *word;             // word_cap letters
    int64_t word_cap;
    int64_t max_ticks;         // stop after this many wall_clock64 ticks (0: no limit)
    EppState *st;
};

struct TraceDesc {
    const u32 *par_f;
    const int64_t *off_f;      // level offsets of the forward side
    const u32 *par_b;
    const int64_t *off_b;
    int64_t i, j;              // meeting pair (ranks in the two levels)
    int32_t f, b, k, pad;
    uint8_t *out;              // f + b letters
};

}  // namespace srw
