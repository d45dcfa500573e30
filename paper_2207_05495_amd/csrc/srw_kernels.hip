// srw_kernels.hip -- gfx950 kernels of one bidirectional-BFS step.
//
// Paper: Szykula & Zyzik, "An Improved Algorithm for Finding the Shortest
// Synchronizing Words".  One step of Alg. 1 (plain variant: duplicate removal
// only) for every segment (automaton) of a batch:
//
//   k_expand    CalculateImages / CalculatePreimages (Alg. 1; the image and
//               preimage definitions of Section 2).  Candidate keys: forward
//               g = i*k + a, inverse g = a*m + i (letter-major), so that key
//               order is the lexicographic order of the words.
//   k_insert    duplicate removal (Alg. 1 removes duplicates of the new list;
//               here a device hash set per side also drops sets seen on an
//               earlier level).  The least key of equal candidates wins.
//   k_count, k_scan, k_compact
//               stream compaction of the winners in key order into the new
//               level, with the parent key stored per row (predecessor
//               pointers, end of the Section 2 intro).
//   k_transpose a new inverse level into 64-set tiles of column words, plus
//               one signature word (OR of the set's words) per set.
//   k_sort_*    bucket sort of a large new forward level into 64-set chunks
//               with their common states, for the chunked meet.
//   k_meet      the meet test of Alg. 1: least (i, j) with X_i subset of Y_j
//               (Section 2: X in the BFS list, Y in the IBFS list).  Bit-
//               sliced: for a tile of 64 sets Y, the AND of the columns of
//               the states of X has bit j set iff X is a subset of Y_j.
//   k_step_small  a whole step of one small segment in one block.
//   k_copy, k_init, k_rehash, k_clear_tables, k_fill
//               growth of buffers and hash tables, level 0.
//   k_trace     walks the parent keys back to the reset word.
//
// All arithmetic is exact integer / bitwise.  Subsets are W = ceil(n/64)
// 64-bit words; state q is bit q%64 of word q/64; bits >= n are zero.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "srw_device.h"

namespace srw {

// ---------------------------------------------------------------- helpers

// Descriptors and block prefixes are written by the host before a launch and
// only read by kernels: they are read through the constant address space, so
// that their fields become scalar loads (through plain pointers they would be
// vector loads once a kernel has stored or done an atomic, since the compiler
// cannot rule out that the store changed them), and the pointers held in them
// are taken as global ones.
#define CONST_AS __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const CONST_AS T &cref(const T *p) {
    return *(const CONST_AS T *)p;
}

__device__ __forceinline__ int find_seg(const int64_t *pre, int nseg, int64_t b) {
    int lo = 0, hi = nseg;  // pre[lo] <= b < pre[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (cref(pre + mid) <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// 64-bit finaliser of MurmurHash3 (Appleby), constants as published
__device__ __forceinline__ u64 fmix64(u64 z) {
    z ^= z >> 33;
    z *= 0xff51afd7ed558ccdull;
    z ^= z >> 33;
    z *= 0xc4ceb9fe1a85ec53ull;
    z ^= z >> 33;
    return z;
}

template <int W>
__device__ __forceinline__ u64 set_hash(const u64 (&x)[W]) {
    u64 h = 0x6a09e667f3bcc909ull;
#pragma unroll
    for (int w = 0; w < W; ++w) h = fmix64(h ^ (x[w] + 0x9E3779B97F4A7C15ull * (u64)(w + 1)));
    return h;
}

__device__ __forceinline__ u64 load_slot(u64 *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ u32 lanes_below(u64 mask) {
    return __builtin_amdgcn_mbcnt_hi((u32)(mask >> 32), __builtin_amdgcn_mbcnt_lo((u32)mask, 0u));
}

__device__ __forceinline__ int lowest_bit(u64 v) { return __ffsll((unsigned long long)v) - 1; }

#define SRW_SWITCH_W(Wv, CALL)                                   \
    switch (Wv) {                                                \
    case 1: { constexpr int W = 1; CALL; } break;                \
    case 2: { constexpr int W = 2; CALL; } break;                \
    case 3: { constexpr int W = 3; CALL; } break;                \
    case 4: { constexpr int W = 4; CALL; } break;                \
    case 5: { constexpr int W = 5; CALL; } break;                \
    case 6: { constexpr int W = 6; CALL; } break;                \
    case 7: { constexpr int W = 7; CALL; } break;                \
    default: { constexpr int W = 8; CALL; } break;               \
    }

// LDS written by some lanes of a wave, then read by others of the same wave
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 64 x 64 bit transpose across a wave: lane r holds row r on entry and
// column r (bit j = bit r of row j) on exit.  Six butterfly stages; stage s
// swaps bit s of the row index with bit s of the column index by exchanging
// the off-diagonal s x s blocks with lane r ^ s.
__device__ __forceinline__ u64 transpose64(u64 v) {
    const int lane = threadIdx.x & 63;
    constexpr u64 kMask[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                              0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int st = 0; st < 6; ++st) {
        const int sh = 32 >> st;
        const u64 m = kMask[st];
        const u64 t = __shfl_xor(v, sh, 64);
        v = (lane & sh) ? (((t >> sh) & m) | (v & ~m)) : ((v & m) | ((t & m) << sh));
    }
    return v;
}

// ---------------------------------------------------------------- expand

// Forward: X = delta(S, a) = { delta(q, a) | q in S }, scattering the set
// bits of S; each thread owns a row of LDS for X (registers cannot be
// indexed by a run-time word).  Inverse: Y = delta^-1(S, a) =
// { q | delta(q, a) in S }, bit-sliced per wave: the wave's 64 parents are
// transposed into columns (column q: which parents hold state q), column q
// of the 64 preimages is column delta(q, a) of the parents (one LDS gather
// per state and letter), and the columns are transposed back into rows.  A
// wave whose candidates span more than two letters (levels under 64 sets)
// gathers one bit per state from the parent row instead.
// D: the step descriptor as the caller holds it -- in the constant address
// space (written by the host) or in LDS (built by a block that runs many
// steps itself).  Every thread of the block calls it (the inverse side
// shuffles within waves).
template <int W, class D>
__device__ void expand_w(const D &d, int64_t lb, u64 *lds) {
    const int tid = threadIdx.x;
    const int64_t g = lb * kBS + tid;
    const int n = d.n;
    if (d.dir == 1) {
        const bool act = g < d.C;
        const u64 live = __ballot(act);
        if (live == 0) return;                         // whole wave
        const int lane = tid & 63;
        const int a = act ? (int)(g / d.m) : 0;
        const int64_t i = act ? g - (int64_t)a * d.m : 0;
        // active lanes are a prefix of the wave and their letters ascend
        const int a_lo = __shfl(a, 0, 64);
        const int a_hi = __shfl(a, 63 - __clzll(live), 64);
        if (a_hi - a_lo > 1) {
            if (!act) return;
            const u64 *S = d.par_rows + i * W;
            const uint16_t *da = d.delta + (int64_t)a * n;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                u64 y = 0;
                const int qn = min(64, n - 64 * w);
                for (int b = 0; b < qn; ++b) {
                    const int t = da[64 * w + b];
                    y |= ((S[t >> 6] >> (t & 63)) & 1ull) << b;
                }
                d.cand[g * W + w] = y;
            }
            return;
        }
        u64 *col = lds + (tid >> 6) * 64 * W;          // this wave's columns, state-indexed
        u64 v[W];
#pragma unroll
        for (int w = 0; w < W; ++w) v[w] = act ? d.par_rows[i * W + w] : 0ull;
        wave_sync_lds();                               // earlier readers of col are done
#pragma unroll
        for (int w = 0; w < W; ++w) col[64 * w + lane] = transpose64(v[w]);
        wave_sync_lds();
#pragma unroll
        for (int w = 0; w < W; ++w) v[w] = 0;
        for (int b = a_lo; b <= a_hi; ++b) {
            const u64 lm = __ballot(act && a == b);    // the preimages under letter b
            const uint16_t *db = d.delta + (int64_t)b * n;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const int q = 64 * w + lane;
                if (q < n) v[w] |= col[db[q]] & lm;
            }
        }
#pragma unroll
        for (int w = 0; w < W; ++w) v[w] = transpose64(v[w]);
        if (act)
#pragma unroll
            for (int w = 0; w < W; ++w) d.cand[g * W + w] = v[w];
        return;
    }
    if (g >= d.C) return;
    {
        const int64_t i = g / d.k;
        const int a = (int)(g - i * d.k);
        const u64 *S = d.par_rows + i * W;
        const uint16_t *da = d.delta + (int64_t)a * n;
#pragma unroll
        for (int w = 0; w < W; ++w) lds[w * kBS + tid] = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            u64 bits = S[w];
            while (bits) {
                const int b = lowest_bit(bits);
                bits &= bits - 1;
                const int t = da[w * 64 + b];
                lds[(t >> 6) * kBS + tid] |= 1ull << (t & 63);
            }
        }
#pragma unroll
        for (int w = 0; w < W; ++w) d.cand[g * W + w] = lds[w * kBS + tid];
    }
}

__global__ void __launch_bounds__(kBS) k_expand(const StepDesc *descs, const int64_t *pre, int nseg) {
    __shared__ u64 lds[kMaxW * kBS];
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS StepDesc &d = cref(descs + s);
    const int64_t lb = (int64_t)blockIdx.x - cref(pre + s);
    SRW_SWITCH_W(d.W, expand_w<W>(d, lb, lds));
}

// ---------------------------------------------------------------- insert

template <int W, class D>
__device__ void insert_w(const D &d, int64_t lb) {
    const int64_t g = lb * kBS + threadIdx.x;
    if (g >= d.C) return;
    u64 x[W];
    u64 any = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) { x[w] = d.cand[g * W + w]; any |= x[w]; }
    if (any == 0) { d.cslot[g] = kDrop; return; }   // empty preimage
    const u64 h = set_hash<W>(x);
    const u32 fp = (u32)(h >> 32);
    const u64 mine = ((u64)fp << 32) | (u64)(kCandBit | (u32)g);
    u64 pos = h & d.tab_mask;
    for (;;) {
        u64 cur = load_slot(&d.tab[pos]);
        if (cur == kEmpty) {
            const u64 prev = atomicCAS(&d.tab[pos], kEmpty, mine);
            if (prev == kEmpty) { d.cslot[g] = (u32)pos; return; }
            cur = prev;
        }
        if ((u32)(cur >> 32) == fp) {
            const u32 ref = (u32)cur;
            const u64 *o = (ref & kCandBit) ? d.cand + (u64)(ref & ~kCandBit) * W
                         : (d.ghost && (ref & kGhostBit)) ? d.ghost + (u64)(ref & ~kGhostBit) * W
                                                          : d.vis_rows + (u64)ref * W;
            bool eq = true;
#pragma unroll
            for (int w = 0; w < W; ++w) eq = eq && (o[w] == x[w]);
            if (eq) {
                if (ref & kCandBit) {
                    // every value this slot ever holds names the same set,
                    // so the minimum is the least key among equal candidates
                    atomicMin(&d.tab[pos], mine);
                    d.cslot[g] = (u32)pos;
                } else {
                    d.cslot[g] = kDrop;   // visited on an earlier level
                }
                return;
            }
        }
        pos = (pos + 1) & d.tab_mask;
    }
}

__global__ void __launch_bounds__(kBS) k_insert(const StepDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS StepDesc &d = cref(descs + s);
    const int64_t lb = (int64_t)blockIdx.x - cref(pre + s);
    SRW_SWITCH_W(d.W, insert_w<W>(d, lb));
}

// ------------------------------------------------------------ compaction

template <class D>
__device__ __forceinline__ bool is_winner(const D &d, int64_t g) {
    const u32 sl = d.cslot[g];
    if (sl == kDrop) return false;
    return (u32)d.tab[sl] == (kCandBit | (u32)g);
}

__global__ void __launch_bounds__(kBS) k_count(const StepDesc *descs, const int64_t *pre, int nseg,
                                               u32 *blk_cnt) {
    __shared__ u32 wsum[kBS / 64];
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS StepDesc &d = cref(descs + s);
    const int64_t lb = (int64_t)blockIdx.x - cref(pre + s);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    u32 c = 0;
#pragma unroll
    for (int t = 0; t < kCB / kBS; ++t) {
        const int64_t g = lb * kCB + t * kBS + tid;
        const bool f = g < d.C && is_winner(d, g);
        c += (u32)__popcll(__ballot(f));
    }
    if (lane == 0) wsum[wave] = c;
    __syncthreads();
    if (tid == 0) {
        u32 tot = 0;
        for (int w = 0; w < kBS / 64; ++w) tot += wsum[w];
        blk_cnt[d.cblk_base + lb] = tot;
    }
}

// one block per segment: exclusive scan of its compaction-block counts
__global__ void __launch_bounds__(kBS) k_scan(const StepDesc *descs, int nseg, const u32 *blk_cnt,
                                              u32 *blk_off) {
    __shared__ u32 wsum[kBS / 64];
    const int s = blockIdx.x;
    if (s >= nseg) return;
    const CONST_AS StepDesc &d = cref(descs + s);
    if (d.small) return;                   // its step runs in k_step_small
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    u64 running = 0;
    for (int64_t c0 = 0; c0 < d.ncblk; c0 += kBS) {
        const int64_t idx = c0 + tid;
        const u32 v = idx < d.ncblk ? blk_cnt[d.cblk_base + idx] : 0u;
        u32 incl = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const u32 o = __shfl_up(incl, off, 64);
            if (lane >= off) incl += o;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        u32 wpre = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kBS / 64; ++w) {
            if (w < wave) wpre += wsum[w];
            tot += wsum[w];
        }
        if (idx < d.ncblk) blk_off[d.cblk_base + idx] = (u32)(running + wpre + incl - v);
        running += tot;
        __syncthreads();
    }
    if (tid == 0) {
        d.res[0] = running;
        d.res[1] = kEmpty;
        d.res[2] = 0;                      // k_compact adds the cardinalities
        d.res[3] = 0;                      // sets a reduction drops
    }
}

__global__ void __launch_bounds__(kBS) k_compact(const StepDesc *descs, const int64_t *pre, int nseg,
                                                 const u32 *blk_off) {
    __shared__ u32 wsum[kBS / 64];
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS StepDesc &d = cref(descs + s);
    const int64_t lb = (int64_t)blockIdx.x - cref(pre + s);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int W = d.W;
    u32 rank0 = blk_off[d.cblk_base + lb];
    u32 card = 0;                          // cardinalities of this lane's winners
#pragma unroll
    for (int t = 0; t < kCB / kBS; ++t) {
        const int64_t g = lb * kCB + t * kBS + tid;
        const bool f = g < d.C && is_winner(d, g);
        const u64 mask = __ballot(f);
        if (lane == 0) wsum[wave] = (u32)__popcll(mask);
        __syncthreads();
        u32 wpre = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kBS / 64; ++w) {
            if (w < wave) wpre += wsum[w];
            tot += wsum[w];
        }
        if (f) {
            const u64 rank = rank0 + wpre + lanes_below(mask);
            for (int w = 0; w < W; ++w) {
                const u64 v = d.cand[g * W + w];
                d.out_rows[rank * W + w] = v;
                card += (u32)__popcll(v);
            }
            d.out_par[rank] = (u32)g;
            const u32 sl = d.cslot[g];
            const u64 e = d.tab[sl];
            d.tab[sl] = (e & 0xFFFFFFFF00000000ull) | (u64)(u32)(d.out_base + (int64_t)rank);
        }
        rank0 += tot;
        __syncthreads();
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) card += (u32)__shfl_xor((int)card, off, 64);
    if (lane == 0 && card) atomicAdd((unsigned long long *)(d.res + 2), (unsigned long long)card);
}

// ------------------------------------------------------ self-reduction

// Self-reduction of a new level (Alg. 1), for segments with d.ghost set.
// Step 1: mark each new set i that has another set of its level inside it
// (forward: i is not minimal) or around it (inverse: i is not maximal), and
// with d.red_hist also each one with a set of an earlier level of its side
// inside (forward) or around it (inverse): the reduction by history.  The
// sets of a level are distinct, so "another" is the index.  Brute force:
// 256 sets per block against the level (then the earlier levels, the
// side's stored rows 0 .. out_base-1), staged 256 sets at a time in LDS and
// read as broadcasts.
template <int W>
__device__ void red_mark_w(const CONST_AS StepDesc &d, int64_t lb, u64 *lds) {
    const int64_t U = (int64_t)d.res[0];
    if (lb * kBS >= U) return;                 // the whole block
    const int tid = threadIdx.x;
    const int64_t i = lb * kBS + tid;
    const bool vi = i < U;
    u64 x[W];
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = vi ? d.out_rows[i * W + w] : 0ull;
    bool marked = !vi;
    // pass 0: the level itself; pass 1: the earlier levels (history)
    for (int pass = 0; pass < (d.red_hist ? 2 : 1); ++pass) {
        const u64 *src = pass == 0 ? d.out_rows : d.vis_rows;
        const int64_t cnt = pass == 0 ? U : d.out_base;
        for (int64_t j0 = 0; j0 < cnt; j0 += kBS) {
            __syncthreads();                   // the last tile is read
            const int64_t j = j0 + tid;
#pragma unroll
            for (int w = 0; w < W; ++w) lds[w * kBS + tid] = j < cnt ? src[j * W + w] : 0ull;
            __syncthreads();
            const int jn = (int)min((int64_t)kBS, cnt - j0);
            for (int t = 0; t < jn && !marked; ++t) {
                if (pass == 0 && j0 + t == i) continue;
                u64 viol = 0;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const u64 y = lds[w * kBS + t];
                    viol |= d.dir == 0 ? (y & ~x[w]) : (x[w] & ~y);
                }
                marked = viol == 0;
            }
        }
    }
    if (vi) d.mark[i] = marked ? 1u : 0u;
}

__global__ void __launch_bounds__(kBS) k_red_mark(const StepDesc *descs, const int64_t *pre, int nseg) {
    __shared__ u64 lds[kMaxW * kBS];
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS StepDesc &d = cref(descs + s);
    if (!d.ghost) return;
    const int64_t lb = (int64_t)blockIdx.x - cref(pre + s);
    SRW_SWITCH_W(d.W, red_mark_w<W>(d, lb, lds));
}

// Step 2: kept sets per compaction block (the step's compaction grid)
__global__ void __launch_bounds__(kBS) k_red_count(const StepDesc *descs, const int64_t *pre, int nseg,
                                                   u32 *blk_cnt) {
    __shared__ u32 wsum[kBS / 64];
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS StepDesc &d = cref(descs + s);
    if (!d.ghost) return;
    const int64_t lb = (int64_t)blockIdx.x - cref(pre + s);
    const int64_t U = (int64_t)d.res[0];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    u32 c = 0;
#pragma unroll
    for (int t = 0; t < kCB / kBS; ++t) {
        const int64_t r = lb * kCB + t * kBS + tid;
        c += (u32)__popcll(__ballot(r < U && d.mark[r] == 0));
    }
    if (lane == 0) wsum[wave] = c;
    __syncthreads();
    if (tid == 0) {
        u32 tot = 0;
        for (int w = 0; w < kBS / 64; ++w) tot += wsum[w];
        blk_cnt[d.cblk_base + lb] = tot;
    }
}

// Step 3, one block per segment: exclusive scan of the kept counts; the
// level size becomes the kept count, res[3] the dropped one
__global__ void __launch_bounds__(kBS) k_red_scan(const StepDesc *descs, int nseg, const u32 *blk_cnt,
                                                  u32 *blk_off) {
    __shared__ u32 wsum[kBS / 64];
    const int s = blockIdx.x;
    if (s >= nseg) return;
    const CONST_AS StepDesc &d = cref(descs + s);
    if (!d.ghost) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    u64 running = 0;
    for (int64_t c0 = 0; c0 < d.ncblk; c0 += kBS) {
        const int64_t idx = c0 + tid;
        const u32 v = idx < d.ncblk ? blk_cnt[d.cblk_base + idx] : 0u;
        u32 incl = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const u32 o = __shfl_up(incl, off, 64);
            if (lane >= off) incl += o;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        u32 wpre = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kBS / 64; ++w) {
            if (w < wave) wpre += wsum[w];
            tot += wsum[w];
        }
        if (idx < d.ncblk) blk_off[d.cblk_base + idx] = (u32)(running + wpre + incl - v);
        running += tot;
        __syncthreads();
    }
    if (tid == 0) {
        d.res[3] = d.res[0] - running;
        d.res[0] = running;
    }
}

// Step 4: kept sets (in key order) to the candidate buffer and their keys
// to red_par, dropped sets to the ghost rows; every moved set's hash slot
// (found through its key: cslot[g]) names its new place, and a dropped
// set's cardinality leaves the level's sum
template <int W>
__device__ void red_compact_w(const CONST_AS StepDesc &d, int64_t lb, const u32 *blk_off, u32 *wsum) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t U = (int64_t)(d.res[0] + d.res[3]);
    u32 rank0 = blk_off[d.cblk_base + lb];
    u64 gone = 0;                              // cardinalities of the dropped sets
#pragma unroll
    for (int t = 0; t < kCB / kBS; ++t) {
        const int64_t r = lb * kCB + t * kBS + tid;
        const bool v = r < U;
        const bool keep = v && d.mark[r] == 0;
        const u64 mask = __ballot(keep);
        if (lane == 0) wsum[wave] = (u32)__popcll(mask);
        __syncthreads();
        u32 wpre = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kBS / 64; ++w) {
            if (w < wave) wpre += wsum[w];
            tot += wsum[w];
        }
        if (v) {
            const u64 rank = rank0 + wpre + lanes_below(mask);     // kept sets before r
            const u32 g = d.out_par[r];
            const u32 sl = d.cslot[g];
            const u64 e = d.tab[sl];
            if (keep) {
#pragma unroll
                for (int w = 0; w < W; ++w) d.cand[rank * W + w] = d.out_rows[r * W + w];
                d.red_par[rank] = g;
                d.tab[sl] = (e & 0xFFFFFFFF00000000ull) | (u64)(u32)(d.out_base + (int64_t)rank);
            } else {
                const int64_t gr = d.ghost_base + (r - (int64_t)rank);
                u32 card = 0;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const u64 x = d.out_rows[r * W + w];
                    d.ghost[gr * W + w] = x;
                    card += (u32)__popcll(x);
                }
                d.tab[sl] = (e & 0xFFFFFFFF00000000ull) | (u64)(kGhostBit | (u32)gr);
                gone += card;
            }
        }
        rank0 += tot;
        __syncthreads();
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) gone += (u64)__shfl_xor((long long)gone, off, 64);
    if (lane == 0 && gone) atomicAdd((unsigned long long *)(d.res + 2), (unsigned long long)(0ull - gone));
}

__global__ void __launch_bounds__(kBS) k_red_compact(const StepDesc *descs, const int64_t *pre, int nseg,
                                                     const u32 *blk_off) {
    __shared__ u32 wsum[kBS / 64];
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS StepDesc &d = cref(descs + s);
    if (!d.ghost) return;
    const int64_t lb = (int64_t)blockIdx.x - cref(pre + s);
    SRW_SWITCH_W(d.W, red_compact_w<W>(d, lb, blk_off, wsum));
}

// Step 5: the kept sets and keys back into the level
__global__ void __launch_bounds__(kBS) k_red_copy(const StepDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS StepDesc &d = cref(descs + s);
    if (!d.ghost) return;
    const int64_t r = ((int64_t)blockIdx.x - cref(pre + s)) * kBS + threadIdx.x;
    if (r >= (int64_t)d.res[0]) return;
    for (int w = 0; w < d.W; ++w) d.out_rows[r * d.W + w] = d.cand[r * d.W + w];
    d.out_par[r] = d.red_par[r];
}

// ------------------------------------------------------------ transpose

// One wave transposes word w of the 64 rows of tile `tile`: lane l ends with
// column q = 64*w + l, bit j = [state q in row 64*tile + j], stored
// state-major at YT[q * nt + tile] (nt = number of tiles) and tile-major at
// YTt[tile * 64W + q].
__device__ __forceinline__ void transpose_tile(const u64 *rows, int64_t count, int W, u64 *YT,
                                               u64 *YTt, u64 *Ysig, int64_t tile, int w,
                                               const u32 *perm = nullptr) {
    const int lane = threadIdx.x & 63;
    const int64_t j = tile * 64 + lane;
    const int64_t nt = (count + 63) / 64;
    const int64_t src = j < count ? (perm ? (int64_t)perm[j] : j) : 0;   // row j of the (sorted) level
    const u64 v = j < count ? rows[src * W + w] : 0ull;
    if (w == 0) {                       // the set's signature (0 past the end)
        u64 f = 0;
        for (int ww = 0; ww < W; ++ww) f |= j < count ? rows[src * W + ww] : 0ull;
        Ysig[j] = f;
    }
    u64 col = 0;
    for (int b = 0; b < 64; ++b) {
        const u64 m = __ballot((v >> b) & 1ull);
        if (lane == b) col = m;
    }
    YT[(int64_t)(64 * w + lane) * nt + tile] = col;
    YTt[(tile * W + w) * 64 + lane] = col;
}

__global__ void __launch_bounds__(kBS) k_transpose(const StepDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS StepDesc &d = cref(descs + s);
    const int64_t lb = (int64_t)blockIdx.x - cref(pre + s);
    const int64_t wv = lb * (kBS / 64) + (threadIdx.x >> 6);
    if (wv >= d.ntr_waves) return;
    const int64_t count = (int64_t)d.res[0];
    const int64_t tile = wv / d.W;
    const int w = (int)(wv - tile * d.W);
    if (tile * 64 >= count) return;
    transpose_tile(d.out_rows, count, d.W, d.YT, d.YTt, d.Ysig, tile, w, d.ysort ? d.ys_idx : nullptr);
}

// ------------------------------------ cardinality order of an inverse level

// A set X can lie in Y only if |X| <= |Y|.  A large new inverse level is
// put in order of decreasing cardinality (ties in any order: the meet
// resolves the least index pair through Yidx, whatever the order), so that a
// chunk of forward sets scans only the tiles of sets at least as large as its
// smallest member.
__global__ void __launch_bounds__(kBS) k_ysort_zero(const StepDesc *descs, int nseg) {
    const CONST_AS StepDesc &d = cref(descs + blockIdx.x);
    if (!d.ysort) return;
    for (int c = threadIdx.x; c <= d.n; c += kBS) d.ys_hist[c] = 0;
}
__global__ void __launch_bounds__(kBS) k_ysort_hist(const StepDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS StepDesc &d = cref(descs + s);
    const int64_t j = ((int64_t)blockIdx.x - cref(pre + s)) * kBS + threadIdx.x;
    if (j >= (int64_t)d.res[0]) return;
    int c = 0;
    for (int w = 0; w < d.W; ++w) c += __popcll(d.out_rows[j * d.W + w]);
    atomicAdd(d.ys_hist + c, 1u);
}
// one block per segment: Ycnt, and ys_hist turned into the first position
// of each cardinality (largest first)
__global__ void __launch_bounds__(kBS) k_ysort_scan(const StepDesc *descs, int nseg) {
    __shared__ u32 h[kMaxW * 64 + 1];       // n + 1 cardinalities
    const CONST_AS StepDesc &d = cref(descs + blockIdx.x);
    if (!d.ysort) return;
    for (int c = threadIdx.x; c <= d.n; c += kBS) h[c] = d.ys_hist[c];
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 acc = 0;                        // sets with more than c states
        for (int c = d.n; c >= 0; --c) {
            const u32 v = h[c];
            h[c] = acc;
            acc += v;
        }
        d.ys_cnt[0] = acc;
    }
    __syncthreads();
    for (int c = threadIdx.x; c <= d.n; c += kBS) {
        d.ys_hist[c] = h[c];
        d.ys_cnt[c + 1] = h[c];
    }
}
__global__ void __launch_bounds__(kBS) k_ysort_scatter(const StepDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS StepDesc &d = cref(descs + s);
    const int64_t j = ((int64_t)blockIdx.x - cref(pre + s)) * kBS + threadIdx.x;
    if (j >= (int64_t)d.res[0]) return;
    int c = 0;
    for (int w = 0; w < d.W; ++w) c += __popcll(d.out_rows[j * d.W + w]);
    d.ys_idx[atomicAdd(d.ys_hist + c, 1u)] = (u32)j;
}

__global__ void __launch_bounds__(kBS) k_transpose_rows(const TransposeDesc *descs, const int64_t *pre,
                                                        int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS TransposeDesc &d = cref(descs + s);
    const int64_t lb = (int64_t)blockIdx.x - cref(pre + s);
    const int64_t wv = lb * (kBS / 64) + (threadIdx.x >> 6);
    const int64_t tiles = (d.count + 63) / 64;
    if (wv >= tiles * d.W) return;
    const int64_t tile = wv / d.W;
    transpose_tile(d.rows, d.count, d.W, d.YT, d.YTt, d.Ysig, tile, (int)(wv - tile * d.W));
}

// ------------------------------------------------------------------ meet

// YS: the inverse level may be in cardinality order (read through d.Yidx
// when it is set); without it the level is in its own order and the paths
// of that order are compiled out.
template <int W, bool YS, class D>
__device__ u32 meet_w(const D &d, int64_t lb, u64 *cols) {
    const u32 *Yidx = YS ? d.Yidx : nullptr;
    const int tid = threadIdx.x;
    const int64_t nX = d.nX >= 0 ? d.nX : (int64_t)d.res[0];
    const int64_t nY = d.nY >= 0 ? d.nY : (int64_t)d.res[0];
    const int64_t xb = lb % d.nXb, yc = lb / d.nXb;
    const int64_t tiles = (nY + 63) / 64;
    const int64_t t0 = yc * d.tpb;
    const int64_t t1 = min(t0 + (int64_t)d.tpb, tiles);
    if (t0 >= t1 || xb * kBS >= nX) return 0;  // whole block
    const int64_t nw = (t1 - t0) * 64 * W;
    const u64 *src = d.YTt + t0 * 64 * W;            // tiles t0..t1-1, contiguous
    for (int64_t e = tid; e < nw; e += kBS) cols[e] = src[e];
    __syncthreads();
    const int64_t i = xb * kBS + tid;
    if (i >= nX) return 0;
    const u64 best = load_slot(d.res + 1);
    if ((best >> 32) < (u64)i) return 0;     // a smaller i already met
    u32 nops = 0;                            // 32-bit lane-ops: 2 per 64-bit AND
    u64 x[W];
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = d.X[i * W + w];
    for (int64_t t = t0; t < t1; ++t) {
        const u64 *c = cols + (t - t0) * 64 * W;
        u64 M = ~0ull;
        bool alive = true;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            if (!alive) break;
            u64 bits = x[w];
            while (bits) {
                const int b = lowest_bit(bits);
                bits &= bits - 1;
                M &= c[64 * w + b];
                nops += 2;
                if (M == 0) { alive = false; break; }
            }
        }
        if (alive) {
            if (!Yidx) {                   // level order: the lowest bit is the least j
                const u64 j = (u64)t * 64 + (u64)lowest_bit(M);
                atomicMin(d.res + 1, ((u64)i << 32) | j);
                return nops;
            }
            for (u64 mm = M; mm; mm &= mm - 1)   // cardinality order: every hit
                atomicMin(d.res + 1, ((u64)i << 32) | (u64)Yidx[(u64)t * 64 + lowest_bit(mm)]);
        }
    }
    return nops;
}

// a / b for a >= 0, b > 0, in 32 bits when both fit
__device__ __forceinline__ int64_t udiv(int64_t a, int64_t b) {
    if (((u64)a | (u64)b) >> 32 == 0) return (int64_t)((u32)a / (u32)b);
    return (int64_t)((u64)a / (u64)b);
}

__device__ __forceinline__ u64 shfl64(u64 v, int src) {
    const u32 lo = (u32)__shfl((int)(u32)v, src, 64);
    const u32 hi = (u32)__shfl((int)(u32)(v >> 32), src, 64);
    return ((u64)hi << 32) | lo;
}

// Mode 1: one wave per work item = (chunk c of 64 sorted sets X, a range of
// groups of 64 tiles).  C = the states common to the whole chunk.  A set Y
// can contain some X of the chunk only if it contains C, so each lane takes
// one tile of a group and ANDs the columns of (at most kCommonMax states of)
// C over it: coalesced loads, issued a few at a time without waiting on each
// other.  The surviving (tile, bit) pairs are the candidate sets Y_j.  Their
// indices are listed in the wave's slice of LDS, the one-word signatures of
// those sets (the OR of a set's words) are gathered next to them in one round
// of independent loads, and every lane tests X minus C against each
// signature: X subset of Y implies OR(X) subset of OR(Y), so a failed test
// rejects exactly; only a lane whose test passes reads the whole row of that
// Y.  Candidates go in increasing j, so a lane's first hit is its least j.
// When a group has very many
// candidates (chunks with almost no common state) the remaining states of
// each X are ANDed over the columns of each surviving tile instead.
// Mode 1 takes a work item apart into (chunk c, group range gi); mode 2
// (BK: the inverse level in buckets) is handed (c, gi) by its queue.
//
// BK: only the tiles of the buckets whose key contains the chunk's key a
// (the split states common to the chunk) can hold a superset of a set of the
// chunk; they are tile list a of the bucketed level, read through the list
// (key 0, or lists that did not fit: every tile in order).  The split states
// of a hold in every set of those buckets, so they are taken out of each X
// and out of the filtering states.  Level indices come through Yidx (the
// bucket order is not the level order, so a hit does not end a lane).
//
// CNT: count the set operations (the returned lane-ops) and the work (into
// d.mstat); a profiling build of the kernel, the other one does neither.
template <int W, bool YS, bool BK, bool CNT>
__device__ u32 meet_chunk_core(const CONST_AS StepDesc &d, int64_t c, int64_t gi, u64 *slice) {
    const int lane = threadIdx.x & 63;
    const u32 *Yidx = YS ? d.Yidx : nullptr;
    const u32 *Ycnt = (YS && !BK) ? d.Ycnt : nullptr;
    const int64_t nX = d.nX >= 0 ? d.nX : (int64_t)d.res[0];
    const int64_t nY = d.nY >= 0 ? d.nY : (int64_t)d.res[0];
    const int64_t nt = BK ? (int64_t)d.yb->nt : (nY + 63) / 64;
    if (c * 64 >= nX) return 0;                    // whole wave
    const int64_t is = c * 64 + lane;
    const bool valid = is < nX;
    // BK: the chunk's key and its split states
    u64 smask[W];
#pragma unroll
    for (int w = 0; w < W; ++w) smask[w] = 0;
    const u32 *tlist = nullptr;                    // the chunk's tile list (null: every tile)
    int64_t nvt = nt;                              // tiles the chunk scans
    if (BK) {
        u32 a = 0;
#pragma unroll
        for (int i = 0; i < kYBits; ++i) {
            const int q = d.yb->split[i];
            if (q >= 0 && ((d.Xcom[c * W + (q >> 6)] >> (q & 63)) & 1ull)) {
                a |= 1u << (kYBits - 1 - i);
                smask[q >> 6] |= 1ull << (q & 63);
            }
        }
        if (a != 0 && d.yb->ok) {
            tlist = d.yb_list + d.yb_loff[a];
            nvt = d.yb_lsize[a];
        } else {
            // every tile is scanned, sets without the split states too: the
            // states stay in X and among the filtering states
#pragma unroll
            for (int w = 0; w < W; ++w) smask[w] = 0;
        }
    }
    const int64_t ngroups = (nvt + 63) / 64;
    const int64_t g0 = gi * d.ngi;
    int64_t g1 = min(g0 + d.ngi, ngroups);
    if (g0 >= g1) return 0;                        // whole wave
    // the first kCommonMax states of C (-1: none); only those are filtered
    // on, so only those (and the split states of the key) are taken out of X
    int cq[kCommonMax];
    u64 x[W];
    {
        u64 cur[W];
#pragma unroll
        for (int w = 0; w < W; ++w) cur[w] = d.Xcom[c * W + w] & ~smask[w];
        u64 used[W];
#pragma unroll
        for (int w = 0; w < W; ++w) used[w] = cur[w];
#pragma unroll
        for (int r = 0; r < kCommonMax; ++r) {
            int qq = -1;
#pragma unroll
            for (int w = 0; w < W; ++w)
                if (qq < 0 && cur[w]) {
                    qq = 64 * w + lowest_bit(cur[w]);
                    cur[w] &= cur[w] - 1;
                }
            cq[r] = qq;
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
            used[w] &= ~cur[w];                    // states of C left unfiltered stay in x
            x[w] = valid ? (d.X[is * W + w] & ~(used[w] | smask[w])) : 0ull;
        }
    }
    int nc = 0;                                    // states of C filtered on
#pragma unroll
    for (int r = 0; r < kCommonMax; ++r) nc += cq[r] >= 0;
    // the set operations this lane performs, in 32-bit lane-ops: 2 per
    // 64-bit AND of a column, 4 per word of a row test (and-not, or)
    u32 nops = 0;
    const u32 orig = valid ? d.Xidx[is] : 0xFFFFFFFFu;
    // inverse level in cardinality order: only its first Ycnt[min |X|] sets
    // can contain a set of this chunk
    int64_t nt_lim = nvt;
    if (Ycnt) {
        int sz = 0x7fffffff;
        if (valid) {
            sz = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) sz += __popcll(x[w]);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) sz = min(sz, __shfl_xor(sz, off, 64));
        int csz = 0;                       // the states of C taken out of each x
#pragma unroll
        for (int r = 0; r < kCommonMax; ++r) csz += cq[r] >= 0;
        nt_lim = ((int64_t)Ycnt[min(sz + csz, d.n + 1)] + 63) / 64;
    }
    bool done = !valid || (load_slot(d.res + 1) >> 32) < (u64)orig;
    // slice: candidate indices (u32) in words 0 .. kRowBatchMax/2-1, their
    // signatures after them
    u32 *jl = (u32 *)slice;
    u64 *sig = slice + kRowBatchMax / 2;
    u64 xs = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) xs |= x[w];
    // first round of common columns of group gg, loaded two groups ahead
    // (a group with no candidate is a few dozen instructions, far shorter than
    // a load).  Lanes past the last tile and unused states load word 0 of YT,
    // so the loads need no branch; the words are used raw and masked where
    // the group consumes them (a select here would wait for the load).
    // the tile of the chunk's vt-th scanned tile
    auto tile_of = [&](int64_t vt) -> int64_t {
        if (!BK || !tlist) return vt;
        return vt < nvt ? (int64_t)tlist[vt] : 0;
    };
    auto first_round = [&](int64_t gg, u64 *v) {
        const int64_t vg = gg * 64 + lane;
        const int64_t tg = tile_of(vg);
#pragma unroll
        for (int r = 0; r < kCommonRound; ++r) {
            const bool ok = vg < nvt && cq[r] >= 0;
            v[r] = d.YT[ok ? (int64_t)cq[r] * nt + tg : 0];
        }
    };
    // the last tile may be partial (buckets are padded with empty sets)
    const u64 last_rows = (BK || (nY & 63) == 0) ? ~0ull : ((1ull << (nY & 63)) - 1ull);
    // one group with its first-round columns in cur; refills cur for group g + 2.
    // false: every lane of the wave is done
    // work counters (the same in every lane; row tests per lane)
    u32 w_groups = 0, w_groups_k = 0, w_cand = 0, w_col_tiles = 0, w_tiles = 0, w_full = 0;
    auto group = [&](int64_t g, u64 *cur) -> bool {
        // every fourth group: a lane whose X has a larger index than a
        // meeting pair found meanwhile is done (the least pair is sought)
        if ((g & 3) == 3 && (load_slot(d.res + 1) >> 32) < (u64)orig) done = true;
        if (__ballot(!done) == 0) return false;
        const int64_t vt = g * 64 + lane;
        const bool tv = vt < nt_lim;
        const int64_t t = tile_of(vt);
        if (CNT) {
            ++w_groups;
            w_tiles += (u32)__popcll(__ballot(tv));
        }
        // lanes past the tiles (t >= nt_lim, so also t >= nt) start from 0,
        // so the raw word they loaded does not matter; an unused state (cq
        // < 0, uniform over the wave) contributes no column
        u64 m = !tv ? 0ull : (t == nt - 1 ? last_rows : ~0ull);
#pragma unroll
        for (int r = 0; r < kCommonRound; ++r) m &= cq[r] >= 0 ? cur[r] : ~0ull;
        if (CNT && tv) nops += 2 * min(nc, kCommonRound);
        // further common columns, in rounds of independent loads (issued
        // before the lookahead of group g + 2, so that waiting for them does
        // not also wait for that lookahead)
#pragma unroll
        for (int r0 = kCommonRound; r0 < kCommonMax; r0 += kCommonRound) {
            if (cq[r0] < 0 || __ballot(m != 0) == 0) break;
            u64 v[kCommonRound];
#pragma unroll
            for (int r = 0; r < kCommonRound; ++r) {
                const bool ok = tv && cq[r0 + r] >= 0;
                v[r] = d.YT[ok ? (int64_t)cq[r0 + r] * nt + t : 0];
            }
#pragma unroll
            for (int r = 0; r < kCommonRound; ++r) m &= cq[r0 + r] >= 0 ? v[r] : ~0ull;
            if (CNT && tv) nops += 2 * min(nc - r0, kCommonRound);
        }
        if (g + 2 < g1) first_round(g + 2, cur);
        if (__ballot(m != 0) == 0) return true;      // the usual case: no candidate in the group
        // number the candidates: lane order (tile), then bit order
        const u32 pc = (u32)__popcll(m);
        u32 incl = pc;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const u32 o = (u32)__shfl_up((int)incl, off, 64);
            if (lane >= off) incl += o;
        }
        const u32 K = (u32)__shfl((int)incl, 63, 64);
        if (K == 0) return true;
        if (CNT) ++w_groups_k;
        if (K <= (u32)d.row_batch_max) {              // row_batch_max <= kRowBatchMax
            if (CNT) w_cand += K;
            wave_sync_lds();                           // the last group's lists are read
            {
                u64 mm = m;
                for (u32 idx = incl - pc; mm; ++idx) {
                    jl[idx] = (u32)(t * 64 + lowest_bit(mm));
                    mm &= mm - 1;
                }
            }
            wave_sync_lds();
            for (u32 b0 = 0; b0 < K; b0 += 4 * 64) {   // 4 independent gathers per lane
                u64 sv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const u32 idx = b0 + 64 * u + lane;
                    sv[u] = idx < K ? d.Ysig[jl[idx]] : 0ull;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const u32 idx = b0 + 64 * u + lane;
                    if (idx < K) sig[idx] = sv[u];
                }
            }
            wave_sync_lds();
            if (CNT && !done) nops += K * 2;
            // K is the same in every lane: loop bounds and the tail test are
            // scalar.  Eight candidates a round: one broadcast LDS read and
            // one branch-free test each; a lane whose X passes a signature
            // test (rare) tests those candidates' rows in full.
            const u32 Ku = __builtin_amdgcn_readfirstlane(K);
            auto full = [&](u32 c0, u32 cnt) {
                for (u32 u = 0; u < cnt; ++u) {
                    const u32 cc = c0 + u;
                    if (done || (xs & ~sig[cc]) != 0) continue;
                    const u32 jc = Yidx ? Yidx[jl[cc]] : jl[cc];   // index in the level
                    u64 out = 0;
#pragma unroll
                    for (int w = 0; w < W; ++w) out |= x[w] & ~d.Yrows[(int64_t)jc * W + w];
                    if (CNT) {
                        nops += 4 * W;
                        ++w_full;
                    }
                    if (out == 0) {
                        atomicMin(d.res + 1, ((u64)orig << 32) | (u64)jc);
                        done = !Yidx;              // another order: a later hit may be smaller
                    }
                }
            };
            u32 c0 = 0;
            for (; c0 + 8 <= Ku; c0 += 8) {
                bool p = false;
#pragma unroll
                for (int u = 0; u < 8; ++u) p |= (xs & ~sig[c0 + u]) == 0;
                if (__ballot(p && !done)) full(c0, 8);
            }
            if (c0 < Ku) {
                bool p = false;
#pragma unroll
                for (int u = 0; u < 8; ++u) p |= c0 + u < Ku && (xs & ~sig[c0 + u]) == 0;
                if (__ballot(p && !done)) full(c0, Ku - c0);
            }
            return true;
        }
        // many candidates: per surviving tile, stage its columns in LDS
        // (coalesced, tile-major) and AND the remaining states of each X
        u64 surv = __ballot(m != 0);
        while (surv) {
            const int lt = lowest_bit(surv);
            surv &= surv - 1;
            const u64 mc = shfl64(m, lt);
            const int64_t tt = BK ? (int64_t)shfl64((u64)t, lt) : g * 64 + lt;
            if (__ballot(!done) == 0) break;
            if (CNT) ++w_col_tiles;
            wave_sync_lds();                       // the last tile is read
#pragma unroll
            for (int w = 0; w < W; ++w) slice[64 * w + lane] = d.YTt[tt * 64 * W + 64 * w + lane];
            wave_sync_lds();
            if (done) continue;
            u64 M = mc;
            bool alive = true;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                if (!alive) break;
                u64 b = x[w];
                while (b) {
                    const int q = 64 * w + lowest_bit(b);
                    b &= b - 1;
                    M &= slice[q];
                    if (M == 0) { alive = false; break; }
                }
                if (CNT) nops += 2 * (u32)(__popcll(x[w]) - __popcll(b));
            }
            if (alive) {
                if (!Yidx) {
                    atomicMin(d.res + 1, ((u64)orig << 32) | (u64)(tt * 64 + lowest_bit(M)));
                    done = true;
                } else {
                    for (u64 mm = M; mm; mm &= mm - 1)
                        atomicMin(d.res + 1, ((u64)orig << 32) | (u64)Yidx[tt * 64 + lowest_bit(mm)]);
                }
            }
        }
        return true;
    };
    g1 = min(g1, (nt_lim + 63) / 64);
    if (g0 >= g1) return nops;
    u64 pa[kCommonRound], pb[kCommonRound];
    if (g0 < g1) first_round(g0, pa);
    if (g0 + 1 < g1) first_round(g0 + 1, pb);
    for (int64_t g = g0; g < g1; g += 2) {
        if (!group(g, pa)) break;
        if (g + 1 < g1 && !group(g + 1, pb)) break;
    }
    if (CNT && d.mstat) {
        u32 full = w_full;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) full += (u32)__shfl_xor((int)full, off, 64);
        if (lane == 0) {
            u64 *m = d.mstat + (blockIdx.x % kMstatSlots) * kOpsStride;
            atomicAdd((unsigned long long *)m + 0, 1ull);
            atomicAdd((unsigned long long *)m + 1, (unsigned long long)w_groups);
            atomicAdd((unsigned long long *)m + 2, (unsigned long long)w_groups_k);
            atomicAdd((unsigned long long *)m + 3, (unsigned long long)w_cand);
            atomicAdd((unsigned long long *)m + 4, (unsigned long long)full);
            atomicAdd((unsigned long long *)m + 5, (unsigned long long)w_col_tiles);
            atomicAdd((unsigned long long *)m + 6, (unsigned long long)w_tiles);
        }
    }
    return nops;
}

template <int W, bool YS, bool CNT>
__device__ u32 meet_chunk_w(const CONST_AS StepDesc &d, int64_t item, u64 *slice) {
    // tile-range-major: the items in flight share one range of tiles, so its
    // columns and rows stay in L2 (every XCD works on the same range)
    int64_t c, gi;
    if (d.item_order == 0) { gi = udiv(item, d.nch_ub); c = item - gi * d.nch_ub; }
    else { c = udiv(item, d.gitems_ub); gi = item - c * d.gitems_ub; }
    return meet_chunk_core<W, YS, false, CNT>(d, c, gi, slice);
}

// Grid-stride over work items: mode 0 items are blocks (256 sets X against
// up to `tpb` tiles staged in LDS), mode 1 items are waves (4 per block).
// The item count can exceed the grid limit.  One launch covers segments
// s0..s1-1, which all have W words per set (a kernel per width keeps the
// register count of the narrow widths low).  With `ops` set, the set
// operations the launch performed (32-bit lane-ops) are added to the
// kOpsSlots counters at ops (kOpsStride words apart).
template <int W, bool YS, bool CNT>
__global__ void __launch_bounds__(kBS) k_meet(const StepDesc *descs, const int64_t *pre, int s0, int s1, u64 *ops) {
    __shared__ u64 cols[kMeetLdsWords];
    const int64_t base = cref(pre + s0), items = cref(pre + s1) - base;
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int s = s0 + find_seg(pre + s0, s1 - s0, base + it);
        const CONST_AS StepDesc &d = cref(descs + s);
        const int64_t li = base + it - cref(pre + s);
        __syncthreads();   // the previous item is done with cols
        u32 nops;
        if (d.meet_mode == 0) {
            nops = meet_w<W, YS>(d, li, cols);
        } else {
            const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wave
            nops = meet_chunk_w<W, YS, CNT>(d, li * (kBS / 64) + wave, cols + wave * kSliceWords);
        }
        if (ops) {
            u32 sum = nops;   // at most a few million per wave and item
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) sum += (u32)__shfl_xor((int)sum, off, 64);
            if ((threadIdx.x & 63) == 0 && sum)
                atomicAdd((unsigned long long *)(ops + (blockIdx.x % kOpsSlots) * kOpsStride), (unsigned long long)sum);
        }
    }
}

// Mode 2: waves take work items from each segment's queue in turn, until
// the queue is empty (its counter passes the item count the plan wrote),
// so every wave of the grid ends.  Work items go in the plan's order (see
// kOrderKeys): per order key, range by range of d.ngi tile groups of the
// key's list, and within a range chunk by chunk.
//
// With d.xcd_granule = G > 0 the items are dealt to eight queues, one per
// XCD: runs of G consecutive items in plan order go to queue 0, 1, ..., 7,
// 0, ... in turn, so the chunks that scan one range of tiles mostly run on
// one XCD and share its L2 (each XCD has its own).  Workgroups are
// dispatched to the XCDs round robin, so block b serves queue b % 8 first;
// a wave whose queue is empty takes from the next queues.  Queue x's j-th
// item is item ((j / G) * 8 + x) * G + j % G of the plan: every item is in
// exactly one queue, and a queue's items rise with j, so a wave that finds
// every queue past the item count has nothing left to take.
template <int W, bool CNT>
__global__ void __launch_bounds__(kBS) k_meet_b(const StepDesc *descs, int s0, int s1, u64 *ops) {
    __shared__ u64 cols[kMeetLdsWords];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    u64 *slice = cols + wave * kSliceWords;
    u32 nops = 0;
    for (int s = s0; s < s1; ++s) {
        const CONST_AS StepDesc &d = cref(descs + s);
        if (d.meet_mode != 2) continue;
        const int64_t nX = d.nX >= 0 ? d.nX : (int64_t)d.res[0];
        const u32 nch = (u32)((nX + 63) / 64);
        // the plan's item count, capped by the host's upper bound of it
        const u32 total = (u32)min((int64_t)__hip_atomic_load(d.queue + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                                   d.nch_ub * d.gitems_ub);
        const u32 G = (u32)d.xcd_granule;
        const u32 x0 = blockIdx.x & 7u;
        for (;;) {
            u32 it = 0xFFFFFFFFu;
            if (lane == 0) {
                if (G == 0) {
                    it = atomicAdd(d.queue, 1u);
                } else {
                    for (u32 t = 0; t < 8; ++t) {
                        const u32 x = (x0 + t) & 7u;
                        const u64 j = atomicAdd(d.queue + 2 + x, 1u);
                        const u64 i = ((j / G) * 8 + x) * G + j % G;
                        if (i < total) { it = (u32)i; break; }
                    }
                }
            }
            it = __builtin_amdgcn_readfirstlane(__shfl((int)it, 0, 64));
            if (it >= total) break;
            const u32 *kpre = d.kinfo + kKPre;
            u32 lo = 0, hi = kOrderKeys;           // kpre[lo] <= it < kpre[hi]
            while (hi - lo > 1) {
                const u32 mid = (lo + hi) >> 1;
                if (kpre[mid] <= it) lo = mid; else hi = mid;
            }
            const u32 cnt = d.kinfo[kKCount + lo];   // chunks of order key lo (> 0: it has items)
            const u32 rem = it - kpre[lo];
            const u32 r = rem / cnt;
            const u32 c = d.korder[d.kinfo[kKStart + lo] + (rem - r * cnt)];
            (void)nch;
            nops += meet_chunk_core<W, true, true, CNT>(d, c, r, slice);
        }
    }
    if (ops) {
        u32 sum = nops;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) sum += (u32)__shfl_xor((int)sum, off, 64);
        if (lane == 0 && sum)
            atomicAdd((unsigned long long *)(ops + (blockIdx.x % kOpsSlots) * kOpsStride), (unsigned long long)sum);
    }
}

// ---------------------------------------- inverse levels in buckets

// key of a set: bit kYBits-1-i is [split[i] in the set]
template <class D>
__device__ __forceinline__ u32 yb_key_of(const D &d, const u64 *row, const int32_t *split) {
    u32 k = 0;
#pragma unroll
    for (int i = 0; i < kYBits; ++i) {
        const int q = split[i];
        const u32 bit = q >= 0 ? (u32)((row[q >> 6] >> (q & 63)) & 1ull) : 0u;
        k |= bit << (kYBits - 1 - i);
    }
    return k;
}

__device__ __forceinline__ int64_t yb_count(const CONST_AS YbDesc &d) {
    return d.cnt ? (int64_t)*d.cnt : d.count;
}

// one block per segment: clear the counters, record the split states
__global__ void __launch_bounds__(kBS) k_yb_zero(const YbDesc *descs, int nseg) {
    const CONST_AS YbDesc &d = cref(descs + blockIdx.x);
    for (int e = threadIdx.x; e < 2 * kYBins; e += kBS) d.bins[e] = 0;
    if (threadIdx.x < kYBits) {
        const int q = d.top[threadIdx.x];
        d.meta->split[threadIdx.x] = q < d.n ? q : -1;
    }
}

// keys and bucket sizes (per-block histogram in LDS)
__global__ void __launch_bounds__(kBS) k_yb_hist(const YbDesc *descs, const int64_t *pre, int nseg) {
    __shared__ u32 h[kYBins];
    __shared__ int32_t split[kYBits];
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS YbDesc &d = cref(descs + s);
    const int64_t j = ((int64_t)blockIdx.x - cref(pre + s)) * kBS + threadIdx.x;
    for (int e = threadIdx.x; e < kYBins; e += kBS) h[e] = 0;
    if (threadIdx.x < kYBits) {
        const int q = d.top[threadIdx.x];
        split[threadIdx.x] = q < d.n ? q : -1;
    }
    __syncthreads();
    if (j < yb_count(d)) {
        const u32 k = yb_key_of(d, d.rows + j * d.W, split);
        d.key[j] = (uint16_t)k;
        atomicAdd(&h[k], 1u);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kYBins; e += kBS)
        if (h[e]) atomicAdd(&d.bins[e], h[e]);
}

// one block per segment: tiles per bucket and their first tiles, the
// insertion cursors, then the list lengths -- for key a, the tiles of all
// buckets b containing a (a sum over supersets, one pass per key bit) --
// and the list offsets; key 0 scans every tile and has no list
__global__ void __launch_bounds__(kBS) k_yb_scan(const YbDesc *descs, int nseg) {
    __shared__ u32 t[kYBins];
    __shared__ u32 wsum[kBS / 64];
    __shared__ u32 carry;
    const CONST_AS YbDesc &d = cref(descs + blockIdx.x);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < kYBins; e += kBS) t[e] = (d.bins[e] + 63) / 64;
    __syncthreads();
    // exclusive scan of t into tb (4 entries per thread, in order)
    auto scan = [&](const u32 *src, u32 *dst, u32 &total) {
        constexpr int kPer = kYBins / kBS;
        u32 v[kPer], run = 0;
#pragma unroll
        for (int i = 0; i < kPer; ++i) { v[i] = src[tid * kPer + i]; run += v[i]; }
        u32 incl = run;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const u32 o = (u32)__shfl_up((int)incl, off, 64);
            if (lane >= off) incl += o;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        u32 wpre = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kBS / 64; ++w) {
            if (w < wave) wpre += wsum[w];
            tot += wsum[w];
        }
        u32 acc = wpre + incl - run;
#pragma unroll
        for (int i = 0; i < kPer; ++i) { dst[tid * kPer + i] = acc; acc += v[i]; }
        total = tot;
        __syncthreads();
    };
    u32 nt = 0;
    scan(t, d.tb, nt);
    if (tid == 0) d.tb[kYBins] = nt;
    __syncthreads();
    for (int e = tid; e < kYBins; e += kBS) d.bins[kYBins + e] = d.tb[e] * 64;   // insertion cursors
    // superset sums of the tile counts
    for (int i = 0; i < kYBits; ++i) {
        const u32 bit = 1u << i;
        for (int e = tid; e < kYBins; e += kBS)
            if (!(e & bit)) t[e] += t[e | bit];
        __syncthreads();
    }
    if (tid == 0) t[0] = 0;
    __syncthreads();
    for (int e = tid; e < kYBins; e += kBS) d.lsize[e] = t[e];
    u32 ent = 0;
    scan(t, d.loff, ent);
    for (int e = tid; e < kYBins; e += kBS) d.lcur[e] = d.loff[e];
    if (tid == 0) {
        d.loff[kYBins] = ent;
        d.meta->nt = (int32_t)nt;
        d.meta->entries = ent;
        d.meta->ok = (int64_t)ent <= d.list_cap ? 1 : 0;
        carry = 0;
    }
}

__global__ void __launch_bounds__(kBS) k_yb_fill(const YbDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS YbDesc &d = cref(descs + s);
    const int64_t e = ((int64_t)blockIdx.x - cref(pre + s)) * kBS + threadIdx.x;
    if (e < d.nt_ub * 64) d.idx[e] = 0xFFFFFFFFu;
}

// every set to a free place of its bucket (any order within a bucket: the
// meet resolves the least index pair through idx).  The block's sets of one
// bucket take one range of places with a single global atomic; within the
// block each set's place comes from an LDS counter.
__global__ void __launch_bounds__(kBS) k_yb_scatter(const YbDesc *descs, const int64_t *pre, int nseg) {
    __shared__ u32 h[kYBins];
    __shared__ u32 base[kYBins];
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS YbDesc &d = cref(descs + s);
    const int64_t j = ((int64_t)blockIdx.x - cref(pre + s)) * kBS + threadIdx.x;
    for (int e = threadIdx.x; e < kYBins; e += kBS) h[e] = 0;
    __syncthreads();
    const bool valid = j < yb_count(d);
    u32 k = 0, lpos = 0;
    if (valid) {
        k = d.key[j];
        lpos = atomicAdd(&h[k], 1u);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kYBins; e += kBS)
        if (h[e]) base[e] = atomicAdd(&d.bins[kYBins + e], h[e]);
    __syncthreads();
    if (valid) d.idx[base[k] + lpos] = (u32)j;
}

// one wave per bucket b: its tiles go into the list of every nonzero key a
// contained in b (any order within a list)
__global__ void __launch_bounds__(kBS) k_yb_list(const YbDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS YbDesc &d = cref(descs + s);
    const int lane = threadIdx.x & 63;
    const u32 b = (u32)(((int64_t)blockIdx.x - cref(pre + s)) * (kBS / 64) + (threadIdx.x >> 6));
    if (b >= (u32)kYBins || !d.meta->ok || b == 0) return;
    const u32 t0 = d.tb[b], nb = d.tb[b + 1] - t0;
    if (nb == 0) return;
    for (u32 a = b; a != 0; a = (a - 1) & b) {
        u32 base = 0;
        if (lane == 0) base = atomicAdd(&d.lcur[a], nb);
        base = (u32)__shfl((int)base, 0, 64);
        for (u32 i = lane; i < nb; i += 64) d.list[base + i] = t0 + i;
    }
}

// the padded level transposed: one wave per (tile, word); padding is empty
__global__ void __launch_bounds__(kBS) k_yb_transpose(const YbDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS YbDesc &d = cref(descs + s);
    const int64_t wv = ((int64_t)blockIdx.x - cref(pre + s)) * (kBS / 64) + (threadIdx.x >> 6);
    const int W = d.W;
    const int64_t nt = d.meta->nt;
    const int64_t tile = wv / W;
    if (tile >= nt) return;
    const int w = (int)(wv - tile * W);
    const int lane = threadIdx.x & 63;
    const int64_t pos = tile * 64 + lane;
    const u32 src = d.idx[pos];
    const bool real = src != 0xFFFFFFFFu;
    const u64 v = real ? d.rows[(int64_t)src * W + w] : 0ull;
    if (w == 0) {
        u64 f = 0;
        for (int ww = 0; ww < W; ++ww) f |= real ? d.rows[(int64_t)src * W + ww] : 0ull;
        d.Ysig[pos] = f;
    }
    u64 col = 0;
    for (int bb = 0; bb < 64; ++bb) {
        const u64 m = __ballot((v >> bb) & 1ull);
        if (lane == bb) col = m;
    }
    d.YT[(int64_t)(64 * w + lane) * nt + tile] = col;
    d.YTt[(tile * W + w) * 64 + lane] = col;
}

// ------------------------------------------------------ meet plan (mode 2)

// chunk key (the split states common to the chunk)
template <class D>
__device__ __forceinline__ u32 chunk_key(const D &d, int64_t c) {
    u32 a = 0;
    for (int i = 0; i < kYBits; ++i) {
        const int q = d.yb->split[i];
        if (q >= 0 && ((d.Xcom[c * d.W + (q >> 6)] >> (q & 63)) & 1ull)) a |= 1u << (kYBits - 1 - i);
    }
    return a;
}

// one block per segment: clear the chunk counts of the order keys
__global__ void __launch_bounds__(kBS) k_mp_zero(const StepDesc *descs, int nseg) {
    const CONST_AS StepDesc &d = cref(descs + blockIdx.x);
    if (d.meet_mode != 2) return;
    for (int e = threadIdx.x; e < kOrderKeys; e += kBS) d.kinfo[kKCount + e] = 0;
}

// per chunk: its order key (index bin of its least index in the level,
// then its bucket key), counted per order key
__global__ void __launch_bounds__(kBS) k_mp_keys(const StepDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS StepDesc &d = cref(descs + s);
    if (d.meet_mode != 2) return;
    const int64_t c = ((int64_t)blockIdx.x - cref(pre + s)) * kBS + threadIdx.x;
    const int64_t nX = d.nX >= 0 ? d.nX : (int64_t)d.res[0];
    if (c * 64 >= nX) return;
    u32 imin = 0xFFFFFFFFu;
    const int64_t e1 = min(c * 64 + 64, nX);
    for (int64_t e = c * 64; e < e1; ++e) imin = min(imin, d.Xidx[e]);
    const u32 bin = (u32)(((u64)imin * kIndexBins) / (u64)nX);
    const u32 ok = bin * kYBins + chunk_key(d, c);
    d.ckey[c] = ok;
    atomicAdd(&d.kinfo[kKCount + ok], 1u);
}

// exclusive scan of cnt = kMpThreads * kMpRun counters by a block of
// kMpThreads threads, each owning a run of kMpRun consecutive ones; returns
// the total (every thread)
constexpr int kMpThreads = 1024;
constexpr int kMpRun = kOrderKeys / kMpThreads;
static_assert(kOrderKeys % kMpThreads == 0, "order keys in whole runs");
__device__ u32 block_scan_runs(const u32 *n, u32 *out, u32 *wsum) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const u32 *src = n + (int64_t)tid * kMpRun;
    u32 sum = 0;
#pragma unroll
    for (int j = 0; j < kMpRun; ++j) sum += src[j];
    u32 incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const u32 o = (u32)__shfl_up((int)incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    u32 acc = incl - sum, tot = 0;
    for (int w = 0; w < kMpThreads / 64; ++w) {
        acc += w < wave ? wsum[w] : 0u;
        tot += wsum[w];
    }
    u32 *dst = out + (int64_t)tid * kMpRun;
#pragma unroll
    for (int j = 0; j < kMpRun; ++j) {
        const u32 v = src[j];
        dst[j] = acc;
        acc += v;
    }
    __syncthreads();                       // wsum is reused by the next scan
    return tot;
}

// one block per segment: per order key its tile ranges (of d.ngi groups of
// its bucket key's list; key 0 and lists that did not fit: every tile) and
// work items, then its first place in korder and first work item, the item
// count and the queue reset
__global__ void __launch_bounds__(kMpThreads) k_mp_scan(const StepDesc *descs, int nseg) {
    __shared__ u32 wsum[kMpThreads / 64];
    const CONST_AS StepDesc &d = cref(descs + blockIdx.x);
    if (d.meet_mode != 2) return;
    for (int e = threadIdx.x; e < kOrderKeys; e += kMpThreads) {
        const u32 cnt = d.kinfo[kKCount + e];
        const u32 a = (u32)e % kYBins;
        const int64_t nvt = (a != 0 && d.yb->ok) ? (int64_t)d.yb_lsize[a] : (int64_t)d.yb->nt;
        const u32 ranges = cnt ? (u32)(((nvt + 63) / 64 + d.ngi - 1) / d.ngi) : 0u;
        d.kinfo[kKRanges + e] = ranges;
        d.kinfo[kKCur + e] = cnt * ranges;        // work items, scanned below
    }
    __syncthreads();
    block_scan_runs(d.kinfo + kKCount, d.kinfo + kKStart, wsum);
    const u32 total = block_scan_runs(d.kinfo + kKCur, d.kinfo + kKPre, wsum);
    for (int e = threadIdx.x; e < kOrderKeys; e += kMpThreads) d.kinfo[kKCur + e] = d.kinfo[kKStart + e];
    if (threadIdx.x == 0) {
        d.kinfo[kKPre + kOrderKeys] = total;
        d.queue[0] = 0;
        d.queue[1] = total;
        for (int x = 0; x < 8; ++x) d.queue[2 + x] = 0;
    }
}

// every chunk to a place of its order key in korder (any order within a key)
__global__ void __launch_bounds__(kBS) k_mp_scatter(const StepDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS StepDesc &d = cref(descs + s);
    if (d.meet_mode != 2) return;
    const int64_t c = ((int64_t)blockIdx.x - cref(pre + s)) * kBS + threadIdx.x;
    const int64_t nX = d.nX >= 0 ? d.nX : (int64_t)d.res[0];
    if (c * 64 >= nX) return;
    d.korder[atomicAdd(&d.kinfo[kKCur + d.ckey[c]], 1u)] = (u32)c;
}

// ------------------------------------------------------ copies

__global__ void __launch_bounds__(kBS) k_copy(const CopyDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS CopyDesc &d = cref(descs + s);
    const int64_t base = ((int64_t)blockIdx.x - cref(pre + s)) * kCopyPerBlock;
    for (int i = threadIdx.x; i < kCopyPerBlock; i += kBS) {
        const int64_t e = base + i;
        if (e < d.count) d.dst[e] = d.src[e];
    }
}

// ------------------------------------------------------ small steps

// One block runs a whole step of one small segment: expansion, insertion,
// compaction in key order (a running rank over the candidates instead of a
// scan across blocks), the transpose of a new inverse level and the LDS-tile
// meet, with a barrier between phases.  The same device functions as the
// per-phase kernels do the work, so the results are the same; what goes is
// six dependent launches per step, which dominate when the lists are tiny (a
// Černý automaton takes (n-1)^2 steps over lists of about n sets).
template <int W, class D>
__device__ u32 step_small_w(const D &d, u64 *lds, u32 *wsum) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t nb = (d.C + kBS - 1) / kBS;
    for (int64_t lb = 0; lb < nb; ++lb) expand_w<W>(d, lb, lds);
    __syncthreads();
    for (int64_t lb = 0; lb < nb; ++lb) insert_w<W>(d, lb);
    __syncthreads();
    u32 rank0 = 0;
    u32 card = 0;                          // cardinalities of this lane's winners
    for (int64_t g0 = 0; g0 < d.C; g0 += kBS) {
        const int64_t g = g0 + tid;
        const bool f = g < d.C && is_winner(d, g);
        const u64 mask = __ballot(f);
        if (lane == 0) wsum[wave] = (u32)__popcll(mask);
        __syncthreads();
        u32 wpre = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kBS / 64; ++w) {
            if (w < wave) wpre += wsum[w];
            tot += wsum[w];
        }
        if (f) {
            const u64 rank = rank0 + wpre + lanes_below(mask);
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const u64 v = d.cand[g * W + w];
                d.out_rows[rank * W + w] = v;
                card += (u32)__popcll(v);
            }
            d.out_par[rank] = (u32)g;
            const u32 sl = d.cslot[g];
            const u64 e = d.tab[sl];
            d.tab[sl] = (e & 0xFFFFFFFF00000000ull) | (u64)(u32)(d.out_base + (int64_t)rank);
        }
        rank0 += tot;
        __syncthreads();
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) card += (u32)__shfl_xor((int)card, off, 64);
    if (lane == 0) wsum[wave] = card;
    __syncthreads();
    if (tid == 0) {
        u64 tc = 0;
        for (int w = 0; w < kBS / 64; ++w) tc += wsum[w];
        d.res[0] = rank0;
        d.res[1] = kEmpty;
        d.res[2] = tc;
        d.res[3] = 0;
    }
    if (d.ntr_waves > 0) {                 // a new inverse level: transpose it
        const int64_t tiles = ((int64_t)rank0 + 63) / 64;
        for (int64_t wv = wave; wv < tiles * W; wv += kBS / 64) {
            const int64_t tile = wv / W;
            transpose_tile(d.out_rows, rank0, W, d.YT, d.YTt, d.Ysig, tile, (int)(wv - tile * W));
        }
    }
    __syncthreads();
    u32 nops = 0;
    const int64_t nmb = d.nXb * d.nYc;
    for (int64_t lb = 0; lb < nmb; ++lb) {
        __syncthreads();                   // the previous tiles are read
        nops += meet_w<W, true>(d, lb, lds);
    }
    return nops;
}

// blocks: one per small segment, listed in segs
__global__ void __launch_bounds__(kBS) k_step_small(const StepDesc *descs, const int32_t *segs, u64 *ops) {
    __shared__ u64 lds[kMaxW * kBS];       // expansion rows, then meet tiles
    __shared__ u32 wsum[kBS / 64];
    static_assert(kMaxW * kBS >= kMeetTileWords * 64, "meet tiles fit the expansion buffer");
    const int s = cref(segs + blockIdx.x);
    const CONST_AS StepDesc &d = cref(descs + s);
    u32 nops = 0;
    SRW_SWITCH_W(d.W, nops = step_small_w<W>(d, lds, wsum));
    if (ops) {
        u32 sum = nops;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) sum += (u32)__shfl_xor((int)sum, off, 64);
        if ((threadIdx.x & 63) == 0 && sum)
            atomicAdd((unsigned long long *)(ops + ((int64_t)(d.W - 1) * kOpsSlots + blockIdx.x % kOpsSlots) * kOpsStride),
                      (unsigned long long)sum);
    }
}

// One block runs one automaton's search step after step, choosing the side
// (smaller current list, ties forward) and building each step's descriptor
// in LDS, for as long as every step stays within what a one-block step
// handles (at most small_cand candidates, an LDS-tile meet of at most
// kSmallMeetBlocks blocks) and within the buffers the host gave it.  Each
// step is the same sequence of device functions as a one-block step launched
// by the host, so the results are those of the step-by-step search; what
// goes is the host round trip per step.  At the first step that does not fit
// the block stops, and the host goes on from the state it left (level
// offsets, row counts).
template <int W>
__device__ u32 run_small_w(const CONST_AS RunDesc &r, StepDesc &sd, u64 *lds, u32 *wsum) {
    __shared__ int64_t cs[2], cn[2], nr[2];   // current level start and size, rows stored
    __shared__ u64 ps[2];                     // cardinality sums of the current levels
    __shared__ int nl[2];                     // levels per side
    __shared__ int go, dir_s;
    RunState *st = r.st;
    const int tid = threadIdx.x;
    const u64 t_start = wall_clock64();
    int steps = 0;
    int64_t cands = 0, uniq = 0, pairs = 0;
    u32 nops = 0;
    if (tid == 0) {
        for (int s = 0; s < 2; ++s) {
            nr[s] = st->nrows[s];
            nl[s] = st->nlev[s];
            if (nl[s] == 1) {               // level 0 only: its offsets are written here
                r.off[s][0] = 0;
                r.off[s][1] = nr[s];
            }
            cs[s] = r.off[s][nl[s] - 1];
            cn[s] = nr[s] - cs[s];
            ps[s] = st->popsum[s];
        }
    }
    __syncthreads();
    for (;;) {
        if (tid == 0) {
            const int dir = cn[1] < cn[0] ? 1 : 0;
            const int64_t m = cn[dir];
            const int64_t C = m * r.k;
            const int64_t nx_ub = dir == 0 ? C : cn[0];
            const int64_t ny_ub = dir == 0 ? cn[1] : C;
            const int tpb = max(1, kMeetTileWords / W);
            const int64_t nXb = (nx_ub + kBS - 1) / kBS;
            const int64_t nYc = ((ny_ub + 63) / 64 + tpb - 1) / tpb;
            const int64_t tiles = (C + 63) / 64;
            bool ok = C <= r.small_cand && C <= r.cand_cap && nr[dir] + C <= r.rows_cap[dir] &&
                      2 * (nr[dir] + C) <= (int64_t)r.tab_mask[dir] + 1 && nl[dir] + 1 < r.max_lev &&
                      nXb * nYc <= kSmallMeetBlocks;
            if (dir == 1) ok = ok && tiles * 64 * W <= r.colT_cap && tiles * 64 <= r.ysig_cap;
            // a deadline: hand the search back to the host, which ends it
            if (r.max_ticks > 0 && (int64_t)(wall_clock64() - t_start) > r.max_ticks) ok = false;
            go = ok;
            dir_s = dir;
            if (ok) {
                StepDesc &d = sd;
                d.n = r.n;
                d.k = r.k;
                d.W = W;
                d.dir = dir;
                d.delta = r.delta;
                d.m = m;
                d.par_rows = r.rows[dir] + cs[dir] * W;
                d.C = C;
                d.cand = r.cand;
                d.cslot = r.cslot;
                d.tab = r.tab[dir];
                d.tab_mask = r.tab_mask[dir];
                d.vis_rows = r.rows[dir];
                d.ghost = nullptr;
                d.out_rows = r.rows[dir] + nr[dir] * W;
                d.out_par = r.par[dir] + nr[dir];
                d.out_base = nr[dir];
                d.YT = r.colT;
                d.YTt = r.colT + r.colT_cap;
                d.Ysig = r.ysig;
                if (dir == 0) {
                    d.X = d.out_rows;
                    d.nX = -1;
                    d.Yrows = r.rows[1] + cs[1] * W;
                    d.nY = cn[1];
                } else {
                    d.X = r.rows[0] + cs[0] * W;
                    d.nX = cn[0];
                    d.Yrows = d.out_rows;
                    d.nY = -1;
                }
                d.nXb = nXb;
                d.nYc = nYc;
                d.tpb = tpb;
                d.small = 1;
                d.ntr_waves = dir == 1 ? tiles * W : 0;
                d.meet_mode = 0;
                d.ysort = 0;
                d.Yidx = nullptr;
                d.Ycnt = nullptr;
                d.Xidx = nullptr;
                d.Xcom = nullptr;
                d.res = st->res;
            }
        }
        __syncthreads();
        if (!go) break;
        nops += step_small_w<W>(sd, lds, wsum);
        __syncthreads();
        if (tid == 0) {
            const int dir = dir_s;
            const int64_t U = (int64_t)load_slot(st->res);
            const u64 best = load_slot(st->res + 1);
            cands += sd.C;
            uniq += U;
            pairs += dir == 0 ? U * cn[1] : cn[0] * U;
            cs[dir] = nr[dir];
            cn[dir] = U;
            ps[dir] = load_slot(st->res + 2);
            nr[dir] += U;
            nl[dir] += 1;
            r.off[dir][nl[dir]] = nr[dir];
            if (dir && steps < 64 * kRunSideWords) st->sides[steps >> 6] |= 1ull << (steps & 63);
            ++steps;
            go = 1;
            if (best != kEmpty) {
                st->best = best;
                st->status = 1;
                go = 0;
            } else if (U == 0) {
                st->status = 2;
                go = 0;
            }
        }
        __syncthreads();
        if (!go) break;
    }
    if (tid == 0) {
        for (int s = 0; s < 2; ++s) {
            st->nrows[s] = nr[s];
            st->nlev[s] = nl[s];
            st->popsum[s] = ps[s];
        }
        st->steps = steps;
        st->candidates = cands;
        st->unique = uniq;
        st->pairs = pairs;
    }
    return nops;
}

// one block per automaton; one launch per set width W (all its automata)
template <int W>
__global__ void __launch_bounds__(kBS) k_run_small(const RunDesc *descs, u64 *ops) {
    __shared__ u64 lds[kMaxW * kBS];       // expansion rows, then meet tiles
    __shared__ u32 wsum[kBS / 64];
    __shared__ StepDesc sd;
    const CONST_AS RunDesc &r = cref(descs + blockIdx.x);
    const u32 nops = run_small_w<W>(r, sd, lds, wsum);
    if (ops) {
        u32 sum = nops;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) sum += (u32)__shfl_xor((int)sum, off, 64);
        if ((threadIdx.x & 63) == 0 && sum)
            atomicAdd((unsigned long long *)(ops + ((int64_t)(r.W - 1) * kOpsSlots + blockIdx.x % kOpsSlots) * kOpsStride),
                      (unsigned long long)sum);
    }
}

// ---------------------------------------------------------- beam search

__device__ __forceinline__ u32 set_card(const u64 *row, int W) {
    u32 c = 0;
    for (int w = 0; w < W; ++w) c += (u32)__popcll(row[w]);
    return c;
}

// One block runs the whole beam search of one automaton (BeamDesc).  Each
// step makes candidates -- at depth 0 the singletons (key q), later the
// preimages of the kept sets of the current level under every letter (key
// a * m + i, letter-major, as on the inverse side of the plain search) --
// and removes duplicates in the automaton's hash set with the same device
// functions as the plain search (least key among equal candidates; sets
// stored before, kept or cut, and empty sets dropped).  Then the cut: with
// U new sets and U > beam, c* is the cardinality of the beam-th largest;
// the sets above c* are kept, and those at c* in key order until the beam
// is full.  Kept sets are stored first, in key order, then the cut ones,
// and their hash slots are pointed at the stored rows.  The search stops at
// the first level that keeps Q (the full set) and traces the word back
// through the keys, at an empty level, when rows or levels run out, or at
// the deadline.
template <int W>
__device__ void beam_w(const CONST_AS BeamDesc &b, StepDesc &sd, u64 *lds, u32 *wsum, u32 *hist) {
    __shared__ int64_t s_nrows, s_start, s_m, s_U, s_K;
    __shared__ int s_nlev, s_go, s_depth;
    __shared__ u32 s_cstar, s_quota, s_qbest;
    BeamState *st = b.st;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = b.n;
    const u64 t_start = wall_clock64();
    if (tid == 0) {
        s_nrows = 0;
        s_nlev = 0;
        s_start = 0;
        s_m = 0;
        s_depth = 0;
        st->status = 0;
        st->R = -1;
        st->candidates = st->kept = st->cut = 0;
        sd.n = n;
        sd.k = b.k;
        sd.W = W;
        sd.dir = 1;
        sd.delta = b.delta;
        sd.cand = b.cand;
        sd.cslot = b.cslot;
        sd.tab = b.tab;
        sd.tab_mask = b.tab_mask;
        sd.vis_rows = b.rows;
        sd.ghost = nullptr;
    }
    __syncthreads();
    for (;;) {
        // candidates of this depth (they must fit the candidate buffer)
        if (tid == 0) {
            sd.m = s_m;
            sd.par_rows = b.rows + s_start * W;
            sd.C = s_depth == 0 ? (int64_t)n : s_m * b.k;
            s_go = sd.C <= b.cand_cap;
            if (!s_go) st->status = 3;
        }
        __syncthreads();
        if (!s_go) break;
        const int64_t C = sd.C;
        if (s_depth == 0) {
            for (int64_t g = tid; g < C; g += kBS)
                for (int w = 0; w < W; ++w)
                    b.cand[g * W + w] = (w == (int)(g >> 6)) ? 1ull << (g & 63) : 0ull;
        } else {
            const int64_t nb = (C + kBS - 1) / kBS;
            for (int64_t lb = 0; lb < nb; ++lb) expand_w<W>(sd, lb, lds);
        }
        __syncthreads();
        {
            const int64_t nb = (C + kBS - 1) / kBS;
            for (int64_t lb = 0; lb < nb; ++lb) insert_w<W>(sd, lb);
        }
        for (int c = tid; c <= n; c += kBS) hist[c] = 0;
        __syncthreads();
        // cardinalities of the new sets
        for (int64_t g = tid; g < C; g += kBS)
            if (is_winner(sd, g)) atomicAdd(&hist[set_card(b.cand + g * W, W)], 1u);
        __syncthreads();
        if (tid == 0) {
            int64_t U = 0;
            for (int c = 0; c <= n; ++c) U += hist[c];
            s_U = U;
            s_qbest = 0xFFFFFFFFu;
            if (U > b.beam) {
                int64_t above = 0;
                int c = n;
                while (above + hist[c] < b.beam) above += hist[c--];
                s_cstar = (u32)c;
                s_quota = (u32)(b.beam - above);
                s_K = b.beam;
            } else {
                s_cstar = 0;
                s_quota = 0xFFFFFFFFu;
                s_K = U;
            }
            int status = 0;
            if (U == 0) status = 2;
            else if (s_nrows + U > b.rows_cap || s_nlev + 1 >= b.max_lev) status = 3;
            else if (b.max_ticks > 0 && (int64_t)(wall_clock64() - t_start) > b.max_ticks) status = 4;
            s_go = status == 0;
            if (status) st->status = status;
            st->candidates += C;
        }
        __syncthreads();
        if (!s_go) break;
        // keep or cut every new set, in key order; store kept sets first
        const bool all = s_U <= b.beam;
        const u32 cstar = s_cstar, quota = s_quota;
        const int64_t base = s_nrows, K = s_K;
        u32 kept_run = 0, cut_run = 0, tie_run = 0;
        for (int64_t g0 = 0; g0 < C; g0 += kBS) {
            const int64_t g = g0 + tid;
            const bool f = g < C && is_winner(sd, g);
            const u32 c = f ? set_card(b.cand + g * W, W) : 0u;
            const bool tie = f && !all && c == cstar;
            const u64 tmask = __ballot(tie);
            if (lane == 0) wsum[wave] = (u32)__popcll(tmask);
            __syncthreads();
            u32 tpre = 0, ttot = 0;
#pragma unroll
            for (int w = 0; w < kBS / 64; ++w) {
                if (w < wave) tpre += wsum[w];
                ttot += wsum[w];
            }
            const bool keep = f && (all || c > cstar || (tie && tie_run + tpre + lanes_below(tmask) < quota));
            const bool cutf = f && !keep;
            const u64 kmask = __ballot(keep), cmask = __ballot(cutf);
            __syncthreads();                       // wsum is read
            if (lane == 0) {
                wsum[wave] = (u32)__popcll(kmask);
                wsum[kBS / 64 + wave] = (u32)__popcll(cmask);
            }
            __syncthreads();
            u32 kpre = 0, ktot = 0, cpre = 0, ctot = 0;
#pragma unroll
            for (int w = 0; w < kBS / 64; ++w) {
                if (w < wave) { kpre += wsum[w]; cpre += wsum[kBS / 64 + w]; }
                ktot += wsum[w];
                ctot += wsum[kBS / 64 + w];
            }
            if (f) {
                const u32 kp = kept_run + kpre + lanes_below(kmask);
                const u32 cp = cut_run + cpre + lanes_below(cmask);
                const int64_t row = keep ? base + kp : base + K + cp;
#pragma unroll
                for (int w = 0; w < W; ++w) b.rows[row * W + w] = b.cand[g * W + w];
                b.par[row] = (u32)g;
                const u32 sl = b.cslot[g];
                const u64 e = b.tab[sl];
                b.tab[sl] = (e & 0xFFFFFFFF00000000ull) | (u64)(u32)row;
                if (keep && (int)c == n) atomicMin(&s_qbest, kp);
            }
            kept_run += ktot;
            cut_run += ctot;
            tie_run += ttot;
            __syncthreads();
        }
        if (tid == 0) {
            const int L = s_nlev;
            b.lev[3 * L] = base;
            b.lev[3 * L + 1] = K;
            b.lev[3 * L + 2] = base + s_U;
            st->kept += K;
            st->cut += s_U - K;
            s_start = base;
            s_m = K;
            s_nrows = base + s_U;
            s_nlev = L + 1;
            if (s_qbest != 0xFFFFFFFFu) {
                // Q at depth L: the letters back through the keys
                int64_t j = s_qbest;
                for (int dd = L; dd > 0; --dd) {
                    const u32 g = b.par[b.lev[3 * dd] + j];
                    const int64_t m = b.lev[3 * (dd - 1) + 1];
                    b.word[L - dd] = (uint8_t)(g / m);
                    j = (int64_t)(g % m);
                }
                st->R = L;
                st->status = 1;
                s_go = 0;
            }
            s_depth = s_depth + 1;
        }
        __syncthreads();
        if (!s_go) break;
    }
    if (tid == 0) {
        st->nlev = s_nlev;
        st->nrows = s_nrows;
    }
}

// one block per automaton; one launch per set width W (all its automata)
template <int W>
__global__ void __launch_bounds__(kBS) k_beam(const BeamDesc *descs) {
    __shared__ u64 lds[kMaxW * kBS];       // expansion rows
    __shared__ u32 wsum[2 * (kBS / 64)];
    __shared__ u32 hist[kMaxW * 64 + 1];
    __shared__ StepDesc sd;
    const CONST_AS BeamDesc &b = cref(descs + blockIdx.x);
    beam_w<W>(b, sd, lds, wsum, hist);
}

// ------------------------------------------------- Eppstein's heuristic
//
// One block per automaton.  First the shortest merging length of every pair
// of states: a breadth-first search over pairs backwards from the pairs some
// letter merges, a pair {x, y} reaching distance d + 1 from {p, q} at
// distance d when delta(x, a) = p and delta(y, a) = q for a letter a (so the
// preimage lists of each letter are built first).  The distance of a pair is
// claimed once by compare-and-swap; the frontier order does not matter.
// Then each pair's first letter: the least letter taking it to a single
// state (distance 1) or to a pair one shorter.  Then the greedy rounds on
// the current set S (flags and a sorted list in LDS): the least (distance,
// p, q) over the pairs of S, a block-wide minimum; one thread walks the pair
// through its first letters, writing the round's word, in chunks that the
// other threads then apply to the states of S; S is rebuilt from the images.
constexpr int kEB = 512;                 // threads per Eppstein block (n <= 512 states, one each)
constexpr int kEppSeg = 2048;            // letters of a round applied at once
constexpr int kEppLdsDelta = 16384;      // k*n entries of delta staged in LDS when they fit

__device__ __forceinline__ u32 pair_no(u32 p, u32 q) {     // p < q
    return q * (q - 1) / 2 + p;
}
__device__ __forceinline__ void pair_of(u32 idx, u32 &p, u32 &q) {
    u32 j = (u32)((1.0f + sqrtf(1.0f + 8.0f * (float)idx)) * 0.5f);
    while (j > 1 && j * (j - 1) / 2 > idx) --j;
    while ((j + 1) * j / 2 <= idx) ++j;
    q = j;
    p = idx - j * (j - 1) / 2;
}

__global__ void __launch_bounds__(kEB) k_eppstein(const EppDesc *descs) {
    __shared__ uint16_t s_delta[kEppLdsDelta];
    __shared__ uint8_t s_in[kMaxW * 64];
    __shared__ uint16_t s_list[kMaxW * 64];
    __shared__ uint8_t s_seg[kEppSeg];
    __shared__ u64 s_wmin[kEB / 64];
    __shared__ u32 s_wcnt[kEB / 64];
    __shared__ u32 s_qlen[2];
    __shared__ u32 s_p, s_q;
    __shared__ int s_m, s_stop;
    const CONST_AS EppDesc &e = cref(descs + blockIdx.x);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = e.n, k = e.k;
    const u32 P = (u32)n * (u32)(n - 1) / 2;
    const u64 t_start = wall_clock64();
    const bool lds_delta = (int64_t)n * k <= kEppLdsDelta;
    const uint16_t *D = lds_delta ? s_delta : e.delta;
    const int K1 = n + 1;
    if (lds_delta)
        for (int t = tid; t < n * k; t += kEB) s_delta[t] = e.delta[t];
    // preimage lists: counts, offsets (one thread per letter), fill
    for (int t = tid; t < k * K1; t += kEB) e.inv_off[t] = 0;
    for (u32 t = tid; t < P; t += kEB) e.dist[t] = 0;
    if (tid == 0) {
        s_qlen[0] = 0;
        s_stop = 0;
    }
    __syncthreads();
    for (int t = tid; t < k * n; t += kEB) {
        const int a = t / n;
        atomicAdd(&e.inv_off[a * K1 + D[t] + 1], 1u);
    }
    __syncthreads();
    for (int a = tid; a < k; a += kEB) {
        u32 acc = (u32)(a * n);            // letter a's lists fill inv[a*n .. a*n + n)
        for (int t = 0; t <= n; ++t) {
            acc += e.inv_off[a * K1 + t];
            e.inv_off[a * K1 + t] = acc;
        }
    }
    __syncthreads();
    for (int t = tid; t < k * n; t += kEB) {
        const int a = t / n, x = t - a * n;
        e.inv_cur[t] = e.inv_off[a * K1 + x];
    }
    __syncthreads();
    for (int t = tid; t < k * n; t += kEB) {
        const int a = t / n, x = t - a * n;
        const u32 pos = atomicAdd(&e.inv_cur[a * n + D[t]], 1u);
        e.inv[pos] = (uint16_t)x;
    }
    // distance 1: pairs some letter merges
    for (u32 idx = tid; idx < P; idx += kEB) {
        u32 p, q;
        pair_of(idx, p, q);
        for (int a = 0; a < k; ++a)
            if (D[a * n + p] == D[a * n + q]) {
                e.dist[idx] = 1;
                e.queue[atomicAdd(&s_qlen[0], 1u)] = idx;
                break;
            }
    }
    __syncthreads();
    // the search over pairs, a level per round
    int cur = 0;
    for (u32 d = 1;; ++d) {
        const u32 len = s_qlen[cur];
        if (len == 0 || s_stop) break;
        if (tid == 0) s_qlen[cur ^ 1] = 0;
        __syncthreads();
        const u32 *in = e.queue + (size_t)cur * P;
        u32 *out = e.queue + (size_t)(cur ^ 1) * P;
        for (u32 i = tid; i < len; i += kEB) {
            u32 p, q;
            pair_of(in[i], p, q);
            for (int a = 0; a < k; ++a) {
                const u32 pb = e.inv_off[a * K1 + p], pe = e.inv_off[a * K1 + p + 1];
                const u32 qb = e.inv_off[a * K1 + q], qe = e.inv_off[a * K1 + q + 1];
                for (u32 u = pb; u < pe; ++u) {
                    const u32 x = e.inv[u];
                    for (u32 v = qb; v < qe; ++v) {
                        const u32 y = e.inv[v];
                        const u32 j = x < y ? pair_no(x, y) : pair_no(y, x);
                        if (atomicCAS(&e.dist[j], 0u, d + 1) == 0u) out[atomicAdd(&s_qlen[cur ^ 1], 1u)] = j;
                    }
                }
            }
        }
        if (tid == 0 && e.max_ticks > 0 && (int64_t)(wall_clock64() - t_start) > e.max_ticks) s_stop = 4;
        __syncthreads();
        cur ^= 1;
    }
    // first letters
    for (u32 idx = tid; idx < P && !s_stop; idx += kEB) {
        u32 p, q;
        pair_of(idx, p, q);
        const u32 d = e.dist[idx];
        uint8_t nx = 255;
        for (int a = 0; d && a < k; ++a) {
            const u32 pp = D[a * n + p], qq = D[a * n + q];
            const bool ok = pp == qq ? d == 1
                                     : e.dist[pp < qq ? pair_no(pp, qq) : pair_no(qq, pp)] + 1 == d && d > 1;
            if (ok) {
                nx = (uint8_t)a;
                break;
            }
        }
        e.next[idx] = nx;
    }
    // the greedy rounds
    if (tid < n) {
        s_in[tid] = 1;
        s_list[tid] = (uint16_t)tid;
    }
    if (tid == 0) s_m = n;
    __syncthreads();
    int64_t total = 0;
    int rounds = 0;
    while (s_m > 1 && !s_stop) {
        const u32 m = (u32)s_m;
        const u32 np = m * (m - 1) / 2;
        u64 best = ~0ull;
        for (u32 idx = tid; idx < np; idx += kEB) {
            u32 i, j;
            pair_of(idx, i, j);
            const u32 p = s_list[i], q = s_list[j];
            const u32 d = e.dist[pair_no(p, q)];
            const u64 key = ((u64)(d ? d : 0xFFFFFFFFu) << 20) | ((u64)p << 10) | q;
            best = key < best ? key : best;
        }
        for (int o = 32; o > 0; o >>= 1) {
            const u64 other = __shfl_xor(best, o, 64);
            best = other < best ? other : best;
        }
        if (lane == 0) s_wmin[wave] = best;
        __syncthreads();
        best = s_wmin[0];
        for (int w = 1; w < kEB / 64; ++w) best = s_wmin[w] < best ? s_wmin[w] : best;
        const u32 bd = (u32)(best >> 20);
        if (bd == 0xFFFFFFFFu) {
            if (tid == 0) s_stop = 5;
            __syncthreads();
            break;
        }
        if (tid == 0) {
            s_p = (u32)(best >> 10) & 1023u;
            s_q = (u32)best & 1023u;
        }
        u32 s = tid < (int)m ? s_list[tid] : 0;
        for (u32 done = 0; done < bd; done += kEppSeg) {
            const u32 c = bd - done < (u32)kEppSeg ? bd - done : (u32)kEppSeg;
            __syncthreads();
            if (tid == 0) {
                u32 p = s_p, q = s_q;
                for (u32 t = 0; t < c; ++t) {
                    // each letter shortens the pair's distance by one, so the
                    // pair stays a pair with a first letter until the last one
                    const uint8_t a = p < q ? e.next[pair_no(p, q)] : (uint8_t)255;
                    if (a >= k) {
                        s_stop = 5;
                        break;
                    }
                    s_seg[t] = a;
                    const int64_t at = total + done + t;
                    if (at < e.word_cap) e.word[at] = a;
                    const u32 pp = D[a * n + p], qq = D[a * n + q];
                    p = pp < qq ? pp : qq;
                    q = pp < qq ? qq : pp;
                }
                s_p = p;
                s_q = q;
            }
            __syncthreads();
            if (s_stop) break;
            if (tid < (int)m)
                for (u32 t = 0; t < c; ++t) s = D[s_seg[t] * n + s];
        }
        total += bd;
        ++rounds;
        __syncthreads();
        if (tid < n) s_in[tid] = 0;
        __syncthreads();
        if (tid < (int)m) s_in[s] = 1;
        __syncthreads();
        const bool f = tid < n && s_in[tid];
        const u64 bal = __ballot(f);
        if (lane == 0) s_wcnt[wave] = (u32)__popcll(bal);
        __syncthreads();
        u32 off = 0, all = 0;
        for (int w = 0; w < kEB / 64; ++w) {
            off += w < wave ? s_wcnt[w] : 0;
            all += s_wcnt[w];
        }
        if (f) s_list[off + (u32)__popcll(bal & ((1ull << lane) - 1))] = (uint16_t)tid;
        // every round merges its pair, so n - 1 rounds leave one state
        if (tid == 0 && all > 1 && rounds >= n - 1) s_stop = 5;
        if (tid == 0 && e.max_ticks > 0 && (int64_t)(wall_clock64() - t_start) > e.max_ticks) s_stop = 4;
        __syncthreads();
        if (tid == 0) s_m = (int)all;
        __syncthreads();
    }
    if (tid == 0) {
        e.st->status = s_stop ? s_stop : 1;
        e.st->rounds = rounds;
        e.st->len = total;
    }
}

// ------------------------------------------------- sort of forward levels

// zero the state histogram and the key bins
__global__ void __launch_bounds__(kBS) k_sort_zero(const SortDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS SortDesc &d = cref(descs + s);
    const int64_t e = ((int64_t)blockIdx.x - cref(pre + s)) * kBS + threadIdx.x;
    if (e < kSortBins) d.bins[e] = 0;
    else if (e < kSortBins + d.n) d.hist[e - kSortBins] = 0;
}

// how many sets of the level contain each state
__global__ void __launch_bounds__(kBS) k_sort_hist(const SortDesc *descs, const int64_t *pre, int nseg) {
    __shared__ u32 h[kMaxW * 64];
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS SortDesc &d = cref(descs + s);
    const int64_t i = ((int64_t)blockIdx.x - cref(pre + s)) * kBS + threadIdx.x;
    const int64_t cnt = (int64_t)*d.cnt;
    for (int q = threadIdx.x; q < kMaxW * 64; q += kBS) h[q] = 0;
    __syncthreads();
    if (i < cnt) {
        for (int w = 0; w < d.W; ++w) {
            u64 b = d.X[i * d.W + w];
            while (b) {
                atomicAdd(&h[64 * w + lowest_bit(b)], 1u);
                b &= b - 1;
            }
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < d.n; q += kBS)
        if (h[q]) atomicAdd(&d.hist[q], h[q]);
}

// one block per segment: the kKeyBits most frequent states (ties: lower q)
__global__ void __launch_bounds__(512) k_sort_top(const SortDesc *descs, int nseg) {
    __shared__ u32 h[kMaxW * 64];
    if ((int)blockIdx.x >= nseg) return;
    const CONST_AS SortDesc &d = cref(descs + blockIdx.x);
    const int q = threadIdx.x;
    h[q] = q < d.n ? d.hist[q] : 0u;
    __syncthreads();
    if (q < kKeyBits && q >= d.n) d.top[q] = -1;
    if (q >= d.n) return;
    const u32 c = h[q];
    int rank = 0;
    for (int o = 0; o < d.n; ++o) rank += (h[o] > c) || (h[o] == c && o < q);
    if (rank < kKeyBits) d.top[rank] = q;
}

__global__ void __launch_bounds__(kBS) k_sort_key(const SortDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS SortDesc &d = cref(descs + s);
    const int64_t i = ((int64_t)blockIdx.x - cref(pre + s)) * kBS + threadIdx.x;
    if (i >= (int64_t)*d.cnt) return;
    u32 key = 0;
    for (int r = 0; r < kKeyBits; ++r) {
        const int q = d.top[r];
        const u32 bit = q >= 0 ? (u32)((d.X[i * d.W + (q >> 6)] >> (q & 63)) & 1ull) : 0u;
        key = (key << 1) | bit;
    }
    d.keys[i] = key;
    atomicAdd(&d.bins[key], 1u);
}

// one block per segment: exclusive scan of the key bins in place.  Each of
// the 1,024 threads owns a run of 64 consecutive bins: it sums its run
// (16-byte loads), the block scans the 1,024 run sums, and each thread
// writes its run's exclusive prefixes.
constexpr int kScanThreads = 1024;
constexpr int kScanRun = kSortBins / kScanThreads;
__global__ void __launch_bounds__(kScanThreads) k_sort_scan(const SortDesc *descs, int nseg) {
    __shared__ u32 wsum[kScanThreads / 64];
    if ((int)blockIdx.x >= nseg) return;
    const CONST_AS SortDesc &d = cref(descs + blockIdx.x);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint4 *run = (uint4 *)(d.bins + (int64_t)tid * kScanRun);
    u32 sum = 0;
#pragma unroll 4
    for (int j = 0; j < kScanRun / 4; ++j) {
        const uint4 v = run[j];
        sum += v.x + v.y + v.z + v.w;
    }
    u32 incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const u32 o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    u32 acc = incl - sum;
    for (int w = 0; w < wave; ++w) acc += wsum[w];
#pragma unroll 4
    for (int j = 0; j < kScanRun / 4; ++j) {
        uint4 v = run[j];
        const uint4 o = {acc, acc + v.x, acc + v.x + v.y, acc + v.x + v.y + v.z};
        acc += v.x + v.y + v.z + v.w;
        run[j] = o;
    }
}

// place every set at its bucket (order inside a bucket is arbitrary: the
// meet keeps the original ranks, so its answer does not depend on it)
__global__ void __launch_bounds__(kBS) k_sort_scatter(const SortDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS SortDesc &d = cref(descs + s);
    const int64_t i = ((int64_t)blockIdx.x - cref(pre + s)) * kBS + threadIdx.x;
    if (i >= (int64_t)*d.cnt) return;
    const u32 pos = atomicAdd(&d.bins[d.keys[i]], 1u);
    for (int w = 0; w < d.W; ++w) d.xs_rows[(int64_t)pos * d.W + w] = d.X[i * d.W + w];
    d.xs_idx[pos] = (u32)i;
}

// AND of the 64 sorted sets of each chunk (one wave per chunk)
__global__ void __launch_bounds__(kBS) k_sort_chunk(const SortDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS SortDesc &d = cref(descs + s);
    const int64_t c = ((int64_t)blockIdx.x - cref(pre + s)) * (kBS / 64) + (threadIdx.x >> 6);
    const int64_t cnt = (int64_t)*d.cnt;
    if (c * 64 >= cnt) return;                     // whole wave
    const int lane = threadIdx.x & 63;
    const int64_t i = c * 64 + lane;
    for (int w = 0; w < d.W; ++w) {
        u64 v = i < cnt ? d.xs_rows[i * d.W + w] : ~0ull;
        u32 lo = (u32)v, hi = (u32)(v >> 32);
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            lo &= (u32)__shfl_xor((int)lo, off, 64);
            hi &= (u32)__shfl_xor((int)hi, off, 64);
        }
        if (lane == 0) d.xs_common[c * d.W + w] = ((u64)hi << 32) | lo;
    }
}

// ------------------------------------------------------- init / rehash

// level 0 of both sides: Q forward, the n singletons inverse (Alg. 1 init)
__global__ void __launch_bounds__(kBS) k_init(const InitDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS InitDesc &d = cref(descs + s);
    const int64_t q = ((int64_t)blockIdx.x - cref(pre + s)) * kBS + threadIdx.x;
    if (q > d.n) return;
    const int W = d.W;
    if (q < d.n)
        for (int a = 0; a < d.k; ++a) d.delta[(int64_t)a * d.n + q] = d.delta_src[(int64_t)a * d.n + q];
    if (q == d.n) {
        for (int w = 0; w < W; ++w) {
            const int lo = 64 * w;
            const int cnt = d.n - lo >= 64 ? 64 : d.n - lo;
            d.rows_f[w] = cnt >= 64 ? ~0ull : ((1ull << cnt) - 1ull);
        }
        d.par_f[0] = kDrop;
        return;
    }
    for (int w = 0; w < W; ++w) d.rows_b[q * W + w] = (w == (q >> 6)) ? (1ull << (q & 63)) : 0ull;
    d.par_b[q] = kDrop;
}

template <int W>
__device__ void rehash_w(const CONST_AS RehashDesc &d, int64_t id) {
    u64 x[W];
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = d.rows[id * W + w];
    const u64 h = set_hash<W>(x);
    const u64 e = (h & 0xFFFFFFFF00000000ull) | (u64)((u32)id | (u32)d.ref_or);
    u64 pos = h & d.tab_mask;
    for (;;) {
        if (load_slot(&d.tab[pos]) == kEmpty && atomicCAS(&d.tab[pos], kEmpty, e) == kEmpty) return;
        pos = (pos + 1) & d.tab_mask;
    }
}

// stored rows are pairwise distinct, so each just needs a free slot
__global__ void __launch_bounds__(kBS) k_rehash(const RehashDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS RehashDesc &d = cref(descs + s);
    const int64_t id = ((int64_t)blockIdx.x - cref(pre + s)) * kBS + threadIdx.x;
    if (id >= d.count) return;
    SRW_SWITCH_W(d.W, rehash_w<W>(d, id));
}

// mark every slot of each segment's (new) hash table free
__global__ void __launch_bounds__(kBS) k_clear_tables(const RehashDesc *descs, const int64_t *pre, int nseg) {
    const int s = find_seg(pre, nseg, blockIdx.x);
    const CONST_AS RehashDesc &d = cref(descs + s);
    const int64_t e = ((int64_t)blockIdx.x - cref(pre + s)) * kBS + threadIdx.x;
    if (e <= (int64_t)d.tab_mask) d.tab[e] = kEmpty;
}

__global__ void __launch_bounds__(kBS) k_fill(u64 *p, int64_t count, u64 v) {
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kBS;
    for (int64_t e = i; e < count; e += stride) p[e] = v;
}

// ------------------------------------------------------------- traceback

// Forward key g = i*k + a: parent i = g / k, letter a = g % k (word position
// L-1).  Inverse key g = a*|L_prev| + i: letter a is the next letter of the
// inverse half, read from its last level down.
__global__ void k_trace(const TraceDesc *descs, int count) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const CONST_AS TraceDesc &d = cref(descs + t);
    int64_t i = d.i;
    for (int L = d.f; L > 0; --L) {
        const u32 g = d.par_f[d.off_f[L] + i];
        d.out[L - 1] = (uint8_t)(g % (u32)d.k);
        i = g / (u32)d.k;
    }
    int64_t j = d.j;
    for (int L = d.b, pos = 0; L > 0; --L, ++pos) {
        const u32 g = d.par_b[d.off_b[L] + j];
        const int64_t prev = d.off_b[L] - d.off_b[L - 1];
        d.out[d.f + pos] = (uint8_t)((int64_t)g / prev);
        j = (int64_t)g % prev;
    }
}

// ------------------------------------------------------------- launchers

static inline hipError_t launch_checked() { return hipGetLastError(); }

// cardinality order of the new inverse levels of the segments with ysort set;
// pre: blocks of kBS sets per such segment
hipError_t launch_ysort(const StepDesc *d, const int64_t *pre, int nseg, int64_t blocks, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ysort_zero, dim3((unsigned)nseg), dim3(kBS), 0, st, d, nseg);
    hipLaunchKernelGGL(k_ysort_hist, dim3((unsigned)blocks), dim3(kBS), 0, st, d, pre, nseg);
    hipLaunchKernelGGL(k_ysort_scan, dim3((unsigned)nseg), dim3(kBS), 0, st, d, nseg);
    hipLaunchKernelGGL(k_ysort_scatter, dim3((unsigned)blocks), dim3(kBS), 0, st, d, pre, nseg);
    return launch_checked();
}
hipError_t launch_copy(const CopyDesc *d, const int64_t *pre, int nseg, int64_t blocks, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(kBS), 0, st, d, pre, nseg);
    return launch_checked();
}
// count automata, all with W words per set
hipError_t launch_run_small(const RunDesc *d, int count, int W, u64 *ops, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    SRW_SWITCH_W(W, hipLaunchKernelGGL(k_run_small<W>, dim3((unsigned)count), dim3(kBS), 0, st, d, ops));
    return launch_checked();
}
// pe: block prefix of ceil(C / kBS) per segment (marks, copy); pc: the
// compaction grid (ceil(C / kCB) per segment)
hipError_t launch_reduce(const StepDesc *d, const int64_t *pe, const int64_t *pc, int nseg, int64_t be,
                         int64_t bc, u32 *cnt, u32 *off, hipStream_t st) {
    if (nseg <= 0) return hipSuccess;
    if (be > 0) hipLaunchKernelGGL(k_red_mark, dim3((unsigned)be), dim3(kBS), 0, st, d, pe, nseg);
    if (bc > 0) hipLaunchKernelGGL(k_red_count, dim3((unsigned)bc), dim3(kBS), 0, st, d, pc, nseg, cnt);
    hipLaunchKernelGGL(k_red_scan, dim3((unsigned)nseg), dim3(kBS), 0, st, d, nseg, cnt, off);
    if (bc > 0) hipLaunchKernelGGL(k_red_compact, dim3((unsigned)bc), dim3(kBS), 0, st, d, pc, nseg, off);
    if (be > 0) hipLaunchKernelGGL(k_red_copy, dim3((unsigned)be), dim3(kBS), 0, st, d, pe, nseg);
    return launch_checked();
}
// count automata, all with W words per set
hipError_t launch_beam(const BeamDesc *d, int count, int W, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    SRW_SWITCH_W(W, hipLaunchKernelGGL(k_beam<W>, dim3((unsigned)count), dim3(kBS), 0, st, d));
    return launch_checked();
}
// count automata, a block each
hipError_t launch_eppstein(const EppDesc *d, int count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eppstein, dim3((unsigned)count), dim3(kEB), 0, st, d);
    return launch_checked();
}
hipError_t launch_step_small(const StepDesc *d, const int32_t *segs, int count, u64 *ops, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_step_small, dim3((unsigned)count), dim3(kBS), 0, st, d, segs, ops);
    return launch_checked();
}
hipError_t launch_expand(const StepDesc *d, const int64_t *pre, int nseg, int64_t blocks, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_expand, dim3((unsigned)blocks), dim3(kBS), 0, st, d, pre, nseg);
    return launch_checked();
}
hipError_t launch_insert(const StepDesc *d, const int64_t *pre, int nseg, int64_t blocks, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_insert, dim3((unsigned)blocks), dim3(kBS), 0, st, d, pre, nseg);
    return launch_checked();
}
hipError_t launch_count(const StepDesc *d, const int64_t *pre, int nseg, int64_t blocks, u32 *cnt,
                        hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count, dim3((unsigned)blocks), dim3(kBS), 0, st, d, pre, nseg, cnt);
    return launch_checked();
}
hipError_t launch_scan(const StepDesc *d, int nseg, const u32 *cnt, u32 *off, hipStream_t st) {
    if (nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan, dim3((unsigned)nseg), dim3(kBS), 0, st, d, nseg, cnt, off);
    return launch_checked();
}
hipError_t launch_compact(const StepDesc *d, const int64_t *pre, int nseg, int64_t blocks,
                          const u32 *off, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact, dim3((unsigned)blocks), dim3(kBS), 0, st, d, pre, nseg, off);
    return launch_checked();
}
hipError_t launch_transpose(const StepDesc *d, const int64_t *pre, int nseg, int64_t blocks,
                            hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_transpose, dim3((unsigned)blocks), dim3(kBS), 0, st, d, pre, nseg);
    return launch_checked();
}
hipError_t launch_transpose_rows(const TransposeDesc *d, const int64_t *pre, int nseg, int64_t blocks,
                                 hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_transpose_rows, dim3((unsigned)blocks), dim3(kBS), 0, st, d, pre, nseg);
    return launch_checked();
}
// segments s0..s1-1 all have width W; `items` = cref(pre + s1) - cref(pre + s0).  At most
// max_grid blocks (each then loops over several items); short-lived blocks
// let kernels of other streams onto the GPU between them.
// ys: some segment of the launch has its inverse level in cardinality order
hipError_t launch_meet(const StepDesc *d, const int64_t *pre, int s0, int s1, int W, int64_t items,
                       int64_t max_grid, bool ys, u64 *ops, hipStream_t st) {
    if (items <= 0) return hipSuccess;
    const int64_t cap = max_grid > 0 ? std::min<int64_t>(max_grid, kMeetMaxGrid) : kMeetMaxGrid;
    const unsigned grid = (unsigned)(items < cap ? items : cap);
    // the counting kernels only when the operations are counted
    if (ys && ops) {
        SRW_SWITCH_W(W, hipLaunchKernelGGL((k_meet<W, true, true>), dim3(grid), dim3(kBS), 0, st, d, pre, s0, s1, ops));
    } else if (ys) {
        SRW_SWITCH_W(W, hipLaunchKernelGGL((k_meet<W, true, false>), dim3(grid), dim3(kBS), 0, st, d, pre, s0, s1, ops));
    } else if (ops) {
        SRW_SWITCH_W(W, hipLaunchKernelGGL((k_meet<W, false, true>), dim3(grid), dim3(kBS), 0, st, d, pre, s0, s1, ops));
    } else {
        SRW_SWITCH_W(W, hipLaunchKernelGGL((k_meet<W, false, false>), dim3(grid), dim3(kBS), 0, st, d, pre, s0, s1, ops));
    }
    return launch_checked();
}
// sort pipeline: pre[0..4] are the block prefixes of zero, hist (= key =
// scatter, rows), chunk; the top and scan kernels take one block per segment
hipError_t launch_sort(const SortDesc *d, const int64_t *const pre[3], const int64_t blocks[3], int nseg,
                       hipStream_t st) {
    if (nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sort_zero, dim3((unsigned)blocks[0]), dim3(kBS), 0, st, d, pre[0], nseg);
    hipLaunchKernelGGL(k_sort_hist, dim3((unsigned)blocks[1]), dim3(kBS), 0, st, d, pre[1], nseg);
    hipLaunchKernelGGL(k_sort_top, dim3((unsigned)nseg), dim3(512), 0, st, d, nseg);
    hipLaunchKernelGGL(k_sort_key, dim3((unsigned)blocks[1]), dim3(kBS), 0, st, d, pre[1], nseg);
    hipLaunchKernelGGL(k_sort_scan, dim3((unsigned)nseg), dim3(kScanThreads), 0, st, d, nseg);
    hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)blocks[1]), dim3(kBS), 0, st, d, pre[1], nseg);
    if (blocks[2] > 0)
        hipLaunchKernelGGL(k_sort_chunk, dim3((unsigned)blocks[2]), dim3(kBS), 0, st, d, pre[2], nseg);
    return launch_checked();
}

// buckets of inverse levels: pre[0] blocks over sets (count_ub), pre[1]
// over padded positions (nt_ub * 64), pre[2] waves over buckets, pre[3]
// waves over (tile, word) pairs
hipError_t launch_ybin(const YbDesc *d, const int64_t *const pre[4], const int64_t blocks[4], int nseg,
                       hipStream_t st) {
    if (nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_yb_zero, dim3((unsigned)nseg), dim3(kBS), 0, st, d, nseg);
    if (blocks[0] > 0) hipLaunchKernelGGL(k_yb_hist, dim3((unsigned)blocks[0]), dim3(kBS), 0, st, d, pre[0], nseg);
    hipLaunchKernelGGL(k_yb_scan, dim3((unsigned)nseg), dim3(kBS), 0, st, d, nseg);
    if (blocks[1] > 0) hipLaunchKernelGGL(k_yb_fill, dim3((unsigned)blocks[1]), dim3(kBS), 0, st, d, pre[1], nseg);
    if (blocks[0] > 0) hipLaunchKernelGGL(k_yb_scatter, dim3((unsigned)blocks[0]), dim3(kBS), 0, st, d, pre[0], nseg);
    if (blocks[2] > 0) hipLaunchKernelGGL(k_yb_list, dim3((unsigned)blocks[2]), dim3(kBS), 0, st, d, pre[2], nseg);
    if (blocks[3] > 0) hipLaunchKernelGGL(k_yb_transpose, dim3((unsigned)blocks[3]), dim3(kBS), 0, st, d, pre[3], nseg);
    return launch_checked();
}
// plan of the mode-2 meets: pre = blocks over chunks per segment
hipError_t launch_meet_plan(const StepDesc *d, const int64_t *pre, int nseg, int64_t blocks, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mp_zero, dim3((unsigned)nseg), dim3(kBS), 0, st, d, nseg);
    hipLaunchKernelGGL(k_mp_keys, dim3((unsigned)blocks), dim3(kBS), 0, st, d, pre, nseg);
    hipLaunchKernelGGL(k_mp_scan, dim3((unsigned)nseg), dim3(kMpThreads), 0, st, d, nseg);
    hipLaunchKernelGGL(k_mp_scatter, dim3((unsigned)blocks), dim3(kBS), 0, st, d, pre, nseg);
    return launch_checked();
}
// mode-2 meets of segments s0..s1-1 (width W), `grid` blocks
hipError_t launch_meet_b(const StepDesc *d, int s0, int s1, int W, int64_t grid, u64 *ops, hipStream_t st) {
    if (grid <= 0 || s1 <= s0) return hipSuccess;
    if (ops) {
        SRW_SWITCH_W(W, hipLaunchKernelGGL((k_meet_b<W, true>), dim3((unsigned)grid), dim3(kBS), 0, st, d, s0, s1, ops));
    } else {
        SRW_SWITCH_W(W, hipLaunchKernelGGL((k_meet_b<W, false>), dim3((unsigned)grid), dim3(kBS), 0, st, d, s0, s1, ops));
    }
    return launch_checked();
}

hipError_t launch_init(const InitDesc *d, const int64_t *pre, int nseg, int64_t blocks, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(kBS), 0, st, d, pre, nseg);
    return launch_checked();
}
hipError_t launch_rehash(const RehashDesc *d, const int64_t *pre, int nseg, int64_t blocks, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rehash, dim3((unsigned)blocks), dim3(kBS), 0, st, d, pre, nseg);
    return launch_checked();
}
// pre: block prefix of ceil(capacity / kBS) per table
hipError_t launch_clear_tables(const RehashDesc *d, const int64_t *pre, int nseg, int64_t blocks,
                               hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear_tables, dim3((unsigned)blocks), dim3(kBS), 0, st, d, pre, nseg);
    return launch_checked();
}

hipError_t launch_fill(u64 *p, int64_t count, u64 v, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + kBS - 1) / kBS;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(kBS), 0, st, p, count, v);
    return launch_checked();
}
hipError_t launch_trace(const TraceDesc *d, int count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_trace, dim3((unsigned)((count + 63) / 64)), dim3(64), 0, st, d, count);
    return launch_checked();
}

}  // namespace srw
