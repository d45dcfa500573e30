// srw_engine.hip -- host side of libsrw: the C ABI, the step orchestration
// of the bidirectional breadth-first search, device memory and serving.
//
// Paper: Szykula & Zyzik, "An Improved Algorithm for Finding the Shortest
// Synchronizing Words".  The search loop follows Alg. 1 in its plain
// variant; see include/srw.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/srw.h"
#include "srw_device.h"

namespace srw {

hipError_t launch_expand(const StepDesc *, const int64_t *, int, int64_t, hipStream_t);
hipError_t launch_insert(const StepDesc *, const int64_t *, int, int64_t, hipStream_t);
hipError_t launch_count(const StepDesc *, const int64_t *, int, int64_t, u32 *, hipStream_t);
hipError_t launch_scan(const StepDesc *, int, const u32 *, u32 *, hipStream_t);
hipError_t launch_compact(const StepDesc *, const int64_t *, int, int64_t, const u32 *, hipStream_t);
hipError_t launch_transpose(const StepDesc *, const int64_t *, int, int64_t, hipStream_t);
hipError_t launch_transpose_rows(const TransposeDesc *, const int64_t *, int, int64_t, hipStream_t);
hipError_t launch_meet(const StepDesc *, const int64_t *, int, int, int, int64_t, int64_t, bool, u64 *, hipStream_t);
hipError_t launch_step_small(const StepDesc *, const int32_t *, int, u64 *, hipStream_t);
hipError_t launch_run_small(const RunDesc *, int, int, u64 *, hipStream_t);
hipError_t launch_ybin(const YbDesc *, const int64_t *const[4], const int64_t[4], int, hipStream_t);
hipError_t launch_meet_plan(const StepDesc *, const int64_t *, int, int64_t, hipStream_t);
hipError_t launch_meet_b(const StepDesc *, int, int, int, int64_t, u64 *, hipStream_t);
hipError_t launch_copy(const CopyDesc *, const int64_t *, int, int64_t, hipStream_t);
hipError_t launch_ysort(const StepDesc *, const int64_t *, int, int64_t, hipStream_t);
hipError_t launch_init(const InitDesc *, const int64_t *, int, int64_t, hipStream_t);
hipError_t launch_rehash(const RehashDesc *, const int64_t *, int, int64_t, hipStream_t);
hipError_t launch_fill(u64 *, int64_t, u64, hipStream_t);
hipError_t launch_clear_tables(const RehashDesc *, const int64_t *, int, int64_t, hipStream_t);
hipError_t launch_trace(const TraceDesc *, int, hipStream_t);
hipError_t launch_beam(const BeamDesc *, int, int, hipStream_t);
hipError_t launch_eppstein(const EppDesc *, int, hipStream_t);
hipError_t launch_reduce(const StepDesc *, const int64_t *, const int64_t *, int, int64_t, int64_t, u32 *, u32 *,
                         hipStream_t);
hipError_t launch_sort(const SortDesc *, const int64_t *const[3], const int64_t[3], int, hipStream_t);

// ------------------------------------------------------------------ errors

static thread_local std::string t_err;

struct HipFailure {
    hipError_t e;
    std::string where;
};

static int set_error(int code, const std::string &msg) {
    t_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) throw HipFailure{e_, std::string(#expr) + " @" +          \
                                                      std::to_string(__LINE__)};        \
    } while (0)

static double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------ host checks

static int check_input(int32_t n, int32_t k, const int32_t *delta) {
    if (!delta) return set_error(SRW_EINVAL, "delta is NULL");
    if (n < 1 || k < 1 || k > 255) return set_error(SRW_EINVAL, "n or k out of range");
    if (n > SRW_MAX_N) return set_error(SRW_EUNSUPPORTED, "n exceeds SRW_MAX_N");
    for (int64_t i = 0; i < (int64_t)n * k; ++i)
        if (delta[i] < 0 || delta[i] >= n) return set_error(SRW_EINVAL, "delta entry outside [0,n)");
    return SRW_OK;
}

// Pair test: every pair {p,q} must be mergeable (Section 2 intro).  Backward
// search in the pair automaton from the diagonal, O(k n^2).
// A word that maps Q to a single state proves the automaton synchronizing
// (Section 1).  Greedy: each step applies the letter with the smallest image
// of the current set (ties: the least letter), a pseudo-random letter
// (xorshift64) when none shrinks it, within a budget of state visits; false
// when no such word turned up (then the pair test decides).
static bool reset_witness(int n, int k, const int32_t *delta) {
    std::vector<int32_t> S(n), T(n);
    std::vector<uint32_t> stamp(n, 0u);
    uint32_t tick = 0;
    for (int q = 0; q < n; ++q) S[q] = q;
    int m = n;
    uint64_t rng = 0x9E3779B97F4A7C15ull;
    int64_t budget = 16 * (int64_t)n * (k + 1) + 4096;
    while (m > 1 && budget > 0) {
        int best = -1, best_c = m;
        for (int a = 0; a < k; ++a) {
            const int32_t *da = delta + (size_t)a * n;
            ++tick;
            int c = 0;
            for (int i = 0; i < m; ++i) {
                const int t = da[S[(size_t)i]];
                if (stamp[(size_t)t] != tick) {
                    stamp[(size_t)t] = tick;
                    ++c;
                }
            }
            budget -= m;
            if (c < best_c) {
                best_c = c;
                best = a;
            }
        }
        if (best < 0) {
            rng ^= rng << 13;
            rng ^= rng >> 7;
            rng ^= rng << 17;
            best = (int)(rng % (uint64_t)k);
        }
        const int a = best;
        const int32_t *da = delta + (size_t)a * n;
        ++tick;
        int c = 0;
        for (int i = 0; i < m; ++i) {
            const int t = da[S[(size_t)i]];
            if (stamp[(size_t)t] != tick) {
                stamp[(size_t)t] = tick;
                T[(size_t)c++] = t;
            }
        }
        budget -= m;
        S.swap(T);
        m = c;
    }
    return m == 1;
}

static bool is_synchronizing(int n, int k, const int32_t *delta) {
    if (n == 1) return true;
    if (reset_witness(n, k, delta)) return true;
    // preimage lists of every letter
    std::vector<int> start((size_t)k * (n + 1), 0), list((size_t)k * n);
    for (int a = 0; a < k; ++a) {
        int *st = &start[(size_t)a * (n + 1)];
        for (int q = 0; q < n; ++q) st[delta[(size_t)a * n + q] + 1]++;
        for (int t = 0; t < n; ++t) st[t + 1] += st[t];
        std::vector<int> fillp(st, st + n);
        for (int q = 0; q < n; ++q) list[(size_t)a * n + fillp[delta[(size_t)a * n + q]]++] = q;
    }
    // unordered pairs {p, q}, p < q, that some word merges: a search
    // backwards from the single states, a pair {x, y} joining when a letter
    // takes it to a merged pair or a single state
    std::vector<uint64_t> merged(((size_t)n * n + 63) / 64, 0);   // bit p*n + q
    std::vector<int32_t> queue;
    queue.reserve((size_t)n * (n + 1));
    for (int p = 0; p < n; ++p) {
        queue.push_back(p);
        queue.push_back(p);
    }
    int64_t count = 0;
    const int64_t want = (int64_t)n * (n - 1) / 2;
    for (size_t h = 0; h < queue.size() && count < want; h += 2) {
        const int s = queue[h], t = queue[h + 1];
        for (int a = 0; a < k; ++a) {
            const int *st = &start[(size_t)a * (n + 1)];
            const int *ls = &list[(size_t)a * n];
            for (int x = st[s]; x < st[s + 1]; ++x)
                for (int y = s == t ? x + 1 : st[t]; y < st[t + 1]; ++y) {
                    const int p = std::min(ls[x], ls[y]), q = std::max(ls[x], ls[y]);
                    const size_t bit = (size_t)p * n + q;
                    uint64_t &m = merged[bit >> 6];
                    if (!(m >> (bit & 63) & 1)) {
                        m |= 1ull << (bit & 63);
                        ++count;
                        queue.push_back(p);
                        queue.push_back(q);
                    }
                }
        }
    }
    return count == want;
}

// check_input and is_synchronizing of every automaton of a batch, on up to
// 16 host threads: rc[i] = 0, an input error or SRW_ENOTSYNC
// fn(i) for i in [0, count) on up to 16 host threads (one when `work`, a
// rough operation count, is small)
template <class F>
static void parallel_for(int64_t count, int64_t work, F &&fn) {
    const int hw = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const int nt = (int)std::min<int64_t>(std::min<int64_t>(hw, count), std::max<int64_t>(1, work / 200000));
    if (nt <= 1) {
        for (int64_t i = 0; i < count; ++i) fn(i);
        return;
    }
    std::atomic<int64_t> next{0};
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&] {
            for (int64_t i; (i = next.fetch_add(1)) < count;) fn(i);
        });
    for (auto &x : th) x.join();
}

// (without `sync`, check_input only)
static void host_checks(int32_t count, const int32_t *n, const int32_t *k, const int64_t *delta_off,
                        const int32_t *delta, std::vector<int> &rc, bool sync = true) {
    rc.assign((size_t)std::max(count, 0), 0);
    auto one = [&](int32_t i) {
        const int32_t *d = delta + delta_off[i];
        int c = check_input(n[i], k[i], d);
        if (!c && sync && !is_synchronizing(n[i], k[i], d)) c = SRW_ENOTSYNC;
        rc[(size_t)i] = c;
    };
    int64_t work = 0;
    if (sync)
        for (int32_t i = 0; i < count; ++i) work += (int64_t)n[i] * n[i] * std::max(1, k[i]);
    parallel_for(count, work, [&](int64_t i) { one((int32_t)i); });
}

static bool verify_word(int n, int k, const int32_t *delta, const uint8_t *w, int64_t len) {
    std::vector<uint8_t> cur(n, 1), nxt(n);
    for (int64_t i = 0; i < len; ++i) {
        if (w[i] >= k) return false;
        std::fill(nxt.begin(), nxt.end(), 0);
        const int32_t *da = delta + (size_t)w[i] * n;
        for (int q = 0; q < n; ++q)
            if (cur[q]) nxt[da[q]] = 1;
        cur.swap(nxt);
    }
    int c = 0;
    for (int q = 0; q < n; ++q) c += cur[q];
    return c == 1;
}

// ------------------------------------------------------------- memory pool

struct Backing {
    void *(*alloc)(size_t, void *) = nullptr;
    void (*free)(void *, void *) = nullptr;
    void *ctx = nullptr;
    bool own_stream_only = false;   // the memory is used on the engine's stream alone
};

// Power-of-two size classes.  Blocks up to 4 MiB are carved from slabs of
// up to 64 MiB; larger ones are separate backing allocations.  Freed blocks are
// cached per class and reused; everything returns to the backing allocator
// when the pool is destroyed.  `budget` caps the bytes taken from backing.
// The search's own buffers may take all but `reserve` bytes of it; the
// engine's small per-step buffers (descriptors, results, counters) may use
// the reserve too, so that a search that fills its share of the budget ends
// in SRW_ENOMEM for that search instead of failing the step of every other.
// Every block is used on stream `st`: before a block goes back to the
// backing allocator, the stream is drained, and after an external
// allocator hands over a block, the stream waits for the legacy default
// stream (on which such an allocator may still have work queued).
class Pool {
  public:
    Pool(Backing b, int64_t budget, hipStream_t st) : b_(b), budget_(budget), st_(st) {
        if (b_.alloc && !b_.own_stream_only) HIPCHK(hipEventCreateWithFlags(&ev_ext_, hipEventDisableTiming));
    }
    ~Pool() {
        if (!chunks_.empty()) (void)hipStreamSynchronize(st_);
        for (auto &c : chunks_) backing_free(c.first);
        if (ev_ext_) (void)hipEventDestroy(ev_ext_);
    }
    void *alloc(size_t bytes, bool internal = false) {
        const int c = cls_of(bytes);
        const size_t size = (size_t)256 << c;
        if (!free_[c].empty()) {
            // a cached block counts against the budget as well (it may have
            // been cut since the block was reserved)
            if (in_use_ + (int64_t)size > budget_ - (internal ? 0 : reserve())) return nullptr;
            void *p = free_[c].back();
            free_[c].pop_back();
            account(size);
            return p;
        }
        void *p = nullptr;
        if (size <= kSmallMax) {
            if (slab_left_ < size) {
                const size_t sl = slab_bytes();
                char *s = (char *)backing_alloc(sl, internal);
                if (!s) {
                    trim();
                    s = (char *)backing_alloc(sl, internal);
                    if (!s) return nullptr;
                }
                slab_ = s;
                slab_left_ = sl;
            }
            p = slab_;
            slab_ += size;
            slab_left_ -= size;
        } else {
            p = backing_alloc(size, internal);
            if (!p) {
                trim();
                p = backing_alloc(size, internal);
                if (!p) return nullptr;
            }
            big_.insert({p, size});
        }
        cls_[p] = c;
        account(size);
        return p;
    }
    void free(void *p) {
        if (!p) return;
        auto it = cls_.find(p);
        if (it == cls_.end()) return;
        free_[it->second].push_back(p);
        in_use_ -= (int64_t)256 << it->second;
    }
    int64_t reserved() const { return reserved_; }
    int64_t in_use() const { return in_use_; }
    // bytes of the pool block at p (0 for NULL or a foreign pointer)
    int64_t size_of(const void *p) const {
        auto it = cls_.find(const_cast<void *>(p));
        return it == cls_.end() ? 0 : (int64_t)256 << it->second;
    }
    int64_t peak() const { return peak_; }
    int64_t budget() const { return budget_; }
    void set_budget(int64_t b) {
        budget_ = b;
        if (reserved_ > budget_) trim();   // cached blocks beyond a cut budget go back
    }
    // bytes of the budget kept for the engine's own per-step buffers
    int64_t reserve() const { return std::min<int64_t>(kReserve, budget_ / 4); }
    // slabs of at most 64 MiB, and at most an eighth of the budget (a small
    // budget must still hold several of them), but never below the largest
    // block they serve
    size_t slab_bytes() const {
        return std::max(kSmallMax, std::min(kSlab, (size_t)std::max<int64_t>(budget_ / 8, 0) & ~(size_t)4095));
    }

  private:
    static int cls_of(size_t bytes) {
        int c = 0;
        size_t s = 256;
        while (s < bytes) { s <<= 1; ++c; }
        return c;
    }
    void account(size_t size) {
        in_use_ += (int64_t)size;
        peak_ = std::max(peak_, in_use_);
    }
    void *backing_alloc(size_t bytes, bool internal) {
        if (reserved_ + (int64_t)bytes > budget_ - (internal ? 0 : reserve())) return nullptr;
        void *p = nullptr;
        if (b_.alloc) {
            p = b_.alloc(bytes, b_.ctx);
            if (!p) return nullptr;
            if (ev_ext_) {
                HIPCHK(hipEventRecord(ev_ext_, nullptr));
                HIPCHK(hipStreamWaitEvent(st_, ev_ext_, 0));
            }
        } else {
            if (hipMalloc(&p, bytes) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
        }
        reserved_ += (int64_t)bytes;
        chunks_.push_back({p, bytes});
        return p;
    }
    void backing_free(void *p) {
        if (b_.free) b_.free(p, b_.ctx);
        else (void)hipFree(p);
    }
    // hand cached large blocks back to the backing allocator, once the
    // stream is done with them
    void trim() {
        bool any = false;
        for (int c = 0; c < 48; ++c)
            if ((size_t)256 << c > kSmallMax && !free_[c].empty()) any = true;
        if (!any) return;
        HIPCHK(hipStreamSynchronize(st_));
        for (int c = 0; c < 48; ++c) {
            const size_t size = (size_t)256 << c;
            if (size <= kSmallMax) continue;
            for (void *p : free_[c]) {
                backing_free(p);
                reserved_ -= (int64_t)size;
                cls_.erase(p);
                big_.erase(p);
                for (size_t i = 0; i < chunks_.size(); ++i)
                    if (chunks_[i].first == p) {
                        chunks_[i] = chunks_.back();
                        chunks_.pop_back();
                        break;
                    }
            }
            free_[c].clear();
        }
    }
    static constexpr size_t kSlab = (size_t)64 << 20;
    static constexpr size_t kSmallMax = (size_t)4 << 20;
    static constexpr int64_t kReserve = (int64_t)128 << 20;
    Backing b_;
    int64_t budget_, reserved_ = 0, in_use_ = 0, peak_ = 0;
    hipStream_t st_;
    hipEvent_t ev_ext_ = nullptr;
    std::vector<void *> free_[48];
    std::unordered_map<void *, int> cls_;
    std::unordered_map<void *, size_t> big_;
    std::vector<std::pair<void *, size_t>> chunks_;
    char *slab_ = nullptr;
    size_t slab_left_ = 0;
};

// pinned host buffer that only grows.  With `pageable` set (an engine that
// may not allocate device or pinned memory) it is ordinary host memory, and
// the next user waits for the whole stream instead of an event.
struct Pinned {
    void *p = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;     // recorded after the last copy that reads the buffer
    bool pageable = false;
    std::vector<char> host;
    hipStream_t last = nullptr;  // pageable: the stream of the last copy out of it
    // the buffer, once the last copy out of it has been done
    void *acquire(size_t bytes) {
        if (pageable) {
            if (last) HIPCHK(hipStreamSynchronize(last));
            last = nullptr;
            return need(bytes);
        }
        if (ev) HIPCHK(hipEventSynchronize(ev));
        return need(bytes);
    }
    // a copy out of the buffer has been enqueued on `st`
    void issued(hipStream_t st) {
        if (pageable) {
            last = st;
            return;
        }
        if (!ev) HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIPCHK(hipEventRecord(ev, st));
    }
    void *need(size_t bytes) {
        if (pageable) {
            if (bytes > host.size()) host.resize(std::max(std::max(bytes, 2 * host.size()), (size_t)1 << 16));
            return host.data();
        }
        if (bytes > cap) {
            if (p) (void)hipHostFree(p);
            p = nullptr;
            size_t nc = std::max(bytes, cap * 2);
            nc = std::max(nc, (size_t)1 << 16);
            HIPCHK(hipHostMalloc(&p, nc, hipHostMallocDefault));
            cap = nc;
        }
        return p;
    }
    ~Pinned() {
        if (ev) (void)hipEventSynchronize(ev);
        if (p) (void)hipHostFree(p);
        if (ev) (void)hipEventDestroy(ev);
    }
};

// --------------------------------------------------------------- problem

struct SideState {
    u64 *rows = nullptr;     // every visited set of the side, level by level
    u32 *par = nullptr;      // parent key per row
    int64_t cap = 0;         // rows of capacity
    u64 *tab = nullptr;      // visited hash set
    int64_t tab_cap = 0;     // slots (power of two)
    int64_t nrows = 0;
    std::vector<int64_t> off;  // level L: rows off[L] .. off[L+1]-1
    u64 popsum = 0;            // sum of the cardinalities of the current level's sets
    u64 *ghost = nullptr;      // sets dropped by the self-reduction (they stay visited)
    int64_t ghost_cap = 0, nghost = 0;
    int nlev() const { return (int)off.size() - 1; }
    int64_t cur() const { return off[off.size() - 1] - off[off.size() - 2]; }
    int64_t cur_start() const { return off[off.size() - 2]; }
    int64_t prev() const { return off.size() >= 3 ? off[off.size() - 2] - off[off.size() - 3] : 0; }
};

struct Problem {
    int n = 0, k = 0, W = 0;
    uint64_t tag = 0;
    int64_t index = -1;
    std::vector<int32_t> delta;
    uint16_t *d_delta = nullptr;
    SideState s[2];
    std::vector<uint8_t> sides;  // side of every step so far (0 forward, 1 inverse)
    u64 *colT = nullptr;      // current inverse level transposed: colT_cap words state-major, then colT_cap tile-major
    int64_t colT_cap = 0;     // words
    u64 *ysig = nullptr;      // signature (OR of the words) of each set of the current inverse level
    int64_t *d_off = nullptr; // level offsets of both sides for k_run_small: 2 x max_lev
    int32_t max_lev = 0;
    int64_t ysig_cap = 0;     // words
    // cardinality order of the current inverse level (ys_valid: it is in that order)
    u32 *ys_hist = nullptr, *ys_cnt = nullptr, *ys_idx = nullptr;
    int64_t ys_cap = 0;
    bool ys_valid = false;
    u64 *cand = nullptr;
    int64_t cand_cap = 0;     // rows
    u32 *cslot = nullptr;
    int64_t cslot_cap = 0;
    u32 *mark = nullptr, *red_par = nullptr;   // self-reduction: flags and moved keys, red_cap each
    int64_t red_cap = 0;
    // the current forward level bucket-sorted for the chunked meet
    u64 *xs_rows = nullptr, *xs_com = nullptr;
    u32 *xs_idx = nullptr, *xs_keys = nullptr, *xs_hist = nullptr, *xs_bins = nullptr;
    int32_t *xs_top = nullptr;
    int64_t xs_cap = 0;       // rows
    bool xs_valid = false;    // xs_* hold the current forward level
    bool sort_now = false;    // this step sorts its new forward level
    // the current inverse level in buckets (yb_valid; colT, ysig and yb_idx
    // are then in bucket order) -- see YbMeta
    bool yb_valid = false;
    bool yb_now = false;      // this step puts an inverse level into buckets
    char *yb_small = nullptr; // YbMeta, then the counters, bucket tiles and list offsets
    uint16_t *yb_key = nullptr;
    int64_t yb_key_cap = 0;
    u32 *yb_idx = nullptr;    // padded position -> index in the level
    int64_t yb_idx_cap = 0;
    u32 *yb_list = nullptr;
    int64_t yb_list_cap = 0;
    // plan of a bucketed meet: per chunk its key, the chunks in key order,
    // per key counts and offsets, the work queue
    u32 *mp_key = nullptr, *mp_order = nullptr, *mp_cpre = nullptr, *mp_kinfo = nullptr, *mp_queue = nullptr;
    int64_t mp_cap = 0;       // chunks
    int status = 1;           // 1 running, else SRW_ status
    int32_t r = -1;
    std::vector<uint8_t> word;
    int steps = 0;
    bool admitted = false;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int64_t est_bytes = 0;
    int64_t dev_bytes = 0;    // device memory its buffers held when it was released
};

// --------------------------------------------------------------- options

// a new forward level is bucket-sorted for the chunked meet when its
// candidates and the pairs it will be tested against are at least these
constexpr int64_t kSortMinCand = 2048;
constexpr double kSortMinPairs = double(1 << 22);

struct Options {
    int meet = 0;             // 0 auto, 1 LDS tiles only, 2 chunks whenever possible
    int schedule = 0;
    uint64_t sched_seed = 1;
    int meet_tiles = 0;
    int64_t meet_rows = kRowBatchMax;   // chunked meet: row tests up to this many candidates per group
    int64_t meet_groups = 16;           // chunked meet: tile groups per work item (upper limit)
    int64_t small_cand = 2048;          // steps with at most this many candidates run in one block (0: never)
    int persist = 1;                    // 1: the small steps of a new automaton run in one launch (k_run_small)
    int64_t bucket = kYMin;             // inverse levels of at least this many sets go into buckets for the meet (0: never)
    int64_t ysort = 0;                  // new inverse levels of at least this many candidates go in cardinality order (0: never)
    int64_t meet_grid = 0;              // meet blocks per launch (0: one per work item)
    int64_t meet_order = 1;             // chunked meet items: 0 tile-range-major, 1 chunk-major
    int64_t meet_xcd = 0;               // bucketed meet: items dealt to per-XCD queues in runs of this many (0: one queue)
    int64_t meet_bgrid = 4096;          // bucketed meet: blocks per launch (they take items from queues)
    int reduce = 0;                     // 1: self-reduction of every new level (Alg. 1), 2: also by history;
                                        // dropped sets kept visited
    int profile = 0;                    // 1: every kernel class and the meet; 2: the meet only
    bool keep_levels = false;
    bool verbose = false;          // one stderr line per step of a single solve
    int64_t max_slots = 4096;
    double deadline_ms = 0;        // per automaton, from admission (0: none)
    // per set width W (index W = 1..8; -1: the value above), e.g. from the
    // autotuner's table
    int64_t meet_groups_w[kMaxW + 1] = {-1, -1, -1, -1, -1, -1, -1, -1, -1};
    int64_t meet_rows_w[kMaxW + 1] = {-1, -1, -1, -1, -1, -1, -1, -1, -1};
    int64_t bucket_w[kMaxW + 1] = {-1, -1, -1, -1, -1, -1, -1, -1, -1};
    int64_t small_cand_w[kMaxW + 1] = {-1, -1, -1, -1, -1, -1, -1, -1, -1};
    int64_t schedule_w[kMaxW + 1] = {-1, -1, -1, -1, -1, -1, -1, -1, -1};
    int64_t groups(int W) const { return meet_groups_w[W] >= 0 ? meet_groups_w[W] : meet_groups; }
    int64_t rows(int W) const { return meet_rows_w[W] >= 0 ? meet_rows_w[W] : meet_rows; }
    int64_t bucket_min(int W) const { return bucket_w[W] >= 0 ? bucket_w[W] : bucket; }
    int64_t small(int W) const { return small_cand_w[W] >= 0 ? small_cand_w[W] : small_cand; }
    int sched(int W) const { return schedule_w[W] >= 0 ? (int)schedule_w[W] : schedule; }
};

// 64-bit finaliser of MurmurHash3 (Appleby), constants as published
static uint64_t mix64(uint64_t z) {
    z ^= z >> 33;
    z *= 0xff51afd7ed558ccdull;
    z ^= z >> 33;
    z *= 0xc4ceb9fe1a85ec53ull;
    z ^= z >> 33;
    return z;
}

// --------------------------------------------------------------- engine

class Engine {
  public:
    // pageable: staging buffers in ordinary host memory (no pinned
    // allocations at all; the no-alloc entry point runs such an engine)
    Engine(int device, Backing backing, int64_t budget, hipStream_t ext_stream, bool pageable = false)
        : device_(device), backing_(backing) {
        HIPCHK(hipSetDevice(device_));
        for (Pinned *q : {&pin_delta_, &pin_step_, &pin_res_, &pin_trace_, &pin_init_, &pin_misc_, &pin_clear_,
                          &pin_copy_, &pin_run_})
            q->pageable = pageable;
        if (ext_stream) {
            stream_ = ext_stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&own_stream_, hipStreamNonBlocking));
            stream_ = own_stream_;
        }
        if (budget <= 0) {
            size_t fr = 0, tot = 0;
            HIPCHK(hipMemGetInfo(&fr, &tot));
            budget = (int64_t)(fr * 0.8);
        }
        pool_.reset(new Pool(backing_, budget, stream_));
        int khz = 0;
        HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device_));
        wall_khz_ = khz > 0 ? (double)khz : 1e5;
        for (int c = 0; c < 16; ++c) HIPCHK(hipEventCreate(&ev_[c]));
        for (int c = 0; c < 2 * kMaxW; ++c) HIPCHK(hipEventCreate(&ev_meet_[c]));
        for (int c = 0; c < 2 * kMaxW; ++c) HIPCHK(hipEventCreate(&ev_meetb_[c]));
        memset(&stats_, 0, sizeof stats_);
    }
    ~Engine() {
        (void)hipSetDevice(device_);
        if (stream_) (void)hipStreamSynchronize(stream_);
        release_kept();
        pool_.reset();
        for (int c = 0; c < 16; ++c) (void)hipEventDestroy(ev_[c]);
        for (int c = 0; c < 2 * kMaxW; ++c) (void)hipEventDestroy(ev_meet_[c]);
        for (int c = 0; c < 2 * kMaxW; ++c) (void)hipEventDestroy(ev_meetb_[c]);
        if (own_stream_) (void)hipStreamDestroy(own_stream_);
    }

    Options opt;
    srw_stats stats_;

    // statistics with the device-side meet counters folded in
    srw_stats stats() {
        srw_stats out = stats_;
        if (d_ops_) {
            u64 *h = (u64 *)pin_misc_.acquire((kOpsWords + kMstatWords) * sizeof(u64));
            HIPCHK(hipMemcpyAsync(h, d_ops_, (kOpsWords + kMstatWords) * sizeof(u64), hipMemcpyDeviceToHost, stream_));
            HIPCHK(hipStreamSynchronize(stream_));
            for (int w = 0; w < kMaxW; ++w) {
                out.meet_ops_w[w] = out.meet_b_ops_w[w] = 0;
                for (int sl = 0; sl < kOpsSlots; ++sl) {
                    const u64 *c = h + ((int64_t)w * kOpsSlots + sl) * kOpsStride;
                    out.meet_b_ops_w[w] += (int64_t)c[1];
                    out.meet_ops_w[w] += (int64_t)(c[0] + c[1]);
                }
            }
            for (int c = 0; c < kMstatCounters - 1; ++c) {   // [7] is counted on the host
                out.meet_work[c] = 0;
                for (int sl = 0; sl < kMstatSlots; ++sl) out.meet_work[c] += (int64_t)h[kOpsWords + sl * kOpsStride + c];
            }
        }
        return out;
    }
    void reset_stats() {
        memset(&stats_, 0, sizeof stats_);
        if (d_ops_) {
            HIPCHK(launch_fill(d_ops_, kOpsWords + kMstatWords, 0, stream_));
            HIPCHK(hipStreamSynchronize(stream_));
        }
    }

    void set_budget(int64_t b) {
        if (b <= 0) {
            size_t fr = 0, tot = 0;
            HIPCHK(hipMemGetInfo(&fr, &tot));
            b = pool_->reserved() + (int64_t)(fr * 0.8);
        }
        pool_->set_budget(b);
    }
    int64_t budget() const { return pool_->budget(); }
    int64_t in_use() const { return pool_->in_use(); }
    int device() const { return device_; }

    // Runs every problem of `probs` to completion, at most opt.max_slots at
    // a time (continuous admission as others finish).
    void run(std::vector<Problem *> &probs) {
        HIPCHK(hipSetDevice(device_));
        std::deque<Problem *> pending(probs.begin(), probs.end());
        std::vector<Problem *> active;
        while (!pending.empty() || !active.empty()) {
            std::vector<Problem *> fresh;
            // in order; one whose estimated footprint does not fit yet waits
            // without blocking smaller ones behind it
            std::deque<Problem *> waiting;
            while (!pending.empty()) {
                Problem *p = pending.front();
                pending.pop_front();
                if ((int64_t)active.size() >= opt.max_slots ||
                    (!active.empty() && in_use() + p->est_bytes > budget())) {
                    waiting.push_back(p);
                    continue;
                }
                if (admit(p)) {
                    active.push_back(p);
                    fresh.push_back(p);
                } else if (active.empty()) {
                    finish_error(p, SRW_ENOMEM);
                } else {
                    waiting.push_back(p);
                }
            }
            pending.swap(waiting);
            if (!fresh.empty()) {
                init(fresh);
                run_small(fresh, opt.deadline_ms);
            }
            if (active.empty()) continue;
            step(active);
            std::vector<Problem *> still;
            for (Problem *p : active) {
                if (p->status == 1 && opt.deadline_ms > 0 && now_ms() - p->t_admit > opt.deadline_ms)
                    finish_error(p, SRW_ETIMEOUT, "deadline passed before the searches met");
                if (p->status == 1) still.push_back(p);
            }
            active.swap(still);
        }
    }

    // --- single steps for the server
    bool admit(Problem *p) {
        const int n = p->n, W = p->W;
        p->t_admit = now_ms();
        bool ok = true;
        auto A = [&](size_t bytes) -> void * {
            void *q = pool_->alloc(bytes);
            if (!q) ok = false;
            return q;
        };
        p->d_delta = (uint16_t *)A((size_t)p->k * n * sizeof(uint16_t));
        const int64_t cap0 = std::max<int64_t>(256, n + 1);
        for (int sd = 0; sd < 2; ++sd) {
            SideState &s = p->s[sd];
            s.cap = cap0;
            s.rows = (u64 *)A((size_t)cap0 * W * 8);
            s.par = (u32 *)A((size_t)cap0 * 4);
            s.tab_cap = 1024;
            while (s.tab_cap < 4 * cap0) s.tab_cap <<= 1;
            s.tab = (u64 *)A((size_t)s.tab_cap * 8);
        }
        int64_t tiles0 = ceil_div(n, 64);
        if (persist_ok(W)) {
            // room for the steps k_run_small may take before the first large
            // one: kPersistRows sets per side, one small step of candidates
            const int64_t cc = std::min<int64_t>(opt.small(W), kPersistCand);
            for (int sd = 0; sd < 2; ++sd) {
                SideState &s = p->s[sd];
                pool_->free(s.rows);
                pool_->free(s.par);
                pool_->free(s.tab);
                s.cap = std::max<int64_t>(cap0, kPersistRows);
                s.rows = (u64 *)A((size_t)s.cap * W * 8);
                s.par = (u32 *)A((size_t)s.cap * 4);
                s.tab_cap = 1024;
                while (s.tab_cap < 4 * s.cap) s.tab_cap <<= 1;
                s.tab = (u64 *)A((size_t)s.tab_cap * 8);
            }
            p->cand_cap = p->cslot_cap = cc;
            p->cand = (u64 *)A((size_t)cc * W * 8);
            p->cslot = (u32 *)A((size_t)cc * 4);
            tiles0 = std::max(tiles0, ceil_div(cc, 64));
            p->max_lev = (int32_t)std::min<int64_t>(kPersistLevels, std::max<int64_t>(128, (int64_t)n * n + 2));
            p->d_off = (int64_t *)A((size_t)2 * p->max_lev * 8);
        }
        p->colT_cap = tiles0 * 64 * W;
        p->colT = (u64 *)A((size_t)p->colT_cap * 16);   // state-major, then tile-major
        p->ysig_cap = tiles0 * 64;
        p->ysig = (u64 *)A((size_t)p->ysig_cap * 8);
        if (!ok) {
            release(p);
            return false;
        }
        p->s[0].off = {0, 1};
        p->s[0].nrows = 1;
        p->s[0].popsum = (u64)n;        // Q
        p->s[1].off = {0, n};
        p->s[1].nrows = n;
        p->s[1].popsum = (u64)n;        // the n singletons
        p->admitted = true;
        return true;
    }

    void init(std::vector<Problem *> &ps) {
        const int nseg = (int)ps.size();
        // deltas as uint16
        size_t dbytes = 0;
        for (Problem *p : ps) dbytes += (size_t)p->k * p->n * 2;
        uint16_t *hd = (uint16_t *)pin_delta_.acquire(dbytes);
        std::vector<size_t> doff(nseg);
        size_t o = 0;
        for (int i = 0; i < nseg; ++i) {
            Problem *p = ps[i];
            const size_t cnt = (size_t)p->k * p->n;
            for (size_t e = 0; e < cnt; ++e) hd[o + e] = (uint16_t)p->delta[e];
            doff[i] = o;
            o += cnt;
        }
        // one copy for all tables; k_init moves each to its automaton
        uint16_t *dsrc = (uint16_t *)dev_need(delta_blob_, delta_blob_cap_, align8(dbytes));
        HIPCHK(hipMemcpyAsync(dsrc, hd, dbytes, hipMemcpyHostToDevice, stream_));
        pin_delta_.issued(stream_);
        // clear both tables, write level 0, insert it, transpose inverse level 0
        std::vector<InitDesc> idesc(nseg);
        std::vector<int64_t> ipre(nseg + 1, 0);
        std::vector<RehashDesc> rdesc;
        std::vector<int64_t> rpre(1, 0);
        std::vector<TransposeDesc> tdesc(nseg);
        std::vector<int64_t> tpre(nseg + 1, 0);
        for (int i = 0; i < nseg; ++i) {
            Problem *p = ps[i];
            idesc[i] = InitDesc{p->n, p->W, p->s[0].rows, p->s[1].rows, p->s[0].par, p->s[1].par,
                                dsrc + doff[i], p->d_delta, p->k, 0};
            ipre[i + 1] = ipre[i] + ceil_div(p->n + 1, kBS);
            for (int sd = 0; sd < 2; ++sd) {
                rdesc.push_back(RehashDesc{p->W, 0, p->s[sd].rows, p->s[sd].nrows, p->s[sd].tab,
                                           (u64)(p->s[sd].tab_cap - 1)});
                rpre.push_back(rpre.back() + ceil_div(p->s[sd].nrows, kBS));
            }
            tdesc[i] = TransposeDesc{p->W, 0, p->s[1].rows, p->n, p->colT, p->colT + p->colT_cap, p->ysig};
            tpre[i + 1] = tpre[i] + ceil_div(ceil_div(p->n, 64) * p->W, kBS / 64);
        }
        prof_begin(6);
        char *blob = upload3(idesc, ipre, rdesc, rpre, tdesc, tpre);
        const size_t a1 = sizeof(InitDesc) * idesc.size(), a2 = 8 * ipre.size();
        const size_t a3 = sizeof(RehashDesc) * rdesc.size(), a4 = 8 * rpre.size();
        const size_t a5 = sizeof(TransposeDesc) * tdesc.size();
        char *b = blob;
        const InitDesc *dI = (const InitDesc *)b; b += align8(a1);
        const int64_t *dIp = (const int64_t *)b; b += align8(a2);
        const RehashDesc *dR = (const RehashDesc *)b; b += align8(a3);
        const int64_t *dRp = (const int64_t *)b; b += align8(a4);
        const TransposeDesc *dT = (const TransposeDesc *)b; b += align8(a5);
        const int64_t *dTp = (const int64_t *)b;
        clear_tables(rdesc);
        HIPCHK(launch_init(dI, dIp, nseg, ipre[nseg], stream_));
        HIPCHK(launch_rehash(dR, dRp, (int)rdesc.size(), rpre.back(), stream_));
        HIPCHK(launch_transpose_rows(dT, dTp, nseg, tpre[nseg], stream_));
        prof_end(6);
        stats_.launches[6] += 4;
    }

    // one launch marks every slot of all these tables free
    void clear_tables(const std::vector<RehashDesc> &t) {
        std::vector<int64_t> cpre(1, 0);
        for (const RehashDesc &r : t) cpre.push_back(cpre.back() + ceil_div((int64_t)r.tab_mask + 1, kBS));
        const size_t a = align8(sizeof(RehashDesc) * t.size()), b = align8(8 * cpre.size());
        char *h = (char *)pin_clear_.acquire(a + b);
        memcpy(h, t.data(), sizeof(RehashDesc) * t.size());
        memcpy(h + a, cpre.data(), 8 * cpre.size());
        char *d = dev_need(clear_blob_, clear_blob_cap_, a + b);
        HIPCHK(hipMemcpyAsync(d, h, a + b, hipMemcpyHostToDevice, stream_));
        pin_clear_.issued(stream_);
        HIPCHK(launch_clear_tables((const RehashDesc *)d, (const int64_t *)(d + a), (int)t.size(),
                                   cpre.back(), stream_));
    }

    // One global step: every active problem expands one side.
    void step(std::vector<Problem *> &act) {
        HIPCHK(hipSetDevice(device_));
        const double t0 = now_ms();
        std::vector<Problem *> segp;
        std::vector<int> segdir;
        std::vector<RehashDesc> grow;
        std::vector<int64_t> growpre(1, 0);
        std::vector<Problem *> waiting;
        prof_begin(6);
        for (Problem *p : act) {
            if (p->status != 1) continue;
            const int dir = choose_side(p);
            const int fail = prepare(p, dir, grow, growpre);
            if (fail == SRW_ENOMEM) {
                waiting.push_back(p);   // sits this step out; others may free memory
                continue;
            }
            if (fail) {
                finish_error(p, fail);
                continue;
            }
            segp.push_back(p);
            segdir.push_back(dir);
        }
        flush_copies();
        if (segp.empty() && !waiting.empty()) {
            // nothing can move: give up on the largest one to free memory
            Problem *big = waiting[0];
            for (Problem *p : waiting)
                if (p->s[0].nrows + p->s[1].nrows > big->s[0].nrows + big->s[1].nrows) big = p;
            finish_error(big, SRW_ENOMEM, "device memory budget exhausted before the searches met");
        }
        if (!grow.empty()) {
            clear_tables(grow);
            const RehashDesc *dR = (const RehashDesc *)upload_simple(grow, growpre, rehash_blob_);
            const int64_t *dRp = (const int64_t *)((char *)dR + align8(sizeof(RehashDesc) * grow.size()));
            HIPCHK(launch_rehash(dR, dRp, (int)grow.size(), growpre.back(), stream_));
            stats_.launches[6] += 2;
        }
        prof_end(6);
        const double t1 = now_ms();
        stats_.host_ms[0] += t1 - t0;
        const int nseg = (int)segp.size();
        if (nseg == 0) return;
        {   // segments of equal width side by side: the meet launches per width
            std::vector<int> ord(nseg);
            for (int i = 0; i < nseg; ++i) ord[i] = i;
            std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return segp[a]->W < segp[b]->W; });
            std::vector<Problem *> sp(nseg);
            std::vector<int> sd(nseg);
            for (int i = 0; i < nseg; ++i) { sp[i] = segp[ord[i]]; sd[i] = segdir[ord[i]]; }
            segp.swap(sp);
            segdir.swap(sd);
        }

        // descriptors
        std::vector<StepDesc> D(nseg);
        std::vector<int64_t> pe(nseg + 1, 0), pc(nseg + 1, 0), pt(nseg + 1, 0), pm(nseg + 1, 0), pq(nseg + 1, 0);
        std::vector<SortDesc> S;
        std::vector<int64_t> pz(1, 0), pr(1, 0), pch(1, 0);
        std::vector<int32_t> small;                // segments whose whole step runs in one block
        std::vector<YbDesc> YB;                    // inverse levels put into buckets in this step
        std::vector<int64_t> pyb[4] = {{0}, {0}, {0}, {0}};
        std::vector<int64_t> pmp(nseg + 1, 0);     // bucketed meets: blocks over chunks
        if ((int64_t)nseg * kResWords > res_cap_) {
            pool_->free(d_res_);
            res_cap_ = std::max<int64_t>((int64_t)nseg * kResWords, 2 * res_cap_);
            d_res_ = (u64 *)pool_->alloc((size_t)res_cap_ * 8, true);
            if (!d_res_) throw HipFailure{hipErrorOutOfMemory, "step result buffer"};
        }
        ensure_ops();
        for (int i = 0; i < nseg; ++i) {
            Problem *p = segp[i];
            const int dir = segdir[i];
            SideState &s = p->s[dir];
            const int W = p->W;
            StepDesc &d = D[i];
            memset(&d, 0, sizeof d);
            d.n = p->n;
            d.k = p->k;
            d.W = W;
            d.dir = dir;
            d.delta = p->d_delta;
            d.m = s.cur();
            d.par_rows = s.rows + s.cur_start() * W;
            d.C = d.m * p->k;
            d.cand = p->cand;
            d.cslot = p->cslot;
            d.tab = s.tab;
            d.tab_mask = (u64)(s.tab_cap - 1);
            d.vis_rows = s.rows;
            if (opt.reduce) {
                d.ghost = s.ghost;
                d.ghost_base = s.nghost;
                d.mark = p->mark;
                d.red_par = p->red_par;
                d.red_hist = opt.reduce == 2;
            }
            d.out_rows = s.rows + s.nrows * W;
            d.out_par = s.par + s.nrows;
            d.out_base = s.nrows;
            d.ncblk = ceil_div(d.C, kCB);
            d.cblk_base = pc[i];
            int64_t nx_ub, ny_ub;
            if (dir == 0) {
                d.X = d.out_rows;
                d.nX = -1;
                nx_ub = d.C;
                d.YT = p->colT;
                d.YTt = p->colT + p->colT_cap;
                d.Yrows = p->s[1].rows + p->s[1].cur_start() * W;
                d.Ysig = p->ysig;
                d.nY = p->s[1].cur();
                ny_ub = d.nY;
            } else {
                d.X = p->s[0].rows + p->s[0].cur_start() * W;
                d.nX = p->s[0].cur();
                nx_ub = d.nX;
                d.YT = p->colT;
                d.YTt = p->colT + p->colT_cap;
                d.Yrows = d.out_rows;
                d.Ysig = p->ysig;
                d.nY = -1;
                ny_ub = d.C;
            }
            d.res = d_res_ + kResWords * i;
            d.mstat = opt.profile == 1 ? d_ops_ + kOpsWords : nullptr;
            // chunked meet over the sorted forward level when it exists
            if ((dir == 0 && p->sort_now) || (dir == 1 && p->xs_valid && opt.meet != 1)) {
                d.meet_mode = bucketed_meet(p, dir) ? 2 : 1;
                d.X = p->xs_rows;
                d.Xidx = p->xs_idx;
                d.Xcom = p->xs_com;
            }
            if (p->yb_now) {                       // the inverse level goes into buckets
                const int64_t yub = dir == 1 ? d.C : d.nY;
                const int64_t nt_ub = ceil_div(yub, 64) + kYBins;
                u32 *w = yb_words(p);
                YbDesc y;
                memset(&y, 0, sizeof y);
                y.n = p->n;
                y.W = W;
                y.rows = dir == 1 ? d.out_rows : d.Yrows;
                y.cnt = dir == 1 ? d.res : nullptr;
                y.count = dir == 1 ? 0 : d.nY;
                y.count_ub = yub;
                y.nt_ub = nt_ub;
                y.top = p->xs_top;
                y.meta = yb_meta(p);
                y.key = p->yb_key;
                y.bins = w;
                y.tb = w + 2 * kYBins;
                y.lsize = y.tb + kYBins + 1;
                y.loff = y.lsize + kYBins;
                y.lcur = y.loff + kYBins + 1;
                y.list = p->yb_list;
                y.list_cap = p->yb_list_cap;
                y.idx = p->yb_idx;
                y.YT = p->colT;
                y.YTt = p->colT + p->colT_cap;
                y.Ysig = p->ysig;
                YB.push_back(y);
                pyb[0].push_back(pyb[0].back() + ceil_div(yub, kBS));
                pyb[1].push_back(pyb[1].back() + ceil_div(nt_ub * 64, kBS));
                pyb[2].push_back(pyb[2].back() + kYBins / (kBS / 64));
                pyb[3].push_back(pyb[3].back() + ceil_div(nt_ub * W, kBS / 64));
            }
            if (d.meet_mode == 2) {
                u32 *w = yb_words(p);
                d.yb = yb_meta(p);
                d.yb_lsize = w + 2 * kYBins + kYBins + 1;
                d.yb_loff = d.yb_lsize + kYBins;
                d.yb_list = p->yb_list;
                d.Yidx = p->yb_idx;
                d.ckey = p->mp_key;
                d.korder = p->mp_order;
                d.kinfo = p->mp_kinfo;
                d.queue = p->mp_queue;
            }
            if (dir == 0 && p->sort_now) {
                S.push_back(SortDesc{p->n, W, d.out_rows, d.res, d.C, p->xs_hist, p->xs_top, p->xs_keys,
                                     p->xs_bins, p->xs_rows, p->xs_idx, p->xs_com});
                pz.push_back(pz.back() + ceil_div(kSortBins + p->n, kBS));
                pr.push_back(pr.back() + ceil_div(d.C, kBS));
                pch.push_back(pch.back() + ceil_div(ceil_div(d.C, 64), kBS / 64));
            }
            if (d.meet_mode == 0) {
                const int tmax = std::max(1, kMeetTileWords / W);   // LDS holds tpb*64*W words
                d.tpb = opt.meet_tiles > 0 ? std::min(opt.meet_tiles, tmax) : tmax;
                d.nXb = ceil_div(nx_ub, kBS);
                d.nYc = ceil_div(ceil_div(ny_ub, 64), d.tpb);
                pm[i + 1] = pm[i] + d.nXb * d.nYc;
            } else {
                const int64_t ng_ub = ceil_div(ceil_div(ny_ub, 64) + (d.meet_mode == 2 ? kYBins : 0), 64);
                d.ngi = std::max<int64_t>(1, std::min<int64_t>(opt.groups(W), ng_ub));
                d.row_batch_max = std::min<int64_t>(opt.rows(W), kRowBatchMax);
                d.nch_ub = ceil_div(nx_ub, 64);
                d.item_order = opt.meet_order;
                d.xcd_granule = opt.meet_xcd;
                d.gitems_ub = ceil_div(ng_ub, d.ngi);
                if (d.meet_mode == 1) pm[i + 1] = pm[i] + ceil_div(ceil_div(nx_ub, 64) * d.gitems_ub, kBS / 64);
                else pm[i + 1] = pm[i];            // its items come from a queue
            }
            pmp[i + 1] = pmp[i] + (d.meet_mode == 2 ? ceil_div(ceil_div(nx_ub, 64), kBS) : 0);
            // the new inverse level is transposed in level order, unless it
            // goes into buckets (transposed in bucket order there)
            d.ntr_waves = (dir == 1 && !p->yb_now) ? ceil_div(d.C, 64) * W : 0;
            d.small = d.meet_mode == 0 && d.C <= opt.small(W) && d.nXb * d.nYc <= kSmallMeetBlocks && !opt.reduce;
            if (d.small) {
                pm[i + 1] = pm[i];
                small.push_back(i);
            }
            if (dir == 0 && p->ys_valid) {         // the current inverse level is in cardinality order
                d.Yidx = p->ys_idx;
                d.Ycnt = p->ys_cnt;
            }
            if (dir == 1 && !d.small && opt.ysort > 0 && d.C >= opt.ysort && ensure_ysort(p, d.C)) {
                d.ysort = 1;
                d.ys_hist = p->ys_hist;
                d.ys_cnt = p->ys_cnt;
                d.ys_idx = p->ys_idx;
                d.Yidx = p->ys_idx;
                d.Ycnt = p->ys_cnt;
            }
            pq[i + 1] = pq[i] + (d.ysort ? ceil_div(d.C, kBS) : 0);
            pe[i + 1] = pe[i] + (d.small ? 0 : ceil_div(d.C, kBS));
            pc[i + 1] = pc[i] + (d.small ? 0 : d.ncblk);
            pt[i + 1] = pt[i] + (d.small ? 0 : ceil_div(d.ntr_waves, kBS / 64));
            stats_.candidates += d.C;
            stats_.cand_words += d.C * W;
            stats_.bytes_expand += 8 * W * (d.m + d.C);
            stats_.bytes_insert += d.C * (8 * W + 8 + 4);
        }
        // compaction block counters
        const int64_t ncb = pc[nseg];
        if (ncb > cblk_cap_) {
            pool_->free(d_cnt_);
            pool_->free(d_off_);
            cblk_cap_ = std::max(ncb, 2 * cblk_cap_);
            d_cnt_ = (u32 *)pool_->alloc((size_t)cblk_cap_ * 4, true);
            d_off_ = (u32 *)pool_->alloc((size_t)cblk_cap_ * 4, true);
            if (!d_cnt_ || !d_off_) throw HipFailure{hipErrorOutOfMemory, "compaction counters"};
        }
        // upload descriptors + the four block prefixes in one copy
        const int nsort = (int)S.size();
        const size_t szD = align8(sizeof(StepDesc) * nseg), szP = align8(8 * (nseg + 1));
        const size_t szS = align8(sizeof(SortDesc) * nsort), szQ = align8(8 * (nsort + 1));
        const int nsmall = (int)small.size();
        const size_t szL = align8(4 * (size_t)std::max(1, nsmall));
        const int nyb = (int)YB.size();
        const size_t szY = align8(sizeof(YbDesc) * nyb), szYP = align8(8 * (nyb + 1));
        const size_t total = szD + 4 * szP + szS + 3 * szQ + szL + szP + szY + 4 * szYP + szP;
        char *h = (char *)pin_step_.need(total);
        memcpy(h, D.data(), sizeof(StepDesc) * nseg);
        memcpy(h + szD, pe.data(), 8 * (nseg + 1));
        memcpy(h + szD + szP, pc.data(), 8 * (nseg + 1));
        memcpy(h + szD + 2 * szP, pt.data(), 8 * (nseg + 1));
        memcpy(h + szD + 3 * szP, pm.data(), 8 * (nseg + 1));
        const size_t oS = szD + 4 * szP;
        if (nsort) memcpy(h + oS, S.data(), sizeof(SortDesc) * nsort);
        memcpy(h + oS + szS, pz.data(), 8 * (nsort + 1));
        memcpy(h + oS + szS + szQ, pr.data(), 8 * (nsort + 1));
        memcpy(h + oS + szS + 2 * szQ, pch.data(), 8 * (nsort + 1));
        const size_t oL = oS + szS + 3 * szQ;
        if (nsmall) memcpy(h + oL, small.data(), 4 * nsmall);
        const size_t oQ = oL + szL;
        memcpy(h + oQ, pq.data(), 8 * (nseg + 1));
        const size_t oY = oQ + szP;
        if (nyb) memcpy(h + oY, YB.data(), sizeof(YbDesc) * nyb);
        for (int k2 = 0; k2 < 4; ++k2) memcpy(h + oY + szY + k2 * szYP, pyb[k2].data(), 8 * (nyb + 1));
        const size_t oMP = oY + szY + 4 * szYP;
        memcpy(h + oMP, pmp.data(), 8 * (nseg + 1));
        char *dblob = dev_need(step_blob_, step_blob_cap_, total);
        HIPCHK(hipMemcpyAsync(dblob, h, total, hipMemcpyHostToDevice, stream_));
        const StepDesc *dD = (const StepDesc *)dblob;
        const int64_t *dpe = (const int64_t *)(dblob + szD);
        const int64_t *dpc = (const int64_t *)(dblob + szD + szP);
        const int64_t *dpt = (const int64_t *)(dblob + szD + 2 * szP);
        const int64_t *dpm = (const int64_t *)(dblob + szD + 3 * szP);
        const SortDesc *dS = (const SortDesc *)(dblob + oS);
        const int64_t *const dsp[3] = {(const int64_t *)(dblob + oS + szS),
                                       (const int64_t *)(dblob + oS + szS + szQ),
                                       (const int64_t *)(dblob + oS + szS + 2 * szQ)};
        const int64_t sblocks[3] = {pz.back(), pr.back(), pch.back()};
        const int32_t *dsmall = (const int32_t *)(dblob + oL);
        const int64_t *dpq = (const int64_t *)(dblob + oQ);
        const YbDesc *dY = (const YbDesc *)(dblob + oY);
        const int64_t *const dyp[4] = {(const int64_t *)(dblob + oY + szY), (const int64_t *)(dblob + oY + szY + szYP),
                                       (const int64_t *)(dblob + oY + szY + 2 * szYP),
                                       (const int64_t *)(dblob + oY + szY + 3 * szYP)};
        const int64_t yblocks[4] = {pyb[0].back(), pyb[1].back(), pyb[2].back(), pyb[3].back()};
        const int64_t *dpmp = (const int64_t *)(dblob + oMP);

        prof_begin(0);
        HIPCHK(launch_step_small(dD, dsmall, nsmall, opt.profile ? d_ops_ : nullptr, stream_));
        HIPCHK(launch_expand(dD, dpe, nseg, pe[nseg], stream_));
        prof_end(0);
        prof_begin(1);
        HIPCHK(launch_insert(dD, dpe, nseg, pe[nseg], stream_));
        prof_end(1);
        prof_begin(2);
        HIPCHK(launch_count(dD, dpc, nseg, pc[nseg], d_cnt_, stream_));
        if (nsmall < nseg) HIPCHK(launch_scan(dD, nseg, d_cnt_, d_off_, stream_));
        HIPCHK(launch_compact(dD, dpc, nseg, pc[nseg], d_off_, stream_));
        if (opt.reduce)        // the new levels' self-reduction, before the meet sees them
            HIPCHK(launch_reduce(dD, dpe, dpc, nseg, pe[nseg], pc[nseg], d_cnt_, d_off_, stream_));
        prof_end(2);
        if (pt[nseg] > 0 || nsort > 0 || nyb > 0 || pmp[nseg] > 0) {
            prof_begin(3);
            HIPCHK(launch_ysort(dD, dpq, nseg, pq[nseg], stream_));
            HIPCHK(launch_transpose(dD, dpt, nseg, pt[nseg], stream_));
            HIPCHK(launch_sort(dS, dsp, sblocks, nsort, stream_));
            // buckets of inverse levels (after the sorts: they take their
            // split states from the forward level's most frequent states)
            HIPCHK(launch_ybin(dY, dyp, yblocks, nyb, stream_));
            HIPCHK(launch_meet_plan(dD, dpmp, nseg, pmp[nseg], stream_));
            prof_end(3);
            stats_.launches[3]++;
        }
        prof_begin(4);
        for (int s0 = 0; s0 < nseg;) {
            int s1 = s0;
            const int W = segp[s0]->W;
            while (s1 < nseg && segp[s1]->W == W) ++s1;
            int64_t bk_items = 0;                  // bucketed meets: their work items (upper bound)
            for (int i = s0; i < s1; ++i)
                if (D[i].meet_mode == 2) bk_items += D[i].nch_ub * D[i].gitems_ub;
            if (pm[s1] == pm[s0] && bk_items == 0) {   // only small segments of this width
                s0 = s1;
                continue;
            }
            if (opt.profile) {
                HIPCHK(hipEventRecord(ev_meet_[2 * (W - 1)], stream_));
                meet_used_[W - 1] = true;
            }
            // operations are counted by the counting kernels, with profile 1
            u64 *ops = opt.profile == 1 ? d_ops_ + (int64_t)(W - 1) * kOpsSlots * kOpsStride : nullptr;
            if (pm[s1] > pm[s0]) {
                bool ys = false;                   // an inverse level in cardinality order
                for (int i = s0; i < s1; ++i) ys = ys || (D[i].meet_mode != 2 && D[i].Yidx != nullptr);
                HIPCHK(launch_meet(dD, dpm, s0, s1, W, pm[s1] - pm[s0], opt.meet_grid, ys, ops, stream_));
            }
            if (bk_items > 0) {
                // its own events and, in the counting build, its own word of
                // each counter slot
                if (opt.profile) {
                    HIPCHK(hipEventRecord(ev_meetb_[2 * (W - 1)], stream_));
                    meetb_used_[W - 1] = true;
                }
                HIPCHK(launch_meet_b(dD, s0, s1, W, std::min<int64_t>(ceil_div(bk_items, kBS / 64), opt.meet_bgrid),
                                     ops ? ops + 1 : nullptr, stream_));
                if (opt.profile) HIPCHK(hipEventRecord(ev_meetb_[2 * (W - 1) + 1], stream_));
                stats_.meet_work[7]++;
                stats_.meet_b_launches_w[W - 1]++;
            }
            if (opt.profile) HIPCHK(hipEventRecord(ev_meet_[2 * (W - 1) + 1], stream_));
            stats_.meet_launches_w[W - 1]++;
            s0 = s1;
        }
        prof_end(4);
        stats_.launches[0]++;
        stats_.launches[1]++;
        stats_.launches[2]++;
        stats_.launches[4]++;
        u64 *hres = (u64 *)pin_res_.need((size_t)nseg * kResWords * 8);
        HIPCHK(hipMemcpyAsync(hres, d_res_, (size_t)nseg * kResWords * 8, hipMemcpyDeviceToHost, stream_));
        const double t2 = now_ms();
        wait_step();
        const double t3 = now_ms();
        stats_.host_ms[1] += t2 - t1;
        stats_.host_ms[2] += t3 - t2;
        prof_collect();
        stats_.global_steps++;

        std::vector<Problem *> met;
        std::vector<u64> metbest;
        for (int i = 0; i < nseg; ++i) {
            Problem *p = segp[i];
            const int dir = segdir[i];
            SideState &s = p->s[dir];
            const int64_t U = (int64_t)hres[kResWords * i];
            const u64 best = hres[kResWords * i + 1];
            const StepDesc &d = D[i];
            s.nrows += U;
            s.off.push_back(s.nrows);
            s.popsum = hres[kResWords * i + 2];
            s.nghost += (int64_t)hres[kResWords * i + 3];
            stats_.reduced += (int64_t)hres[kResWords * i + 3];
            p->sides.push_back((uint8_t)dir);
            if (dir == 0) p->xs_valid = p->sort_now;
            if (dir == 1) p->ys_valid = d.ysort != 0;
            if (dir == 1) p->yb_valid = p->yb_now;   // a new inverse level: bucketed or not
            else if (p->yb_now) p->yb_valid = true;  // the current one put into buckets
            p->sort_now = false;
            p->yb_now = false;
            p->steps++;
            stats_.steps++;
            stats_.unique += U;
            stats_.bytes_compact += d.C * 24 + U * (16 * p->W + 12);
            const int64_t nx = dir == 0 ? U : d.nX;
            const int64_t ny = dir == 0 ? d.nY : U;
            stats_.pairs += nx * ny;
            stats_.pair_words += nx * ny * p->W;
            stats_.pair_words_w[p->W - 1] += nx * ny * p->W;
            if (opt.verbose && nseg == 1)
                fprintf(stderr, "srw step %d %s f=%d b=%d cand=%lld new=%lld |X|=%lld |Y|=%lld meet=%s %.1f ms\n",
                        p->steps, dir ? "inv" : "fwd", p->s[0].nlev() - 1, p->s[1].nlev() - 1,
                        (long long)d.C, (long long)U, (long long)nx, (long long)ny,
                        d.meet_mode ? "chunks" : "tiles", now_ms() - t0);
            if (best != kEmpty) {
                met.push_back(p);
                metbest.push_back(best);
            } else if (U == 0) {
                finish_error(p, SRW_EINTERNAL, "a list became empty before the searches met");
            }
        }
        if (!met.empty()) trace(met, metbest);
        const double t4 = now_ms();
        stats_.host_ms[3] += t4 - t3;
        stats_.ms[7] += t4 - t0;
    }

    // The steps of newly admitted automata, in one launch per set width: a
    // block per automaton steps it until the searches meet or until a step
    // is too large for one block; the host then takes over from the state
    // the block left (rows, level offsets).  Met automata are traced here.
    // deadline_ms: per automaton, from its admission (0: none)
    void run_small(std::vector<Problem *> &ps, double deadline_ms) {
        std::vector<Problem *> q;
        for (Problem *p : ps)
            if (p->status == 1 && p->d_off && p->s[0].nlev() == 1 && p->s[1].nlev() == 1) q.push_back(p);
        if (q.empty()) return;
        std::stable_sort(q.begin(), q.end(), [](Problem *a, Problem *b) { return a->W < b->W; });
        const int nq = (int)q.size();
        const size_t szD = align8(sizeof(RunDesc) * nq), szS = align8(sizeof(RunState) * nq);
        char *dblob = dev_need(run_blob_, run_blob_cap_, szD + szS);
        char *h = (char *)pin_run_.acquire(szD + szS);
        RunDesc *D = (RunDesc *)h;
        RunState *S = (RunState *)(h + szD);
        RunState *dS = (RunState *)(dblob + szD);
        for (int i = 0; i < nq; ++i) {
            Problem *p = q[i];
            RunDesc &r = D[i];
            memset(&r, 0, sizeof r);
            r.n = p->n;
            r.k = p->k;
            r.W = p->W;
            r.max_lev = p->max_lev;
            r.delta = p->d_delta;
            for (int sd = 0; sd < 2; ++sd) {
                SideState &s = p->s[sd];
                r.rows[sd] = s.rows;
                r.par[sd] = s.par;
                r.tab[sd] = s.tab;
                r.tab_mask[sd] = (u64)(s.tab_cap - 1);
                r.rows_cap[sd] = s.cap;
                r.off[sd] = p->d_off + (int64_t)sd * p->max_lev;
            }
            r.cand = p->cand;
            r.cslot = p->cslot;
            r.cand_cap = std::min(p->cand_cap, p->cslot_cap);
            r.colT = p->colT;
            r.colT_cap = p->colT_cap;
            r.ysig = p->ysig;
            r.ysig_cap = p->ysig_cap;
            r.small_cand = opt.small(p->W);
            if (deadline_ms > 0) {
                const double left = deadline_ms - (now_ms() - p->t_admit);
                r.max_ticks = std::max<int64_t>(1, (int64_t)(left * wall_khz_));
            }
            r.st = dS + i;
            RunState &st = S[i];
            memset(&st, 0, sizeof st);
            for (int sd = 0; sd < 2; ++sd) {
                st.nrows[sd] = p->s[sd].nrows;
                st.nlev[sd] = p->s[sd].nlev();
                st.popsum[sd] = p->s[sd].popsum;
            }
        }
        ensure_ops();
        prof_begin(0);
        HIPCHK(hipMemcpyAsync(dblob, h, szD + szS, hipMemcpyHostToDevice, stream_));
        pin_run_.issued(stream_);
        for (int i0 = 0; i0 < nq;) {
            int i1 = i0;
            while (i1 < nq && q[i1]->W == q[i0]->W) ++i1;
            HIPCHK(launch_run_small((const RunDesc *)dblob + i0, i1 - i0, q[i0]->W,
                                    opt.profile ? d_ops_ : nullptr, stream_));
            i0 = i1;
        }
        prof_end(0);
        stats_.launches[0]++;
        RunState *hS = (RunState *)pin_res_.need(szS);
        HIPCHK(hipMemcpyAsync(hS, dS, szS, hipMemcpyDeviceToHost, stream_));
        wait_step();
        prof_collect();
        // every automaton's level offsets, packed into one buffer by one copy launch
        std::vector<CopyDesc> cp;
        std::vector<int64_t> pre(1, 0);
        int64_t words = 0;
        for (int i = 0; i < nq; ++i)
            for (int sd = 0; sd < 2; ++sd) words += 2 * ((int64_t)hS[i].nlev[sd] + 1);
        char *dpack = dev_need(pack_blob_, pack_blob_cap_, (size_t)words * 4);
        int64_t o = 0;
        for (int i = 0; i < nq; ++i)
            for (int sd = 0; sd < 2; ++sd) {
                const int64_t cnt = 2 * ((int64_t)hS[i].nlev[sd] + 1);
                cp.push_back(CopyDesc{(const u32 *)(q[i]->d_off + (int64_t)sd * q[i]->max_lev),
                                      (u32 *)dpack + o, cnt});
                pre.push_back(pre.back() + ceil_div(cnt, kCopyPerBlock));
                o += cnt;
            }
        const size_t a = align8(sizeof(CopyDesc) * cp.size()), b = align8(8 * pre.size());
        char *hc = (char *)pin_copy_.acquire(a + b);
        memcpy(hc, cp.data(), sizeof(CopyDesc) * cp.size());
        memcpy(hc + a, pre.data(), 8 * pre.size());
        char *dc = dev_need(copy_blob_, copy_blob_cap_, a + b);
        HIPCHK(hipMemcpyAsync(dc, hc, a + b, hipMemcpyHostToDevice, stream_));
        pin_copy_.issued(stream_);
        HIPCHK(launch_copy((const CopyDesc *)dc, (const int64_t *)(dc + a), (int)cp.size(), pre.back(), stream_));
        stats_.launches[6]++;
        int64_t *hoff = (int64_t *)pin_trace_.need((size_t)words * 4);
        HIPCHK(hipMemcpyAsync(hoff, dpack, (size_t)words * 4, hipMemcpyDeviceToHost, stream_));
        HIPCHK(hipStreamSynchronize(stream_));
        std::vector<Problem *> met;
        std::vector<u64> metbest;
        o = 0;
        for (int i = 0; i < nq; ++i) {
            Problem *p = q[i];
            const RunState &st = hS[i];
            for (int sd = 0; sd < 2; ++sd) {
                SideState &s = p->s[sd];
                s.off.assign(hoff + o, hoff + o + st.nlev[sd] + 1);
                o += st.nlev[sd] + 1;
                s.nrows = st.nrows[sd];
                s.popsum = st.popsum[sd];
            }
            for (int t = 0; t < st.steps; ++t)
                p->sides.push_back(t < 64 * kRunSideWords ? (uint8_t)((st.sides[t >> 6] >> (t & 63)) & 1) : 255);
            p->steps += st.steps;
            stats_.steps += st.steps;
            stats_.candidates += st.candidates;
            stats_.cand_words += st.candidates * p->W;
            stats_.unique += st.unique;
            stats_.pairs += st.pairs;
            stats_.pair_words += st.pairs * p->W;
            stats_.pair_words_w[p->W - 1] += st.pairs * p->W;
            stats_.bytes_expand += 8 * p->W * (st.candidates / p->k + st.candidates);
            stats_.bytes_insert += st.candidates * (8 * p->W + 8 + 4);
            stats_.bytes_compact += st.candidates * 24 + st.unique * (16 * p->W + 12);
            if (st.status == 1) {
                met.push_back(p);
                metbest.push_back(st.best);
            } else if (st.status == 2) {
                finish_error(p, SRW_EINTERNAL, "a list became empty before the searches met");
            }
        }
        if (!met.empty()) trace(met, metbest);
    }

    void finish_error(Problem *p, int code, const char *msg = nullptr) {
        p->status = code;
        p->r = -1;
        p->t_done = now_ms();
        if (msg) t_err = msg;
        release(p);
    }

    // After a step failed on the device memory budget (an allocation of the
    // engine's own per-step buffers found no room even in the reserve): let
    // the queued work finish and drop the copies that step had planned.  The
    // caller then fails the problems of that step with SRW_ENOMEM.
    void recover() {
        (void)hipStreamSynchronize(stream_);
        (void)hipGetLastError();
        for (void *q : pend_free_) pool_->free(q);
        pend_copy_.clear();
        pend_free_.clear();
    }

    // lists of the last kept problem
    Problem *kept() { return kept_; }
    void release_kept() {
        if (kept_) {
            release(kept_, true);
            delete kept_;
            kept_ = nullptr;
        }
    }
    void keep(Problem *p) {
        release_kept();
        kept_ = p;
    }
    hipStream_t stream() const { return stream_; }

    // Beam searches (k_beam), a block per automaton, in groups whose buffers
    // fit the budget.  A search that runs out of rows, candidates or levels
    // is run again with four times the room, up to kBeamTries times.
    struct BeamJob {
        int n = 0, k = 0;
        const int32_t *delta = nullptr;
        int64_t width = 0;
        int64_t index = -1;
        int status = 1;            // 1: not run yet
        int32_t R = -1;
        std::vector<uint8_t> word;
        int64_t rows_cap = 0, max_lev = 0;
        int64_t stats[3] = {0, 0, 0};   // candidates, kept, cut
        bool want_sizes = false;
        std::vector<int64_t> sizes;     // with want_sizes: new sets of each level before its cut
    };
    static constexpr int kBeamTries = 4;
    // rows and candidates of one search at most: its hash table then stays
    // below 2^31 slots (slot positions are 32-bit)
    static constexpr int64_t kBeamMaxRows = (int64_t)1 << 28;
    static constexpr int kBeamGroup = 256;

    void beam(std::vector<BeamJob *> &jobs) {
        HIPCHK(hipSetDevice(device_));
        for (BeamJob *j : jobs) {
            const int64_t wk = std::min<int64_t>(j->width, (int64_t)1 << 24);
            j->rows_cap = std::min<int64_t>(std::max<int64_t>(65536, 32 * (int64_t)j->k * wk + j->n),
                                            (int64_t)1 << 22);
            j->max_lev = std::min<int64_t>((int64_t)j->n * j->n + 2, 4096);
        }
        for (int attempt = 0; attempt < kBeamTries; ++attempt) {
            std::vector<BeamJob *> todo;
            for (BeamJob *j : jobs)
                if (j->status == 1) todo.push_back(j);
            if (todo.empty()) break;
            std::stable_sort(todo.begin(), todo.end(), [](BeamJob *a, BeamJob *b) {
                return (a->n + 63) / 64 < (b->n + 63) / 64;
            });
            for (size_t i0 = 0; i0 < todo.size(); i0 += kBeamGroup) {
                std::vector<BeamJob *> grp(todo.begin() + i0,
                                           todo.begin() + std::min(todo.size(), i0 + kBeamGroup));
                beam_group(grp);
            }
            for (BeamJob *j : todo)
                if (j->status == 1) {          // out of room: more of it next time
                    j->rows_cap = std::min<int64_t>(4 * j->rows_cap, kBeamMaxRows);
                    j->max_lev = std::min<int64_t>(4 * j->max_lev, (int64_t)1 << 20);
                }
        }
        for (BeamJob *j : jobs)
            if (j->status == 1) j->status = SRW_ENOMEM;
    }

    // Eppstein's heuristic (k_eppstein), a block per automaton, in groups
    // whose buffers fit the budget.  The word buffer starts at a guess; a
    // longer word (its length is always returned) is computed again with
    // room for all of it, so that every word is checked on the host.
    struct EppJob {
        int n = 0, k = 0;
        const int32_t *delta = nullptr;
        int64_t index = -1;
        int status = 1;            // 1: not done yet
        int64_t len = -1, dcap = 0;
        int32_t rounds = 0;
        std::vector<uint8_t> word;
    };
    static constexpr int kEppGroup = 2048;    // blocks of one launch (about 1.7 MB each at n = 512)
    void eppstein(std::vector<EppJob *> &jobs) {
        HIPCHK(hipSetDevice(device_));
        for (EppJob *j : jobs) j->dcap = 4 * (int64_t)j->n + 64;
        for (int attempt = 0; attempt < 2; ++attempt) {
            std::vector<EppJob *> todo;
            for (EppJob *j : jobs)
                if (j->status == 1) todo.push_back(j);
            for (size_t i0 = 0; i0 < todo.size(); i0 += kEppGroup) {
                std::vector<EppJob *> grp(todo.begin() + i0,
                                          todo.begin() + std::min(todo.size(), i0 + kEppGroup));
                eppstein_group(grp);
            }
            for (EppJob *j : todo)
                if (j->status == 1) j->dcap = j->len;     // the whole word next time
        }
        for (EppJob *j : jobs)
            if (j->status == 1) j->status = SRW_EINTERNAL;
    }

  private:
    static size_t align8(size_t x) { return (x + 7) & ~(size_t)7; }

    void eppstein_group(std::vector<EppJob *> &grp) {
        const int cnt = (int)grp.size();
        std::vector<EppDesc> D(cnt);
        std::vector<size_t> at(cnt + 1, 0);
        // [states | words | descriptors | tables | per-automaton buffers]:
        // states and words come back in one copy
        std::vector<size_t> woff(cnt + 1, 0);
        for (int i = 0; i < cnt; ++i) woff[i + 1] = woff[i] + (size_t)grp[i]->dcap;
        const size_t wbase = align8(sizeof(EppState) * (size_t)cnt);
        size_t head = wbase + align8(woff[cnt]) + align8(sizeof(EppDesc) * (size_t)cnt);
        std::vector<int64_t> doff(cnt + 1, 0);
        for (int i = 0; i < cnt; ++i) doff[i + 1] = doff[i] + (int64_t)grp[i]->n * grp[i]->k;
        head += align8((size_t)doff[cnt] * 2);
        at[0] = head;
        for (int i = 0; i < cnt; ++i) {
            const size_t n = (size_t)grp[i]->n, k = (size_t)grp[i]->k, P = n * (n - 1) / 2;
            at[i + 1] = at[i] + align8(4 * P) + align8(P) + align8(8 * P) + align8(2 * k * n) +
                        align8(4 * k * (n + 1)) + align8(4 * k * n);
        }
        char *base = (char *)pool_->alloc(at[cnt]);
        if (!base) {
            if (cnt == 1) {
                grp[0]->status = SRW_ENOMEM;
                return;
            }
            std::vector<EppJob *> a(grp.begin(), grp.begin() + cnt / 2), b(grp.begin() + cnt / 2, grp.end());
            eppstein_group(a);
            eppstein_group(b);
            return;
        }
        EppState *dst = (EppState *)base;
        uint8_t *dwords = (uint8_t *)(base + wbase);
        EppDesc *dd = (EppDesc *)(base + wbase + align8(woff[cnt]));
        uint16_t *dl = (uint16_t *)((char *)dd + align8(sizeof(EppDesc) * (size_t)cnt));
        std::vector<uint16_t> d16((size_t)doff[cnt]);
        for (int i = 0; i < cnt; ++i)
            for (int64_t t = 0; t < doff[i + 1] - doff[i]; ++t) d16[(size_t)(doff[i] + t)] = (uint16_t)grp[i]->delta[t];
        for (int i = 0; i < cnt; ++i) {
            EppJob *j = grp[i];
            const size_t n = (size_t)j->n, k = (size_t)j->k, P = n * (n - 1) / 2;
            EppDesc &e = D[i];
            memset(&e, 0, sizeof e);
            char *c = base + at[i];
            e.n = j->n;
            e.k = j->k;
            e.delta = dl + doff[i];
            e.dist = (u32 *)c;            c += align8(4 * P);
            e.next = (uint8_t *)c;        c += align8(P);
            e.queue = (u32 *)c;           c += align8(8 * P);
            e.inv = (uint16_t *)c;        c += align8(2 * k * n);
            e.inv_off = (u32 *)c;         c += align8(4 * k * (n + 1));
            e.inv_cur = (u32 *)c;
            e.word = dwords + woff[i];
            e.word_cap = j->dcap;
            if (opt.deadline_ms > 0) e.max_ticks = std::max<int64_t>(1, (int64_t)(opt.deadline_ms * wall_khz_));
            e.st = dst + i;
        }
        HIPCHK(hipMemcpyAsync(dl, d16.data(), d16.size() * 2, hipMemcpyHostToDevice, stream_));
        HIPCHK(hipMemcpyAsync(dd, D.data(), sizeof(EppDesc) * (size_t)cnt, hipMemcpyHostToDevice, stream_));
        HIPCHK(launch_eppstein(dd, cnt, stream_));
        std::vector<char> back(wbase + woff[cnt]);
        HIPCHK(hipMemcpyAsync(back.data(), base, back.size(), hipMemcpyDeviceToHost, stream_));
        HIPCHK(hipStreamSynchronize(stream_));
        const EppState *S = (const EppState *)back.data();
        std::vector<char> check(cnt, 0);
        int64_t vwork = 0;
        for (int i = 0; i < cnt; ++i) {
            EppJob *j = grp[i];
            const EppState &t = S[i];
            j->rounds = t.rounds;
            if (t.status == 4) {
                j->status = SRW_ETIMEOUT;
            } else if (t.status == 5) {
                // a pair of the current set that no word merges: the
                // automaton is not synchronizing (the pair test of the
                // search over pairs)
                j->status = SRW_ENOTSYNC;
            } else if (t.status != 1) {
                j->status = SRW_EINTERNAL;
                t_err = "Eppstein: unexpected kernel status";
            } else if (t.len > j->dcap) {
                j->len = t.len;                    // again, with room for all of it
            } else {
                j->len = t.len;
                j->word.assign(back.data() + wbase + woff[i], back.data() + wbase + woff[i] + t.len);
                check[i] = 1;
                vwork += t.len * j->n;
            }
        }
        pool_->free(base);
        // every word is checked on the host, on host threads
        parallel_for(cnt, vwork, [&](int64_t i) {
            if (!check[(size_t)i]) return;
            EppJob *j = grp[(size_t)i];
            j->status = verify_word(j->n, j->k, j->delta, j->word.data(), j->len) ? SRW_OK : SRW_EINTERNAL;
        });
        for (int i = 0; i < cnt; ++i)
            if (check[i] && grp[i]->status != SRW_OK) t_err = "Eppstein word does not reset the automaton";
    }

    // one group of beam searches: buffers, one launch per set width, results
    void beam_group(std::vector<BeamJob *> &grp) {
        const int cnt = (int)grp.size();
        std::vector<BeamDesc> D(cnt);
        std::vector<void *> blocks;
        auto A = [&](size_t bytes) -> void * {
            void *q = pool_->alloc(bytes);
            if (q) blocks.push_back(q);
            return q;
        };
        char *dst = (char *)A(sizeof(BeamState) * (size_t)cnt);
        BeamDesc *dd = (BeamDesc *)A(sizeof(BeamDesc) * (size_t)cnt);
        // every transition table of the group in one upload
        std::vector<int64_t> doff(cnt + 1, 0);
        for (int i = 0; i < cnt; ++i) doff[i + 1] = doff[i] + (int64_t)grp[i]->n * grp[i]->k;
        std::vector<uint16_t> d16((size_t)doff[cnt]);
        for (int i = 0; i < cnt; ++i)
            for (int64_t t = 0; t < doff[i + 1] - doff[i]; ++t) d16[(size_t)(doff[i] + t)] = (uint16_t)grp[i]->delta[t];
        uint16_t *dl = (uint16_t *)A(d16.size() * 2);
        bool ok = dst && dd && dl;
        for (int i = 0; i < cnt && ok; ++i) {
            BeamJob *j = grp[i];
            const int W = (j->n + 63) / 64;
            BeamDesc &b = D[i];
            memset(&b, 0, sizeof b);
            b.n = j->n;
            b.k = j->k;
            b.W = W;
            b.max_lev = (int32_t)j->max_lev;
            b.beam = j->width;
            b.rows_cap = j->rows_cap;
            b.cand_cap = std::min<int64_t>(kBeamMaxRows, std::max<int64_t>(
                j->n, (int64_t)j->k * std::min<int64_t>(j->width, j->rows_cap)));
            int64_t slots = 1;
            while (slots < 2 * (b.rows_cap + b.cand_cap)) slots <<= 1;
            b.tab_mask = (u64)(slots - 1);
            b.rows = (u64 *)A((size_t)b.rows_cap * W * 8);
            b.par = (u32 *)A((size_t)b.rows_cap * 4);
            b.tab = (u64 *)A((size_t)slots * 8);
            b.cand = (u64 *)A((size_t)b.cand_cap * W * 8);
            b.cslot = (u32 *)A((size_t)b.cand_cap * 4);
            b.lev = (int64_t *)A((size_t)j->max_lev * 3 * 8);
            b.word = (uint8_t *)A((size_t)j->max_lev);
            b.st = (BeamState *)(dst + sizeof(BeamState) * (size_t)i);
            if (opt.deadline_ms > 0) b.max_ticks = std::max<int64_t>(1, (int64_t)(opt.deadline_ms * wall_khz_));
            ok = b.rows && b.par && b.tab && b.cand && b.cslot && b.lev && b.word;
            if (!ok) break;
            b.delta = dl + doff[i];
            HIPCHK(launch_fill(b.tab, slots, kEmpty, stream_));
        }
        if (!ok) {
            // no room for the whole group: halve it (one automaton that does
            // not fit ends with SRW_ENOMEM)
            HIPCHK(hipStreamSynchronize(stream_));
            for (void *q : blocks) pool_->free(q);
            if (cnt == 1) {
                grp[0]->status = SRW_ENOMEM;
                return;
            }
            std::vector<BeamJob *> a(grp.begin(), grp.begin() + cnt / 2), b(grp.begin() + cnt / 2, grp.end());
            beam_group(a);
            beam_group(b);
            return;
        }
        HIPCHK(hipMemcpyAsync(dl, d16.data(), d16.size() * 2, hipMemcpyHostToDevice, stream_));
        HIPCHK(hipMemcpyAsync(dd, D.data(), sizeof(BeamDesc) * (size_t)cnt, hipMemcpyHostToDevice, stream_));
        for (int i0 = 0; i0 < cnt;) {
            int i1 = i0;
            const int W = D[i0].W;
            while (i1 < cnt && D[i1].W == W) ++i1;
            HIPCHK(launch_beam(dd + i0, i1 - i0, W, stream_));
            i0 = i1;
        }
        std::vector<BeamState> S(cnt);
        HIPCHK(hipMemcpyAsync(S.data(), dst, sizeof(BeamState) * (size_t)cnt, hipMemcpyDeviceToHost, stream_));
        HIPCHK(hipStreamSynchronize(stream_));
        for (int i = 0; i < cnt; ++i) {
            BeamJob *j = grp[i];
            const BeamState &t = S[i];
            j->stats[0] = t.candidates;
            j->stats[1] = t.kept;
            j->stats[2] = t.cut;
            if (j->want_sizes && (t.status == 1 || t.status == 2) && t.nlev > 0) {
                std::vector<int64_t> lev((size_t)t.nlev * 3);
                HIPCHK(hipMemcpy(lev.data(), D[i].lev, lev.size() * 8, hipMemcpyDeviceToHost));
                j->sizes.resize((size_t)t.nlev);
                for (int L = 0; L < t.nlev; ++L) j->sizes[(size_t)L] = lev[3 * (size_t)L + 2] - lev[3 * (size_t)L];
            }
            if (t.status == 1) {
                j->R = t.R;
                j->word.resize((size_t)t.R);
                if (t.R > 0)
                    HIPCHK(hipMemcpy(j->word.data(), D[i].word, (size_t)t.R, hipMemcpyDeviceToHost));
                j->status = verify_word(j->n, j->k, j->delta, j->word.data(), t.R) ? SRW_OK : SRW_EINTERNAL;
                if (j->status != SRW_OK) t_err = "beam word does not reset the automaton";
            } else if (t.status == 2) {
                j->status = SRW_ENOBOUND;
            } else if (t.status == 4) {
                j->status = SRW_ETIMEOUT;
            } else {
                j->status = 1;                   // out of room: again, larger
            }
        }
        for (void *q : blocks) pool_->free(q);
    }

    // the automata of this engine start with k_run_small (it keeps the side
    // rule of schedule 0 and the LDS-tile meet of one-block steps)
    // the meet's operation counters, once profiling is on
    void ensure_ops() {
        if (opt.profile && !d_ops_) {
            d_ops_ = (u64 *)pool_->alloc((kOpsWords + kMstatWords) * sizeof(u64), true);
            if (!d_ops_) throw HipFailure{hipErrorOutOfMemory, "meet counters"};
            HIPCHK(launch_fill(d_ops_, kOpsWords + kMstatWords, 0, stream_));
        }
    }

    // (schedule 3 leaves the first, small steps to the runner's side rule)
    bool persist_ok(int W) const {
        return opt.persist && opt.small(W) > 0 && (opt.sched(W) == 0 || opt.sched(W) == 3) && opt.meet != 2 &&
               !opt.reduce;
    }
    static constexpr int64_t kPersistRows = 16384;   // rows per side while k_run_small steps
    static constexpr int64_t kPersistCand = 8192;    // candidates of its largest step
    static constexpr int64_t kPersistLevels = 4096;  // levels per side it can record

    int choose_side(Problem *p) {
        const int64_t lf = p->s[0].cur(), lb = p->s[1].cur();
        switch (opt.sched(p->W)) {
            case 1: return (int)(mix64(opt.sched_seed * 0x9E3779B97F4A7C15ull + (uint64_t)p->steps +
                                       ((uint64_t)p->index << 32)) & 1);
            case 2: return p->steps & 1;
            case 3: return cost_side(*p);
            default: return lb < lf ? 1 : 0;   // smaller list first, ties forward
        }
    }

    // The estimate ExpMark (Section 2.1.2) of the subset tests of marking
    // the sets of a list of Bs sets of density Bd that contain one of a list
    // of As sets of density Ad.
    static double exp_mark(double As, double Bs, double Ad, double Bd) {
        if (As <= 0 || Bs <= 0) return 0.0;
        const double w = (1.0 + Bd) / (1.0 + Ad * Bd - Ad);
        const double e = std::log1p(Bd) / std::log(w);
        return Bs * ((1.0 + Bd) / Bd + 1.0 / (Ad - Ad * Bd)) * std::pow(As, e);
    }

    // Schedule 3: the step of lower estimated cost (Section 2.1.2, Eq. 1-4)
    // among the two this search has, BFS and IBFS, both with their history
    // (there is no step without it and no DFS phase, so the rule is the
    // paper's greedy comparison of the two single-step costs).  A step costs
    // SetCost (512) per candidate plus ExpMark of its meet test; the terms
    // of Eq. 2 and 3 price inclusion reductions that this search does not
    // make, and are zero.  The fraction of candidates a side's duplicate
    // removal keeps is taken from its last step (1 before its first);
    // densities are clamped to [1/(2n), 1 - 1/(2n)].  Ties go forward.
    int cost_side(const Problem &p) const {
        const double n = p.n, k = p.k, set_cost = 512.0;
        const double lo = 0.5 / n, hi = 1.0 - 0.5 / n;
        const SideState &F = p.s[0], &B = p.s[1];
        const double lf = (double)F.cur(), lb = (double)B.cur();
        auto dens = [&](const SideState &s, double m) {
            return std::min(hi, std::max(lo, m > 0 ? (double)s.popsum / (n * m) : lo));
        };
        auto keep = [&](const SideState &s) {
            return s.prev() > 0 ? (double)s.cur() / (k * (double)s.prev()) : 1.0;
        };
        const double df = dens(F, lf), db = dens(B, lb);
        const double bfs = set_cost * k * lf + exp_mark(k * keep(F) * lf, lb, df, db);
        const double ibfs = set_cost * k * lb + exp_mark(lf, k * keep(B) * lb, df, db);
        return ibfs < bfs ? 1 : 0;
    }

    bool dev_grow(void *&ptr, int64_t &cap, int64_t need, size_t elem, int64_t keep) {
        if (need <= cap) return true;
        const int64_t nc = std::max(need, cap * 2);
        void *q = pool_->alloc((size_t)nc * elem);
        if (!q) return false;
        if (ptr && keep > 0) {
            // copied by flush_copies in one launch with the step's other
            // grown buffers; the old block stays allocated until that launch
            // is enqueued, so no buffer grown in the same step can reuse it
            pend_copy_.push_back(CopyDesc{(const u32 *)ptr, (u32 *)q, (int64_t)((size_t)keep * elem / 4)});
            pend_free_.push_back(ptr);
        } else {
            pool_->free(ptr);
        }
        ptr = q;
        cap = nc;
        return true;
    }

    // buffers for the cardinality order of an inverse level of up to C sets
    bool ensure_ysort(Problem *p, int64_t C) {
        if (!p->ys_hist) {
            p->ys_hist = (u32 *)pool_->alloc((size_t)(p->n + 1) * 4);
            p->ys_cnt = (u32 *)pool_->alloc((size_t)(p->n + 2) * 4);
            if (!p->ys_hist || !p->ys_cnt) return false;
        }
        void *pp = p->ys_idx;
        int64_t cap = p->ys_cap;
        if (!dev_grow(pp, cap, C, 4, 0)) return false;
        p->ys_idx = (u32 *)pp;
        p->ys_cap = cap;
        return true;
    }

    void flush_copies() {
        if (pend_copy_.empty()) return;
        std::vector<int64_t> pre(1, 0);
        for (const CopyDesc &c : pend_copy_) pre.push_back(pre.back() + ceil_div(c.count, kCopyPerBlock));
        const size_t a = align8(sizeof(CopyDesc) * pend_copy_.size()), b = align8(8 * pre.size());
        char *h = (char *)pin_copy_.acquire(a + b);
        memcpy(h, pend_copy_.data(), sizeof(CopyDesc) * pend_copy_.size());
        memcpy(h + a, pre.data(), 8 * pre.size());
        char *d = dev_need(copy_blob_, copy_blob_cap_, a + b);
        HIPCHK(hipMemcpyAsync(d, h, a + b, hipMemcpyHostToDevice, stream_));
        pin_copy_.issued(stream_);
        HIPCHK(launch_copy((const CopyDesc *)d, (const int64_t *)(d + a), (int)pend_copy_.size(), pre.back(),
                           stream_));
        stats_.launches[6]++;
        for (void *q : pend_free_) pool_->free(q);
        pend_copy_.clear();
        pend_free_.clear();
    }

    // make room for one step of side `dir`; returns 0 or an SRW_ error
    int prepare(Problem *p, int dir, std::vector<RehashDesc> &grow, std::vector<int64_t> &growpre) {
        SideState &s = p->s[dir];
        const int W = p->W;
        const int64_t C = s.cur() * p->k;
        if (C >= (int64_t)kCandBit - 1 || s.nrows + C >= (int64_t)kCandBit - 1)
            return set_error(SRW_ENOMEM, "list size beyond 2^31");
        void *pp;
        int64_t cap;
        if (opt.reduce) {
            // rows and ghosts are named by refs below kGhostBit
            if (s.nrows + s.nghost + C >= (int64_t)kGhostBit)
                return set_error(SRW_ENOMEM, "list size beyond 2^30 with reductions");
            pp = s.ghost; cap = s.ghost_cap;
            if (!dev_grow(pp, cap, s.nghost + C, (size_t)W * 8, s.nghost))
                return set_error(SRW_ENOMEM, "device budget (dropped sets)");
            s.ghost = (u64 *)pp; s.ghost_cap = cap;
            pp = p->mark; cap = p->red_cap;
            if (!dev_grow(pp, cap, C, 4, 0)) return set_error(SRW_ENOMEM, "device budget (reduction)");
            p->mark = (u32 *)pp;
            pp = p->red_par; cap = p->red_cap;
            if (!dev_grow(pp, cap, C, 4, 0)) return set_error(SRW_ENOMEM, "device budget (reduction)");
            p->red_par = (u32 *)pp; p->red_cap = cap;
        }
        pp = p->cand; cap = p->cand_cap;
        if (!dev_grow(pp, cap, C, (size_t)W * 8, 0)) return set_error(SRW_ENOMEM, "device budget (candidates)");
        p->cand = (u64 *)pp; p->cand_cap = cap;
        pp = p->cslot; cap = p->cslot_cap;
        if (!dev_grow(pp, cap, C, 4, 0)) return set_error(SRW_ENOMEM, "device budget (slots)");
        p->cslot = (u32 *)pp; p->cslot_cap = cap;
        if (s.nrows + C > s.cap) {
            int64_t c1 = s.cap, c2 = s.cap;
            pp = s.rows;
            if (!dev_grow(pp, c1, s.nrows + C, (size_t)W * 8, s.nrows)) return set_error(SRW_ENOMEM, "device budget (rows)");
            s.rows = (u64 *)pp;
            pp = s.par;
            if (!dev_grow(pp, c2, s.nrows + C, 4, s.nrows)) return set_error(SRW_ENOMEM, "device budget (parents)");
            s.par = (u32 *)pp;
            s.cap = c1;
        }
        if (2 * (s.nrows + s.nghost + C) > s.tab_cap) {
            int64_t nc = s.tab_cap;
            while (2 * (s.nrows + s.nghost + C) > nc) nc <<= 1;
            nc = std::max(nc, 2 * s.tab_cap);
            if (nc > ((int64_t)1 << 31)) return set_error(SRW_ENOMEM, "hash table beyond 2^31 slots");
            void *t = pool_->alloc((size_t)nc * 8);
            if (!t) return set_error(SRW_ENOMEM, "device budget (hash table)");
            pool_->free(s.tab);
            s.tab = (u64 *)t;
            s.tab_cap = nc;
            grow.push_back(RehashDesc{W, 0, s.rows, s.nrows, s.tab, (u64)(nc - 1)});
            growpre.push_back(growpre.back() + ceil_div(s.nrows, kBS));
            if (s.nghost > 0) {                  // the dropped sets stay visited
                grow.push_back(RehashDesc{W, (int32_t)kGhostBit, s.ghost, s.nghost, s.tab, (u64)(nc - 1)});
                growpre.push_back(growpre.back() + ceil_div(s.nghost, kBS));
            }
        }
        if (dir == 1) {
            pp = p->colT; cap = p->colT_cap;
            if (!dev_grow(pp, cap, ceil_div(C, 64) * 64 * W, 16, 0)) return set_error(SRW_ENOMEM, "device budget (tiles)");
            p->colT = (u64 *)pp; p->colT_cap = cap;
            pp = p->ysig; cap = p->ysig_cap;
            if (!dev_grow(pp, cap, ceil_div(C, 64) * 64, 8, 0)) return set_error(SRW_ENOMEM, "device budget (signatures)");
            p->ysig = (u64 *)pp; p->ysig_cap = cap;
        }
        p->sort_now = false;
        p->yb_now = false;
        const int64_t nY = p->s[1].cur();
        if (dir == 0 && opt.meet != 1) {
            // a bucketed inverse level is met only by a sorted forward level
            const bool want = opt.meet == 2 || p->yb_valid ||
                              (C >= kSortMinCand && (double)C * (double)nY >= kSortMinPairs);
            if (want) p->sort_now = ensure_sort(p, C);   // no room: the LDS-tile meet serves
            if (!p->sort_now && p->yb_valid) return set_error(SRW_ENOMEM, "device budget (sort)");
            if (p->sort_now && !p->yb_valid && bucket_ok(W) && nY >= opt.bucket_min(W)) p->yb_now = true;
        } else if (dir == 1 && bucket_ok(W) && p->xs_valid && C >= opt.bucket_min(W)) {
            p->yb_now = true;
        }
        if (p->yb_now) {
            const int64_t yub = dir == 1 ? C : nY;    // sets of the level to bucket
            const int64_t nt_ub = ceil_div(yub, 64) + kYBins;
            if (!ensure_ybin(p, yub, nt_ub)) {
                p->yb_now = false;                     // no room: level order
            } else {
                pp = p->colT; cap = p->colT_cap;
                if (!dev_grow(pp, cap, nt_ub * 64 * W, 16, 0)) return set_error(SRW_ENOMEM, "device budget (tiles)");
                p->colT = (u64 *)pp; p->colT_cap = cap;
                pp = p->ysig; cap = p->ysig_cap;
                if (!dev_grow(pp, cap, nt_ub * 64, 8, 0)) return set_error(SRW_ENOMEM, "device budget (signatures)");
                p->ysig = (u64 *)pp; p->ysig_cap = cap;
            }
        }
        if (bucketed_meet(p, dir)) {
            const int64_t nch = ceil_div(dir == 0 ? C : p->s[0].cur(), 64) + 1;
            if (!ensure_plan(p, nch)) return set_error(SRW_ENOMEM, "device budget (meet plan)");
        }
        return 0;
    }

    bool bucket_ok(int W) const { return opt.bucket_min(W) > 0 && opt.ysort == 0 && opt.meet != 1; }
    // this step's meet runs against the inverse level in buckets (mode 2)
    static bool bucketed_meet(const Problem *p, int dir) {
        return dir == 0 ? (p->sort_now && (p->yb_valid || p->yb_now)) : (p->xs_valid && p->yb_now);
    }

    static constexpr size_t kYbSmallWords = 2 * kYBins + (kYBins + 1) + kYBins + (kYBins + 1) + kYBins;
    static size_t yb_small_bytes() { return 256 + kYbSmallWords * 4; }
    static YbMeta *yb_meta(Problem *p) { return (YbMeta *)p->yb_small; }
    static u32 *yb_words(Problem *p) { return (u32 *)(p->yb_small + 256); }

    // buffers for bucketing an inverse level of up to `count` sets
    bool ensure_ybin(Problem *p, int64_t count, int64_t nt_ub) {
        if (!p->yb_small) {
            p->yb_small = (char *)pool_->alloc(yb_small_bytes());
            if (!p->yb_small) return false;
        }
        void *q = p->yb_key;
        int64_t cap = p->yb_key_cap;
        if (!dev_grow(q, cap, count, 2, 0)) return false;
        p->yb_key = (uint16_t *)q;
        p->yb_key_cap = cap;
        q = p->yb_idx;
        cap = p->yb_idx_cap;
        if (!dev_grow(q, cap, nt_ub * 64, 4, 0)) return false;
        p->yb_idx = (u32 *)q;
        p->yb_idx_cap = cap;
        q = p->yb_list;
        cap = p->yb_list_cap;
        if (!dev_grow(q, cap, kYListPerTile * nt_ub, 4, 0)) return false;
        p->yb_list = (u32 *)q;
        p->yb_list_cap = cap;
        return true;
    }

    // plan buffers of a bucketed meet over `nch` chunks
    bool ensure_plan(Problem *p, int64_t nch) {
        if (nch <= p->mp_cap && p->mp_queue) return true;
        pool_->free(p->mp_key);
        pool_->free(p->mp_order);
        pool_->free(p->mp_cpre);
        const int64_t nc = std::max(nch, 2 * p->mp_cap);
        p->mp_key = (u32 *)pool_->alloc((size_t)nc * 4);
        p->mp_order = (u32 *)pool_->alloc((size_t)nc * 4);
        p->mp_cpre = (u32 *)pool_->alloc((size_t)(nc + 1) * 4);
        if (!p->mp_kinfo) p->mp_kinfo = (u32 *)pool_->alloc((size_t)kKInfoWords * 4);
        if (!p->mp_queue) p->mp_queue = (u32 *)pool_->alloc(256);
        p->mp_cap = (p->mp_key && p->mp_order && p->mp_cpre && p->mp_kinfo && p->mp_queue) ? nc : 0;
        return p->mp_cap > 0;
    }

    bool ensure_sort(Problem *p, int64_t rows) {
        const int W = p->W;
        if (!p->xs_bins) {
            p->xs_bins = (u32 *)pool_->alloc((size_t)kSortBins * 4);
            p->xs_hist = (u32 *)pool_->alloc((size_t)kMaxW * 64 * 4);
            p->xs_top = (int32_t *)pool_->alloc((size_t)kKeyBits * 4);
            if (!p->xs_bins || !p->xs_hist || !p->xs_top) return false;
        }
        if (rows > p->xs_cap) {
            p->xs_valid = false;
            pool_->free(p->xs_rows);
            pool_->free(p->xs_idx);
            pool_->free(p->xs_keys);
            pool_->free(p->xs_com);
            const int64_t nc = std::max(rows, 2 * p->xs_cap);
            p->xs_rows = (u64 *)pool_->alloc((size_t)nc * W * 8);
            p->xs_idx = (u32 *)pool_->alloc((size_t)nc * 4);
            p->xs_keys = (u32 *)pool_->alloc((size_t)nc * 4);
            p->xs_com = (u64 *)pool_->alloc((size_t)ceil_div(nc, 64) * W * 8);
            p->xs_cap = (p->xs_rows && p->xs_idx && p->xs_keys && p->xs_com) ? nc : 0;
            if (!p->xs_cap) return false;
        }
        return true;
    }

    void trace(std::vector<Problem *> &met, std::vector<u64> &best) {
        const int cnt = (int)met.size();
        size_t offs = 0, words = 0;
        for (Problem *p : met) {
            offs += p->s[0].off.size() + p->s[1].off.size();
            words += p->s[0].nlev() - 1 + p->s[1].nlev() - 1;
        }
        const size_t szT = align8(sizeof(TraceDesc) * cnt), szO = align8(8 * offs);
        const size_t total = szT + szO + align8(words);
        char *h = (char *)pin_trace_.need(total);
        char *dblob = dev_need(trace_blob_, trace_blob_cap_, total);
        TraceDesc *T = (TraceDesc *)h;
        int64_t *O = (int64_t *)(h + szT);
        size_t oo = 0, wo = 0;
        for (int t = 0; t < cnt; ++t) {
            Problem *p = met[t];
            const int f = p->s[0].nlev() - 1, b = p->s[1].nlev() - 1;
            TraceDesc &d = T[t];
            d.par_f = p->s[0].par;
            d.off_f = (const int64_t *)(dblob + szT) + oo;
            memcpy(O + oo, p->s[0].off.data(), 8 * p->s[0].off.size());
            oo += p->s[0].off.size();
            d.par_b = p->s[1].par;
            d.off_b = (const int64_t *)(dblob + szT) + oo;
            memcpy(O + oo, p->s[1].off.data(), 8 * p->s[1].off.size());
            oo += p->s[1].off.size();
            d.i = (int64_t)(best[t] >> 32);
            d.j = (int64_t)(best[t] & 0xFFFFFFFFull);
            d.f = f;
            d.b = b;
            d.k = p->k;
            d.out = (uint8_t *)(dblob + szT + szO + wo);
            p->r = f + b;
            wo += (size_t)(f + b);
        }
        prof_begin(5);
        HIPCHK(hipMemcpyAsync(dblob, h, szT + szO, hipMemcpyHostToDevice, stream_));
        HIPCHK(launch_trace((const TraceDesc *)dblob, cnt, stream_));
        if (words) HIPCHK(hipMemcpyAsync(h + szT + szO, dblob + szT + szO, words, hipMemcpyDeviceToHost, stream_));
        prof_end(5);
        stats_.launches[5]++;
        HIPCHK(hipStreamSynchronize(stream_));
        prof_collect();
        wo = 0;
        for (int t = 0; t < cnt; ++t) {
            Problem *p = met[t];
            p->word.assign((uint8_t *)h + szT + szO + wo, (uint8_t *)h + szT + szO + wo + p->r);
            wo += p->r;
            p->t_done = now_ms();
            if (!verify_word(p->n, p->k, p->delta.data(), p->word.data(), p->r)) {
                p->status = SRW_EINTERNAL;
                t_err = "returned word does not reset the automaton";
            } else {
                p->status = SRW_OK;
            }
            stats_.solves++;
            if (!opt.keep_levels) release(p);
        }
    }

  public:
    // device bytes held by the problem's buffers (they only grow, so at the
    // end of a search this is its footprint)
    int64_t footprint(const Problem *p) const {
        int64_t b = 0;
        for (const void *q : {(const void *)p->d_delta, (const void *)p->colT, (const void *)p->ysig,
                              (const void *)p->d_off, (const void *)p->yb_small, (const void *)p->yb_key,
                              (const void *)p->yb_idx, (const void *)p->yb_list, (const void *)p->mp_key,
                              (const void *)p->mp_order, (const void *)p->mp_cpre, (const void *)p->mp_kinfo,
                              (const void *)p->mp_queue, (const void *)p->ys_hist, (const void *)p->ys_cnt,
                              (const void *)p->ys_idx, (const void *)p->cand, (const void *)p->cslot,
                              (const void *)p->xs_rows, (const void *)p->xs_com, (const void *)p->xs_idx,
                              (const void *)p->xs_keys, (const void *)p->xs_hist, (const void *)p->xs_bins,
                              (const void *)p->xs_top, (const void *)p->mark, (const void *)p->red_par})
            b += pool_->size_of(q);
        for (int sd = 0; sd < 2; ++sd)
            b += pool_->size_of(p->s[sd].rows) + pool_->size_of(p->s[sd].par) + pool_->size_of(p->s[sd].tab) +
                 pool_->size_of(p->s[sd].ghost);
        return b;
    }

    void release(Problem *p, bool force = false) {
        (void)force;
        p->dev_bytes = std::max(p->dev_bytes, footprint(p));
        pool_->free(p->d_delta); p->d_delta = nullptr;
        for (int sd = 0; sd < 2; ++sd) {
            pool_->free(p->s[sd].rows); p->s[sd].rows = nullptr;
            pool_->free(p->s[sd].par); p->s[sd].par = nullptr;
            pool_->free(p->s[sd].tab); p->s[sd].tab = nullptr;
            pool_->free(p->s[sd].ghost); p->s[sd].ghost = nullptr;
            p->s[sd].ghost_cap = p->s[sd].nghost = 0;
            p->s[sd].cap = p->s[sd].tab_cap = 0;
        }
        pool_->free(p->colT); p->colT = nullptr; p->colT_cap = 0;
        pool_->free(p->ysig); p->ysig = nullptr; p->ysig_cap = 0;
        pool_->free(p->d_off); p->d_off = nullptr; p->max_lev = 0;
        for (void *q : {(void *)p->yb_small, (void *)p->yb_key, (void *)p->yb_idx, (void *)p->yb_list,
                        (void *)p->mp_key, (void *)p->mp_order, (void *)p->mp_cpre, (void *)p->mp_kinfo,
                        (void *)p->mp_queue})
            pool_->free(q);
        p->yb_small = nullptr;
        p->yb_key = nullptr;
        p->yb_idx = p->yb_list = nullptr;
        p->yb_key_cap = p->yb_idx_cap = p->yb_list_cap = 0;
        p->mp_key = nullptr;
        p->mp_order = p->mp_cpre = p->mp_kinfo = p->mp_queue = nullptr;
        p->mp_cap = 0;
        p->yb_valid = p->yb_now = false;
        pool_->free(p->ys_hist); pool_->free(p->ys_cnt); pool_->free(p->ys_idx);
        p->ys_hist = p->ys_cnt = p->ys_idx = nullptr;
        p->ys_cap = 0;
        p->ys_valid = false;
        pool_->free(p->cand); p->cand = nullptr; p->cand_cap = 0;
        pool_->free(p->mark); pool_->free(p->red_par);
        p->mark = p->red_par = nullptr;
        p->red_cap = 0;
        pool_->free(p->cslot); p->cslot = nullptr; p->cslot_cap = 0;
        for (void *q : {(void *)p->xs_rows, (void *)p->xs_com, (void *)p->xs_idx, (void *)p->xs_keys,
                        (void *)p->xs_hist, (void *)p->xs_bins, (void *)p->xs_top})
            pool_->free(q);
        p->xs_rows = p->xs_com = nullptr;
        p->xs_idx = p->xs_keys = p->xs_hist = p->xs_bins = nullptr;
        p->xs_top = nullptr;
        p->xs_cap = 0;
        p->xs_valid = false;
        stats_.peak_device_bytes = std::max<int64_t>(stats_.peak_device_bytes, pool_->peak());
    }

  private:
    char *dev_need(void *&p, int64_t &cap, size_t bytes) {
        if ((int64_t)bytes > cap) {
            pool_->free(p);
            cap = std::max<int64_t>((int64_t)bytes, 2 * cap);
            p = pool_->alloc((size_t)cap, true);
            if (!p) throw HipFailure{hipErrorOutOfMemory, "descriptor blob"};
        }
        return (char *)p;
    }

    template <class T>
    void *upload_simple(const std::vector<T> &v, const std::vector<int64_t> &pre, void *&blob) {
        const size_t a = align8(sizeof(T) * v.size()), b = align8(8 * pre.size());
        char *h = (char *)pin_misc_.acquire(a + b);
        memcpy(h, v.data(), sizeof(T) * v.size());
        memcpy(h + a, pre.data(), 8 * pre.size());
        char *d = dev_need(blob, misc_blob_cap_, a + b);
        HIPCHK(hipMemcpyAsync(d, h, a + b, hipMemcpyHostToDevice, stream_));
        pin_misc_.issued(stream_);
        return d;
    }

    char *upload3(const std::vector<InitDesc> &a, const std::vector<int64_t> &ap,
                  const std::vector<RehashDesc> &b, const std::vector<int64_t> &bp,
                  const std::vector<TransposeDesc> &c, const std::vector<int64_t> &cp) {
        const size_t s1 = align8(sizeof(InitDesc) * a.size()), s2 = align8(8 * ap.size());
        const size_t s3 = align8(sizeof(RehashDesc) * b.size()), s4 = align8(8 * bp.size());
        const size_t s5 = align8(sizeof(TransposeDesc) * c.size()), s6 = align8(8 * cp.size());
        const size_t total = s1 + s2 + s3 + s4 + s5 + s6;
        char *h = (char *)pin_init_.acquire(total);
        char *q = h;
        memcpy(q, a.data(), sizeof(InitDesc) * a.size()); q += s1;
        memcpy(q, ap.data(), 8 * ap.size()); q += s2;
        memcpy(q, b.data(), sizeof(RehashDesc) * b.size()); q += s3;
        memcpy(q, bp.data(), 8 * bp.size()); q += s4;
        memcpy(q, c.data(), sizeof(TransposeDesc) * c.size()); q += s5;
        memcpy(q, cp.data(), 8 * cp.size());
        char *d = dev_need(init_blob_, init_blob_cap_, total);
        HIPCHK(hipMemcpyAsync(d, h, total, hipMemcpyHostToDevice, stream_));
        pin_init_.issued(stream_);
        return d;
    }

    // Waits for the step's results.  Short steps (many of them: a Černý
    // automaton takes (n-1)^2 steps) finish within tens of microseconds, and
    // polling the stream answers sooner than a blocking wait; after
    // kSpinMs of polling it blocks.
    void wait_step() {
        const double t0 = now_ms();
        for (;;) {
            const hipError_t e = hipStreamQuery(stream_);
            if (e == hipSuccess) return;
            if (e != hipErrorNotReady) throw HipFailure{e, "step"};
            if (now_ms() - t0 > kSpinMs) break;
        }
        HIPCHK(hipStreamSynchronize(stream_));
    }
    static constexpr double kSpinMs = 2.0;

    void prof_begin(int c) {
        if (opt.profile == 1) {
            HIPCHK(hipEventRecord(ev_[2 * c], stream_));
            prof_used_[c] = true;
        }
    }
    void prof_end(int c) {
        if (opt.profile == 1) HIPCHK(hipEventRecord(ev_[2 * c + 1], stream_));
    }
    void prof_collect() {
        if (!opt.profile) return;
        for (int c = 0; c < 7; ++c) {
            if (!prof_used_[c]) continue;
            float ms = 0;
            HIPCHK(hipEventSynchronize(ev_[2 * c + 1]));
            HIPCHK(hipEventElapsedTime(&ms, ev_[2 * c], ev_[2 * c + 1]));
            stats_.ms[c] += ms;
            prof_used_[c] = false;
        }
        for (int w = 0; w < kMaxW; ++w) {
            if (!meet_used_[w]) continue;
            float ms = 0;
            HIPCHK(hipEventSynchronize(ev_meet_[2 * w + 1]));
            HIPCHK(hipEventElapsedTime(&ms, ev_meet_[2 * w], ev_meet_[2 * w + 1]));
            stats_.meet_ms_w[w] += ms;
            meet_used_[w] = false;
        }
        for (int w = 0; w < kMaxW; ++w) {
            if (!meetb_used_[w]) continue;
            float ms = 0;
            HIPCHK(hipEventSynchronize(ev_meetb_[2 * w + 1]));
            HIPCHK(hipEventElapsedTime(&ms, ev_meetb_[2 * w], ev_meetb_[2 * w + 1]));
            stats_.meet_b_ms_w[w] += ms;
            meetb_used_[w] = false;
        }
    }

    int device_;
    double wall_khz_ = 1e5;    // ticks of the device's wall clock per millisecond
    Backing backing_;
    hipStream_t stream_ = nullptr, own_stream_ = nullptr;
    std::unique_ptr<Pool> pool_;
    hipEvent_t ev_[16], ev_meet_[2 * kMaxW], ev_meetb_[2 * kMaxW];
    bool meet_used_[kMaxW] = {};
    bool meetb_used_[kMaxW] = {};
    bool prof_used_[8] = {};
    Pinned pin_delta_, pin_step_, pin_res_, pin_trace_, pin_init_, pin_misc_, pin_clear_, pin_copy_, pin_run_;
    std::vector<CopyDesc> pend_copy_;
    std::vector<void *> pend_free_;
    void *copy_blob_ = nullptr, *delta_blob_ = nullptr, *run_blob_ = nullptr, *pack_blob_ = nullptr;
    int64_t copy_blob_cap_ = 0, delta_blob_cap_ = 0, run_blob_cap_ = 0, pack_blob_cap_ = 0;
    void *step_blob_ = nullptr, *trace_blob_ = nullptr, *init_blob_ = nullptr, *rehash_blob_ = nullptr,
         *clear_blob_ = nullptr;
    int64_t step_blob_cap_ = 0, trace_blob_cap_ = 0, init_blob_cap_ = 0, misc_blob_cap_ = 0,
            clear_blob_cap_ = 0;
    u64 *d_res_ = nullptr, *d_ops_ = nullptr;
    int64_t res_cap_ = 0;
    u32 *d_cnt_ = nullptr, *d_off_ = nullptr;
    int64_t cblk_cap_ = 0;
    Problem *kept_ = nullptr;
};

// Rough device footprint of a solve, used for admission only (growth is
// checked against the budget anyway).  Visited sets of random automata grow
// about exponentially in n: log10(sets) ~ 2.7 + n/80 (k = 2), 3.2 + n/56
// (k = 3), 3.0 + n/42 (k >= 4), fitted on sizes measured with the oracle;
// the device footprints the server reported for a 400-request serving mix
// were a median 2.6-2.8 times these estimates in every letter count, so
// the intercepts carry log10(2.7) more.
static int64_t estimate_bytes(int n, int k) {
    const int W = (n + 63) / 64;
    const double c = 0.43;
    double e;
    if (k <= 2) e = c + 2.7 + n / 80.0;
    else if (k == 3) e = c + 3.2 + n / 56.0;
    else e = c + 3.0 + n / 42.0;
    const double sets = std::pow(10.0, std::min(e, 10.0));
    const double bytes = sets * (8.0 * W * 1.5 + 4 + 16) + 4.0 * 64 * (1 << 20) / 64;
    return (int64_t)std::min(bytes, 4e11);
}

static Problem *make_problem(int32_t n, int32_t k, const int32_t *delta) {
    Problem *p = new Problem();
    p->n = n;
    p->k = k;
    p->W = (n + 63) / 64;
    p->delta.assign(delta, delta + (size_t)n * k);
    p->t_submit = now_ms();
    p->est_bytes = estimate_bytes(n, k);
    return p;
}

// ------------------------------------------------------- default context

struct Context {
    std::mutex mu;
    Backing backing;
    hipStream_t stream = nullptr;
    std::unique_ptr<Engine> eng;
    Options opt;
    int64_t budget = 0;
};

// never destroyed: a destructor running after the HIP runtime (or the
// caller's allocator) has shut down at process exit would crash
static Context &ctx() {
    static Context *c = new Context();
    return *c;
}

static Engine *engine_locked(Context &c) {
    if (!c.eng) {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
            (void)hipGetLastError();
            throw HipFailure{hipErrorNoDevice, "no HIP device"};
        }
        c.eng.reset(new Engine(0, c.backing, c.budget, c.stream));
        c.eng->opt = c.opt;
    }
    return c.eng.get();
}

static int device_error(const HipFailure &f) {
    return set_error(SRW_EDEVICE, std::string("HIP error ") + hipGetErrorString(f.e) + " in " + f.where);
}

}  // namespace srw

using namespace srw;

// ================================================================ C ABI

extern "C" {

const char *srw_last_error(void) { return t_err.c_str(); }

int srw_check_sync(int32_t n, int32_t k, const int32_t *delta) {
    const int rc = check_input(n, k, delta);
    if (rc) return rc;
    return is_synchronizing(n, k, delta) ? 1 : 0;
}

int srw_verify(int32_t n, int32_t k, const int32_t *delta, const uint8_t *word, int64_t len) {
    const int rc = check_input(n, k, delta);
    if (rc) return rc;
    if (len < 0 || (len > 0 && !word)) return set_error(SRW_EINVAL, "bad word");
    return verify_word(n, k, delta, word, len) ? 1 : 0;
}

int srw_set_allocator(void *(*alloc)(size_t, void *), void (*free_fn)(void *, void *), void *c) {
    if ((alloc == nullptr) != (free_fn == nullptr)) return set_error(SRW_EINVAL, "set both or neither");
    Context &x = ctx();
    std::lock_guard<std::mutex> g(x.mu);
    x.backing = Backing{alloc, free_fn, c};
    x.eng.reset();
    return SRW_OK;
}

int srw_set_stream(void *s) {
    Context &x = ctx();
    std::lock_guard<std::mutex> g(x.mu);
    if (x.stream != (hipStream_t)s) {
        x.stream = (hipStream_t)s;
        x.eng.reset();
    }
    return SRW_OK;
}

int srw_set_option(const char *key, int64_t v) {
    if (!key) return set_error(SRW_EINVAL, "key is NULL");
    Context &x = ctx();
    std::lock_guard<std::mutex> g(x.mu);
    std::string k(key);
    if (k == "budget") {
        if (v < 0) return set_error(SRW_EINVAL, "budget < 0");
        x.budget = v;
        if (x.eng) {
            try {
                x.eng->set_budget(v);
            } catch (const HipFailure &f) {
                return device_error(f);
            }
        }
        return SRW_OK;
    }
    const size_t at = k.find('@');
    if (at != std::string::npos) {       // a per-width value: "<key>@<W>", -1 removes it
        const std::string base = k.substr(0, at), ws = k.substr(at + 1);
        const int W = (ws.size() == 1 && ws[0] >= '1' && ws[0] <= '8') ? ws[0] - '0' : 0;
        if (W == 0) return set_error(SRW_EINVAL, "width in " + k + " must be 1..8");
        int64_t *slot = base == "meet_groups" ? x.opt.meet_groups_w : base == "meet_rows" ? x.opt.meet_rows_w
                      : base == "bucket" ? x.opt.bucket_w : base == "small_cand" ? x.opt.small_cand_w
                      : base == "schedule" ? x.opt.schedule_w : nullptr;
        if (!slot) return set_error(SRW_EINVAL, "no per-width option " + base);
        if (v < -1 || (base == "meet_groups" && (v == 0 || v > 4096)) || (base == "small_cand" && v > (1 << 20)) ||
            (base == "schedule" && v > 3))
            return set_error(SRW_EINVAL, "value of " + k);
        slot[W] = v;
        if (x.eng) x.eng->opt = x.opt;
        return SRW_OK;
    }
    if (k == "max_slots") { if (v < 1) return set_error(SRW_EINVAL, "max_slots < 1"); x.opt.max_slots = v; }
    else if (k == "profile") { if (v < 0 || v > 2) return set_error(SRW_EINVAL, "profile"); x.opt.profile = (int)v; }
    else if (k == "schedule") { if (v < 0 || v > 3) return set_error(SRW_EINVAL, "schedule"); x.opt.schedule = (int)v; }
    else if (k == "sched_seed") x.opt.sched_seed = (uint64_t)v;
    else if (k == "meet_tiles") { if (v < 0 || v > kMeetTileWords) return set_error(SRW_EINVAL, "meet_tiles"); x.opt.meet_tiles = (int)v; }
    else if (k == "keep_levels") x.opt.keep_levels = v != 0;
    else if (k == "verbose") x.opt.verbose = v != 0;
    else if (k == "deadline_ms") { if (v < 0) return set_error(SRW_EINVAL, "deadline_ms"); x.opt.deadline_ms = (double)v; }
    else if (k == "meet") { if (v < 0 || v > 2) return set_error(SRW_EINVAL, "meet"); x.opt.meet = (int)v; }
    else if (k == "meet_rows") { if (v < 0) return set_error(SRW_EINVAL, "meet_rows"); x.opt.meet_rows = v; }
    else if (k == "ysort") { if (v < 0) return set_error(SRW_EINVAL, "ysort"); x.opt.ysort = v; }
    else if (k == "small_cand") { if (v < 0 || v > (1 << 20)) return set_error(SRW_EINVAL, "small_cand"); x.opt.small_cand = v; }
    else if (k == "persist") { if (v < 0 || v > 1) return set_error(SRW_EINVAL, "persist"); x.opt.persist = (int)v; }
    else if (k == "bucket") { if (v < 0) return set_error(SRW_EINVAL, "bucket"); x.opt.bucket = v; }
    else if (k == "meet_groups") { if (v < 1 || v > 4096) return set_error(SRW_EINVAL, "meet_groups"); x.opt.meet_groups = v; }
    else if (k == "meet_grid") { if (v < 0) return set_error(SRW_EINVAL, "meet_grid"); x.opt.meet_grid = v; }
    else if (k == "meet_order") { if (v < 0 || v > 1) return set_error(SRW_EINVAL, "meet_order"); x.opt.meet_order = v; }
    else if (k == "meet_xcd") { if (v < 0 || v > 65536) return set_error(SRW_EINVAL, "meet_xcd"); x.opt.meet_xcd = v; }
    else if (k == "meet_bgrid") { if (v < 1 || v > 65536) return set_error(SRW_EINVAL, "meet_bgrid"); x.opt.meet_bgrid = v; }
    else if (k == "reduce") { if (v < 0 || v > 2) return set_error(SRW_EINVAL, "reduce"); x.opt.reduce = (int)v; }
    else return set_error(SRW_EINVAL, "unknown option " + k);
    if (x.eng) x.eng->opt = x.opt;
    return SRW_OK;
}

int srw_get_stats(srw_stats *out) {
    if (!out) return set_error(SRW_EINVAL, "out is NULL");
    Context &x = ctx();
    std::lock_guard<std::mutex> g(x.mu);
    if (!x.eng) {
        memset(out, 0, sizeof *out);
        return SRW_OK;
    }
    try {
        *out = x.eng->stats();
    } catch (const HipFailure &e) {
        return device_error(e);
    }
    return SRW_OK;
}

int srw_reset_stats(void) {
    Context &x = ctx();
    std::lock_guard<std::mutex> g(x.mu);
    if (!x.eng) return SRW_OK;
    try {
        x.eng->reset_stats();
    } catch (const HipFailure &e) {
        return device_error(e);
    }
    return SRW_OK;
}

int srw_solve_batch(int32_t count, const int32_t *n, const int32_t *k, const int64_t *delta_off,
                    const int32_t *delta, int32_t *r, int32_t *status, const int64_t *word_off,
                    uint8_t *words, const int64_t *word_cap) {
    if (count < 0 || (count > 0 && (!n || !k || !delta_off || !delta || !r || !status)))
        return set_error(SRW_EINVAL, "null argument");
    if (words && (!word_off || !word_cap)) return set_error(SRW_EINVAL, "words without offsets");
    Context &x = ctx();
    std::lock_guard<std::mutex> g(x.mu);
    std::vector<int> hc;
    host_checks(count, n, k, delta_off, delta, hc);
    std::vector<std::unique_ptr<Problem>> own;
    std::vector<Problem *> work;
    for (int32_t i = 0; i < count; ++i) {
        r[i] = -1;
        const int32_t *d = delta + delta_off[i];
        int rc = hc[(size_t)i];
        if (rc) { status[i] = rc; continue; }
        if (n[i] == 1) { status[i] = SRW_OK; r[i] = 0; continue; }
        Problem *p = make_problem(n[i], k[i], d);
        p->index = i;
        own.emplace_back(p);
        work.push_back(p);
    }
    if (!work.empty()) {
        try {
            Engine *e = engine_locked(x);
            e->release_kept();
            const bool keep = e->opt.keep_levels;
            e->opt.keep_levels = false;
            e->run(work);
            e->opt.keep_levels = keep;
        } catch (const HipFailure &f) {
            // members that finished keep their results; the others fail with
            // SRW_ENOMEM (the engine's budget) or SRW_EDEVICE (a HIP error)
            const bool oom = f.e == hipErrorOutOfMemory;
            for (Problem *p : work)
                if (p->status == 1) p->status = oom ? SRW_ENOMEM : SRW_EDEVICE;
            x.eng.reset();
            if (!oom) {
                for (Problem *p : work) status[p->index] = p->status;
                return device_error(f);
            }
            set_error(SRW_ENOMEM, "device memory budget exhausted in " + f.where);
        }
    }
    for (Problem *p : work) {
        const int i = (int)p->index;
        status[i] = p->status;
        r[i] = p->status == SRW_OK ? p->r : -1;
        if (p->status == SRW_OK && words) {
            if (word_cap[i] < p->r) status[i] = SRW_EWORDCAP;
            else memcpy(words + word_off[i], p->word.data(), p->r);
        }
    }
    return SRW_OK;
}

int srw_beam_batch(int32_t count, const int32_t *n, const int32_t *k, const int64_t *delta_off,
                   const int32_t *delta, const int64_t *width, int32_t *R, int32_t *status,
                   const int64_t *word_off, uint8_t *words, const int64_t *word_cap) {
    if (count < 0 || (count > 0 && (!n || !k || !delta_off || !delta || !width || !R || !status)))
        return set_error(SRW_EINVAL, "null argument");
    if (words && (!word_off || !word_cap)) return set_error(SRW_EINVAL, "words without offsets");
    Context &x = ctx();
    std::lock_guard<std::mutex> g(x.mu);
    std::vector<int> hc;
    host_checks(count, n, k, delta_off, delta, hc);
    std::vector<Engine::BeamJob> jobs((size_t)std::max(count, 0));
    std::vector<Engine::BeamJob *> work;
    for (int32_t i = 0; i < count; ++i) {
        R[i] = -1;
        const int32_t *d = delta + delta_off[i];
        int rc = hc[(size_t)i];
        if (!rc && width[i] < 1) rc = SRW_EINVAL;
        if (rc) { status[i] = rc; continue; }
        if (n[i] == 1) { status[i] = SRW_OK; R[i] = 0; continue; }
        Engine::BeamJob &j = jobs[(size_t)i];
        j.n = n[i];
        j.k = k[i];
        j.delta = d;
        j.width = width[i];
        j.index = i;
        work.push_back(&j);
    }
    if (!work.empty()) {
        try {
            engine_locked(x)->beam(work);
        } catch (const HipFailure &f) {
            const bool oom = f.e == hipErrorOutOfMemory;
            for (Engine::BeamJob *j : work)
                if (j->status == 1) j->status = oom ? SRW_ENOMEM : SRW_EDEVICE;
            x.eng.reset();
            if (!oom) {
                for (Engine::BeamJob *j : work) status[j->index] = j->status;
                return device_error(f);
            }
        }
    }
    for (Engine::BeamJob *j : work) {
        const int i = (int)j->index;
        status[i] = j->status;
        R[i] = j->status == SRW_OK ? j->R : -1;
        if (j->status == SRW_OK && words) {
            if (word_cap[i] < j->R) status[i] = SRW_EWORDCAP;
            else memcpy(words + word_off[i], j->word.data(), (size_t)j->R);
        }
    }
    return SRW_OK;
}

int srw_eppstein_batch(int32_t count, const int32_t *n, const int32_t *k, const int64_t *delta_off,
                       const int32_t *delta, int64_t *len, int32_t *status, const int64_t *word_off,
                       uint8_t *words, const int64_t *word_cap) {
    if (count < 0 || (count > 0 && (!n || !k || !delta_off || !delta || !len || !status)))
        return set_error(SRW_EINVAL, "null argument");
    if (words && (!word_off || !word_cap)) return set_error(SRW_EINVAL, "words without offsets");
    Context &x = ctx();
    std::lock_guard<std::mutex> g(x.mu);
    std::vector<int> hc;
    host_checks(count, n, k, delta_off, delta, hc, false);   // non-synchronizing: found on the device
    std::vector<Engine::EppJob> jobs((size_t)std::max(count, 0));
    std::vector<Engine::EppJob *> work;
    for (int32_t i = 0; i < count; ++i) {
        len[i] = -1;
        const int32_t *d = delta + delta_off[i];
        int rc = hc[(size_t)i];
        if (rc) { status[i] = rc; continue; }
        if (n[i] == 1) { status[i] = SRW_OK; len[i] = 0; continue; }
        Engine::EppJob &j = jobs[(size_t)i];
        j.n = n[i];
        j.k = k[i];
        j.delta = d;
        j.index = i;
        work.push_back(&j);
    }
    if (!work.empty()) {
        try {
            engine_locked(x)->eppstein(work);
        } catch (const HipFailure &f) {
            const bool oom = f.e == hipErrorOutOfMemory;
            for (Engine::EppJob *j : work)
                if (j->status == 1) j->status = oom ? SRW_ENOMEM : SRW_EDEVICE;
            x.eng.reset();
            if (!oom) {
                for (Engine::EppJob *j : work) status[j->index] = j->status;
                return device_error(f);
            }
        }
    }
    for (Engine::EppJob *j : work) {
        const int i = (int)j->index;
        status[i] = j->status;
        len[i] = j->status == SRW_OK ? j->len : -1;
        if (j->status == SRW_OK && words) {
            if (word_cap[i] < j->len) status[i] = SRW_EWORDCAP;
            else memcpy(words + word_off[i], j->word.data(), (size_t)j->len);
        }
    }
    return SRW_OK;
}

namespace {
// The beam size of the second beam search of srw_bound: the exact search's
// cost estimated from the first beam's level sizes (exact up to the first
// level larger than w0, growing by that level's ratio to the one before
// beyond it), over both sides to depth ceil(B/2); the beam takes 1/16 of it
// at about width * B sets.  w0 when the first beam cut no level.
constexpr int kBoundFraction = 16;
constexpr int64_t kBoundMaxWidth = (int64_t)1 << 20;
int64_t bound_width(const std::vector<int64_t> &sizes, int64_t w0, int64_t B) {
    size_t c = 0;
    while (c < sizes.size() && sizes[c] <= w0) ++c;
    if (c == sizes.size() || c == 0) return w0;
    const double g = (double)sizes[c] / (double)sizes[c - 1];
    const int64_t h = (B + 1) / 2;
    double total = 0.0, u = 0.0;
    for (int64_t d = 0; d <= h; ++d) {
        u = (size_t)d <= c ? (double)sizes[(size_t)d] : u * g;
        total += u;
        if (total > 1e30) break;
    }
    const double w = std::ceil(2.0 * total / ((double)kBoundFraction * (double)B));
    if (w >= (double)kBoundMaxWidth) return kBoundMaxWidth;
    return std::max<int64_t>(w0, (int64_t)w);
}
}  // namespace

int srw_bound_batch(int32_t count, const int32_t *n, const int32_t *k, const int64_t *delta_off,
                    const int32_t *delta, int32_t *R, int64_t *width, int32_t *status,
                    const int64_t *word_off, uint8_t *words, const int64_t *word_cap) {
    if (count < 0 || (count > 0 && (!n || !k || !delta_off || !delta || !R || !width || !status)))
        return set_error(SRW_EINVAL, "null argument");
    if (words && (!word_off || !word_cap)) return set_error(SRW_EINVAL, "words without offsets");
    Context &x = ctx();
    std::lock_guard<std::mutex> g(x.mu);
    std::vector<int> hc;
    host_checks(count, n, k, delta_off, delta, hc, false);   // non-synchronizing: found on the device
    const size_t cn = (size_t)std::max(count, 0);
    std::vector<Engine::EppJob> ej(cn);
    std::vector<Engine::BeamJob> b0(cn), b1(cn);
    std::vector<Engine::EppJob *> ework;
    std::vector<Engine::BeamJob *> w0work, w1work;
    for (int32_t i = 0; i < count; ++i) {
        R[i] = -1;
        width[i] = 0;
        const int32_t *d = delta + delta_off[i];
        int rc = hc[(size_t)i];
        if (rc) { status[i] = rc; continue; }
        if (n[i] == 1) { status[i] = SRW_OK; R[i] = 0; width[i] = 1; continue; }
        status[i] = 1;
        ej[(size_t)i].n = b0[(size_t)i].n = n[i];
        ej[(size_t)i].k = b0[(size_t)i].k = k[i];
        ej[(size_t)i].delta = b0[(size_t)i].delta = d;
        ej[(size_t)i].index = b0[(size_t)i].index = i;
        b0[(size_t)i].width = n[i];
        b0[(size_t)i].want_sizes = true;
        ework.push_back(&ej[(size_t)i]);
        w0work.push_back(&b0[(size_t)i]);
    }
    try {
        if (!ework.empty()) {
            Engine *eng = engine_locked(x);
            eng->eppstein(ework);
            std::vector<Engine::BeamJob *> run0;
            for (Engine::BeamJob *j : w0work)
                if (ej[(size_t)j->index].status == SRW_OK) run0.push_back(j);
            eng->beam(run0);
            for (Engine::BeamJob *j : w0work) {
                const size_t i = (size_t)j->index;
                const Engine::EppJob &e = ej[i];
                if (e.status != SRW_OK && e.status != SRW_EWORDCAP) { status[i] = e.status; continue; }
                if (j->status != SRW_OK && j->status != SRW_ENOBOUND) { status[i] = j->status; continue; }
                int64_t B = e.len;
                if (j->status == SRW_OK) B = std::min<int64_t>(B, j->R);
                width[i] = bound_width(j->sizes, j->width, B);
                if (width[i] > j->width) {
                    Engine::BeamJob &s = b1[i];
                    s.n = j->n;
                    s.k = j->k;
                    s.delta = j->delta;
                    s.index = j->index;
                    s.width = width[i];
                    w1work.push_back(&s);
                }
            }
            if (!w1work.empty()) eng->beam(w1work);
        }
    } catch (const HipFailure &f) {
        x.eng.reset();
        if (f.e != hipErrorOutOfMemory) {
            for (int32_t i = 0; i < count; ++i)
                if (status[i] == 1) status[i] = SRW_EDEVICE;
            return device_error(f);
        }
        for (int32_t i = 0; i < count; ++i)
            if (status[i] == 1) status[i] = SRW_ENOMEM;
        return SRW_OK;
    }
    for (Engine::EppJob *e : ework) {
        const size_t i = (size_t)e->index;
        if (status[i] != 1) continue;
        // the least bound; ties to Eppstein, then the first beam, then the second
        const std::vector<uint8_t> *best = &e->word;
        int64_t len = e->len;
        for (const Engine::BeamJob *j : {&b0[i], &b1[i]})
            if (j->status == SRW_OK && j->R < len) {
                len = j->R;
                best = &j->word;
            }
        if (b1[i].index >= 0 && b1[i].status != SRW_OK && b1[i].status != SRW_ENOBOUND) {
            status[i] = b1[i].status;
            continue;
        }
        R[i] = (int32_t)len;
        status[i] = SRW_OK;
        if (words) {
            if (word_cap[i] < len) status[i] = SRW_EWORDCAP;
            else if ((int64_t)best->size() == len) memcpy(words + word_off[i], best->data(), (size_t)len);
            else status[i] = SRW_EWORDCAP;
        }
    }
    return SRW_OK;
}

int srw_bound(int32_t n, int32_t k, const int32_t *delta, int32_t *R, int64_t *width, uint8_t *word,
              int64_t word_cap) {
    if (!R || !width) return set_error(SRW_EINVAL, "R or width is NULL");
    const int64_t off = 0;
    int32_t st = SRW_OK;
    int rc = srw_bound_batch(1, &n, &k, &off, delta, R, width, &st, word ? &off : nullptr, word,
                             word ? &word_cap : nullptr);
    return rc ? rc : st;
}

int srw_eppstein(int32_t n, int32_t k, const int32_t *delta, int64_t *len, uint8_t *word, int64_t word_cap) {
    if (!len) return set_error(SRW_EINVAL, "len is NULL");
    const int64_t off = 0;
    int32_t st = SRW_OK;
    int rc = srw_eppstein_batch(1, &n, &k, &off, delta, len, &st, word ? &off : nullptr, word,
                                word ? &word_cap : nullptr);
    return rc ? rc : st;
}

int srw_beam(int32_t n, int32_t k, const int32_t *delta, int64_t width, int32_t *R, uint8_t *word,
             int64_t word_cap) {
    if (!R) return set_error(SRW_EINVAL, "R is NULL");
    const int64_t off = 0;
    int32_t st = SRW_OK;
    int rc = srw_beam_batch(1, &n, &k, &off, delta, &width, R, &st, word ? &off : nullptr, word,
                            word ? &word_cap : nullptr);
    return rc ? rc : st;
}

int srw_solve(int32_t n, int32_t k, const int32_t *delta, int32_t *r, uint8_t *word, int64_t word_cap) {
    if (!r) return set_error(SRW_EINVAL, "r is NULL");
    *r = -1;
    int rc = check_input(n, k, delta);
    if (rc) return rc;
    if (!is_synchronizing(n, k, delta)) return set_error(SRW_ENOTSYNC, "automaton is not synchronizing");
    if (n == 1) { *r = 0; return SRW_OK; }
    Context &x = ctx();
    std::lock_guard<std::mutex> g(x.mu);
    Problem *p = make_problem(n, k, delta);
    p->index = 0;
    std::vector<Problem *> work{p};
    try {
        Engine *e = engine_locked(x);
        e->release_kept();
        e->run(work);
        if (e->opt.keep_levels) e->keep(p);
    } catch (const HipFailure &f) {
        x.eng.reset();
        delete p;
        if (f.e == hipErrorOutOfMemory)   // the budget, even its reserve, ran out
            return set_error(SRW_ENOMEM, "device memory budget exhausted in " + f.where);
        return device_error(f);
    }
    rc = p->status;
    if (rc == SRW_OK) {
        *r = p->r;
        if (word) {
            if (word_cap < p->r) rc = set_error(SRW_EWORDCAP, "word_cap too small");
            else memcpy(word, p->word.data(), p->r);
        }
    } else if (rc < 0 && t_err.empty()) {
        set_error(rc, "solve failed");
    }
    if (!x.eng || x.eng->kept() != p) delete p;
    return rc;
}

int srw_last_sides(int32_t *steps, uint8_t *sides, int64_t cap) {
    if (!steps || cap < 0 || (cap > 0 && !sides)) return set_error(SRW_EINVAL, "bad arguments");
    Context &x = ctx();
    std::lock_guard<std::mutex> g(x.mu);
    if (!x.eng || !x.eng->kept()) return set_error(SRW_EINVAL, "no kept solve (set keep_levels)");
    const std::vector<uint8_t> &v = x.eng->kept()->sides;
    *steps = (int32_t)v.size();
    if ((int64_t)v.size() > cap && sides) return set_error(SRW_EINVAL, "cap below the step count");
    if (sides) memcpy(sides, v.data(), v.size());
    return SRW_OK;
}

int srw_last_levels(int32_t side, int32_t *nlev, int64_t *nrows, int64_t *off, uint64_t *rows, uint32_t *par) {
    if (side < 0 || side > 1 || !nlev || !nrows) return set_error(SRW_EINVAL, "bad arguments");
    Context &x = ctx();
    std::lock_guard<std::mutex> g(x.mu);
    if (!x.eng || !x.eng->kept()) return set_error(SRW_EINVAL, "no kept solve (set keep_levels)");
    Problem *p = x.eng->kept();
    const SideState &s = p->s[side];
    *nlev = s.nlev();
    *nrows = s.nrows;
    if (!rows) return SRW_OK;
    if (!off || !par) return set_error(SRW_EINVAL, "off/par NULL");
    try {
        HIPCHK(hipSetDevice(x.eng->device()));
        memcpy(off, s.off.data(), 8 * s.off.size());
        HIPCHK(hipMemcpyAsync(rows, s.rows, (size_t)s.nrows * p->W * 8, hipMemcpyDeviceToHost, x.eng->stream()));
        HIPCHK(hipMemcpyAsync(par, s.par, (size_t)s.nrows * 4, hipMemcpyDeviceToHost, x.eng->stream()));
        HIPCHK(hipStreamSynchronize(x.eng->stream()));
    } catch (const HipFailure &f) {
        return device_error(f);
    }
    return SRW_OK;
}

}  // extern "C"

// ========================================================= no-alloc solves

namespace srw {

// Device memory of srw_solve_noalloc: one array per GPU in the library's
// code object, taken when that code is loaded on the GPU and held until the
// process ends.  Host code reaches it only through the address that
// hipGetSymbolAddress gives for the current device (the array's name in
// host code is a host-side stand-in, not a device address).
constexpr int64_t kScratchBytes = (int64_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// First-fit allocator over one device's scratch array; the bookkeeping is
// on the host.  Blocks are 256-byte aligned.
class Arena {
  public:
    void init(char *base, int64_t size) {
        base_ = base;
        free_.clear();
        used_.clear();
        free_[0] = size;
    }
    void *alloc(size_t bytes) {
        const int64_t need = (int64_t)((bytes + 255) & ~(size_t)255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const int64_t off = it->first, left = it->second - need;
            free_.erase(it);
            if (left) free_[off + need] = left;
            used_[off] = need;
            return base_ + off;
        }
        return nullptr;
    }
    void free(void *p) {
        const int64_t off = (char *)p - base_;
        auto u = used_.find(off);
        if (u == used_.end()) return;
        int64_t start = off, len = u->second;
        used_.erase(u);
        auto nx = free_.lower_bound(start);
        if (nx != free_.end() && nx->first == start + len) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == start) {
                start = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = len;
    }

  private:
    char *base_ = nullptr;
    std::map<int64_t, int64_t> free_;            // offset -> bytes
    std::unordered_map<int64_t, int64_t> used_;  // offset -> bytes
};
static void *arena_alloc(size_t b, void *c) { return ((Arena *)c)->alloc(b); }
static void arena_free(void *p, void *c) { ((Arena *)c)->free(p); }

struct NoAllocDevice {
    std::mutex mu;               // serializes the calls on this device
    char *ptr = nullptr;         // this device's scratch array
    Arena arena;
    std::unique_ptr<Engine> eng; // its pool draws on the arena; pageable staging
};
constexpr int kNoAllocDevices = 64;
static NoAllocDevice &noalloc_dev(int d) {
    static NoAllocDevice *devs = new NoAllocDevice[kNoAllocDevices];   // never destroyed
    return devs[d];
}

// Set-up, once per device with that device current: the scratch address,
// then an engine over it (its stream and events are created here, so that
// the calls themselves create nothing).
static Engine *noalloc_engine(NoAllocDevice &nd, int device) {
    if (!nd.ptr) {
        HIPCHK(hipSetDevice(device));
        void *ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        nd.ptr = (char *)ptr;
    }
    if (!nd.eng) {
        nd.arena.init(nd.ptr, kScratchBytes);
        Backing b;
        b.alloc = arena_alloc;
        b.free = arena_free;
        b.ctx = &nd.arena;
        b.own_stream_only = true;
        nd.eng.reset(new Engine(device, b, kScratchBytes, nullptr, true));
    }
    return nd.eng.get();
}

}  // namespace srw

extern "C" {

int srw_solve_noalloc(int32_t n, int32_t k, const int32_t *delta, int32_t *r, uint8_t *word,
                      int64_t word_cap) {
    if (!r) return set_error(SRW_EINVAL, "r is NULL");
    *r = -1;
    int rc = check_input(n, k, delta);
    if (rc) return rc;
    if (!is_synchronizing(n, k, delta)) return set_error(SRW_ENOTSYNC, "automaton is not synchronizing");
    if (n == 1) {
        *r = 0;
        return SRW_OK;
    }
    int device = -1, count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1 || hipGetDevice(&device) != hipSuccess ||
        device < 0 || device >= kNoAllocDevices) {
        (void)hipGetLastError();
        return set_error(SRW_EDEVICE, "no usable HIP device");
    }
    NoAllocDevice &nd = noalloc_dev(device);
    std::lock_guard<std::mutex> g(nd.mu);
    std::unique_ptr<Problem> p(make_problem(n, k, delta));
    p->index = 0;
    std::vector<Problem *> work{p.get()};
    try {
        noalloc_engine(nd, device)->run(work);
    } catch (const HipFailure &f) {
        nd.eng.reset();           // the next call sets up a fresh engine over the same array
        return device_error(f);
    }
    rc = p->status;
    if (rc == SRW_OK) {
        *r = p->r;
        if (word) {
            if (word_cap < p->r) rc = set_error(SRW_EWORDCAP, "word_cap too small");
            else memcpy(word, p->word.data(), p->r);
        }
    } else if (rc == SRW_ENOMEM) {
        set_error(rc, "the search needs more device memory than the 256 MiB no-alloc scratch; "
                      "srw_solve has no such limit");
    } else if (rc < 0 && t_err.empty()) {
        set_error(rc, "solve failed");
    }
    return rc;
}

}  // extern "C"

// ================================================================ serving

// Requests go to one of three lanes by estimated footprint.  Each lane has
// its own engine, stream and worker thread and batches its requests
// continuously; a global step of a heavier lane (seconds at large n) never
// holds up the steps of a lighter one, and the streams share the GPU.
constexpr int kLanes = 3;
constexpr int64_t kLaneBytes[kLanes - 1] = {(int64_t)64 << 20, (int64_t)2 << 30};
constexpr double kLaneShare[kLanes] = {0.10, 0.25, 0.65};   // of the memory budget

static int lane_of(int64_t est) {
    int li = 0;
    while (li < kLanes - 1 && est > kLaneBytes[li]) ++li;
    return li;
}

struct ServerLane {
    std::unique_ptr<Engine> eng;
    std::thread worker;
    std::deque<Problem *> inbox;
};

struct srw_server {
    ServerLane lane[kLanes];
    std::mutex mu;
    std::condition_variable cv_in, cv_out;
    std::deque<Problem *> outbox;
    std::vector<Problem *> returned;   // owned until the next poll
    bool stop = false;
    int64_t submitted = 0, polled = 0;
    int max_slots = 4096;
    double deadline_ms = 0;
    std::string fatal;
};

static void server_loop(srw_server *s, int li) {
    std::deque<Problem *> pending;
    std::vector<Problem *> active;
    std::vector<Problem *> done_now;        // finished in this round, not yet returned
    Engine *eng = s->lane[li].eng.get();
    std::deque<Problem *> &inbox = s->lane[li].inbox;
    try {
        HIPCHK(hipSetDevice(eng->device()));
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(s->mu);
                if (active.empty() && pending.empty())
                    s->cv_in.wait(lk, [&] { return s->stop || !inbox.empty(); });
                if (s->stop) break;
                while (!inbox.empty()) {
                    pending.push_back(inbox.front());
                    inbox.pop_front();
                }
            }
            std::vector<Problem *> fresh;
            done_now.clear();
            // admit in arrival order; a request whose estimated footprint
            // does not fit waits without blocking smaller ones behind it
            std::deque<Problem *> waiting;
            while (!pending.empty()) {
                Problem *p = pending.front();
                pending.pop_front();
                if ((int)active.size() >= s->max_slots ||
                    (!active.empty() && eng->in_use() + p->est_bytes > eng->budget())) {
                    waiting.push_back(p);
                    continue;
                }
                if (eng->admit(p)) {
                    active.push_back(p);
                    fresh.push_back(p);
                } else if (active.empty()) {
                    eng->finish_error(p, SRW_ENOMEM);
                    done_now.push_back(p);
                } else {
                    waiting.push_back(p);
                }
            }
            pending.swap(waiting);
            try {
                if (!fresh.empty()) {
                    eng->init(fresh);
                    eng->run_small(fresh, s->deadline_ms);
                }
                if (!active.empty()) eng->step(active);
            } catch (const HipFailure &f) {
                if (f.e != hipErrorOutOfMemory) throw;
                // the lane's memory budget, not the device: the problems of
                // this step fail with SRW_ENOMEM and the lane goes on
                eng->recover();
                for (Problem *p : active)
                    if (p->status == 1) eng->finish_error(p, SRW_ENOMEM, "device memory budget exhausted");
            }
            std::vector<Problem *> still;
            for (Problem *p : active) {
                if (p->status == 1 && s->deadline_ms > 0 && now_ms() - p->t_admit > s->deadline_ms)
                    eng->finish_error(p, SRW_ETIMEOUT, "deadline passed before the searches met");
                (p->status == 1 ? still : done_now).push_back(p);
            }
            active.swap(still);
            if (!done_now.empty()) {
                std::lock_guard<std::mutex> lk(s->mu);
                for (Problem *p : done_now) s->outbox.push_back(p);
                done_now.clear();
                s->cv_out.notify_all();
            }
        }
    } catch (const HipFailure &f) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->fatal = std::string("HIP error ") + hipGetErrorString(f.e) + " in " + f.where;
        const double t = now_ms();
        for (Problem *p : done_now) s->outbox.push_back(p);   // their own status stands
        for (Problem *p : active) {
            if (p->status == 1) {
                p->status = SRW_EDEVICE;
                p->t_done = t;
            }
            if (std::find(done_now.begin(), done_now.end(), p) == done_now.end()) s->outbox.push_back(p);
        }
        for (Problem *p : pending) {
            p->status = SRW_EDEVICE;
            p->t_admit = p->t_done = t;
            s->outbox.push_back(p);
        }
        s->cv_out.notify_all();
        return;
    }
    for (Problem *p : active) delete p;     // stopped with work in flight
    for (Problem *p : pending) delete p;
}

extern "C" {

int srw_server_create(srw_server **out, const srw_config *cfg) {
    if (!out) return set_error(SRW_EINVAL, "out is NULL");
    *out = nullptr;
    srw_config c{0, 0, 0, 0};
    if (cfg) c = *cfg;
    Backing b;
    {
        Context &x = ctx();
        std::lock_guard<std::mutex> g(x.mu);
        b = x.backing;
    }
    srw_server *s = new srw_server();
    try {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count <= c.device) {
            (void)hipGetLastError();
            delete s;
            return set_error(SRW_EDEVICE, "no such HIP device");
        }
        int64_t total = c.hbm_budget;
        if (total <= 0) {
            size_t fr = 0, tot = 0;
            HIPCHK(hipSetDevice(c.device));
            HIPCHK(hipMemGetInfo(&fr, &tot));
            total = (int64_t)(fr * 0.8);
        }
        // the lanes search with the default context's options as they are now
        // (its tuning, e.g. the autotuner's per-width values); the rest are
        // the server's own or off
        Options so;
        {
            Context &x = ctx();
            std::lock_guard<std::mutex> g(x.mu);
            so = x.opt;
        }
        so.profile = 0;
        so.keep_levels = false;
        so.verbose = false;
        so.deadline_ms = 0;
        so.max_slots = Options().max_slots;
        for (int li = 0; li < kLanes; ++li) {
            s->lane[li].eng.reset(new Engine(c.device, b, (int64_t)(total * kLaneShare[li]), nullptr));
            s->lane[li].eng->opt = so;
        }
    } catch (const HipFailure &f) {
        delete s;
        return device_error(f);
    }
    s->max_slots = c.max_slots > 0 ? c.max_slots : 4096;
    s->deadline_ms = c.deadline_ms > 0 ? (double)c.deadline_ms : 0.0;
    for (int li = 0; li < kLanes; ++li) s->lane[li].worker = std::thread(server_loop, s, li);
    *out = s;
    return SRW_OK;
}

int srw_server_submit(srw_server *s, int32_t n, int32_t k, const int32_t *delta, uint64_t tag) {
    if (!s) return set_error(SRW_EINVAL, "server is NULL");
    int rc = check_input(n, k, delta);
    if (rc) return rc;
    Problem *p = make_problem(n, k, delta);
    p->tag = tag;
    bool immediate = false;
    if (!is_synchronizing(n, k, delta)) {
        p->status = SRW_ENOTSYNC;
        immediate = true;
    } else if (n == 1) {
        p->status = SRW_OK;
        p->r = 0;
        immediate = true;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->fatal.empty()) {
        delete p;
        return set_error(SRW_EDEVICE, s->fatal);
    }
    s->submitted++;
    if (immediate) {
        p->t_admit = p->t_done = now_ms();
        s->outbox.push_back(p);
        s->cv_out.notify_all();
    } else {
        s->lane[lane_of(p->est_bytes)].inbox.push_back(p);
        s->cv_in.notify_all();
    }
    return SRW_OK;
}

int srw_server_poll(srw_server *s, srw_result *out, int32_t max, int32_t timeout_us) {
    if (!s || !out || max < 1) return set_error(SRW_EINVAL, "bad arguments");
    std::unique_lock<std::mutex> lk(s->mu);
    for (Problem *p : s->returned) delete p;
    s->returned.clear();
    if (s->outbox.empty() && timeout_us > 0)
        s->cv_out.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return !s->outbox.empty(); });
    if (s->outbox.empty()) return SRW_ETIMEOUT;
    int cnt = 0;
    while (cnt < max && !s->outbox.empty()) {
        Problem *p = s->outbox.front();
        s->outbox.pop_front();
        srw_result &r = out[cnt++];
        r.tag = p->tag;
        r.status = p->status;
        r.r = p->status == SRW_OK ? p->r : -1;
        r.word = p->word.empty() ? nullptr : p->word.data();
        r.latency_ms = p->t_done - p->t_submit;
        r.queue_ms = p->t_admit - p->t_submit;
        r.est_bytes = p->est_bytes;
        r.dev_bytes = p->dev_bytes;
        s->returned.push_back(p);
        s->polled++;
    }
    return cnt;
}

int64_t srw_server_pending(srw_server *s) {
    if (!s) return set_error(SRW_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    return s->submitted - s->polled;
}

void srw_server_destroy(srw_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_in.notify_all();
    }
    for (int li = 0; li < kLanes; ++li)
        if (s->lane[li].worker.joinable()) s->lane[li].worker.join();
    for (Problem *p : s->returned) delete p;
    for (Problem *p : s->outbox) delete p;
    for (int li = 0; li < kLanes; ++li) {
        for (Problem *p : s->lane[li].inbox) delete p;
        s->lane[li].eng.reset();
    }
    delete s;
}

}  // extern "C"
