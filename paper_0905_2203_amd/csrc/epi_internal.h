// Internal declarations of the episode-counting engine (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <limits>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/epi.h"

namespace epi {

constexpr int kMaxN = EPI_MAX_N;
constexpr int kMaxK = 4096;        // LDS histogram bound of the index build
constexpr int kMaxQueue = 16;      // deepest merged-interval ring (LDS) per node
constexpr int kTile = 4096;        // largest number of events per stream tile (the stream picks its own, Stream::T)
constexpr int kDefaultTile = 2048; // largest a stream picks unless the autotuner raises or lowers it
constexpr int kMinTile = 256;      // smallest tile a stream may pick
constexpr int kMlpHidden = 64;     // hidden units of the cost model
constexpr int kFeatures = 24;      // cost-model features per candidate
constexpr int kBaseFeature = 23;   // the cost model predicts log work as this feature + the network's correction
constexpr int kWork = 5;           // work-log counters per candidate

// Device error flags (int32 each), set by kernels with atomicOr / atomicAdd.
enum DevFlag { kFlagQueueOverflow = 0, kFlagUnsorted = 1, kFlagBadType = 2, kFlagBadTime = 3, kNumFlags = 4 };

template <typename T>
struct TsLimits {
    static constexpr T lo() { return std::numeric_limits<T>::min(); }
    static constexpr T hi() { return std::numeric_limits<T>::max(); }
};

// Device blocks kept for reuse, for work that runs on one stream only: a
// block given back while kernels queued on that stream still use it is handed
// out again only to later work of the same stream, which runs after them.
// Blocks are taken best fit among those at most twice the request (plus
// 1 MiB); new ones come from hipMalloc.  Every block is freed by release(),
// which the owner calls after synchronising the stream.
class BlockCache {
public:
    BlockCache() = default;
    BlockCache(const BlockCache &) = delete;
    BlockCache &operator=(const BlockCache &) = delete;
    ~BlockCache() { release(); }
    hipError_t get(size_t b, void **p, size_t *got) {
        b = (b + 255) & ~(size_t)255;
        auto it = free_.lower_bound(b);
        if (it != free_.end() && it->first <= 2 * b + ((size_t)1 << 20)) {
            *p = it->second;
            *got = it->first;
            free_.erase(it);
            return hipSuccess;
        }
        hipError_t e = hipMalloc(p, b);
        if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
            // give the kept blocks back to the device (once no queued work
            // can use them) and try once more
            (void)hipGetLastError();
            (void)hipDeviceSynchronize();
            release();
            e = hipMalloc(p, b);
        }
        if (e != hipSuccess) return e;
        *got = b;
        return hipSuccess;
    }
    void put(void *p, size_t bytes) { free_.emplace(bytes, p); }
    void release() {
        for (auto &kv : free_) (void)hipFree(kv.second);
        free_.clear();
    }

private:
    std::multimap<size_t, void *> free_;
};

// While a CacheScope is alive, DevBuf::alloc of the calling thread takes its
// blocks from the scope's cache (and gives them back to it); otherwise it
// uses hipMalloc and hipFree.
struct CacheScope {
    static BlockCache *&current() {
        static thread_local BlockCache *c = nullptr;
        return c;
    }
    BlockCache *prev;
    explicit CacheScope(BlockCache *c) : prev(current()) { current() = c; }
    ~CacheScope() { current() = prev; }
    CacheScope(const CacheScope &) = delete;
    CacheScope &operator=(const CacheScope &) = delete;
};

// Owning device allocation (from the thread's cache scope, if any, which it
// must not outlive).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    BlockCache *cache = nullptr;  // where the block goes back to (null: hipFree)
    size_t block = 0;             // the cached block's size
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), cache(o.cache), block(o.block) {
        o.p = nullptr;
        o.bytes = 0;
        o.cache = nullptr;
    }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            reset();
            p = o.p;
            bytes = o.bytes;
            cache = o.cache;
            block = o.block;
            o.p = nullptr;
            o.bytes = 0;
            o.cache = nullptr;
        }
        return *this;
    }
    ~DevBuf() { reset(); }
    void reset() {
        if (p) {
            if (cache) cache->put(p, block);
            else (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
        cache = nullptr;
    }
    hipError_t alloc(size_t b) {
        reset();
        if (b == 0) b = 16;
        hipError_t e;
        if (BlockCache *c = CacheScope::current()) {
            e = c->get(b, &p, &block);
            if (e == hipSuccess) cache = c;
        } else {
            e = hipMalloc(&p, b);
        }
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        bytes = b;
        return hipSuccess;
    }
    template <typename U>
    U *as() const {
        return static_cast<U *>(p);
    }
};

struct Stream {
    int64_t n = 0;
    int32_t K = 0;
    int ts_kind = EPI_TS_I32;
    int64_t tmin = 0, tmax = 0;
    DevBuf types;       // int32[n]
    DevBuf times;       // T[n]
    DevBuf type_off;    // int32[K+1]
    DevBuf ts_by_type;  // T[n], grouped by type, each group in time order
    DevBuf pos_by_type; // int32[n], stream position of each ts_by_type entry
    // Tile-major copy of the index: tile b holds stream positions
    // [b*T, (b+1)*T); inside a tile the events are grouped by type (each
    // group in time order) starting at tile_loff[b*(K+1) + type].  T is the
    // largest power of two from tile_cap down to 256 whose tiles span less
    // than 2^29 - 1 time units (relative times of a tile then leave 3 bits
    // for a node index in a 32-bit unsigned key), else the largest spanning
    // less than 2^30, else tile_cap.
    int T = kDefaultTile;  // events per tile
    int tile_cap = kDefaultTile;  // largest T the stream may pick (the autotuner sets it)
    int64_t B = 0;      // number of tiles
    DevBuf tiled_ts;    // T[B*T] (the last tile is padded)
    DevBuf tile_loff;   // uint16[B*(K+1)]
    DevBuf tile_t0;     // T[B+1]: time of each tile's first event; [B] = type maximum
    std::vector<int32_t> h_off;  // host copy of type_off
    std::vector<int64_t> h_tile_t0;  // host copy of tile_t0 (widened)
    int64_t max_tile_span = -1;      // longest time from a tile's first event to the next tile's (or the last event)
    size_t ts_bytes() const { return ts_kind == EPI_TS_I64 ? 8 : 4; }
};

// Candidates of one launch class: same episode size N and queue capacity Q.
struct Group {
    int N = 0;
    int Q = 0;                   // ring capacity class of the deepest interval (LDS-ring machines)
    int C = 0;                   // most ring entries of one episode: sum of its intervals' bounds (lane machines)
    int64_t begin = 0, end = 0;  // slots [begin, end) of the grouped layout
    int64_t hspan = -1;          // longest span (sum of upper bounds) of its episodes (-1: unknown)
};

// Launch classes of the register-indexed lane machines: an episode's ring
// entries (the sum of its intervals' bounds) rounded up to one of these.
constexpr int kCapClasses = 23;
inline int cap_class_index(int c) {
    static constexpr int kC[kCapClasses] = {1,  2,  3,  4,  5,  6,  7,  8,  10, 12, 14, 16,
                                            20, 24, 28, 32, 40, 48, 56, 64, 80, 96, 112};
    for (int i = 0; i < kCapClasses; ++i)
        if (kC[i] >= c) return i;
    return kCapClasses - 1;
}
inline int cap_class_value(int i) {
    static constexpr int kC[kCapClasses] = {1,  2,  3,  4,  5,  6,  7,  8,  10, 12, 14, 16,
                                            20, 24, 28, 32, 40, 48, 56, 64, 80, 96, 112};
    return kC[i < 0 ? 0 : (i >= kCapClasses ? kCapClasses - 1 : i)];
}

// Ring capacity of a launch class: the smallest of 1, 2, 3, 4, 6, 8, 12, 16
// that holds queue bound b.
inline int queue_class(int64_t b) {
    static constexpr int kQ[] = {1, 2, 3, 4, 6, 8, 12, 16};
    for (int q : kQ)
        if (q >= b) return q;
    return 16;
}

struct CandSet {
    int32_t stream_id = 0;
    int64_t m = 0;
    // Grouped (launch-class-major) structure-of-arrays on the device; slot s
    // holds submission index orig[s].
    DevBuf types;   // int32 [8][m]
    DevBuf lo, hi;  // T [7][m]
    DevBuf orig;    // int32 [m]
    DevBuf counts;  // int32 [m], submission order
    DevBuf tau;     // T [m], submission order: each episode's last completion (type minimum: none)
    int64_t counted_n = -1;  // stream events covered by the counts (-1: never counted)
    DevBuf scratch; // per-segment speculative records of the last count
    DevBuf work;    // work log: int32 [m][kWork] (submission order) when enabled
    int64_t n_items = 0;  // work items of the last count
    bool logged = false;  // the last count recorded a work log
    DevBuf dmeasured;             // EPI_SCHED_MEASURED: logged work per grouped slot (float [m]), taken before a count resets the log
    bool has_measured = false;
    uint64_t cycles_plan = 0;     // batched plan whose per-item times the work log of the last count keeps (0: none)
    uint64_t last_plan = 0;       // batched plan of the last batched count that included the set (0: none)
    // Compact layout (level-wise mining): one episode size, types uint16
    // [N][m], interval ids uint8 [N-1][m] into a menu of (lo, hi) pairs
    // (T[2*n_menu]); slots are in submission order (orig unused).
    bool compact = false;
    DevBuf t16, iv, menu;
    // Optional pair-existence bitmaps of the menu (compact layout only; not
    // owned): bit (i, x, pos) of pred_bits says the event at tiled position
    // pos has an event of type x at a gap in menu interval i before it;
    // succ_bits the same after it.  Rows of B*T bits (T: the stream's tile).
    const uint64_t *pred_bits = nullptr;
    const uint64_t *succ_bits = nullptr;
    std::vector<Group> groups;
    bool counted = false;
    // host copy of the candidates (submission order; not for the compact
    // layout): sizes [m], types [m][8], lo and hi [m][7]
    std::vector<uint8_t> h_N;
    std::vector<int32_t> h_order;  // grouped slot -> submission index (the host copy of orig)
    std::vector<int32_t> h_types;
    std::vector<int64_t> h_lo, h_hi;
    DevBuf track_work, track_desc;  // working set of the tracking engine, kept for the next count
    bool stream_order = false;      // overlap decided in stream order (counted by the tracking engine only)
    int64_t max_span = 0;           // longest span (sum of upper bounds) of its episodes
    // Episodes with an interval deeper than the state machines' rings
    // (bound > kLaneMaxQ) sit in the last slots of the grouped layout, in no
    // group; the tracking engine counts them as this sub-set, whose counts
    // and last completions are then scattered to deep_idx (submission indices).
    std::unique_ptr<CandSet> deep;
    DevBuf deep_idx;  // int32 [deep->m]
};

// Launch options (epi_set_option).
struct CountOptions {
    int64_t segments = 0;          // 0: automatic; k >= 1: k segments per launch class
    int lanes = 0;                 // 0: automatic; else lanes per workgroup (64, 128 or 256)
    int64_t target_lanes = 262144; // automatic segmentation aims at this many (candidate, segment) lanes
    bool pair_filter = true;       // level-wise discovery: skip events with no constrained neighbour
    int mine_engine = 1;           // level-wise discovery: 1 extension engine, 0 state machines
    bool worklog = false;          // record per-candidate work counts and per-item times
    int64_t target_items = 0;      // batched mode: work items aimed at (0: 8 per compute unit)
    int64_t pair_filter_max_bytes = int64_t(1) << 30;
    int64_t mine_list_bytes = int64_t(8) << 30;  // extension engine: list-path budget per level
    bool allow_repeats = false;    // epi_submit_candidates accepts a type at several nodes
    int64_t mine_list_alphas = 65536;  // extension engine: list path below this many parent episodes
    bool stream_order = false;     // sets submitted now decide overlap in stream order
    bool lane_engine = true;       // state machines: register-indexed lane machines where they apply
    int ring_classes = 0;          // batched mode: 0 submission groups, 1 one group per size, 2 three per size
};

// One level of a level-wise discovery run: candidates of size N in
// structure-of-arrays form (types[k*m + i], interval ids iv[k*m + i]).
struct MineLevel {
    int N = 0;
    int64_t m = 0;
    // explicit candidates (state-machine engine): types [N][m], ids [N-1][m]
    std::vector<uint16_t> types;
    std::vector<uint8_t> iv;
    std::vector<int32_t> counts;  // [m] (host copy; for device-counted levels made on demand)
    DevBuf dcounts;               // int32 [m] on the device (extension engine)
    std::vector<int64_t> freq;    // indices with count > threshold (extension engine: host copy on demand)
    double gen_ms = 0, count_ms = 0, kernel_ms = 0;
    int64_t alg_bytes = -1;       // bytes the counting method must read and write (-1: not yet computed)
    int64_t nf = 0;                // frequent episodes
    // Extension engine: candidate c of level N >= 2 is alpha + one node, where
    // alpha indexes the frequent episodes of level N-1 (alpha-major order).
    // Level 2: alpha's extensions are every other frequent type x the menu.
    // Level >= 3: they are the frequent episodes [rlo, rlo + n) of level N-1
    // whose prefix is alpha's suffix, less [xlo, xhi), those whose last type
    // is alpha's first.
    bool implicit = false;
    int64_t nA = 0;
    DevBuf d_out_off;              // int64 [nA + 1] first candidate of each alpha (level >= 3)
    DevBuf d_rlo, d_xlo, d_xhi;    // int32 [nA] (level >= 3)
    // Frequent episodes on the device: candidate index, prefix parent (alpha:
    // the level N-1 episode it extends; level 1: unused), suffix parent (the
    // level N-1 episode its last N-1 nodes form), last type, last interval
    // id, first type, end-event count.  Level 1 keeps only flast = ffirst =
    // the frequent types.
    DevBuf d_fcand, d_fpar, d_fsuf, d_flast, d_fliv, d_ffirst, d_fnv;
    // host copies, made on demand for reading back (extend_host_view)
    bool host_view = false;
    std::vector<int64_t> out_off;
    std::vector<int32_t> rlo, xlo, xhi, h_fpar;
    std::vector<uint16_t> h_flast;
    std::vector<uint8_t> h_fliv;
    // chain lists of the frequent episodes: for every end event with an
    // occurrence, in time order, its time, the latest start of an occurrence
    // ending there, and its stream position
    DevBuf chain;                  // {T time, T start, int32 position} entries
    DevBuf cbeg;                   // int64 [nf + 1]: first entry of each chain list (length: d_fnv)
    int64_t chain_total = 0;       // entries in the chain lists of the frequent episodes
    int32_t list_seg = 0;          // list path: pieces per alpha (0: not taken)
    int64_t walked = 0;            // stream positions the extension walk visited (counting pass)
};

struct Mine {
    int engine = 1;  // 1: extension engine (default), 0: state-machine engine
    int32_t stream_id = 0;
    int64_t max_span = 0;  // longest span of any episode the run may count (longest menu end x (sizes - 1))
    std::vector<int64_t> menu_lo, menu_hi;
    int64_t threshold = 0;
    std::vector<MineLevel> levels;
    DevBuf pred_bits, succ_bits;  // pair-existence bitmaps of the menu (may be empty)
    // extension engine: the stream's types as uint16 and, for every position
    // p, the first position whose time exceeds time[p] + H (H = the longest
    // menu interval end)
    DevBuf ty16, wend;
    DevBuf chain1;  // the per-type index as chain entries (level 2's alphas)
    // list path: device bytes the end-event lists of every candidate of a
    // level may take (larger: count and write walks)
    int64_t list_budget = 0;
    int64_t list_alphas = 65536;  // levels with fewer alphas than this take the list path
    double bits_ms = 0;
    // pinned host slots (the context's) that device scalars are copied to,
    // several per synchronisation
    int64_t *stage = nullptr;
};

// Cost model (epi_mlp.hip): parameters, Adam moments, gradient, activations.
struct Mlp {
    int F = 0;
    int step = 0;
    float lr = 1e-3f, b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    DevBuf p, m, v, g, act;
    size_t cap = 0;
    // standardisation of the cost model around the network:
    // prediction = y_sd * net((x - x_mu) * x_isd) + y_mu (identity after init)
    std::vector<float> x_mu, x_isd;
    float y_mu = 0.f, y_sd = 1.f;
    DevBuf norm;  // x_mu[F], x_isd[F] on the device
    bool ready() const { return p.p != nullptr; }
};

// A batched count, planned once and kept as an instantiated graph: the
// scheduler kernels (costs, device sorts, item order), the queue clear, the
// persistent launches (parallel branches) and the reconciliation.  A later
// count of the same sets, schedule and options replays it.
struct BatchPlan {
    std::vector<int64_t> key;      // identity (sets, streams, buffers, options, schedule, model)
    std::vector<int32_t> set_ids;
    uint64_t id = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    DevBuf units, tmpl, items, queue, rec, cycles;
    DevBuf ssets, sgroups, gid, sunits, X, y, k0, k1, v0, v1, ik0, ik1, iv0, iv1, hist;
    int64_t n_items = 0;
    int64_t launches = 0;
    // the schedule, for reading back: each set's first global slot, the
    // permutation buffer (null: submission order within each group) and the
    // units' (set, first slot, size, lane width)
    std::vector<int64_t> soff;
    const int32_t *perm = nullptr;
    struct UnitView {
        int set;
        int64_t begin, G;
        int W;
    };
    std::vector<UnitView> uview;
    BatchPlan() = default;
    BatchPlan(const BatchPlan &) = delete;
    BatchPlan &operator=(const BatchPlan &) = delete;
    ~BatchPlan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// The context's batched plans (most recently used last) and the branch
// streams and events the plans' graphs were captured with (created once).
struct BatchCache {
    static constexpr size_t kMaxPlans = 8;
    static constexpr int kBranches = 4;
    std::vector<std::unique_ptr<BatchPlan>> plans;
    hipStream_t br[kBranches] = {};
    hipEvent_t joined[kBranches] = {};
    hipEvent_t fork = nullptr;
    uint64_t next_id = 1;
    int64_t built = 0;     // plans captured and instantiated
    int64_t replays = 0;   // graph launches of a kept plan
    BatchCache() = default;
    BatchCache(const BatchCache &) = delete;
    BatchCache &operator=(const BatchCache &) = delete;
    ~BatchCache() { clear(); }
    hipError_t branches();
    BatchPlan *find(const std::vector<int64_t> &key);
    BatchPlan *find_id(uint64_t id);
    // plans are dropped only after the device is idle (their graphs may run)
    void evict_set(int32_t id);
    void evict_all();
    void clear();
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // blocks of the mining working set (all of it runs on `stream`), kept for
    // reuse until the context is destroyed
    BlockCache cache;
    int64_t *stage = nullptr;  // pinned host slots of the mining runs (kStageSlots)
    std::string err;
    std::map<int32_t, std::unique_ptr<Stream>> streams;
    std::map<int32_t, std::unique_ptr<CandSet>> sets;
    std::map<int32_t, std::unique_ptr<Mine>> mines;
    int32_t next_id = 1;
    DevBuf flags;  // int32[kNumFlags]
    CountOptions opt;
    Mlp mlp;
    BatchCache batch;
};

// Queue capacity bound of one constraint (lo, hi]: at most
// 1 + floor(hi / (hi - lo + 1)) disjoint merged acceptance intervals can be
// live at once.
inline int64_t queue_bound(int64_t lo, int64_t hi) {
    return 1 + hi / (hi - lo + 1);
}

// ---- launchers -------------------------------------------------------------
hipError_t build_type_index(Stream &s, hipStream_t st);
hipError_t validate_stream_device(const int32_t *d_types, const void *d_times, int64_t n, int ts_kind,
                                  int32_t K, int32_t *d_flags, hipStream_t st);
// ext_scratch (optional): device memory of ext_bytes for the segment records,
// used instead of the set's own (then nothing is allocated and nothing waits
// on the host; hipErrorOutOfMemory if a group's records do not fit).
hipError_t launch_count(const Stream &s, CandSet &c, const CountOptions &opt, int32_t *d_flags, hipStream_t st,
                        unsigned char *ext_scratch = nullptr, size_t ext_bytes = 0);
// Static device scratch of the allocation-free count (epi_noalloc.hip):
// noalloc_init looks up its address on the current device (once per device),
// noalloc_scratch returns it (null before init), noalloc_scratch_bytes its size.
hipError_t noalloc_init(int device);
unsigned char *noalloc_scratch(int device);
size_t noalloc_scratch_bytes();
// Segments of a plain count of a group of G episodes on stream s (and the
// tiles per segment, *S_out), and the bytes of its segment records.
int64_t plain_segments(const Stream &s, int64_t G, const CountOptions &opt, int64_t *S_out);
size_t plain_record_bytes(const Stream &s, int64_t P, int64_t G);
// Count set c by per-event tracking of each episode's nodes and the greedy
// over the latest-start intervals (epi_track.hip); returns when done.
hipError_t launch_count_tracking(const Stream &s, CandSet &c, hipStream_t st);
// Count set c's deep episodes (CandSet::deep) by tracking and scatter their
// counts and last completions into c's; returns when done (no-op without).
hipError_t count_deep_subset(const Stream &s, CandSet &c, hipStream_t st);
// Add to set c's counts the occurrences completed by the stream's events
// after the first c.counted_n (B = the first of their times).
hipError_t launch_count_append(const Stream &s, CandSet &c, int64_t B, int32_t *d_flags, hipStream_t st);
// Batched count of several candidate sets (possibly on different streams) in
// one graph launch of persistent kernels, one per episode size.  sched:
// EPI_SCHED_RR (submission order), EPI_SCHED_LEARNED (the cost model's
// predictions; round robin without a model), EPI_SCHED_MEASURED (the work
// the set's previous count logged) or EPI_SCHED_HEURISTIC (sum of
// the types' event counts).
struct BatchRef {
    const Stream *s;
    CandSet *c;
};
// ids: the sets' ids (plan identity).  Returns after queuing the graph on st
// (asynchronous).
hipError_t launch_count_batched(std::vector<BatchRef> &sets, const std::vector<int32_t> &ids, int sched,
                                const CountOptions &opt, Mlp &mlp, BatchCache &cache, int32_t *d_flags,
                                hipStream_t st);
// Count every candidate of one mining level on the device (compact layout);
// fills L.counts and the timing fields.
hipError_t count_mine_level(const Stream &s, const Mine &mn, MineLevel &L, const CountOptions &opt, int32_t *d_flags,
                            hipStream_t st);
int queue_class_of(int64_t bound);
// Extension engine of level-wise discovery (epi_extend.hip): count level 1,
// then count level N (>= 2) from level N-1's frequent episodes and chain lists,
// select its frequent episodes and write their chain lists.  Menus of up to
// kExtMaxMenu intervals.
constexpr int kStageSlots = 8;     // pinned host slots of a mining run
constexpr int kExtMaxMenu = 8;
hipError_t extend_prepare(const Stream &s, Mine &mn, hipStream_t st);
hipError_t extend_level1(const Stream &s, Mine &mn, hipStream_t st);
hipError_t extend_level(const Stream &s, Mine &mn, int N, hipStream_t st);
// algorithmic bytes of an extension-engine level (computed on first use)
int64_t extend_level_bytes(const Stream &s, Mine &mn, int level);
// Host copies of an extension-engine run's levels 2..level, for reading back.
hipError_t extend_host_view(Mine &mn, int level);
// Candidate c / frequent episode f of an implicit level (after
// extend_host_view): types[N], interval ids[N-1].
void implicit_candidate(const Mine &mn, int level, int64_t c, int32_t *types, int *ivs);
void extend_frequent(const Mine &mn, int level, int64_t f, int32_t *types, int *ivs);
// Cost model (epi_mlp.hip).
int64_t mlp_n_params(int F);
hipError_t mlp_init(Mlp &net, int F, uint64_t seed);
hipError_t mlp_forward_device(Mlp &net, const float *dX, int64_t B, float *dy, hipStream_t st);
hipError_t mlp_grad_device(Mlp &net, const float *dX, const float *dt, int64_t B, float *dg, float *loss,
                           hipStream_t st);
hipError_t mlp_adam_device(Mlp &net, const float *dg, hipStream_t st);
hipError_t mlp_set_scaling(Mlp &net, const float *x_mu, const float *x_isd, float y_mu, float y_sd);
// the cost model's prediction for B device samples; standardises dX in place
hipError_t costmodel_predict_device(Mlp &net, float *dX, int64_t B, float *dy, hipStream_t st);
// Cost-model features of every candidate of a set, in grouped slot order
// (float [G][kFeatures]) (epi_sched.hip).
hipError_t candidate_features(const Stream &s, const CandSet &c, float *dX, hipStream_t st);
// Pair-existence bitmaps of an interval menu over a stream (epi_pairs.hip).
hipError_t build_pair_bits(const Stream &s, Mine &mn, hipStream_t st);
// Candidate generation of level-wise discovery (epi_mine.hip).
void gen_level1(int32_t K, MineLevel &L);
void gen_level2(const MineLevel &F1, int n_menu, MineLevel &L);
void gen_join(const MineLevel &prev, MineLevel &L);
void select_frequent(MineLevel &L, int64_t threshold);

}  // namespace epi
