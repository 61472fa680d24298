// Arguments of the state-machine counting kernels (shared by the LDS-ring
// machines of epi_tiled.hip and the register-indexed machines of
// epi_lane.hip) and the interface of the latter.
#pragma once

#include "epi_fsm.h"

namespace epi {

constexpr int kRecFirst = 4;  // speculative completion times recorded per segment

template <typename T>
struct CountArgs {
    const T *tiled;
    const uint16_t *loff;
    const T *tile_t0;
    const T *ts_by_type;
    const int32_t *type_off;
    int64_t B;
    int32_t K;
    const int32_t *ctypes;
    const T *clo;
    const T *chi;
    const uint16_t *t16;  // compact layout (when non-null): types
    const uint8_t *iv;    //   interval ids into menu
    const T *menu;        //   (lo, hi) pairs
    const uint64_t *pbits;  // pair-existence bitmaps (filtered mode)
    const uint64_t *sbits;
    int64_t rwords;         // words per bitmap row (B * T / 64)
    int32_t tile;           // events per tile of the stream
    int64_t m;
    int64_t begin;  // first slot of the group
    int64_t G;      // group size
    int32_t Q;
    int32_t P;
    int64_t S;  // tiles per segment
    const int32_t *orig;
    int32_t *counts;
    int32_t *rec_cnt;
    T *rec_last;
    T *rec_first;
    // reconciliation pre-pass: each segment's true completions and last true
    // completion when re-run from pre_tau, the last completion the records
    // of the earlier segments give (null: no pre-pass)
    int32_t *pre_cnt;
    T *pre_last;
    T *pre_tau;
    // each candidate's last completion (submission order; the type minimum
    // for none), kept for counting appended events (null: not kept)
    T *tau;
    int32_t *flags;
    uint32_t off_qse, off_tbuf, off_qh, off_obuf, off_misc;
    int32_t C;            // epi_lane.hip: ring entries per lane (off_qse: the rings)
    const int32_t *perm;  // lane slot -> candidate slot (scheduler order); null = identity
    int32_t *work;        // work log: kWork counters per candidate (submission order); null = off
    int64_t *cycles;      // work log: wall-clock start/end per work item; null = off
};

// Persistent form: one work item = (unit, lane block, segment).
struct WorkItem {
    int32_t unit;
    int32_t p;
    int64_t blk;
};

// ---- device scheduler of the batched count (epi_sched.hip) -------------------
// One set of a batched count, as the scheduler kernels see it.
struct SchedSet {
    const int32_t *type_off;  // the stream's per-type offsets [K+1]
    const int32_t *ctypes;    // grouped types [8][m]
    const void *clo, *chi;    // grouped bounds [7][m] (the stream's time type)
    const float *measured;    // logged work per grouped slot (null: none)
    int64_t m;
    int64_t off;              // the set's first slot in the count's global slot order
};
// One launch group (set, episode size) of the global slot order.
struct SchedGroup {
    int32_t set;
    int32_t N;
};
// One unit of the batched count: its first global slot, size, the lane width
// of its launch class, its segments and the rank of its launch class.
struct SchedUnit {
    int64_t gbase;
    int64_t G;
    int32_t W;
    int32_t P;
    int32_t cls;
    int32_t pad;
};
// Cost of every global slot into y: the cost model's log-work prediction
// (EPI_SCHED_LEARNED; X: feature scratch [M][kFeatures]), the summed event
// counts of the types (EPI_SCHED_HEURISTIC) or the logged work (EPI_SCHED_MEASURED).
hipError_t sched_costs(int ts_kind, int sched, const SchedSet *sets, const SchedGroup *groups, const int32_t *gid,
                       int64_t M, Mlp &mlp, float *X, float *y, hipStream_t st);
// Sort keys (group, descending cost) and values (local slot) of every global slot.
hipError_t sched_keys(const SchedSet *sets, const SchedGroup *groups, const int32_t *gid, int64_t M, const float *y,
                      bool log_cost, uint64_t *key, int32_t *val, hipStream_t st);
// Sort keys (class rank, descending cost) and values (index) of the work items
// tmpl, from the candidates' sorted keys skey.
hipError_t sched_item_keys(const WorkItem *tmpl, int64_t n, const SchedUnit *units, const uint64_t *skey,
                           uint64_t *key, int32_t *val, hipStream_t st);
hipError_t sched_gather_items(const WorkItem *tmpl, const int32_t *idx, int64_t n, WorkItem *out, hipStream_t st);
// c.dmeasured = each grouped slot's logged work (visits + records + queries).
hipError_t measured_costs(const CandSet &c, hipStream_t st);

// ---- register-indexed lane machines (epi_lane.hip) --------------------------
// A group of episodes can be counted by them when the stream's tiles are
// short enough for int32 relative times (lane_rel_ok) and every interval's
// ring bound is at most kLaneMaxQ.  pk: relative times stay below 2^29 - 1,
// so (time, node) pack into one 32-bit unsigned key below its all-ones end
// marker.
constexpr int kLaneMaxQ = 15;

inline bool lane_rel_ok(int64_t max_tile_span, int64_t hspan) {
    return max_tile_span >= 0 && hspan >= 0 && hspan < (int64_t(1) << 29) && max_tile_span < (int64_t(1) << 30) &&
           max_tile_span + 2 * hspan < (int64_t(1) << 31) - 64;
}
inline bool lane_pk_ok(int64_t max_tile_span) {
    return max_tile_span >= 0 && max_tile_span < (int64_t(1) << 29) - 1;
}

// Ring entries of an episode: sum over its intervals of the ring bound.
inline int lane_ring_entries(int N, const int64_t *lo, const int64_t *hi) {
    int c = 0;
    for (int j = 0; j + 1 < N; ++j) c += (int)(1 + hi[j] / (hi[j] - lo[j] + 1));
    return c;
}

struct LaneLayout {
    uint32_t off_ring, off_tbuf, off_obuf, off_misc, total;
};
LaneLayout lane_layout(int C, int W, int K, int tile);

// Kernel symbols (for attributes and occupancy) and launches; wl: the work
// log is kept (a.work set).
template <typename T>
const void *lane_tiled_fn(int N, bool pk, bool wl);
template <typename T>
const void *lane_persistent_fn(int N, bool pk, bool wl);
template <typename T>
hipError_t lane_launch_tiled(const CountArgs<T> &a, int N, bool pk, dim3 grid, int W, uint32_t lds, hipStream_t st);
template <typename T>
hipError_t lane_launch_persistent(int N, bool pk, bool wl, unsigned grid, int W, uint32_t lds, hipStream_t st,
                                  const CountArgs<T> *units, const WorkItem *items, int64_t n_items, int64_t item_base,
                                  unsigned long long *queue);

}  // namespace epi
