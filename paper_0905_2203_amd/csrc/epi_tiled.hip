// Tiled counting engine and exact segment reconciliation.
//
// k_count_tiled: a workgroup holds W candidate episodes of one size N (one
// lane each) and walks a range of stream tiles.  Each tile (T stream
// positions, grouped by type) is copied into LDS with coalesced 16-byte
// loads and shared by all W lanes; a lane merges, in time order, the tile's
// events of its own N types only (the per-tile type offsets give each
// group) and feeds them to its state machine (epi_fsm.h).
//
// Segments.  With P > 1 the tiles are cut into P segments at tile starts;
// segment p owns times [B_p, B_{p+1}).  Every occurrence ending at or after
// B_p starts at or after B_p - H (H = sum of the upper bounds), so workgroup
// (block, p) runs the machine speculatively from B_p - H as if nothing had
// happened before (last completion = B_p - H - 1) and records, for times in
// its own segment, the number of completions, the first kRecFirst completion
// times and the last one.
//
// k_reconcile: one lane per candidate walks the segments in order carrying
// tau, the last true completion before the segment.  If tau < B_p - H the
// speculative record is exact: the true machine holds only partial
// occurrences that started before B_p - H, and those can complete neither
// before B_p (tau is the last completion before B_p) nor after it (they are
// too old).  Otherwise the lane re-runs the machine from the state right
// after the completion at tau (last completion = tau, no partial state) over
// the events after tau, from the global per-type index.  Both machines are in
// the same state right after any completion time they share, so as soon as
// the re-run completes at a time the speculative run also recorded, the rest
// of the speculative count is taken as is; otherwise the re-run covers the
// whole segment.  It also stops at B_p + H if neither machine has completed
// by then: from there on both hold the same state.
//
// The walk over the segments is sequential in tau, but tau is nearly always
// the last completion the earlier segments' records give (a re-run that
// meets the speculative run ends on the record's last completion).  So a
// pre-pass (k_reconcile_pre, one lane per candidate and segment, all in
// parallel) re-runs every segment from that predicted tau, and the
// sequential walk takes the pre-pass result whenever its true tau equals the
// prediction, re-running itself only when it does not.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include <cstring>
#include <type_traits>

#include "epi_count.h"
#include "epi_sort.h"

namespace epi {

namespace {

template <typename T, int N, typename R>
__device__ __forceinline__ T load_candidate(const CountArgs<T> &a, LaneFsm<R, N> &f, int64_t slot, int32_t *ty,
                                           T *lo, T *hi) {
    T H = 0;
    if (a.t16) {
#pragma unroll
        for (int k = 0; k < N; ++k) ty[k] = a.t16[(int64_t)k * a.m + slot];
#pragma unroll
        for (int k = 0; k + 1 < N; ++k) {
            const int id = a.iv[(int64_t)k * a.m + slot];
            lo[k] = a.menu[2 * id];
            hi[k] = a.menu[2 * id + 1];
        }
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) ty[k] = a.ctypes[(int64_t)k * a.m + slot];
#pragma unroll
        for (int k = 0; k + 1 < N; ++k) {
            lo[k] = a.clo[(int64_t)k * a.m + slot];
            hi[k] = a.chi[(int64_t)k * a.m + slot];
        }
    }
#pragma unroll
    for (int k = 0; k + 1 < N; ++k) {
        Pair<R> v;
        v.s = (R)lo[k];
        v.e = (R)hi[k];
        f.lohi[k * f.W + f.lane] = v;
        H += hi[k];
    }
    return H;
}

// One work item: lane block `blk` of a launch unit, time segment p.  REL
// (int64 streams whose tiles are short enough, rel_ok): the machines and the
// staged tile hold int32 offsets from the current tile's first time, which
// halves their LDS.
template <typename T, int N, bool FILT, bool REL>
__device__ __forceinline__ void count_item(const CountArgs<T> &a, int64_t blk, int p, int64_t item,
                                           unsigned char *smem) {
    using R = std::conditional_t<REL, int32_t, T>;
    constexpr T kMin = TsLimits<T>::lo();
    constexpr T kEnd = TsLimits<T>::hi();
    constexpr R rEnd = TsLimits<R>::hi();
    constexpr int L = N > 1 ? N - 1 : 1;
    const int W = blockDim.x, lane = threadIdx.x;
    const int64_t s = blk * W + lane;
    const bool active = s < a.G;
    const int64_t lslot = a.begin + (active ? s : 0);
    const int64_t slot = a.perm ? (int64_t)a.perm[lslot] : lslot;
    if (a.cycles && lane == 0) a.cycles[2 * item] = (int64_t)wall_clock64();
    R *tbuf = reinterpret_cast<R *>(smem + a.off_tbuf);
    uint16_t *obuf = reinterpret_cast<uint16_t *>(smem + a.off_obuf);
    T *misc = reinterpret_cast<T *>(smem + a.off_misc);

    LaneFsm<R, N> f;
    f.lohi = reinterpret_cast<Pair<R> *>(smem);
    f.qse = reinterpret_cast<Pair<R> *>(smem + a.off_qse);
    f.qh = reinterpret_cast<uint32_t *>(smem + a.off_qh);
    f.W = W;
    f.lane = lane;
    f.Q = a.Q;
    f.gen = 0;
    int32_t ty[N];
    T lo[L], hi[L];
    const T H = load_candidate<T, N, R>(a, f, slot, ty, lo, hi);
    R hiR[L];
#pragma unroll
    for (int k = 0; k + 1 < N; ++k) hiR[k] = (R)hi[k];
    f.clear_all();
    // vf[k] (k >= 1): no node-k event before this time can meet constraint k
    // with the intervals currently recorded at node k-1 (a lower bound on the
    // earliest interval start + 1; the type maximum when none is recorded).
    R vf[N];
#pragma unroll
    for (int k = 0; k < N; ++k) vf[k] = rEnd;
    // pair-existence rows of each node (filtered mode)
    int64_t prow[N], srow[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        prow[k] = 0;
        srow[k] = 0;
        if (FILT) {
            if (k >= 1) prow[k] = ((int64_t)a.iv[(int64_t)(k - 1) * a.m + slot] * a.K + ty[k - 1]) * a.rwords;
            if (k + 1 < N) srow[k] = ((int64_t)a.iv[(int64_t)k * a.m + slot] * a.K + ty[k + 1]) * a.rwords;
        }
    }

    const int64_t b0 = (int64_t)p * a.S;
    const int64_t b1 = b0 + a.S < a.B ? b0 + a.S : a.B;
    const T Bp = p == 0 ? kMin : a.tile_t0[b0];
    const T Ep = p == a.P - 1 ? kEnd : a.tile_t0[b1];
    const T e0 = p == 0 ? kMin : (T)(Bp - H - 1);

    // first tile: the last one starting before B_p - max H of the workgroup
    int64_t bs = b0;
    if (p > 0) {
        T hm = active ? H : T(0);
        for (int d = 32; d >= 1; d >>= 1) {
            const T o = __shfl_xor(hm, d, 64);
            hm = o > hm ? o : hm;
        }
        if ((lane & 63) == 0) misc[lane >> 6] = hm;
        __syncthreads();
        if (lane == 0) {
            T mx = 0;
            for (int w = 0; w < (W + 63) / 64; ++w) mx = misc[w] > mx ? misc[w] : mx;
            const T target = (T)(Bp - mx);
            int64_t blo = 0, bhi = b0;  // last b in [0, b0] with tile_t0[b] < target, else 0
            if (a.tile_t0[0] >= target) {
                bhi = 0;
            } else {
                while (blo < bhi) {
                    const int64_t mid = (blo + bhi + 1) / 2;
                    if (a.tile_t0[mid] < target) blo = mid; else bhi = mid - 1;
                }
            }
            misc[8] = (T)blo;
        }
        __syncthreads();
        bs = (int64_t)misc[8];
    }

    // origin of the relative times (REL): the first time of the tile walked
    T t0b = REL ? a.tile_t0[bs] : T(0);
    if (REL) {
        // e0 - t0b, or -2 (before the tile) when e0 is earlier than that
        const bool before = e0 < t0b && (uint64_t)t0b - (uint64_t)e0 > 2u;
        f.e = before ? R(-2) : (R)(int64_t)((uint64_t)e0 - (uint64_t)t0b);
    } else {
        f.e = (R)e0;
    }
    int32_t cnt = 0;
    T last = kMin;
    uint32_t w_visits = 0, w_records = 0, w_queries = 0, w_done = 0;
    for (int64_t b = bs; b < b1; ++b) {
        __syncthreads();
        R BpR, EpR;  // segment bounds in the machine's time
        if (REL) {
            const T nb = a.tile_t0[b];
            const R d = (R)(nb - t0b);  // the previous tile's span (0 for the first)
            if (d != 0) {
                f.rebase(d);
#pragma unroll
                for (int k = 0; k < N; ++k)
                    if (vf[k] != rEnd) vf[k] = vf[k] - d < R(-1) ? R(-1) : (R)(vf[k] - d);
                f.e = f.e - d < R(-2) ? R(-2) : (R)(f.e - d);
            }
            t0b = nb;
            const T *src = a.tiled + b * a.tile;
            // (the last tile's padding is never read; wrapping keeps it defined)
            for (int i = lane; i < a.tile; i += W) {
                const int64_t v = (int64_t)((uint64_t)src[i] - (uint64_t)t0b);
                tbuf[i] = v > (int64_t)INT32_MAX ? INT32_MAX : (v < -1 ? R(-1) : (R)v);
            }
            BpR = Bp <= t0b ? R(-1) : (Bp - t0b >= (T)INT32_MAX ? rEnd : (R)(Bp - t0b));
            EpR = (Ep == kEnd || Ep - t0b >= (T)INT32_MAX) ? rEnd : (R)(Ep - t0b);
        } else {
            const uint4 *src = reinterpret_cast<const uint4 *>(a.tiled + b * a.tile);
            uint4 *dst = reinterpret_cast<uint4 *>(tbuf);
            for (int i = lane; i < (int)(a.tile * sizeof(T) / 16); i += W) dst[i] = src[i];
            BpR = (R)Bp;
            EpR = (R)Ep;
        }
        for (int i = lane; i <= a.K; i += W) obuf[i] = a.loff[b * (a.K + 1) + i];
        __syncthreads();
        if (!active) continue;
        // Per node: the tile range [rs, re) of its type; unfiltered lanes walk
        // it with a cursor, filtered lanes walk the set bits of the words of
        // (range & predecessor-exists & successor-exists).
        int cur[N], stop[N];
        int wi[N], we[N];
        uint64_t msk[N], nmsk[N];  // current word's bits, next word's (prefetched)
        R head[N];
        const int64_t wbase = b * (a.tile / 64);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            cur[k] = obuf[ty[k]];
            stop[k] = obuf[ty[k] + 1];
            wi[k] = 0;
            we[k] = -1;
            msk[k] = 0;
            nmsk[k] = 0;
        }
        // bits of word w of node k's range that may matter
        auto word_bits = [&](const int k, const int w) -> uint64_t {
            const int base = w << 6;
            const int l0 = (cur[k] > base ? cur[k] : base) - base;
            const int l1 = (stop[k] < base + 64 ? stop[k] : base + 64) - base;
            if (l1 <= l0) return 0;
            uint64_t m = (l1 - l0 == 64 ? ~0ull : ((1ull << (l1 - l0)) - 1ull)) << l0;
            if (k >= 1) m &= a.pbits[prow[k] + wbase + w];
            if (k + 1 < N) m &= a.sbits[srow[k] + wbase + w];
            return m;
        };
        auto filt_head = [&](const int k) -> R {
            while (msk[k] == 0 && wi[k] < we[k]) {
                ++wi[k];
                msk[k] = nmsk[k];
                nmsk[k] = wi[k] < we[k] ? word_bits(k, wi[k] + 1) : 0ull;
            }
            if (msk[k] == 0) return rEnd;
            const R v = tbuf[(wi[k] << 6) + (int)__builtin_ctzll(msk[k])];
            return v < EpR ? v : rEnd;
        };
#pragma unroll
        for (int k = 0; k < N; ++k) {
            if (FILT) {
                if (cur[k] < stop[k]) {
                    wi[k] = cur[k] >> 6;
                    we[k] = (stop[k] - 1) >> 6;
                    msk[k] = word_bits(k, wi[k]);
                    nmsk[k] = wi[k] < we[k] ? word_bits(k, wi[k] + 1) : 0ull;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            if (FILT) {
                head[k] = filt_head(k);
            } else {
                const R v = cur[k] < stop[k] ? tbuf[cur[k]] : rEnd;
                head[k] = v < EpR ? v : rEnd;
            }
        }
        while (true) {
            // next event of the lane's types (any order among equal times)
            R t = head[0];
            int j = 0;
#pragma unroll
            for (int k = 1; k < N; ++k) {
                if (head[k] < t) {
                    t = head[k];
                    j = k;
                }
            }
            if (t == rEnd) break;
            ++w_visits;
            // per-node values of the selected node
            R vfj = vf[0], nxt = rEnd, hij = R(0);
#pragma unroll
            for (int k = 1; k < N; ++k)
                if (k == j) vfj = vf[k];
#pragma unroll
            for (int k = 0; k + 1 < N; ++k) {
                if (k == j) {
                    nxt = head[k + 1];
                    hij = hiR[k];
                }
            }
            // Exact rejections that need no LDS state: a start not after the
            // last completion; a query below vf; a record whose acceptance
            // interval ends before the next event of the following node
            // (only when that event is known, i.e. inside this tile).
            const bool late_next = j + 1 < N && nxt != rEnd && nxt > (R)(t + hij);
            const bool useless = (j == 0 ? t <= f.e : t < vfj) || late_next;
            if (!useless) {
                bool done = false;
                if (j == 0) {
                    if (N == 1) {
                        f.e = t;
                        done = true;
                    } else {
                        const R ns = f.record(0, t, a.flags);
                        ++w_records;
                        vf[1] = vf[1] < (R)(ns + 1) ? vf[1] : (R)(ns + 1);
                    }
                } else {
                    R nv;
                    ++w_queries;
                    const bool ok = f.query(j - 1, t, &nv);
                    if (!ok) {
#pragma unroll
                        for (int k = 1; k < N; ++k)
                            if (k == j) vf[k] = nv;
                    } else if (j == N - 1) {
                        f.e = t;
                        f.gen ^= 1u;
#pragma unroll
                        for (int k = 0; k < N; ++k) vf[k] = rEnd;
                        done = true;
                    } else {
                        const R ns = f.record(j, t, a.flags);
                        ++w_records;
#pragma unroll
                        for (int k = 1; k + 1 < N; ++k)
                            if (k == j) vf[k + 1] = vf[k + 1] < (R)(ns + 1) ? vf[k + 1] : (R)(ns + 1);
                    }
                }
                if (done) ++w_done;
                if (done && t >= BpR) {
                    const T ta = (T)t + t0b;  // absolute
                    if (a.P > 1 && cnt < kRecFirst) a.rec_first[((int64_t)p * kRecFirst + cnt) * a.G + s] = ta;
                    ++cnt;
                    last = ta;
                }
            }
            // advance the selected node
            if (FILT) {
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    if (k == j) {
                        msk[k] &= msk[k] - 1ull;
                        head[k] = filt_head(k);
                    }
                }
            } else {
                int c = cur[0], st = stop[0];
#pragma unroll
                for (int k = 1; k < N; ++k) {
                    if (k == j) {
                        c = cur[k];
                        st = stop[k];
                    }
                }
                ++c;
                R v = c < st ? tbuf[c] : rEnd;
                v = v < EpR ? v : rEnd;
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    if (k == j) {
                        cur[k] = c;
                        head[k] = v;
                    }
                }
            }
        }
    }
    if (a.cycles && lane == 0) a.cycles[2 * item + 1] = (int64_t)wall_clock64();
    if (!active) return;
    const int64_t o = a.orig ? a.orig[slot] : slot;
    if (a.work) {
        int32_t *w = a.work + o * kWork;
        atomicAdd(w + 0, (int32_t)w_visits);
        atomicAdd(w + 1, (int32_t)w_records);
        atomicAdd(w + 2, (int32_t)w_queries);
        atomicAdd(w + 3, (int32_t)w_done);
        atomicMax(w + 4, (int32_t)f.maxq);
    }
    if (a.P == 1) {
        a.counts[o] = cnt;
        if (a.tau) a.tau[o] = last;
    } else {
        a.rec_cnt[(int64_t)p * a.G + s] = cnt;
        a.rec_last[(int64_t)p * a.G + s] = last;
    }
}

template <typename T, int N, bool FILT, bool REL>
__global__ __launch_bounds__(256) void k_count_tiled(CountArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    count_item<T, N, FILT, REL>(a, blockIdx.x, blockIdx.y, (int64_t)blockIdx.y * gridDim.x + blockIdx.x, smem);
}

// Persistent form: every workgroup takes work items (unit, lane block,
// segment) from a device queue until it is empty.  Units may belong to
// different streams and candidate sets; they share the LDS layout.

template <typename T, int N, bool FILT, bool REL>
__global__ __launch_bounds__(256) void k_count_persistent(const CountArgs<T> *__restrict__ units,
                                                          const WorkItem *__restrict__ items, int64_t n_items,
                                                          int64_t item_base, unsigned long long *__restrict__ queue) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int64_t next;
    while (true) {
        if (threadIdx.x == 0) next = (int64_t)atomicAdd(queue, 1ull);
        __syncthreads();
        const int64_t it = next;
        __syncthreads();
        // uniform: every wave of the group exits; unsigned, so that a counter
        // that was not cleared (any value) ends the loop instead of indexing
        // items[] out of range
        if ((uint64_t)it >= (uint64_t)n_items) break;
        const WorkItem w = items[it];
        const CountArgs<T> a = units[w.unit];
        count_item<T, N, FILT, REL>(a, w.blk, w.p, item_base + it, smem);
    }
}

// p[0..n) = v, any n (one workgroup strides over it)
__global__ void k_fill_u64(unsigned long long *p, int n, unsigned long long v) {
    for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) p[i] = v;
}

template <typename T>
__global__ void k_zero_counts(const int32_t *__restrict__ orig, int64_t G, int32_t *__restrict__ counts,
                              T *__restrict__ tau) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < G) {
        counts[orig ? orig[i] : i] = 0;
        if (tau) tau[orig ? orig[i] : i] = TsLimits<T>::lo();
    }
}

// first index in [lo, hi) with ts[index] > x
template <typename T>
__device__ __forceinline__ int32_t upper_bound(const T *ts, int32_t lo, int32_t hi, T x) {
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (ts[mid] <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// First index after time x in each node's range [lo_k, hi_k) of the per-type
// index: the N binary searches advance in lockstep, so that each step's
// loads are issued together.
template <typename T, int N>
__device__ __forceinline__ void first_after(const T *ts, const int32_t (&lo_)[N], const int32_t (&hi_)[N], T x,
                                            int32_t (&cur)[N]) {
    int32_t hb[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        cur[k] = lo_[k];
        hb[k] = hi_[k];
    }
    for (;;) {
        bool any = false;
        int32_t mid[N];
        T v[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            mid[k] = cur[k] + (hb[k] - cur[k]) / 2;
            any |= cur[k] < hb[k];
        }
        if (!any) break;
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = cur[k] < hb[k] ? ts[mid[k]] : T(0);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            if (cur[k] < hb[k]) {
                if (v[k] <= x) cur[k] = mid[k] + 1;
                else hb[k] = mid[k];
            }
        }
    }
}

// Segment p of candidate lane s, given tau (the last true completion before
// B_p): returns the segment's true completions and moves tau to the last
// true completion up to the segment's end.  f holds the lane's machine (LDS).
template <typename T, int N>
__device__ int64_t rerun_segment(const CountArgs<T> &a, LaneFsm<T, N> &f, const int32_t (&lo_)[N],
                                 const int32_t (&hi_)[N], T H, int p, int64_t s, T &tau) {
    constexpr T kMin = TsLimits<T>::lo();
    constexpr T kEnd = TsLimits<T>::hi();
    const int64_t b0 = (int64_t)p * a.S;
    const int64_t b1 = b0 + a.S < a.B ? b0 + a.S : a.B;
    const T Bp = p == 0 ? kMin : a.tile_t0[b0];
    const T Ep = p == a.P - 1 ? kEnd : a.tile_t0[b1];
    const int32_t c = a.rec_cnt[(int64_t)p * a.G + s];
    const T last = a.rec_last[(int64_t)p * a.G + s];
    if (p == 0 || tau < (T)(Bp - H)) {
        if (c > 0) tau = last;
        return c;
    }
    // re-run from the state right after the completion at tau
    f.e = tau;
    f.clear_all();
    // first event after tau of every node
    int32_t cur[N];
    first_after<T, N>(a.ts_by_type, lo_, hi_, tau, cur);
    T head[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const T v = cur[k] < hi_[k] ? a.ts_by_type[cur[k]] : kEnd;
        head[k] = v < Ep ? v : kEnd;
    }
    const int nspec = c < kRecFirst ? c : kRecFirst;
    // From B_p + H on, every partial occurrence either machine holds
    // started after B_p, hence after both machines' last completion
    // (tau < B_p; the speculative one's, if any, is before B_p as long as
    // it has none in the segment yet): until one of them completes, both
    // hold the same state, and from then on they agree.
    const T sync_t = (T)(Bp + H);
    const T first0 = c > 0 ? a.rec_first[((int64_t)p * kRecFirst) * a.G + s] : kEnd;
    int qi = 0;
    int32_t fcount = 0;
    T flast = tau;
    while (true) {
        T t = head[0];
        int j = 0;
#pragma unroll
        for (int k = 1; k < N; ++k) {
            if (head[k] < t) {
                t = head[k];
                j = k;
            }
        }
        if (t == kEnd) break;
        if (fcount == 0 && t >= sync_t && first0 >= t) {
            if (c > 0) tau = last;
            return c;
        }
        if (f.step(j, t, a.flags)) {
            ++fcount;
            flast = t;
            while (qi < nspec && a.rec_first[((int64_t)p * kRecFirst + qi) * a.G + s] < t) ++qi;
            if (qi < nspec && a.rec_first[((int64_t)p * kRecFirst + qi) * a.G + s] == t) {
                tau = last;
                return fcount + (c - qi - 1);
            }
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            if (k == j) {
                ++cur[k];
                const T v = cur[k] < hi_[k] ? a.ts_by_type[cur[k]] : kEnd;
                head[k] = v < Ep ? v : kEnd;
            }
        }
    }
    tau = flast;
    return fcount;
}

// The lane's machine in LDS and its candidate's per-node index ranges.
template <typename T, int N>
__device__ __forceinline__ T reconcile_lane(const CountArgs<T> &a, unsigned char *smem, int W, int lane, int64_t slot,
                                            LaneFsm<T, N> &f, int32_t (&lo_)[N], int32_t (&hi_)[N]) {
    f.lohi = reinterpret_cast<Pair<T> *>(smem);
    f.qse = reinterpret_cast<Pair<T> *>(smem + a.off_qse);
    f.qh = reinterpret_cast<uint32_t *>(smem + a.off_qh);
    f.W = W;
    f.lane = lane;
    f.Q = a.Q;
    f.gen = 0;
    constexpr int L = N > 1 ? N - 1 : 1;
    int32_t ty[N];
    T lo[L], hi[L];
    const T H = load_candidate<T, N>(a, f, slot, ty, lo, hi);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        lo_[k] = a.type_off[ty[k]];
        hi_[k] = a.type_off[ty[k] + 1];
    }
    return H;
}

// Pre-pass: lane (s, p = blockIdx.y + 1) re-runs segment p from the last
// completion the records of segments 0..p-1 give.
template <typename T, int N>
__global__ __launch_bounds__(64) void k_reconcile_pre(CountArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int W = blockDim.x, lane = threadIdx.x;
    const int64_t s = (int64_t)blockIdx.x * W + lane;
    if (s >= a.G) return;  // no barriers below
    const int p = (int)blockIdx.y + 1;
    const int64_t slot = a.perm ? (int64_t)a.perm[a.begin + s] : a.begin + s;
    LaneFsm<T, N> f;
    int32_t lo_[N], hi_[N];
    const T H = reconcile_lane<T, N>(a, smem, W, lane, slot, f, lo_, hi_);
    T tau = TsLimits<T>::lo();
    for (int q = p - 1; q >= 0; --q) {
        if (a.rec_cnt[(int64_t)q * a.G + s] > 0) {
            tau = a.rec_last[(int64_t)q * a.G + s];
            break;
        }
    }
    const int64_t o = (int64_t)p * a.G + s;
    a.pre_tau[o] = tau;
    a.pre_cnt[o] = (int32_t)rerun_segment<T, N>(a, f, lo_, hi_, H, p, s, tau);
    a.pre_last[o] = tau;
}

template <typename T, int N>
__global__ __launch_bounds__(256) void k_reconcile(CountArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int W = blockDim.x, lane = threadIdx.x;
    const int64_t s = (int64_t)blockIdx.x * W + lane;
    if (s >= a.G) return;  // no barriers below
    const int64_t slot = a.perm ? (int64_t)a.perm[a.begin + s] : a.begin + s;
    LaneFsm<T, N> f;
    int32_t lo_[N], hi_[N];
    const T H = reconcile_lane<T, N>(a, smem, W, lane, slot, f, lo_, hi_);
    T tau = TsLimits<T>::lo();
    int64_t total = 0;
    for (int p = 0; p < a.P; ++p) {
        const int64_t o = (int64_t)p * a.G + s;
        if (p > 0 && a.pre_cnt && a.pre_tau[o] == tau) {
            total += a.pre_cnt[o];
            tau = a.pre_last[o];
        } else {
            total += rerun_segment<T, N>(a, f, lo_, hi_, H, p, s, tau);
        }
    }
    const int64_t o = a.orig ? a.orig[slot] : slot;
    a.counts[o] = (int32_t)total;
    if (a.tau) a.tau[o] = tau;
}

// Appended events (streaming).  A set counted up to the stream's first n0
// events holds, per candidate, its count and last completion tau.  After an
// append (first new time B) the machine resumes from the state right after
// max(tau, B - H - 1): every occurrence ending at or after B starts at or
// after B - H, so the earlier partial occurrences cannot complete any more
// when tau < B - H, and none completes in [B - H, B) (tau is the last
// completion before B); when tau >= B - H, the machine re-runs from tau over
// the events after it, which reproduces its true state.  Either way every
// completion it finds is at or after B and is added to the count.
template <typename T, int N>
__global__ __launch_bounds__(64) void k_count_append(CountArgs<T> a, T B) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr T kEnd = TsLimits<T>::hi();
    const int W = blockDim.x, lane = threadIdx.x;
    const int64_t s = (int64_t)blockIdx.x * W + lane;
    if (s >= a.G) return;  // no barriers below
    const int64_t slot = a.begin + s;
    LaneFsm<T, N> f;
    int32_t lo_[N], hi_[N];
    const T H = reconcile_lane<T, N>(a, smem, W, lane, slot, f, lo_, hi_);
    const int64_t o = a.orig ? a.orig[slot] : slot;
    const T tau = a.tau[o];
    const T from = tau > (T)(B - H - 1) ? tau : (T)(B - H - 1);
    f.e = from;
    f.clear_all();
    int32_t cur[N];
    first_after<T, N>(a.ts_by_type, lo_, hi_, from, cur);
    T head[N];
#pragma unroll
    for (int k = 0; k < N; ++k) head[k] = cur[k] < hi_[k] ? a.ts_by_type[cur[k]] : kEnd;
    int32_t add = 0;
    T last = tau;
    while (true) {
        T t = head[0];
        int j = 0;
#pragma unroll
        for (int k = 1; k < N; ++k) {
            if (head[k] < t) {
                t = head[k];
                j = k;
            }
        }
        if (t == kEnd) break;
        if (f.step(j, t, a.flags)) {
            ++add;
            last = t;
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            if (k == j) {
                ++cur[k];
                head[k] = cur[k] < hi_[k] ? a.ts_by_type[cur[k]] : kEnd;
            }
        }
    }
    a.counts[o] += add;
    a.tau[o] = last;
}

template <typename T>
using KFn = void (*)(CountArgs<T>);

template <typename T>
using AFn = void (*)(CountArgs<T>, T);

template <typename T>
AFn<T> pick_append(int N) {
    switch (N) {
        case 1: return k_count_append<T, 1>;
        case 2: return k_count_append<T, 2>;
        case 3: return k_count_append<T, 3>;
        case 4: return k_count_append<T, 4>;
        case 5: return k_count_append<T, 5>;
        case 6: return k_count_append<T, 6>;
        case 7: return k_count_append<T, 7>;
        case 8: return k_count_append<T, 8>;
        default: return nullptr;
    }
}

template <typename T, bool F, bool REL>
KFn<T> pick_count_f(int N) {
    switch (N) {
        case 1: return k_count_tiled<T, 1, F, REL>;
        case 2: return k_count_tiled<T, 2, F, REL>;
        case 3: return k_count_tiled<T, 3, F, REL>;
        case 4: return k_count_tiled<T, 4, F, REL>;
        case 5: return k_count_tiled<T, 5, F, REL>;
        case 6: return k_count_tiled<T, 6, F, REL>;
        case 7: return k_count_tiled<T, 7, F, REL>;
        case 8: return k_count_tiled<T, 8, F, REL>;
        default: return nullptr;
    }
}

// REL: the int32 relative-time machines (int64 streams only).
template <typename T>
KFn<T> pick_count(int N, bool filtered, bool rel) {
    if constexpr (sizeof(T) == 8) {
        if (rel) return filtered ? pick_count_f<T, true, true>(N) : pick_count_f<T, false, true>(N);
    }
    return filtered ? pick_count_f<T, true, false>(N) : pick_count_f<T, false, false>(N);
}

template <typename T>
KFn<T> pick_reconcile(int N) {
    switch (N) {
        case 1: return k_reconcile<T, 1>;
        case 2: return k_reconcile<T, 2>;
        case 3: return k_reconcile<T, 3>;
        case 4: return k_reconcile<T, 4>;
        case 5: return k_reconcile<T, 5>;
        case 6: return k_reconcile<T, 6>;
        case 7: return k_reconcile<T, 7>;
        case 8: return k_reconcile<T, 8>;
        default: return nullptr;
    }
}

template <typename T>
KFn<T> pick_reconcile_pre(int N) {
    switch (N) {
        case 1: return k_reconcile_pre<T, 1>;
        case 2: return k_reconcile_pre<T, 2>;
        case 3: return k_reconcile_pre<T, 3>;
        case 4: return k_reconcile_pre<T, 4>;
        case 5: return k_reconcile_pre<T, 5>;
        case 6: return k_reconcile_pre<T, 6>;
        case 7: return k_reconcile_pre<T, 7>;
        case 8: return k_reconcile_pre<T, 8>;
        default: return nullptr;
    }
}

inline uint32_t al16(size_t x) { return (uint32_t)((x + 15) & ~size_t(15)); }


template <typename T>
struct Layout {
    uint32_t off_qse, off_tbuf, off_qh, off_obuf, off_misc, total;
};

// rel: the machines and the staged tile hold int32 relative times; tile:
// events per tile of the stream(s).
template <typename T>
Layout<T> layout(int N, int Q, int W, int K, bool tiles, bool rel, int tile) {
    Layout<T> L;
    const size_t lv = N > 1 ? N - 1 : 0;
    const size_t ts = rel ? sizeof(int32_t) : sizeof(T);  // machine time
    size_t o = al16(lv * W * 2 * ts);
    L.off_qse = (uint32_t)o;
    o += al16(lv * Q * W * 2 * ts);
    L.off_tbuf = (uint32_t)o;
    o += tiles ? al16((size_t)tile * ts) : 0;
    L.off_qh = (uint32_t)o;
    o += al16(lv * W * sizeof(uint32_t));
    L.off_obuf = (uint32_t)o;
    o += tiles ? al16((K + 1) * sizeof(uint16_t)) : 0;
    L.off_misc = (uint32_t)o;
    o += 16 * sizeof(T);
    L.total = (uint32_t)o;
    return L;
}

// Whether the int32 relative-time machines can count a group of the stream:
// an int64 stream whose longest tile plus twice the group's longest episode
// span stays below 2^31 - 64.  Relative times lie in [-2, tile span], and the
// machine only forms a time plus one interval bound (record, rejection test)
// or minus a tile span (rebase), so every value then fits int32.
template <typename T>
bool rel_ok(const Stream &s, int64_t hspan) {
    return sizeof(T) == 8 && s.max_tile_span >= 0 && hspan >= 0 && hspan < (int64_t(1) << 29) &&
           s.max_tile_span < (int64_t(1) << 31) && s.max_tile_span + 2 * hspan < (int64_t(1) << 31) - 64;
}

constexpr uint32_t kLdsSoft = 64 * 1024;
constexpr uint32_t kLdsHard = 160 * 1024;

// Widest workgroup (at most max_lanes) whose LDS fits comfortably; else the
// widest that fits at all.
template <typename T>
int pick_lanes(int N, int Q, int K, int max_lanes, bool rel, int tile) {
    int fit = 64;
    bool any = false;
    for (int W : {256, 128, 64}) {
        if (max_lanes > 0 && W > max_lanes) continue;
        const Layout<T> L = layout<T>(N, Q, W, K, true, rel, tile);
        if (L.total <= kLdsSoft) return W;
        if (!any && L.total <= kLdsHard) {
            fit = W;
            any = true;
        }
    }
    return fit;
}

// Lane width of a launch of kernel fn: the one (of 256, 128, 64, at most
// max_lanes) whose workgroups keep the most waves resident on a CU, as the
// runtime counts them (LDS and registers); ties go to the wider one, whose
// waves share one staged tile.  Falls back to pick_lanes.
template <typename T>
int pick_lanes_fn(const void *fn, int N, int Q, int K, int max_lanes, bool rel, int tile) {
    int best = 0, bestW = 0;
    for (int W : {256, 128, 64}) {
        if (max_lanes > 0 && W > max_lanes) continue;
        const Layout<T> L = layout<T>(N, Q, W, K, true, rel, tile);
        if (L.total > kLdsHard) continue;
        if (L.total > kLdsSoft &&
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total) != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        int per = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, W, L.total) != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        const int waves = per * (W / 64);
        if (waves > best) {
            best = waves;
            bestW = W;
        }
    }
    return best > 0 ? bestW : pick_lanes<T>(N, Q, K, max_lanes, rel, tile);
}

template <typename T>
hipError_t ensure_lds_attr(KFn<T> fn, uint32_t bytes) {
    if (bytes <= kLdsSoft) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

constexpr int kRecLanes = 64;  // lanes per reconciliation workgroup

// Bytes of the segment records of a unit of G lanes and P segments: per
// (segment, lane) the speculative last and first completions and count, and
// the pre-pass's assumed tau, last completion and count.
template <typename T>
size_t record_bytes(int64_t P, int64_t G) {
    return (size_t)P * (size_t)G * (sizeof(T) * (3 + kRecFirst) + 2 * sizeof(int32_t));
}

template <typename T>
void set_records(CountArgs<T> &a, unsigned char *base, int64_t P, int64_t G) {
    const size_t PG = (size_t)P * (size_t)G;
    a.rec_last = reinterpret_cast<T *>(base);
    a.rec_first = a.rec_last + PG;
    a.pre_last = a.rec_first + PG * kRecFirst;
    a.pre_tau = a.pre_last + PG;
    a.rec_cnt = reinterpret_cast<int32_t *>(a.pre_tau + PG);
    a.pre_cnt = a.rec_cnt + PG;
}

// Reconciliation of a unit's segments: the pre-pass over every (lane,
// segment > 0) in parallel, then the walk over the segments.
template <typename T>
hipError_t launch_reconcile(const CountArgs<T> &a, int N, const Layout<T> &RL, hipStream_t st) {
    if (a.P < 2 || a.P > 65536 || !a.pre_cnt) return hipErrorInvalidValue;
    CountArgs<T> r = a;
    r.off_qse = RL.off_qse;
    r.off_qh = RL.off_qh;
    r.off_tbuf = RL.off_tbuf;
    r.off_obuf = RL.off_obuf;
    r.off_misc = RL.off_misc;
    KFn<T> pf = pick_reconcile_pre<T>(N), rf = pick_reconcile<T>(N);
    if (!pf || !rf) return hipErrorInvalidValue;
    hipError_t e;
    if ((e = ensure_lds_attr<T>(pf, RL.total)) != hipSuccess) return e;
    if ((e = ensure_lds_attr<T>(rf, RL.total)) != hipSuccess) return e;
    const unsigned gx = (unsigned)((r.G + kRecLanes - 1) / kRecLanes);
    pf<<<dim3(gx, (unsigned)(r.P - 1)), kRecLanes, RL.total, st>>>(r);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    rf<<<gx, kRecLanes, RL.total, st>>>(r);
    return hipGetLastError();
}

// Lane width of a launch of the lane-machine kernel fn with ring entries C:
// the one (of 256, 128, 64, at most max_lanes) whose workgroups keep the most
// waves resident on a CU; ties go to the wider one.
int lane_pick_width(const void *fn, int C, int K, int tile, int max_lanes) {
    int best = 0, bestW = 64;
    for (int W : {256, 128, 64}) {
        if (max_lanes > 0 && W > max_lanes) continue;
        const LaneLayout L = lane_layout(C, W, K, tile);
        if (L.total > kLdsHard) continue;
        if (L.total > kLdsSoft &&
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total) != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        int per = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, W, L.total) != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        const int waves = per * (W / 64);
        if (waves > best) {
            best = waves;
            bestW = W;
        }
    }
    return bestW;
}

hipError_t lane_lds_attr(const void *fn, uint32_t bytes) {
    if (bytes <= kLdsSoft) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Whether the register-indexed lane machines count group g of stream s.
template <typename T>
bool lane_group_ok(const Stream &s, const CandSet &c, const Group &g, const CountOptions &opt) {
    const bool filtered = c.compact && c.pred_bits && c.succ_bits;
    return opt.lane_engine && !filtered && (g.N == 1 || (g.C > 0 && g.C <= cap_class_value(kCapClasses - 1))) &&
           lane_rel_ok(s.max_tile_span, g.hspan);
}

template <typename T>
hipError_t count_t(const Stream &s, CandSet &c, const CountOptions &opt, int32_t *d_flags, hipStream_t st,
                   unsigned char *ext_scratch, size_t ext_bytes) {
    hipError_t e;
    for (const Group &g : c.groups) {
        const int64_t G = g.end - g.begin;
        if (G <= 0) continue;
        if (s.n == 0) {  // no events: every count is zero
            k_zero_counts<T><<<(unsigned)((G + 255) / 256), 256, 0, st>>>(
                c.compact ? nullptr : c.orig.as<int32_t>() + g.begin, G, c.counts.as<int32_t>() + (c.compact ? g.begin : 0),
                !c.compact && c.tau.p ? c.tau.as<T>() : nullptr);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            continue;
        }
        const bool lane = lane_group_ok<T>(s, c, g, opt);
        const bool pk = lane && lane_pk_ok(s.max_tile_span);
        const bool rel = !lane && rel_ok<T>(s, g.hspan);
        const bool filtered = c.compact && c.pred_bits && c.succ_bits;
        KFn<T> fn = lane ? nullptr : pick_count<T>(g.N, filtered, rel);
        const bool wl = opt.worklog && c.work.p;  // (a.work below)
        const void *lfn = lane ? lane_tiled_fn<T>(g.N, pk, wl) : nullptr;
        if (!fn && !lfn) return hipErrorInvalidValue;
        const int C = std::max(1, g.C);
        const int W = lane ? lane_pick_width(lfn, C, s.K, s.T, opt.lanes)
                           : pick_lanes_fn<T>(reinterpret_cast<const void *>(fn), g.N, g.Q, s.K, opt.lanes, rel, s.T);
        const Layout<T> L = layout<T>(g.N, g.Q, W, s.K, true, rel, s.T);
        const LaneLayout LL = lane_layout(C, W, s.K, s.T);
        const uint32_t lds = lane ? LL.total : L.total;
        if (lds > kLdsHard) return hipErrorInvalidConfiguration;
        int64_t S = 1;
        int64_t P = plain_segments(s, G, opt, &S);

        CountArgs<T> a{};
        a.tiled = s.tiled_ts.as<T>();
        a.loff = s.tile_loff.as<uint16_t>();
        a.tile_t0 = s.tile_t0.as<T>();
        a.ts_by_type = s.ts_by_type.as<T>();
        a.type_off = s.type_off.as<int32_t>();
        a.B = s.B;
        a.K = s.K;
        a.ctypes = c.types.as<int32_t>();
        a.clo = c.lo.as<T>();
        a.chi = c.hi.as<T>();
        a.t16 = c.compact ? c.t16.as<uint16_t>() : nullptr;
        a.iv = c.compact ? c.iv.as<uint8_t>() : nullptr;
        a.menu = c.compact ? c.menu.as<T>() : nullptr;
        a.m = c.m;
        a.begin = g.begin;
        a.G = G;
        a.Q = g.Q;
        a.C = C;
        a.P = (int32_t)P;
        a.S = S;
        a.orig = c.compact ? nullptr : c.orig.as<int32_t>();
        a.counts = c.counts.as<int32_t>();
        a.tau = !c.compact && c.tau.p ? c.tau.as<T>() : nullptr;
        a.flags = d_flags;
        a.perm = nullptr;
        a.work = wl ? c.work.as<int32_t>() : nullptr;
        a.cycles = nullptr;
        if (lane) {
            a.off_qse = LL.off_ring;
            a.off_tbuf = LL.off_tbuf;
            a.off_qh = 0;
            a.off_obuf = LL.off_obuf;
            a.off_misc = LL.off_misc;
        } else {
            a.off_qse = L.off_qse;
            a.off_tbuf = L.off_tbuf;
            a.off_qh = L.off_qh;
            a.off_obuf = L.off_obuf;
            a.off_misc = L.off_misc;
        }
        if (P > 1) {
            const size_t need = record_bytes<T>(P, G);
            if (ext_scratch) {
                // the caller's scratch (no allocation); groups run one after
                // another on st, so each reuses it from the start
                if (need > ext_bytes) return hipErrorOutOfMemory;
                set_records<T>(a, ext_scratch, P, G);
            } else {
                if (c.scratch.bytes < need) {
                    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
                    if ((e = c.scratch.alloc(need)) != hipSuccess) return e;
                }
                set_records<T>(a, c.scratch.as<unsigned char>(), P, G);
            }
        }
        a.pbits = filtered ? c.pred_bits : nullptr;
        a.sbits = filtered ? c.succ_bits : nullptr;
        a.rwords = s.B * (s.T / 64);
        a.tile = s.T;
        const dim3 grid((unsigned)((G + W - 1) / W), (unsigned)P);
        if (lane) {
            if ((e = lane_lds_attr(lfn, lds)) != hipSuccess) return e;
            if ((e = lane_launch_tiled<T>(a, g.N, pk, grid, W, lds, st)) != hipSuccess) return e;
        } else {
            if ((e = ensure_lds_attr<T>(fn, lds)) != hipSuccess) return e;
            fn<<<grid, W, lds, st>>>(a);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        if (P > 1 && (e = launch_reconcile<T>(a, g.N, layout<T>(g.N, g.Q, kRecLanes, s.K, false, false, 0), st)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// The events of the stream appended since set c was counted (B: the first
// appended time): one lane per candidate resumes its machine (k_count_append).
template <typename T>
hipError_t count_append_t(const Stream &s, CandSet &c, int64_t B, int32_t *d_flags, hipStream_t st) {
    hipError_t e;
    if (c.compact || !c.tau.p) return hipErrorInvalidValue;
    for (const Group &g : c.groups) {
        const int64_t G = g.end - g.begin;
        if (G <= 0) continue;
        AFn<T> fn = pick_append<T>(g.N);
        if (!fn) return hipErrorInvalidValue;
        const Layout<T> L = layout<T>(g.N, g.Q, kRecLanes, s.K, false, false, 0);
        CountArgs<T> a{};
        a.ts_by_type = s.ts_by_type.as<T>();
        a.type_off = s.type_off.as<int32_t>();
        a.K = s.K;
        a.ctypes = c.types.as<int32_t>();
        a.clo = c.lo.as<T>();
        a.chi = c.hi.as<T>();
        a.m = c.m;
        a.begin = g.begin;
        a.G = G;
        a.Q = g.Q;
        a.P = 1;
        a.orig = c.orig.as<int32_t>();
        a.counts = c.counts.as<int32_t>();
        a.tau = c.tau.as<T>();
        a.flags = d_flags;
        a.off_qse = L.off_qse;
        a.off_qh = L.off_qh;
        a.off_tbuf = L.off_tbuf;
        a.off_obuf = L.off_obuf;
        a.off_misc = L.off_misc;
        if ((e = ensure_lds_attr<T>(reinterpret_cast<KFn<T>>(fn), L.total)) != hipSuccess) return e;
        fn<<<(unsigned)((G + kRecLanes - 1) / kRecLanes), kRecLanes, L.total, st>>>(a, (T)B);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_count_append(const Stream &s, CandSet &c, int64_t B, int32_t *d_flags, hipStream_t st) {
    if (s.ts_kind == EPI_TS_I64) return count_append_t<int64_t>(s, c, B, d_flags, st);
    return count_append_t<int32_t>(s, c, B, d_flags, st);
}

hipError_t launch_count(const Stream &s, CandSet &c, const CountOptions &opt, int32_t *d_flags, hipStream_t st,
                        unsigned char *ext_scratch, size_t ext_bytes) {
    if (s.ts_kind == EPI_TS_I64) return count_t<int64_t>(s, c, opt, d_flags, st, ext_scratch, ext_bytes);
    return count_t<int32_t>(s, c, opt, d_flags, st, ext_scratch, ext_bytes);
}

int64_t plain_segments(const Stream &s, int64_t G, const CountOptions &opt, int64_t *S_out) {
    int64_t P = 1;
    if (opt.segments > 0) {
        P = opt.segments;
    } else if (opt.segments == 0) {
        const int64_t target = opt.target_lanes;
        P = G >= target ? 1 : (target + G - 1) / G;
    }
    // at most one segment per 4 tiles (the look-back before each segment
    // start is re-read), and within the grid's y limit
    const int64_t pmax = std::max<int64_t>(1, std::min<int64_t>(s.B / 4, 65535));
    if (opt.segments == 0 && P > pmax) P = pmax;
    if (P > s.B) P = s.B;
    if (P > 65535) P = 65535;
    if (P < 1) P = 1;
    const int64_t S = (std::max<int64_t>(s.B, 1) + P - 1) / P;
    P = (s.B + S - 1) / S;
    if (P < 1) P = 1;
    if (S_out) *S_out = S;
    return P;
}

size_t plain_record_bytes(const Stream &s, int64_t P, int64_t G) {
    return P > 1 ? (s.ts_kind == EPI_TS_I64 ? record_bytes<int64_t>(P, G) : record_bytes<int32_t>(P, G)) : 0;
}

}  // namespace epi

// ---------------------------------------------------------------------------
// Batched mode and its scheduler.
// ---------------------------------------------------------------------------
namespace epi {

namespace {

template <typename T>
using PFn = void (*)(const CountArgs<T> *, const WorkItem *, int64_t, int64_t, unsigned long long *);

template <typename T, bool F, bool REL>
PFn<T> pick_persistent_rf(int N) {
    switch (N) {
        case 1: return k_count_persistent<T, 1, F, REL>;
        case 2: return k_count_persistent<T, 2, F, REL>;
        case 3: return k_count_persistent<T, 3, F, REL>;
        case 4: return k_count_persistent<T, 4, F, REL>;
        case 5: return k_count_persistent<T, 5, F, REL>;
        case 6: return k_count_persistent<T, 6, F, REL>;
        case 7: return k_count_persistent<T, 7, F, REL>;
        case 8: return k_count_persistent<T, 8, F, REL>;
        default: return nullptr;
    }
}

template <typename T, bool F>
PFn<T> pick_persistent_f(int N, bool rel) {
    if constexpr (sizeof(T) == 8) {
        if (rel) return pick_persistent_rf<T, F, true>(N);
    }
    return pick_persistent_rf<T, F, false>(N);
}

// Identity of a batched plan: everything its graph bakes in (buffers, sizes,
// launch groups, options, schedule and, for the learned schedule, the model's
// buffers and output scaling).
std::vector<int64_t> plan_key(const std::vector<BatchRef> &sets, const std::vector<int32_t> &ids, int sched,
                              const CountOptions &opt, const Mlp &mlp, const int32_t *d_flags) {
    std::vector<int64_t> k;
    auto P = [&](const void *p) { k.push_back((int64_t)(intptr_t)p); };
    k.push_back(sched);
    k.push_back(opt.segments);
    k.push_back(opt.lanes);
    k.push_back(opt.target_lanes);
    k.push_back(opt.worklog);
    k.push_back(opt.lane_engine);
    k.push_back(opt.ring_classes);
    P(d_flags);
    if (sched == EPI_SCHED_LEARNED) {
        k.push_back(mlp.ready() ? mlp.F : -1);
        P(mlp.p.p);
        P(mlp.norm.p);
        uint32_t a, b;
        std::memcpy(&a, &mlp.y_mu, 4);
        std::memcpy(&b, &mlp.y_sd, 4);
        k.push_back(((int64_t)a << 32) | b);
    }
    for (size_t i = 0; i < sets.size(); ++i) {
        const Stream &s = *sets[i].s;
        const CandSet &c = *sets[i].c;
        k.push_back(ids[i]);
        P(&s);
        k.push_back(s.n);
        k.push_back(s.K);
        k.push_back(s.B);
        k.push_back(s.T);
        k.push_back(s.max_tile_span);
        P(s.tiled_ts.p);
        P(s.tile_loff.p);
        P(s.tile_t0.p);
        P(s.type_off.p);
        P(s.ts_by_type.p);
        P(&c);
        k.push_back(c.m);
        k.push_back(c.compact);
        P(c.types.p);
        P(c.lo.p);
        P(c.hi.p);
        P(c.orig.p);
        P(c.counts.p);
        P(c.tau.p);
        P(c.work.p);
        P(c.dmeasured.p);
        P(c.t16.p);
        P(c.iv.p);
        P(c.menu.p);
        P(c.pred_bits);
        P(c.succ_bits);
        k.push_back((int64_t)c.groups.size());
        for (const Group &g : c.groups) {
            k.push_back(g.N);
            k.push_back(g.Q);
            k.push_back(g.C);
            k.push_back(g.begin);
            k.push_back(g.end);
            k.push_back(g.hspan);
        }
    }
    return k;
}

// Plan a batched count: launch units (set, episode size group) with their
// segment counts, launch classes with their lane widths and LDS layouts, the
// work-item template (class-major), the device tables of the scheduler, and
// one captured graph: [costs -> candidate sort -> item keys -> item sort ->
// item gather] (costed schedules only), clear of the queue counters,
// persistent launches (parallel branches), reconciliation.
template <typename T>
hipError_t plan_t(std::vector<BatchRef> &sets, int sched, const CountOptions &opt, Mlp &mlp, int32_t *d_flags,
                  BatchCache &cache, BatchPlan &plan, hipStream_t st) {
    hipError_t e;
    int dev = 0, ncu = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = cache.branches()) != hipSuccess) return e;

    // the schedule: round robin without costs, for compact (level-wise) sets
    // and for the learned schedule without a model
    bool costed = sched != EPI_SCHED_RR;
    if (sched == EPI_SCHED_LEARNED && !(mlp.ready() && mlp.F == kFeatures)) costed = false;
    for (auto &r : sets)
        if (r.c->compact) costed = false;
    if (sched == EPI_SCHED_MEASURED)
        for (auto &r : sets)
            if (!r.c->has_measured) costed = false;

    // launch groups: the submission groups (episode size x ring entries
    // class), adjacent ones of one size merged per EPI_OPT_RING_CLASSES
    // (fewer, larger groups: the cost order spans more episodes, so each
    // wave's lanes are closer in work; the rings take the group's largest)
    std::vector<std::vector<Group>> mg(sets.size());
    for (size_t si = 0; si < sets.size(); ++si) {
        auto bucket = [&](const Group &g) {
            const int L = std::max(1, g.N - 1);
            if (opt.ring_classes == 1) return 0;
            if (opt.ring_classes == 2) return g.C <= 2 * L ? 0 : (g.C <= 3 * L ? 1 : 2);
            return cap_class_index(std::max(1, g.C));
        };
        for (const Group &g : sets[si].c->groups) {
            if (g.end <= g.begin) continue;
            if (!mg[si].empty()) {
                Group &b = mg[si].back();
                if (b.N == g.N && b.end == g.begin && bucket(b) == bucket(g) && opt.ring_classes != 0) {
                    b.end = g.end;
                    b.Q = std::max(b.Q, g.Q);
                    b.C = std::max(b.C, g.C);
                    b.hspan = std::max(b.hspan, g.hspan);
                    continue;
                }
            }
            mg[si].push_back(g);
        }
    }

    // global slot order: the sets back to back; launch groups numbered in
    // that order (each set's deep tail, counted elsewhere, is a group too)
    std::vector<int64_t> soff(sets.size() + 1, 0);
    for (size_t si = 0; si < sets.size(); ++si) soff[si + 1] = soff[si] + sets[si].c->m;
    const int64_t M = soff.back();
    std::vector<SchedGroup> sgroups;
    std::vector<int32_t> gid(costed ? M : 0);
    std::vector<SchedSet> ssets(sets.size());
    for (size_t si = 0; si < sets.size(); ++si) {
        const Stream &s = *sets[si].s;
        const CandSet &c = *sets[si].c;
        ssets[si] = SchedSet{s.type_off.as<int32_t>(), c.types.as<int32_t>(), c.lo.p, c.hi.p,
                             c.has_measured ? c.dmeasured.as<float>() : nullptr, c.m, soff[si]};
        if (!costed) continue;
        int64_t end = 0;
        for (const Group &g : mg[si]) {
            for (int64_t i = g.begin; i < g.end; ++i) gid[soff[si] + i] = (int32_t)sgroups.size();
            sgroups.push_back(SchedGroup{(int32_t)si, g.N});
            end = std::max(end, g.end);
        }
        if (end < c.m) {
            for (int64_t i = end; i < c.m; ++i) gid[soff[si] + i] = (int32_t)sgroups.size();
            sgroups.push_back(SchedGroup{(int32_t)si, 1});
        }
    }

    // 1. launch units: one per (set, group), segments as in plain mode
    struct UnitH {
        int set, N, Q, W;
        int64_t begin, G, P, S;
        bool filt, rel, lane, pk;
        int C;
    };
    std::vector<UnitH> units;
    std::vector<std::pair<size_t, Group>> empty_groups;  // groups of sets on streams without events
    for (size_t si = 0; si < sets.size(); ++si) {
        const Stream &s = *sets[si].s;
        CandSet &c = *sets[si].c;
        for (const Group &g : mg[si]) {
            const int64_t G = g.end - g.begin;
            if (G <= 0) continue;
            if (s.n == 0) {
                empty_groups.emplace_back(si, g);
                continue;
            }
            UnitH u{};
            u.set = (int)si;
            u.N = g.N;
            u.Q = g.Q;
            u.begin = g.begin;
            u.G = G;
            u.filt = c.compact && c.pred_bits && c.succ_bits;
            u.lane = lane_group_ok<T>(s, c, g, opt);
            u.pk = u.lane && lane_pk_ok(s.max_tile_span);
            u.rel = !u.lane && rel_ok<T>(s, g.hspan);
            u.C = std::max(1, g.C);
            const int64_t pmax = std::max<int64_t>(1, std::min<int64_t>(s.B / 4, 65535));
            int64_t P = G >= opt.target_lanes ? 1 : (opt.target_lanes + G - 1) / G;
            if (opt.segments > 0) P = opt.segments;
            P = std::max<int64_t>(1, std::min<int64_t>(P, opt.segments > 0 ? s.B : pmax));
            P = std::min<int64_t>(P, 65535);
            u.S = (s.B + P - 1) / P;
            u.P = (s.B + u.S - 1) / u.S;
            units.push_back(u);
        }
    }
    // 2. launch classes: the LDS-ring machines by (episode size, queue class,
    // time type); the lane machines by (episode size, ring-entries class,
    // key form); each with one lane width and LDS layout for its units
    constexpr int kQClasses = 8;  // Q = 1, 2, 3, 4, 6, 8, 12, 16
    constexpr int kRingClasses = (kMaxN + 1) * kQClasses * 2;
    constexpr int kClasses = kRingClasses + (kMaxN + 1) * kCapClasses * 2;
    auto cls_of = [](const UnitH &u) {
        if (u.lane) return kRingClasses + (u.N * kCapClasses + cap_class_index(u.C)) * 2 + (u.pk ? 1 : 0);
        static constexpr int kQ[kQClasses] = {1, 2, 3, 4, 6, 8, 12, 16};
        int q = 0;
        while (q + 1 < kQClasses && kQ[q] < u.Q) ++q;
        return (u.N * kQClasses + q) * 2 + (u.rel ? 1 : 0);
    };
    std::vector<int> clsN(kClasses, 0), clsQ(kClasses, 1), clsC(kClasses, 1), maxK(kClasses, 1), maxT(kClasses, 64),
        Wn(kClasses, 256);
    std::vector<bool> filtN(kClasses, false), relN(kClasses, false), laneN(kClasses, false), pkN(kClasses, false);
    for (const UnitH &u : units) {
        const Stream &s = *sets[u.set].s;
        const int cl = cls_of(u);
        clsN[cl] = u.N;
        relN[cl] = u.rel;
        laneN[cl] = u.lane;
        pkN[cl] = u.pk;
        clsQ[cl] = std::max(clsQ[cl], u.Q);
        clsC[cl] = std::max(clsC[cl], u.C);
        maxK[cl] = std::max(maxK[cl], (int)s.K);
        maxT[cl] = std::max(maxT[cl], s.T);
        filtN[cl] = filtN[cl] || u.filt;
    }
    std::vector<int> crank(kClasses, -1), corder;
    for (int cl = 0; cl < kClasses; ++cl) {
        if (clsN[cl] <= 0) continue;
        crank[cl] = (int)corder.size();
        corder.push_back(cl);
        if (laneN[cl]) {
            Wn[cl] = lane_pick_width(lane_persistent_fn<T>(clsN[cl], pkN[cl], opt.worklog), clsC[cl], maxK[cl], maxT[cl],
                                     opt.lanes);
            continue;
        }
        const PFn<T> pfn = filtN[cl] ? pick_persistent_f<T, true>(clsN[cl], relN[cl])
                                     : pick_persistent_f<T, false>(clsN[cl], relN[cl]);
        if (!pfn) return hipErrorInvalidValue;
        Wn[cl] = pick_lanes_fn<T>(reinterpret_cast<const void *>(pfn), clsN[cl], clsQ[cl], maxK[cl], opt.lanes,
                                  relN[cl], maxT[cl]);
    }

    // 3. the candidate sort's passes (decided now: the permutation's buffer
    // is the one the last pass writes)
    int gpass = 1;
    while (gpass < 4 && ((int64_t)sgroups.size() >> (8 * gpass)) > 0) ++gpass;
    std::vector<int> cshift = {0, 8, 16, 24};
    for (int i = 0; i < gpass; ++i) cshift.push_back(32 + 8 * i);
    int ipass = 1;
    while (ipass < 4 && ((int64_t)corder.size() >> (8 * ipass)) > 0) ++ipass;
    std::vector<int> ishift = {0, 8, 16, 24};
    for (int i = 0; i < ipass; ++i) ishift.push_back(32 + 8 * i);
    if (costed && M > 0) {
        if ((e = plan.k0.alloc(sizeof(uint64_t) * M)) != hipSuccess) return e;
        if ((e = plan.k1.alloc(sizeof(uint64_t) * M)) != hipSuccess) return e;
        if ((e = plan.v0.alloc(sizeof(int32_t) * M)) != hipSuccess) return e;
        if ((e = plan.v1.alloc(sizeof(int32_t) * M)) != hipSuccess) return e;
        if ((e = plan.y.alloc(sizeof(float) * M)) != hipSuccess) return e;
        if (sched == EPI_SCHED_LEARNED && (e = plan.X.alloc(sizeof(float) * M * kFeatures)) != hipSuccess) return e;
    }
    const bool perm_second = (cshift.size() % 2) == 1;
    const int32_t *perm_base = !(costed && M > 0) ? nullptr : (perm_second ? plan.v1.as<int32_t>() : plan.v0.as<int32_t>());
    const uint64_t *skey_base =
        !(costed && M > 0) ? nullptr : (perm_second ? plan.k1.as<uint64_t>() : plan.k0.as<uint64_t>());

    // 4. per-unit arguments, records and the work-item template (class-major)
    size_t rec_bytes = 0;
    for (const UnitH &u : units)
        if (u.P > 1) rec_bytes += record_bytes<T>(u.P, u.G) + 64;
    if ((e = plan.rec.alloc(rec_bytes)) != hipSuccess) return e;
    std::vector<CountArgs<T>> ua(units.size());
    std::vector<SchedUnit> su(units.size());
    size_t ro = 0;
    for (size_t ui = 0; ui < units.size(); ++ui) {
        const UnitH &u = units[ui];
        const Stream &s = *sets[u.set].s;
        CandSet &c = *sets[u.set].c;
        const int cl = cls_of(u);
        CountArgs<T> a{};
        a.tiled = s.tiled_ts.as<T>();
        a.loff = s.tile_loff.as<uint16_t>();
        a.tile_t0 = s.tile_t0.as<T>();
        a.ts_by_type = s.ts_by_type.as<T>();
        a.type_off = s.type_off.as<int32_t>();
        a.B = s.B;
        a.K = s.K;
        a.ctypes = c.types.as<int32_t>();
        a.clo = c.lo.as<T>();
        a.chi = c.hi.as<T>();
        a.t16 = c.compact ? c.t16.as<uint16_t>() : nullptr;
        a.iv = c.compact ? c.iv.as<uint8_t>() : nullptr;
        a.menu = c.compact ? c.menu.as<T>() : nullptr;
        a.pbits = u.filt ? c.pred_bits : nullptr;
        a.sbits = u.filt ? c.succ_bits : nullptr;
        a.rwords = s.B * (s.T / 64);
        a.tile = s.T;
        a.m = c.m;
        a.begin = u.begin;
        a.G = u.G;
        a.Q = clsQ[cl];
        a.C = clsC[cl];
        a.P = (int32_t)u.P;
        a.S = u.S;
        a.orig = c.compact ? nullptr : c.orig.as<int32_t>();
        a.counts = c.counts.as<int32_t>();
        a.tau = !c.compact && c.tau.p ? c.tau.template as<T>() : nullptr;
        a.flags = d_flags;
        a.perm = perm_base ? perm_base + soff[u.set] : nullptr;
        a.work = opt.worklog ? c.work.as<int32_t>() : nullptr;
        if (u.P > 1) {
            set_records<T>(a, plan.rec.as<unsigned char>() + ro, u.P, u.G);
            ro += (record_bytes<T>(u.P, u.G) + 64) & ~size_t(15);
        }
        if (laneN[cl]) {
            const LaneLayout L = lane_layout(clsC[cl], Wn[cl], maxK[cl], maxT[cl]);
            a.off_qse = L.off_ring;
            a.off_tbuf = L.off_tbuf;
            a.off_qh = 0;
            a.off_obuf = L.off_obuf;
            a.off_misc = L.off_misc;
        } else {
            const Layout<T> L = layout<T>(clsN[cl], clsQ[cl], Wn[cl], maxK[cl], true, relN[cl], maxT[cl]);
            a.off_qse = L.off_qse;
            a.off_tbuf = L.off_tbuf;
            a.off_qh = L.off_qh;
            a.off_obuf = L.off_obuf;
            a.off_misc = L.off_misc;
        }
        ua[ui] = a;
        su[ui] = SchedUnit{soff[u.set] + u.begin, u.G, Wn[cl], (int32_t)u.P, crank[cl], 0};
    }
    std::vector<WorkItem> tmpl;
    std::vector<int64_t> ioff(kClasses + 1, 0);
    // the branch balance: each class's work as the summed event counts of
    // its episodes' types (the events its lanes visit), from host copies
    std::vector<double> ccost(kClasses, 0.0);
    for (size_t ui = 0; ui < units.size(); ++ui) {
        const UnitH &u = units[ui];
        const Stream &s = *sets[u.set].s;
        const CandSet &c = *sets[u.set].c;
        double w = 0;
        if (!c.compact && (int64_t)c.h_N.size() == c.m && (int64_t)s.h_off.size() == (int64_t)s.K + 1) {
            // slots -> submission indices are the set's grouping order; the
            // unit's slots hold the candidates of one launch group, whose
            // work the host knows per candidate
            for (int64_t i = 0; i < u.G; ++i) {
                const int64_t o = c.h_order.empty() ? u.begin + i : c.h_order[u.begin + i];
                const int32_t *ty = c.h_types.data() + o * kMaxN;
                for (int j = 0; j < c.h_N[o]; ++j) w += (double)(s.h_off[ty[j] + 1] - s.h_off[ty[j]]);
            }
        } else {
            w = (double)u.G * (double)u.N * (double)s.n / std::max(1.0, (double)s.K);
        }
        ccost[cls_of(u)] += w;
    }
    for (int cl = 0; cl < kClasses; ++cl) {
        ioff[cl] = (int64_t)tmpl.size();
        for (size_t ui = 0; ui < units.size(); ++ui) {
            const UnitH &u = units[ui];
            if (cls_of(u) != cl) continue;
            const int64_t nb = (u.G + Wn[cl] - 1) / Wn[cl];
            for (int64_t b = 0; b < nb; ++b)
                for (int64_t p = 0; p < u.P; ++p) tmpl.push_back(WorkItem{(int32_t)ui, (int32_t)p, b});
        }
    }
    ioff[kClasses] = (int64_t)tmpl.size();
    const int64_t n_items = (int64_t)tmpl.size();
    plan.n_items = n_items;
    plan.soff = soff;
    plan.perm = perm_base;
    for (const UnitH &u : units) plan.uview.push_back(BatchPlan::UnitView{u.set, u.begin, u.G, Wn[cls_of(u)]});
    if (opt.worklog) {
        if ((e = plan.cycles.alloc(sizeof(int64_t) * 2 * std::max<int64_t>(1, n_items))) != hipSuccess) return e;
        for (auto &a : ua) a.cycles = plan.cycles.as<int64_t>();
    }
    // device tables
    auto up = [&](DevBuf &d, const void *h, size_t bytes) -> hipError_t {
        hipError_t x = d.alloc(std::max<size_t>(bytes, 16));
        if (x != hipSuccess || bytes == 0) return x;
        return hipMemcpy(d.p, h, bytes, hipMemcpyHostToDevice);
    };
    if ((e = up(plan.units, ua.data(), sizeof(CountArgs<T>) * ua.size())) != hipSuccess) return e;
    if ((e = up(plan.tmpl, tmpl.data(), sizeof(WorkItem) * tmpl.size())) != hipSuccess) return e;
    if ((e = plan.items.alloc(sizeof(WorkItem) * std::max<int64_t>(1, n_items))) != hipSuccess) return e;
    if ((e = plan.queue.alloc(sizeof(unsigned long long) * kClasses)) != hipSuccess) return e;
    if (!costed && n_items > 0 &&
        (e = hipMemcpy(plan.items.p, tmpl.data(), sizeof(WorkItem) * n_items, hipMemcpyHostToDevice)) != hipSuccess)
        return e;
    if (costed) {
        if ((e = up(plan.ssets, ssets.data(), sizeof(SchedSet) * ssets.size())) != hipSuccess) return e;
        if ((e = up(plan.sgroups, sgroups.data(), sizeof(SchedGroup) * sgroups.size())) != hipSuccess) return e;
        if ((e = up(plan.gid, gid.data(), sizeof(int32_t) * gid.size())) != hipSuccess) return e;
        if ((e = up(plan.sunits, su.data(), sizeof(SchedUnit) * su.size())) != hipSuccess) return e;
        if ((e = plan.ik0.alloc(sizeof(uint64_t) * std::max<int64_t>(1, n_items))) != hipSuccess) return e;
        if ((e = plan.ik1.alloc(sizeof(uint64_t) * std::max<int64_t>(1, n_items))) != hipSuccess) return e;
        if ((e = plan.iv0.alloc(sizeof(int32_t) * std::max<int64_t>(1, n_items))) != hipSuccess) return e;
        if ((e = plan.iv1.alloc(sizeof(int32_t) * std::max<int64_t>(1, n_items))) != hipSuccess) return e;
        if ((e = plan.hist.alloc(sizeof(uint32_t) * radix_hist_words(std::max<int64_t>(M, n_items)))) != hipSuccess)
            return e;
    }

    // 5. capture: scheduler, queue clear, persistent launches on parallel
    // branches (costliest classes first, each onto the least loaded branch),
    // join, reconciliation
    std::vector<int> border = corder;
    std::stable_sort(border.begin(), border.end(), [&](int x, int y) { return ccost[x] > ccost[y]; });
    const int nb = std::max(1, std::min<int>(BatchCache::kBranches, (int)border.size()));
    if ((e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    if (costed && M > 0) {
        bool second = false;
        e = sched_costs(sizeof(T) == 8 ? EPI_TS_I64 : EPI_TS_I32, sched, plan.ssets.as<SchedSet>(),
                        plan.sgroups.as<SchedGroup>(), plan.gid.as<int32_t>(), M, mlp, plan.X.as<float>(),
                        plan.y.as<float>(), st);
        if (e == hipSuccess)
            e = sched_keys(plan.ssets.as<SchedSet>(), plan.sgroups.as<SchedGroup>(), plan.gid.as<int32_t>(), M,
                           plan.y.as<float>(), sched == EPI_SCHED_LEARNED, plan.k0.as<uint64_t>(),
                           plan.v0.as<int32_t>(), st);
        if (e == hipSuccess)
            e = radix_sort(plan.k0.as<uint64_t>(), plan.v0.as<int32_t>(), plan.k1.as<uint64_t>(),
                           plan.v1.as<int32_t>(), M, cshift.data(), (int)cshift.size(), plan.hist.as<uint32_t>(), st,
                           &second);
        if (e == hipSuccess && second != perm_second) e = hipErrorInvalidValue;
        if (e == hipSuccess && n_items > 0) {
            bool isec = false;
            e = sched_item_keys(plan.tmpl.as<WorkItem>(), n_items, plan.sunits.as<SchedUnit>(), skey_base,
                                plan.ik0.as<uint64_t>(), plan.iv0.as<int32_t>(), st);
            if (e == hipSuccess)
                e = radix_sort(plan.ik0.as<uint64_t>(), plan.iv0.as<int32_t>(), plan.ik1.as<uint64_t>(),
                               plan.iv1.as<int32_t>(), n_items, ishift.data(), (int)ishift.size(),
                               plan.hist.as<uint32_t>(), st, &isec);
            if (e == hipSuccess)
                e = sched_gather_items(plan.tmpl.as<WorkItem>(), isec ? plan.iv1.as<int32_t>() : plan.iv0.as<int32_t>(),
                                       n_items, plan.items.as<WorkItem>(), st);
        }
    } else if (costed && M == 0) {
        // nothing to order
    }
    for (auto &eg : empty_groups) {
        if (e != hipSuccess) break;
        CandSet &c = *sets[eg.first].c;
        const Group &g = eg.second;
        const int64_t G = g.end - g.begin;
        k_zero_counts<T><<<(unsigned)((G + 255) / 256), 256, 0, st>>>(
            c.compact ? nullptr : c.orig.as<int32_t>() + g.begin, G, c.counts.as<int32_t>() + (c.compact ? g.begin : 0),
            !c.compact && c.tau.p ? c.tau.template as<T>() : nullptr);
        e = hipGetLastError();
    }
    static_assert(kClasses <= 65536, "queue counters");
    if (e == hipSuccess) {
        k_fill_u64<<<1, 256, 0, st>>>(plan.queue.as<unsigned long long>(), kClasses, 0ull);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(cache.fork, st);
    for (int i = 0; i < nb && e == hipSuccess; ++i) e = hipStreamWaitEvent(cache.br[i], cache.fork, 0);
    // the segmented units of a class are reconciled on the class's branch
    // (their records are all written by its kernel), after the branch's last
    // persistent kernel: a reconciliation queued between two classes waits
    // for CUs that the other branches' persistent kernels hold and keeps its
    // branch's next class waiting too; at the branch's end it overlaps the
    // other branches' last kernels instead
    auto reconcile_class = [&](int cl, hipStream_t bst) -> hipError_t {
        for (size_t ui = 0; ui < units.size(); ++ui) {
            if (units[ui].P <= 1 || cls_of(units[ui]) != cl) continue;
            const int N = units[ui].N;
            const hipError_t x = launch_reconcile<T>(ua[ui], N, layout<T>(N, clsQ[cl], kRecLanes, maxK[cl], false, false, 0), bst);
            if (x != hipSuccess) return x;
        }
        return hipSuccess;
    };
    std::vector<double> load(nb, 0.0);
    std::vector<std::vector<int>> brcls(nb);
    for (int cl : border) {
        if (e != hipSuccess) break;
        const int bi = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[bi] += ccost[cl];
        const int N = clsN[cl];
        const int64_t ncl = ioff[cl + 1] - ioff[cl];
        if (ncl <= 0) continue;
        int per = 0;
        if (laneN[cl]) {
            const void *lfn = lane_persistent_fn<T>(N, pkN[cl], opt.worklog);
            const LaneLayout L = lane_layout(clsC[cl], Wn[cl], maxK[cl], maxT[cl]);
            if (L.total > kLdsHard) {
                e = hipErrorInvalidConfiguration;
                break;
            }
            if ((e = lane_lds_attr(lfn, L.total)) != hipSuccess) break;
            if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, lfn, Wn[cl], L.total)) != hipSuccess) break;
            const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(ncl, (int64_t)ncu * std::max(per, 1)));
            e = lane_launch_persistent<T>(N, pkN[cl], opt.worklog, (unsigned)grid, Wn[cl], L.total, cache.br[bi],
                                          plan.units.as<CountArgs<T>>(), plan.items.as<WorkItem>() + ioff[cl], ncl,
                                          ioff[cl], plan.queue.as<unsigned long long>() + cl);
            brcls[bi].push_back(cl);
            continue;
        }
        PFn<T> fn = filtN[cl] ? pick_persistent_f<T, true>(N, relN[cl]) : pick_persistent_f<T, false>(N, relN[cl]);
        const Layout<T> L = layout<T>(N, clsQ[cl], Wn[cl], maxK[cl], true, relN[cl], maxT[cl]);
        if (L.total > kLdsHard) {
            e = hipErrorInvalidConfiguration;
            break;
        }
        if ((e = ensure_lds_attr<T>(reinterpret_cast<KFn<T>>(fn), L.total)) != hipSuccess) break;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void *>(fn), Wn[cl],
                                                              L.total)) != hipSuccess)
            break;
        const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(ncl, (int64_t)ncu * std::max(per, 1)));
        fn<<<(unsigned)grid, Wn[cl], L.total, cache.br[bi]>>>(plan.units.as<CountArgs<T>>(),
                                                             plan.items.as<WorkItem>() + ioff[cl], ncl, ioff[cl],
                                                             plan.queue.as<unsigned long long>() + cl);
        e = hipGetLastError();
        brcls[bi].push_back(cl);
    }
    for (int bi = 0; bi < nb && e == hipSuccess; ++bi)
        for (int cl : brcls[bi])
            if (e == hipSuccess) e = reconcile_class(cl, cache.br[bi]);
    // every branch joins back (also after an error, so that the capture ends
    // cleanly)
    for (int i = 0; i < nb; ++i) {
        hipError_t ej = hipEventRecord(cache.joined[i], cache.br[i]);
        if (ej == hipSuccess) ej = hipStreamWaitEvent(st, cache.joined[i], 0);
        if (e == hipSuccess) e = ej;
    }
    hipError_t ec = hipStreamEndCapture(st, &plan.graph);
    if (e == hipSuccess) e = ec;
    if (e == hipSuccess) e = hipGraphInstantiate(&plan.exec, plan.graph, nullptr, nullptr, 0);
    return e;
}

}  // namespace

hipError_t BatchCache::branches() {
    if (fork) return hipSuccess;
    hipError_t e = hipSuccess;
    for (int i = 0; i < kBranches && e == hipSuccess; ++i) {
        if (!br[i]) e = hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking);
        if (e == hipSuccess && !joined[i]) e = hipEventCreateWithFlags(&joined[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    return e;
}

BatchPlan *BatchCache::find(const std::vector<int64_t> &key) {
    for (size_t i = 0; i < plans.size(); ++i) {
        if (plans[i]->key != key) continue;
        std::unique_ptr<BatchPlan> p = std::move(plans[i]);
        plans.erase(plans.begin() + (std::ptrdiff_t)i);
        plans.push_back(std::move(p));
        return plans.back().get();
    }
    return nullptr;
}

BatchPlan *BatchCache::find_id(uint64_t id) {
    for (auto &p : plans)
        if (p->id == id) return p.get();
    return nullptr;
}

void BatchCache::evict_set(int32_t id) {
    bool any = false;
    for (auto &p : plans)
        for (int32_t x : p->set_ids) any = any || x == id;
    if (!any) return;
    (void)hipDeviceSynchronize();
    std::vector<std::unique_ptr<BatchPlan>> keep;
    for (auto &p : plans) {
        bool hit = false;
        for (int32_t x : p->set_ids) hit = hit || x == id;
        if (!hit) keep.push_back(std::move(p));
    }
    plans = std::move(keep);
}

void BatchCache::evict_all() {
    if (plans.empty()) return;
    (void)hipDeviceSynchronize();
    plans.clear();
}

void BatchCache::clear() {
    evict_all();
    for (int i = 0; i < kBranches; ++i) {
        if (joined[i]) (void)hipEventDestroy(joined[i]);
        if (br[i]) (void)hipStreamDestroy(br[i]);
        joined[i] = nullptr;
        br[i] = nullptr;
    }
    if (fork) (void)hipEventDestroy(fork);
    fork = nullptr;
}

hipError_t launch_count_batched(std::vector<BatchRef> &sets, const std::vector<int32_t> &ids, int sched,
                                const CountOptions &opt, Mlp &mlp, BatchCache &cache, int32_t *d_flags,
                                hipStream_t st) {
    if (sets.empty()) return hipSuccess;
    const int kind = sets[0].s->ts_kind;
    for (auto &r : sets)
        if (r.s->ts_kind != kind) return hipErrorInvalidValue;
    const std::vector<int64_t> key = plan_key(sets, ids, sched, opt, mlp, d_flags);
    BatchPlan *p = cache.find(key);
    if (p) {
        ++cache.replays;
    } else {
        if (cache.plans.size() >= BatchCache::kMaxPlans) {
            (void)hipDeviceSynchronize();
            cache.plans.erase(cache.plans.begin());
        }
        auto np = std::make_unique<BatchPlan>();
        np->key = key;
        np->set_ids = ids;
        np->id = cache.next_id++;
        hipError_t e = kind == EPI_TS_I64 ? plan_t<int64_t>(sets, sched, opt, mlp, d_flags, cache, *np, st)
                                          : plan_t<int32_t>(sets, sched, opt, mlp, d_flags, cache, *np, st);
        if (e != hipSuccess) {
            (void)hipDeviceSynchronize();  // the plan's uploads end before its buffers are freed
            return e;
        }
        ++cache.built;
        cache.plans.push_back(std::move(np));
        p = cache.plans.back().get();
    }
    hipError_t e = hipGraphLaunch(p->exec, st);
    if (e != hipSuccess) return e;
    ++p->launches;
    for (auto &r : sets) {
        r.c->n_items = p->n_items;
        r.c->cycles_plan = 0;
        r.c->last_plan = p->id;
    }
    sets[0].c->cycles_plan = opt.worklog ? p->id : 0;
    return hipSuccess;
}

}  // namespace epi
