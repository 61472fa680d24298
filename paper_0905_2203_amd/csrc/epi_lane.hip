// Register-indexed lane machines: the state-machine count of a workgroup of W
// candidate episodes (one lane each) over a range of stream tiles, with the
// machine's bookkeeping in registers and only the interval rings in LDS.
//
// The machine is the one of epi_fsm.h (Sec. III-A with starts admitted only
// strictly after the last completion, so that its completions are the greedy
// choices of Alg. 1), with the same merged acceptance intervals: a record at
// node j at time t' matters only through (t' + lo_j, t' + hi_j], node j keeps
// the union of those intervals as a ring of disjoint intervals in time order,
// and at most q_j = 1 + floor(hi_j / (hi_j - lo_j + 1)) of them are live (end
// at or after the latest event) at once.  What differs is where the state
// lives and what the step costs:
//
//   * each node has its own ring of exactly q_j entries (not the episode's
//     deepest), laid out back to back per lane in LDS (lane-interleaved, so a
//     wave-wide access to one entry index touches consecutive words); the
//     ring's head and fill (4 bits each), capacity (4 bits) and base entry
//     (8 bits) are bit fields of a few registers, selected by the node index
//     with one shift;
//   * dead intervals (end before the current time) are dropped lazily: a
//     query skips them from the head; a record drops the head only when the
//     ring is full, and then the head is dead (at most q_j - 1 intervals other
//     than the new one can be live);
//   * a completion empties every ring by clearing the fill fields (two
//     register writes);
//   * the lane's next event is the minimum over its N per-node heads; when
//     relative times fit 28 bits, a head is the 31-bit key time * 8 + node and
//     the minimum is N - 1 integer minimum instructions (PK).
//
// Times are int32 offsets from the first time of the tile being walked
// (tiles are short enough: lane_rel_ok); at every tile the live intervals and
// the last completion move by the previous tile's span, with interval starts
// before the new origin kept at -1 and ends at -2, which every later query or
// record (at a time >= 0) compares exactly as the true values.
//
// Segments (P > 1) and their records are those of epi_tiled.hip: segment p
// owns times [B_p, B_{p+1}); its run starts at the last tile starting before
// B_p - H (H: the workgroup's longest episode span) as if the last completion
// were B_p - H - 1 and records the completions in its own segment.
#include <type_traits>

#include "epi_count.h"

namespace epi {

namespace {

// 8-bit field k (k < 8) of the register pair (r0: fields 0-3, r1: 4-7).
template <int NS>
__device__ __forceinline__ uint32_t f8(uint32_t r0, uint32_t r1, int k) {
    const uint32_t sh = (uint32_t)(k & 3) << 3;
    if constexpr (NS <= 4) return (r0 >> sh) & 0xffu;
    return ((k < 4 ? r0 : r1) >> sh) & 0xffu;
}

template <int NS>
__device__ __forceinline__ void set8(uint32_t &r0, uint32_t &r1, int k, uint32_t v) {
    const uint32_t sh = (uint32_t)(k & 3) << 3, m = 0xffu << sh;
    if constexpr (NS <= 4) {
        r0 = (r0 & ~m) | (v << sh);
    } else {
        if (k < 4) r0 = (r0 & ~m) | (v << sh);
        else r1 = (r1 & ~m) | (v << sh);
    }
}

template <typename T, int N, bool PK>
__device__ __forceinline__ void lane_item(const CountArgs<T> &a, int64_t blk, int p, int64_t item,
                                          unsigned char *smem) {
    using R = int32_t;
    constexpr T kMin = TsLimits<T>::lo();
    constexpr T kEnd = TsLimits<T>::hi();
    constexpr R rEnd = INT32_MAX;
    constexpr int L = N > 1 ? N - 1 : 1;  // interval slots (array size)
    constexpr int NS = N > 1 ? N - 1 : 1;
    const int W = blockDim.x, lane = threadIdx.x;
    const int64_t s = blk * W + lane;
    const bool active = s < a.G;
    const int64_t lslot = a.begin + (active ? s : 0);
    const int64_t slot = a.perm ? (int64_t)a.perm[lslot] : lslot;
    if (a.cycles && lane == 0) a.cycles[2 * item] = (int64_t)wall_clock64();
    R *tbuf = reinterpret_cast<R *>(smem + a.off_tbuf);
    uint16_t *obuf = reinterpret_cast<uint16_t *>(smem + a.off_obuf);
    T *misc = reinterpret_cast<T *>(smem + a.off_misc);
    // this lane's ring entry i: rl[i << wsh] (W is a power of two)
    int2 *rl = reinterpret_cast<int2 *>(smem + a.off_qse) + lane;
    const int wsh = 31 - __clz(W);

    // the episode: types, interval bounds, ring capacities and bases
    int32_t ty[N];
    R loR[L], hiR[L];
    T H = 0;
    uint32_t qpk = 0, bp0 = 0, bp1 = 0;
    {
        uint32_t base = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) ty[k] = a.t16 ? (int32_t)a.t16[(int64_t)k * a.m + slot] : a.ctypes[(int64_t)k * a.m + slot];
#pragma unroll
        for (int k = 0; k + 1 < N; ++k) {
            T lo, hi;
            if (a.t16) {
                const int id = a.iv[(int64_t)k * a.m + slot];
                lo = a.menu[2 * id];
                hi = a.menu[2 * id + 1];
            } else {
                lo = a.clo[(int64_t)k * a.m + slot];
                hi = a.chi[(int64_t)k * a.m + slot];
            }
            H += hi;
            loR[k] = (R)lo;
            hiR[k] = (R)hi;
            uint32_t q = (uint32_t)(1 + (int64_t)hi / ((int64_t)hi - (int64_t)lo + 1));
            if (q > (uint32_t)kLaneMaxQ) {  // never: the host keeps deeper episodes away
                atomicAdd(&a.flags[kFlagQueueOverflow], 1);
                q = kLaneMaxQ;
            }
            qpk |= q << (4 * k);
            set8<NS>(bp0, bp1, k, base);
            base += q;
        }
    }
    uint32_t hn0 = 0, hn1 = 0;  // per ring: head | fill << 4

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

    // origin of the relative times: the first time of the tile walked
    T t0b = a.tile_t0[bs];
    R e;  // last completion, relative
    {
        const bool before = e0 < t0b && (uint64_t)t0b - (uint64_t)e0 > 2u;
        e = before ? R(-2) : (R)(int64_t)((uint64_t)e0 - (uint64_t)t0b);
    }
    int32_t cnt = 0;
    T last = kMin;
    uint32_t w_visits = 0, w_records = 0, w_queries = 0, w_done = 0, w_maxq = 0;
    for (int64_t b = bs; b < b1; ++b) {
        __syncthreads();
        const T nb = a.tile_t0[b];
        const R d = (R)(nb - t0b);  // the previous tile's span (0 for the first)
        if (d != 0 && active) {
#pragma unroll
            for (int k = 0; k + 1 < N; ++k) {
                const uint32_t hn = f8<NS>(hn0, hn1, k), Q = (qpk >> (4 * k)) & 15u, base = f8<NS>(bp0, bp1, k);
                uint32_t hd = hn & 15u;
                for (uint32_t i = 0; i < (hn >> 4); ++i) {
                    int2 &v = rl[(int)(base + hd) << wsh];
                    const R vs = v.x - d, ve = v.y - d;
                    v.x = vs < R(-1) ? R(-1) : vs;
                    v.y = ve < R(-2) ? R(-2) : ve;
                    hd = hd + 1 == Q ? 0u : hd + 1;
                }
            }
            e = e - d < R(-2) ? R(-2) : (R)(e - d);
        }
        t0b = nb;
        {
            const T *src = a.tiled + b * a.tile;
            // (the last tile's padding is never read; wrapping keeps it defined)
            for (int i = lane; i < a.tile; i += W) {
                const int64_t v = (int64_t)((uint64_t)src[i] - (uint64_t)t0b);
                tbuf[i] = v > (int64_t)INT32_MAX ? INT32_MAX : (v < -1 ? R(-1) : (R)v);
            }
        }
        const R BpR = Bp <= t0b ? R(-1) : (Bp - t0b >= (T)INT32_MAX ? rEnd : (R)(Bp - t0b));
        const R EpR = (Ep == kEnd || Ep - t0b >= (T)INT32_MAX) ? rEnd : (R)(Ep - t0b);
        for (int i = lane; i <= a.K; i += W) obuf[i] = a.loff[b * (a.K + 1) + i];
        __syncthreads();
        if (!active) continue;
        int cur[N], stp[N];
        R head[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            cur[k] = obuf[ty[k]];
            stp[k] = obuf[ty[k] + 1];
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            R v = cur[k] < stp[k] ? tbuf[cur[k]] : rEnd;
            v = v < EpR ? v : rEnd;
            head[k] = PK ? (v == rEnd ? rEnd : (R)((v << 3) | k)) : v;
        }
        while (true) {
            // next event of the lane's types (lowest node first among equal times)
            R t;
            int j;
            if constexpr (PK) {
                R key = head[0];
#pragma unroll
                for (int k = 1; k < N; ++k) key = head[k] < key ? head[k] : key;
                if (key == rEnd) break;
                j = key & 7;
                t = key >> 3;
            } else {
                t = head[0];
                j = 0;
#pragma unroll
                for (int k = 1; k < N; ++k) {
                    if (head[k] < t) {
                        t = head[k];
                        j = k;
                    }
                }
                if (t == rEnd) break;
            }
            ++w_visits;
            bool done = false;
            if constexpr (N == 1) {
                if (t > e) {
                    e = t;
                    done = true;
                }
            } else {
                bool ok;
                if (j == 0) {
                    ok = t > e;
                } else {
                    // query the ring of node j - 1: drop dead intervals from the head,
                    // then t is covered iff the first live one starts before it
                    ++w_queries;
                    const int q = j - 1;
                    const uint32_t hn = f8<NS>(hn0, hn1, q), Q = (qpk >> (4 * q)) & 15u, base = f8<NS>(bp0, bp1, q);
                    uint32_t hd = hn & 15u, n = hn >> 4;
                    int2 f = make_int2(0, 0);
                    while (n > 0) {
                        f = rl[(int)(base + hd) << wsh];
                        if (f.y >= t) break;
                        hd = hd + 1 == Q ? 0u : hd + 1;
                        --n;
                    }
                    ok = n > 0 && f.x < t;
                    const uint32_t nh = hd | (n << 4);
                    if (nh != hn) set8<NS>(hn0, hn1, q, nh);
                }
                if (ok) {
                    if (j == N - 1) {
                        e = t;
                        done = true;
                        hn0 = 0;
                        hn1 = 0;
                    } else {
                        // record at node j: merge into the newest interval when they
                        // touch, else append (dropping the head, dead, when full)
                        ++w_records;
                        R lj = loR[0], hj = hiR[0];
#pragma unroll
                        for (int k = 1; k + 1 < N; ++k) {
                            if (k == j) {
                                lj = loR[k];
                                hj = hiR[k];
                            }
                        }
                        const R ns = t + lj, ne = t + hj;
                        const uint32_t hn = f8<NS>(hn0, hn1, j), Q = (qpk >> (4 * j)) & 15u,
                                       base = f8<NS>(bp0, bp1, j);
                        uint32_t hd = hn & 15u, n = hn >> 4;
                        bool merged = Q == 0;  // (no ring: never, j < N - 1)
                        if (n > 0 && !merged) {
                            uint32_t bk = hd + n - 1;
                            if (bk >= Q) bk -= Q;
                            int2 &be = rl[(int)(base + bk) << wsh];
                            if (ns <= be.y) {
                                be.y = ne;
                                merged = true;
                            }
                        }
                        if (!merged) {
                            if (n == Q) {
                                hd = hd + 1 == Q ? 0u : hd + 1;
                                --n;
                            }
                            uint32_t tl = hd + n;
                            if (tl >= Q) tl -= Q;
                            rl[(int)(base + tl) << wsh] = make_int2(ns, ne);
                            ++n;
                            w_maxq = n > w_maxq ? n : w_maxq;
                            set8<NS>(hn0, hn1, j, hd | (n << 4));
                        }
                    }
                }
            }
            if (done) {
                ++w_done;
                if (t >= BpR) {
                    const T ta = (T)t + t0b;  // absolute
                    if (a.P > 1 && cnt < kRecFirst) a.rec_first[((int64_t)p * kRecFirst + cnt) * a.G + s] = ta;
                    ++cnt;
                    last = ta;
                }
            }
            // advance node j
            int c = cur[0], st = stp[0];
#pragma unroll
            for (int k = 1; k < N; ++k) {
                if (k == j) {
                    c = cur[k];
                    st = stp[k];
                }
            }
            ++c;
            R v = c < st ? tbuf[c] : rEnd;
            v = v < EpR ? v : rEnd;
            const R nk = PK ? (v == rEnd ? rEnd : (R)((v << 3) | j)) : v;
#pragma unroll
            for (int k = 0; k < N; ++k) {
                if (k == j) {
                    cur[k] = c;
                    head[k] = nk;
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
        atomicMax(w + 4, (int32_t)w_maxq);
    }
    if (a.P == 1) {
        a.counts[o] = cnt;
        if (a.tau) a.tau[o] = last;
    } else {
        a.rec_cnt[(int64_t)p * a.G + s] = cnt;
        a.rec_last[(int64_t)p * a.G + s] = last;
    }
}

template <typename T, int N, bool PK>
__global__ __launch_bounds__(256) void k_lane_tiled(CountArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    lane_item<T, N, PK>(a, blockIdx.x, blockIdx.y, (int64_t)blockIdx.y * gridDim.x + blockIdx.x, smem);
}

// Persistent form: every workgroup takes work items (unit, lane block,
// segment) from a device queue until it is empty.
template <typename T, int N, bool PK>
__global__ __launch_bounds__(256) void k_lane_persistent(const CountArgs<T> *__restrict__ units,
                                                         const WorkItem *__restrict__ items, int64_t n_items,
                                                         int64_t item_base, unsigned long long *__restrict__ queue) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int64_t next;
    while (true) {
        if (threadIdx.x == 0) next = (int64_t)atomicAdd(queue, 1ull);
        __syncthreads();
        const int64_t it = next;
        __syncthreads();
        // uniform: every wave of the group exits (unsigned: any counter value
        // beyond the items ends the loop)
        if ((uint64_t)it >= (uint64_t)n_items) break;
        const WorkItem w = items[it];
        const CountArgs<T> a = units[w.unit];
        lane_item<T, N, PK>(a, w.blk, w.p, item_base + it, smem);
    }
}

template <typename T, bool PK>
const void *tiled_sym(int N) {
    switch (N) {
        case 1: return reinterpret_cast<const void *>(k_lane_tiled<T, 1, PK>);
        case 2: return reinterpret_cast<const void *>(k_lane_tiled<T, 2, PK>);
        case 3: return reinterpret_cast<const void *>(k_lane_tiled<T, 3, PK>);
        case 4: return reinterpret_cast<const void *>(k_lane_tiled<T, 4, PK>);
        case 5: return reinterpret_cast<const void *>(k_lane_tiled<T, 5, PK>);
        case 6: return reinterpret_cast<const void *>(k_lane_tiled<T, 6, PK>);
        case 7: return reinterpret_cast<const void *>(k_lane_tiled<T, 7, PK>);
        case 8: return reinterpret_cast<const void *>(k_lane_tiled<T, 8, PK>);
        default: return nullptr;
    }
}

template <typename T, bool PK>
const void *persistent_sym(int N) {
    switch (N) {
        case 1: return reinterpret_cast<const void *>(k_lane_persistent<T, 1, PK>);
        case 2: return reinterpret_cast<const void *>(k_lane_persistent<T, 2, PK>);
        case 3: return reinterpret_cast<const void *>(k_lane_persistent<T, 3, PK>);
        case 4: return reinterpret_cast<const void *>(k_lane_persistent<T, 4, PK>);
        case 5: return reinterpret_cast<const void *>(k_lane_persistent<T, 5, PK>);
        case 6: return reinterpret_cast<const void *>(k_lane_persistent<T, 6, PK>);
        case 7: return reinterpret_cast<const void *>(k_lane_persistent<T, 7, PK>);
        case 8: return reinterpret_cast<const void *>(k_lane_persistent<T, 8, PK>);
        default: return nullptr;
    }
}

inline uint32_t al16(size_t x) { return (uint32_t)((x + 15) & ~size_t(15)); }

}  // namespace

LaneLayout lane_layout(int C, int W, int K, int tile) {
    LaneLayout L;
    size_t o = 0;
    L.off_ring = (uint32_t)o;
    o += al16((size_t)(C > 0 ? C : 1) * W * sizeof(int2));
    L.off_tbuf = (uint32_t)o;
    o += al16((size_t)tile * sizeof(int32_t));
    L.off_obuf = (uint32_t)o;
    o += al16((size_t)(K + 1) * sizeof(uint16_t));
    L.off_misc = (uint32_t)o;
    o += 16 * sizeof(int64_t);
    L.total = (uint32_t)o;
    return L;
}

template <typename T>
const void *lane_tiled_fn(int N, bool pk) {
    return pk ? tiled_sym<T, true>(N) : tiled_sym<T, false>(N);
}

template <typename T>
const void *lane_persistent_fn(int N, bool pk) {
    return pk ? persistent_sym<T, true>(N) : persistent_sym<T, false>(N);
}

template <typename T>
hipError_t lane_launch_tiled(const CountArgs<T> &a, int N, bool pk, dim3 grid, int W, uint32_t lds, hipStream_t st) {
    const void *fn = lane_tiled_fn<T>(N, pk);
    if (!fn) return hipErrorInvalidValue;
    CountArgs<T> arg = a;
    void *args[] = {&arg};
    return hipLaunchKernel(fn, grid, dim3((unsigned)W), args, lds, st);
}

template <typename T>
hipError_t lane_launch_persistent(int N, bool pk, unsigned grid, int W, uint32_t lds, hipStream_t st,
                                  const CountArgs<T> *units, const WorkItem *items, int64_t n_items, int64_t item_base,
                                  unsigned long long *queue) {
    const void *fn = lane_persistent_fn<T>(N, pk);
    if (!fn) return hipErrorInvalidValue;
    void *args[] = {&units, &items, &n_items, &item_base, &queue};
    return hipLaunchKernel(fn, dim3(grid), dim3((unsigned)W), args, lds, st);
}

template const void *lane_tiled_fn<int32_t>(int, bool);
template const void *lane_tiled_fn<int64_t>(int, bool);
template const void *lane_persistent_fn<int32_t>(int, bool);
template const void *lane_persistent_fn<int64_t>(int, bool);
template hipError_t lane_launch_tiled<int32_t>(const CountArgs<int32_t> &, int, bool, dim3, int, uint32_t, hipStream_t);
template hipError_t lane_launch_tiled<int64_t>(const CountArgs<int64_t> &, int, bool, dim3, int, uint32_t, hipStream_t);
template hipError_t lane_launch_persistent<int32_t>(int, bool, unsigned, int, uint32_t, hipStream_t,
                                                    const CountArgs<int32_t> *, const WorkItem *, int64_t, int64_t,
                                                    unsigned long long *);
template hipError_t lane_launch_persistent<int64_t>(int, bool, unsigned, int, uint32_t, hipStream_t,
                                                    const CountArgs<int64_t> *, const WorkItem *, int64_t, int64_t,
                                                    unsigned long long *);

}  // namespace epi
