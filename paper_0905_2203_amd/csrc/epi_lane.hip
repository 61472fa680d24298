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
//   * node 0's admission test (a start only strictly after the last
//     completion e) is a ring too: ring 0 holds the one interval (e, +inf],
//     ring r >= 1 holds node r-1's records, i.e. node r's acceptance
//     intervals; so every event, whatever its node j, queries ring j and, if
//     covered, records into ring j+1 (or completes, at j = N-1): one path for
//     every node, and a completion rewrites ring 0 and empties the others;
//   * ring r >= 1 has exactly q_{r-1} entries (not the episode's deepest),
//     the rings of a lane back to back and lane-interleaved in LDS (a
//     wave-wide access to one entry index touches consecutive words); each
//     ring's head and fill (4 bits each) are a byte of one 64-bit register,
//     its capacity (4 bits) and base entry (8 bits) fields of two more,
//     selected by the ring index with one shift;
//   * dead intervals (end before the current time) are dropped lazily: a
//     query skips them from the head; a record drops the head only when the
//     ring is full, and then the head is dead (at most q - 1 intervals other
//     than the new one can be live);
//   * each node's tile cursor and end are one packed register, its head the
//     next event; the lane's next event is the minimum over the N heads; when
//     relative times stay below 2^29 - 1, a head is the 32-bit unsigned key
//     time * 8 + node and the minimum is N - 1 integer minimum instructions
//     (PK).
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

// WL: the work log is kept (its counters cost nothing in the visit loop
// without it).
template <typename T, int N, bool PK, bool WL>
__device__ __forceinline__ void lane_item(const CountArgs<T> &a, int64_t blk, int p, int64_t item,
                                          unsigned char *smem) {
    using R = int32_t;
    // heads: PK, the unsigned key time * 8 + node (times below 2^29 - 1),
    // all ones when the node has no event left; else the relative time
    using HK = std::conditional_t<PK, uint32_t, int32_t>;
    constexpr HK kNoHead = PK ? HK(0xffffffffu) : HK(INT32_MAX);
    constexpr T kMin = TsLimits<T>::lo();
    constexpr T kEnd = TsLimits<T>::hi();
    constexpr R rEnd = INT32_MAX;
    constexpr int L = N > 1 ? N - 1 : 1;  // interval slots (array size)
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

    // the episode: types, interval bounds, ring capacities and bases.  Ring 0
    // is node 0's: the one interval (e, +inf] of the starts the machine admits
    // (e: the last completion); ring r >= 1 holds node r-1's records, i.e. the
    // acceptance intervals of node r.  A query at node j reads ring j, a record
    // at node j < N-1 writes ring j+1: one path for every node.
    int32_t ty[N];
    R loR[L], hiR[L];
    T H = 0;
    uint32_t capk = 1;   // 4 bits per ring: capacity
    uint64_t basek = 0;  // 8 bits per ring: first entry
    {
        uint32_t base = 1;
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
            capk |= q << (4 * (k + 1));
            basek |= (uint64_t)base << (8 * (k + 1));
            base += q;
        }
    }
    // per ring: head (4 bits) | fill << 4, 8 bits each
    uint64_t hf = uint64_t(1) << 4;  // ring 0 holds its interval

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
    {
        // ring 0's interval (e, +inf]; any e before the origin reads as -1
        const bool before = e0 < t0b && (uint64_t)t0b - (uint64_t)e0 > 1u;
        const R e = before ? R(-1) : (R)(int64_t)((uint64_t)e0 - (uint64_t)t0b);
        if (active) rl[0] = make_int2(e, rEnd);
    }
    int32_t cnt = 0;
    T last = kMin;
    uint32_t w_visits = 0, w_records = 0, w_queries = 0, w_done = 0, w_maxq = 0;
    for (int64_t b = bs; b < b1; ++b) {
        __syncthreads();
        const T nb = a.tile_t0[b];
        const R d = (R)(nb - t0b);  // the previous tile's span (0 for the first)
        if (d != 0 && active) {
            // move every live interval by the span: starts before the new
            // origin read as -1, ends as -2 (ring 0's +inf end stays)
#pragma unroll
            for (int r = 0; r < N; ++r) {
                const uint32_t m = (uint32_t)(hf >> (8 * r)) & 0xffu;
                const uint32_t Q = (capk >> (4 * r)) & 15u, base = (uint32_t)(basek >> (8 * r)) & 0xffu;
                uint32_t hd = m & 15u;
                for (uint32_t i = 0; i < (m >> 4); ++i) {
                    int2 &v = rl[(int)(base + hd) << wsh];
                    const R vs = v.x - d, ve = v.y - d;
                    v.x = vs < R(-1) ? R(-1) : vs;
                    v.y = v.y == rEnd ? rEnd : (ve < R(-2) ? R(-2) : ve);
                    hd = hd + 1 == Q ? 0u : hd + 1;
                }
            }
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
        // per node: tile cursor | end << 16, and the head (next event)
        uint32_t cs[N];
        HK head[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const uint32_t c = obuf[ty[k]], st = obuf[ty[k] + 1];
            cs[k] = c | st << 16;
            R v = c < st ? tbuf[c] : rEnd;
            v = v < EpR ? v : rEnd;
            head[k] = PK ? (v == rEnd ? kNoHead : (HK)(((uint32_t)v << 3) | (uint32_t)k)) : (HK)v;
        }
        while (true) {
            // next event of the lane's types (lowest node first among equal times)
            // A lane whose events are all visited stays in the loop until
            // the wave leaves together: it visits nothing (live = false: its
            // query fails and its cursor stays), so no value of it is
            // carried round the loop.
            R t;
            int j;
            bool live;
            if constexpr (PK) {
                HK key = head[0];
#pragma unroll
                for (int k = 1; k < N; ++k) key = head[k] < key ? head[k] : key;
                live = key != kNoHead;
                j = live ? (int)(key & 7u) : 0;
                t = (R)(key >> 3);
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
                live = t != rEnd;
            }
            if (__ballot(live) == 0) break;  // uniform
            // node j's cursor (selected here, where the node tests dominate the
            // record's interval select, which then reuses them)
            uint32_t c = cs[0];
#pragma unroll
            for (int k = 1; k < N; ++k) c = k == j ? cs[k] : c;
            // query ring j: skip dead intervals from the head; t is covered iff
            // the first live one starts before it (ring 0: iff t > e)
            bool ok;
            {
                const uint32_t sh = 8u * (uint32_t)j;
                const uint32_t m = (uint32_t)(hf >> sh) & 0xffu;
                const uint32_t Q = (capk >> (4 * j)) & 15u, base = (uint32_t)(basek >> sh) & 0xffu;
                uint32_t hd = m & 15u, n = m >> 4;
                int2 f = make_int2(0, 0);
                while (n > 0) {
                    f = rl[(int)(base + hd) << wsh];
                    if (f.y >= t) break;
                    hd = hd + 1 == Q ? 0u : hd + 1;
                    --n;
                }
                ok = live && n > 0 && f.x < t;
                const uint32_t nm = hd | (n << 4);
                hf ^= (uint64_t)(nm ^ m) << sh;  // ring j's byte m becomes nm
            }
            if (ok) {
                if (j == N - 1) {
                    // completion: ring 0 becomes (t, +inf], every other ring empties
                    rl[0] = make_int2(t, rEnd);
                    hf = uint64_t(1) << 4;
                    if constexpr (WL) ++w_done;
                    if (t >= BpR) {
                        const T ta = (T)t + t0b;  // absolute
                        if (a.P > 1 && cnt < kRecFirst) a.rec_first[((int64_t)p * kRecFirst + cnt) * a.G + s] = ta;
                        ++cnt;
                        last = ta;
                    }
                } else {
                    // record at node j into ring j+1: merge into its newest
                    // interval when they touch, else append (dropping the
                    // head, dead, when full)
                    if constexpr (WL) ++w_records;
                    R lj = loR[0], hj = hiR[0];
#pragma unroll
                    for (int k = 1; k + 1 < N; ++k) {
                        if (k == j) {
                            lj = loR[k];
                            hj = hiR[k];
                        }
                    }
                    const R ns = t + lj, ne = t + hj;
                    const uint32_t r = (uint32_t)j + 1u, sh = 8u * r;
                    const uint32_t m = (uint32_t)(hf >> sh) & 0xffu;
                    const uint32_t Q = (capk >> (4 * r)) & 15u, base = (uint32_t)(basek >> sh) & 0xffu;
                    uint32_t hd = m & 15u, n = m >> 4;
                    bool merged = false;
                    if (n > 0) {
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
                        if constexpr (WL) w_maxq = n > w_maxq ? n : w_maxq;
                        hf ^= (uint64_t)((hd | (n << 4)) ^ m) << sh;  // ring r's byte m becomes the new one
                    }
                }
            }
            // advance node j
            c += live ? 1u : 0u;
            const uint32_t cl = c & 0xffffu;
            R v = cl < (c >> 16) ? tbuf[cl] : rEnd;
            v = v < EpR ? v : rEnd;
            const HK nk = PK ? (v == rEnd ? kNoHead : (HK)(((uint32_t)v << 3) | (uint32_t)j)) : (HK)v;
#pragma unroll
            for (int k = 0; k < N; ++k) {
                if (k == j) {
                    cs[k] = c;
                    head[k] = nk;
                }
            }
        }
        if constexpr (WL) {
            // visits of this tile: each node's events its cursor moved past
            // (a query at every node but node 0)
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const uint32_t v = (cs[k] & 0xffffu) - (uint32_t)obuf[ty[k]];
                w_visits += v;
                if (k > 0) w_queries += v;
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

template <typename T, int N, bool PK, bool WL>
__global__ __launch_bounds__(256) void k_lane_tiled(CountArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    lane_item<T, N, PK, WL>(a, blockIdx.x, blockIdx.y, (int64_t)blockIdx.y * gridDim.x + blockIdx.x, smem);
}

// Persistent form: every workgroup takes work items (unit, lane block,
// segment) from a device queue until it is empty.
template <typename T, int N, bool PK, bool WL>
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
        lane_item<T, N, PK, WL>(a, w.blk, w.p, item_base + it, smem);
    }
}

template <typename T, bool PK, bool WL>
const void *tiled_sym(int N) {
    switch (N) {
        case 1: return reinterpret_cast<const void *>(k_lane_tiled<T, 1, PK, WL>);
        case 2: return reinterpret_cast<const void *>(k_lane_tiled<T, 2, PK, WL>);
        case 3: return reinterpret_cast<const void *>(k_lane_tiled<T, 3, PK, WL>);
        case 4: return reinterpret_cast<const void *>(k_lane_tiled<T, 4, PK, WL>);
        case 5: return reinterpret_cast<const void *>(k_lane_tiled<T, 5, PK, WL>);
        case 6: return reinterpret_cast<const void *>(k_lane_tiled<T, 6, PK, WL>);
        case 7: return reinterpret_cast<const void *>(k_lane_tiled<T, 7, PK, WL>);
        case 8: return reinterpret_cast<const void *>(k_lane_tiled<T, 8, PK, WL>);
        default: return nullptr;
    }
}

template <typename T, bool PK, bool WL>
const void *persistent_sym(int N) {
    switch (N) {
        case 1: return reinterpret_cast<const void *>(k_lane_persistent<T, 1, PK, WL>);
        case 2: return reinterpret_cast<const void *>(k_lane_persistent<T, 2, PK, WL>);
        case 3: return reinterpret_cast<const void *>(k_lane_persistent<T, 3, PK, WL>);
        case 4: return reinterpret_cast<const void *>(k_lane_persistent<T, 4, PK, WL>);
        case 5: return reinterpret_cast<const void *>(k_lane_persistent<T, 5, PK, WL>);
        case 6: return reinterpret_cast<const void *>(k_lane_persistent<T, 6, PK, WL>);
        case 7: return reinterpret_cast<const void *>(k_lane_persistent<T, 7, PK, WL>);
        case 8: return reinterpret_cast<const void *>(k_lane_persistent<T, 8, PK, WL>);
        default: return nullptr;
    }
}

inline uint32_t al16(size_t x) { return (uint32_t)((x + 15) & ~size_t(15)); }

}  // namespace

LaneLayout lane_layout(int C, int W, int K, int tile) {
    LaneLayout L;
    size_t o = 0;
    L.off_ring = (uint32_t)o;
    o += al16((size_t)((C > 0 ? C : 1) + 1) * W * sizeof(int2));  // + ring 0 (node 0's starts)
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
const void *lane_tiled_fn(int N, bool pk, bool wl) {
    if (wl) return pk ? tiled_sym<T, true, true>(N) : tiled_sym<T, false, true>(N);
    return pk ? tiled_sym<T, true, false>(N) : tiled_sym<T, false, false>(N);
}

template <typename T>
const void *lane_persistent_fn(int N, bool pk, bool wl) {
    if (wl) return pk ? persistent_sym<T, true, true>(N) : persistent_sym<T, false, true>(N);
    return pk ? persistent_sym<T, true, false>(N) : persistent_sym<T, false, false>(N);
}

template <typename T>
hipError_t lane_launch_tiled(const CountArgs<T> &a, int N, bool pk, dim3 grid, int W, uint32_t lds, hipStream_t st) {
    const void *fn = lane_tiled_fn<T>(N, pk, a.work != nullptr);
    if (!fn) return hipErrorInvalidValue;
    CountArgs<T> arg = a;
    void *args[] = {&arg};
    return hipLaunchKernel(fn, grid, dim3((unsigned)W), args, lds, st);
}

template <typename T>
hipError_t lane_launch_persistent(int N, bool pk, bool wl, unsigned grid, int W, uint32_t lds, hipStream_t st,
                                  const CountArgs<T> *units, const WorkItem *items, int64_t n_items, int64_t item_base,
                                  unsigned long long *queue) {
    const void *fn = lane_persistent_fn<T>(N, pk, wl);
    if (!fn) return hipErrorInvalidValue;
    void *args[] = {&units, &items, &n_items, &item_base, &queue};
    return hipLaunchKernel(fn, dim3(grid), dim3((unsigned)W), args, lds, st);
}

template const void *lane_tiled_fn<int32_t>(int, bool, bool);
template const void *lane_tiled_fn<int64_t>(int, bool, bool);
template const void *lane_persistent_fn<int32_t>(int, bool, bool);
template const void *lane_persistent_fn<int64_t>(int, bool, bool);
template hipError_t lane_launch_tiled<int32_t>(const CountArgs<int32_t> &, int, bool, dim3, int, uint32_t, hipStream_t);
template hipError_t lane_launch_tiled<int64_t>(const CountArgs<int64_t> &, int, bool, dim3, int, uint32_t, hipStream_t);
template hipError_t lane_launch_persistent<int32_t>(int, bool, bool, unsigned, int, uint32_t, hipStream_t,
                                                    const CountArgs<int32_t> *, const WorkItem *, int64_t, int64_t,
                                                    unsigned long long *);
template hipError_t lane_launch_persistent<int64_t>(int, bool, bool, unsigned, int, uint32_t, hipStream_t,
                                                    const CountArgs<int64_t> *, const WorkItem *, int64_t, int64_t,
                                                    unsigned long long *);

}  // namespace epi
