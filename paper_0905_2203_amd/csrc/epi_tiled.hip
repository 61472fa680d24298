// Tiled counting engine and exact segment reconciliation.
//
// k_count_tiled: a workgroup holds W candidate episodes of one size N (one
// lane each) and walks a range of stream tiles.  Each tile (kTile stream
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
// whole segment.
#include <algorithm>
#include <vector>

#include "epi_fsm.h"

namespace epi {

namespace {

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
    int64_t rwords;         // words per bitmap row (B * kTile / 64)
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
    int32_t *flags;
    uint32_t off_qse, off_tbuf, off_qh, off_obuf, off_misc;
};

template <typename T, int N>
__device__ __forceinline__ T load_candidate(const CountArgs<T> &a, LaneFsm<T, N> &f, int64_t slot, int32_t *ty,
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
        Pair<T> v;
        v.s = lo[k];
        v.e = hi[k];
        f.lohi[k * f.W + f.lane] = v;
        H += hi[k];
    }
    return H;
}

template <typename T, int N, bool FILT>
__global__ __launch_bounds__(256) void k_count_tiled(CountArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr T kMin = TsLimits<T>::lo();
    constexpr T kEnd = TsLimits<T>::hi();
    constexpr int L = N > 1 ? N - 1 : 1;
    const int W = blockDim.x, lane = threadIdx.x;
    const int64_t s = (int64_t)blockIdx.x * W + lane;
    const bool active = s < a.G;
    const int64_t slot = a.begin + (active ? s : 0);
    const int p = blockIdx.y;
    T *tbuf = reinterpret_cast<T *>(smem + a.off_tbuf);
    uint16_t *obuf = reinterpret_cast<uint16_t *>(smem + a.off_obuf);
    T *misc = reinterpret_cast<T *>(smem + a.off_misc);

    LaneFsm<T, N> f;
    f.lohi = reinterpret_cast<Pair<T> *>(smem);
    f.qse = reinterpret_cast<Pair<T> *>(smem + a.off_qse);
    f.qh = reinterpret_cast<uint32_t *>(smem + a.off_qh);
    f.W = W;
    f.lane = lane;
    f.Q = a.Q;
    f.gen = 0;
    int32_t ty[N];
    T lo[L], hi[L];
    const T H = load_candidate<T, N>(a, f, slot, ty, lo, hi);
    f.clear_all();
    // vf[k] (k >= 1): no node-k event before this time can meet constraint k
    // with the intervals currently recorded at node k-1 (a lower bound on the
    // earliest interval start + 1; the type maximum when none is recorded).
    T vf[N];
#pragma unroll
    for (int k = 0; k < N; ++k) vf[k] = kEnd;
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
    f.e = p == 0 ? kMin : (T)(Bp - H - 1);

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

    int32_t cnt = 0;
    T last = kMin;
    for (int64_t b = bs; b < b1; ++b) {
        __syncthreads();
        const uint4 *src = reinterpret_cast<const uint4 *>(a.tiled + b * kTile);
        uint4 *dst = reinterpret_cast<uint4 *>(tbuf);
        for (int i = lane; i < (int)(kTile * sizeof(T) / 16); i += W) dst[i] = src[i];
        for (int i = lane; i <= a.K; i += W) obuf[i] = a.loff[b * (a.K + 1) + i];
        __syncthreads();
        if (!active) continue;
        // Per node: the tile range [rs, re) of its type; unfiltered lanes walk
        // it with a cursor, filtered lanes walk the set bits of the words of
        // (range & predecessor-exists & successor-exists).
        int cur[N], stop[N];
        int wi[N], we[N];
        uint64_t msk[N], nmsk[N];  // current word's bits, next word's (prefetched)
        T head[N];
        const int64_t wbase = b * (kTile / 64);
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
        auto filt_head = [&](const int k) -> T {
            while (msk[k] == 0 && wi[k] < we[k]) {
                ++wi[k];
                msk[k] = nmsk[k];
                nmsk[k] = wi[k] < we[k] ? word_bits(k, wi[k] + 1) : 0ull;
            }
            if (msk[k] == 0) return kEnd;
            const T v = tbuf[(wi[k] << 6) + (int)__builtin_ctzll(msk[k])];
            return v < Ep ? v : kEnd;
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
                const T v = cur[k] < stop[k] ? tbuf[cur[k]] : kEnd;
                head[k] = v < Ep ? v : kEnd;
            }
        }
        while (true) {
            // next event of the lane's types (any order among equal times)
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
            // per-node values of the selected node
            T vfj = vf[0], nxt = kEnd, hij = T(0);
#pragma unroll
            for (int k = 1; k < N; ++k)
                if (k == j) vfj = vf[k];
#pragma unroll
            for (int k = 0; k + 1 < N; ++k) {
                if (k == j) {
                    nxt = head[k + 1];
                    hij = hi[k];
                }
            }
            // Exact rejections that need no LDS state: a start not after the
            // last completion; a query below vf; a record whose acceptance
            // interval ends before the next event of the following node
            // (only when that event is known, i.e. inside this tile).
            const bool late_next = j + 1 < N && nxt != kEnd && nxt > (T)(t + hij);
            const bool useless = (j == 0 ? t <= f.e : t < vfj) || late_next;
            if (!useless) {
                bool done = false;
                if (j == 0) {
                    if (N == 1) {
                        f.e = t;
                        done = true;
                    } else {
                        const T ns = f.record(0, t, a.flags);
                        vf[1] = vf[1] < (T)(ns + 1) ? vf[1] : (T)(ns + 1);
                    }
                } else {
                    T nv;
                    const bool ok = f.query(j - 1, t, &nv);
                    if (!ok) {
#pragma unroll
                        for (int k = 1; k < N; ++k)
                            if (k == j) vf[k] = nv;
                    } else if (j == N - 1) {
                        f.e = t;
                        f.gen ^= 1u;
#pragma unroll
                        for (int k = 0; k < N; ++k) vf[k] = kEnd;
                        done = true;
                    } else {
                        const T ns = f.record(j, t, a.flags);
#pragma unroll
                        for (int k = 1; k + 1 < N; ++k)
                            if (k == j) vf[k + 1] = vf[k + 1] < (T)(ns + 1) ? vf[k + 1] : (T)(ns + 1);
                    }
                }
                if (done && t >= Bp) {
                    if (a.P > 1 && cnt < kRecFirst) a.rec_first[((int64_t)p * kRecFirst + cnt) * a.G + s] = t;
                    ++cnt;
                    last = t;
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
                T v = c < st ? tbuf[c] : kEnd;
                v = v < Ep ? v : kEnd;
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
    if (!active) return;
    if (a.P == 1) {
        a.counts[a.orig ? a.orig[slot] : slot] = cnt;
    } else {
        a.rec_cnt[(int64_t)p * a.G + s] = cnt;
        a.rec_last[(int64_t)p * a.G + s] = last;
    }
}

__global__ void k_zero_counts(const int32_t *__restrict__ orig, int64_t G, int32_t *__restrict__ counts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < G) counts[orig ? orig[i] : i] = 0;
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

template <typename T, int N>
__global__ __launch_bounds__(256) void k_reconcile(CountArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr T kMin = TsLimits<T>::lo();
    constexpr T kEnd = TsLimits<T>::hi();
    const int W = blockDim.x, lane = threadIdx.x;
    const int64_t s = (int64_t)blockIdx.x * W + lane;
    if (s >= a.G) return;  // no barriers below
    const int64_t slot = a.begin + s;
    LaneFsm<T, N> f;
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
    int32_t lo_[N], hi_[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        lo_[k] = a.type_off[ty[k]];
        hi_[k] = a.type_off[ty[k] + 1];
    }
    T tau = kMin;
    int64_t total = 0;
    for (int p = 0; p < a.P; ++p) {
        const int64_t b0 = (int64_t)p * a.S;
        const int64_t b1 = b0 + a.S < a.B ? b0 + a.S : a.B;
        const T Bp = p == 0 ? kMin : a.tile_t0[b0];
        const T Ep = p == a.P - 1 ? kEnd : a.tile_t0[b1];
        const int32_t c = a.rec_cnt[(int64_t)p * a.G + s];
        const T last = a.rec_last[(int64_t)p * a.G + s];
        if (p == 0 || tau < (T)(Bp - H)) {
            total += c;
            if (c > 0) tau = last;
            continue;
        }
        // re-run from the state right after the completion at tau
        f.e = tau;
        f.clear_all();
        int32_t cur[N];
        T head[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            cur[k] = upper_bound(a.ts_by_type, lo_[k], hi_[k], tau);
            const T v = cur[k] < hi_[k] ? a.ts_by_type[cur[k]] : kEnd;
            head[k] = v < Ep ? v : kEnd;
        }
        const int nspec = c < kRecFirst ? c : kRecFirst;
        int qi = 0;
        int32_t fcount = 0;
        T flast = tau;
        bool synced = false;
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
                ++fcount;
                flast = t;
                while (qi < nspec && a.rec_first[((int64_t)p * kRecFirst + qi) * a.G + s] < t) ++qi;
                if (qi < nspec && a.rec_first[((int64_t)p * kRecFirst + qi) * a.G + s] == t) {
                    total += fcount + (c - qi - 1);
                    tau = last;
                    synced = true;
                    break;
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
        if (!synced) {
            total += fcount;
            tau = flast;
        }
    }
    a.counts[a.orig ? a.orig[slot] : slot] = (int32_t)total;
}

template <typename T>
using KFn = void (*)(CountArgs<T>);

template <typename T, bool F>
KFn<T> pick_count_f(int N) {
    switch (N) {
        case 1: return k_count_tiled<T, 1, F>;
        case 2: return k_count_tiled<T, 2, F>;
        case 3: return k_count_tiled<T, 3, F>;
        case 4: return k_count_tiled<T, 4, F>;
        case 5: return k_count_tiled<T, 5, F>;
        case 6: return k_count_tiled<T, 6, F>;
        case 7: return k_count_tiled<T, 7, F>;
        case 8: return k_count_tiled<T, 8, F>;
        default: return nullptr;
    }
}

template <typename T>
KFn<T> pick_count(int N, bool filtered) {
    return filtered ? pick_count_f<T, true>(N) : pick_count_f<T, false>(N);
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

inline uint32_t al16(size_t x) { return (uint32_t)((x + 15) & ~size_t(15)); }

template <typename T>
struct Layout {
    uint32_t off_qse, off_tbuf, off_qh, off_obuf, off_misc, total;
};

template <typename T>
Layout<T> layout(int N, int Q, int W, int K, bool tiles) {
    Layout<T> L;
    const size_t lv = N > 1 ? N - 1 : 0;
    size_t o = al16(lv * W * sizeof(Pair<T>));
    L.off_qse = (uint32_t)o;
    o += al16(lv * Q * W * sizeof(Pair<T>));
    L.off_tbuf = (uint32_t)o;
    o += tiles ? al16(kTile * sizeof(T)) : 0;
    L.off_qh = (uint32_t)o;
    o += al16(lv * W * sizeof(uint32_t));
    L.off_obuf = (uint32_t)o;
    o += tiles ? al16((K + 1) * sizeof(uint16_t)) : 0;
    L.off_misc = (uint32_t)o;
    o += 16 * sizeof(T);
    L.total = (uint32_t)o;
    return L;
}

constexpr uint32_t kLdsSoft = 64 * 1024;
constexpr uint32_t kLdsHard = 160 * 1024;

// Widest workgroup (at most max_lanes) whose LDS fits comfortably; else the
// widest that fits at all.
template <typename T>
int pick_lanes(int N, int Q, int K, int max_lanes) {
    int fit = 64;
    bool any = false;
    for (int W : {256, 128, 64}) {
        if (max_lanes > 0 && W > max_lanes) continue;
        const Layout<T> L = layout<T>(N, Q, W, K, true);
        if (L.total <= kLdsSoft) return W;
        if (!any && L.total <= kLdsHard) {
            fit = W;
            any = true;
        }
    }
    return fit;
}

template <typename T>
hipError_t ensure_lds_attr(KFn<T> fn, uint32_t bytes) {
    if (bytes <= kLdsSoft) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

template <typename T>
hipError_t count_t(const Stream &s, CandSet &c, const CountOptions &opt, int32_t *d_flags, hipStream_t st) {
    hipError_t e;
    for (const Group &g : c.groups) {
        const int64_t G = g.end - g.begin;
        if (G <= 0) continue;
        if (s.n == 0) {  // no events: every count is zero
            k_zero_counts<<<(unsigned)((G + 255) / 256), 256, 0, st>>>(
                c.compact ? nullptr : c.orig.as<int32_t>() + g.begin, G, c.counts.as<int32_t>() + (c.compact ? g.begin : 0));
            if ((e = hipGetLastError()) != hipSuccess) return e;
            continue;
        }
        const int W = pick_lanes<T>(g.N, g.Q, s.K, opt.lanes);
        const Layout<T> L = layout<T>(g.N, g.Q, W, s.K, true);
        const uint32_t lds = L.total;
        if (lds > kLdsHard) return hipErrorInvalidConfiguration;
        // segments
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
        const int64_t S = (s.B + P - 1) / P;
        P = (s.B + S - 1) / S;

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
        a.P = (int32_t)P;
        a.S = S;
        a.orig = c.compact ? nullptr : c.orig.as<int32_t>();
        a.counts = c.counts.as<int32_t>();
        a.flags = d_flags;
        a.off_qse = L.off_qse;
        a.off_tbuf = L.off_tbuf;
        a.off_qh = L.off_qh;
        a.off_obuf = L.off_obuf;
        a.off_misc = L.off_misc;
        if (P > 1) {
            const size_t need = (size_t)P * G * (sizeof(int32_t) + sizeof(T) * (1 + kRecFirst));
            if (c.scratch.bytes < need) {
                if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
                if ((e = c.scratch.alloc(need)) != hipSuccess) return e;
            }
            unsigned char *base = c.scratch.as<unsigned char>();
            a.rec_last = reinterpret_cast<T *>(base);
            a.rec_first = a.rec_last + (size_t)P * G;
            a.rec_cnt = reinterpret_cast<int32_t *>(a.rec_first + (size_t)P * G * kRecFirst);
        }
        const bool filtered = c.compact && c.pred_bits && c.succ_bits;
        a.pbits = filtered ? c.pred_bits : nullptr;
        a.sbits = filtered ? c.succ_bits : nullptr;
        a.rwords = s.B * (kTile / 64);
        KFn<T> fn = pick_count<T>(g.N, filtered);
        if (!fn) return hipErrorInvalidValue;
        if ((e = ensure_lds_attr<T>(fn, lds)) != hipSuccess) return e;
        const dim3 grid((unsigned)((G + W - 1) / W), (unsigned)P);
        fn<<<grid, W, lds, st>>>(a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (P > 1) {
            KFn<T> rf = pick_reconcile<T>(g.N);
            const int RW = 64;
            const Layout<T> RL = layout<T>(g.N, g.Q, RW, s.K, false);
            CountArgs<T> r = a;
            r.off_qse = RL.off_qse;
            r.off_qh = RL.off_qh;
            r.off_tbuf = RL.off_tbuf;
            r.off_obuf = RL.off_obuf;
            r.off_misc = RL.off_misc;
            if ((e = ensure_lds_attr<T>(rf, RL.total)) != hipSuccess) return e;
            rf<<<(unsigned)((G + RW - 1) / RW), RW, RL.total, st>>>(r);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_count(const Stream &s, CandSet &c, const CountOptions &opt, int32_t *d_flags, hipStream_t st) {
    if (s.ts_kind == EPI_TS_I64) return count_t<int64_t>(s, c, opt, d_flags, st);
    return count_t<int32_t>(s, c, opt, d_flags, st);
}

}  // namespace epi
