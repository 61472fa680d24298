// Counting by Parallel Local Tracking (Sec. IV-C) followed by the greedy of
// Alg. 1 (Sec. IV-A): the engine for a few long episodes over a long stream,
// where one lane per episode would leave most of the GPU idle.  It is
// parallel over the events of each node's type instead of over episodes.
//
// For an episode alpha, the chain events of node k are the events x of type
// alpha[k] that end an occurrence of alpha[1..k]; each carries the latest
// start L_k(x) of such an occurrence.  Keeping only the latest start per end
// event is exact for the greedy (Sec. IV-A: the non-overlapped subset is
// taken in order of end times, and of two occurrences with one end the later
// start dominates) and keeps every list no longer than its type's events.
// L_1(x) = t_x.  Along the chain events of a node, in time order, L is
// non-decreasing, so the predecessor with the latest start is the latest
// chain event y of node k-1 with lo < t_x - t_y <= hi: one binary search per
// event, which is the backward tracking of Alg. 2 with the search replacing
// the scan.  The events with a chain are compacted in time order by a
// search (which counts) / scan / write pass (the order-preserving compaction
// of Sec. IV-D/E).  The count is Alg. 1 over the intervals (L_N(x), t_x) in
// time order: after keeping x the next kept interval is the first with
// L > t_x, a binary search over the non-decreasing L; the kept intervals form
// the successor chain of the first interval, whose length and last element
// pointer jumping finds (first inside blocks of intervals in LDS, then across
// blocks).
//
// Under stream-order overlap the starts L and the ends compared with them are
// stream positions instead of times (the predecessor windows stay in time);
// along a node's chain events in (time, position) order the latest start
// position is still non-decreasing, so nothing else changes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "epi_internal.h"

namespace epi {
namespace {

constexpr int kTB = 256;               // threads per block of the per-event kernels
constexpr int kTBLog = 8;
static_assert((1 << kTBLog) == kTB, "kTBLog");
constexpr int kTPer = 4;               // events per thread
constexpr int kTChunk = kTB * kTPer;   // events per block
constexpr int kTWaves = kTB / 64;
constexpr int kScanT = 1024;           // threads of the per-episode scan
constexpr int kStage = 2048;           // chain events of node k-1 staged in LDS per block
constexpr int kJPer = 4;               // intervals per thread of a pointer-jumping round
constexpr int kMaxJobs = 65535;        // episodes per launch (grid y)
constexpr size_t kChunkBytes = size_t(2) << 30;  // working set of one group of episodes

template <typename T>
struct TrackJob {
    const T *pt;         // chain events of node k-1: times (non-decreasing)
    const T *pL;         // and their latest starts (non-decreasing)
    const int32_t *pn;   // how many (on the device; null: pn_host)
    int32_t pn_host;
    int32_t ne;          // events of node k's type
    const T *et;         // their times, in order
    T lo, hi;            // constraint (lo, hi] from node k-1 to node k
    const int32_t *ep;   // stream positions of node k's events (stream-order overlap), else null
    T *tl;               // per event of node k: its latest start, or the type minimum (no chain)
    T *ot, *oL;          // chain events of node k (written in time order)
    T *oK;               // and their stream positions (stream-order overlap), else null
    int32_t *on;         // how many (written by the scan)
    int32_t *blk;        // per-block counts, then offsets: max(1, ceil(ne / kTChunk)) entries
};

// (next uncovered interval, intervals covered, last covered interval) of the
// pointer jumping
struct Hop {
    int32_t nx, d, last, pad;
};

template <typename T>
struct GreedyJob {
    const T *t, *L;      // intervals (L_N(x), t_x) in time order
    const T *key;        // the ends compared with the starts: t, or stream positions (then L holds
                         // the first events' stream positions)
    const int32_t *pn;   // how many (device; null: pn_host)
    int32_t pn_host;
    int32_t bound;       // capacity of the arrays below
    Hop *h[2];
    int32_t slot;        // submission index of the episode
};

__device__ __forceinline__ int32_t n_blocks(int32_t ne) { return max(1, (ne + kTChunk - 1) / kTChunk); }

// first index in [a, b) of ts with ts[index] >= x (b if none)
template <typename T>
__device__ __forceinline__ int32_t lower_idx(const T *ts, int32_t a, int32_t b, T x) {
    while (a < b) {
        const int32_t mid = a + (b - a) / 2;
        if (ts[mid] < x) a = mid + 1;
        else b = mid;
    }
    return a;
}

// The same by one wave: 64 probes per step, so a few dependent loads instead
// of one per halving (the value is uniform across the wave).
template <typename T>
__device__ __forceinline__ int32_t lower_idx_wave(const T *ts, int32_t a, int32_t b, T x) {
    const int lane = threadIdx.x & 63;
    while (b - a > 64) {
        const int32_t step = (b - a + 63) / 64;
        const int64_t p = (int64_t)a + (int64_t)lane * step;
        const int cnt = __popcll(__ballot(p < b && ts[p] < x));
        if (cnt == 0) return a;
        // the first index at or above x lies in (a + (cnt-1) step, a + cnt step]
        const int64_t na = (int64_t)a + (int64_t)(cnt - 1) * step + 1;
        const int64_t nb = (int64_t)a + (int64_t)cnt * step;
        a = (int32_t)na;
        b = (int32_t)min<int64_t>(nb, b);
    }
    return a + __popcll(__ballot(a + lane < b && ts[a + lane] < x));
}

// Backward tracking of one block of node k's events: each finds the latest
// chain event y of node k-1 with t - hi <= t_y < t - lo and takes its latest
// start.  The chain events any event of the block can reach (from the block's
// first time - lo back by one entry to its last time - lo) are staged in LDS
// when they fit, else searched in place.  Writes every event's latest start
// (tl) and the block's number of chain events.
template <typename T>
__global__ __launch_bounds__(kTB) void k_track_search(const TrackJob<T> *__restrict__ jobs) {
    const TrackJob<T> j = jobs[blockIdx.y];
    if ((int32_t)blockIdx.x >= n_blocks(j.ne)) return;
    const int32_t np = j.pn ? *j.pn : j.pn_host;
    __shared__ T st[kStage], sL[kStage];
    __shared__ int32_t rng[2], tot;
    const int64_t base = (int64_t)blockIdx.x * kTChunk;
    const int64_t end = min<int64_t>(base + kTChunk, j.ne);
    if (threadIdx.x < 128) {  // waves 0 and 1: the range of the first and of the last event
        const int w = threadIdx.x >> 6;
        int32_t a = 0;
        if (base < end) a = lower_idx_wave(j.pt, 0, np, (w == 0 ? j.et[base] : j.et[end - 1]) - j.lo);
        if ((threadIdx.x & 63) == 0) rng[w] = a;
    }
    if (threadIdx.x == 0) tot = 0;
    __syncthreads();
    const int32_t s0 = max(rng[0] - 1, 0), len = rng[1] - s0;
    const bool staged = len <= kStage;
    if (staged)
        for (int32_t q = threadIdx.x; q < len; q += kTB) {
            st[q] = j.pt[s0 + q];
            sL[q] = j.pL[s0 + q];
        }
    __syncthreads();
    int32_t c = 0;
    for (int r = 0; r < kTPer; ++r) {
        const int64_t i = base + r * kTB + threadIdx.x;
        if (i >= end) break;
        const T t = j.et[i];
        T L = TsLimits<T>::lo();
        if (staged) {
            const int32_t a = lower_idx(st, 0, len, t - j.lo);
            if (a > 0 && st[a - 1] >= t - j.hi) L = sL[a - 1];
        } else {
            const int32_t a = lower_idx(j.pt, 0, np, t - j.lo);
            if (a > 0 && j.pt[a - 1] >= t - j.hi) L = j.pL[a - 1];
        }
        j.tl[i] = L;
        c += L != TsLimits<T>::lo();
    }
    atomicAdd(&tot, c);
    __syncthreads();
    if (threadIdx.x == 0) j.blk[blockIdx.x] = tot;
}

// Exclusive scan of one episode's block counts (one workgroup per episode);
// the total is the node's number of chain events.
template <typename T>
__global__ __launch_bounds__(kScanT) void k_track_scan(const TrackJob<T> *__restrict__ jobs) {
    const TrackJob<T> j = jobs[blockIdx.y];
    const int32_t nb = n_blocks(j.ne);
    __shared__ int32_t wsum[kScanT / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t carry = 0;
    for (int32_t b0 = 0; b0 < nb; b0 += kScanT) {
        const int32_t b = b0 + (int32_t)threadIdx.x;
        const int32_t v = b < nb ? j.blk[b] : 0;
        int32_t x = v;
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        int32_t woff = 0, total = 0;
        for (int q = 0; q < kScanT / 64; ++q) {
            const int32_t s = wsum[q];
            if (q < w) woff += s;
            total += s;
        }
        if (b < nb) j.blk[b] = carry + woff + x - v;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *j.on = carry;
}

// Order-preserving compaction of the events with a chain.
template <typename T>
__global__ __launch_bounds__(kTB) void k_track_write(const TrackJob<T> *__restrict__ jobs) {
    const TrackJob<T> j = jobs[blockIdx.y];
    if ((int32_t)blockIdx.x >= n_blocks(j.ne)) return;
    __shared__ int32_t wc[kTWaves];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t pos = j.blk[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kTChunk;
    for (int r = 0; r < kTPer; ++r) {
        const int64_t i = base + r * kTB + threadIdx.x;
        T t = 0, L = TsLimits<T>::lo();
        if (i < j.ne) {
            t = j.et[i];
            L = j.tl[i];
        }
        const bool ok = L != TsLimits<T>::lo();
        const uint64_t bal = __ballot(ok);
        const int32_t below = __popcll(bal & ((uint64_t(1) << lane) - 1));
        if (lane == 0) wc[w] = __popcll(bal);
        __syncthreads();
        int32_t woff = 0, total = 0;
        for (int q = 0; q < kTWaves; ++q) {
            if (q < w) woff += wc[q];
            total += wc[q];
        }
        if (ok) {
            j.ot[pos + woff + below] = t;
            j.oL[pos + woff + below] = L;
            if (j.oK) j.oK[pos + woff + below] = (T)j.ep[i];
        }
        pos += total;
        __syncthreads();
    }
}

// Successor of every interval under the greedy: the first later interval
// whose start is after its end (the end of the list if none).  Each block of
// kTB intervals then follows its successors inside the block by pointer
// jumping in LDS, so every record leaves the block: (first successor at or
// after the block's end, intervals covered, last covered).  The chain from any
// interval then takes at most one record per block.
template <typename T>
__global__ __launch_bounds__(kTB) void k_track_next(const GreedyJob<T> *__restrict__ jobs) {
    const GreedyJob<T> j = jobs[blockIdx.y];
    const int32_t n = j.pn ? *j.pn : j.pn_host;
    const int64_t b0 = (int64_t)blockIdx.x * kTB;
    if (b0 >= n) return;  // the whole block
    const int t = threadIdx.x;
    const int64_t i = b0 + t;
    const int32_t bend = (int32_t)min<int64_t>(b0 + kTB, n);
    __shared__ int32_t snx[2][kTB], sd[2][kTB], sl[2][kTB];
    int32_t nx = n, d = 0, last = 0;
    if (i < n) {
        const T ki = j.key[i];
        int32_t a = (int32_t)i + 1, b = n;
        while (a < b) {
            const int32_t mid = a + (b - a) / 2;
            if (j.L[mid] <= ki) a = mid + 1;
            else b = mid;
        }
        nx = a;
        d = 1;
        last = (int32_t)i;
    }
    snx[0][t] = nx;
    sd[0][t] = d;
    sl[0][t] = last;
    __syncthreads();
    for (int r = 0; r < kTBLog; ++r) {
        const int src = r & 1;
        int32_t x = snx[src][t], dd = sd[src][t], ll = sl[src][t];
        if (i < n && x < bend) {  // a successor inside the block (x > i >= b0)
            const int k = x - (int32_t)b0;
            dd += sd[src][k];
            ll = sl[src][k];
            x = snx[src][k];
        }
        snx[src ^ 1][t] = x;
        sd[src ^ 1][t] = dd;
        sl[src ^ 1][t] = ll;
        __syncthreads();
    }
    if (i < n) j.h[0][i] = Hop{snx[kTBLog & 1][t], sd[kTBLog & 1][t], sl[kTBLog & 1][t], 0};
}

// One pointer-jumping round: every interval's (next uncovered interval,
// covered count, last covered interval) over twice the distance.
// Each thread takes kJPer intervals, so that their loads are in flight together.
template <typename T>
__global__ __launch_bounds__(kTB) void k_track_jump(const GreedyJob<T> *__restrict__ jobs, int r) {
    const GreedyJob<T> j = jobs[blockIdx.y];
    const int32_t n = j.pn ? *j.pn : j.pn_host;
    const int64_t i0 = (int64_t)blockIdx.x * kTB * kJPer + threadIdx.x;
    if (i0 >= n) return;
    const Hop *src = j.h[r & 1];
    Hop *dst = j.h[(r & 1) ^ 1];
    Hop x[kJPer];
#pragma unroll
    for (int q = 0; q < kJPer; ++q)
        if (i0 + q * kTB < n) x[q] = src[i0 + q * kTB];
#pragma unroll
    for (int q = 0; q < kJPer; ++q)
        if (i0 + q * kTB < n && x[q].nx < n) {
            const Hop y = src[x[q].nx];
            x[q] = Hop{y.nx, x[q].d + y.d, y.last, 0};
        }
#pragma unroll
    for (int q = 0; q < kJPer; ++q)
        if (i0 + q * kTB < n) dst[i0 + q * kTB] = x[q];
}

template <typename T>
__global__ __launch_bounds__(kTB) void k_track_final(const GreedyJob<T> *__restrict__ jobs, int32_t njobs, int R,
                                                     int32_t *__restrict__ counts, T *__restrict__ tau) {
    const int32_t q = blockIdx.x * kTB + threadIdx.x;
    if (q >= njobs) return;
    const GreedyJob<T> j = jobs[q];
    const int32_t n = j.pn ? *j.pn : j.pn_host;
    const Hop h0 = n > 0 ? j.h[R & 1][0] : Hop{0, 0, 0, 0};
    counts[j.slot] = n > 0 ? h0.d : 0;
    if (tau) tau[j.slot] = n > 0 ? j.t[h0.last] : TsLimits<T>::lo();
}

// stream positions of a type's events, widened to the time type
template <typename T>
__global__ __launch_bounds__(kTB) void k_track_pos(const int32_t *__restrict__ pos, int32_t n, T *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x;
    if (i < n) out[i] = (T)pos[i];
}

size_t round_up(size_t b) { return (b + 255) & ~size_t(255); }

template <typename T>
hipError_t count_tracking_t(const Stream &s, CandSet &c, hipStream_t st) {
    const int64_t m = c.m;
    if (m == 0) return hipSuccess;
    auto nt = [&](int32_t E) -> int32_t { return s.h_off[E + 1] - s.h_off[E]; };
    const bool so = c.stream_order;
    const int nbuf = so ? 8 : 5;  // (t, L) x 2 and tl; with stream order also K x 2 and node 1's positions
    auto job_bytes = [&](int64_t q) -> size_t {
        const int N = c.h_N[q];
        const int32_t *ty = c.h_types.data() + q * kMaxN;
        size_t maxl = so ? (size_t)nt(ty[0]) : 0, nbm = 1;
        for (int k = 1; k < N; ++k) {
            maxl = std::max<size_t>(maxl, (size_t)nt(ty[k]));
            nbm = std::max<size_t>(nbm, ((size_t)nt(ty[k]) + kTChunk - 1) / kTChunk);
        }
        const size_t nN = std::max<size_t>(1, (size_t)nt(ty[N - 1]));
        return nbuf * round_up(sizeof(T) * std::max<size_t>(maxl, 1)) + 2 * round_up(sizeof(Hop) * nN) +
               round_up(4 * nbm) + round_up(4 * kMaxN);
    };
    const T *tsb = s.ts_by_type.as<T>();
    hipError_t e;
    for (int64_t q0 = 0; q0 < m;) {
        // a group of episodes whose working set fits the budget (at least one)
        int64_t q1 = q0;
        size_t total = 0;
        while (q1 < m && q1 - q0 < kMaxJobs) {
            const size_t b = job_bytes(q1);
            if (q1 > q0 && total + b > kChunkBytes) break;
            total += b;
            ++q1;
        }
        DevBuf &work = c.track_work;
        if (work.bytes < total && (e = work.alloc(total)) != hipSuccess) return e;
        std::vector<std::vector<TrackJob<T>>> lv(kMaxN + 1);
        std::vector<GreedyJob<T>> gj;
        int32_t max_bound = 1;
        char *p = work.as<char>();
        for (int64_t q = q0; q < q1; ++q) {
            const int N = c.h_N[q];
            const int32_t *ty = c.h_types.data() + q * kMaxN;
            size_t maxl = so ? (size_t)nt(ty[0]) : 0, nbm = 1;
            for (int k = 1; k < N; ++k) {
                maxl = std::max<size_t>(maxl, (size_t)nt(ty[k]));
                nbm = std::max<size_t>(nbm, ((size_t)nt(ty[k]) + kTChunk - 1) / kTChunk);
            }
            const size_t nN = std::max<size_t>(1, (size_t)nt(ty[N - 1]));
            const size_t lb = round_up(sizeof(T) * std::max<size_t>(maxl, 1));
            T *buf[2][2] = {{(T *)p, (T *)(p + lb)}, {(T *)(p + 2 * lb), (T *)(p + 3 * lb)}};
            T *tl = (T *)(p + 4 * lb);
            T *kb[2] = {so ? (T *)(p + 5 * lb) : nullptr, so ? (T *)(p + 6 * lb) : nullptr};
            T *l1 = so ? (T *)(p + 7 * lb) : nullptr;
            p += nbuf * lb;
            Hop *ga[2];
            for (int a = 0; a < 2; ++a) {
                ga[a] = (Hop *)p;
                p += round_up(sizeof(Hop) * nN);
            }
            int32_t *blk = (int32_t *)p;
            p += round_up(4 * nbm);
            int32_t *on = (int32_t *)p;
            p += round_up(4 * kMaxN);
            // node 1: the type's events, each its own start (its time, or its stream position)
            const T *pt = tsb + s.h_off[ty[0]], *pL = pt, *pK = pt;
            if (so) {
                if (nt(ty[0]) > 0)
                    k_track_pos<T><<<(unsigned)((nt(ty[0]) + kTB - 1) / kTB), kTB, 0, st>>>(
                        s.pos_by_type.as<int32_t>() + s.h_off[ty[0]], nt(ty[0]), l1);
                pL = pK = l1;
            }
            const int32_t *pn = nullptr;
            int32_t pn_host = nt(ty[0]);
            for (int k = 1; k < N; ++k) {
                TrackJob<T> j;
                j.pt = pt;
                j.pL = pL;
                j.pn = pn;
                j.pn_host = pn_host;
                j.ne = nt(ty[k]);
                j.et = tsb + s.h_off[ty[k]];
                j.lo = (T)c.h_lo[q * (kMaxN - 1) + k - 1];
                j.hi = (T)c.h_hi[q * (kMaxN - 1) + k - 1];
                j.ep = so ? s.pos_by_type.as<int32_t>() + s.h_off[ty[k]] : nullptr;
                j.tl = tl;
                j.oK = kb[k & 1];
                j.ot = buf[k & 1][0];
                j.oL = buf[k & 1][1];
                j.on = on + k;
                j.blk = blk;
                lv[k].push_back(j);
                pt = j.ot;
                pL = j.oL;
                pK = so ? j.oK : j.ot;
                pn = j.on;
            }
            GreedyJob<T> g;
            g.t = pt;
            g.L = pL;
            g.key = pK;
            g.pn = pn;
            g.pn_host = pn_host;
            g.bound = (int32_t)nN;
            g.h[0] = ga[0];
            g.h[1] = ga[1];
            g.slot = (int32_t)q;
            gj.push_back(g);
            max_bound = std::max<int32_t>(max_bound, g.bound);
        }
        // descriptors: the levels' jobs, then the greedy's
        size_t db = 0;
        std::vector<size_t> loff(kMaxN + 1, 0);
        for (int k = 1; k < kMaxN; ++k) {
            loff[k] = db;
            db += round_up(sizeof(TrackJob<T>) * lv[k].size());
        }
        const size_t goff = db;
        db += round_up(sizeof(GreedyJob<T>) * gj.size());
        std::vector<char> hd(db);
        for (int k = 1; k < kMaxN; ++k)
            if (!lv[k].empty()) std::copy_n((const char *)lv[k].data(), sizeof(TrackJob<T>) * lv[k].size(), &hd[loff[k]]);
        std::copy_n((const char *)gj.data(), sizeof(GreedyJob<T>) * gj.size(), &hd[goff]);
        DevBuf &desc = c.track_desc;
        if (desc.bytes < db && (e = desc.alloc(db)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(desc.p, hd.data(), db, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
        for (int k = 1; k < kMaxN; ++k) {
            if (lv[k].empty()) continue;
            int32_t gx = 1;
            for (const auto &j : lv[k]) gx = std::max<int32_t>(gx, (j.ne + kTChunk - 1) / kTChunk);
            const auto *dj = (const TrackJob<T> *)(desc.as<char>() + loff[k]);
            const dim3 grid((unsigned)gx, (unsigned)lv[k].size());
            k_track_search<T><<<grid, kTB, 0, st>>>(dj);
            k_track_scan<T><<<dim3(1, (unsigned)lv[k].size()), kScanT, 0, st>>>(dj);
            k_track_write<T><<<grid, kTB, 0, st>>>(dj);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        const auto *dg = (const GreedyJob<T> *)(desc.as<char>() + goff);
        const dim3 ggrid((unsigned)((max_bound + kTB - 1) / kTB), (unsigned)gj.size());
        k_track_next<T><<<ggrid, kTB, 0, st>>>(dg);
        // records leave their block of kTB intervals: at most one per block on any chain
        const int64_t max_blocks = (max_bound + kTB - 1) / kTB;
        int R = 0;
        while ((int64_t(1) << R) < max_blocks) ++R;
        const dim3 jgrid((unsigned)((max_bound + kTB * kJPer - 1) / (kTB * kJPer)), (unsigned)gj.size());
        for (int r = 0; r < R; ++r) k_track_jump<T><<<jgrid, kTB, 0, st>>>(dg, r);
        k_track_final<T><<<(unsigned)((gj.size() + kTB - 1) / kTB), kTB, 0, st>>>(
            dg, (int32_t)gj.size(), R, c.counts.as<int32_t>(), c.tau.p ? c.tau.as<T>() : nullptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // the host descriptors die here, and the next group reuses the working set
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        q0 = q1;
    }
    return hipSuccess;
}

template <typename T>
__global__ void k_scatter_deep(int64_t md, const int32_t *__restrict__ idx, const int32_t *__restrict__ dc,
                               const T *__restrict__ dtau, int32_t *__restrict__ counts, T *__restrict__ tau) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= md) return;
    counts[idx[i]] = dc[i];
    if (tau) tau[idx[i]] = dtau[i];
}

}  // namespace

hipError_t count_deep_subset(const Stream &s, CandSet &c, hipStream_t st) {
    if (!c.deep || c.deep->m == 0) return hipSuccess;
    CandSet &d = *c.deep;
    hipError_t e = launch_count_tracking(s, d, st);
    if (e != hipSuccess) return e;
    const unsigned blocks = (unsigned)((d.m + 255) / 256);
    if (s.ts_kind == EPI_TS_I64)
        k_scatter_deep<int64_t><<<blocks, 256, 0, st>>>(d.m, c.deep_idx.as<int32_t>(), d.counts.as<int32_t>(),
                                                       d.tau.as<int64_t>(), c.counts.as<int32_t>(),
                                                       c.tau.p ? c.tau.as<int64_t>() : nullptr);
    else
        k_scatter_deep<int32_t><<<blocks, 256, 0, st>>>(d.m, c.deep_idx.as<int32_t>(), d.counts.as<int32_t>(),
                                                       d.tau.as<int32_t>(), c.counts.as<int32_t>(),
                                                       c.tau.p ? c.tau.as<int32_t>() : nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

hipError_t launch_count_tracking(const Stream &s, CandSet &c, hipStream_t st) {
    if (c.compact || (int64_t)c.h_N.size() != c.m) return hipErrorInvalidValue;
    return s.ts_kind == EPI_TS_I64 ? count_tracking_t<int64_t>(s, c, st) : count_tracking_t<int32_t>(s, c, st);
}

}  // namespace epi
