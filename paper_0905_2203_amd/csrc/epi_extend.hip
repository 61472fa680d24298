// Extension engine of level-wise discovery: the decomposition of Sec. IV-A
// organised around Apriori's candidate families.
//
// Subproblem-1 (Sec. IV-A) needs only, for every end event x of an episode,
// the latest start s(x) among its occurrences ending at x: an occurrence set
// holding one such occurrence per end event has the same optimum.  For a
// candidate alpha + (B, (lo, hi]), where alpha is a frequent episode of the
// previous level, an event y of type B ends an occurrence iff some end event
// x of alpha has lo < t_y - t_x <= hi, and then
//     s(y) = max over such x of s(x).
// Over alpha's end events s is non-decreasing in time (the latest occurrence
// end before a window edge carries the latest start), so the maximum is taken
// at the latest x with t_x < t_y - lo, provided t_x >= t_y - hi.  The greedy
// of Alg. 1 over the y in time order (keep y when s(y) > the last kept end,
// starting from minus infinity) gives the count.
//
// Window walk.  Every candidate of alpha needs only the stream events that
// follow one of alpha's end events by at most H (the longest interval end of
// the menu): the union U(alpha) of the windows (t_x, t_x + H].  One wave per
// alpha walks U(alpha) once, 64 stream positions at a time, for all of
// alpha's extensions together:
//   * the runs of U are cut from alpha's chain list 64 entries at a time
//     (entry x covers stream positions (p_x, wend(p_x)); overlaps are
//     removed with a prefix maximum) and packed into full batches;
//   * each lane of a batch holds one stream event y and finds, for every menu
//     interval m, s_m(y) from the few end events that precede the batch by at
//     most H (uniform loop, scalar reads);
//   * each extension type B of alpha owns a lane that keeps one greedy state
//     per menu interval; a batch's events reach the lanes of their types
//     through one LDS mask per lane (an atomic OR per event), and each lane
//     runs its greedy over its events in time order, reading them with
//     cross-lane permutes.
// This is the tracking step of Parallel Local Tracking (Sec. IV-C) done for
// all extensions of an episode at once: the work per alpha is |U(alpha)|
// stream events whatever the number of its extensions.
//
// Level 1 counts distinct timestamps per type.  Level 2 extends a frequent
// type (its chain list is its own events, s = t).  The chain lists of a
// level's frequent episodes are written by a second walk over the alphas that
// have frequent extensions, at offsets from an exclusive scan of their
// end-event counts (the count / scan / write compaction of Sec. IV-E).
#include <algorithm>
#include <chrono>
#include <numeric>
#include <thread>

#include "epi_internal.h"

namespace epi {

namespace {

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0) { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }

constexpr int kWave = 64;
constexpr uint16_t kNoSlot = 0;  // owner-slot entry of a type no lane counts (no intervals)
// List path: taken for levels with fewer alphas than Mine::list_alphas, whose
// walks are cut into pieces so that about kListJobs workgroups run.  Chain
// lists of levels with fewer write jobs than kWritePieced are written by
// walks cut into pieces likewise (a size walk and a list walk over the
// frequent extensions, about kWriteJobs workgroups each), so that no long
// walk runs alone; with more jobs one walk per job keeps the GPU busy and
// costs half the work.
constexpr int64_t kListJobs = 65536;
constexpr int64_t kWritePieced = 32768;
constexpr int64_t kWriteJobs = 262144;

// One entry of a chain list: an end event of an episode (time, stream
// position) and the latest start of an occurrence ending there.
template <typename T>
struct ChainEntry {
    T t, s;
    int32_t p;
};

template <typename T>
struct WalkArgs {
    const uint16_t *ty16;     // [n] event types, stream order
    const T *times;           // [n]
    const int32_t *wend;      // [n] first position whose time exceeds times[p] + H
    T H;                      // longest menu interval end
    // the alphas' chain lists: level >= 3, those of the previous level's
    // frequent episodes ([coff[alpha], coff[alpha + 1])); level 2, a frequent
    // type's own events (the per-type index as chain entries, s = t)
    const ChainEntry<T> *chain;
    const int64_t *cbeg;      // level >= 3: first entry of each alpha's chain list
    const int32_t *clen;      // level >= 3: its length
    const int32_t *type_off;
    const uint16_t *f1;       // level 2: the frequent types
    int32_t nf1;
    // one job per workgroup: an alpha, or (nseg > 1) one of nseg pieces of
    // an alpha's chain list (workgroup = job slot * nseg + piece)
    const int32_t *job_alpha; // alpha of each job (null: the job index)
    const int32_t *order;     // order in which the workgroups take the jobs (null: index order)
    int32_t nseg;
    // counting pass (level >= 3): alpha's extensions are the frequent
    // episodes beta = rlo..rlo+n of the previous level, skipping [xlo, xhi)
    const int64_t *out_off;   // [nA + 1] first candidate of each alpha
    const int32_t *rlo, *xlo, *xhi;
    const uint16_t *flast;    // last type of each frequent episode of the previous level
    const uint8_t *fliv;      // its last interval id
    int32_t *counts, *nvalid;
    unsigned long long *walked;  // stream positions walked, summed over the jobs
    // write pass: each job's range of the frequent list
    const int64_t *job_f;     // [njobs + 1]
    const uint16_t *w_type;
    const uint8_t *w_iv;
    const int64_t *w_off;     // first chain-list slot of each frequent episode
    ChainEntry<T> *wchain;
    // list pass: first slot of each (candidate, piece) list
    const int64_t *lst_off;   // [m * nseg + 1]
    T menu_lo[kExtMaxMenu], menu_hi[kExtMaxMenu];
    int32_t M;
    int32_t K;
    bool level2;              // alphas are frequent types (level 2)
};

// Read-only data seen through the constant address space: uniform reads of
// it become scalar loads (scalar cache) instead of vector loads.
template <typename T>
using const_ptr = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ __forceinline__ T read_lane(T v, int l) {
    if constexpr (sizeof(T) == 4) {
        return (T)__builtin_amdgcn_readlane((int)v, l);
    } else {
        const uint64_t u = (uint64_t)v;
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
        return (T)(((uint64_t)hi << 32) | lo);
    }
}

// An entry's (t, s) as one scalar load of both words.
template <typename T>
__device__ __forceinline__ void load_ts(const_ptr<ChainEntry<T>> e, T &t, T &s) {
    // (the entries are 4-byte aligned: the types say so)
    if constexpr (sizeof(T) == 4) {
        typedef uint64_t u64a4 __attribute__((aligned(4)));
        const uint64_t v = *(const_ptr<u64a4>)e;
        t = (T)(uint32_t)v;
        s = (T)(uint32_t)(v >> 32);
    } else {
        typedef unsigned u4 __attribute__((ext_vector_type(4), aligned(8)));
        const u4 v = *(const_ptr<u4>)e;
        t = (T)(((uint64_t)v.y << 32) | v.x);
        s = (T)(((uint64_t)v.w << 32) | v.z);
    }
}

// Walk kinds: count (greedy counts and end-event counts per candidate),
// write (chain lists of the frequent episodes), size (end events per
// candidate and piece), list (end events of every candidate, per piece), and
// size and list over the frequent extensions only (chain lists written by
// pieces).
enum WalkMode { kCount = 0, kWrite = 1, kSize = 2, kList = 3, kWSize = 4, kWList = 5 };

// walks over a write job's frequent extensions
template <int MODE>
constexpr bool kFreqJob = MODE == kWrite || MODE == kWSize || MODE == kWList;

// Extension r of a job: its new type B, interval id and key (count and size:
// the candidate's index; write: the first slot of its chain list).  Within a
// job the extensions are ordered by B.
template <typename T, int MODE>
__device__ __forceinline__ void extension(const WalkArgs<T> &a, int64_t job, int64_t alpha, int64_t r, int32_t &B,
                                          int &iv, int64_t &key) {
    if (kFreqJob<MODE>) {
        const int64_t f = a.job_f[job] + r;
        B = a.w_type[f];
        iv = a.w_iv[f];
        key = MODE == kWrite ? a.w_off[f] : f;
    } else if (a.level2) {
        const int64_t bi0 = r / a.M;
        iv = (int)(r - bi0 * a.M);
        const int64_t bi = bi0 >= alpha ? bi0 + 1 : bi0;
        B = a.f1[bi];
        key = alpha * (int64_t)(a.nf1 - 1) * a.M + r;
    } else {
        int64_t beta = a.rlo[alpha] + r;
        if (beta >= a.xlo[alpha]) beta += a.xhi[alpha] - a.xlo[alpha];
        B = a.flast[beta];
        iv = a.fliv[beta];
        key = a.out_off[alpha] + r;
    }
}

template <typename T, int MODE>
__device__ __forceinline__ int64_t n_extensions(const WalkArgs<T> &a, int64_t job, int64_t alpha) {
    if (kFreqJob<MODE>) return a.job_f[job + 1] - a.job_f[job];
    if (a.level2) return (int64_t)(a.nf1 - 1) * a.M;
    return a.out_off[alpha + 1] - a.out_off[alpha];
}

// A batch event in LDS: its time, its start per menu interval (minimum of
// the type: no occurrence ends there) and, counting, the next leader event of
// the same owner.  One record per event, so that a greedy step reads it with
// one address.
template <typename T, int MP>
struct alignas(16) EvRec {
    T t;
    T s[MP];
    int32_t n;
};

// One job: alpha (or a piece of its chain list) and all of its extensions
// (or, writing, its frequent ones).  MP greedy states per lane, one per menu
// interval: MP = M for menus of up to 4 intervals, else 8 with the unused
// states idle.
template <typename T, int MP, int MODE>
__global__ __launch_bounds__(kWave) void k_ext_walk(WalkArgs<T> a) {
    constexpr bool WRITE = MODE == kWrite || MODE == kList || MODE == kWList;
    constexpr T kMin = TsLimits<T>::lo();
    constexpr T kMax = TsLimits<T>::hi();
    constexpr bool kExact = MP <= 4;
    extern __shared__ uint16_t slot_of[];           // [K] owner lane of each type this round | its intervals << 8
    __shared__ unsigned long long want[kWave];      // batch lanes holding each owner's events
    __shared__ int32_t gtype[kWave];
    __shared__ int64_t gkey[MP][kWave];
    // the batch's events (slot 64: a null event that no greedy keeps; its
    // next leader, 64, is none)
    __shared__ EvRec<T, MP> evr[kWave + 1];
    // counting: each owner's end events per interval
    __shared__ int32_t cnv[MODE == kCount ? MP : 1][kWave];
    // writing: each owner's first slot and entries so far, per interval
    __shared__ int64_t okey[WRITE ? MP : 1][kWave];
    __shared__ int32_t onv[WRITE ? MP : 1][kWave];
    const int lane = threadIdx.x;
    const int64_t slot = (int64_t)blockIdx.x / a.nseg;
    const int32_t seg = (int32_t)((int64_t)blockIdx.x - slot * a.nseg);
    const int64_t job = a.order ? (int64_t)a.order[slot] : slot;
    const int64_t alpha = a.job_alpha ? (int64_t)a.job_alpha[job] : job;
    const int M = kExact ? MP : a.M;
    // alpha's chain list
    int64_t c0;
    int32_t clen;
    if (a.level2) {
        const int32_t ty = a.f1[alpha];
        c0 = a.type_off[ty];
        clen = a.type_off[ty + 1] - (int32_t)c0;
    } else {
        c0 = a.cbeg[alpha];
        clen = a.clen[alpha];
    }
    const_ptr<ChainEntry<T>> xc = (const_ptr<ChainEntry<T>>)(a.chain + c0);
    const ChainEntry<T> *xg = a.chain + c0;  // the same entries, read per lane
    // this job's piece of the chain list
    const int32_t e0 = (int32_t)((int64_t)clen * seg / a.nseg);
    const int32_t e1 = (int32_t)((int64_t)clen * (seg + 1) / a.nseg);
    // the menu, uniform
    T mlo[MP], mhi[MP];
#pragma unroll
    for (int m = 0; m < MP; ++m) {
        mlo[m] = a.menu_lo[m];
        mhi[m] = a.menu_hi[m];
    }
    const int64_t R = n_extensions<T, MODE>(a, job, alpha);
    for (int k = lane; k < a.K; k += kWave) slot_of[k] = kNoSlot;
    want[lane] = 0;
    if (lane == 0) {
        evr[kWave].t = kMin;
        evr[kWave].n = kWave;
#pragma unroll
        for (int m = 0; m < MP; ++m) evr[kWave].s[m] = kMin;
    }
    unsigned long long walked = 0;
    // rounds of up to 64 distinct extension types (one lane each)
    for (int64_t r_start = 0; r_start < R;) {
        gtype[lane] = -1;
#pragma unroll
        for (int m = 0; m < MP; ++m) gkey[m][lane] = -1;
        __syncthreads();
        int32_t ng = 0, prevB = -1;
        int64_t r_next = R;
        for (int64_t rb = r_start; rb < R; rb += kWave) {  // uniform
            const int64_t r = rb + lane;
            const bool in = r < R;
            int32_t B = -1;
            int iv = 0;
            int64_t key = -1;
            if (in) {
                extension<T, MODE>(a, job, alpha, r, B, iv, key);
                if (MODE == kSize || MODE == kWSize) key = key * a.nseg + seg;
                if (MODE == kList || MODE == kWList) key = a.lst_off[key * a.nseg + seg];
            }
            int32_t pB = __shfl_up(B, 1, kWave);
            if (lane == 0) pB = prevB;
            const uint64_t st = __ballot(in && B != pB);
            const int32_t g = ng + __popcll(st & (~0ull >> (63 - lane))) - 1;
            if (in && g < kWave) {
                gtype[g] = B;
                gkey[iv][g] = key;
            }
            const uint64_t over = __ballot(in && g >= kWave);
            if (over) {
                r_next = rb + __builtin_ctzll(over);
                ng = kWave;
                break;
            }
            ng += __popcll(st);
            prevB = __shfl(B, 63 - __builtin_clzll(__ballot(in)), kWave);
        }
        __syncthreads();
        const bool has = lane < ng;
        const int32_t myB = has ? gtype[lane] : -1;
        int64_t key[MP];
        bool own[MP];
        T pe[MP];
        int32_t cnt[MP], nv[MP];
#pragma unroll
        for (int m = 0; m < MP; ++m) {
            key[m] = has ? gkey[m][lane] : -1;
            own[m] = key[m] >= 0;
            pe[m] = own[m] ? kMin : kMax;  // an interval the lane does not count keeps nothing
            cnt[m] = 0;
            nv[m] = 0;
        }
        uint32_t ownm = 0;
#pragma unroll
        for (int m = 0; m < MP; ++m) ownm |= (uint32_t)own[m] << m;
        if (has) slot_of[myB] = (uint16_t)(lane | ownm << 8);
        if (WRITE) {
#pragma unroll
            for (int m = 0; m < MP; ++m) {
                okey[m][lane] = key[m];
                onv[m][lane] = 0;
            }
        }
        if (MODE == kCount) {
#pragma unroll
            for (int m = 0; m < MP; ++m) cnv[m][lane] = 0;
        }
        __syncthreads();
        // ---- the walk over U(alpha) (this piece: the runs of entries e0..e1-1)
        int32_t carry = e0 > 0 ? a.wend[xc[e0 - 1].p] : 0;  // coverage end of the entries already taken
        int32_t ilo = e0;  // first entry that can still be a predecessor
        if (e0 < e1) {
            const T t0 = xc[e0].t;
            while (ilo > 0 && xc[ilo - 1].t >= (T)(t0 - a.H)) --ilo;
        }
        for (int32_t i0 = e0; i0 < e1; i0 += kWave) {  // uniform
            const int32_t i = i0 + lane;
            const bool ci = i < e1;
            const int32_t p = ci ? xc[i].p : 0;
            const int32_t e = ci ? a.wend[p] : 0;
            int32_t prev_e = __shfl_up(e, 1, kWave);
            if (lane == 0) prev_e = carry;
            const int32_t beg = max(p + 1, prev_e);
            const int32_t len = ci ? max(0, e - beg) : 0;
            int32_t S = len;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const int32_t y = __shfl_up(S, d, kWave);
                if (lane >= d) S += y;
            }
            const int32_t X = S - len;
            const int32_t total = __builtin_amdgcn_readlane(S, 63);
            carry = max(carry, __builtin_amdgcn_readlane(e, 63 - __builtin_clzll(__ballot(ci))));
            walked += (unsigned long long)total;
            // stream position of this lane in the batch at b: the runs
            // meeting [b, b + 64) are visited in order
            auto position = [&](int32_t b) -> int32_t {
                const int32_t o = b + lane;
                uint64_t runs = __ballot(len > 0 && X < b + kWave && S > b);
                int32_t P = 0;
                while (runs) {
                    const int j = __builtin_ctzll(runs);
                    runs &= runs - 1;
                    const int32_t Xj = __builtin_amdgcn_readlane(X, j);
                    const int32_t bj = __builtin_amdgcn_readlane(beg, j);
                    if (o >= Xj) P = bj + (o - Xj);
                }
                return P;
            };
            // the next batch's events are loaded before this batch is
            // processed (its loads then wait behind this batch's work)
            int32_t Pn = 0, tyn = 0;
            T tn = kMax;
            if (total > 0) {
                Pn = position(0);
                if (lane < total) {
                    tyn = (int32_t)a.ty16[Pn];
                    tn = a.times[Pn];
                }
            }
            for (int32_t b = 0; b < total; b += kWave) {  // uniform
                const int32_t o = b + lane;
                const bool ev = o < total;
                const int32_t P = Pn;
                const int32_t ty = tyn;
                const T t = tn;
                if (b + kWave < total) {  // uniform
                    Pn = position(b + kWave);
                    tyn = 0;
                    tn = kMax;
                    if (o + kWave < total) {
                        tyn = (int32_t)a.ty16[Pn];
                        tn = a.times[Pn];
                    }
                }
                const int nb = min(total - b, kWave);
                const T tf = read_lane(t, 0), tl = read_lane(t, nb - 1);
                // s_m(y): start of the latest end event x with
                // t_x < t - lo_m, when t_x >= t - hi_m
                while (ilo < clen && xc[ilo].t < (T)(tf - a.H)) ++ilo;  // (entries past e1 can precede too)
                T cx[MP], cxs[MP];
#pragma unroll
                for (int m = 0; m < MP; ++m) {
                    cx[m] = kMin;
                    cxs[m] = kMin;
                }
                for (int32_t q = ilo; q < clen; ++q) {  // uniform
                    // (t, s) in one load: one wait per entry
                    T qt, qs;
                    load_ts(xc + q, qt, qs);
                    if (qt >= tl) break;
#pragma unroll
                    for (int m = 0; m < MP; ++m) {
                        const bool c = (T)(qt + mlo[m]) < t;
                        cx[m] = c ? qt : cx[m];
                        cxs[m] = c ? qs : cxs[m];
                    }
                }
                T sv[MP];
                uint32_t vm = 0;  // menu intervals for which this event ends an occurrence
#pragma unroll
                for (int m = 0; m < MP; ++m) {
                    // bitwise, not short-circuit: keeps the code branch-free
                    const uint32_t v = (uint32_t)(kExact || m < M) & (uint32_t)ev &
                                       (uint32_t)(cx[m] != kMin) & (uint32_t)((T)(cx[m] + mhi[m]) >= t);
                    sv[m] = v ? cxs[m] : kMin;
                    vm |= v << m;
                }
                // the event in LDS, for its owner and its same-type neighbours
                evr[lane].t = t;
#pragma unroll
                for (int m = 0; m < MP; ++m) evr[lane].s[m] = sv[m];
                // delivered to the owner of its type when that owner counts
                // one of those intervals
                const uint32_t sl = vm ? (uint32_t)slot_of[ty] : 0u;
                const bool dl = (vm & (sl >> 8)) != 0;
                const int ow = (int)(sl & 0xFF);
                if (dl) atomicOr(&want[ow], 1ull << lane);
                uint64_t vb[MP];  // delivered events that end an occurrence, per interval
                if (MODE == kCount) {
                    // counted by the events themselves, for the intervals
                    // their owner counts
                    const uint32_t dv = dl ? vm & (sl >> 8) : 0u;
#pragma unroll
                    for (int m = 0; m < MP; ++m)
                        if ((dv >> m) & 1u) atomicAdd(&cnv[m][ow], 1);
                } else {
#pragma unroll
                    for (int m = 0; m < MP; ++m) vb[m] = __ballot(dl & (sv[m] != kMin));
                }
                __syncthreads();
                const uint64_t below = (1ull << lane) - 1ull;
                const uint64_t wo = dl ? want[ow] : 0ull;  // the batch's events of the same owner
                uint64_t lb = 0;
                if (MODE == kCount) {
                    // leaders: events whose s_m differs from that of the
                    // previous same-owner event; the others can never be kept
                    // (an earlier event with the same start was kept or
                    // rejected first)
                    uint32_t lead = 0;
                    const uint64_t bm = wo & below;
                    if (bm == 0) {
                        lead = vm;
                    } else {
                        const int pl = 63 - __builtin_clzll(bm);
#pragma unroll
                        for (int m = 0; m < MP; ++m)
                            lead |= (uint32_t)((sv[m] != kMin) & (sv[m] != evr[pl].s[m])) << m;
                    }
                    lb = __ballot(dl & ((lead & (sl >> 8)) != 0));
                    // the owner's leaders as a list in time order
                    const uint64_t nx = wo & lb & ~((2ull << lane) - 1ull);
                    evr[lane].n = nx ? __builtin_ctzll(nx) : kWave;
                }
                if (WRITE && dl) {
                    // each event writes itself, after the owner's entries so
                    // far and the batch's earlier ones
#pragma unroll
                    for (int m = 0; m < MP; ++m) {
                        if ((sv[m] != kMin) & (((sl >> 8) >> m) & 1u)) {
                            const int64_t w = okey[m][ow] + onv[m][ow] + __popcll(wo & vb[m] & below);
                            a.wchain[w] = ChainEntry<T>{t, sv[m], P};
                        }
                    }
                }
                __syncthreads();  // every read of want and of the owners' published counts is done
                uint64_t wm = want[lane];
                want[lane] = 0;
                if (MODE != kCount) {
#pragma unroll
                    for (int m = 0; m < MP; ++m) nv[m] += __popcll(wm & vb[m]);
                }
                if (WRITE) {
#pragma unroll
                    for (int m = 0; m < MP; ++m) onv[m][lane] = nv[m];
                }
                if (MODE == kCount) {
                    // each owner lane runs its greedies over its leaders in
                    // time order, following the list; lanes with none left
                    // read the null event
                    const uint64_t wl = wm & lb;
                    int k = wl ? __builtin_ctzll(wl) : kWave;
                    if (__ballot(k < kWave)) do {  // uniform
                        const EvRec<T, MP> y = evr[k];
#pragma unroll
                        for (int m = 0; m < MP; ++m) {
                            const bool g = y.s[m] > pe[m];
                            unsigned co;  // (an add with carry-in: no select of 0 or 1)
                            cnt[m] = (int32_t)__builtin_addc((unsigned)cnt[m], 0u, (unsigned)g, &co);
                            pe[m] = g ? y.t : pe[m];
                        }
                        k = y.n;
                    } while (__ballot(k < kWave));
                }
            }
        }
        if (MODE == kCount) {
#pragma unroll
            for (int m = 0; m < MP; ++m) nv[m] = cnv[m][lane];
        }
        if (MODE == kCount || MODE == kSize || MODE == kWSize) {
#pragma unroll
            for (int m = 0; m < MP; ++m) {
                if (own[m]) {
                    if (MODE == kCount) a.counts[key[m]] = cnt[m];
                    a.nvalid[key[m]] = nv[m];
                }
            }
        }
        if (has) slot_of[myB] = kNoSlot;
        __syncthreads();
        r_start = r_next;
    }
    if ((MODE == kCount || MODE == kSize) && a.walked && lane == 0) atomicAdd(a.walked, walked);
}

// Every array a walk of this kind reads or writes must be present.
template <typename T, int MODE>
bool walk_args_complete(const WalkArgs<T> &a) {
    bool ok = a.ty16 && a.times && a.wend && a.M >= 1 && a.M <= kExtMaxMenu && a.K >= 1 && a.nseg >= 1;
    ok = ok && a.chain;
    if (a.level2) ok = ok && a.f1 && a.type_off && a.nf1 >= 2;
    else ok = ok && a.cbeg && a.clen;
    if (kFreqJob<MODE>) ok = ok && a.job_alpha && a.job_f && a.w_type && a.w_iv;
    else ok = ok && (a.level2 || (a.out_off && a.rlo && a.xlo && a.xhi && a.flast && a.fliv));
    if (MODE == kWrite) ok = ok && a.w_off && a.wchain;
    if (MODE == kCount) ok = ok && a.counts && a.nvalid;
    if (MODE == kSize || MODE == kWSize) ok = ok && a.nvalid;
    if (MODE == kList || MODE == kWList) ok = ok && a.lst_off && a.wchain;
    if (MODE == kWrite || MODE == kCount) ok = ok && a.nseg == 1;
    return ok;
}

// njobs workgroups (jobs times pieces).
template <typename T, int MODE>
hipError_t launch_walk(const WalkArgs<T> &a, int64_t njobs, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    if (!walk_args_complete<T, MODE>(a)) return hipErrorInvalidValue;
    const size_t lds = (size_t)(2 * a.K + 15) / 16 * 16;
    const unsigned g = (unsigned)njobs;
    switch (a.M) {
        case 1: k_ext_walk<T, 1, MODE><<<g, kWave, lds, st>>>(a); break;
        case 2: k_ext_walk<T, 2, MODE><<<g, kWave, lds, st>>>(a); break;
        case 3: k_ext_walk<T, 3, MODE><<<g, kWave, lds, st>>>(a); break;
        case 4: k_ext_walk<T, 4, MODE><<<g, kWave, lds, st>>>(a); break;
        default: k_ext_walk<T, 8, MODE><<<g, kWave, lds, st>>>(a); break;
    }
    return hipGetLastError();
}

// The per-type index as chain entries (the chain lists of 1-node episodes).
template <typename T>
__global__ void k_type_chain(const T *__restrict__ ts, const int32_t *__restrict__ pos, int64_t n,
                             ChainEntry<T> *__restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) out[q] = ChainEntry<T>{ts[q], ts[q], pos[q]};
}

// Types as uint16 and the window end of every position.
template <typename T>
__global__ void k_walk_prep(const int32_t *__restrict__ types, const T *__restrict__ times, int64_t n, T H,
                            uint16_t *__restrict__ ty16, int32_t *__restrict__ wend) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ty16[i] = (uint16_t)types[i];
    const T lim = (T)(times[i] + H);
    int64_t lo = i + 1, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (times[mid] <= lim) lo = mid + 1;
        else hi = mid;
    }
    wend[i] = (int32_t)lo;
}

// ---- device-side bookkeeping of the levels ----------------------------------

constexpr int kBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

// Block-wide exclusive scan of one int64 per thread.
__device__ __forceinline__ int64_t block_scan64(int64_t v, int64_t *total) {
    __shared__ int64_t wsum[kBlock / kWave];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    int64_t x = v;
    for (int d = 1; d < kWave; d <<= 1) {
        const int64_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    int64_t off = 0, tot = 0;
    for (int k = 0; k < kBlock / kWave; ++k) {
        if (k < w) off += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

// Exclusive scan of in[len] into int64 out[len + 1] (out[len] = total), in
// three passes: tile sums, a one-block scan of the tile sums, tile scans.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_scan_tiles(const V *__restrict__ in, int64_t len,
                                                       int64_t *__restrict__ sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t acc = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        if (i < len) acc += (int64_t)in[i];
    }
    int64_t tot;
    (void)block_scan64(acc, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_sums64(int64_t *__restrict__ sums, int64_t nb) {
    int64_t carry = 0;
    for (int64_t r = 0; r < nb; r += kBlock) {
        const int64_t i = r + threadIdx.x;
        const int64_t v = i < nb ? sums[i] : 0;
        int64_t tot;
        const int64_t ex = block_scan64(v, &tot);
        if (i < nb) sums[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_scan_apply64(const V *__restrict__ in, int64_t len,
                                                         const int64_t *__restrict__ sums, int64_t nb,
                                                         int64_t *__restrict__ out) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t v[kScanItems];
    int64_t acc = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        v[k] = i < len ? (int64_t)in[i] : 0;
        acc += v[k];
    }
    int64_t tot;
    int64_t run = block_scan64(acc, &tot) + sums[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        if (i < len) out[i] = run;
        run += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[len] = sums[nb];
}

// out[len + 1] = exclusive scan of in[len]; the total is left in out[len].
template <typename V>
hipError_t scan64(const V *in, int64_t len, int64_t *out, DevBuf &tmp, hipStream_t st) {
    const int64_t nb = len > 0 ? (len + kScanTile - 1) / kScanTile : 1;
    hipError_t e;
    if ((e = tmp.alloc(sizeof(int64_t) * (nb + 1))) != hipSuccess) return e;
    k_scan_tiles<V><<<(unsigned)nb, kBlock, 0, st>>>(in, len, tmp.as<int64_t>());
    k_scan_sums64<<<1, kBlock, 0, st>>>(tmp.as<int64_t>(), nb);
    k_scan_apply64<V><<<(unsigned)nb, kBlock, 0, st>>>(in, len, tmp.as<int64_t>(), nb, out);
    return hipGetLastError();
}

// Frequent selection (count > threshold), order preserving: per-block flag
// counts, their scan, then each block writes its candidates at its offset.
constexpr int kSelItems = 8;
constexpr int kSelTile = kBlock * kSelItems;

__global__ __launch_bounds__(kBlock) void k_sel_count(const int32_t *__restrict__ counts, int64_t m, int32_t thr,
                                                      int32_t *__restrict__ bcnt) {
    __shared__ int32_t red[kBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kSelTile;
    int32_t c = 0;
    for (int k = 0; k < kSelItems; ++k) {
        const int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
        if (i < m && counts[i] > thr) ++c;
    }
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, kWave);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < kBlock / kWave; ++w) t += red[w];
        bcnt[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_sel_write(const int32_t *__restrict__ counts,
                                                      const int32_t *__restrict__ nvalid, int64_t m, int32_t thr,
                                                      const int64_t *__restrict__ boff, int64_t *__restrict__ fcand,
                                                      int32_t *__restrict__ fnv) {
    __shared__ int32_t wsum[kBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kSelTile;
    int64_t off = boff[blockIdx.x];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = 0; k < kSelItems; ++k) {  // uniform
        const int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
        const bool f = i < m && counts[i] > thr;
        const uint64_t bal = __ballot(f);
        if (lane == 0) wsum[w] = __popcll(bal);
        __syncthreads();
        int32_t before = 0, total = 0;
        for (int q = 0; q < kBlock / kWave; ++q) {
            if (q < w) before += wsum[q];
            total += wsum[q];
        }
        if (f) {
            const int64_t o = off + before + __popcll(bal & ((1ull << lane) - 1ull));
            fcand[o] = i;
            fnv[o] = nvalid[i];
        }
        off += total;
        __syncthreads();
    }
}

// Level 1: distinct timestamps of each type, one wave per type.
template <typename T>
__global__ __launch_bounds__(kWave) void k_level1(const T *__restrict__ ts, const int32_t *__restrict__ type_off,
                                                  int32_t *__restrict__ counts) {
    const int k = blockIdx.x;
    const int lane = threadIdx.x;
    const int32_t b = type_off[k], e = type_off[k + 1];
    int32_t c = 0;
    for (int32_t i = b + lane; i < e; i += kWave) c += (i == b || ts[i] != ts[i - 1]) ? 1 : 0;
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, kWave);
    if (lane == 0) counts[k] = c;
}

// Apriori join on the device.  Every frequent episode of level N-1 >= 2
// records its prefix parent fpar (the episode of level N-2 it extends) and its
// suffix parent fsuf (the frequent episode of level N-2 equal to its last N-2
// nodes: the join took its last node from it).  The candidates of level N
// are alpha + last(beta) for frequent alpha, beta of level N-1 with
// fpar[beta] == fsuf[alpha] and a new type other than alpha's first.  The
// frequent list is in candidate order, hence sorted by fpar and, within one
// parent, by (last type, interval): the betas of one parent are a contiguous
// bucket, sorted by last type.
//
// Bucket offsets: boff[p] = first f with fpar[f] >= p, p = 0..np.
__global__ __launch_bounds__(kBlock) void k_bucket_off(const int32_t *__restrict__ fpar, int64_t nf, int64_t np,
                                                       int32_t *__restrict__ boff) {
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f > nf) return;
    const int64_t prev = f == 0 ? -1 : fpar[f - 1];
    const int64_t cur = f == nf ? np : fpar[f];
    for (int64_t p = prev + 1; p <= cur; ++p) boff[p] = (int32_t)f;
}

// Per alpha: its bucket [rlo, rhi) of betas, the run [xlo, xhi) of betas whose
// last type is alpha's first type (excluded), and its number of candidates.
__global__ __launch_bounds__(kBlock) void k_join(const int32_t *__restrict__ fsuf, const uint16_t *__restrict__ ffirst,
                                                 const uint16_t *__restrict__ flast, const int32_t *__restrict__ boff,
                                                 int64_t nA, int32_t *__restrict__ rlo, int32_t *__restrict__ xlo,
                                                 int32_t *__restrict__ xhi, int64_t *__restrict__ cnt) {
    const int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (a >= nA) return;
    const int32_t p = fsuf[a];
    const int32_t lo = boff[p], hi = boff[p + 1];
    const uint16_t first = ffirst[a];
    int32_t l = lo, h = hi;
    while (l < h) {
        const int32_t mid = (l + h) >> 1;
        if (flast[mid] < first) l = mid + 1;
        else h = mid;
    }
    const int32_t xl = l;
    h = hi;
    while (l < h) {
        const int32_t mid = (l + h) >> 1;
        if (flast[mid] <= first) l = mid + 1;
        else h = mid;
    }
    rlo[a] = lo;
    xlo[a] = xl;
    xhi[a] = l;
    cnt[a] = (int64_t)(hi - lo) - (l - xl);
}

// Fields of each frequent episode of level N from its candidate index.
struct FreqArgs {
    int64_t nf;
    const int64_t *fcand;
    bool level2;
    int64_t per;                 // level 2: candidates per alpha ((nf1 - 1) * M)
    int32_t M;
    const int64_t *out_off;      // level >= 3: [nA + 1]
    int64_t nA;
    const int32_t *rlo, *xlo, *xhi;
    const uint16_t *pflast;      // level N-1: last type (level 1: the type)
    const uint8_t *pfliv;        // level N-1: last interval id
    const uint16_t *pffirst;     // level N-1: first type
    int32_t *fpar, *fsuf;
    uint16_t *flast, *ffirst;
    uint8_t *fliv;
};

__global__ __launch_bounds__(kBlock) void k_freq_fields(FreqArgs a) {
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f >= a.nf) return;
    const int64_t c = a.fcand[f];
    int64_t alpha, beta;
    uint16_t B;
    uint8_t iv;
    if (a.level2) {
        alpha = c / a.per;
        const int64_t r = c - alpha * a.per;
        const int64_t bi0 = r / a.M;
        iv = (uint8_t)(r - bi0 * a.M);
        beta = bi0 >= alpha ? bi0 + 1 : bi0;
        B = a.pflast[beta];
    } else {
        int64_t l = 0, h = a.nA;  // last alpha with out_off[alpha] <= c
        while (h - l > 1) {
            const int64_t mid = (l + h) >> 1;
            if (a.out_off[mid] <= c) l = mid;
            else h = mid;
        }
        alpha = l;
        int64_t rr = a.rlo[alpha] + (c - a.out_off[alpha]);
        if (rr >= a.xlo[alpha]) rr += a.xhi[alpha] - a.xlo[alpha];
        beta = rr;
        B = a.pflast[beta];
        iv = a.pfliv[beta];
    }
    a.fpar[f] = (int32_t)alpha;
    a.fsuf[f] = (int32_t)beta;
    a.flast[f] = B;
    a.fliv[f] = iv;
    a.ffirst[f] = a.pffirst[alpha];
}

// Write jobs: the alphas with frequent extensions (runs of equal fpar).
__global__ __launch_bounds__(kBlock) void k_job_flags(const int32_t *__restrict__ fpar, int64_t nf,
                                                      int32_t *__restrict__ flag) {
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f < nf) flag[f] = (f == 0 || fpar[f] != fpar[f - 1]) ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_job_write(const int32_t *__restrict__ fpar, const int32_t *__restrict__ flag,
                                                      const int64_t *__restrict__ jidx, int64_t nf,
                                                      int32_t *__restrict__ job_alpha, int64_t *__restrict__ job_f) {
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f > nf) return;
    if (f == nf) {
        job_f[jidx[nf]] = nf;
        return;
    }
    if (flag[f]) {
        job_alpha[jidx[f]] = fpar[f];
        job_f[jidx[f]] = f;
    }
}

// Length class of each job's alpha: leading zeros of its chain-list length,
// so that ordering by the key takes the longest walks first.
__global__ __launch_bounds__(kBlock) void k_len_key(const int32_t *__restrict__ clen, const int32_t *__restrict__ idx,
                                                    int64_t n, uint16_t *__restrict__ key) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const int32_t a = idx ? idx[j] : (int32_t)j;
    key[j] = (uint16_t)__clz((uint32_t)clen[a] | 1u);
}

// Jobs grouped by a uint16 key (the alphas' last type): a counting sort whose
// histogram is kept per block in LDS (kKeyItems jobs per block), so that a
// block adds each key once; the order inside a key is arbitrary.
constexpr int kKeyItems = 16;

__global__ __launch_bounds__(kBlock) void k_key_count(const uint16_t *__restrict__ key, const int32_t *__restrict__ idx,
                                                      int64_t n, int32_t K, int32_t *__restrict__ cnt) {
    extern __shared__ int32_t h[];
    for (int k = threadIdx.x; k < K; k += kBlock) h[k] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kBlock * kKeyItems;
    for (int q = 0; q < kKeyItems; ++q) {
        const int64_t j = base + (int64_t)q * kBlock + threadIdx.x;
        if (j < n) atomicAdd(&h[key[idx ? idx[j] : j]], 1);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += kBlock) cnt[(int64_t)k * gridDim.x + blockIdx.x] = h[k];
}

// off: exclusive scan of cnt in key-major order (key, block)
__global__ __launch_bounds__(kBlock) void k_key_place(const uint16_t *__restrict__ key, const int32_t *__restrict__ idx,
                                                      int64_t n, int32_t K, const int64_t *__restrict__ off,
                                                      int32_t *__restrict__ order) {
    extern __shared__ int32_t h[];
    for (int k = threadIdx.x; k < K; k += kBlock) h[k] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kBlock * kKeyItems;
    for (int q = 0; q < kKeyItems; ++q) {
        const int64_t j = base + (int64_t)q * kBlock + threadIdx.x;
        if (j < n) {
            const int32_t k = key[idx ? idx[j] : j];
            const int32_t r = atomicAdd(&h[k], 1);
            order[off[(int64_t)k * gridDim.x + blockIdx.x] + r] = (int32_t)j;
        }
    }
}

// List path: the count of candidate c is the greedy of Alg. 1 over its end
// events in time order (its lists of the nseg pieces, consecutive); one wave
// per candidate loads 64 entries at a time and the greedy steps through them
// in scalar registers.
template <typename T>
__global__ __launch_bounds__(kWave) void k_list_count(const ChainEntry<T> *__restrict__ lst,
                                                      const int64_t *__restrict__ lst_off, int32_t nseg,
                                                      int32_t *__restrict__ counts, int32_t *__restrict__ nvalid) {
    constexpr T kMin = TsLimits<T>::lo();
    const int64_t c = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t b = lst_off[c * nseg], e = lst_off[(c + 1) * nseg];
    T pe = kMin;
    int32_t cnt = 0;
    for (int64_t q0 = b; q0 < e; q0 += kWave) {  // uniform
        const int64_t q = q0 + lane;
        T t = kMin, s = kMin;
        if (q < e) {
            t = lst[q].t;
            s = lst[q].s;
        }
        const int nb = (int)(e - q0 < kWave ? e - q0 : kWave);
        for (int k = 0; k < nb; ++k) {
            const T sk = read_lane(s, k);
            if (sk > pe) {
                ++cnt;
                pe = read_lane(t, k);
            }
        }
    }
    if (lane == 0) {
        counts[c] = cnt;
        nvalid[c] = (int32_t)(e - b);
    }
}

// The same with one lane per candidate (many candidates).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_list_count_lane(const ChainEntry<T> *__restrict__ lst,
                                                            const int64_t *__restrict__ lst_off, int32_t nseg,
                                                            int64_t m, int32_t *__restrict__ counts,
                                                            int32_t *__restrict__ nvalid) {
    constexpr T kMin = TsLimits<T>::lo();
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= m) return;
    const int64_t b = lst_off[c * nseg], e = lst_off[(c + 1) * nseg];
    T pe = kMin;
    int32_t cnt = 0;
    int64_t q = b;
    for (; q + 4 <= e; q += 4) {
        ChainEntry<T> v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = lst[q + u];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (v[u].s > pe) {
                ++cnt;
                pe = v[u].t;
            }
        }
    }
    for (; q < e; ++q) {
        const ChainEntry<T> v = lst[q];
        if (v.s > pe) {
            ++cnt;
            pe = v.t;
        }
    }
    counts[c] = cnt;
    nvalid[c] = (int32_t)(e - b);
}

// List path: the chain list of frequent episode f is its candidate's list.
__global__ __launch_bounds__(kBlock) void k_list_begin(const int64_t *__restrict__ fcand,
                                                       const int64_t *__restrict__ lst_off, int32_t nseg, int64_t nf,
                                                       int64_t *__restrict__ cbeg) {
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f < nf) cbeg[f] = lst_off[fcand[f] * nseg];
}

unsigned grid_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <typename V>
hipError_t read_scalar(const DevBuf &b, int64_t at, V *out, hipStream_t st) {
    hipError_t e = hipMemcpyAsync(out, b.as<V>() + at, sizeof(V), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

// jobs j = 0..n-1 ordered by key[idx[j]] (idx null: key[j]), key < K
hipError_t order_by_key(const uint16_t *key, const int32_t *idx, int64_t n, int32_t K, DevBuf &order,
                        hipStream_t st) {
    hipError_t e;
    if ((e = order.alloc(sizeof(int32_t) * std::max<int64_t>(1, n))) != hipSuccess) return e;
    if (n == 0) return hipSuccess;
    const int64_t nb = (n + kBlock * kKeyItems - 1) / (kBlock * kKeyItems);
    DevBuf cnt, off, tmp;
    if ((e = cnt.alloc(sizeof(int32_t) * nb * K)) != hipSuccess) return e;
    if ((e = off.alloc(sizeof(int64_t) * (nb * K + 1))) != hipSuccess) return e;
    const size_t lds = sizeof(int32_t) * (size_t)K;
    k_key_count<<<(unsigned)nb, kBlock, lds, st>>>(key, idx, n, K, cnt.as<int32_t>());
    if ((e = scan64(cnt.as<int32_t>(), nb * K, off.as<int64_t>(), tmp, st)) != hipSuccess) return e;
    k_key_place<<<(unsigned)nb, kBlock, lds, st>>>(key, idx, n, K, off.as<int64_t>(), order.as<int32_t>());
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the temporaries die here: blocks of a cache scope go back for later
    // work of this stream, others are freed after it
    return CacheScope::current() ? hipGetLastError() : hipStreamSynchronize(st);
}

template <typename T>
hipError_t level_t(const Stream &s, Mine &mn, int N, hipStream_t st) {
    hipError_t e;
    if (!mn.stage) return hipErrorInvalidValue;
    MineLevel &P = mn.levels.back();  // level N-1
    MineLevel L;
    L.N = N;
    L.implicit = true;
    const int M = (int)mn.menu_lo.size();
    auto t0 = Clock::now();
    const int64_t nA = P.nf;
    L.nA = nA;
    // ---- the candidates: alpha-major, alpha's extensions in (type, interval) order
    int64_t m;
    DevBuf d_order, tmp;
    if (N == 2) {
        m = nA * (nA - 1) * M;
    } else {
        const MineLevel &PP = mn.levels[mn.levels.size() - 2];  // level N-2
        DevBuf boff, cnt;
        if ((e = boff.alloc(sizeof(int32_t) * (PP.nf + 1))) != hipSuccess) return e;
        if ((e = cnt.alloc(sizeof(int64_t) * std::max<int64_t>(1, nA))) != hipSuccess) return e;
        if ((e = L.d_rlo.alloc(sizeof(int32_t) * nA)) != hipSuccess) return e;
        if ((e = L.d_xlo.alloc(sizeof(int32_t) * nA)) != hipSuccess) return e;
        if ((e = L.d_xhi.alloc(sizeof(int32_t) * nA)) != hipSuccess) return e;
        if ((e = L.d_out_off.alloc(sizeof(int64_t) * (nA + 1))) != hipSuccess) return e;
        k_bucket_off<<<grid_of(nA + 1), kBlock, 0, st>>>(P.d_fpar.as<int32_t>(), nA, PP.nf, boff.as<int32_t>());
        k_join<<<grid_of(nA), kBlock, 0, st>>>(P.d_fsuf.as<int32_t>(), P.d_ffirst.as<uint16_t>(),
                                               P.d_flast.as<uint16_t>(), boff.as<int32_t>(), nA,
                                               L.d_rlo.as<int32_t>(), L.d_xlo.as<int32_t>(), L.d_xhi.as<int32_t>(),
                                               cnt.as<int64_t>());
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = scan64(cnt.as<int64_t>(), nA, L.d_out_off.as<int64_t>(), tmp, st)) != hipSuccess) return e;
        if ((e = read_scalar(L.d_out_off, nA, &m, st)) != hipSuccess) return e;
        // workgroups take the alphas grouped by their last type: the waves in
        // flight then walk the neighbourhoods of the same type's events
        {
            DevBuf lkey;
            if ((e = lkey.alloc(sizeof(uint16_t) * std::max<int64_t>(1, nA))) != hipSuccess) return e;
            k_len_key<<<grid_of(nA), kBlock, 0, st>>>(P.d_fnv.as<int32_t>(), nullptr, nA, lkey.as<uint16_t>());
            if ((e = order_by_key(lkey.as<uint16_t>(), nullptr, nA, 33, d_order, st)) != hipSuccess) return e;
        }
    }
    L.m = m;
    WalkArgs<T> a{};
    a.ty16 = mn.ty16.as<uint16_t>();
    a.times = s.times.as<T>();
    a.wend = mn.wend.as<int32_t>();
    a.H = (T)*std::max_element(mn.menu_hi.begin(), mn.menu_hi.end());
    a.chain = mn.chain1.as<ChainEntry<T>>();  // level 2; level >= 3 below
    a.type_off = s.type_off.as<int32_t>();
    a.M = M;
    a.K = s.K;
    a.level2 = N == 2;
    for (int i = 0; i < M; ++i) {
        a.menu_lo[i] = (T)mn.menu_lo[i];
        a.menu_hi[i] = (T)mn.menu_hi[i];
    }
    a.f1 = P.d_flast.as<uint16_t>();  // level 2: the frequent types
    a.nf1 = (int32_t)nA;
    a.nseg = 1;
    if (N > 2) {
        a.chain = P.chain.as<ChainEntry<T>>();
        a.cbeg = P.cbeg.as<int64_t>();
        a.clen = P.d_fnv.as<int32_t>();
        a.flast = P.d_flast.as<uint16_t>();
        a.fliv = P.d_fliv.as<uint8_t>();
        a.out_off = L.d_out_off.as<int64_t>();
        a.rlo = L.d_rlo.as<int32_t>();
        a.xlo = L.d_xlo.as<int32_t>();
        a.xhi = L.d_xhi.as<int32_t>();
        a.order = d_order.as<int32_t>();
    }
    DevBuf d_nval, d_walked;
    if ((e = L.dcounts.alloc(sizeof(int32_t) * m)) != hipSuccess) return e;
    if ((e = d_nval.alloc(sizeof(int32_t) * m)) != hipSuccess) return e;
    if ((e = d_walked.alloc(sizeof(unsigned long long))) != hipSuccess) return e;
    if ((e = hipMemsetAsync(d_walked.p, 0, sizeof(unsigned long long), st)) != hipSuccess) return e;
    a.counts = L.dcounts.as<int32_t>();
    a.nvalid = d_nval.as<int32_t>();
    a.walked = d_walked.as<unsigned long long>();
    L.gen_ms = ms_since(t0);
    auto t1 = Clock::now();
    // ---- count
    hipEvent_t ev0, ev1;
    if ((e = hipEventCreate(&ev0)) != hipSuccess) return e;
    if ((e = hipEventCreate(&ev1)) != hipSuccess) return e;
    (void)hipEventRecord(ev0, st);
    // With few alphas (level 2 has as many as frequent types) one walk per
    // alpha leaves the GPU idle: the walks are cut into pieces and every
    // candidate's end events are listed (list path), when they fit the budget.
    bool listed = false;
    DevBuf lst_off;
    if (m > 0 && nA < mn.list_alphas) {
        const int32_t nseg = (int32_t)std::max<int64_t>(1, std::min<int64_t>(64, (kListJobs + nA - 1) / nA));
        if ((e = lst_off.alloc(sizeof(int64_t) * (m * nseg + 1))) != hipSuccess) return e;
        DevBuf nvseg;
        if ((e = nvseg.alloc(sizeof(int32_t) * m * nseg)) != hipSuccess) return e;
        WalkArgs<T> b = a;
        b.nseg = nseg;
        b.nvalid = nvseg.as<int32_t>();
        if ((e = launch_walk<T, kSize>(b, nA * nseg, st)) != hipSuccess) return e;
        if ((e = scan64(nvseg.as<int32_t>(), m * nseg, lst_off.as<int64_t>(), tmp, st)) != hipSuccess) return e;
        int64_t total = 0;
        if ((e = read_scalar(lst_off, m * nseg, &total, st)) != hipSuccess) return e;
        if (total * (int64_t)sizeof(ChainEntry<T>) <= mn.list_budget) {
            if ((e = L.chain.alloc(sizeof(ChainEntry<T>) * (size_t)total)) != hipSuccess) return e;
            b.lst_off = lst_off.as<int64_t>();
            b.wchain = L.chain.as<ChainEntry<T>>();
            if ((e = launch_walk<T, kList>(b, nA * nseg, st)) != hipSuccess) return e;
            if (m < kListJobs)
                k_list_count<T><<<(unsigned)m, kWave, 0, st>>>(L.chain.as<ChainEntry<T>>(), lst_off.as<int64_t>(),
                                                              nseg, a.counts, a.nvalid);
            else
                k_list_count_lane<T><<<grid_of(m), kBlock, 0, st>>>(L.chain.as<ChainEntry<T>>(), lst_off.as<int64_t>(),
                                                                   nseg, m, a.counts, a.nvalid);
            e = hipGetLastError();
            listed = true;
            L.list_seg = nseg;
        }
    }
    if (m > 0 && !listed && e == hipSuccess) e = launch_walk<T, kCount>(a, nA, st);
    (void)hipEventRecord(ev1, st);
    // the walked positions and the number of frequent episodes reach the host
    // at one synchronisation (pinned slots 0 and 1)
    int64_t *stage = mn.stage;
    if (e == hipSuccess) e = hipMemcpyAsync(&stage[0], d_walked.p, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    // ---- frequent episodes, selected on the device
    const int64_t nb = m > 0 ? (m + kSelTile - 1) / kSelTile : 0;
    int64_t nf = 0;
    DevBuf bcnt, boffs;
    if (e == hipSuccess) e = bcnt.alloc(sizeof(int32_t) * std::max<int64_t>(1, nb));
    if (e == hipSuccess) e = boffs.alloc(sizeof(int64_t) * (nb + 1));
    const int32_t thr = (int32_t)std::max<int64_t>(INT32_MIN, std::min<int64_t>(mn.threshold, INT32_MAX));
    if (nb > 0 && e == hipSuccess) {
        k_sel_count<<<(unsigned)nb, kBlock, 0, st>>>(a.counts, m, thr, bcnt.as<int32_t>());
        e = hipGetLastError();
        if (e == hipSuccess) e = scan64(bcnt.as<int32_t>(), nb, boffs.as<int64_t>(), tmp, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&stage[1], boffs.as<int64_t>() + nb, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    float kms = 0;
    if (e == hipSuccess) (void)hipEventElapsedTime(&kms, ev0, ev1);
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (e != hipSuccess) return e;
    L.kernel_ms = kms;
    L.walked = stage[0];
    if (nb > 0) nf = stage[1];
    L.nf = nf;
    const size_t nfa = (size_t)std::max<int64_t>(1, nf);
    if ((e = L.d_fcand.alloc(sizeof(int64_t) * nfa)) != hipSuccess) return e;
    if ((e = L.d_fnv.alloc(sizeof(int32_t) * nfa)) != hipSuccess) return e;
    if ((e = L.d_fpar.alloc(sizeof(int32_t) * nfa)) != hipSuccess) return e;
    if ((e = L.d_fsuf.alloc(sizeof(int32_t) * nfa)) != hipSuccess) return e;
    if ((e = L.d_flast.alloc(sizeof(uint16_t) * nfa)) != hipSuccess) return e;
    if ((e = L.d_ffirst.alloc(sizeof(uint16_t) * nfa)) != hipSuccess) return e;
    if ((e = L.d_fliv.alloc(nfa)) != hipSuccess) return e;
    if ((e = L.cbeg.alloc(sizeof(int64_t) * (nf + 1))) != hipSuccess) return e;
    L.chain_total = 0;
    if (nf > 0) {
        k_sel_write<<<(unsigned)nb, kBlock, 0, st>>>(a.counts, a.nvalid, m, thr, boffs.as<int64_t>(),
                                                    L.d_fcand.as<int64_t>(), L.d_fnv.as<int32_t>());
        FreqArgs fa{};
        fa.nf = nf;
        fa.fcand = L.d_fcand.as<int64_t>();
        fa.level2 = N == 2;
        fa.per = (nA - 1) * M;
        fa.M = M;
        fa.out_off = L.d_out_off.as<int64_t>();
        fa.nA = nA;
        fa.rlo = L.d_rlo.as<int32_t>();
        fa.xlo = L.d_xlo.as<int32_t>();
        fa.xhi = L.d_xhi.as<int32_t>();
        fa.pflast = P.d_flast.as<uint16_t>();
        fa.pfliv = P.d_fliv.as<uint8_t>();
        fa.pffirst = P.d_ffirst.as<uint16_t>();
        fa.fpar = L.d_fpar.as<int32_t>();
        fa.fsuf = L.d_fsuf.as<int32_t>();
        fa.flast = L.d_flast.as<uint16_t>();
        fa.ffirst = L.d_ffirst.as<uint16_t>();
        fa.fliv = L.d_fliv.as<uint8_t>();
        k_freq_fields<<<grid_of(nf), kBlock, 0, st>>>(fa);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // chain lists: offsets from the scan of the end-event counts (the
        // list path keeps every candidate's list; its frequent ones are the
        // chain lists)
        DevBuf tmp2, flag, jidx, job_alpha, job_f, w_order;
        if ((e = scan64(L.d_fnv.as<int32_t>(), nf, L.cbeg.as<int64_t>(), tmp2, st)) != hipSuccess) return e;
        // the chain entries in all (pinned slot 2), read at the next synchronisation
        if ((e = hipMemcpyAsync(&stage[2], L.cbeg.as<int64_t>() + nf, sizeof(int64_t), hipMemcpyDeviceToHost,
                                st)) != hipSuccess)
            return e;
        if (listed) {
            k_list_begin<<<grid_of(nf), kBlock, 0, st>>>(L.d_fcand.as<int64_t>(), lst_off.as<int64_t>(), L.list_seg,
                                                         nf, L.cbeg.as<int64_t>());
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
            L.chain_total = stage[2];
            L.count_ms = ms_since(t1);
            goto done;
        }
        // write jobs: the alphas with frequent extensions
        if ((e = flag.alloc(sizeof(int32_t) * nf)) != hipSuccess) return e;
        if ((e = jidx.alloc(sizeof(int64_t) * (nf + 1))) != hipSuccess) return e;
        k_job_flags<<<grid_of(nf), kBlock, 0, st>>>(L.d_fpar.as<int32_t>(), nf, flag.as<int32_t>());
        if ((e = scan64(flag.as<int32_t>(), nf, jidx.as<int64_t>(), tmp, st)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(&stage[3], jidx.as<int64_t>() + nf, sizeof(int64_t), hipMemcpyDeviceToHost, st)) !=
            hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        L.chain_total = stage[2];
        const int64_t nj = stage[3];
        if ((e = job_alpha.alloc(sizeof(int32_t) * nj)) != hipSuccess) return e;
        if ((e = job_f.alloc(sizeof(int64_t) * (nj + 1))) != hipSuccess) return e;
        k_job_write<<<grid_of(nf + 1), kBlock, 0, st>>>(L.d_fpar.as<int32_t>(), flag.as<int32_t>(),
                                                       jidx.as<int64_t>(), nf, job_alpha.as<int32_t>(),
                                                       job_f.as<int64_t>());
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (N > 2) {
            // few jobs: the longest walks first, so that none is left alone at the end
            DevBuf lkey;
            if ((e = lkey.alloc(sizeof(uint16_t) * std::max<int64_t>(1, nj))) != hipSuccess) return e;
            k_len_key<<<grid_of(nj), kBlock, 0, st>>>(P.d_fnv.as<int32_t>(), job_alpha.as<int32_t>(), nj,
                                                      lkey.as<uint16_t>());
            if ((e = order_by_key(lkey.as<uint16_t>(), nullptr, nj, 33, w_order, st)) != hipSuccess) return e;
        }
        const size_t tot = (size_t)L.chain_total;
        if ((e = L.chain.alloc(sizeof(ChainEntry<T>) * tot)) != hipSuccess) return e;
        a.job_alpha = job_alpha.as<int32_t>();
        a.job_f = job_f.as<int64_t>();
        a.order = N > 2 ? w_order.as<int32_t>() : nullptr;
        a.w_type = L.d_flast.as<uint16_t>();
        a.w_iv = L.d_fliv.as<uint8_t>();
        a.w_off = L.cbeg.as<int64_t>();
        a.wchain = L.chain.as<ChainEntry<T>>();
        DevBuf wseg, woff;
        if (mn.list_budget > 0 && nj < kWritePieced) {
            // few write jobs: walks cut into pieces; the end events of each
            // (frequent episode, piece), scanned in that order, give every
            // piece its offset in the chain lists (the same layout)
            const int32_t nseg = (int32_t)std::max<int64_t>(1, std::min<int64_t>(64, (kWriteJobs + nj - 1) / nj));
            if ((e = wseg.alloc(sizeof(int32_t) * (size_t)nf * nseg)) != hipSuccess) return e;
            if ((e = woff.alloc(sizeof(int64_t) * ((size_t)nf * nseg + 1))) != hipSuccess) return e;
            a.nseg = nseg;
            a.nvalid = wseg.as<int32_t>();
            a.walked = nullptr;
            if ((e = launch_walk<T, kWSize>(a, nj * nseg, st)) != hipSuccess) return e;
            if ((e = scan64(wseg.as<int32_t>(), nf * nseg, woff.as<int64_t>(), tmp, st)) != hipSuccess) return e;
            a.lst_off = woff.as<int64_t>();
            if ((e = launch_walk<T, kWList>(a, nj * nseg, st)) != hipSuccess) return e;
        } else {
            a.nseg = 1;
            if ((e = launch_walk<T, kWrite>(a, nj, st)) != hipSuccess) return e;
        }
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;  // the job buffers die here
    } else {
        if ((e = hipMemsetAsync(L.cbeg.p, 0, sizeof(int64_t), st)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    }
    L.count_ms = ms_since(t1);
done:
    // chain lists two levels back are no longer needed
    if (mn.levels.size() >= 2) {
        MineLevel &Q = mn.levels[mn.levels.size() - 2];
        Q.chain.reset();
        Q.cbeg.reset();
    }
    mn.levels.push_back(std::move(L));
    return hipSuccess;
}

template <typename T>
hipError_t level1_t(const Stream &s, Mine &mn, hipStream_t st) {
    hipError_t e;
    MineLevel L;
    L.N = 1;
    L.m = s.K;
    L.implicit = false;
    auto t1 = Clock::now();
    if ((e = L.dcounts.alloc(sizeof(int32_t) * s.K)) != hipSuccess) return e;
    k_level1<T><<<s.K, kWave, 0, st>>>(s.ts_by_type.as<T>(), s.type_off.as<int32_t>(), L.dcounts.as<int32_t>());
    if ((e = hipGetLastError()) != hipSuccess) return e;
    L.counts.resize(s.K);
    if ((e = hipMemcpyAsync(L.counts.data(), L.dcounts.p, sizeof(int32_t) * s.K, hipMemcpyDeviceToHost, st)) !=
        hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    L.types.resize(s.K);
    for (int32_t k = 0; k < s.K; ++k) L.types[k] = (uint16_t)k;
    std::vector<uint16_t> f1;
    for (int32_t k = 0; k < s.K; ++k) {
        if (L.counts[k] > mn.threshold) {
            L.freq.push_back(k);
            f1.push_back((uint16_t)k);
        }
    }
    L.nf = (int64_t)L.freq.size();
    // a 1-node episode's first and last node is its type
    if ((e = L.d_flast.alloc(sizeof(uint16_t) * std::max<size_t>(1, f1.size()))) != hipSuccess) return e;
    if ((e = L.d_ffirst.alloc(sizeof(uint16_t) * std::max<size_t>(1, f1.size()))) != hipSuccess) return e;
    if (!f1.empty()) {
        if ((e = hipMemcpyAsync(L.d_flast.p, f1.data(), sizeof(uint16_t) * f1.size(), hipMemcpyHostToDevice, st)) !=
            hipSuccess)
            return e;
        if ((e = hipMemcpyAsync(L.d_ffirst.p, f1.data(), sizeof(uint16_t) * f1.size(), hipMemcpyHostToDevice,
                                st)) != hipSuccess)
            return e;
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    L.count_ms = ms_since(t1);
    L.alg_bytes = s.n * (int64_t)s.ts_bytes() + 4 * (int64_t)s.K;
    mn.levels.push_back(std::move(L));
    return hipSuccess;
}

template <typename V>
hipError_t to_host(const DevBuf &d, int64_t n, std::vector<V> &h) {
    h.resize((size_t)std::max<int64_t>(0, n));
    if (n <= 0) return hipSuccess;
    return hipMemcpy(h.data(), d.p, sizeof(V) * (size_t)n, hipMemcpyDeviceToHost);
}

// Types and interval ids of frequent episode f of a level (host copies).
void frequent_nodes(const Mine &mn, int level, int64_t f, int32_t *types, int *ivs) {
    for (int L = level; L >= 1; --L) {
        const MineLevel &V = mn.levels[L - 1];
        if (L == 1) {
            types[0] = (int32_t)V.freq[f];
            break;
        }
        types[L - 1] = V.h_flast[f];
        ivs[L - 2] = V.h_fliv[f];
        f = V.h_fpar[f];
    }
}

}  // namespace

hipError_t extend_level1(const Stream &s, Mine &mn, hipStream_t st) {
    if (s.ts_kind == EPI_TS_I64) return level1_t<int64_t>(s, mn, st);
    return level1_t<int32_t>(s, mn, st);
}

hipError_t extend_level(const Stream &s, Mine &mn, int N, hipStream_t st) {
    if (s.ts_kind == EPI_TS_I64) return level_t<int64_t>(s, mn, N, st);
    return level_t<int32_t>(s, mn, N, st);
}

// Bytes the window walk of a level must read and write: the stream positions
// it walked (type and time of each), the alphas' chain lists (one entry and
// its window end each), and each candidate's count and end-event count.
int64_t extend_level_bytes(const Stream &s, Mine &mn, int level) {
    MineLevel &L = mn.levels[level - 1];
    if (L.alg_bytes >= 0) return L.alg_bytes;
    const MineLevel &P = mn.levels[level - 2];
    const int64_t tsb = s.ts_bytes();
    int64_t entries = 0;
    if (L.N == 2) {
        for (int64_t f : P.freq) entries += s.h_off[f + 1] - s.h_off[f];
    } else {
        entries = P.chain_total;
    }
    const int64_t entry = tsb == 8 ? (int64_t)sizeof(ChainEntry<int64_t>) : (int64_t)sizeof(ChainEntry<int32_t>);
    L.alg_bytes = L.walked * (2 + tsb) + entries * (entry + 4) + L.m * 8;
    return L.alg_bytes;
}

hipError_t extend_prepare(const Stream &s, Mine &mn, hipStream_t st) {
    hipError_t e;
    if ((e = mn.ty16.alloc(sizeof(uint16_t) * (size_t)s.n)) != hipSuccess) return e;
    if ((e = mn.wend.alloc(sizeof(int32_t) * (size_t)s.n)) != hipSuccess) return e;
    if (s.n == 0) return hipSuccess;
    const int64_t H = *std::max_element(mn.menu_hi.begin(), mn.menu_hi.end());
    const unsigned blocks = (unsigned)((s.n + 255) / 256);
    if (s.ts_kind == EPI_TS_I64) {
        if ((e = mn.chain1.alloc(sizeof(ChainEntry<int64_t>) * (size_t)s.n)) != hipSuccess) return e;
        k_walk_prep<int64_t><<<blocks, 256, 0, st>>>(s.types.as<int32_t>(), s.times.as<int64_t>(), s.n, H,
                                                     mn.ty16.as<uint16_t>(), mn.wend.as<int32_t>());
        k_type_chain<int64_t><<<blocks, 256, 0, st>>>(s.ts_by_type.as<int64_t>(), s.pos_by_type.as<int32_t>(), s.n,
                                                      mn.chain1.as<ChainEntry<int64_t>>());
    } else {
        if ((e = mn.chain1.alloc(sizeof(ChainEntry<int32_t>) * (size_t)s.n)) != hipSuccess) return e;
        k_walk_prep<int32_t><<<blocks, 256, 0, st>>>(s.types.as<int32_t>(), s.times.as<int32_t>(), s.n, (int32_t)H,
                                                     mn.ty16.as<uint16_t>(), mn.wend.as<int32_t>());
        k_type_chain<int32_t><<<blocks, 256, 0, st>>>(s.ts_by_type.as<int32_t>(), s.pos_by_type.as<int32_t>(), s.n,
                                                      mn.chain1.as<ChainEntry<int32_t>>());
    }
    return hipGetLastError();
}

// Host copies of the device-side bookkeeping of levels 2..level (made once).
hipError_t extend_host_view(Mine &mn, int level) {
    hipError_t e;
    for (int Lv = 2; Lv <= level; ++Lv) {
        MineLevel &L = mn.levels[Lv - 1];
        if (!L.implicit || L.host_view) continue;
        std::vector<int64_t> fc;
        if ((e = to_host(L.d_fcand, L.nf, fc)) != hipSuccess) return e;
        L.freq = std::move(fc);
        if ((e = to_host(L.d_fpar, L.nf, L.h_fpar)) != hipSuccess) return e;
        if ((e = to_host(L.d_flast, L.nf, L.h_flast)) != hipSuccess) return e;
        if ((e = to_host(L.d_fliv, L.nf, L.h_fliv)) != hipSuccess) return e;
        if (Lv >= 3) {
            if ((e = to_host(L.d_out_off, L.nA + 1, L.out_off)) != hipSuccess) return e;
            if ((e = to_host(L.d_rlo, L.nA, L.rlo)) != hipSuccess) return e;
            if ((e = to_host(L.d_xlo, L.nA, L.xlo)) != hipSuccess) return e;
            if ((e = to_host(L.d_xhi, L.nA, L.xhi)) != hipSuccess) return e;
        }
        L.host_view = true;
    }
    return hipSuccess;
}

void extend_frequent(const Mine &mn, int level, int64_t f, int32_t *types, int *ivs) {
    frequent_nodes(mn, level, f, types, ivs);
}

void implicit_candidate(const Mine &mn, int level, int64_t c, int32_t *types, int *ivs) {
    const MineLevel &L = mn.levels[level - 1];
    const int M = (int)mn.menu_lo.size();
    const int N = L.N;
    if (N == 2) {
        const MineLevel &P = mn.levels[0];
        const int64_t per = (L.nA - 1) * M;
        const int64_t a = c / per, r = c - a * per;
        const int64_t bi0 = r / M;
        const int64_t bi = bi0 >= a ? bi0 + 1 : bi0;
        types[0] = (int32_t)P.freq[a];
        types[1] = (int32_t)P.freq[bi];
        ivs[0] = (int)(r - bi0 * M);
        return;
    }
    const MineLevel &P = mn.levels[level - 2];
    const int64_t alpha = std::upper_bound(L.out_off.begin(), L.out_off.end(), c) - L.out_off.begin() - 1;
    int64_t rr = L.rlo[alpha] + (c - L.out_off[alpha]);
    if (rr >= L.xlo[alpha]) rr += L.xhi[alpha] - L.xlo[alpha];
    frequent_nodes(mn, level - 1, alpha, types, ivs);
    types[N - 1] = P.h_flast[rr];
    ivs[N - 2] = P.h_fliv[rr];
}

}  // namespace epi
