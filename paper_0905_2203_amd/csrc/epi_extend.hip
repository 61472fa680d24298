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
constexpr uint8_t kNoSlot = 0xFF;

template <typename T>
struct WalkArgs {
    const uint16_t *ty16;     // [n] event types, stream order
    const T *times;           // [n]
    const int32_t *wend;      // [n] first position whose time exceeds times[p] + H
    T H;                      // longest menu interval end
    // the alphas' chain lists
    const T *ct, *cs;         // level >= 3: end times, latest starts
    const int32_t *cp;        // level >= 3: stream positions
    const int64_t *coff;      // level >= 3: [nA + 1]
    const T *ts_by_type;      // level 2: a frequent type's chain is its own events
    const int32_t *pos_by_type;
    const int32_t *type_off;
    const uint16_t *f1;       // level 2: the frequent types
    int32_t nf1;
    // one job per workgroup
    const int32_t *job_alpha; // alpha of each job (null: the job index)
    const int32_t *order;     // order in which the workgroups take the jobs (null: index order)
    // counting pass: each alpha's extensions and their outputs
    const int64_t *out_off;   // [nA + 1]
    const int32_t *rlo, *rhi, *xlo, *xhi, *byprefix;
    const uint16_t *flast;    // last type of each frequent episode of the previous level
    const uint8_t *fliv;      // its last interval id
    int32_t *counts, *nvalid;
    unsigned long long *walked;  // stream positions walked, summed over the jobs
    // write pass: each job's range of the frequent list
    const int64_t *job_f;     // [njobs + 1]
    const uint16_t *w_type;
    const uint8_t *w_iv;
    const int64_t *w_off;     // first chain-list slot of each frequent episode
    T *wct, *wcs;
    int32_t *wcp;
    T menu_lo[kExtMaxMenu], menu_hi[kExtMaxMenu];
    int32_t M;
    int32_t K;
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

template <typename T>
__device__ __forceinline__ T lane_value(T v, int src) {
    if constexpr (sizeof(T) == 4) {
        return (T)__shfl((int)v, src, kWave);
    } else {
        const uint64_t u = (uint64_t)v;
        const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)u, src, kWave);
        const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(u >> 32), src, kWave);
        return (T)(((uint64_t)hi << 32) | lo);
    }
}

// Extension r of a job: its new type B, interval id and key (counting: the
// candidate's index; writing: the first slot of its chain list).  Within a
// job the extensions are ordered by B.
template <typename T, bool L2, bool WRITE>
__device__ __forceinline__ void extension(const WalkArgs<T> &a, int64_t job, int64_t alpha, int64_t r, int32_t &B,
                                          int &iv, int64_t &key) {
    if (WRITE) {
        const int64_t f = a.job_f[job] + r;
        B = a.w_type[f];
        iv = a.w_iv[f];
        key = a.w_off[f];
    } else if (L2) {
        const int64_t bi0 = r / a.M;
        iv = (int)(r - bi0 * a.M);
        const int64_t bi = bi0 >= alpha ? bi0 + 1 : bi0;
        B = a.f1[bi];
        key = a.out_off[alpha] + r;
    } else {
        int64_t rr = a.rlo[alpha] + r;
        if (rr >= a.xlo[alpha]) rr += a.xhi[alpha] - a.xlo[alpha];
        const int32_t beta = a.byprefix[rr];
        B = a.flast[beta];
        iv = a.fliv[beta];
        key = a.out_off[alpha] + r;
    }
}

template <typename T, bool L2, bool WRITE>
__device__ __forceinline__ int64_t n_extensions(const WalkArgs<T> &a, int64_t job, int64_t alpha) {
    if (WRITE) return a.job_f[job + 1] - a.job_f[job];
    if (L2) return (int64_t)(a.nf1 - 1) * a.M;
    return (int64_t)(a.rhi[alpha] - a.rlo[alpha]) - (a.xhi[alpha] - a.xlo[alpha]);
}

// One job: alpha, all of its extensions (or, writing, its frequent ones).
// MP >= M greedy states per lane, one per menu interval.
template <typename T, int MP, bool L2, bool WRITE>
__global__ __launch_bounds__(kWave) void k_ext_walk(WalkArgs<T> a) {
    constexpr T kMin = TsLimits<T>::lo();
    constexpr T kMax = TsLimits<T>::hi();
    extern __shared__ uint8_t slot_of[];            // [K] lane owning each type this round
    __shared__ unsigned long long want[kWave];      // batch lanes holding each owner's events
    __shared__ int32_t gtype[kWave];
    __shared__ int64_t gkey[MP][kWave];
    const int lane = threadIdx.x;
    const int64_t job = a.order ? (int64_t)a.order[blockIdx.x] : (int64_t)blockIdx.x;
    const int64_t alpha = a.job_alpha ? (int64_t)a.job_alpha[job] : job;
    const int M = a.M;
    // alpha's chain list
    const_ptr<T> xt, xs;
    const int32_t *xp;
    int32_t clen;
    if (L2) {
        const int32_t ty = a.f1[alpha];
        const int32_t o = a.type_off[ty];
        clen = a.type_off[ty + 1] - o;
        xt = (const_ptr<T>)(a.ts_by_type + o);
        xs = xt;
        xp = a.pos_by_type + o;
    } else {
        const int64_t o = a.coff[alpha];
        clen = (int32_t)(a.coff[alpha + 1] - o);
        xt = (const_ptr<T>)(a.ct + o);
        xs = (const_ptr<T>)(a.cs + o);
        xp = a.cp + o;
    }
    const int64_t R = n_extensions<T, L2, WRITE>(a, job, alpha);
    for (int k = lane; k < a.K; k += kWave) slot_of[k] = kNoSlot;
    want[lane] = 0;
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
            if (in) extension<T, L2, WRITE>(a, job, alpha, r, B, iv, key);
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
        T pe[MP];
        int32_t cnt[MP], nv[MP];
#pragma unroll
        for (int m = 0; m < MP; ++m) {
            key[m] = has ? gkey[m][lane] : -1;
            pe[m] = kMin;
            cnt[m] = 0;
            nv[m] = 0;
        }
        if (has) slot_of[myB] = (uint8_t)lane;
        __syncthreads();
        // ---- the walk over U(alpha)
        int32_t carry = 0;  // coverage end of the entries already taken
        int32_t ilo = 0;    // first entry that can still be a predecessor
        for (int32_t i0 = 0; i0 < clen; i0 += kWave) {  // uniform
            const int32_t i = i0 + lane;
            const bool ci = i < clen;
            const int32_t p = ci ? xp[i] : 0;
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
            for (int32_t b = 0; b < total; b += kWave) {  // uniform
                const int32_t o = b + lane;
                const bool ev = o < total;
                uint64_t runs = __ballot(len > 0 && X < b + kWave && S > b);
                int32_t P = 0;
                while (runs) {
                    const int j = __builtin_ctzll(runs);
                    runs &= runs - 1;
                    const int32_t Xj = __builtin_amdgcn_readlane(X, j);
                    const int32_t bj = __builtin_amdgcn_readlane(beg, j);
                    if (o >= Xj) P = bj + (o - Xj);
                }
                const int32_t ty = ev ? (int32_t)a.ty16[P] : 0;
                const T t = ev ? a.times[P] : kMax;
                const int nb = min(total - b, kWave);
                const T tf = read_lane(t, 0), tl = read_lane(t, nb - 1);
                while (ilo < clen && xt[ilo] < (T)(tf - a.H)) ++ilo;
                T cx[MP], cxs[MP], lim[MP];
#pragma unroll
                for (int m = 0; m < MP; ++m) {
                    cx[m] = kMin;
                    cxs[m] = kMin;
                    lim[m] = m < M ? (T)(t - a.menu_lo[m]) : kMin;
                }
                for (int32_t q = ilo; q < clen; ++q) {  // uniform
                    const T qt = xt[q];
                    if (qt >= tl) break;
                    const T qs = xs[q];
#pragma unroll
                    for (int m = 0; m < MP; ++m) {
                        if (qt < lim[m]) {
                            cx[m] = qt;
                            cxs[m] = qs;
                        }
                    }
                }
                T sv[MP];
                bool any = false;
#pragma unroll
                for (int m = 0; m < MP; ++m) {
                    sv[m] = (m < M && ev && cx[m] >= (T)(t - a.menu_hi[m])) ? cxs[m] : kMin;
                    any |= sv[m] != kMin;
                }
                if (any) {
                    const uint8_t sl = slot_of[ty];
                    if (sl != kNoSlot) atomicOr(&want[sl], 1ull << lane);
                }
                __syncthreads();
                uint64_t wm = want[lane];
                want[lane] = 0;
                while (__ballot(wm != 0)) {  // uniform
                    const int k = wm ? __builtin_ctzll(wm) : lane;
                    const T yt = lane_value(t, k);
                    const int32_t yp = __shfl(P, k, kWave);
                    T ys[MP];
#pragma unroll
                    for (int m = 0; m < MP; ++m) ys[m] = m < M ? lane_value(sv[m], k) : kMin;
                    if (wm) {
#pragma unroll
                        for (int m = 0; m < MP; ++m) {
                            if (key[m] >= 0 && ys[m] != kMin) {
                                if (WRITE) {
                                    const int64_t w = key[m] + nv[m];
                                    a.wct[w] = yt;
                                    a.wcs[w] = ys[m];
                                    a.wcp[w] = yp;
                                }
                                ++nv[m];
                                if (ys[m] > pe[m]) {
                                    ++cnt[m];
                                    pe[m] = yt;
                                }
                            }
                        }
                        wm &= wm - 1;
                    }
                }
            }
        }
        if (!WRITE) {
#pragma unroll
            for (int m = 0; m < MP; ++m) {
                if (key[m] >= 0) {
                    a.counts[key[m]] = cnt[m];
                    a.nvalid[key[m]] = nv[m];
                }
            }
        }
        if (has) slot_of[myB] = kNoSlot;
        __syncthreads();
        r_start = r_next;
    }
    if (!WRITE && a.walked && lane == 0) atomicAdd(a.walked, walked);
}

template <typename T, bool L2, bool WRITE>
hipError_t launch_walk(const WalkArgs<T> &a, int64_t njobs, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    const size_t lds = (size_t)(a.K + 15) / 16 * 16;
    if (a.M <= 4) k_ext_walk<T, 4, L2, WRITE><<<(unsigned)njobs, kWave, lds, st>>>(a);
    else k_ext_walk<T, 8, L2, WRITE><<<(unsigned)njobs, kWave, lds, st>>>(a);
    return hipGetLastError();
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

// Frequent selection (count > threshold), order preserving: per-block flag
// counts, then each block writes its indices at its scanned offset.
constexpr int kSelBlock = 256;
constexpr int kSelItems = 8;

__global__ __launch_bounds__(kSelBlock) void k_sel_count(const int32_t *__restrict__ counts, int64_t m, int32_t thr,
                                                         int32_t *__restrict__ bcnt) {
    __shared__ int32_t red[kSelBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kSelBlock * kSelItems;
    int32_t c = 0;
    for (int k = 0; k < kSelItems; ++k) {
        const int64_t i = base + (int64_t)k * kSelBlock + threadIdx.x;
        if (i < m && counts[i] > thr) ++c;
    }
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < kSelBlock / 64; ++w) t += red[w];
        bcnt[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kSelBlock) void k_sel_write(const int32_t *__restrict__ counts,
                                                         const int32_t *__restrict__ nvalid, int64_t m, int32_t thr,
                                                         const int64_t *__restrict__ boff, int64_t *__restrict__ idx,
                                                         int32_t *__restrict__ nv) {
    __shared__ int32_t wsum[kSelBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kSelBlock * kSelItems;
    int64_t off = boff[blockIdx.x];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = 0; k < kSelItems; ++k) {  // uniform
        const int64_t i = base + (int64_t)k * kSelBlock + threadIdx.x;
        const bool f = i < m && counts[i] > thr;
        const uint64_t bal = __ballot(f);
        if (lane == 0) wsum[w] = __popcll(bal);
        __syncthreads();
        int32_t before = 0, total = 0;
        for (int q = 0; q < kSelBlock / 64; ++q) {
            if (q < w) before += wsum[q];
            total += wsum[q];
        }
        if (f) {
            const int64_t o = off + before + __popcll(bal & ((1ull << lane) - 1ull));
            idx[o] = i;
            nv[o] = nvalid[i];
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

template <typename U>
hipError_t upload(DevBuf &d, const std::vector<U> &h, hipStream_t st) {
    hipError_t e = d.alloc(sizeof(U) * h.size());
    if (e != hipSuccess) return e;
    if (!h.empty()) e = hipMemcpyAsync(d.p, h.data(), sizeof(U) * h.size(), hipMemcpyHostToDevice, st);
    return e;
}

int nthreads() { return (int)std::max<unsigned>(1, std::min<unsigned>(32, std::thread::hardware_concurrency())); }

template <typename F>
void parallel_for(int64_t n, F &&body) {
    const int nt = nthreads();
    if (n < 4096 || nt == 1) {
        body(0, n);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (n + nt - 1) / nt;
    for (int q = 0; q < nt; ++q) {
        const int64_t x0 = q * chunk, x1 = std::min(n, x0 + chunk);
        if (x0 >= x1) break;
        th.emplace_back([&, x0, x1] { body(x0, x1); });
    }
    for (auto &t : th) t.join();
}

// Indices 0..n-1 stably ordered by key(i) in [0, K) (counting sort).
template <typename F>
std::vector<int32_t> order_by_key(int64_t n, int32_t K, F &&key) {
    std::vector<int64_t> start(K + 1, 0);
    for (int64_t i = 0; i < n; ++i) ++start[key(i) + 1];
    for (int32_t k = 0; k < K; ++k) start[k + 1] += start[k];
    std::vector<int32_t> out(n);
    for (int64_t i = 0; i < n; ++i) out[start[key(i)]++] = (int32_t)i;
    return out;
}

// local extension index e of alpha (level >= 3) -> position r in byprefix
// (the excluded extensions, those repeating alpha's first type, are the
// contiguous range [xlo, xhi) of alpha's range)
int32_t ext_position(const MineLevel &L, int64_t alpha, int64_t e) {
    const int64_t r = L.rlo[alpha] + e;
    return (int32_t)(r < L.xlo[alpha] ? r : r + (L.xhi[alpha] - L.xlo[alpha]));
}

// Sort with a strict weak order on nt threads: sorted chunks, then merged
// pairwise in rounds.
template <typename It, typename Less>
void parallel_sort(It first, It last, Less less) {
    const int64_t n = last - first;
    const int nt = nthreads();
    if (n < 65536 || nt == 1) {
        std::sort(first, last, less);
        return;
    }
    std::vector<int64_t> cut(nt + 1);
    for (int q = 0; q <= nt; ++q) cut[q] = n * q / nt;
    {
        std::vector<std::thread> th;
        for (int q = 0; q < nt; ++q) th.emplace_back([&, q] { std::sort(first + cut[q], first + cut[q + 1], less); });
        for (auto &t : th) t.join();
    }
    for (int width = 1; width < nt; width *= 2) {
        std::vector<std::thread> th;
        for (int q = 0; q + width < nt; q += 2 * width) {
            const int64_t a = cut[q], b = cut[q + width], c = cut[std::min(nt, q + 2 * width)];
            th.emplace_back([=] { std::inplace_merge(first + a, first + b, first + c, less); });
        }
        for (auto &t : th) t.join();
    }
}

template <typename T>
hipError_t level_t(const Stream &s, Mine &mn, int N, int32_t *d_flags, hipStream_t st) {
    (void)d_flags;
    hipError_t e;
    MineLevel &P = mn.levels.back();  // level N-1
    MineLevel L;
    L.N = N;
    L.implicit = true;
    const int M = (int)mn.menu_lo.size();
    auto t0 = Clock::now();
    // ---- the candidate family of each alpha
    int64_t nA = P.nf;
    L.out_off.assign(nA + 1, 0);
    if (N == 2) {
        for (int64_t a = 0; a < nA; ++a) L.out_off[a + 1] = L.out_off[a] + (nA - 1) * M;
    } else {
        const int Pn = P.N;  // episodes of the previous level have Pn = N-1 nodes
        auto pty = [&](int64_t i, int k) { return P.ftypes[(size_t)k * P.nf + i]; };
        auto piv = [&](int64_t i, int k) { return P.fiv[(size_t)k * P.nf + i]; };
        L.byprefix.resize(P.nf);
        std::iota(L.byprefix.begin(), L.byprefix.end(), 0);
        // prefix of beta = its first Pn-1 nodes and Pn-2 intervals; within a
        // prefix, by the last node (type, then interval)
        auto prefix_less = [&](int32_t a, int32_t b) {
            for (int k = 0; k < Pn - 1; ++k) {
                if (pty(a, k) != pty(b, k)) return pty(a, k) < pty(b, k);
                if (k < Pn - 2 && piv(a, k) != piv(b, k)) return piv(a, k) < piv(b, k);
            }
            if (pty(a, Pn - 1) != pty(b, Pn - 1)) return pty(a, Pn - 1) < pty(b, Pn - 1);
            return piv(a, Pn - 2) < piv(b, Pn - 2);
        };
        parallel_sort(L.byprefix.begin(), L.byprefix.end(), prefix_less);
        // compare prefix(beta) with suffix(alpha) = last Pn-1 nodes of alpha
        auto cmp = [&](int32_t beta, int64_t alpha) {
            for (int k = 0; k < Pn - 1; ++k) {
                if (pty(beta, k) != pty(alpha, k + 1)) return pty(beta, k) < pty(alpha, k + 1) ? -1 : 1;
                if (k < Pn - 2 && piv(beta, k) != piv(alpha, k + 1)) return piv(beta, k) < piv(alpha, k + 1) ? -1 : 1;
            }
            return 0;
        };
        L.rlo.resize(nA);
        L.rhi.resize(nA);
        L.xlo.resize(nA);
        L.xhi.resize(nA);
        std::vector<int64_t> cnt(nA, 0);
        parallel_for(nA, [&](int64_t x0, int64_t x1) {
            for (int64_t a = x0; a < x1; ++a) {
                const auto lo = std::partition_point(L.byprefix.begin(), L.byprefix.end(),
                                                     [&](int32_t b) { return cmp(b, a) < 0; });
                const auto hi =
                    std::partition_point(lo, L.byprefix.end(), [&](int32_t b) { return cmp(b, a) == 0; });
                L.rlo[a] = (int32_t)(lo - L.byprefix.begin());
                L.rhi[a] = (int32_t)(hi - L.byprefix.begin());
                // extensions whose new type is alpha's first: one run in the range
                const uint16_t first = pty(a, 0);
                const auto xl = std::partition_point(lo, hi, [&](int32_t b) { return pty(b, Pn - 1) < first; });
                const auto xh = std::partition_point(xl, hi, [&](int32_t b) { return pty(b, Pn - 1) == first; });
                L.xlo[a] = (int32_t)(xl - L.byprefix.begin());
                L.xhi[a] = (int32_t)(xh - L.byprefix.begin());
                cnt[a] = (hi - lo) - (xh - xl);
            }
        });
        for (int64_t a = 0; a < nA; ++a) L.out_off[a + 1] = L.out_off[a] + cnt[a];
    }
    const int64_t m = L.out_off[nA];
    L.m = m;
    // ---- device inputs
    DevBuf d_out_off, d_f1, d_rlo, d_rhi, d_xlo, d_xhi, d_by, d_fl, d_fliv, d_counts, d_nval, d_order, d_walked;
    if ((e = upload(d_out_off, L.out_off, st)) != hipSuccess) return e;
    WalkArgs<T> a{};
    a.ty16 = mn.ty16.as<uint16_t>();
    a.times = s.times.as<T>();
    a.wend = mn.wend.as<int32_t>();
    a.H = (T)*std::max_element(mn.menu_hi.begin(), mn.menu_hi.end());
    a.ts_by_type = s.ts_by_type.as<T>();
    a.pos_by_type = s.pos_by_type.as<int32_t>();
    a.type_off = s.type_off.as<int32_t>();
    a.out_off = d_out_off.as<int64_t>();
    a.M = M;
    a.K = s.K;
    for (int i = 0; i < M; ++i) {
        a.menu_lo[i] = (T)mn.menu_lo[i];
        a.menu_hi[i] = (T)mn.menu_hi[i];
    }
    // host sources of asynchronous uploads live until the level's last sync
    std::vector<uint16_t> f1, fl;
    std::vector<uint8_t> fliv;
    std::vector<int32_t> order;
    if (N == 2) {
        f1.assign(P.ftypes.begin(), P.ftypes.begin() + P.nf);
        if ((e = upload(d_f1, f1, st)) != hipSuccess) return e;
        a.f1 = d_f1.as<uint16_t>();
        a.nf1 = (int32_t)P.nf;
    } else {
        fl.assign(P.ftypes.begin() + (size_t)(P.N - 1) * P.nf, P.ftypes.begin() + (size_t)P.N * P.nf);
        fliv.assign(P.fiv.begin() + (size_t)(P.N - 2) * P.nf, P.fiv.begin() + (size_t)(P.N - 1) * P.nf);
        if ((e = upload(d_fl, fl, st)) != hipSuccess) return e;
        if ((e = upload(d_fliv, fliv, st)) != hipSuccess) return e;
        if ((e = upload(d_rlo, L.rlo, st)) != hipSuccess) return e;
        if ((e = upload(d_rhi, L.rhi, st)) != hipSuccess) return e;
        if ((e = upload(d_xlo, L.xlo, st)) != hipSuccess) return e;
        if ((e = upload(d_xhi, L.xhi, st)) != hipSuccess) return e;
        if ((e = upload(d_by, L.byprefix, st)) != hipSuccess) return e;
        a.ct = P.ct.as<T>();
        a.cs = P.cs.as<T>();
        a.cp = P.cp.as<int32_t>();
        a.coff = P.chain_off.as<int64_t>();
        a.flast = d_fl.as<uint16_t>();
        a.fliv = d_fliv.as<uint8_t>();
        a.rlo = d_rlo.as<int32_t>();
        a.rhi = d_rhi.as<int32_t>();
        a.xlo = d_xlo.as<int32_t>();
        a.xhi = d_xhi.as<int32_t>();
        a.byprefix = d_by.as<int32_t>();
        // workgroups take the alphas grouped by their last type: the waves in
        // flight then walk the neighbourhoods of the same type's events
        order = order_by_key(nA, s.K, [&](int64_t x) { return (int32_t)fl[x]; });
        if ((e = upload(d_order, order, st)) != hipSuccess) return e;
        a.order = d_order.as<int32_t>();
    }
    if ((e = d_counts.alloc(sizeof(int32_t) * m)) != hipSuccess) return e;
    if ((e = d_nval.alloc(sizeof(int32_t) * m)) != hipSuccess) return e;
    if ((e = d_walked.alloc(sizeof(unsigned long long))) != hipSuccess) return e;
    if ((e = hipMemsetAsync(d_walked.p, 0, sizeof(unsigned long long), st)) != hipSuccess) return e;
    a.counts = d_counts.as<int32_t>();
    a.nvalid = d_nval.as<int32_t>();
    a.walked = d_walked.as<unsigned long long>();
    L.gen_ms = ms_since(t0);
    auto t1 = Clock::now();
    // ---- count
    hipEvent_t ev0, ev1;
    if ((e = hipEventCreate(&ev0)) != hipSuccess) return e;
    if ((e = hipEventCreate(&ev1)) != hipSuccess) return e;
    (void)hipEventRecord(ev0, st);
    if (m > 0) e = N == 2 ? launch_walk<T, true, false>(a, nA, st) : launch_walk<T, false, false>(a, nA, st);
    (void)hipEventRecord(ev1, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    float kms = 0;
    if (e == hipSuccess) (void)hipEventElapsedTime(&kms, ev0, ev1);
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (e != hipSuccess) return e;
    L.kernel_ms = kms;
    {
        unsigned long long wk = 0;
        if ((e = hipMemcpy(&wk, d_walked.p, sizeof(wk), hipMemcpyDeviceToHost)) != hipSuccess) return e;
        L.walked = (int64_t)wk;
    }
    // ---- frequent episodes, selected on the device (counts stay there)
    std::vector<int32_t> nval;
    {
        const int64_t per = (int64_t)kSelBlock * kSelItems;
        const int64_t nb = m > 0 ? (m + per - 1) / per : 0;
        DevBuf d_bcnt, d_boff;
        if ((e = d_bcnt.alloc(sizeof(int32_t) * (nb + 1))) != hipSuccess) return e;
        const int32_t thr = (int32_t)std::min<int64_t>(mn.threshold, INT32_MAX);
        int64_t nf = 0;
        std::vector<int64_t> boff(nb + 1, 0);
        if (nb > 0) {
            if (mn.threshold < 0) {
                // every candidate is frequent
                for (int64_t b = 0; b < nb; ++b) boff[b + 1] = boff[b] + std::min(per, m - b * per);
            } else {
                k_sel_count<<<(unsigned)nb, kSelBlock, 0, st>>>(a.counts, m, thr, d_bcnt.as<int32_t>());
                if ((e = hipGetLastError()) != hipSuccess) return e;
                std::vector<int32_t> bc(nb);
                if ((e = hipMemcpyAsync(bc.data(), d_bcnt.p, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, st)) !=
                    hipSuccess)
                    return e;
                if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
                for (int64_t b = 0; b < nb; ++b) boff[b + 1] = boff[b] + bc[b];
            }
            nf = boff[nb];
        }
        L.freq.assign(nf, 0);
        nval.assign(nf, 0);
        if (nf > 0) {
            DevBuf d_idx, d_nv;
            if ((e = upload(d_boff, boff, st)) != hipSuccess) return e;
            if ((e = d_idx.alloc(sizeof(int64_t) * nf)) != hipSuccess) return e;
            if ((e = d_nv.alloc(sizeof(int32_t) * nf)) != hipSuccess) return e;
            k_sel_write<<<(unsigned)nb, kSelBlock, 0, st>>>(a.counts, a.nvalid, m, mn.threshold < 0 ? INT32_MIN : thr,
                                                            d_boff.as<int64_t>(), d_idx.as<int64_t>(),
                                                            d_nv.as<int32_t>());
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((e = hipMemcpyAsync(L.freq.data(), d_idx.p, sizeof(int64_t) * nf, hipMemcpyDeviceToHost, st)) !=
                hipSuccess)
                return e;
            if ((e = hipMemcpyAsync(nval.data(), d_nv.p, sizeof(int32_t) * nf, hipMemcpyDeviceToHost, st)) !=
                hipSuccess)
                return e;
            if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        }
    }
    L.dcounts = std::move(d_counts);
    const int64_t nf = (int64_t)L.freq.size();
    L.nf = nf;
    L.ftypes.assign((size_t)N * nf, 0);
    L.fiv.assign((size_t)(N - 1) * nf, 0);
    std::vector<int32_t> w_alpha(nf);
    std::vector<uint16_t> w_type(nf);
    std::vector<uint8_t> w_iv(nf);
    parallel_for(nf, [&](int64_t x0, int64_t x1) {
        for (int64_t f = x0; f < x1; ++f) {
            const int64_t c = L.freq[f];
            const int64_t alpha = std::upper_bound(L.out_off.begin(), L.out_off.end(), c) - L.out_off.begin() - 1;
            const int64_t le = c - L.out_off[alpha];
            uint16_t bt;
            uint8_t biv;
            if (N == 2) {
                int64_t r = le < alpha * M ? le : le + M;
                bt = P.ftypes[r / M];
                biv = (uint8_t)(r % M);
            } else {
                const int32_t r = ext_position(L, alpha, le);
                const int32_t beta = L.byprefix[r];
                bt = P.ftypes[(size_t)(P.N - 1) * P.nf + beta];
                biv = P.fiv[(size_t)(P.N - 2) * P.nf + beta];
            }
            for (int k = 0; k < N - 1; ++k) L.ftypes[(size_t)k * nf + f] = P.ftypes[(size_t)k * P.nf + alpha];
            L.ftypes[(size_t)(N - 1) * nf + f] = bt;
            for (int k = 0; k < N - 2; ++k) L.fiv[(size_t)k * nf + f] = P.fiv[(size_t)k * P.nf + alpha];
            L.fiv[(size_t)(N - 2) * nf + f] = biv;
            w_alpha[f] = (int32_t)alpha;
            w_type[f] = bt;
            w_iv[f] = biv;
        }
    });
    L.h_chain_off.assign(nf + 1, 0);
    for (int64_t f = 0; f < nf; ++f) L.h_chain_off[f + 1] = L.h_chain_off[f] + nval[f];
    // write jobs: the alphas with frequent extensions (the frequent list is in
    // candidate order, so each alpha's frequent extensions are contiguous)
    std::vector<int32_t> job_alpha;
    std::vector<int64_t> job_f;
    for (int64_t f = 0; f < nf; ++f) {
        if (f == 0 || w_alpha[f] != w_alpha[f - 1]) {
            job_alpha.push_back(w_alpha[f]);
            job_f.push_back(f);
        }
    }
    job_f.push_back(nf);
    const int64_t nj = (int64_t)job_alpha.size();
    // taken grouped by alpha's last type, as the counting pass takes them
    std::vector<int32_t> w_order = order_by_key(nj, s.K, [&](int64_t j) {
        const int64_t al = job_alpha[j];
        return (int32_t)(N == 2 ? P.ftypes[al] : P.ftypes[(size_t)(P.N - 1) * P.nf + al]);
    });
    DevBuf d_ja, d_jf, d_wt, d_wi, d_wo;
    if ((e = upload(d_ja, job_alpha, st)) != hipSuccess) return e;
    if ((e = upload(d_jf, job_f, st)) != hipSuccess) return e;
    if ((e = upload(d_wo, w_order, st)) != hipSuccess) return e;
    if ((e = upload(d_wt, w_type, st)) != hipSuccess) return e;
    if ((e = upload(d_wi, w_iv, st)) != hipSuccess) return e;
    if ((e = upload(L.chain_off, L.h_chain_off, st)) != hipSuccess) return e;
    const size_t tot = (size_t)L.h_chain_off[nf];
    if ((e = L.ct.alloc(sizeof(T) * tot)) != hipSuccess) return e;
    if ((e = L.cs.alloc(sizeof(T) * tot)) != hipSuccess) return e;
    if ((e = L.cp.alloc(sizeof(int32_t) * tot)) != hipSuccess) return e;
    if (nj > 0) {
        a.job_alpha = d_ja.as<int32_t>();
        a.job_f = d_jf.as<int64_t>();
        a.order = d_wo.as<int32_t>();
        a.w_type = d_wt.as<uint16_t>();
        a.w_iv = d_wi.as<uint8_t>();
        a.w_off = L.chain_off.as<int64_t>();
        a.wct = L.ct.as<T>();
        a.wcs = L.cs.as<T>();
        a.wcp = L.cp.as<int32_t>();
        e = N == 2 ? launch_walk<T, true, true>(a, nj, st) : launch_walk<T, false, true>(a, nj, st);
        if (e != hipSuccess) return e;
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    L.count_ms = ms_since(t1);
    // chain lists two levels back are no longer needed
    if (mn.levels.size() >= 2) {
        MineLevel &Q = mn.levels[mn.levels.size() - 2];
        Q.ct.reset();
        Q.cs.reset();
        Q.cp.reset();
        Q.chain_off.reset();
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
    DevBuf d_counts;
    if ((e = d_counts.alloc(sizeof(int32_t) * s.K)) != hipSuccess) return e;
    k_level1<T><<<s.K, kWave, 0, st>>>(s.ts_by_type.as<T>(), s.type_off.as<int32_t>(), d_counts.as<int32_t>());
    if ((e = hipGetLastError()) != hipSuccess) return e;
    L.counts.resize(s.K);
    if ((e = hipMemcpyAsync(L.counts.data(), d_counts.p, sizeof(int32_t) * s.K, hipMemcpyDeviceToHost, st)) !=
        hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    L.count_ms = ms_since(t1);
    L.types.resize(s.K);
    for (int32_t k = 0; k < s.K; ++k) L.types[k] = (uint16_t)k;
    for (int32_t k = 0; k < s.K; ++k)
        if (L.counts[k] > mn.threshold) L.freq.push_back(k);
    L.nf = (int64_t)L.freq.size();
    for (int64_t f : L.freq) L.ftypes.push_back((uint16_t)f);
    L.alg_bytes = s.n * (int64_t)s.ts_bytes() + 4 * (int64_t)s.K;
    mn.levels.push_back(std::move(L));
    return hipSuccess;
}

}  // namespace

hipError_t extend_level1(const Stream &s, Mine &mn, hipStream_t st) {
    if (s.ts_kind == EPI_TS_I64) return level1_t<int64_t>(s, mn, st);
    return level1_t<int32_t>(s, mn, st);
}

hipError_t extend_level(const Stream &s, Mine &mn, int N, int32_t *d_flags, hipStream_t st) {
    if (s.ts_kind == EPI_TS_I64) return level_t<int64_t>(s, mn, N, d_flags, st);
    return level_t<int32_t>(s, mn, N, d_flags, st);
}

// Bytes the window walk of a level must read and write: the stream positions
// it walked (type and time of each), the alphas' chain lists (time, start,
// position and window end of each entry), and each candidate's count and
// end-event count.
int64_t extend_level_bytes(const Stream &s, Mine &mn, int level) {
    MineLevel &L = mn.levels[level - 1];
    if (L.alg_bytes >= 0) return L.alg_bytes;
    const MineLevel &P = mn.levels[level - 2];
    const int64_t tsb = s.ts_bytes();
    int64_t entries = 0;
    if (L.N == 2) {
        for (int64_t a = 0; a < P.nf; ++a) entries += s.h_off[P.ftypes[a] + 1] - s.h_off[P.ftypes[a]];
    } else {
        entries = P.h_chain_off.empty() ? 0 : P.h_chain_off.back();
    }
    L.alg_bytes = L.walked * (2 + tsb) + entries * (2 * tsb + 8) + L.m * 8;
    return L.alg_bytes;
}

hipError_t extend_prepare(const Stream &s, Mine &mn, hipStream_t st) {
    hipError_t e;
    if ((e = mn.ty16.alloc(sizeof(uint16_t) * (size_t)s.n)) != hipSuccess) return e;
    if ((e = mn.wend.alloc(sizeof(int32_t) * (size_t)s.n)) != hipSuccess) return e;
    if (s.n == 0) return hipSuccess;
    const int64_t H = *std::max_element(mn.menu_hi.begin(), mn.menu_hi.end());
    const unsigned blocks = (unsigned)((s.n + 255) / 256);
    if (s.ts_kind == EPI_TS_I64)
        k_walk_prep<int64_t><<<blocks, 256, 0, st>>>(s.types.as<int32_t>(), s.times.as<int64_t>(), s.n, H,
                                                     mn.ty16.as<uint16_t>(), mn.wend.as<int32_t>());
    else
        k_walk_prep<int32_t><<<blocks, 256, 0, st>>>(s.types.as<int32_t>(), s.times.as<int32_t>(), s.n, (int32_t)H,
                                                     mn.ty16.as<uint16_t>(), mn.wend.as<int32_t>());
    return hipGetLastError();
}

void implicit_candidate(const Mine &mn, int level, int64_t c, int32_t *types, int *ivs) {
    const MineLevel &L = mn.levels[level - 1];
    const MineLevel &P = mn.levels[level - 2];
    const int M = (int)mn.menu_lo.size();
    const int N = L.N;
    const int64_t alpha = std::upper_bound(L.out_off.begin(), L.out_off.end(), c) - L.out_off.begin() - 1;
    const int64_t le = c - L.out_off[alpha];
    for (int k = 0; k < N - 1; ++k) types[k] = P.ftypes[(size_t)k * P.nf + alpha];
    for (int k = 0; k < N - 2; ++k) ivs[k] = P.fiv[(size_t)k * P.nf + alpha];
    if (N == 2) {
        const int64_t r = le < alpha * M ? le : le + M;
        types[1] = P.ftypes[r / M];
        ivs[0] = (int)(r % M);
    } else {
        const int32_t r = ext_position(L, alpha, le);
        const int32_t beta = L.byprefix[r];
        types[N - 1] = P.ftypes[(size_t)(P.N - 1) * P.nf + beta];
        ivs[N - 2] = P.fiv[(size_t)(P.N - 2) * P.nf + beta];
    }
}

}  // namespace epi
