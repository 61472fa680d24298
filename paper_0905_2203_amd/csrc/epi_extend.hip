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
// at the latest x with t_x < t_y - lo, provided t_x >= t_y - hi.  So with
// alpha's chain list -- its end events in time order with their latest
// starts -- one merge of two sorted lists gives s(y) for every y, and the
// greedy of Alg. 1 over the y in time order (keep y when s(y) > the last kept
// end, starting from minus infinity) gives the count.  This is Parallel Local
// Tracking (Sec. IV-C) advanced by one node per level, with book-keeping of
// start times and the end-ordered list for free.
//
// Level 1 counts distinct timestamps per type.  Level 2 candidates extend a
// frequent type (its chain list is its own events, s = t).  The chain lists
// of a level's frequent episodes are written by a second pass over those
// episodes only, at offsets from an exclusive scan of their end-event counts
// (the count / scan / write compaction of Sec. IV-E).
//
// Counting: one wave per alpha; its lanes take alpha's extensions (the
// Apriori join's matches, minus the one repeating alpha's first type),
// 64 at a time; every lane of the wave reads the same chain list.
#include <algorithm>
#include <chrono>
#include <numeric>
#include <thread>

#include "epi_fsm.h"

namespace epi {

namespace {

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0) { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }

template <typename T>
struct ExtArgs {
    const T *ts;             // per-type index (time order per type)
    const int32_t *type_off; // [K+1]
    int64_t nA;              // number of alphas
    // level 2 (MODE 0): alphas are frequent types
    const uint16_t *f1;      // [nf1] frequent types
    int32_t nf1;
    // level >= 3 (MODE 1): alphas are frequent episodes of the previous level
    const Pair<T> *chains;   // chain lists of the previous level's frequent episodes
    const int64_t *coff;     // [nfprev + 1]
    const uint16_t *ftype0;  // [nfprev] first type
    const uint16_t *flast;   // [nfprev] last type
    const uint8_t *fliv;     // [nfprev] last interval id
    const int32_t *rlo, *rhi, *byprefix;
    const int64_t *out_off;  // [nA + 1]
    const int32_t *aorder;   // order in which the workgroups take the alphas (null: index order)
    const T *menu;           // (lo, hi) pairs
    int32_t M;
    const uint64_t *xbits;   // predecessor bits (interval, type, index position) or null
    int64_t xwords;
    int32_t K;
    int32_t *counts;         // [m]
    int32_t *nvalid;         // [m]
    // write pass: explicit list of candidates
    int64_t nw;
    const int32_t *w_alpha;
    const uint16_t *w_type;
    const uint8_t *w_iv;
    const int64_t *w_off;
    const int32_t *w_order;  // order in which the threads take the write list (null: list order)
    Pair<T> *w_out;
};

// One candidate: merge alpha's chain list with the events of type B; returns
// the count, the number of end events, and optionally writes the new chain.
//
// The lanes of a wave read 64 different type lists, far more lines than the
// L1 keeps between a lane's visits; so each lane reads its list in whole
// 64-byte lines (16-byte loads from a line-aligned address) and consumes
// them from registers; the elements before the first line boundary and after
// the last whole line are read one by one.  Alpha's chain list is shared by
// the wave; its next two entries are held ahead.
template <typename T, int MODE, bool WRITE, bool FILT>
__device__ __forceinline__ int32_t ext_core(const ExtArgs<T> &a, int64_t alpha, int32_t X, int32_t B, int iv,
                                            int32_t *nval, Pair<T> *out) {
    constexpr T kMin = TsLimits<T>::lo();
    constexpr T kMax = TsLimits<T>::hi();
    constexpr int kLineBytes = 64;
    constexpr int kLine = kLineBytes / (int)sizeof(T);
    constexpr int kVec = kLineBytes / 16;
    const T lo = a.menu[2 * iv], hi = a.menu[2 * iv + 1];
    // alpha's chain list
    const T *at = nullptr;
    const Pair<T> *ap = nullptr;
    int32_t alen;
    if (MODE == 0) {
        const int32_t ty = a.f1[alpha];
        at = a.ts + a.type_off[ty];
        alen = a.type_off[ty + 1] - a.type_off[ty];
    } else {
        ap = a.chains + a.coff[alpha];
        alen = (int32_t)(a.coff[alpha + 1] - a.coff[alpha]);
    }
    auto chain_at = [&](int32_t q) {
        Pair<T> v;
        if (q < alen) {
            if (MODE == 0) {
                v.s = at[q];
                v.e = v.s;
            } else {
                v = ap[q];
            }
        } else {
            v.s = kMax;
            v.e = kMax;
        }
        return v;
    };
    const int32_t y0 = a.type_off[B];
    const int32_t ylen = a.type_off[B + 1] - y0;
    const T *y = a.ts + y0;
    int32_t p = 0, cnt = 0, nv = 0;
    T prev_e = kMin;
    T xt = kMin, xs = kMin;  // latest entry with time < t_y - lo (when p > 0)
    Pair<T> n1 = chain_at(0), n2 = chain_at(1);
    auto step = [&](const T ty) {
        const T lim = (T)(ty - lo);
        while (n1.s < lim) {
            xt = n1.s;
            xs = n1.e;
            ++p;
            n1 = n2;
            n2 = chain_at(p + 1);
        }
        if (p > 0 && xt >= (T)(ty - hi)) {
            if (WRITE) {
                Pair<T> w;
                w.s = ty;
                w.e = xs;
                out[nv] = w;
            }
            ++nv;
            if (xs > prev_e) {
                ++cnt;
                prev_e = ty;
            }
        }
    };
    if (FILT) {
        // only the events of B with an event of alpha's last type X at a gap
        // in the interval before them can end an occurrence: visit those
        if (ylen > 0) {
            const uint64_t *pb = a.xbits + ((int64_t)iv * a.K + X) * a.xwords;
            const int32_t q1 = y0 + ylen;
            const int32_t w0 = y0 >> 6, w1 = (q1 - 1) >> 6;
            for (int32_t w = w0; w <= w1; ++w) {
                uint64_t bits = pb[w];
                if (w == w0) bits &= ~0ull << (y0 & 63);
                if (w == w1 && (q1 & 63)) bits &= (1ull << (q1 & 63)) - 1ull;
                const T *yw = a.ts + ((int64_t)w << 6);
                while (bits) {
                    // up to four loads in flight
                    T v[4];
                    int k = 0;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (bits) {
                            v[u] = yw[__builtin_ctzll(bits)];
                            bits &= bits - 1ull;
                            k = u + 1;
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (u < k) step(v[u]);
                }
            }
        }
        *nval = nv;
        return cnt;
    }
    // elements up to the first line boundary
    const int32_t lead = (int32_t)((uint32_t)y0 & (uint32_t)(kLine - 1));
    const int32_t head = lead == 0 ? 0 : min(ylen, kLine - lead);
    int32_t i = 0;
    for (; i < head; ++i) step(y[i]);
    // whole lines
    for (; i + kLine <= ylen; i += kLine) {
        uint4 raw[kVec];
        const uint4 *src = reinterpret_cast<const uint4 *>(y + i);
#pragma unroll
        for (int k = 0; k < kVec; ++k) raw[k] = src[k];
        const T *v = reinterpret_cast<const T *>(raw);
#pragma unroll
        for (int u = 0; u < kLine; ++u) step(v[u]);
    }
    // the rest
    for (; i < ylen; ++i) step(y[i]);
    *nval = nv;
    return cnt;
}

template <typename T, bool FILT>
__global__ __launch_bounds__(64) void k_ext_count0(ExtArgs<T> a) {
    const int64_t alpha = blockIdx.x;
    const int lane = threadIdx.x;
    const int32_t R = a.nf1 * a.M;
    const int64_t o0 = a.out_off[alpha];
    for (int32_t rb = 0; rb < R; rb += 64) {
        const int32_t r = rb + lane;
        if (r >= R) break;
        const int32_t bi = r / a.M, iv = r % a.M;
        if (bi == alpha) continue;
        const int64_t c = o0 + (bi < alpha ? r : r - a.M);
        int32_t nv;
        a.counts[c] = ext_core<T, 0, false, FILT>(a, alpha, a.f1[alpha], a.f1[bi], iv, &nv, nullptr);
        a.nvalid[c] = nv;
    }
}

template <typename T, bool FILT>
__global__ __launch_bounds__(64) void k_ext_count1(ExtArgs<T> a) {
    const int64_t alpha = a.aorder ? a.aorder[blockIdx.x] : (int64_t)blockIdx.x;
    const int lane = threadIdx.x;
    const int32_t r0 = a.rlo[alpha], r1 = a.rhi[alpha];
    const int64_t o0 = a.out_off[alpha];
    const uint16_t first = a.ftype0[alpha];
    const int32_t X = a.flast[alpha];
    int32_t skipped = 0;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int32_t rb = r0; rb < r1; rb += 64) {  // uniform across the wave
        const int32_t r = rb + lane;
        const bool in = r < r1;
        const int32_t beta = in ? a.byprefix[r] : 0;
        const bool excl = in && a.flast[beta] == first;
        const uint64_t em = __ballot(excl);
        if (in && !excl) {
            const int64_t c = o0 + (r - r0) - skipped - __popcll(em & lt);
            int32_t nv;
            a.counts[c] = ext_core<T, 1, false, FILT>(a, alpha, X, a.flast[beta], a.fliv[beta], &nv, nullptr);
            a.nvalid[c] = nv;
        }
        skipped += __popcll(em);
    }
}

template <typename T, int MODE, bool FILT>
__global__ __launch_bounds__(256) void k_ext_write(ExtArgs<T> a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.nw) return;
    const int64_t f = a.w_order ? a.w_order[g] : g;
    int32_t nv;
    const int32_t alpha = a.w_alpha[f];
    const int32_t X = MODE == 0 ? a.f1[alpha] : a.flast[alpha];
    (void)ext_core<T, MODE, true, FILT>(a, alpha, X, a.w_type[f], a.w_iv[f], &nv, a.w_out + a.w_off[f]);
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

template <typename T>
__global__ void k_level1(const T *__restrict__ ts, const int32_t *__restrict__ type_off, int32_t K,
                         int32_t *__restrict__ counts) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    int32_t c = 0;
    for (int32_t i = type_off[k]; i < type_off[k + 1]; ++i)
        if (i == type_off[k] || ts[i] != ts[i - 1]) ++c;
    counts[k] = c;
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
    const size_t tsb = sizeof(T);
    auto t0 = Clock::now();
    const std::vector<int32_t> &off = s.h_off;
    auto ntype = [&](int32_t ty) { return (int64_t)off[ty + 1] - off[ty]; };
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
    DevBuf d_out_off, d_f1, d_menu, d_rlo, d_rhi, d_by, d_f0, d_fl, d_fliv, d_counts, d_nval, d_order;
    std::vector<T> menu(2 * M);
    for (int i = 0; i < M; ++i) {
        menu[2 * i] = (T)mn.menu_lo[i];
        menu[2 * i + 1] = (T)mn.menu_hi[i];
    }
    if ((e = upload(d_out_off, L.out_off, st)) != hipSuccess) return e;
    if ((e = upload(d_menu, menu, st)) != hipSuccess) return e;
    ExtArgs<T> a{};
    a.ts = s.ts_by_type.as<T>();
    a.type_off = s.type_off.as<int32_t>();
    a.nA = nA;
    a.out_off = d_out_off.as<int64_t>();
    a.menu = d_menu.as<T>();
    a.M = M;
    a.K = s.K;
    a.xbits = mn.xpred.p ? mn.xpred.as<uint64_t>() : nullptr;
    a.xwords = mn.xwords;
    // host sources of asynchronous uploads live until the level's last sync
    std::vector<uint16_t> f1, f0, fl;
    std::vector<uint8_t> fliv;
    std::vector<int32_t> order;
    if (N == 2) {
        f1.assign(P.ftypes.begin(), P.ftypes.begin() + P.nf);
        if ((e = upload(d_f1, f1, st)) != hipSuccess) return e;
        a.f1 = d_f1.as<uint16_t>();
        a.nf1 = (int32_t)P.nf;
    } else {
        f0.assign(P.ftypes.begin(), P.ftypes.begin() + P.nf);
        fl.assign(P.ftypes.begin() + (size_t)(P.N - 1) * P.nf, P.ftypes.begin() + (size_t)P.N * P.nf);
        fliv.assign(P.fiv.begin() + (size_t)(P.N - 2) * P.nf, P.fiv.begin() + (size_t)(P.N - 1) * P.nf);
        if ((e = upload(d_f0, f0, st)) != hipSuccess) return e;
        if ((e = upload(d_fl, fl, st)) != hipSuccess) return e;
        if ((e = upload(d_fliv, fliv, st)) != hipSuccess) return e;
        if ((e = upload(d_rlo, L.rlo, st)) != hipSuccess) return e;
        if ((e = upload(d_rhi, L.rhi, st)) != hipSuccess) return e;
        if ((e = upload(d_by, L.byprefix, st)) != hipSuccess) return e;
        a.chains = P.chains.as<Pair<T>>();
        a.coff = P.chain_off.as<int64_t>();
        a.ftype0 = d_f0.as<uint16_t>();
        a.flast = d_fl.as<uint16_t>();
        a.fliv = d_fliv.as<uint8_t>();
        a.rlo = d_rlo.as<int32_t>();
        a.rhi = d_rhi.as<int32_t>();
        a.byprefix = d_by.as<int32_t>();
        // workgroups take the alphas grouped by their last type: the waves in
        // flight then read the same type's predecessor bits and nearly the
        // same type lists, which stay in each XCD's L2
        order = order_by_key(nA, s.K, [&](int64_t x) { return (int32_t)fl[x]; });
        if ((e = upload(d_order, order, st)) != hipSuccess) return e;
        a.aorder = d_order.as<int32_t>();
    }
    if ((e = d_counts.alloc(sizeof(int32_t) * m)) != hipSuccess) return e;
    if ((e = d_nval.alloc(sizeof(int32_t) * m)) != hipSuccess) return e;
    a.counts = d_counts.as<int32_t>();
    a.nvalid = d_nval.as<int32_t>();
    L.gen_ms = ms_since(t0);
    auto t1 = Clock::now();
    // ---- count
    hipEvent_t ev0, ev1;
    if ((e = hipEventCreate(&ev0)) != hipSuccess) return e;
    if ((e = hipEventCreate(&ev1)) != hipSuccess) return e;
    (void)hipEventRecord(ev0, st);
    if (m > 0) {
        if (N == 2) {
            if (a.xbits) k_ext_count0<T, true><<<(unsigned)nA, 64, 0, st>>>(a);
            else k_ext_count0<T, false><<<(unsigned)nA, 64, 0, st>>>(a);
        } else {
            if (a.xbits) k_ext_count1<T, true><<<(unsigned)nA, 64, 0, st>>>(a);
            else k_ext_count1<T, false><<<(unsigned)nA, 64, 0, st>>>(a);
        }
    }
    (void)hipEventRecord(ev1, st);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    float kms = 0;
    if (e == hipSuccess) (void)hipEventElapsedTime(&kms, ev0, ev1);
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (e != hipSuccess) return e;
    L.kernel_ms = kms;
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
    DevBuf d_wa, d_wt, d_wi, d_wo;
    // the write pass takes the frequent episodes grouped by alpha's last type
    // (as the counting pass takes the alphas)
    std::vector<int32_t> w_order = order_by_key(nf, s.K, [&](int64_t f) {
        const int64_t al = w_alpha[f];
        return (int32_t)(N == 2 ? P.ftypes[al] : P.ftypes[(size_t)(P.N - 1) * P.nf + al]);
    });
    if ((e = upload(d_wo, w_order, st)) != hipSuccess) return e;
    if ((e = upload(d_wa, w_alpha, st)) != hipSuccess) return e;
    if ((e = upload(d_wt, w_type, st)) != hipSuccess) return e;
    if ((e = upload(d_wi, w_iv, st)) != hipSuccess) return e;
    if ((e = upload(L.chain_off, L.h_chain_off, st)) != hipSuccess) return e;
    if ((e = L.chains.alloc(sizeof(Pair<T>) * (size_t)L.h_chain_off[nf])) != hipSuccess) return e;
    if (nf > 0) {
        a.nw = nf;
        a.w_alpha = d_wa.as<int32_t>();
        a.w_type = d_wt.as<uint16_t>();
        a.w_iv = d_wi.as<uint8_t>();
        a.w_off = L.chain_off.as<int64_t>();
        a.w_order = d_wo.as<int32_t>();
        a.w_out = L.chains.as<Pair<T>>();
        const unsigned blocks = (unsigned)((nf + 255) / 256);
        if (N == 2) {
            if (a.xbits) k_ext_write<T, 0, true><<<blocks, 256, 0, st>>>(a);
            else k_ext_write<T, 0, false><<<blocks, 256, 0, st>>>(a);
        } else {
            if (a.xbits) k_ext_write<T, 1, true><<<blocks, 256, 0, st>>>(a);
            else k_ext_write<T, 1, false><<<blocks, 256, 0, st>>>(a);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    L.count_ms = ms_since(t1);
    // chain lists two levels back are no longer needed
    if (mn.levels.size() >= 2) {
        MineLevel &Q = mn.levels[mn.levels.size() - 2];
        Q.chains.reset();
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
    k_level1<T><<<(s.K + 63) / 64, 64, 0, st>>>(s.ts_by_type.as<T>(), s.type_off.as<int32_t>(), s.K,
                                              d_counts.as<int32_t>());
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

// Bytes read and written per candidate: the events of the new node's type
// that the merge visits (with predecessor bits: the bit words over the
// type's index range and the events whose bit is set), alpha's chain list,
// the count and the end-event count.
int64_t extend_level_bytes(const Stream &s, Mine &mn, int level) {
    MineLevel &L = mn.levels[level - 1];
    if (L.alg_bytes >= 0) return L.alg_bytes;
    const MineLevel &P = mn.levels[level - 2];
    const int N = L.N;
    const int M = (int)mn.menu_lo.size();
    const int64_t tsb = s.ts_bytes();
    const std::vector<int32_t> &off = s.h_off;
    auto ntype = [&](int32_t ty) { return (int64_t)off[ty + 1] - off[ty]; };
    const bool filt = mn.xpred.p != nullptr && !mn.xpop.empty();
    auto node_bytes = [&](int iv, int32_t X, int32_t B) -> int64_t {
        if (!filt) return ntype(B) * tsb;
        const int64_t y0 = off[B], q1 = off[B + 1];
        const int64_t words = q1 > y0 ? ((q1 - 1) >> 6) - (y0 >> 6) + 1 : 0;
        return words * 8 + (int64_t)mn.xpop[((int64_t)iv * s.K + X) * s.K + B] * tsb;
    };
    const int64_t nA = P.nf;
    std::vector<int64_t> part(nA, 0);
    parallel_for(nA, [&](int64_t x0, int64_t x1) {
        for (int64_t a = x0; a < x1; ++a) {
            const int64_t k = L.out_off[a + 1] - L.out_off[a];
            if (k == 0) continue;
            const int64_t alen = N == 2 ? ntype(P.ftypes[a]) : P.h_chain_off[a + 1] - P.h_chain_off[a];
            int64_t b = k * (alen * (N == 2 ? 1 : 2) * tsb + 8);
            if (N == 2) {
                for (int64_t bi = 0; bi < nA; ++bi)
                    if (bi != a)
                        for (int iv = 0; iv < M; ++iv) b += node_bytes(iv, P.ftypes[a], P.ftypes[bi]);
            } else {
                const int32_t X = P.ftypes[(size_t)(P.N - 1) * P.nf + a];
                for (int64_t e = 0; e < k; ++e) {
                    const int32_t beta = L.byprefix[ext_position(L, a, e)];
                    b += node_bytes(P.fiv[(size_t)(P.N - 2) * P.nf + beta], X, P.ftypes[(size_t)(P.N - 1) * P.nf + beta]);
                }
            }
            part[a] = b;
        }
    });
    int64_t total = 0;
    for (int64_t a = 0; a < nA; ++a) total += part[a];
    L.alg_bytes = total;
    return total;
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
