// Pair-existence bitmaps for level-wise discovery over an interval menu.
//
// For every event e (at tiled position pos), every type x and every menu
// interval i = (lo, hi]:
//   pred(i, x, pos) = some event of type x lies at a gap in (lo, hi] before e,
//                     i.e. in [t_e - hi, t_e - lo);
//   succ(i, x, pos) = some event of type x lies at a gap in (lo, hi] after e,
//                     i.e. in (t_e + lo, t_e + hi].
// This is the tracking step of Parallel Local Tracking (Sec. IV-C: from each
// event, look for events of the next type inside the constraint window),
// done once for every (type, interval) pair instead of once per episode.
// An event of node j of an episode can change that episode's count only if
// it has a node-(j-1) predecessor (for j > 1) and a node-(j+1) successor
// (for j < N) under the episode's constraints, so the counting kernel skips
// every other event exactly.
//
// One wave builds one 64-bit word (64 consecutive tiled positions) for one
// type x: each lane binary-searches the per-type index of x and the wave
// ballots the bits.
#include <algorithm>

#include "epi_internal.h"

namespace epi {

namespace {

template <typename T>
__device__ __forceinline__ int32_t lower_bound_ts(const T *ts, int32_t lo, int32_t hi, T x) {
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (ts[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <typename T>
__device__ __forceinline__ int32_t upper_bound_ts(const T *ts, int32_t lo, int32_t hi, T x) {
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (ts[mid] <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <typename T>
__global__ __launch_bounds__(256) void k_pair_bits(const T *__restrict__ tiled, const uint16_t *__restrict__ loff,
                                                   int64_t B, int32_t K, const T *__restrict__ ts,
                                                   const int32_t *__restrict__ type_off, const T *__restrict__ menu,
                                                   int32_t M, uint64_t *__restrict__ pbits,
                                                   uint64_t *__restrict__ sbits) {
    const int lane = threadIdx.x & 63;
    const int64_t words = B * (kTile / 64);
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;  // uniform per wave
    if (w >= words) return;
    const int x = blockIdx.y;
    const int64_t b = w / (kTile / 64);
    const int pos = (int)(w % (kTile / 64)) * 64 + lane;
    const bool valid = pos < loff[b * (K + 1) + K];
    const T t = valid ? tiled[b * kTile + pos] : T(0);
    const int32_t xlo = type_off[x], xhi = type_off[x + 1];
    for (int i = 0; i < M; ++i) {
        const T lo = menu[2 * i], hi = menu[2 * i + 1];
        bool pb = false, sb = false;
        if (valid && xlo < xhi) {
            const int32_t a = lower_bound_ts(ts, xlo, xhi, (T)(t - hi));
            pb = a < xhi && ts[a] < (T)(t - lo);
            const int32_t c = upper_bound_ts(ts, xlo, xhi, (T)(t + lo));
            sb = c < xhi && ts[c] <= (T)(t + hi);
        }
        const uint64_t pw = __ballot(pb);
        const uint64_t sw = __ballot(sb);
        if (lane == 0) {
            const int64_t row = (int64_t)i * K + x;
            pbits[row * words + w] = pw;
            sbits[row * words + w] = sw;
        }
    }
}

// Predecessor bits in per-type index order: one wave per 64 consecutive
// positions of ts_by_type, one grid row per type x.
template <typename T>
__global__ __launch_bounds__(256) void k_index_pred_bits(const T *__restrict__ ts, int64_t n,
                                                         const int32_t *__restrict__ type_off,
                                                         const T *__restrict__ menu, int32_t M, int32_t K,
                                                         int64_t words, uint64_t *__restrict__ bits) {
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;  // uniform per wave
    if (w >= words) return;
    const int x = blockIdx.y;
    const int64_t q = w * 64 + lane;
    const bool valid = q < n;
    const T t = valid ? ts[q] : T(0);
    const int32_t xlo = type_off[x], xhi = type_off[x + 1];
    for (int i = 0; i < M; ++i) {
        const T lo = menu[2 * i], hi = menu[2 * i + 1];
        bool pb = false;
        if (valid && xlo < xhi) {
            const int32_t a = lower_bound_ts(ts, xlo, xhi, (T)(t - hi));
            pb = a < xhi && ts[a] < (T)(t - lo);
        }
        const uint64_t pw = __ballot(pb);
        if (lane == 0) bits[((int64_t)i * K + x) * words + w] = pw;
    }
}

// Number of set bits of row (i, x) over the index range of each type B.
__global__ void k_index_pred_popcount(const uint64_t *__restrict__ bits, const int32_t *__restrict__ type_off,
                                      int32_t M, int32_t K, int64_t words, int32_t *__restrict__ pop) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)M * K * K) return;
    const int32_t B = (int32_t)(q % K);
    const int64_t row = q / K;  // i * K + x
    const int32_t y0 = type_off[B], q1 = type_off[B + 1];
    int32_t c = 0;
    if (q1 > y0) {
        const uint64_t *pb = bits + row * words;
        const int32_t w0 = y0 >> 6, w1 = (q1 - 1) >> 6;
        for (int32_t w = w0; w <= w1; ++w) {
            uint64_t v = pb[w];
            if (w == w0) v &= ~0ull << (y0 & 63);
            if (w == w1 && (q1 & 63)) v &= (1ull << (q1 & 63)) - 1ull;
            c += __popcll(v);
        }
    }
    pop[q] = c;
}

}  // namespace

hipError_t build_index_pred_bits(const Stream &s, Mine &mn, hipStream_t st) {
    const int M = (int)mn.menu_lo.size();
    const int64_t words = (s.n + 63) / 64;
    hipError_t e;
    mn.xwords = words;
    if ((e = mn.xpred.alloc(sizeof(uint64_t) * (size_t)std::max<int64_t>(1, M * s.K * words))) != hipSuccess) return e;
    if (words == 0) return hipSuccess;
    DevBuf menu;
    const int wpb = 4;  // waves (words) per block
    const dim3 grid((unsigned)((words + wpb - 1) / wpb), (unsigned)s.K);
    if (s.ts_kind == EPI_TS_I64) {
        std::vector<int64_t> h(2 * M);
        for (int i = 0; i < M; ++i) {
            h[2 * i] = mn.menu_lo[i];
            h[2 * i + 1] = mn.menu_hi[i];
        }
        if ((e = menu.alloc(sizeof(int64_t) * 2 * M)) != hipSuccess) return e;
        if ((e = hipMemcpy(menu.p, h.data(), sizeof(int64_t) * 2 * M, hipMemcpyHostToDevice)) != hipSuccess) return e;
        k_index_pred_bits<int64_t><<<grid, 64 * wpb, 0, st>>>(s.ts_by_type.as<int64_t>(), s.n, s.type_off.as<int32_t>(),
                                                             menu.as<int64_t>(), M, s.K, words,
                                                             mn.xpred.as<uint64_t>());
    } else {
        std::vector<int32_t> h(2 * M);
        for (int i = 0; i < M; ++i) {
            h[2 * i] = (int32_t)mn.menu_lo[i];
            h[2 * i + 1] = (int32_t)mn.menu_hi[i];
        }
        if ((e = menu.alloc(sizeof(int32_t) * 2 * M)) != hipSuccess) return e;
        if ((e = hipMemcpy(menu.p, h.data(), sizeof(int32_t) * 2 * M, hipMemcpyHostToDevice)) != hipSuccess) return e;
        k_index_pred_bits<int32_t><<<grid, 64 * wpb, 0, st>>>(s.ts_by_type.as<int32_t>(), s.n, s.type_off.as<int32_t>(),
                                                             menu.as<int32_t>(), M, s.K, words,
                                                             mn.xpred.as<uint64_t>());
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // per (interval, x, B) counts of set bits: the events the filtered merge visits
    const int64_t np = (int64_t)M * s.K * s.K;
    DevBuf dpop;
    if ((e = dpop.alloc(sizeof(int32_t) * np)) != hipSuccess) return e;
    k_index_pred_popcount<<<(unsigned)((np + 255) / 256), 256, 0, st>>>(mn.xpred.as<uint64_t>(), s.type_off.as<int32_t>(),
                                                                      M, s.K, words, dpop.as<int32_t>());
    if ((e = hipGetLastError()) != hipSuccess) return e;
    mn.xpop.resize(np);
    if ((e = hipMemcpyAsync(mn.xpop.data(), dpop.p, sizeof(int32_t) * np, hipMemcpyDeviceToHost, st)) != hipSuccess)
        return e;
    return hipStreamSynchronize(st);  // the menu and count buffers die here
}

hipError_t build_pair_bits(const Stream &s, Mine &mn, hipStream_t st) {
    const int M = (int)mn.menu_lo.size();
    const int64_t words = s.B * (kTile / 64);
    const size_t bytes = sizeof(uint64_t) * (size_t)M * s.K * words;
    hipError_t e;
    if ((e = mn.pred_bits.alloc(bytes)) != hipSuccess) return e;
    if ((e = mn.succ_bits.alloc(bytes)) != hipSuccess) return e;
    if (words == 0) return hipSuccess;
    DevBuf menu;
    std::vector<int64_t> h(2 * M);
    for (int i = 0; i < M; ++i) {
        h[2 * i] = mn.menu_lo[i];
        h[2 * i + 1] = mn.menu_hi[i];
    }
    const int wpb = 4;  // waves (words) per block
    const dim3 grid((unsigned)((words + wpb - 1) / wpb), (unsigned)s.K);
    if (s.ts_kind == EPI_TS_I64) {
        if ((e = menu.alloc(sizeof(int64_t) * 2 * M)) != hipSuccess) return e;
        if ((e = hipMemcpy(menu.p, h.data(), sizeof(int64_t) * 2 * M, hipMemcpyHostToDevice)) != hipSuccess) return e;
        k_pair_bits<int64_t><<<grid, 64 * wpb, 0, st>>>(s.tiled_ts.as<int64_t>(), s.tile_loff.as<uint16_t>(), s.B, s.K,
                                                       s.ts_by_type.as<int64_t>(), s.type_off.as<int32_t>(),
                                                       menu.as<int64_t>(), M, mn.pred_bits.as<uint64_t>(),
                                                       mn.succ_bits.as<uint64_t>());
    } else {
        std::vector<int32_t> h32(2 * M);
        for (int i = 0; i < 2 * M; ++i) h32[i] = (int32_t)h[i];
        if ((e = menu.alloc(sizeof(int32_t) * 2 * M)) != hipSuccess) return e;
        if ((e = hipMemcpy(menu.p, h32.data(), sizeof(int32_t) * 2 * M, hipMemcpyHostToDevice)) != hipSuccess)
            return e;
        k_pair_bits<int32_t><<<grid, 64 * wpb, 0, st>>>(s.tiled_ts.as<int32_t>(), s.tile_loff.as<uint16_t>(), s.B, s.K,
                                                       s.ts_by_type.as<int32_t>(), s.type_off.as<int32_t>(),
                                                       menu.as<int32_t>(), M, mn.pred_bits.as<uint64_t>(),
                                                       mn.succ_bits.as<uint64_t>());
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipStreamSynchronize(st);  // the menu buffer dies here
}

}  // namespace epi
