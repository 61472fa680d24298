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
                                                   uint64_t *__restrict__ sbits, int32_t TT) {
    const int lane = threadIdx.x & 63;
    const int64_t words = B * (TT / 64);
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;  // uniform per wave
    if (w >= words) return;
    const int x = blockIdx.y;
    const int64_t b = w / (TT / 64);
    const int pos = (int)(w % (TT / 64)) * 64 + lane;
    const bool valid = pos < loff[b * (K + 1) + K];
    const T t = valid ? tiled[b * TT + pos] : T(0);
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

}  // namespace

hipError_t build_pair_bits(const Stream &s, Mine &mn, hipStream_t st) {
    const int M = (int)mn.menu_lo.size();
    const int64_t words = s.B * (s.T / 64);
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
                                                       mn.succ_bits.as<uint64_t>(), s.T);
    } else {
        std::vector<int32_t> h32(2 * M);
        for (int i = 0; i < 2 * M; ++i) h32[i] = (int32_t)h[i];
        if ((e = menu.alloc(sizeof(int32_t) * 2 * M)) != hipSuccess) return e;
        if ((e = hipMemcpy(menu.p, h32.data(), sizeof(int32_t) * 2 * M, hipMemcpyHostToDevice)) != hipSuccess)
            return e;
        k_pair_bits<int32_t><<<grid, 64 * wpb, 0, st>>>(s.tiled_ts.as<int32_t>(), s.tile_loff.as<uint16_t>(), s.B, s.K,
                                                       s.ts_by_type.as<int32_t>(), s.type_off.as<int32_t>(),
                                                       menu.as<int32_t>(), M, mn.pred_bits.as<uint64_t>(),
                                                       mn.succ_bits.as<uint64_t>(), s.T);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipStreamSynchronize(st);  // the menu buffer dies here
}

}  // namespace epi
