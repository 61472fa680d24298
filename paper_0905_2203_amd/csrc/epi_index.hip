// Per-type index of an event stream (the pre-processing step of Sec. IV-A):
// the events of each type, in time order, stored contiguously.
//
//   1. k_hist:    one wave per chunk of C events; LDS histogram over the K
//                 types; writes cnt[type * B + chunk] (type-major).
//   2. scan:      exclusive prefix sum over cnt in type-major order; entry
//                 (type, chunk) is then the global output position of the
//                 chunk's first event of that type, and (type, 0) is the
//                 type's offset.
//   3. k_scatter: each wave re-reads its chunk 64 events at a time; the
//                 rank of a lane among earlier lanes of the same type comes
//                 from a wave-wide compare loop, so the scatter is stable.
//                 It writes the per-type index (times, and the stream
//                 position of every entry) and a tile-major copy in
//                 which each chunk of T stream positions (a "tile") holds
//                 its own events grouped by type, with per-tile uint16
//                 offsets, so that a workgroup can stage a time window of
//                 every type list with one contiguous, coalesced copy.
#include <algorithm>
#include <vector>

#include "epi_internal.h"

namespace epi {

namespace {

constexpr int kWave = 64;

__global__ __launch_bounds__(kWave) void k_hist(const int32_t *__restrict__ types, int64_t n, int32_t K,
                                                int64_t chunk, int64_t B, int32_t *__restrict__ cnt) {
    __shared__ int32_t h[kMaxK];
    const int lane = threadIdx.x;
    const int64_t b = blockIdx.x;
    for (int k = lane; k < K; k += kWave) h[k] = 0;
    __syncthreads();
    const int64_t beg = b * chunk;
    const int64_t end = beg + chunk < n ? beg + chunk : n;
    for (int64_t i = beg + lane; i < end; i += kWave) atomicAdd(&h[types[i]], 1);
    __syncthreads();
    for (int k = lane; k < K; k += kWave) cnt[(int64_t)k * B + b] = h[k];
}

template <typename T>
__global__ __launch_bounds__(kWave) void k_scatter(const int32_t *__restrict__ types, const T *__restrict__ times,
                                                   int64_t n, int32_t K, int64_t B,
                                                   const int32_t *__restrict__ cnt, const int32_t *__restrict__ base,
                                                   T *__restrict__ out, int32_t *__restrict__ pos_out,
                                                   T *__restrict__ tiled,
                                                   uint16_t *__restrict__ loff, T *__restrict__ tile_t0,
                                                   int32_t TT) {
    __shared__ int32_t rank[kMaxK];   // next rank of each type inside this tile
    __shared__ int32_t start[kMaxK];  // tile-local start of each type group
    __shared__ int32_t wsum[kWave];
    const int lane = threadIdx.x;
    const int64_t b = blockIdx.x;
    // tile-local offsets: exclusive scan over types of this tile's counts
    const int per = (K + kWave - 1) / kWave;
    int32_t acc = 0;
    for (int q = 0; q < per; ++q) {
        const int k = lane * per + q;
        if (k < K) acc += cnt[(int64_t)k * B + b];
    }
    int32_t x = acc;
    for (int d = 1; d < kWave; d <<= 1) {
        const int32_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    wsum[lane] = x - acc;
    __syncthreads();
    int32_t run = wsum[lane];
    for (int q = 0; q < per; ++q) {
        const int k = lane * per + q;
        if (k < K) {
            start[k] = run;
            rank[k] = 0;
            loff[b * (K + 1) + k] = (uint16_t)run;
            run += cnt[(int64_t)k * B + b];
        }
    }
    if (lane == kWave - 1) loff[b * (K + 1) + K] = (uint16_t)(x);
    const int64_t beg = b * TT;
    const int64_t end = beg + TT < n ? beg + TT : n;
    if (lane == 0) {
        tile_t0[b] = times[beg];
        if (b == B - 1) tile_t0[B] = TsLimits<T>::hi();
    }
    __syncthreads();
    for (int64_t r = beg; r < end; r += kWave) {
        const int64_t i = r + lane;
        const bool valid = i < end;
        const int32_t ty = valid ? types[i] : -1;
        const T t = valid ? times[i] : T(0);
        int before = 0, after = 0;
        for (int l = 0; l < kWave; ++l) {
            const int32_t o = __shfl(ty, l, kWave);
            before += (l < lane && o == ty) ? 1 : 0;
            after += (l > lane && o == ty) ? 1 : 0;
        }
        int32_t rk = 0;
        if (valid) rk = rank[ty] + before;
        __syncthreads();
        if (valid) {
            const int64_t q = base[(int64_t)ty * B + b] + rk;
            out[q] = t;
            pos_out[q] = (int32_t)i;
            tiled[beg + start[ty] + rk] = t;
            if (after == 0) rank[ty] = rk + 1;
        }
        __syncthreads();
    }
}

// ---- exclusive scan of int32 (values and total fit int32) -------------------
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;  // per thread
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t *total) {
    __shared__ int32_t wsum[kScanBlock / kWave];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    int32_t x = v;
    for (int d = 1; d < kWave; d <<= 1) {
        const int32_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    int32_t off = 0, tot = 0;
    for (int k = 0; k < kScanBlock / kWave; ++k) {
        if (k < w) off += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const int32_t *__restrict__ in, int64_t len,
                                                            int32_t *__restrict__ sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int32_t acc = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        if (i < len) acc += in[i];
    }
    int32_t tot;
    (void)block_exclusive_scan(acc, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Single block: exclusive scan of the tile sums, in place.
__global__ __launch_bounds__(kScanBlock) void k_scan_sums(int32_t *__restrict__ sums, int64_t nb) {
    int32_t carry = 0;
    for (int64_t r = 0; r < nb; r += kScanBlock) {
        const int64_t i = r + threadIdx.x;
        const int32_t v = i < nb ? sums[i] : 0;
        int32_t tot;
        const int32_t ex = block_exclusive_scan(v, &tot);
        if (i < nb) sums[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const int32_t *__restrict__ in, int64_t len,
                                                           const int32_t *__restrict__ sums,
                                                           int32_t *__restrict__ out) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int32_t v[kScanItems];
    int32_t acc = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        v[k] = i < len ? in[i] : 0;
        acc += v[k];
    }
    int32_t tot;
    int32_t run = block_exclusive_scan(acc, &tot) + sums[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        if (i < len) out[i] = run;
        run += v[k];
    }
}

__global__ void k_offsets(const int32_t *__restrict__ base, int32_t K, int64_t B, int64_t n,
                          int32_t *__restrict__ off) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < K) off[k] = base[(int64_t)k * B];
    if (k == K) off[K] = (int32_t)n;
}

// g[i] = times[min(i * step, n - 1)], i < ng
template <typename T>
__global__ void k_sample_times(const T *__restrict__ times, int64_t n, int64_t step, int64_t ng, T *__restrict__ g) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ng) g[i] = times[i * step < n ? i * step : n - 1];
}

template <typename T>
__global__ void k_validate(const int32_t *__restrict__ types, const T *__restrict__ times, int64_t n, int32_t K,
                           int32_t *__restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t ty = types[i];
    const T t = times[i];
    if (ty < 0 || ty >= K) atomicOr(&flags[kFlagBadType], 1);
    if (t == TsLimits<T>::lo() || t == TsLimits<T>::hi()) atomicOr(&flags[kFlagBadTime], 1);
    if (i + 1 < n && times[i + 1] < t) atomicOr(&flags[kFlagUnsorted], 1);
}

}  // namespace

hipError_t validate_stream_device(const int32_t *d_types, const void *d_times, int64_t n, int ts_kind,
                                  int32_t K, int32_t *d_flags, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int threads = 256;
    const int64_t blocks = (n + threads - 1) / threads;
    if (ts_kind == EPI_TS_I64)
        k_validate<int64_t><<<blocks, threads, 0, st>>>(d_types, (const int64_t *)d_times, n, K, d_flags);
    else
        k_validate<int32_t><<<blocks, threads, 0, st>>>(d_types, (const int32_t *)d_times, n, K, d_flags);
    return hipGetLastError();
}

namespace {

// Longest tile of T events (T a multiple of kMinTile): from its first time
// to the next tile's first time, the last tile to the stream's last time;
// g holds the times at every kMinTile-th position (and the last one).
int64_t longest_tile(const std::vector<int64_t> &g, int64_t n, int T) {
    const int64_t per = T / kMinTile, B = (n + T - 1) / T;
    uint64_t best = 0;
    for (int64_t b = 0; b < B; ++b) {
        const int64_t i1 = (b + 1) * per;
        const int64_t end = b + 1 < B ? g[i1] : g.back();
        best = std::max<uint64_t>(best, (uint64_t)end - (uint64_t)g[b * per]);
    }
    return best > (uint64_t)INT64_MAX ? INT64_MAX : (int64_t)best;
}

// Events per tile of a stream (Stream::T).
hipError_t pick_tile(Stream &s, hipStream_t st) {
    const int cap = std::max(kMinTile, std::min(kTile, s.tile_cap));
    s.T = cap;
    if (s.n <= kMinTile) return hipSuccess;
    const int64_t ng = (s.n + kMinTile - 1) / kMinTile + 1;
    DevBuf d;
    hipError_t e;
    if ((e = d.alloc(sizeof(int64_t) * ng)) != hipSuccess) return e;
    std::vector<int64_t> g(ng);
    const unsigned blocks = (unsigned)((ng + 255) / 256);
    if (s.ts_kind == EPI_TS_I64) {
        k_sample_times<int64_t><<<blocks, 256, 0, st>>>(s.times.as<int64_t>(), s.n, kMinTile, ng, d.as<int64_t>());
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(g.data(), d.p, 8 * ng, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    } else {
        std::vector<int32_t> g32(ng);
        k_sample_times<int32_t><<<blocks, 256, 0, st>>>(s.times.as<int32_t>(), s.n, kMinTile, ng, d.as<int32_t>());
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(g32.data(), d.p, 4 * ng, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        for (int64_t i = 0; i < ng; ++i) g[i] = g32[i];
    }
    // the last sample is the last time (index n - 1)
    for (int64_t bound : {(int64_t(1) << 29) - 1, int64_t(1) << 30}) {
        for (int T = cap; T >= kMinTile; T /= 2) {
            if (longest_tile(g, s.n, T) < bound) {
                s.T = T;
                return hipSuccess;
            }
        }
    }
    return hipSuccess;
}

}  // namespace

hipError_t build_type_index(Stream &s, hipStream_t st) {
    hipError_t e;
    const int64_t n = s.n;
    const int32_t K = s.K;
    if ((e = pick_tile(s, st)) != hipSuccess) return e;
    const int TT = s.T;
    const int64_t B = n > 0 ? (n + TT - 1) / TT : 0;
    s.B = B;
    if ((e = s.type_off.alloc(sizeof(int32_t) * (K + 1))) != hipSuccess) return e;
    if ((e = s.ts_by_type.alloc(s.ts_bytes() * (size_t)n)) != hipSuccess) return e;
    if ((e = s.pos_by_type.alloc(sizeof(int32_t) * (size_t)n)) != hipSuccess) return e;
    if ((e = s.tiled_ts.alloc(s.ts_bytes() * (size_t)B * TT)) != hipSuccess) return e;
    if ((e = s.tile_loff.alloc(sizeof(uint16_t) * (size_t)B * (K + 1))) != hipSuccess) return e;
    if ((e = s.tile_t0.alloc(s.ts_bytes() * (size_t)(B + 1))) != hipSuccess) return e;
    const int64_t Bc = B > 0 ? B : 1;
    const int64_t len = Bc * K;
    DevBuf cnt, base, sums;
    const int64_t nb = (len + kScanTile - 1) / kScanTile;
    if ((e = cnt.alloc(sizeof(int32_t) * len)) != hipSuccess) return e;
    if ((e = base.alloc(sizeof(int32_t) * len)) != hipSuccess) return e;
    if ((e = sums.alloc(sizeof(int32_t) * nb)) != hipSuccess) return e;
    if (n > 0) {
        k_hist<<<B, kWave, 0, st>>>(s.types.as<int32_t>(), n, K, TT, B, cnt.as<int32_t>());
    } else {
        if ((e = hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * len, st)) != hipSuccess) return e;
    }
    k_scan_reduce<<<nb, kScanBlock, 0, st>>>(cnt.as<int32_t>(), len, sums.as<int32_t>());
    k_scan_sums<<<1, kScanBlock, 0, st>>>(sums.as<int32_t>(), nb);
    k_scan_apply<<<nb, kScanBlock, 0, st>>>(cnt.as<int32_t>(), len, sums.as<int32_t>(), base.as<int32_t>());
    k_offsets<<<(K + 1 + 255) / 256, 256, 0, st>>>(base.as<int32_t>(), K, Bc, n, s.type_off.as<int32_t>());
    if (n > 0) {
        if (s.ts_kind == EPI_TS_I64)
            k_scatter<int64_t><<<B, kWave, 0, st>>>(s.types.as<int32_t>(), s.times.as<int64_t>(), n, K, B,
                                                    cnt.as<int32_t>(), base.as<int32_t>(),
                                                    s.ts_by_type.as<int64_t>(), s.pos_by_type.as<int32_t>(),
                                                    s.tiled_ts.as<int64_t>(),
                                                    s.tile_loff.as<uint16_t>(), s.tile_t0.as<int64_t>(), TT);
        else
            k_scatter<int32_t><<<B, kWave, 0, st>>>(s.types.as<int32_t>(), s.times.as<int32_t>(), n, K, B,
                                                    cnt.as<int32_t>(), base.as<int32_t>(),
                                                    s.ts_by_type.as<int32_t>(), s.pos_by_type.as<int32_t>(),
                                                    s.tiled_ts.as<int32_t>(),
                                                    s.tile_loff.as<uint16_t>(), s.tile_t0.as<int32_t>(), TT);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the temporaries are freed when this returns: wait for the kernels first
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    s.h_off.resize(K + 1);
    if ((e = hipMemcpy(s.h_off.data(), s.type_off.p, sizeof(int32_t) * (K + 1), hipMemcpyDeviceToHost)) !=
        hipSuccess)
        return e;
    s.h_tile_t0.assign(B + 1, 0);
    if (B > 0) {
        if (s.ts_kind == EPI_TS_I64) {
            if ((e = hipMemcpy(s.h_tile_t0.data(), s.tile_t0.p, 8 * (B + 1), hipMemcpyDeviceToHost)) != hipSuccess)
                return e;
        } else {
            std::vector<int32_t> t32(B + 1);
            if ((e = hipMemcpy(t32.data(), s.tile_t0.p, 4 * (B + 1), hipMemcpyDeviceToHost)) != hipSuccess)
                return e;
            for (int64_t b = 0; b <= B; ++b) s.h_tile_t0[b] = t32[b];
        }
    }
    // longest tile: from its first time to the next tile's (the last tile:
    // to the last event), saturated
    s.max_tile_span = 0;
    for (int64_t b = 0; b < B; ++b) {
        const int64_t end = b + 1 < B ? s.h_tile_t0[b + 1] : s.tmax;
        const uint64_t d = (uint64_t)end - (uint64_t)s.h_tile_t0[b];
        s.max_tile_span = std::max<int64_t>(s.max_tile_span, d > (uint64_t)INT64_MAX ? INT64_MAX : (int64_t)d);
    }
    return hipSuccess;
}

}  // namespace epi
