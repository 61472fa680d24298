// Stable least-significant-digit radix sort of (64-bit key, int32 value)
// pairs on the device, 8 bits per pass, for the scheduler's orderings (the
// candidates of each launch class by predicted cost, the work items of each
// persistent launch longest first).
//
// One pass = three launches:
//   k_radix_hist     each workgroup counts the digits of its chunk of 2048
//                    keys (LDS histogram) -> hist[digit][workgroup]
//   k_radix_scan     one workgroup: exclusive scan of hist in (digit,
//                    workgroup) order -> the first output slot of every
//                    (digit, workgroup) pair
//   k_radix_scatter  each workgroup walks its chunk in order, 256 keys per
//                    round; a key's rank among equal digits of its wave comes
//                    from eight ballots (one per digit bit) and a popcount,
//                    its offset among the earlier waves of the round from a
//                    per-(wave, digit) count in LDS: equal keys keep their
//                    order, so the pass is stable.
// All launches are plain kernels on one stream (no host synchronisation),
// so a sort can be captured into a graph.
#include "epi_sort.h"

namespace epi {

namespace {

constexpr int kThreads = 256;
constexpr int kRounds = kSortChunk / kThreads;
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint64_t *__restrict__ key, int64_t n, int shift,
                                                         uint32_t *__restrict__ hist, int64_t nblk) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortChunk;
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = base + r * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(key[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of total (< 2^32) counts in place, by one workgroup.
__global__ __launch_bounds__(kScanThreads) void k_radix_scan(uint32_t *__restrict__ hist, int64_t total) {
    __shared__ uint32_t part[kScanThreads];
    const int t = threadIdx.x;
    const int64_t per = (total + kScanThreads - 1) / kScanThreads;
    const int64_t lo = (int64_t)t * per;
    const int64_t hi = lo + per < total ? lo + per : total;
    uint32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += hist[i];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const uint32_t v = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = t > 0 ? part[t - 1] : 0u;
    for (int64_t i = lo; i < hi; ++i) {
        const uint32_t v = hist[i];
        hist[i] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kThreads) void k_radix_scatter(const uint64_t *__restrict__ kin,
                                                            const int32_t *__restrict__ vin,
                                                            uint64_t *__restrict__ kout, int32_t *__restrict__ vout,
                                                            int64_t n, int shift, const uint32_t *__restrict__ hist,
                                                            int64_t nblk) {
    constexpr int kWaves = kThreads / 64;
    __shared__ uint32_t run[256];          // next output slot of each digit for this chunk
    __shared__ uint32_t wcnt[kWaves][256]; // per wave: digit counts, then first slots
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    run[t] = hist[(int64_t)t * nblk + blockIdx.x];
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wcnt[w][t] = 0;
    __syncthreads();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));  // lanes before this one
    const int64_t base = (int64_t)blockIdx.x * kSortChunk;
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = base + r * kThreads + t;
        const bool ok = i < n;
        const uint64_t k = ok ? kin[i] : 0ull;
        const int32_t v = ok ? vin[i] : 0;
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        uint64_t same = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            same &= bit ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(same & below);
        if (ok && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(same);
        __syncthreads();
        {
            uint32_t s = run[t];
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t c = wcnt[w][t];
                wcnt[w][t] = s;
                s += c;
            }
            run[t] = s;
        }
        __syncthreads();
        if (ok) {
            const uint32_t pos = wcnt[wave][d] + rank;
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < kWaves; ++w) wcnt[w][t] = 0;
        __syncthreads();
    }
}

}  // namespace

int64_t radix_hist_words(int64_t n) { return 256 * std::max<int64_t>(1, (n + kSortChunk - 1) / kSortChunk); }

hipError_t radix_sort(uint64_t *k0, int32_t *v0, uint64_t *k1, int32_t *v1, int64_t n, const int *shifts, int npass,
                      uint32_t *hist, hipStream_t st, bool *in_second) {
    *in_second = false;
    if (n <= 0 || npass <= 0) return hipSuccess;
    if (n >= (int64_t(1) << 32)) return hipErrorInvalidValue;
    const int64_t nblk = (n + kSortChunk - 1) / kSortChunk;
    uint64_t *ka = k0, *kb = k1;
    int32_t *va = v0, *vb = v1;
    for (int p = 0; p < npass; ++p) {
        k_radix_hist<<<(unsigned)nblk, kThreads, 0, st>>>(ka, n, shifts[p], hist, nblk);
        k_radix_scan<<<1, kScanThreads, 0, st>>>(hist, 256 * nblk);
        k_radix_scatter<<<(unsigned)nblk, kThreads, 0, st>>>(ka, va, kb, vb, n, shifts[p], hist, nblk);
        std::swap(ka, kb);
        std::swap(va, vb);
        *in_second = !*in_second;
    }
    return hipGetLastError();
}

}  // namespace epi
