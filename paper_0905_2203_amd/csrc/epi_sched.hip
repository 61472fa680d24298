// Scheduler inputs: the cost-model features of each candidate episode.
//
// Features (kFeatures = 24), from the stream's per-type event counts and the
// episode's constraints, in stream time units:
//   [0..7]   log1p(number of events of node j's type), 0 for absent nodes
//   [8..14]  log1p(hi_j - lo_j) (window width of constraint j), 0 if absent
//   [15..21] log1p(hi_j), 0 if absent
//   [22]     N
//   [23]     log1p(sum over the nodes of their types' event counts): the
//            events a lane visits, which the per-node features give only
//            through a sum of exponentials the network would have to learn
// The number of events a lane visits grows with the first group, and the
// number of partial occurrences it tracks with the window widths and
// offsets (the runtime of Sec. V-C grows with episode frequency and length).
#include "epi_internal.h"

namespace epi {

namespace {

template <typename T>
__global__ void k_features(const int32_t *__restrict__ type_off, const int32_t *__restrict__ ctypes,
                           const T *__restrict__ clo, const T *__restrict__ chi, const int32_t *__restrict__ orig,
                           int64_t m, const uint8_t *__restrict__ Nof, float *__restrict__ X) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= m) return;
    const int N = Nof[s];
    float *x = X + s * kFeatures;
    int64_t visits = 0;
    for (int k = 0; k < 8; ++k) {
        float v = 0.f;
        if (k < N) {
            const int32_t ty = ctypes[(int64_t)k * m + s];
            const int32_t n_ty = type_off[ty + 1] - type_off[ty];
            visits += n_ty;
            v = log1pf((float)n_ty);
        }
        x[k] = v;
    }
    for (int k = 0; k < 7; ++k) {
        float w = 0.f, h = 0.f;
        if (k + 1 < N) {
            const T lo = clo[(int64_t)k * m + s], hi = chi[(int64_t)k * m + s];
            w = log1pf((float)(hi - lo));
            h = log1pf((float)hi);
        }
        x[8 + k] = w;
        x[15 + k] = h;
    }
    x[22] = (float)N;
    x[23] = log1pf((float)visits);
}

}  // namespace

hipError_t candidate_features(const Stream &s, const CandSet &c, float *dX, hipStream_t st) {
    hipError_t e;
    // episode size per grouped slot
    std::vector<uint8_t> hN(c.m);
    for (const Group &g : c.groups)
        for (int64_t i = g.begin; i < g.end; ++i) hN[i] = (uint8_t)g.N;
    DevBuf dN;
    if ((e = dN.alloc(c.m)) != hipSuccess) return e;
    if (c.m == 0) return hipSuccess;
    if ((e = hipMemcpyAsync(dN.p, hN.data(), c.m, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
    const unsigned blocks = (unsigned)((c.m + 255) / 256);
    if (s.ts_kind == EPI_TS_I64)
        k_features<int64_t><<<blocks, 256, 0, st>>>(s.type_off.as<int32_t>(), c.types.as<int32_t>(), c.lo.as<int64_t>(),
                                                    c.hi.as<int64_t>(), c.orig.as<int32_t>(), c.m, dN.as<uint8_t>(), dX);
    else
        k_features<int32_t><<<blocks, 256, 0, st>>>(s.type_off.as<int32_t>(), c.types.as<int32_t>(), c.lo.as<int32_t>(),
                                                    c.hi.as<int32_t>(), c.orig.as<int32_t>(), c.m, dN.as<uint8_t>(), dX);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipStreamSynchronize(st);  // dN dies here
}

}  // namespace epi
