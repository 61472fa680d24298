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
#include "epi_count.h"

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

// ---------------------------------------------------------------------------
// Device scheduler of the batched count: every step from the candidates to
// the ordered work items runs in kernels on one stream (captured with the
// count into the batched graph, so a replay re-predicts and re-orders).
//
//   k_sched_features / k_sched_cost  a cost per candidate: the cost model's
//       features (learned), the summed event counts of its types (heuristic)
//       or its own logged work (measured), over all sets of the count
//   k_sched_keys     key = (launch group << 32) | ~bits(cost): sorting the
//       keys ascending orders each group's candidates by descending cost and
//       keeps every group on its own slots (costs are >= 0, so their float
//       bits order like the values)
//   (radix sort)     -> per set, the lane-slot -> candidate-slot permutation
//   k_item_keys      work item (unit, lane block, segment) cost = the block's
//       first (costliest) candidate x its lanes / the unit's segments; key =
//       (launch class rank << 32) | ~bits(cost)
//   (radix sort)     -> each class's items longest first
//   k_gather_items   the work items in that order
// ---------------------------------------------------------------------------
namespace epi {

namespace {

__device__ __forceinline__ uint32_t cost_key(float c) {
    if (!(c >= 0.f)) c = 0.f;  // NaN and negatives: cheapest
    return ~__float_as_uint(c);
}

__device__ __forceinline__ float key_cost(uint64_t k) { return __uint_as_float(~(uint32_t)k); }

template <typename T>
__global__ void k_sched_features(const SchedSet *__restrict__ sets, const SchedGroup *__restrict__ groups,
                                 const int32_t *__restrict__ gid, int64_t M, float *__restrict__ X) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= M) return;
    const SchedGroup gr = groups[gid[g]];
    const SchedSet st = sets[gr.set];
    const int64_t s = g - st.off, m = st.m;
    const int N = gr.N;
    const T *clo = static_cast<const T *>(st.clo), *chi = static_cast<const T *>(st.chi);
    float *x = X + g * kFeatures;
    int64_t visits = 0;
    for (int k = 0; k < 8; ++k) {
        float v = 0.f;
        if (k < N) {
            const int32_t ty = st.ctypes[(int64_t)k * m + s];
            const int32_t n_ty = st.type_off[ty + 1] - st.type_off[ty];
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

__global__ void k_sched_cost(const SchedSet *__restrict__ sets, const SchedGroup *__restrict__ groups,
                             const int32_t *__restrict__ gid, int64_t M, int measured, float *__restrict__ y) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= M) return;
    const SchedGroup gr = groups[gid[g]];
    const SchedSet st = sets[gr.set];
    const int64_t s = g - st.off;
    if (measured) {
        y[g] = st.measured ? st.measured[s] : 0.f;
        return;
    }
    int64_t v = 0;
    for (int k = 0; k < gr.N; ++k) {
        const int32_t ty = st.ctypes[(int64_t)k * st.m + s];
        v += st.type_off[ty + 1] - st.type_off[ty];
    }
    y[g] = (float)v;
}

__global__ void k_sched_keys(const SchedSet *__restrict__ sets, const SchedGroup *__restrict__ groups,
                             const int32_t *__restrict__ gid, int64_t M, const float *__restrict__ y, int log_cost,
                             uint64_t *__restrict__ key, int32_t *__restrict__ val) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= M) return;
    const int32_t gi = gid[g];
    float c = y[g];
    if (log_cost) c = expf(fminf(c, 60.f));  // the model predicts log1p(work)
    key[g] = ((uint64_t)(uint32_t)gi << 32) | cost_key(c);
    val[g] = (int32_t)(g - sets[groups[gi].set].off);
}

__global__ void k_item_keys(const WorkItem *__restrict__ tmpl, int64_t n, const SchedUnit *__restrict__ units,
                            const uint64_t *__restrict__ skey, uint64_t *__restrict__ key, int32_t *__restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const WorkItem w = tmpl[i];
    const SchedUnit u = units[w.unit];
    const int64_t first = w.blk * u.W;
    const int64_t lanes = u.G - first < u.W ? u.G - first : u.W;
    const float c = key_cost(skey[u.gbase + first]) * (float)lanes / (float)u.P;
    key[i] = ((uint64_t)(uint32_t)u.cls << 32) | cost_key(c);
    val[i] = (int32_t)i;
}

__global__ void k_gather_items(const WorkItem *__restrict__ tmpl, const int32_t *__restrict__ idx, int64_t n,
                               WorkItem *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = tmpl[idx[i]];
}

__global__ void k_measured(const int32_t *__restrict__ work, const int32_t *__restrict__ orig, int64_t m,
                           float *__restrict__ out) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= m) return;
    const int32_t *x = work + (int64_t)orig[s] * kWork;
    out[s] = (float)x[0] + (float)x[1] + (float)x[2];
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t sched_costs(int ts_kind, int sched, const SchedSet *sets, const SchedGroup *groups, const int32_t *gid,
                       int64_t M, Mlp &mlp, float *X, float *y, hipStream_t st) {
    if (M <= 0) return hipSuccess;
    if (sched == EPI_SCHED_LEARNED) {
        if (ts_kind == EPI_TS_I64) k_sched_features<int64_t><<<nblocks(M), 256, 0, st>>>(sets, groups, gid, M, X);
        else k_sched_features<int32_t><<<nblocks(M), 256, 0, st>>>(sets, groups, gid, M, X);
        hipError_t e;
        if ((e = hipGetLastError()) != hipSuccess) return e;
        return costmodel_predict_device(mlp, X, M, y, st);
    }
    k_sched_cost<<<nblocks(M), 256, 0, st>>>(sets, groups, gid, M, sched == EPI_SCHED_MEASURED ? 1 : 0, y);
    return hipGetLastError();
}

hipError_t sched_keys(const SchedSet *sets, const SchedGroup *groups, const int32_t *gid, int64_t M, const float *y,
                      bool log_cost, uint64_t *key, int32_t *val, hipStream_t st) {
    if (M <= 0) return hipSuccess;
    k_sched_keys<<<nblocks(M), 256, 0, st>>>(sets, groups, gid, M, y, log_cost ? 1 : 0, key, val);
    return hipGetLastError();
}

hipError_t sched_item_keys(const WorkItem *tmpl, int64_t n, const SchedUnit *units, const uint64_t *skey,
                           uint64_t *key, int32_t *val, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_item_keys<<<nblocks(n), 256, 0, st>>>(tmpl, n, units, skey, key, val);
    return hipGetLastError();
}

hipError_t sched_gather_items(const WorkItem *tmpl, const int32_t *idx, int64_t n, WorkItem *out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_gather_items<<<nblocks(n), 256, 0, st>>>(tmpl, idx, n, out);
    return hipGetLastError();
}

hipError_t measured_costs(const CandSet &c, hipStream_t st) {
    if (c.m <= 0) return hipSuccess;
    k_measured<<<nblocks(c.m), 256, 0, st>>>(c.work.as<int32_t>(), c.orig.as<int32_t>(), c.m, c.dmeasured.as<float>());
    return hipGetLastError();
}

}  // namespace epi
