// C ABI of the episode-counting engine: contexts, validation, stream and
// candidate ingest, counting and readback.  Kernels live in epi_index.hip
// (per-type index) and epi_tiled.hip (counting and reconciliation).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>

#include "epi_count.h"

using namespace epi;

struct epi_ctx {
    Ctx c;
};

namespace {

thread_local std::string g_create_err;

epi_status fail(epi_ctx *ctx, epi_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->c.err = buf;
    return code;
}

epi_status hipfail(epi_ctx *ctx, hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(ctx, EPI_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(ctx, EPI_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPTRY(ctx, expr, what)                          \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hipfail(ctx, e_, what); \
    } while (0)

template <typename T>
epi_status check_stream_t(const int32_t *types, const T *times, int64_t n, int32_t K, std::string *msg) {
    for (int64_t i = 0; i < n; ++i) {
        if (types[i] < 0 || types[i] >= K) {
            if (msg) *msg = "event " + std::to_string(i) + " has type " + std::to_string(types[i]) + " outside [0, K)";
            return EPI_ETYPE;
        }
        if (times[i] == TsLimits<T>::lo() || times[i] == TsLimits<T>::hi()) {
            if (msg) *msg = "event " + std::to_string(i) + " uses a reserved timestamp (type minimum or maximum)";
            return EPI_EOVERFLOW;
        }
        if (i > 0 && times[i] < times[i - 1]) {
            if (msg) *msg = "times decrease at event " + std::to_string(i);
            return EPI_EUNSORTED;
        }
    }
    return EPI_OK;
}

epi_status check_stream(const int32_t *types, const void *times, int64_t n, int ts_kind, int32_t K,
                        std::string *msg) {
    if (ts_kind != EPI_TS_I32 && ts_kind != EPI_TS_I64) {
        if (msg) *msg = "ts_kind must be EPI_TS_I32 or EPI_TS_I64";
        return EPI_EINVAL;
    }
    if (n < 0 || n >= (int64_t(1) << 31)) {
        if (msg) *msg = "n must be in [0, 2^31)";
        return EPI_ESIZE;
    }
    if (K < 1 || K > kMaxK) {
        if (msg) *msg = "K must be in [1, " + std::to_string(kMaxK) + "]";
        return EPI_ESIZE;
    }
    if (n > 0 && (!types || !times)) {
        if (msg) *msg = "null stream pointer";
        return EPI_EINVAL;
    }
    if (ts_kind == EPI_TS_I64) return check_stream_t(types, (const int64_t *)times, n, K, msg);
    return check_stream_t(types, (const int32_t *)times, n, K, msg);
}

// Sum of the upper bounds of candidate c (its longest possible span), or -1
// on overflow.
int64_t span_of(int N, const int64_t *hi) {
    int64_t s = 0;
    for (int j = 0; j + 1 < N; ++j) {
        if (hi[j] > INT64_MAX - s) return -1;
        s += hi[j];
    }
    return s;
}

// repeats: accept a type at several nodes of an episode (EPI_OPT_ALLOW_REPEATS)
epi_status check_candidates(int64_t m, const uint8_t *N, const int32_t *types, const int64_t *lo,
                            const int64_t *hi, int32_t K, int ts_kind, std::string *msg, bool repeats = false) {
    if (ts_kind != EPI_TS_I32 && ts_kind != EPI_TS_I64) {
        if (msg) *msg = "ts_kind must be EPI_TS_I32 or EPI_TS_I64";
        return EPI_EINVAL;
    }
    if (m < 0 || m >= (int64_t(1) << 31)) {
        if (msg) *msg = "m must be in [0, 2^31)";
        return EPI_ESIZE;
    }
    if (m > 0 && (!N || !types || !lo || !hi)) {
        if (msg) *msg = "null candidate pointer";
        return EPI_EINVAL;
    }
    const int64_t tmax = ts_kind == EPI_TS_I64 ? INT64_MAX : INT32_MAX;
    for (int64_t c = 0; c < m; ++c) {
        const int n = N[c];
        auto say = [&](const std::string &s) {
            if (msg) *msg = "candidate " + std::to_string(c) + ": " + s;
        };
        if (n < 1 || n > kMaxN) {
            say("size must be in 1..8");
            return EPI_ESIZE;
        }
        const int32_t *ty = types + c * kMaxN;
        for (int j = 0; j < n; ++j) {
            if (ty[j] < 0 || ty[j] >= K) {
                say("type outside [0, K)");
                return EPI_ETYPE;
            }
            for (int k = 0; k < j && !repeats; ++k)
                if (ty[k] == ty[j]) {
                    say("repeated event type");
                    return EPI_EREPEAT;
                }
        }
        const int64_t *l = lo + c * (kMaxN - 1), *h = hi + c * (kMaxN - 1);
        for (int j = 0; j + 1 < n; ++j) {
            if (!(0 <= l[j] && l[j] < h[j])) {
                say("interval must satisfy 0 <= lo < hi");
                return EPI_EINTERVAL;
            }
        }
        const int64_t sp = span_of(n, h);
        if (sp < 0 || sp >= tmax) {
            say("episode span overflows the timestamp type");
            return EPI_EOVERFLOW;
        }
    }
    return EPI_OK;
}

// An episode with an interval whose ring bound exceeds kLaneMaxQ is "deep":
// the state machines do not take it; the per-event tracking engine, which
// keeps no rings, counts it in every mode.
bool is_deep(int N, const int64_t *lo, const int64_t *hi) {
    for (int j = 0; j + 1 < N; ++j)
        if (queue_bound(lo[j], hi[j]) > kLaneMaxQ) return true;
    return false;
}

template <typename T>
hipError_t upload_candidates(CandSet &cs, int64_t m, const uint8_t *N, const int32_t *types, const int64_t *lo,
                             const int64_t *hi, hipStream_t st) {
    // launch class of each candidate: (N, ring entries class); deep ones last
    constexpr int kDeepKey = 1 << 20;
    std::vector<int> key(m);
    for (int64_t c = 0; c < m; ++c) {
        if (is_deep(N[c], lo + c * 7, hi + c * 7)) {
            key[c] = kDeepKey;
            continue;
        }
        key[c] = N[c] * 64 + cap_class_index(std::max(1, lane_ring_entries(N[c], lo + c * 7, hi + c * 7)));
    }
    std::vector<int32_t> order(m);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    std::vector<int32_t> h_types((size_t)kMaxN * m, 0);
    std::vector<T> h_lo((size_t)(kMaxN - 1) * m, 0), h_hi((size_t)(kMaxN - 1) * m, 0);
    cs.groups.clear();
    for (int64_t s = 0; s < m; ++s) {
        const int32_t c = order[s];
        for (int j = 0; j < kMaxN; ++j) h_types[(size_t)j * m + s] = j < N[c] ? types[(int64_t)c * 8 + j] : 0;
        for (int j = 0; j + 1 < kMaxN; ++j) {
            h_lo[(size_t)j * m + s] = j + 1 < N[c] ? (T)lo[(int64_t)c * 7 + j] : T(0);
            h_hi[(size_t)j * m + s] = j + 1 < N[c] ? (T)hi[(int64_t)c * 7 + j] : T(0);
        }
        if (key[c] == kDeepKey) continue;  // no group: the tracking engine counts it
        if (cs.groups.empty() || s == 0 || key[c] != key[order[s - 1]]) {
            Group g;
            g.N = N[c];
            g.Q = 1;
            g.C = 0;
            g.begin = s;
            g.end = s;
            g.hspan = 0;
            cs.groups.push_back(g);
        }
        Group &g = cs.groups.back();
        g.end = s + 1;
        int64_t sp = 0;
        for (int j = 0; j + 1 < N[c]; ++j) {
            sp += hi[(int64_t)c * 7 + j];
            g.Q = std::max<int>(g.Q, queue_class(queue_bound(lo[(int64_t)c * 7 + j], hi[(int64_t)c * 7 + j])));
        }
        g.hspan = std::max(g.hspan, sp);
        g.C = std::max(g.C, lane_ring_entries(N[c], lo + (int64_t)c * 7, hi + (int64_t)c * 7));
    }
    hipError_t e;
    if ((e = cs.types.alloc(sizeof(int32_t) * h_types.size())) != hipSuccess) return e;
    if ((e = cs.lo.alloc(sizeof(T) * h_lo.size())) != hipSuccess) return e;
    if ((e = cs.hi.alloc(sizeof(T) * h_hi.size())) != hipSuccess) return e;
    if ((e = cs.orig.alloc(sizeof(int32_t) * m)) != hipSuccess) return e;
    if ((e = cs.counts.alloc(sizeof(int32_t) * m)) != hipSuccess) return e;
    if ((e = cs.tau.alloc(sizeof(T) * m)) != hipSuccess) return e;
    if (m > 0) {
        if ((e = hipMemcpyAsync(cs.types.p, h_types.data(), sizeof(int32_t) * h_types.size(), hipMemcpyHostToDevice,
                                st)) != hipSuccess)
            return e;
        if ((e = hipMemcpyAsync(cs.lo.p, h_lo.data(), sizeof(T) * h_lo.size(), hipMemcpyHostToDevice, st)) !=
            hipSuccess)
            return e;
        if ((e = hipMemcpyAsync(cs.hi.p, h_hi.data(), sizeof(T) * h_hi.size(), hipMemcpyHostToDevice, st)) !=
            hipSuccess)
            return e;
        if ((e = hipMemcpyAsync(cs.orig.p, order.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st)) !=
            hipSuccess)
            return e;
    }
    cs.h_order = order;
    // host staging vectors die here: wait for the copies
    return hipStreamSynchronize(st);
}

epi_status check_flags(epi_ctx *ctx) {
    int32_t f[kNumFlags];
    HIPTRY(ctx, hipMemcpy(f, ctx->c.flags.p, sizeof(f), hipMemcpyDeviceToHost), "reading device flags");
    if (f[kFlagQueueOverflow] | f[kFlagUnsorted] | f[kFlagBadType] | f[kFlagBadTime]) {
        HIPTRY(ctx, hipMemset(ctx->c.flags.p, 0, sizeof(f)), "clearing device flags");
        if (f[kFlagUnsorted]) return fail(ctx, EPI_EUNSORTED, "device check: stream times decrease");
        if (f[kFlagBadType]) return fail(ctx, EPI_ETYPE, "device check: event type outside [0, K)");
        if (f[kFlagBadTime]) return fail(ctx, EPI_EOVERFLOW, "device check: reserved timestamp value in stream");
        return fail(ctx, EPI_EDEVICE, "device check: interval queue overflow (%d)", f[kFlagQueueOverflow]);
    }
    return EPI_OK;
}

Stream *find_stream(epi_ctx *ctx, int32_t id) {
    auto it = ctx->c.streams.find(id);
    return it == ctx->c.streams.end() ? nullptr : it->second.get();
}

CandSet *find_set(epi_ctx *ctx, int32_t id) {
    auto it = ctx->c.sets.find(id);
    return it == ctx->c.sets.end() ? nullptr : it->second.get();
}

hipStream_t pick_stream(epi_ctx *ctx, void *s) { return s ? (hipStream_t)s : ctx->c.stream; }

}  // namespace

extern "C" {

epi_status epi_create(int device, epi_ctx **out) {
    if (!out) return EPI_EINVAL;
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || device < 0 || device >= ndev) {
        g_create_err = std::string("no HIP device ") + std::to_string(device) + ": " +
                       (e != hipSuccess ? hipGetErrorString(e) : "index out of range");
        return EPI_EDEVICE;
    }
    if ((e = hipSetDevice(device)) != hipSuccess) {
        g_create_err = hipGetErrorString(e);
        return EPI_EDEVICE;
    }
    epi_ctx *ctx = new (std::nothrow) epi_ctx();
    if (!ctx) return EPI_ENOMEM;
    ctx->c.device = device;
    if ((e = hipStreamCreateWithFlags(&ctx->c.stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = ctx->c.flags.alloc(sizeof(int32_t) * kNumFlags)) != hipSuccess ||
        (e = hipMemset(ctx->c.flags.p, 0, sizeof(int32_t) * kNumFlags)) != hipSuccess ||
        (e = hipHostMalloc((void **)&ctx->c.stage, sizeof(int64_t) * kStageSlots, hipHostMallocDefault)) !=
            hipSuccess ||
        (e = noalloc_init(device)) != hipSuccess) {
        g_create_err = hipGetErrorString(e);
        delete ctx;
        return EPI_EDEVICE;
    }
    *out = ctx;
    return EPI_OK;
}

void epi_destroy(epi_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->c.device);
    (void)hipDeviceSynchronize();
    ctx->c.batch.clear();
    ctx->c.mines.clear();
    ctx->c.sets.clear();
    ctx->c.streams.clear();
    ctx->c.flags.reset();
    ctx->c.cache.release();
    if (ctx->c.stage) (void)hipHostFree(ctx->c.stage);
    if (ctx->c.stream) (void)hipStreamDestroy(ctx->c.stream);
    delete ctx;
}

const char *epi_last_error(const epi_ctx *ctx) { return ctx ? ctx->c.err.c_str() : g_create_err.c_str(); }

const char *epi_status_string(epi_status s) {
    switch (s) {
        case EPI_OK: return "EPI_OK";
        case EPI_EINVAL: return "EPI_EINVAL";
        case EPI_EUNSORTED: return "EPI_EUNSORTED";
        case EPI_ETYPE: return "EPI_ETYPE";
        case EPI_EINTERVAL: return "EPI_EINTERVAL";
        case EPI_ESIZE: return "EPI_ESIZE";
        case EPI_EREPEAT: return "EPI_EREPEAT";
        case EPI_EOVERFLOW: return "EPI_EOVERFLOW";
        case EPI_ENOMEM: return "EPI_ENOMEM";
        case EPI_EDEVICE: return "EPI_EDEVICE";
        case EPI_ESTATE: return "EPI_ESTATE";
        default: return "EPI_UNKNOWN";
    }
}

epi_status epi_validate_stream(const int32_t *types, const void *times, int64_t n, int ts_kind, int32_t K) {
    return check_stream(types, times, n, ts_kind, K, nullptr);
}

epi_status epi_validate_candidates(int64_t m, const uint8_t *N, const int32_t *types, const int64_t *lo,
                                   const int64_t *hi, int32_t K, int ts_kind) {
    return check_candidates(m, N, types, lo, hi, K, ts_kind, nullptr);
}

epi_status epi_load_stream(epi_ctx *ctx, const int32_t *types, const void *times, int64_t n, int ts_kind,
                           int32_t K, int32_t *stream_id) {
    if (!ctx || !stream_id) return fail(ctx, EPI_EINVAL, "null argument");
    std::string msg;
    epi_status v = check_stream(types, times, n, ts_kind, K, &msg);
    if (v != EPI_OK) return fail(ctx, v, "%s", msg.c_str());
    HIPTRY(ctx, hipSetDevice(ctx->c.device), "hipSetDevice");
    auto s = std::make_unique<Stream>();
    s->n = n;
    s->K = K;
    s->ts_kind = ts_kind;
    if (n > 0) {
        s->tmin = ts_kind == EPI_TS_I64 ? ((const int64_t *)times)[0] : ((const int32_t *)times)[0];
        s->tmax = ts_kind == EPI_TS_I64 ? ((const int64_t *)times)[n - 1] : ((const int32_t *)times)[n - 1];
    }
    HIPTRY(ctx, s->types.alloc(sizeof(int32_t) * n), "allocating stream types");
    HIPTRY(ctx, s->times.alloc(s->ts_bytes() * n), "allocating stream times");
    if (n > 0) {
        HIPTRY(ctx, hipMemcpy(s->types.p, types, sizeof(int32_t) * n, hipMemcpyHostToDevice), "copying types");
        HIPTRY(ctx, hipMemcpy(s->times.p, times, s->ts_bytes() * n, hipMemcpyHostToDevice), "copying times");
    }
    HIPTRY(ctx, build_type_index(*s, ctx->c.stream), "building the per-type index");
    const int32_t id = ctx->c.next_id++;
    ctx->c.streams[id] = std::move(s);
    *stream_id = id;
    return EPI_OK;
}

epi_status epi_load_stream_device(epi_ctx *ctx, const int32_t *d_types, const void *d_times, int64_t n, int ts_kind,
                                  int32_t K, void *hip_stream, int32_t *stream_id) {
    if (!ctx || !stream_id) return fail(ctx, EPI_EINVAL, "null argument");
    std::string msg;
    // shape checks only; the element checks run on the device
    epi_status v = check_stream(nullptr, nullptr, 0, ts_kind, K, &msg);
    if (v != EPI_OK) return fail(ctx, v, "%s", msg.c_str());
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(ctx, EPI_ESIZE, "n must be in [0, 2^31)");
    if (n > 0 && (!d_types || !d_times)) return fail(ctx, EPI_EINVAL, "null stream pointer");
    HIPTRY(ctx, hipSetDevice(ctx->c.device), "hipSetDevice");
    hipStream_t st = pick_stream(ctx, hip_stream);
    auto s = std::make_unique<Stream>();
    s->n = n;
    s->K = K;
    s->ts_kind = ts_kind;
    HIPTRY(ctx, s->types.alloc(sizeof(int32_t) * n), "allocating stream types");
    HIPTRY(ctx, s->times.alloc(s->ts_bytes() * n), "allocating stream times");
    if (n > 0) {
        HIPTRY(ctx, hipMemcpyAsync(s->types.p, d_types, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st),
               "copying types");
        HIPTRY(ctx, hipMemcpyAsync(s->times.p, d_times, s->ts_bytes() * n, hipMemcpyDeviceToDevice, st),
               "copying times");
        HIPTRY(ctx, validate_stream_device(s->types.as<int32_t>(), s->times.p, n, ts_kind, K,
                                           ctx->c.flags.as<int32_t>(), st),
               "validating the stream");
        HIPTRY(ctx, hipStreamSynchronize(st), "validating the stream");
        epi_status f = check_flags(ctx);
        if (f != EPI_OK) return f;
        int64_t ends[2] = {0, 0};
        if (ts_kind == EPI_TS_I64) {
            HIPTRY(ctx, hipMemcpy(&ends[0], s->times.as<int64_t>(), 8, hipMemcpyDeviceToHost), "reading times");
            HIPTRY(ctx, hipMemcpy(&ends[1], s->times.as<int64_t>() + (n - 1), 8, hipMemcpyDeviceToHost),
                   "reading times");
        } else {
            int32_t a = 0, b = 0;
            HIPTRY(ctx, hipMemcpy(&a, s->times.as<int32_t>(), 4, hipMemcpyDeviceToHost), "reading times");
            HIPTRY(ctx, hipMemcpy(&b, s->times.as<int32_t>() + (n - 1), 4, hipMemcpyDeviceToHost), "reading times");
            ends[0] = a;
            ends[1] = b;
        }
        s->tmin = ends[0];
        s->tmax = ends[1];
    }
    HIPTRY(ctx, build_type_index(*s, st), "building the per-type index");
    const int32_t id = ctx->c.next_id++;
    ctx->c.streams[id] = std::move(s);
    *stream_id = id;
    return EPI_OK;
}

epi_status epi_stream_info(epi_ctx *ctx, int32_t stream_id, int64_t *n, int32_t *K, int *ts_kind) {
    if (!ctx) return EPI_EINVAL;
    Stream *s = find_stream(ctx, stream_id);
    if (!s) return fail(ctx, EPI_ESTATE, "unknown stream id %d", stream_id);
    if (n) *n = s->n;
    if (K) *K = s->K;
    if (ts_kind) *ts_kind = s->ts_kind;
    return EPI_OK;
}

epi_status epi_read_type_index(epi_ctx *ctx, int32_t stream_id, int32_t *off, void *ts_by_type) {
    if (!ctx || !off || !ts_by_type) return fail(ctx, EPI_EINVAL, "null argument");
    Stream *s = find_stream(ctx, stream_id);
    if (!s) return fail(ctx, EPI_ESTATE, "unknown stream id %d", stream_id);
    HIPTRY(ctx, hipStreamSynchronize(ctx->c.stream), "sync");
    HIPTRY(ctx, hipMemcpy(off, s->type_off.p, sizeof(int32_t) * (s->K + 1), hipMemcpyDeviceToHost), "copy");
    if (s->n > 0)
        HIPTRY(ctx, hipMemcpy(ts_by_type, s->ts_by_type.p, s->ts_bytes() * s->n, hipMemcpyDeviceToHost), "copy");
    return EPI_OK;
}

epi_status epi_release_stream(epi_ctx *ctx, int32_t stream_id) {
    if (!ctx) return EPI_EINVAL;
    if (!find_stream(ctx, stream_id)) return fail(ctx, EPI_ESTATE, "unknown stream id %d", stream_id);
    for (auto &kv : ctx->c.sets)
        if (kv.second->stream_id == stream_id)
            return fail(ctx, EPI_ESTATE, "stream %d still has candidate set %d", stream_id, kv.first);
    ctx->c.batch.evict_all();
    (void)hipDeviceSynchronize();
    ctx->c.streams.erase(stream_id);
    return EPI_OK;
}

epi_status epi_submit_candidates(epi_ctx *ctx, int32_t stream_id, int64_t m, const uint8_t *N, const int32_t *types,
                                 const int64_t *lo, const int64_t *hi, int32_t *set_id) {
    if (!ctx || !set_id) return fail(ctx, EPI_EINVAL, "null argument");
    Stream *s = find_stream(ctx, stream_id);
    if (!s) return fail(ctx, EPI_ESTATE, "unknown stream id %d", stream_id);
    std::string msg;
    epi_status v = check_candidates(m, N, types, lo, hi, s->K, s->ts_kind, &msg, ctx->c.opt.allow_repeats);
    if (v != EPI_OK) return fail(ctx, v, "%s", msg.c_str());
    // times +- span must stay strictly inside the timestamp type
    const int64_t tlo = s->ts_kind == EPI_TS_I64 ? INT64_MIN : INT32_MIN;
    const int64_t thi = s->ts_kind == EPI_TS_I64 ? INT64_MAX : INT32_MAX;
    int64_t max_span = 0;
    for (int64_t c = 0; c < m; ++c) {
        const int64_t sp = span_of(N[c], hi + c * 7);
        max_span = std::max(max_span, sp);
        if (s->n > 0 && (s->tmax > thi - 1 - sp || s->tmin < tlo + 1 + sp))
            return fail(ctx, EPI_EOVERFLOW, "candidate %lld: stream times +- its span leave the timestamp type",
                        (long long)c);
    }
    HIPTRY(ctx, hipSetDevice(ctx->c.device), "hipSetDevice");
    auto cs = std::make_unique<CandSet>();
    cs->stream_id = stream_id;
    cs->m = m;
    hipError_t e = s->ts_kind == EPI_TS_I64 ? upload_candidates<int64_t>(*cs, m, N, types, lo, hi, ctx->c.stream)
                                            : upload_candidates<int32_t>(*cs, m, N, types, lo, hi, ctx->c.stream);
    if (e != hipSuccess) return hipfail(ctx, e, "uploading candidates");
    cs->stream_order = ctx->c.opt.stream_order;
    cs->max_span = max_span;
    {
        // deep episodes: a sub-set counted by the tracking engine
        std::vector<int32_t> didx;
        for (int64_t c = 0; c < m; ++c)
            if (is_deep(N[c], lo + c * 7, hi + c * 7)) didx.push_back((int32_t)c);
        if (!didx.empty()) {
            auto d = std::make_unique<CandSet>();
            const int64_t md = (int64_t)didx.size();
            d->stream_id = stream_id;
            d->m = md;
            for (int32_t c : didx) {
                d->h_N.push_back(N[c]);
                d->h_types.insert(d->h_types.end(), types + (int64_t)c * kMaxN, types + (int64_t)(c + 1) * kMaxN);
                d->h_lo.insert(d->h_lo.end(), lo + (int64_t)c * (kMaxN - 1), lo + (int64_t)(c + 1) * (kMaxN - 1));
                d->h_hi.insert(d->h_hi.end(), hi + (int64_t)c * (kMaxN - 1), hi + (int64_t)(c + 1) * (kMaxN - 1));
            }
            HIPTRY(ctx, d->counts.alloc(sizeof(int32_t) * md), "deep episodes");
            HIPTRY(ctx, d->tau.alloc(s->ts_bytes() * md), "deep episodes");
            HIPTRY(ctx, cs->deep_idx.alloc(sizeof(int32_t) * md), "deep episodes");
            HIPTRY(ctx, hipMemcpy(cs->deep_idx.p, didx.data(), sizeof(int32_t) * md, hipMemcpyHostToDevice),
                   "deep episodes");
            cs->deep = std::move(d);
        }
    }
    cs->h_N.assign(N, N + m);
    cs->h_types.assign(types, types + m * kMaxN);
    cs->h_lo.assign(lo, lo + m * (kMaxN - 1));
    cs->h_hi.assign(hi, hi + m * (kMaxN - 1));
    const int32_t id = ctx->c.next_id++;
    ctx->c.sets[id] = std::move(cs);
    *set_id = id;
    return EPI_OK;
}

epi_status epi_release_set(epi_ctx *ctx, int32_t set_id) {
    if (!ctx) return EPI_EINVAL;
    if (!find_set(ctx, set_id)) return fail(ctx, EPI_ESTATE, "unknown set id %d", set_id);
    ctx->c.batch.evict_set(set_id);
    (void)hipDeviceSynchronize();
    ctx->c.sets.erase(set_id);
    return EPI_OK;
}

epi_status epi_count(epi_ctx *ctx, const int32_t *set_ids, int32_t k, int mode, int sched, void *hip_stream) {
    if (!ctx) return EPI_EINVAL;
    if (k < 0 || (k > 0 && !set_ids)) return fail(ctx, EPI_EINVAL, "bad set list");
    if (mode != EPI_MODE_PLAIN && mode != EPI_MODE_BATCHED && mode != EPI_MODE_INCREMENTAL &&
        mode != EPI_MODE_TRACKING)
        return fail(ctx, EPI_EINVAL, "unknown mode %d", mode);
    if (sched != EPI_SCHED_RR && sched != EPI_SCHED_LEARNED && sched != EPI_SCHED_HEURISTIC &&
        sched != EPI_SCHED_MEASURED)
        return fail(ctx, EPI_EINVAL, "unknown sched %d", sched);
    for (int32_t i = 0; i < k; ++i) {
        CandSet *cs = find_set(ctx, set_ids[i]);
        if (!cs) return fail(ctx, EPI_ESTATE, "unknown set id %d", set_ids[i]);
        if (cs->stream_order && mode != EPI_MODE_TRACKING)
            return fail(ctx, EPI_EINVAL, "set %d decides overlap in stream order: count it with EPI_MODE_TRACKING",
                        set_ids[i]);
        if (mode == EPI_MODE_BATCHED && sched == EPI_SCHED_MEASURED && !(cs->counted && cs->logged) &&
            !cs->has_measured)
            return fail(ctx, EPI_ESTATE, "set %d has no work log to schedule by", set_ids[i]);
    }
    HIPTRY(ctx, hipSetDevice(ctx->c.device), "hipSetDevice");
    hipStream_t st = pick_stream(ctx, hip_stream);
    if (mode == EPI_MODE_INCREMENTAL) {
        // sets never counted: a full count; sets counted before an append:
        // only the occurrences the appended events complete
        for (int32_t i = 0; i < k; ++i) {
            CandSet *cs = find_set(ctx, set_ids[i]);
            if (cs->compact) return fail(ctx, EPI_EINVAL, "set %d cannot be counted incrementally", set_ids[i]);
        }
        for (int32_t i = 0; i < k; ++i) {
            CandSet *cs = find_set(ctx, set_ids[i]);
            Stream *s = find_stream(ctx, cs->stream_id);
            cs->logged = false;
            if (!cs->counted || cs->counted_n < 0) {
                HIPTRY(ctx, launch_count(*s, *cs, ctx->c.opt, ctx->c.flags.as<int32_t>(), st), "launching the count");
                HIPTRY(ctx, count_deep_subset(*s, *cs, st), "counting deep episodes");
            } else if (cs->counted_n < s->n && cs->m > 0) {
                int64_t B = 0;
                if (s->ts_kind == EPI_TS_I64) {
                    HIPTRY(ctx, hipMemcpy(&B, s->times.as<int64_t>() + cs->counted_n, 8, hipMemcpyDeviceToHost),
                           "reading times");
                } else {
                    int32_t b32 = 0;
                    HIPTRY(ctx, hipMemcpy(&b32, s->times.as<int32_t>() + cs->counted_n, 4, hipMemcpyDeviceToHost),
                           "reading times");
                    B = b32;
                }
                HIPTRY(ctx, launch_count_append(*s, *cs, B, ctx->c.flags.as<int32_t>(), st), "counting appended events");
                // deep episodes: counted again over the whole stream
                HIPTRY(ctx, count_deep_subset(*s, *cs, st), "counting deep episodes");
            }
            cs->counted = true;
            cs->counted_n = s->n;
        }
        return EPI_OK;
    }
    if (mode == EPI_MODE_TRACKING) {
        for (int32_t i = 0; i < k; ++i)
            if (find_set(ctx, set_ids[i])->compact)
                return fail(ctx, EPI_EINVAL, "set %d cannot be counted by tracking", set_ids[i]);
        for (int32_t i = 0; i < k; ++i) {
            CandSet *cs = find_set(ctx, set_ids[i]);
            Stream *s = find_stream(ctx, cs->stream_id);
            cs->logged = false;
            HIPTRY(ctx, launch_count_tracking(*s, *cs, st), "counting by tracking");
            cs->counted = true;
            cs->counted_n = s->n;
        }
        return EPI_OK;
    }
    // measured costs: the logged work, per grouped slot, taken before the log
    // is reset (kept for later counts that log nothing)
    if (mode == EPI_MODE_BATCHED && sched == EPI_SCHED_MEASURED) {
        for (int32_t i = 0; i < k; ++i) {
            CandSet *cs = find_set(ctx, set_ids[i]);
            if (!(cs->counted && cs->logged)) continue;
            if (cs->dmeasured.bytes < sizeof(float) * (size_t)std::max<int64_t>(cs->m, 1))
                HIPTRY(ctx, cs->dmeasured.alloc(sizeof(float) * std::max<int64_t>(cs->m, 1)), "measured costs");
            HIPTRY(ctx, measured_costs(*cs, st), "measured costs");
            cs->has_measured = true;
        }
    }
    // work log: cleared before the count
    for (int32_t i = 0; i < k; ++i) {
        CandSet *cs = find_set(ctx, set_ids[i]);
        cs->logged = ctx->c.opt.worklog;
        if (ctx->c.opt.worklog) {
            if (cs->work.bytes < sizeof(int32_t) * kWork * (size_t)std::max<int64_t>(cs->m, 1))
                HIPTRY(ctx, cs->work.alloc(sizeof(int32_t) * kWork * std::max<int64_t>(cs->m, 1)), "work log");
            HIPTRY(ctx, hipMemsetAsync(cs->work.p, 0, cs->work.bytes, st), "work log");
        }
    }
    if (mode == EPI_MODE_BATCHED) {
        std::vector<BatchRef> refs;
        std::vector<int32_t> ids(set_ids, set_ids + k);
        int kind = -1;
        for (int32_t i = 0; i < k; ++i) {
            CandSet *cs = find_set(ctx, set_ids[i]);
            Stream *s = find_stream(ctx, cs->stream_id);
            if (kind >= 0 && s->ts_kind != kind)
                return fail(ctx, EPI_EINVAL, "a batched count needs streams of one timestamp kind");
            kind = s->ts_kind;
            refs.push_back(BatchRef{s, cs});
        }
        HIPTRY(ctx,
               launch_count_batched(refs, ids, sched, ctx->c.opt, ctx->c.mlp, ctx->c.batch, ctx->c.flags.as<int32_t>(),
                                    st),
               "batched count");
        for (auto &r : refs) {
            HIPTRY(ctx, count_deep_subset(*r.s, *r.c, st), "counting deep episodes");
            r.c->counted = true;
            r.c->counted_n = r.s->n;
        }
        return EPI_OK;
    }
    for (int32_t i = 0; i < k; ++i) {
        CandSet *cs = find_set(ctx, set_ids[i]);
        Stream *s = find_stream(ctx, cs->stream_id);
        HIPTRY(ctx, launch_count(*s, *cs, ctx->c.opt, ctx->c.flags.as<int32_t>(), st), "launching the count");
        HIPTRY(ctx, count_deep_subset(*s, *cs, st), "counting deep episodes");
        cs->counted = true;
        cs->counted_n = s->n;
    }
    return EPI_OK;
}

epi_status epi_append_stream(epi_ctx *ctx, int32_t stream_id, const int32_t *types, const void *times, int64_t n) {
    if (!ctx) return EPI_EINVAL;
    Stream *s = find_stream(ctx, stream_id);
    if (!s) return fail(ctx, EPI_ESTATE, "unknown stream id %d", stream_id);
    std::string msg;
    epi_status v = check_stream(types, times, n, s->ts_kind, s->K, &msg);
    if (v != EPI_OK) return fail(ctx, v, "%s", msg.c_str());
    if (n == 0) return EPI_OK;
    if (s->n + n >= (int64_t(1) << 31)) return fail(ctx, EPI_ESIZE, "the stream would reach 2^31 events");
    const bool i64 = s->ts_kind == EPI_TS_I64;
    const int64_t first = i64 ? ((const int64_t *)times)[0] : ((const int32_t *)times)[0];
    const int64_t last = i64 ? ((const int64_t *)times)[n - 1] : ((const int32_t *)times)[n - 1];
    if (s->n > 0 && first < s->tmax)
        return fail(ctx, EPI_EUNSORTED, "appended times must not precede the stream's last time");
    // the stream's times +- the span of every set and mining run on it must
    // stay strictly inside the timestamp type after the append, as at
    // submission (the state machines form t + hi, the tracking engine t - hi)
    {
        const int64_t tlo = i64 ? INT64_MIN : INT32_MIN;
        const int64_t thi = i64 ? INT64_MAX : INT32_MAX;
        const int64_t nmin = s->n > 0 ? s->tmin : first;
        auto fits = [&](int64_t sp) { return !(last > thi - 1 - sp || nmin < tlo + 1 + sp); };
        for (auto &kv : ctx->c.sets)
            if (kv.second->stream_id == stream_id && !fits(kv.second->max_span))
                return fail(ctx, EPI_EOVERFLOW, "set %d: appended times +- its longest span leave the timestamp type",
                            kv.first);
        for (auto &kv : ctx->c.mines)
            if (kv.second->stream_id == stream_id && !fits(kv.second->max_span))
                return fail(ctx, EPI_EOVERFLOW,
                            "mining run %d: appended times +- its longest span leave the timestamp type", kv.first);
    }
    HIPTRY(ctx, hipSetDevice(ctx->c.device), "hipSetDevice");
    // the work queued on the stream's arrays ends before they are replaced;
    // batched plans over the old arrays are dropped
    HIPTRY(ctx, hipDeviceSynchronize(), "sync");
    ctx->c.batch.evict_all();
    const size_t tb = s->ts_bytes();
    DevBuf ty, tm;
    HIPTRY(ctx, ty.alloc(sizeof(int32_t) * (size_t)(s->n + n)), "allocating stream types");
    HIPTRY(ctx, tm.alloc(tb * (size_t)(s->n + n)), "allocating stream times");
    if (s->n > 0) {
        HIPTRY(ctx, hipMemcpy(ty.p, s->types.p, sizeof(int32_t) * s->n, hipMemcpyDeviceToDevice), "copying types");
        HIPTRY(ctx, hipMemcpy(tm.p, s->times.p, tb * s->n, hipMemcpyDeviceToDevice), "copying times");
    }
    HIPTRY(ctx, hipMemcpy(ty.as<int32_t>() + s->n, types, sizeof(int32_t) * n, hipMemcpyHostToDevice), "copying types");
    HIPTRY(ctx, hipMemcpy(tm.as<unsigned char>() + tb * s->n, times, tb * n, hipMemcpyHostToDevice), "copying times");
    s->types = std::move(ty);
    s->times = std::move(tm);
    if (s->n == 0) s->tmin = first;
    s->tmax = last;
    s->n += n;
    HIPTRY(ctx, build_type_index(*s, ctx->c.stream), "building the per-type index");
    HIPTRY(ctx, hipStreamSynchronize(ctx->c.stream), "sync");
    return EPI_OK;
}

epi_status epi_set_option(epi_ctx *ctx, int option, int64_t value) {
    if (!ctx) return EPI_EINVAL;
    switch (option) {
        case EPI_OPT_SEGMENTS:
            if (value < 0) return fail(ctx, EPI_EINVAL, "segments must be >= 0");
            ctx->c.opt.segments = value;
            return EPI_OK;
        case EPI_OPT_LANES:
            if (value != 0 && value != 64 && value != 128 && value != 256)
                return fail(ctx, EPI_EINVAL, "lanes must be 0, 64, 128 or 256");
            ctx->c.opt.lanes = (int)value;
            return EPI_OK;
        case EPI_OPT_TARGET_LANES:
            if (value < 1) return fail(ctx, EPI_EINVAL, "target lanes must be >= 1");
            ctx->c.opt.target_lanes = value;
            return EPI_OK;
        case EPI_OPT_PAIR_FILTER:
            if (value != 0 && value != 1) return fail(ctx, EPI_EINVAL, "pair filter must be 0 or 1");
            ctx->c.opt.pair_filter = value != 0;
            return EPI_OK;
        case EPI_OPT_MINE_ENGINE:
            if (value != 0 && value != 1) return fail(ctx, EPI_EINVAL, "mining engine must be 0 or 1");
            ctx->c.opt.mine_engine = (int)value;
            return EPI_OK;
        case EPI_OPT_WORKLOG:
            if (value != 0 && value != 1) return fail(ctx, EPI_EINVAL, "work log must be 0 or 1");
            ctx->c.opt.worklog = value != 0;
            return EPI_OK;
        case EPI_OPT_TARGET_ITEMS:
            if (value < 0) return fail(ctx, EPI_EINVAL, "target items must be >= 0");
            ctx->c.opt.target_items = value;
            return EPI_OK;
        case EPI_OPT_MINE_LIST_BYTES:
            if (value < 0) return fail(ctx, EPI_EINVAL, "list bytes must be >= 0");
            ctx->c.opt.mine_list_bytes = value;
            return EPI_OK;
        case EPI_OPT_MINE_LIST_ALPHAS:
            if (value < 0) return fail(ctx, EPI_EINVAL, "list alphas must be >= 0");
            ctx->c.opt.mine_list_alphas = value;
            return EPI_OK;
        case EPI_OPT_ALLOW_REPEATS:
            if (value != 0 && value != 1) return fail(ctx, EPI_EINVAL, "allow-repeats must be 0 or 1");
            ctx->c.opt.allow_repeats = value != 0;
            return EPI_OK;
        case EPI_OPT_STREAM_ORDER:
            if (value != 0 && value != 1) return fail(ctx, EPI_EINVAL, "stream order must be 0 or 1");
            ctx->c.opt.stream_order = value != 0;
            return EPI_OK;
        case EPI_OPT_LANE_ENGINE:
            if (value != 0 && value != 1) return fail(ctx, EPI_EINVAL, "lane engine must be 0 or 1");
            ctx->c.opt.lane_engine = value != 0;
            return EPI_OK;
        case EPI_OPT_RING_CLASSES:
            if (value < 0 || value > 2) return fail(ctx, EPI_EINVAL, "ring classes must be 0, 1 or 2");
            ctx->c.opt.ring_classes = (int)value;
            return EPI_OK;
        default:
            return fail(ctx, EPI_EINVAL, "unknown option %d", option);
    }
}

epi_status epi_sync(epi_ctx *ctx) {
    if (!ctx) return EPI_EINVAL;
    HIPTRY(ctx, hipSetDevice(ctx->c.device), "hipSetDevice");
    HIPTRY(ctx, hipDeviceSynchronize(), "synchronising");
    return check_flags(ctx);
}

epi_status epi_read_counts(epi_ctx *ctx, int32_t set_id, int32_t *counts, int64_t m) {
    if (!ctx) return EPI_EINVAL;
    CandSet *cs = find_set(ctx, set_id);
    if (!cs) return fail(ctx, EPI_ESTATE, "unknown set id %d", set_id);
    if (!cs->counted) return fail(ctx, EPI_ESTATE, "set %d has not been counted", set_id);
    if (m != cs->m) return fail(ctx, EPI_EINVAL, "set %d holds %lld candidates, not %lld", set_id,
                                (long long)cs->m, (long long)m);
    if (m > 0 && !counts) return fail(ctx, EPI_EINVAL, "null counts");
    epi_status f = epi_sync(ctx);
    if (f != EPI_OK) return f;
    if (m > 0) HIPTRY(ctx, hipMemcpy(counts, cs->counts.p, sizeof(int32_t) * m, hipMemcpyDeviceToHost), "copy");
    return EPI_OK;
}

epi_status epi_mine(epi_ctx *ctx, int32_t stream_id, int32_t n_menu, const int64_t *menu_lo, const int64_t *menu_hi,
                    int32_t max_size, int64_t threshold, void *hip_stream, int32_t *mine_id) {
    if (!ctx || !mine_id) return fail(ctx, EPI_EINVAL, "null argument");
    Stream *s = find_stream(ctx, stream_id);
    if (!s) return fail(ctx, EPI_ESTATE, "unknown stream id %d", stream_id);
    if (n_menu < 1 || n_menu > 255 || !menu_lo || !menu_hi)
        return fail(ctx, EPI_EINVAL, "the interval menu must hold 1..255 intervals");
    if (max_size < 1 || max_size > kMaxN) return fail(ctx, EPI_ESIZE, "max_size must be in 1..8");
    int64_t hmax = 0;
    for (int i = 0; i < n_menu; ++i) {
        if (!(0 <= menu_lo[i] && menu_lo[i] < menu_hi[i]))
            return fail(ctx, EPI_EINTERVAL, "menu interval %d must satisfy 0 <= lo < hi", i);
        // the extension engine keeps no rings; the state-machine engine (menus
        // of more than kExtMaxMenu intervals, or chosen) holds kMaxQueue
        if (queue_bound(menu_lo[i], menu_hi[i]) > kMaxQueue && (n_menu > kExtMaxMenu || ctx->c.opt.mine_engine == 0))
            return fail(ctx, EPI_EINTERVAL, "menu interval %d exceeds the state-machine engine's ring depth", i);
        hmax = std::max(hmax, menu_hi[i]);
    }
    const int64_t tlo = s->ts_kind == EPI_TS_I64 ? INT64_MIN : INT32_MIN;
    const int64_t thi = s->ts_kind == EPI_TS_I64 ? INT64_MAX : INT32_MAX;
    if (hmax > (thi / 2) / kMaxN) return fail(ctx, EPI_EOVERFLOW, "menu interval too long for the timestamp type");
    const int64_t span = hmax * (max_size - 1);
    if (s->n > 0 && (s->tmax > thi - 1 - span || s->tmin < tlo + 1 + span))
        return fail(ctx, EPI_EOVERFLOW, "stream times +- the longest span leave the timestamp type");
    HIPTRY(ctx, hipSetDevice(ctx->c.device), "hipSetDevice");
    // the levels run on the context's stream, after the work already queued
    // on the caller's; every buffer of the run comes from the context's cache
    hipStream_t st = ctx->c.stream;
    if (hip_stream && (hipStream_t)hip_stream != st) {
        hipEvent_t ev;
        HIPTRY(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
        hipError_t e = hipEventRecord(ev, (hipStream_t)hip_stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, ev, 0);
        (void)hipEventDestroy(ev);
        HIPTRY(ctx, e, "ordering after the caller's stream");
    }
    CacheScope scope(&ctx->c.cache);
    auto mn = std::make_unique<Mine>();
    mn->stream_id = stream_id;
    mn->max_span = span;
    mn->stage = ctx->c.stage;
    mn->menu_lo.assign(menu_lo, menu_lo + n_menu);
    mn->menu_hi.assign(menu_hi, menu_hi + n_menu);
    mn->threshold = threshold;
    // the extension engine takes menus of up to kExtMaxMenu intervals; longer
    // menus go to the state-machine engine
    mn->engine = n_menu <= kExtMaxMenu ? ctx->c.opt.mine_engine : 0;
    mn->list_budget = ctx->c.opt.mine_list_bytes;
    mn->list_alphas = ctx->c.opt.mine_list_alphas;
    if (mn->engine == 1) {
        // extension engine: each level extends the previous level's chain lists
        auto tb = std::chrono::steady_clock::now();
        HIPTRY(ctx, extend_prepare(*s, *mn, st), "preparing the window walk");
        mn->bits_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tb).count();
        HIPTRY(ctx, extend_level1(*s, *mn, st), "counting level 1");
        mn->levels.back().gen_ms = 0;
        for (int N = 2; N <= max_size; ++N) {
            const MineLevel &prev = mn->levels.back();
            if (prev.nf == 0 || (N == 2 && prev.nf < 2)) break;
            HIPTRY(ctx, extend_level(*s, *mn, N, st), "counting a level");
            epi_status f = check_flags(ctx);
            if (f != EPI_OK) return f;
            if (mn->levels.back().m == 0) {
                mn->levels.pop_back();
                break;
            }
        }
    } else {
        // pair-existence bitmaps of the menu (skipped when they would be too big)
        const double bits_bytes = 2.0 * 8.0 * n_menu * (double)s->K * (double)s->B * (s->T / 64);
        if (ctx->c.opt.pair_filter && max_size > 1 && s->n > 0 &&
            bits_bytes <= (double)ctx->c.opt.pair_filter_max_bytes) {
            auto tb = std::chrono::steady_clock::now();
            HIPTRY(ctx, build_pair_bits(*s, *mn, st), "building pair-existence bitmaps");
            mn->bits_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tb).count();
        }
        for (int N = 1; N <= max_size; ++N) {
            MineLevel L;
            auto t0 = std::chrono::steady_clock::now();
            if (N == 1) gen_level1(s->K, L);
            else if (N == 2) gen_level2(mn->levels.back(), n_menu, L);
            else gen_join(mn->levels.back(), L);
            L.gen_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (L.m == 0) break;
            HIPTRY(ctx, count_mine_level(*s, *mn, L, ctx->c.opt, ctx->c.flags.as<int32_t>(), st), "counting a level");
            epi_status f = check_flags(ctx);
            if (f != EPI_OK) return f;
            select_frequent(L, threshold);
            const bool none = L.freq.empty();
            mn->levels.push_back(std::move(L));
            if (none) break;
        }
    }
    const int32_t id = ctx->c.next_id++;
    ctx->c.mines[id] = std::move(mn);
    *mine_id = id;
    return EPI_OK;
}

epi_status epi_mine_levels(epi_ctx *ctx, int32_t mine_id, int32_t *n_levels) {
    if (!ctx || !n_levels) return fail(ctx, EPI_EINVAL, "null argument");
    auto it = ctx->c.mines.find(mine_id);
    if (it == ctx->c.mines.end()) return fail(ctx, EPI_ESTATE, "unknown mining id %d", mine_id);
    *n_levels = (int32_t)it->second->levels.size();
    return EPI_OK;
}

epi_status epi_mine_level_info(epi_ctx *ctx, int32_t mine_id, int32_t level, int64_t *n_candidates,
                               int64_t *n_frequent, double *times_ms) {
    if (!ctx) return EPI_EINVAL;
    auto it = ctx->c.mines.find(mine_id);
    if (it == ctx->c.mines.end()) return fail(ctx, EPI_ESTATE, "unknown mining id %d", mine_id);
    const auto &lv = it->second->levels;
    if (level < 1 || level > (int32_t)lv.size()) return fail(ctx, EPI_ESTATE, "no level %d", level);
    const MineLevel &L = lv[level - 1];
    if (n_candidates) *n_candidates = L.m;
    if (n_frequent) *n_frequent = L.nf;
    if (times_ms) {
        times_ms[0] = L.gen_ms;
        times_ms[1] = L.count_ms;
        times_ms[2] = L.kernel_ms;
    }
    return EPI_OK;
}

namespace {

// Host copy of a level's counts (levels counted by the extension engine keep
// them on the device until read).
hipError_t host_counts(MineLevel &L) {
    if ((int64_t)L.counts.size() == L.m || !L.dcounts.p) return hipSuccess;
    L.counts.resize(L.m);
    if (L.m == 0) return hipSuccess;
    return hipMemcpy(L.counts.data(), L.dcounts.p, sizeof(int32_t) * L.m, hipMemcpyDeviceToHost);
}

// Episode r of a level: explicit candidate, implicit candidate, or (when
// frequent) the frequent-episode arrays; writes the ABI layout.
void mine_episode(const Mine &mn, int level, bool frequent, int64_t r, uint8_t *N, int32_t *types, int64_t *lo,
                  int64_t *hi, int32_t *counts) {
    const MineLevel &L = mn.levels[level - 1];
    int32_t ty[kMaxN];
    int ivs[kMaxN];
    int64_t c;
    if (frequent && L.implicit) {
        c = L.freq[r];
        extend_frequent(mn, level, r, ty, ivs);
    } else {
        c = frequent ? L.freq[r] : r;
        if (L.implicit) {
            implicit_candidate(mn, level, c, ty, ivs);
        } else {
            for (int k = 0; k < L.N; ++k) ty[k] = L.types[(size_t)k * L.m + c];
            for (int k = 0; k + 1 < L.N; ++k) ivs[k] = L.iv[(size_t)k * L.m + c];
        }
    }
    N[0] = (uint8_t)L.N;
    for (int k = 0; k < kMaxN; ++k) types[k] = k < L.N ? ty[k] : -1;
    for (int k = 0; k < kMaxN - 1; ++k) {
        const bool live = k + 1 < L.N;
        lo[k] = live ? mn.menu_lo[ivs[k]] : 0;
        hi[k] = live ? mn.menu_hi[ivs[k]] : 0;
    }
    counts[0] = L.counts[c];
}

}  // namespace

epi_status epi_mine_read(epi_ctx *ctx, int32_t mine_id, int32_t level, int frequent_only, int64_t m, uint8_t *N,
                         int32_t *types, int64_t *lo, int64_t *hi, int32_t *counts) {
    if (!ctx) return EPI_EINVAL;
    auto it = ctx->c.mines.find(mine_id);
    if (it == ctx->c.mines.end()) return fail(ctx, EPI_ESTATE, "unknown mining id %d", mine_id);
    Mine &mn = *it->second;
    if (level < 1 || level > (int32_t)mn.levels.size()) return fail(ctx, EPI_ESTATE, "no level %d", level);
    MineLevel &L = mn.levels[level - 1];
    HIPTRY(ctx, host_counts(L), "reading counts");
    if (mn.engine == 1) HIPTRY(ctx, extend_host_view(mn, level), "reading a level");
    const int64_t want = frequent_only ? L.nf : L.m;
    if (m != want) return fail(ctx, EPI_EINVAL, "level %d has %lld entries, not %lld", level, (long long)want,
                               (long long)m);
    if (m > 0 && (!N || !types || !lo || !hi || !counts)) return fail(ctx, EPI_EINVAL, "null output");
    for (int64_t r = 0; r < m; ++r)
        mine_episode(mn, level, frequent_only != 0, r, N + r, types + r * 8, lo + r * 7, hi + r * 7, counts + r);
    return EPI_OK;
}

epi_status epi_mine_read_at(epi_ctx *ctx, int32_t mine_id, int32_t level, int64_t k, const int64_t *idx, uint8_t *N,
                            int32_t *types, int64_t *lo, int64_t *hi, int32_t *counts) {
    if (!ctx) return EPI_EINVAL;
    auto it = ctx->c.mines.find(mine_id);
    if (it == ctx->c.mines.end()) return fail(ctx, EPI_ESTATE, "unknown mining id %d", mine_id);
    Mine &mn = *it->second;
    if (level < 1 || level > (int32_t)mn.levels.size()) return fail(ctx, EPI_ESTATE, "no level %d", level);
    MineLevel &L = mn.levels[level - 1];
    if (k < 0 || (k > 0 && (!idx || !N || !types || !lo || !hi || !counts))) return fail(ctx, EPI_EINVAL, "bad arguments");
    HIPTRY(ctx, host_counts(L), "reading counts");
    if (mn.engine == 1) HIPTRY(ctx, extend_host_view(mn, level), "reading a level");
    for (int64_t r = 0; r < k; ++r) {
        if (idx[r] < 0 || idx[r] >= L.m) return fail(ctx, EPI_EINVAL, "index %lld outside the level", (long long)idx[r]);
        mine_episode(mn, level, false, idx[r], N + r, types + r * 8, lo + r * 7, hi + r * 7, counts + r);
    }
    return EPI_OK;
}

epi_status epi_mine_level_bytes(epi_ctx *ctx, int32_t mine_id, int32_t level, int64_t *alg_bytes) {
    if (!ctx || !alg_bytes) return fail(ctx, EPI_EINVAL, "null argument");
    auto it = ctx->c.mines.find(mine_id);
    if (it == ctx->c.mines.end()) return fail(ctx, EPI_ESTATE, "unknown mining id %d", mine_id);
    Mine &mn = *it->second;
    if (level < 1 || level > (int32_t)mn.levels.size()) return fail(ctx, EPI_ESTATE, "no level %d", level);
    MineLevel &L = mn.levels[level - 1];
    if (L.alg_bytes < 0 && L.implicit && level >= 2) {
        Stream *s = find_stream(ctx, mn.stream_id);
        if (!s) return fail(ctx, EPI_ESTATE, "the mined stream has been released");
        extend_level_bytes(*s, mn, level);
    }
    *alg_bytes = std::max<int64_t>(0, L.alg_bytes);
    return EPI_OK;
}

epi_status epi_mine_release(epi_ctx *ctx, int32_t mine_id) {
    if (!ctx) return EPI_EINVAL;
    if (!ctx->c.mines.erase(mine_id)) return fail(ctx, EPI_ESTATE, "unknown mining id %d", mine_id);
    return EPI_OK;
}

// ---- cost model ------------------------------------------------------------

namespace {

struct HostToDev {
    DevBuf d;
    hipError_t put(const void *h, size_t bytes, hipStream_t st) {
        hipError_t e = d.alloc(bytes);
        if (e != hipSuccess) return e;
        if (bytes) e = hipMemcpyAsync(d.p, h, bytes, hipMemcpyHostToDevice, st);
        return e;
    }
};

epi_status need_mlp(epi_ctx *ctx, int64_t F) {
    if (!ctx->c.mlp.ready()) return fail(ctx, EPI_ESTATE, "the cost model has not been initialised");
    if (F >= 0 && F != ctx->c.mlp.F) return fail(ctx, EPI_EINVAL, "the cost model takes %d features", ctx->c.mlp.F);
    return EPI_OK;
}

}  // namespace

epi_status epi_mlp_init(epi_ctx *ctx, int32_t n_features, uint64_t seed) {
    if (!ctx) return EPI_EINVAL;
    if (n_features < 1 || n_features > 4096) return fail(ctx, EPI_EINVAL, "n_features must be in 1..4096");
    HIPTRY(ctx, hipSetDevice(ctx->c.device), "hipSetDevice");
    HIPTRY(ctx, mlp_init(ctx->c.mlp, n_features, seed), "initialising the cost model");
    return EPI_OK;
}

epi_status epi_mlp_params(epi_ctx *ctx, int32_t *n_features, int64_t *n_params) {
    if (!ctx) return EPI_EINVAL;
    epi_status v = need_mlp(ctx, -1);
    if (v != EPI_OK) return v;
    if (n_features) *n_features = ctx->c.mlp.F;
    if (n_params) *n_params = mlp_n_params(ctx->c.mlp.F);
    return EPI_OK;
}

epi_status epi_mlp_get_params(epi_ctx *ctx, float *p, int64_t n) {
    if (!ctx || !p) return fail(ctx, EPI_EINVAL, "null argument");
    epi_status v = need_mlp(ctx, -1);
    if (v != EPI_OK) return v;
    if (n != mlp_n_params(ctx->c.mlp.F)) return fail(ctx, EPI_EINVAL, "expected %lld parameters",
                                                     (long long)mlp_n_params(ctx->c.mlp.F));
    HIPTRY(ctx, hipStreamSynchronize(ctx->c.stream), "sync");
    HIPTRY(ctx, hipMemcpy(p, ctx->c.mlp.p.p, sizeof(float) * n, hipMemcpyDeviceToHost), "copy");
    return EPI_OK;
}

epi_status epi_mlp_set_params(epi_ctx *ctx, const float *p, int64_t n) {
    if (!ctx || !p) return fail(ctx, EPI_EINVAL, "null argument");
    epi_status v = need_mlp(ctx, -1);
    if (v != EPI_OK) return v;
    if (n != mlp_n_params(ctx->c.mlp.F)) return fail(ctx, EPI_EINVAL, "expected %lld parameters",
                                                     (long long)mlp_n_params(ctx->c.mlp.F));
    HIPTRY(ctx, hipMemcpy(ctx->c.mlp.p.p, p, sizeof(float) * n, hipMemcpyHostToDevice), "copy");
    HIPTRY(ctx, hipMemset(ctx->c.mlp.m.p, 0, sizeof(float) * n), "reset");
    HIPTRY(ctx, hipMemset(ctx->c.mlp.v.p, 0, sizeof(float) * n), "reset");
    ctx->c.mlp.step = 0;
    return EPI_OK;
}

epi_status epi_mlp_forward(epi_ctx *ctx, const float *X, int64_t B, float *y) {
    if (!ctx || (B > 0 && (!X || !y))) return fail(ctx, EPI_EINVAL, "null argument");
    epi_status v = need_mlp(ctx, -1);
    if (v != EPI_OK) return v;
    hipStream_t st = ctx->c.stream;
    HostToDev dx;
    DevBuf dy;
    HIPTRY(ctx, dx.put(X, sizeof(float) * B * ctx->c.mlp.F, st), "copy");
    HIPTRY(ctx, dy.alloc(sizeof(float) * B), "alloc");
    HIPTRY(ctx, mlp_forward_device(ctx->c.mlp, dx.d.as<float>(), B, dy.as<float>(), st), "forward");
    HIPTRY(ctx, hipStreamSynchronize(st), "sync");
    if (B > 0) HIPTRY(ctx, hipMemcpy(y, dy.p, sizeof(float) * B, hipMemcpyDeviceToHost), "copy");
    return EPI_OK;
}

epi_status epi_mlp_grad(epi_ctx *ctx, const float *X, const float *t, int64_t B, float *loss, float *g) {
    if (!ctx || B < 1 || !X || !t || !g) return fail(ctx, EPI_EINVAL, "bad arguments");
    epi_status v = need_mlp(ctx, -1);
    if (v != EPI_OK) return v;
    hipStream_t st = ctx->c.stream;
    const int64_t np = mlp_n_params(ctx->c.mlp.F);
    HostToDev dx, dt;
    HIPTRY(ctx, dx.put(X, sizeof(float) * B * ctx->c.mlp.F, st), "copy");
    HIPTRY(ctx, dt.put(t, sizeof(float) * B, st), "copy");
    float L = 0;
    HIPTRY(ctx, mlp_grad_device(ctx->c.mlp, dx.d.as<float>(), dt.d.as<float>(), B, ctx->c.mlp.g.as<float>(), &L, st),
           "gradient");
    HIPTRY(ctx, hipStreamSynchronize(st), "sync");
    HIPTRY(ctx, hipMemcpy(g, ctx->c.mlp.g.p, sizeof(float) * np, hipMemcpyDeviceToHost), "copy");
    if (loss) *loss = L;
    return EPI_OK;
}

epi_status epi_mlp_adam_step(epi_ctx *ctx, const float *g, float lr) {
    if (!ctx || !g) return fail(ctx, EPI_EINVAL, "null argument");
    epi_status v = need_mlp(ctx, -1);
    if (v != EPI_OK) return v;
    const int64_t np = mlp_n_params(ctx->c.mlp.F);
    HIPTRY(ctx, hipMemcpy(ctx->c.mlp.g.p, g, sizeof(float) * np, hipMemcpyHostToDevice), "copy");
    ctx->c.mlp.lr = lr;
    HIPTRY(ctx, mlp_adam_device(ctx->c.mlp, ctx->c.mlp.g.as<float>(), ctx->c.stream), "adam");
    HIPTRY(ctx, hipStreamSynchronize(ctx->c.stream), "sync");
    return EPI_OK;
}

epi_status epi_mlp_train(epi_ctx *ctx, const float *X, const float *t, int64_t B, int32_t epochs, int32_t batch,
                         float lr, float *losses) {
    if (!ctx || B < 1 || !X || !t || epochs < 1 || batch < 1) return fail(ctx, EPI_EINVAL, "bad arguments");
    epi_status v = need_mlp(ctx, -1);
    if (v != EPI_OK) return v;
    hipStream_t st = ctx->c.stream;
    Mlp &net = ctx->c.mlp;
    net.lr = lr;
    HostToDev dx, dt;
    HIPTRY(ctx, dx.put(X, sizeof(float) * B * net.F, st), "copy");
    HIPTRY(ctx, dt.put(t, sizeof(float) * B, st), "copy");
    for (int32_t ep = 0; ep < epochs; ++ep) {
        double acc = 0;
        for (int64_t b0 = 0; b0 < B; b0 += batch) {
            const int64_t nb = std::min<int64_t>(batch, B - b0);
            float L = 0;
            HIPTRY(ctx, mlp_grad_device(net, dx.d.as<float>() + b0 * net.F, dt.d.as<float>() + b0, nb,
                                        net.g.as<float>(), losses ? &L : nullptr, st),
                   "gradient");
            HIPTRY(ctx, mlp_adam_device(net, net.g.as<float>(), st), "adam");
            acc += (double)L * nb;
        }
        if (losses) losses[ep] = (float)(acc / (double)B);
    }
    HIPTRY(ctx, hipStreamSynchronize(st), "sync");
    return EPI_OK;
}

epi_status epi_costmodel_features(epi_ctx *ctx, int32_t set_id, float *X, int64_t m) {
    if (!ctx) return EPI_EINVAL;
    CandSet *cs = find_set(ctx, set_id);
    if (!cs) return fail(ctx, EPI_ESTATE, "unknown set id %d", set_id);
    if (cs->compact) return fail(ctx, EPI_EINVAL, "set %d has no features", set_id);
    if (m != cs->m || (m > 0 && !X)) return fail(ctx, EPI_EINVAL, "set %d holds %lld candidates", set_id,
                                                 (long long)cs->m);
    Stream *s = find_stream(ctx, cs->stream_id);
    hipStream_t st = ctx->c.stream;
    DevBuf dX;
    HIPTRY(ctx, dX.alloc(sizeof(float) * m * kFeatures), "alloc");
    HIPTRY(ctx, candidate_features(*s, *cs, dX.as<float>(), st), "features");
    std::vector<float> grouped((size_t)m * kFeatures);
    std::vector<int32_t> orig(m);
    if (m > 0) {
        HIPTRY(ctx, hipMemcpy(grouped.data(), dX.p, sizeof(float) * grouped.size(), hipMemcpyDeviceToHost), "copy");
        HIPTRY(ctx, hipMemcpy(orig.data(), cs->orig.p, sizeof(int32_t) * m, hipMemcpyDeviceToHost), "copy");
    }
    for (int64_t i = 0; i < m; ++i)
        std::copy(grouped.begin() + i * kFeatures, grouped.begin() + (i + 1) * kFeatures, X + (int64_t)orig[i] * kFeatures);
    return EPI_OK;
}

epi_status epi_read_worklog(epi_ctx *ctx, int32_t set_id, int32_t *work, int64_t m) {
    if (!ctx) return EPI_EINVAL;
    CandSet *cs = find_set(ctx, set_id);
    if (!cs) return fail(ctx, EPI_ESTATE, "unknown set id %d", set_id);
    if (!cs->counted || !cs->logged) return fail(ctx, EPI_ESTATE, "set %d has no work log", set_id);
    if (m != cs->m || (m > 0 && !work)) return fail(ctx, EPI_EINVAL, "set %d holds %lld candidates", set_id,
                                                    (long long)cs->m);
    epi_status f = epi_sync(ctx);
    if (f != EPI_OK) return f;
    if (m > 0) HIPTRY(ctx, hipMemcpy(work, cs->work.p, sizeof(int32_t) * kWork * m, hipMemcpyDeviceToHost), "copy");
    return EPI_OK;
}

epi_status epi_read_item_cycles(epi_ctx *ctx, int32_t set_id, int64_t *cycles, int64_t n_items, int64_t *n_out) {
    if (!ctx) return EPI_EINVAL;
    CandSet *cs = find_set(ctx, set_id);
    if (!cs) return fail(ctx, EPI_ESTATE, "unknown set id %d", set_id);
    const BatchPlan *pl = cs->cycles_plan ? ctx->c.batch.find_id(cs->cycles_plan) : nullptr;
    const bool have = pl && pl->cycles.p;
    if (n_out) *n_out = have ? pl->n_items : 0;
    if (!cycles) return EPI_OK;
    if (!have || n_items != pl->n_items)
        return fail(ctx, EPI_EINVAL, "the last batched count of set %d stamped %lld items", set_id,
                    (long long)(have ? pl->n_items : 0));
    epi_status f = epi_sync(ctx);
    if (f != EPI_OK) return f;
    HIPTRY(ctx, hipMemcpy(cycles, pl->cycles.p, sizeof(int64_t) * 2 * n_items, hipMemcpyDeviceToHost), "copy");
    return EPI_OK;
}

epi_status epi_costmodel_train(epi_ctx *ctx, const int32_t *set_ids, int32_t k, int32_t epochs, uint64_t seed,
                               float *losses) {
    if (!ctx || k < 1 || !set_ids || epochs < 1) return fail(ctx, EPI_EINVAL, "bad arguments");
    std::vector<float> X, t;
    for (int32_t i = 0; i < k; ++i) {
        CandSet *cs = find_set(ctx, set_ids[i]);
        if (!cs) return fail(ctx, EPI_ESTATE, "unknown set id %d", set_ids[i]);
        if (!cs->counted || !cs->logged) return fail(ctx, EPI_ESTATE, "set %d has no work log", set_ids[i]);
        std::vector<float> Xi((size_t)cs->m * kFeatures);
        std::vector<int32_t> w((size_t)cs->m * kWork);
        epi_status v = epi_costmodel_features(ctx, set_ids[i], Xi.data(), cs->m);
        if (v != EPI_OK) return v;
        v = epi_read_worklog(ctx, set_ids[i], w.data(), cs->m);
        if (v != EPI_OK) return v;
        X.insert(X.end(), Xi.begin(), Xi.end());
        // target: log1p of the lane's work (events visited + state-machine
        // operations) less the base feature, log1p of the summed event counts
        // of the episode's types (the network learns the correction to it)
        for (int64_t c = 0; c < cs->m; ++c)
            t.push_back(std::log1p((float)w[c * kWork + 0] + (float)w[c * kWork + 1] + (float)w[c * kWork + 2]) -
                        Xi[c * kFeatures + kBaseFeature]);
    }
    const int64_t B = (int64_t)t.size();
    // shuffle once (SplitMix64-driven Fisher-Yates) so mini-batches mix sets
    std::vector<int64_t> ord(B);
    std::iota(ord.begin(), ord.end(), 0);
    uint64_t st = seed ^ 0x5DEECE66Dull;
    for (int64_t i = B - 1; i > 0; --i) {
        st += 0x9E3779B97F4A7C15ull;
        uint64_t z = st;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        std::swap(ord[i], ord[(int64_t)(z % (uint64_t)(i + 1))]);
    }
    // standardise inputs and target on the training set (a constant feature
    // gets a zero scale and drops out); the network learns the standardised
    // problem and the scaling is kept with it
    std::vector<double> mu(kFeatures, 0.0), var(kFeatures, 0.0);
    double tmu = 0, tvar = 0;
    for (int64_t i = 0; i < B; ++i) {
        for (int f = 0; f < kFeatures; ++f) mu[f] += X[i * kFeatures + f];
        tmu += t[i];
    }
    for (int f = 0; f < kFeatures; ++f) mu[f] /= (double)B;
    tmu /= (double)B;
    for (int64_t i = 0; i < B; ++i) {
        for (int f = 0; f < kFeatures; ++f) {
            const double d = X[i * kFeatures + f] - mu[f];
            var[f] += d * d;
        }
        tvar += (t[i] - tmu) * (t[i] - tmu);
    }
    std::vector<float> x_mu(kFeatures), x_isd(kFeatures);
    for (int f = 0; f < kFeatures; ++f) {
        const double sd = std::sqrt(var[f] / (double)B);
        x_mu[f] = (float)mu[f];
        x_isd[f] = sd > 1e-6 ? (float)(1.0 / sd) : 0.f;
    }
    const double tsd = std::sqrt(tvar / (double)B);
    const float y_sd = tsd > 1e-6 ? (float)tsd : 1.f;
    std::vector<float> Xs((size_t)B * kFeatures), ts(B);
    for (int64_t i = 0; i < B; ++i) {
        for (int f = 0; f < kFeatures; ++f)
            Xs[i * kFeatures + f] = (X[ord[i] * kFeatures + f] - x_mu[f]) * x_isd[f];
        ts[i] = (float)((t[ord[i]] - tmu) / y_sd);
    }
    epi_status v = epi_mlp_init(ctx, kFeatures, seed);
    if (v != EPI_OK) return v;
    HIPTRY(ctx, mlp_set_scaling(ctx->c.mlp, x_mu.data(), x_isd.data(), (float)tmu, y_sd), "scaling");
    return epi_mlp_train(ctx, Xs.data(), ts.data(), B, epochs, 512, 3e-3f, losses);
}

epi_status epi_costmodel_scaling(epi_ctx *ctx, float *x_mu, float *x_isd, float *y_mu_sd) {
    if (!ctx) return EPI_EINVAL;
    epi_status v = need_mlp(ctx, -1);
    if (v != EPI_OK) return v;
    const Mlp &net = ctx->c.mlp;
    if (x_mu) std::copy(net.x_mu.begin(), net.x_mu.end(), x_mu);
    if (x_isd) std::copy(net.x_isd.begin(), net.x_isd.end(), x_isd);
    if (y_mu_sd) {
        y_mu_sd[0] = net.y_mu;
        y_mu_sd[1] = net.y_sd;
    }
    return EPI_OK;
}

namespace {
constexpr char kModelMagic[8] = {'E', 'P', 'I', 'C', 'R', '0', '0', '1'};
}

epi_status epi_costmodel_save(epi_ctx *ctx, const char *path) {
    if (!ctx || !path) return fail(ctx, EPI_EINVAL, "bad arguments");
    epi_status v = need_mlp(ctx, -1);
    if (v != EPI_OK) return v;
    const Mlp &net = ctx->c.mlp;
    const int32_t F = net.F;
    const int64_t np = mlp_n_params(F);
    std::vector<float> p(np);
    HIPTRY(ctx, hipMemcpy(p.data(), net.p.p, sizeof(float) * np, hipMemcpyDeviceToHost), "copy");
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(ctx, EPI_EINVAL, "cannot write %s", path);
    const float y[2] = {net.y_mu, net.y_sd};
    bool ok = std::fwrite(kModelMagic, 1, 8, f) == 8 && std::fwrite(&F, sizeof F, 1, f) == 1 &&
              std::fwrite(&np, sizeof np, 1, f) == 1 && std::fwrite(p.data(), sizeof(float), np, f) == (size_t)np &&
              std::fwrite(net.x_mu.data(), sizeof(float), F, f) == (size_t)F &&
              std::fwrite(net.x_isd.data(), sizeof(float), F, f) == (size_t)F && std::fwrite(y, sizeof(float), 2, f) == 2;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? EPI_OK : fail(ctx, EPI_EINVAL, "writing %s failed", path);
}

epi_status epi_costmodel_load(epi_ctx *ctx, const char *path) {
    if (!ctx || !path) return fail(ctx, EPI_EINVAL, "bad arguments");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(ctx, EPI_EINVAL, "cannot read %s", path);
    char magic[8];
    int32_t F = 0;
    int64_t np = 0;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kModelMagic, 8) == 0 &&
              std::fread(&F, sizeof F, 1, f) == 1 && F >= 1 && F <= 4096 && std::fread(&np, sizeof np, 1, f) == 1 &&
              np == mlp_n_params(F);
    std::vector<float> p, mu, isd;
    float y[2] = {0.f, 1.f};
    if (ok) {
        p.resize(np);
        mu.resize(F);
        isd.resize(F);
        ok = std::fread(p.data(), sizeof(float), np, f) == (size_t)np &&
             std::fread(mu.data(), sizeof(float), F, f) == (size_t)F &&
             std::fread(isd.data(), sizeof(float), F, f) == (size_t)F && std::fread(y, sizeof(float), 2, f) == 2 &&
             std::fgetc(f) == EOF;
    }
    std::fclose(f);
    if (!ok) return fail(ctx, EPI_EINVAL, "%s is not a cost model file of this library", path);
    for (float x : p)
        if (!std::isfinite(x)) return fail(ctx, EPI_EINVAL, "%s holds non-finite parameters", path);
    if (!(y[1] > 0.f) || !std::isfinite(y[0])) return fail(ctx, EPI_EINVAL, "%s holds a bad output scale", path);
    epi_status v = epi_mlp_init(ctx, F, 0);
    if (v != EPI_OK) return v;
    v = epi_mlp_set_params(ctx, p.data(), np);
    if (v != EPI_OK) return v;
    HIPTRY(ctx, mlp_set_scaling(ctx->c.mlp, mu.data(), isd.data(), y[0], y[1]), "scaling");
    return EPI_OK;
}

epi_status epi_costmodel_predict(epi_ctx *ctx, int32_t set_id, float *y, int64_t m) {
    if (!ctx) return EPI_EINVAL;
    epi_status v = need_mlp(ctx, kFeatures);
    if (v != EPI_OK) return v;
    CandSet *cs = find_set(ctx, set_id);
    if (!cs) return fail(ctx, EPI_ESTATE, "unknown set id %d", set_id);
    if (cs->compact) return fail(ctx, EPI_EINVAL, "set %d has no features", set_id);
    if (m != cs->m || (m > 0 && !y)) return fail(ctx, EPI_EINVAL, "set %d holds %lld candidates", set_id,
                                                 (long long)cs->m);
    if (m == 0) return EPI_OK;
    Stream *s = find_stream(ctx, cs->stream_id);
    hipStream_t st = ctx->c.stream;
    DevBuf dX, dy;
    HIPTRY(ctx, dX.alloc(sizeof(float) * m * kFeatures), "alloc");
    HIPTRY(ctx, dy.alloc(sizeof(float) * m), "alloc");
    HIPTRY(ctx, candidate_features(*s, *cs, dX.as<float>(), st), "features");
    HIPTRY(ctx, costmodel_predict_device(ctx->c.mlp, dX.as<float>(), m, dy.as<float>(), st), "predict");
    std::vector<float> grouped(m);
    std::vector<int32_t> orig(m);
    HIPTRY(ctx, hipMemcpyAsync(grouped.data(), dy.p, sizeof(float) * m, hipMemcpyDeviceToHost, st), "copy");
    HIPTRY(ctx, hipMemcpyAsync(orig.data(), cs->orig.p, sizeof(int32_t) * m, hipMemcpyDeviceToHost, st), "copy");
    HIPTRY(ctx, hipStreamSynchronize(st), "sync");
    for (int64_t i = 0; i < m; ++i) y[orig[i]] = grouped[i];
    return EPI_OK;
}

// ---- autotuner ---------------------------------------------------------------

namespace {

int log2_bucket(int64_t x) {
    int b = 0;
    while (x > 1) {
        x >>= 1;
        ++b;
    }
    return b;
}

// Workload shape: timestamp kind, schedule, max K, and log2 buckets of the
// events, of the candidates and of the candidates of each episode size.
std::string tune_key(epi_ctx *ctx, const int32_t *set_ids, int32_t k, int sched) {
    int64_t n = 0, m = 0;
    int32_t K = 0;
    int kind = 0;
    int64_t byN[kMaxN + 1] = {0};
    for (int32_t i = 0; i < k; ++i) {
        CandSet *cs = find_set(ctx, set_ids[i]);
        Stream *s = find_stream(ctx, cs->stream_id);
        n += s->n;
        m += cs->m;
        K = std::max(K, s->K);
        kind = s->ts_kind;
        for (const Group &g : cs->groups) byN[g.N] += g.end - g.begin;
    }
    std::string key = "ts" + std::to_string(kind) + "_s" + std::to_string(sched) + "_K" + std::to_string(K) + "_n" +
                      std::to_string(log2_bucket(n)) + "_m" + std::to_string(log2_bucket(m)) + "_N";
    for (int N = 1; N <= kMaxN; ++N) key += "." + std::to_string(byN[N] ? log2_bucket(byN[N]) + 1 : 0);
    return key;
}

// One tuned setting of the batched engine.
struct TuneSetting {
    int64_t tile = kDefaultTile; // largest events per tile of the sets' streams
    int64_t rings = 0;           // EPI_OPT_RING_CLASSES
    int64_t lanes = 0;           // EPI_OPT_LANES (0: automatic)
    int64_t target = 262144;     // EPI_OPT_TARGET_LANES
};

bool tune_valid(const TuneSetting &t) {
    return (t.tile == 4096 || t.tile == 2048 || t.tile == 1024 || t.tile == 512 || t.tile == 256) && t.rings >= 0 &&
           t.rings <= 2 &&
           (t.lanes == 0 || t.lanes == 64 || t.lanes == 128 || t.lanes == 256) && t.target >= 1024 &&
           t.target <= (int64_t(1) << 26);
}

bool cache_lookup(const char *path, const std::string &key, TuneSetting *out) {
    if (!path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[1024], kb[512];
    long long a, b, c, d;
    bool found = false;
    // one entry per line: key tile rings lanes target; other lines are ignored
    while (fgets(line, sizeof line, f)) {
        char extra;
        if (sscanf(line, "%511s %lld %lld %lld %lld %c", kb, &a, &b, &c, &d, &extra) != 5) continue;
        const TuneSetting t{a, b, c, d};
        if (key == kb && tune_valid(t)) {
            *out = t;
            found = true;  // the last valid entry wins
        }
    }
    fclose(f);
    return found;
}

// Re-tile every stream of the sets to tile cap `cap` (plans over the old
// tiles are dropped first).
epi_status retile(epi_ctx *ctx, const int32_t *set_ids, int32_t k, int64_t cap) {
    std::vector<Stream *> ss;
    for (int32_t i = 0; i < k; ++i) {
        Stream *s = find_stream(ctx, find_set(ctx, set_ids[i])->stream_id);
        if (std::find(ss.begin(), ss.end(), s) == ss.end()) ss.push_back(s);
    }
    bool any = false;
    for (Stream *s : ss) any = any || s->tile_cap != cap;
    if (!any) return EPI_OK;
    for (auto &kv : ctx->c.mines)
        for (Stream *s : ss)
            if (find_stream(ctx, kv.second->stream_id) == s)
                return fail(ctx, EPI_ESTATE, "a level-wise discovery run (%d) uses a stream to be re-tiled", kv.first);
    HIPTRY(ctx, hipDeviceSynchronize(), "sync");
    ctx->c.batch.evict_all();
    for (Stream *s : ss) {
        if (s->tile_cap == cap) continue;
        s->tile_cap = (int)cap;
        HIPTRY(ctx, build_type_index(*s, ctx->c.stream), "re-tiling a stream");
    }
    HIPTRY(ctx, hipStreamSynchronize(ctx->c.stream), "sync");
    return EPI_OK;
}

void apply_setting(epi_ctx *ctx, const TuneSetting &t) {
    ctx->c.opt.ring_classes = (int)t.rings;
    ctx->c.opt.lanes = (int)t.lanes;
    ctx->c.opt.target_lanes = t.target;
}

}  // namespace

epi_status epi_autotune(epi_ctx *ctx, const int32_t *set_ids, int32_t k, int sched, const char *cache_path,
                        int64_t *chosen) {
    if (!ctx || k < 1 || !set_ids) return fail(ctx, EPI_EINVAL, "bad arguments");
    for (int32_t i = 0; i < k; ++i) {
        CandSet *cs = find_set(ctx, set_ids[i]);
        if (!cs) return fail(ctx, EPI_ESTATE, "unknown set id %d", set_ids[i]);
        if (cs->compact || cs->stream_order)
            return fail(ctx, EPI_EINVAL, "set %d cannot be counted in batched mode", set_ids[i]);
    }
    const std::string key = tune_key(ctx, set_ids, k, sched);
    TuneSetting best;
    best.target = ctx->c.opt.target_lanes;
    if (!cache_lookup(cache_path, key, &best)) {
        // coordinate descent from the defaults: tile cap, then launch-group
        // merging, then lanes per workgroup, then the segment target; each
        // trial is a batched count whose plan is built first and then timed
        // as a replay (hipEvents on the context's stream)
        const CountOptions saved = ctx->c.opt;
        hipEvent_t a = nullptr, b = nullptr;
        hipError_t he = hipEventCreate(&a);
        if (he == hipSuccess && (he = hipEventCreate(&b)) != hipSuccess) (void)hipEventDestroy(a);
        if (he != hipSuccess) return hipfail(ctx, he, "event");
        auto trial = [&](const TuneSetting &t, float *ms) -> epi_status {
            *ms = INFINITY;
            epi_status v = retile(ctx, set_ids, k, t.tile);
            if (v != EPI_OK) return v;
            apply_setting(ctx, t);
            if (epi_count(ctx, set_ids, k, EPI_MODE_BATCHED, sched, nullptr) != EPI_OK || epi_sync(ctx) != EPI_OK) {
                (void)hipGetLastError();
                return EPI_OK;  // a setting that cannot run loses
            }
            // the faster of two replays (a replay's time varies by a few %)
            for (int rep = 0; rep < 2; ++rep) {
                (void)hipEventRecord(a, ctx->c.stream);
                v = epi_count(ctx, set_ids, k, EPI_MODE_BATCHED, sched, nullptr);
                (void)hipEventRecord(b, ctx->c.stream);
                if (v != EPI_OK) {
                    (void)hipGetLastError();
                    *ms = INFINITY;
                    return EPI_OK;
                }
                HIPTRY(ctx, hipEventSynchronize(b), "sync");
                float x = INFINITY;
                (void)hipEventElapsedTime(&x, a, b);
                *ms = std::min(*ms, x);
            }
            return epi_sync(ctx);
        };
        float best_ms = INFINITY;
        epi_status v = trial(best, &best_ms);
        const int64_t menus[4][3] = {{4096, 1024, 512}, {0, 1, 2}, {0, 128, 64}, {131072, 524288, 1048576}};
        // a second pass when the first moved (the knobs interact: wider
        // groups change which lane width keeps the most waves resident)
        for (int pass = 0; v == EPI_OK && pass < 2; ++pass) {
            const TuneSetting start = best;
            for (int d = 0; v == EPI_OK && d < 4; ++d) {
                for (int64_t x : menus[d]) {
                    TuneSetting t = best;
                    int64_t *field = d == 0 ? &t.tile : d == 1 ? &t.rings : d == 2 ? &t.lanes : &t.target;
                    if (*field == x) continue;
                    *field = x;
                    float ms = INFINITY;
                    if ((v = trial(t, &ms)) != EPI_OK) break;
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = t;
                    }
                }
            }
            if (best.tile == start.tile && best.rings == start.rings && best.lanes == start.lanes &&
                best.target == start.target)
                break;
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        ctx->c.opt = saved;
        if (v != EPI_OK) return v;
        if (cache_path) {
            FILE *f = fopen(cache_path, "a");
            if (f) {
                fprintf(f, "%s %lld %lld %lld %lld\n", key.c_str(), (long long)best.tile, (long long)best.rings,
                        (long long)best.lanes, (long long)best.target);
                fclose(f);
            }
        }
    }
    epi_status v = retile(ctx, set_ids, k, best.tile);
    if (v != EPI_OK) return v;
    apply_setting(ctx, best);
    if (chosen) {
        chosen[0] = best.tile;
        chosen[1] = best.rings;
        chosen[2] = best.lanes;
        chosen[3] = best.target;
    }
    return EPI_OK;
}

epi_status epi_count_noalloc(epi_ctx *ctx, int32_t set_id, int64_t segments, void *hip_stream) {
    if (!ctx) return EPI_EINVAL;
    if (segments < 0) return fail(ctx, EPI_EINVAL, "segments must be >= 0");
    CandSet *cs = find_set(ctx, set_id);
    if (!cs) return fail(ctx, EPI_ESTATE, "unknown set id %d", set_id);
    if (cs->stream_order) return fail(ctx, EPI_EINVAL, "set %d decides overlap in stream order", set_id);
    if (cs->compact) return fail(ctx, EPI_EINVAL, "set %d cannot be counted here", set_id);
    if (cs->deep)
        return fail(ctx, EPI_EINVAL, "set %d holds episodes deeper than the rings (counted with working memory)",
                    set_id);
    Stream *s = find_stream(ctx, cs->stream_id);
    unsigned char *scr = noalloc_scratch(ctx->c.device);
    if (!scr) return fail(ctx, EPI_EDEVICE, "no scratch address for device %d", ctx->c.device);
    CountOptions opt = ctx->c.opt;
    opt.segments = segments;
    opt.worklog = false;
    for (const Group &g : cs->groups) {
        const int64_t G = g.end - g.begin;
        if (G <= 0 || s->n == 0) continue;
        const int64_t P = plain_segments(*s, G, opt, nullptr);
        const size_t need = plain_record_bytes(*s, P, G);
        if (need > noalloc_scratch_bytes())
            return fail(ctx, EPI_ESIZE, "%lld segments x %lld episodes need %zu B of records, the scratch holds %zu B",
                        (long long)P, (long long)G, need, noalloc_scratch_bytes());
    }
    HIPTRY(ctx, hipSetDevice(ctx->c.device), "hipSetDevice");
    hipStream_t st = pick_stream(ctx, hip_stream);
    HIPTRY(ctx, launch_count(*s, *cs, opt, ctx->c.flags.as<int32_t>(), st, scr, noalloc_scratch_bytes()),
           "launching the count");
    cs->logged = false;
    cs->counted = true;
    cs->counted_n = s->n;
    return EPI_OK;
}

epi_status epi_batched_stats(epi_ctx *ctx, int64_t *plans_built, int64_t *replays, int64_t *plans_kept) {
    if (!ctx) return EPI_EINVAL;
    if (plans_built) *plans_built = ctx->c.batch.built;
    if (replays) *replays = ctx->c.batch.replays;
    if (plans_kept) *plans_kept = (int64_t)ctx->c.batch.plans.size();
    return EPI_OK;
}

epi_status epi_read_schedule(epi_ctx *ctx, int32_t set_id, int32_t *order, int32_t *block, int64_t m) {
    if (!ctx) return EPI_EINVAL;
    CandSet *cs = find_set(ctx, set_id);
    if (!cs) return fail(ctx, EPI_ESTATE, "unknown set id %d", set_id);
    if (m != cs->m || (m > 0 && (!order || !block)))
        return fail(ctx, EPI_EINVAL, "set %d holds %lld candidates", set_id, (long long)cs->m);
    const BatchPlan *pl = cs->last_plan ? ctx->c.batch.find_id(cs->last_plan) : nullptr;
    if (!pl) return fail(ctx, EPI_ESTATE, "set %d has no kept batched schedule", set_id);
    int si = -1;
    for (size_t i = 0; i < pl->set_ids.size(); ++i)
        if (pl->set_ids[i] == set_id) si = (int)i;
    if (si < 0) return fail(ctx, EPI_ESTATE, "set %d has no kept batched schedule", set_id);
    epi_status f = epi_sync(ctx);
    if (f != EPI_OK) return f;
    if (m == 0) return EPI_OK;
    std::vector<int32_t> orig(m), perm(m);
    HIPTRY(ctx, hipMemcpy(orig.data(), cs->orig.p, sizeof(int32_t) * m, hipMemcpyDeviceToHost), "copy");
    if (pl->perm)
        HIPTRY(ctx, hipMemcpy(perm.data(), pl->perm + pl->soff[si], sizeof(int32_t) * m, hipMemcpyDeviceToHost),
               "copy");
    else
        std::iota(perm.begin(), perm.end(), 0);
    for (int64_t i = 0; i < m; ++i) {
        order[i] = orig[perm[i]];
        block[i] = -1;
    }
    int32_t nb = 0;
    for (const auto &u : pl->uview) {
        if (u.set != si) continue;
        for (int64_t i = 0; i < u.G; ++i) block[u.begin + i] = nb + (int32_t)(i / u.W);
        nb += (int32_t)((u.G + u.W - 1) / u.W);
    }
    return EPI_OK;
}

epi_status epi_counts_device(epi_ctx *ctx, int32_t set_id, const int32_t **d_counts) {
    if (!ctx || !d_counts) return fail(ctx, EPI_EINVAL, "null argument");
    CandSet *cs = find_set(ctx, set_id);
    if (!cs) return fail(ctx, EPI_ESTATE, "unknown set id %d", set_id);
    *d_counts = cs->counts.as<int32_t>();
    return EPI_OK;
}

}  // extern "C"
