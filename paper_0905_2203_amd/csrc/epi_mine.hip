// Level-wise discovery of frequent serial episodes (Sec. II-C): level N
// candidates are generated from the frequent episodes of level N-1, counted
// in one pass over the stream, and those whose count is greater than the
// threshold are kept.
//   level 1: every event type as a 1-node episode;
//   level 2: ordered pairs of distinct frequent types, with every interval
//            of the menu;
//   level N+1: alpha + last(beta) for frequent N-node alpha, beta whose
//            overlap agrees (types 2..N of alpha and their intervals equal
//            types 1..N-1 of beta and theirs), when the new type is not
//            alpha's first (episode types are distinct).
// Candidates live in structure-of-arrays form with interval ids into the
// menu; each level is counted by the engine in compact layout.
#include <algorithm>
#include <chrono>
#include <numeric>
#include <thread>

#include "epi_count.h"

namespace epi {

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

template <typename T>
hipError_t count_level_t(const Stream &s, const Mine &mn, MineLevel &L, const CountOptions &opt, int32_t *d_flags,
                         hipStream_t st) {
    hipError_t e;
    const auto t0 = Clock::now();
    const int64_t m = L.m;
    CandSet cs;
    cs.compact = true;
    cs.m = m;
    const int nm = (int)mn.menu_lo.size();
    std::vector<T> menu(2 * nm);
    int Q = 1;
    int64_t qmax = 1;
    for (int i = 0; i < nm; ++i) {
        menu[2 * i] = (T)mn.menu_lo[i];
        menu[2 * i + 1] = (T)mn.menu_hi[i];
        if (L.N > 1) Q = std::max(Q, queue_class_of(queue_bound(mn.menu_lo[i], mn.menu_hi[i])));
        qmax = std::max(qmax, queue_bound(mn.menu_lo[i], mn.menu_hi[i]));
    }
    if ((e = cs.t16.alloc(sizeof(uint16_t) * L.types.size())) != hipSuccess) return e;
    if ((e = cs.iv.alloc(L.iv.size())) != hipSuccess) return e;
    if ((e = cs.menu.alloc(sizeof(T) * menu.size())) != hipSuccess) return e;
    if ((e = cs.counts.alloc(sizeof(int32_t) * m)) != hipSuccess) return e;
    if (!L.types.empty() &&
        (e = hipMemcpyAsync(cs.t16.p, L.types.data(), sizeof(uint16_t) * L.types.size(), hipMemcpyHostToDevice,
                            st)) != hipSuccess)
        return e;
    if (!L.iv.empty() &&
        (e = hipMemcpyAsync(cs.iv.p, L.iv.data(), L.iv.size(), hipMemcpyHostToDevice, st)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(cs.menu.p, menu.data(), sizeof(T) * menu.size(), hipMemcpyHostToDevice, st)) !=
        hipSuccess)
        return e;
    Group g;
    g.N = L.N;
    g.Q = Q;
    // lane machines: every interval's ring as deep as the menu's deepest
    g.C = qmax <= kLaneMaxQ ? (int)qmax * (L.N - 1) : 0;
    g.begin = 0;
    g.end = m;
    g.hspan = 0;
    for (int i = 0; i < nm; ++i) g.hspan = std::max<int64_t>(g.hspan, mn.menu_hi[i] * (L.N - 1));
    cs.groups.push_back(g);
    if (mn.pred_bits.p && mn.succ_bits.p && L.N > 1) {
        cs.pred_bits = mn.pred_bits.as<uint64_t>();
        cs.succ_bits = mn.succ_bits.as<uint64_t>();
    }
    hipEvent_t ev0, ev1;
    if ((e = hipEventCreate(&ev0)) != hipSuccess) return e;
    if ((e = hipEventCreate(&ev1)) != hipSuccess) return e;
    (void)hipEventRecord(ev0, st);
    e = launch_count(s, cs, opt, d_flags, st);
    (void)hipEventRecord(ev1, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    float kms = 0;
    if (e == hipSuccess) (void)hipEventElapsedTime(&kms, ev0, ev1);
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (e != hipSuccess) return e;
    L.counts.assign(m, 0);
    if (m > 0 && (e = hipMemcpy(L.counts.data(), cs.counts.p, sizeof(int32_t) * m, hipMemcpyDeviceToHost)) !=
                     hipSuccess)
        return e;
    L.kernel_ms = kms;
    L.count_ms = ms_since(t0);
    // bytes the state-machine method reads per candidate: the times of each of
    // its N types, its descriptor, and its count
    int64_t ab = 0;
    for (int k = 0; k < L.N; ++k)
        for (int64_t i = 0; i < m; ++i) {
            const int ty = L.types[(size_t)k * m + i];
            ab += (int64_t)(s.h_off[ty + 1] - s.h_off[ty]) * (int64_t)sizeof(T);
        }
    L.alg_bytes = ab + m * (int64_t)(2 * L.N + (L.N - 1) + 4);
    return hipSuccess;
}

}  // namespace

int queue_class_of(int64_t b) { return queue_class(b); }

hipError_t count_mine_level(const Stream &s, const Mine &mn, MineLevel &L, const CountOptions &opt, int32_t *d_flags,
                            hipStream_t st) {
    if (s.ts_kind == EPI_TS_I64) return count_level_t<int64_t>(s, mn, L, opt, d_flags, st);
    return count_level_t<int32_t>(s, mn, L, opt, d_flags, st);
}

// ---- candidate generation --------------------------------------------------

void gen_level1(int32_t K, MineLevel &L) {
    L.N = 1;
    L.m = K;
    L.types.resize(K);
    for (int32_t k = 0; k < K; ++k) L.types[k] = (uint16_t)k;
    L.iv.clear();
}

void gen_level2(const MineLevel &F1, int nm, MineLevel &L) {
    std::vector<uint16_t> f;
    for (int64_t i : F1.freq) f.push_back(F1.types[i]);
    const int64_t nf = (int64_t)f.size();
    const int64_t m = nf * (nf - 1) * nm;
    L.N = 2;
    L.m = m;
    L.types.resize(2 * m);
    L.iv.resize(m);
    int64_t c = 0;
    for (int64_t a = 0; a < nf; ++a)
        for (int64_t b = 0; b < nf; ++b) {
            if (a == b) continue;
            for (int i = 0; i < nm; ++i) {
                L.types[c] = f[a];
                L.types[m + c] = f[b];
                L.iv[c] = (uint8_t)i;
                ++c;
            }
        }
}

// Join of level P (size N >= 2) into level N+1.
void gen_join(const MineLevel &P, MineLevel &L) {
    const int N = P.N;
    const int64_t mp = P.m;
    const std::vector<int64_t> &F = P.freq;
    auto ty = [&](int64_t i, int k) { return P.types[(size_t)k * mp + i]; };
    auto iv = [&](int64_t i, int k) { return P.iv[(size_t)k * mp + i]; };
    // order frequent episodes by their first N-1 nodes (types and intervals)
    std::vector<int64_t> byprefix(F);
    auto prefix_less = [&](int64_t a, int64_t b) {
        for (int k = 0; k < N - 1; ++k) {
            if (ty(a, k) != ty(b, k)) return ty(a, k) < ty(b, k);
            if (k < N - 2 && iv(a, k) != iv(b, k)) return iv(a, k) < iv(b, k);
        }
        return false;
    };
    std::sort(byprefix.begin(), byprefix.end(), prefix_less);
    // compare the prefix of beta with the suffix (last N-1 nodes) of alpha
    auto cmp_prefix_suffix = [&](int64_t beta, int64_t alpha) {
        for (int k = 0; k < N - 1; ++k) {
            if (ty(beta, k) != ty(alpha, k + 1)) return ty(beta, k) < ty(alpha, k + 1) ? -1 : 1;
            if (k < N - 2 && iv(beta, k) != iv(alpha, k + 1)) return iv(beta, k) < iv(alpha, k + 1) ? -1 : 1;
        }
        return 0;
    };
    const int64_t nf = (int64_t)F.size();
    std::vector<int64_t> rlo(nf), rhi(nf), cnt(nf + 1, 0);
    // both passes split the frequent episodes over host threads
    const int nt = (int)std::max<unsigned>(1, std::min<unsigned>(32, std::thread::hardware_concurrency()));
    auto parallel = [&](auto &&body) {
        std::vector<std::thread> th;
        const int64_t chunk = (nf + nt - 1) / nt;
        for (int q = 0; q < nt; ++q) {
            const int64_t x0 = q * chunk, x1 = std::min(nf, x0 + chunk);
            if (x0 >= x1) break;
            th.emplace_back([&, x0, x1] { body(x0, x1); });
        }
        for (auto &t : th) t.join();
    };
    parallel([&](int64_t x0, int64_t x1) {
        for (int64_t x = x0; x < x1; ++x) {
            const int64_t a = F[x];
            const auto lo = std::partition_point(byprefix.begin(), byprefix.end(),
                                                 [&](int64_t b) { return cmp_prefix_suffix(b, a) < 0; });
            const auto hi =
                std::partition_point(lo, byprefix.end(), [&](int64_t b) { return cmp_prefix_suffix(b, a) == 0; });
            rlo[x] = lo - byprefix.begin();
            rhi[x] = hi - byprefix.begin();
            int64_t c = 0;
            for (int64_t r = rlo[x]; r < rhi[x]; ++r)
                if (ty(byprefix[r], N - 1) != ty(a, 0)) ++c;
            cnt[x + 1] = c;
        }
    });
    for (int64_t x = 0; x < nf; ++x) cnt[x + 1] += cnt[x];
    const int64_t m = cnt[nf];
    L.N = N + 1;
    L.m = m;
    L.types.resize((size_t)(N + 1) * m);
    L.iv.resize((size_t)N * m);
    parallel([&](int64_t x0, int64_t x1) {
        for (int64_t x = x0; x < x1; ++x) {
            const int64_t a = F[x];
            int64_t c = cnt[x];
            for (int64_t r = rlo[x]; r < rhi[x]; ++r) {
                const int64_t b = byprefix[r];
                if (ty(b, N - 1) == ty(a, 0)) continue;
                for (int k = 0; k < N; ++k) L.types[(size_t)k * m + c] = ty(a, k);
                L.types[(size_t)N * m + c] = ty(b, N - 1);
                for (int k = 0; k < N - 1; ++k) L.iv[(size_t)k * m + c] = iv(a, k);
                L.iv[(size_t)(N - 1) * m + c] = iv(b, N - 2);
                ++c;
            }
        }
    });
}

void select_frequent(MineLevel &L, int64_t threshold) {
    L.freq.clear();
    for (int64_t i = 0; i < L.m; ++i)
        if (L.counts[i] > threshold) L.freq.push_back(i);
    L.nf = (int64_t)L.freq.size();
}

}  // namespace epi
