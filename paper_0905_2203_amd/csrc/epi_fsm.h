// Per-lane serial-episode state machine with its per-node state in LDS.
//
// The machine is the one of Sec. III-A, with the reading that overlap is
// decided on times (a start is admitted only strictly after the last
// completion e), so that its completions are exactly the greedy choices of
// Alg. 1 (earliest end among occurrences starting after e):
//   node 1 event at t:  if t > e, open a partial occurrence at t;
//   node j > 1 at t:    extends a partial occurrence recorded at node j-1 at
//                       time t' iff lo_{j-1} < t - t' <= hi_{j-1};
//   node N extension:   completion; e = t; all partial state is dropped.
// A record at node j at time t' matters only through its acceptance interval
// (t' + lo_j, t' + hi_j] for node j+1, so node j keeps the union of those
// intervals as a ring of disjoint intervals ordered by time: a query at t
// drops intervals ending before t and tests the front; a record first drops
// intervals ending before its own time (no later query can reach them), then
// merges into the back interval when they touch.  All live intervals end at
// or after the latest record, are pairwise separated and at least hi - lo
// long, so at most 1 + floor(hi / (hi - lo + 1)) are live at once: that bound
// sizes the ring.
//
// Dropping every partial record at a completion costs one bit: each
// completion at node N needs a record at every node since the previous
// completion, so every ring header is rewritten in every generation; a header
// whose generation bit differs from the lane's current one is empty.
//
// The machine's times are of type T: the stream's timestamps, or (int64
// streams whose tiles are short enough) int32 offsets from the start of the
// tile being walked, moved along with rebase() at every tile.
//
// LDS layout (W lanes, node slots k = 0..N-2, all lane-interleaved so that a
// wave-wide access to one slot touches consecutive words):
//   lohi[k*W + lane]           (lo_k, hi_k)
//   qh[k*W + lane]             count | head << 8 | generation << 16
//   qse[(k*Q + i)*W + lane]    interval i of the ring: (start, end]
#pragma once

#include "epi_internal.h"

namespace epi {

template <typename T>
struct __attribute__((aligned(2 * sizeof(T)))) Pair {
    T s, e;
};

template <typename T, int N>
struct LaneFsm {
    Pair<T> *lohi;
    uint32_t *qh;
    Pair<T> *qse;
    int W, lane, Q;
    T e;            // time of the last completion (type minimum: none)
    uint32_t gen;   // generation bit
    uint32_t maxq = 0;  // deepest ring seen (work log)

    __device__ __forceinline__ uint32_t pack(uint32_t hd, uint32_t n) const { return n | (hd << 8) | (gen << 16); }

    __device__ __forceinline__ void load_hdr(int k, uint32_t &hd, uint32_t &n) const {
        const uint32_t h = qh[k * W + lane];
        n = (h >> 16) == gen ? (h & 0xffu) : 0u;
        hd = (h >> 8) & 0xffu;
    }

    __device__ __forceinline__ uint32_t next(uint32_t i) const { return i + 1 == (uint32_t)Q ? 0u : i + 1; }

    __device__ __forceinline__ Pair<T> &slot(int k, uint32_t i) const { return qse[(k * Q + (int)i) * W + lane]; }

    // Empty every ring (explicitly, not through the generation bit).
    __device__ __forceinline__ void clear_all() {
        for (int k = 0; k < N - 1; ++k) qh[k * W + lane] = gen << 16;
    }

    // Relative times: move the origin d later.  Interval starts before the
    // new origin become -1 and ends before it -2: every later query or record
    // is at a time >= 0, for which both compare as they did (a start before
    // it, an end before it, i.e. dead).
    __device__ __forceinline__ void rebase(T d) {
        for (int k = 0; k < N - 1; ++k) {
            uint32_t hd, n;
            load_hdr(k, hd, n);
            for (uint32_t i = 0; i < n; ++i) {
                Pair<T> &v = slot(k, hd);
                const T s = v.s - d, e = v.e - d;
                v.s = s < T(-1) ? T(-1) : s;
                v.e = e < T(-2) ? T(-2) : e;
                hd = next(hd);
            }
        }
    }

    // Is t inside the acceptance intervals recorded at node slot k?  On a
    // miss, *nv receives the earliest time a later query can succeed with the
    // current intervals (front start + 1, or the type maximum when empty).
    __device__ __forceinline__ bool query(int k, T t, T *nv) {
        uint32_t hd, n;
        load_hdr(k, hd, n);
        const uint32_t n0 = n;
        Pair<T> f;
        f.s = T(0);
        f.e = T(0);
        while (n > 0) {
            f = slot(k, hd);
            if (f.e >= t) break;
            hd = next(hd);
            --n;
        }
        if (n != n0) qh[k * W + lane] = pack(hd, n);
        const bool ok = n > 0 && f.s < t;
        *nv = n > 0 ? (T)(f.s + 1) : TsLimits<T>::hi();
        return ok;
    }

    // Record an event of node slot k at time t; returns the start of its
    // acceptance interval.
    __device__ __forceinline__ T record(int k, T t, int32_t *flags) {
        const Pair<T> lh = lohi[k * W + lane];
        const T ns = t + lh.s, ne = t + lh.e;
        uint32_t hd, n;
        load_hdr(k, hd, n);
        Pair<T> f;
        f.s = T(0);
        f.e = T(0);
        while (n > 0) {
            f = slot(k, hd);
            if (f.e >= t) break;
            hd = next(hd);
            --n;
        }
        if (n > 0) {
            uint32_t bk = hd + n - 1;
            if (bk >= (uint32_t)Q) bk -= Q;
            const T be = n == 1 ? f.e : slot(k, bk).e;
            if (ns <= be) {
                slot(k, bk).e = ne;
                qh[k * W + lane] = pack(hd, n);
                return ns;
            }
        }
        if (n >= (uint32_t)Q) {
            atomicAdd(&flags[kFlagQueueOverflow], 1);  // cannot happen within the bound
            return ns;
        }
        uint32_t tl = hd + n;
        if (tl >= (uint32_t)Q) tl -= Q;
        if (n + 1 > maxq) maxq = n + 1;
        Pair<T> v;
        v.s = ns;
        v.e = ne;
        slot(k, tl) = v;
        qh[k * W + lane] = pack(hd, n + 1);
        return ns;
    }

    // One event of node j (0-based) at time t; true on a completion.
    __device__ __forceinline__ bool step(int j, T t, int32_t *flags) {
        T nv;
        const bool ok = j == 0 ? t > e : query(j - 1, t, &nv);
        if (!ok) return false;
        if (j == N - 1) {
            e = t;
            gen ^= 1u;
            return true;
        }
        (void)record(j, t, flags);
        return false;
    }
};

// LDS bytes of the state of W lanes.
template <typename T>
inline size_t fsm_lds_bytes(int N, int Q, int W) {
    if (N <= 1) return 0;
    return (size_t)(N - 1) * W * (sizeof(Pair<T>) * (1 + (size_t)Q) + sizeof(uint32_t));
}

}  // namespace epi
