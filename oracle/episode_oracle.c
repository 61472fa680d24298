/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Plain, slow, obviously-correct counting of non-overlapped occurrences of
 * serial episodes with inter-event constraints.  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark may load this library; the
 * product (the HIP engine) never calls it, and the two share no code.
 *
 * Definitions (Sec. II-C of the paper):
 *   - event stream: (E_i, t_i), i = 1..n, with t_i <= t_{i+1}           (Def. 1)
 *   - serial episode alpha = (A_1 .. A_N) of event types                  (Def. 2)
 *     (a type may occur at several nodes; an occurrence's times strictly
 *     increase, so one event never fills two nodes of an occurrence)
 *   - inter-event constraint j: lo_j < t(A_{j+1}) - t(A_j) <= hi_j        (Sec. II-C)
 *   - an occurrence is a tuple of events, one per node, meeting every
 *     constraint; its span is [start, end] = [t(A_1), t(A_N)]
 *   - two occurrences are non-overlapped iff one ends strictly before the
 *     other starts (the strict test of Alg. 1)
 *   - frequency = size of the largest set of pairwise non-overlapped
 *     occurrences (Sec. II-C, Sec. IV-A).
 *
 * Two formulations are implemented, independently of each other:
 *   ORACLE_DECOMP -- the decomposition of Sec. IV-A.  Subproblem-1 keeps,
 *     for every event x of type A_N, the occurrence ending at x with the
 *     latest start (a superset sufficient for the optimum); Subproblem-2 is
 *     the greedy interval scheduling of Alg. 1 over those (start, end) pairs
 *     in end order, with the previous end initialised to minus infinity.
 *   ORACLE_FSM -- the serial state machine of Sec. III-A: one list of times
 *     per node, old entries pruned when they can no longer satisfy the
 *     upper bound, a new event is recorded when a predecessor satisfies the
 *     constraint, and a completion at the last node counts one occurrence
 *     and clears every list.  Starts are admitted only strictly after the
 *     last completion, which makes the state machine compute exactly the
 *     greedy of Alg. 1 under the time-based overlap test.
 *
 *   ORACLE_FSM_STREAM -- the same state machine with the reset of the
 *     listing of Sec. III-A taken in stream order: after a completion, any
 *     event that comes later in the stream may start an occurrence (a start
 *     is admitted iff its stream position is after the last completion's),
 *     so two occurrences are non-overlapped iff one's last event precedes
 *     the other's first event in the stream.  It equals ORACLE_FSM on streams
 *     without equal timestamps and differs only at ties.
 *
 * Readings adopted where the paper is silent or inconsistent:
 *   - previous end starts at minus infinity (Alg. 1 writes 0);
 *   - completion is tested at the last node N (the commented listing tests
 *     one node earlier);
 *   - overlap is decided on times, so occurrences sharing a timestamp
 *     overlap; the result does not depend on the order of equal-time events;
 *   - a 1-node episode counts the distinct timestamps of its type.
 *
 * All arithmetic is in int64; times are widened on entry.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_DECOMP 0
#define ORACLE_FSM 1
#define ORACLE_FSM_STREAM 2
#define ORACLE_MAXN 8
#define NONE INT64_MIN

/* ---------------------------------------------------------------------------
 * Pre-processing (Sec. IV-A): the positions of the events of each type, in
 * stream order.  off[k]..off[k+1] indexes pos[] for type k.
 * ------------------------------------------------------------------------- */
typedef struct {
    int64_t K;
    int64_t *off;  /* K + 1 */
    int64_t *pos;  /* n */
} type_index;

static int build_index(const int32_t *types, int64_t n, int32_t K, type_index *ix) {
    ix->K = K;
    ix->off = (int64_t *)calloc((size_t)K + 1, sizeof(int64_t));
    ix->pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!ix->off || !ix->pos) return -1;
    for (int64_t i = 0; i < n; i++) ix->off[types[i] + 1]++;
    for (int32_t k = 0; k < K; k++) ix->off[k + 1] += ix->off[k];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(K > 0 ? K : 1));
    if (!fill) return -1;
    for (int32_t k = 0; k < K; k++) fill[k] = ix->off[k];
    for (int64_t i = 0; i < n; i++) ix->pos[fill[types[i]]++] = i;
    free(fill);
    return 0;
}

static void free_index(type_index *ix) {
    free(ix->off);
    free(ix->pos);
}

/* ---------------------------------------------------------------------------
 * Decomposition (Sec. IV-A) + Alg. 1.
 *   latest[k][x] = latest start over chains A_1..A_k that end at the x-th
 *   event of type A_k, or NONE when no such chain exists:
 *     latest[1][x] = t_x
 *     latest[k][x] = max over events y of type A_{k-1} with
 *                    lo_{k-1} < t_x - t_y <= hi_{k-1} of latest[k-1][y]
 *   Alg. 1 then walks the events of type A_N in time (= end) order.
 * ------------------------------------------------------------------------- */
static int64_t count_decomp(const int64_t *t, const type_index *ix, int N, const int32_t *ep,
                            const int64_t *lo, const int64_t *hi) {
    const int64_t *p0 = ix->pos + ix->off[ep[0]];
    int64_t n0 = ix->off[ep[0] + 1] - ix->off[ep[0]];
    int64_t *prev = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n0 > 0 ? n0 : 1));
    for (int64_t x = 0; x < n0; x++) prev[x] = t[p0[x]];
    const int64_t *pprev = p0;
    int64_t nprev = n0;
    for (int k = 1; k < N; k++) {
        const int64_t *pk = ix->pos + ix->off[ep[k]];
        int64_t nk = ix->off[ep[k] + 1] - ix->off[ep[k]];
        int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nk > 0 ? nk : 1));
        int64_t a = 0; /* first y with t_y >= tx - hi; tx only grows, so a only moves forward */
        for (int64_t x = 0; x < nk; x++) {
            int64_t tx = t[pk[x]];
            while (a < nprev && t[pprev[a]] < tx - hi[k - 1]) a++;
            int64_t best = NONE;
            for (int64_t y = a; y < nprev; y++) {
                int64_t d = tx - t[pprev[y]];
                if (d <= lo[k - 1]) break;          /* t_y too recent: later y are too */
                if (d > hi[k - 1]) continue;        /* cannot happen: a starts the window */
                if (prev[y] != NONE && prev[y] > best) best = prev[y];
            }
            cur[x] = best;
        }
        free(prev);
        prev = cur;
        pprev = pk;
        nprev = nk;
    }
    /* Alg. 1 over (start, end) = (prev[x], t_x), end-ordered */
    int64_t count = 0, prev_e = NONE;
    for (int64_t x = 0; x < nprev; x++) {
        if (prev[x] == NONE) continue;
        if (prev_e < prev[x]) {
            prev_e = t[pprev[x]];
            count++;
        }
    }
    free(prev);
    return count;
}

/* ---------------------------------------------------------------------------
 * Serial state machine (Sec. III-A).  s[j] holds, in time order, the times
 * of events of type A_{j+1} that close a valid chain A_1..A_{j+1} begun after
 * the last completion.  Lists are plain arrays with a moving front.
 * ------------------------------------------------------------------------- */
typedef struct {
    int64_t *v;
    int64_t head, len, cap;
} tlist;

static void tl_push(tlist *l, int64_t x) {
    if (l->len == l->cap) {
        /* compact the deleted front before growing */
        if (l->head > 0) {
            memmove(l->v, l->v + l->head, sizeof(int64_t) * (size_t)(l->len - l->head));
            l->len -= l->head;
            l->head = 0;
        }
        if (l->len == l->cap) {
            l->cap = l->cap ? 2 * l->cap : 16;
            l->v = (int64_t *)realloc(l->v, sizeof(int64_t) * (size_t)l->cap);
        }
    }
    l->v[l->len++] = x;
}

static int64_t count_fsm(const int32_t *types, const int64_t *t, int64_t n, int N,
                         const int32_t *ep, const int64_t *lo, const int64_t *hi, int stream_order) {
    tlist s[ORACLE_MAXN];
    memset(s, 0, sizeof(s));
    int64_t count = 0, e = NONE, pe = -1; /* time and stream position of the last completion */
    for (int64_t i = 0; i < n; i++) {
        int32_t E = types[i];
        /* nodes are scanned from the last to the first, as in Sec. III-A */
        for (int j = N - 1; j >= 0; j--) {
            if (E != ep[j]) continue;
            if (j == 0) {
                if (stream_order ? i > pe : t[i] > e) {
                    if (N == 1) {
                        count++;
                        e = t[i];
                        pe = i;
                    } else {
                        tl_push(&s[0], t[i]);
                    }
                }
            } else {
                tlist *pl = &s[j - 1];
                /* remove entries that can no longer meet the upper bound */
                while (pl->head < pl->len && pl->v[pl->head] < t[i] - hi[j - 1]) pl->head++;
                int found = 0;
                for (int64_t q = pl->len - 1; q >= pl->head; q--) {
                    int64_t d = t[i] - pl->v[q];
                    if (lo[j - 1] < d && d <= hi[j - 1]) {
                        found = 1;
                        break;
                    }
                }
                if (found) {
                    if (j == N - 1) {
                        count++;
                        e = t[i];
                        pe = i;
                        for (int k = 0; k < N; k++) s[k].head = s[k].len = 0;
                    } else {
                        tl_push(&s[j], t[i]);
                    }
                }
            }
            /* a type at several nodes: the event is taken at each of them,
             * last node first (a record at time t never admits a query at
             * the same t, so the order does not change the result) */
        }
    }
    for (int k = 0; k < ORACLE_MAXN; k++) free(s[k].v);
    return count;
}

/* ---------------------------------------------------------------------------
 * Exported entry points.
 *   cand_types: m x 8 (int32, unused slots ignored); cand_lo/hi: m x 7.
 *   method: ORACLE_DECOMP or ORACLE_FSM.  nthreads <= 0: runtime default.
 *   Returns 0, or -1 on allocation failure / bad input.
 * ------------------------------------------------------------------------- */
int oracle_count_batch(const int32_t *types, const int64_t *times, int64_t n, int32_t K, int64_t m,
                       const int32_t *cand_N, const int32_t *cand_types, const int64_t *cand_lo,
                       const int64_t *cand_hi, int method, int nthreads, int64_t *out_counts) {
    for (int64_t i = 0; i < n; i++)
        if (types[i] < 0 || types[i] >= K) return -1;
    for (int64_t c = 0; c < m; c++)
        if (cand_N[c] < 1 || cand_N[c] > ORACLE_MAXN) return -1;
    type_index ix;
    if (build_index(types, n, K, &ix) != 0) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < m; c++) {
        const int32_t *ep = cand_types + c * ORACLE_MAXN;
        const int64_t *lo = cand_lo + c * (ORACLE_MAXN - 1);
        const int64_t *hi = cand_hi + c * (ORACLE_MAXN - 1);
        if (method == ORACLE_FSM || method == ORACLE_FSM_STREAM)
            out_counts[c] = count_fsm(types, times, n, cand_N[c], ep, lo, hi, method == ORACLE_FSM_STREAM);
        else
            out_counts[c] = count_decomp(times, &ix, cand_N[c], ep, lo, hi);
    }
    free_index(&ix);
    return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
