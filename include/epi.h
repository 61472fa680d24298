/*
 * epi.h -- C ABI of the MI355X (gfx950) serial-episode counting engine.
 *
 * The engine counts, exactly, the non-overlapped occurrences of serial
 * episodes with inter-event constraints in a long event stream:
 *   - event stream (E_i, t_i), i = 0..n-1, integer times, t_i <= t_{i+1},
 *     E_i in 0..K-1                                          (paper, Def. 1)
 *   - serial episode alpha = (A_1 .. A_N), distinct types, 1 <= N <= 8
 *                                                            (paper, Def. 2)
 *   - constraint j (j = 1..N-1):  lo_j < t(A_{j+1}) - t(A_j) <= hi_j,
 *     0 <= lo_j < hi_j                                 (paper, Sec. II-C)
 *   - frequency = size of the largest set of occurrences no two of which
 *     overlap in time; occurrences sharing a timestamp overlap
 *                                      (paper, Sec. II-C, Sec. IV-A, Alg. 1)
 *
 * Conventions for every entry point:
 *   - the return value is a status: EPI_OK (0) or a negative error code;
 *     nothing aborts or throws across the ABI, and the message of the last
 *     error of a context is available from epi_last_error();
 *   - HIP runtime failures map to EPI_EDEVICE (message = hipError string);
 *   - a context is not thread-safe: use one per host thread;
 *   - host inputs are copied before the call returns; "_device" inputs are
 *     borrowed until epi_sync() returns;
 *   - outputs go to caller-owned buffers; device memory made by the library
 *     is owned by the context and freed by epi_release_* and epi_destroy;
 *   - there is no CPU fallback: every count is computed by HIP kernels.
 *
 * Timestamps are unit-agnostic integers, int32 (EPI_TS_I32) or int64
 * (EPI_TS_I64); by convention microseconds and nanoseconds.  Candidate
 * interval bounds are always passed as int64 and must fit the stream's
 * timestamp type together with the stream's times (see EPI_EOVERFLOW).
 */
#ifndef EPI_H
#define EPI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct epi_ctx epi_ctx;
typedef int32_t epi_status;

enum {
    EPI_OK = 0,
    EPI_EINVAL = -1,    /* null pointer, bad enum, bad size argument            */
    EPI_EUNSORTED = -2, /* stream times decrease somewhere                       */
    EPI_ETYPE = -3,     /* event or episode type outside [0, K)                  */
    EPI_EINTERVAL = -4, /* an interval violates 0 <= lo < hi                     */
    EPI_ESIZE = -5,     /* episode size outside 1..8, or n / K / m out of range  */
    EPI_EREPEAT = -6,   /* a type occurs twice in one episode (unless allowed)   */
    EPI_EOVERFLOW = -7, /* times +- the episode span leave the timestamp type    */
    EPI_ENOMEM = -8,    /* device or host allocation failed                      */
    EPI_EDEVICE = -9,   /* HIP runtime error or a device-side check failed       */
    EPI_ESTATE = -10    /* unknown id, or counts read before a count was issued  */
};

enum { EPI_TS_I32 = 0, EPI_TS_I64 = 1 };
enum { EPI_MODE_PLAIN = 0, EPI_MODE_BATCHED = 1, EPI_MODE_INCREMENTAL = 2, EPI_MODE_TRACKING = 3 };
enum { EPI_SCHED_RR = 0, EPI_SCHED_LEARNED = 1, EPI_SCHED_HEURISTIC = 2, EPI_SCHED_MEASURED = 3 };

#define EPI_MAX_N 8 /* largest episode size */

/* ------------------------------------------------------------------------
 * Contexts
 * ---------------------------------------------------------------------- */

/* Create a context bound to HIP device `device` (0-based).  *out receives the
 * context.  EPI_EDEVICE if the device cannot be selected. */
epi_status epi_create(int device, epi_ctx **out);

/* Free every device buffer of the context and the context itself.  Waits
 * for outstanding work.  Null is accepted. */
void epi_destroy(epi_ctx *ctx);

/* Message of the context's last error ("" if none).  Valid until the next
 * call on the context.  Null ctx: the message of the last failed
 * epi_create on this thread. */
const char *epi_last_error(const epi_ctx *ctx);

/* Static name of a status code. */
const char *epi_status_string(epi_status s);

/* ------------------------------------------------------------------------
 * Host-only validators (no GPU touched; also used internally)
 * ---------------------------------------------------------------------- */

/* Check a host stream: n >= 0 (n < 2^31), 1 <= K <= 65536, every type in
 * [0, K), times non-decreasing (Def. 1), and every time strictly inside the
 * timestamp type's range (its minimum and maximum are reserved).
 * `times` is int32_t[n] or int64_t[n] according to ts_kind. */
epi_status epi_validate_stream(const int32_t *types, const void *times, int64_t n, int ts_kind,
                               int32_t K);

/* Check m candidate episodes (Def. 2, Sec. II-C):
 *   N[c] in 1..8; types[c*8 + j] in [0, K) and distinct for j < N[c]
 *   (epi_submit_candidates admits repeats under EPI_OPT_ALLOW_REPEATS);
 *   0 <= lo[c*7 + j] < hi[c*7 + j] for j < N[c]-1; the span sum_j hi
 *   fits the timestamp type.  Slots beyond N[c] are ignored. */
epi_status epi_validate_candidates(int64_t m, const uint8_t *N, const int32_t *types,
                                   const int64_t *lo, const int64_t *hi, int32_t K,
                                   int ts_kind);

/* ------------------------------------------------------------------------
 * Streams (Def. 1) and the per-type index (pre-processing of Sec. IV-A)
 * ---------------------------------------------------------------------- */

/* Copy a host stream to the device, validate it, and build its per-type
 * index (events grouped by type, each group in time order).  *stream_id
 * receives a handle.  Errors: the validator's codes, EPI_ENOMEM, EPI_EDEVICE. */
epi_status epi_load_stream(epi_ctx *ctx, const int32_t *types, const void *times, int64_t n,
                           int ts_kind, int32_t K, int32_t *stream_id);

/* Same, from device buffers (int32 types, int32/int64 times) enqueued on
 * `hip_stream` (hipStream_t; null = the context's stream).  The inputs are
 * validated on the device; a violation is reported as EPI_EUNSORTED or
 * EPI_ETYPE by this call (it synchronises once to read the result). */
epi_status epi_load_stream_device(epi_ctx *ctx, const int32_t *d_types, const void *d_times,
                                  int64_t n, int ts_kind, int32_t K, void *hip_stream,
                                  int32_t *stream_id);

/* Number of events, K and timestamp kind of a loaded stream. */
epi_status epi_stream_info(epi_ctx *ctx, int32_t stream_id, int64_t *n, int32_t *K,
                           int *ts_kind);

/* Copy the per-type index back: off[K+1] (int32) and the timestamps grouped
 * by type (ts_kind width, n entries).  For inspection and tests. */
epi_status epi_read_type_index(epi_ctx *ctx, int32_t stream_id, int32_t *off, void *ts_by_type);

epi_status epi_release_stream(epi_ctx *ctx, int32_t stream_id);

/* ------------------------------------------------------------------------
 * Candidate sets
 * ---------------------------------------------------------------------- */

/* Validate m host candidates against the stream (see epi_validate_candidates
 * and EPI_EOVERFLOW: min time - span and max time + span must stay inside the
 * timestamp type) and copy them to the device.  m may be 0.
 * Layout: N[m] (uint8), types[m*8] (int32), lo[m*7], hi[m*7] (int64). */
epi_status epi_submit_candidates(epi_ctx *ctx, int32_t stream_id, int64_t m, const uint8_t *N,
                                 const int32_t *types, const int64_t *lo, const int64_t *hi,
                                 int32_t *set_id);

epi_status epi_release_set(epi_ctx *ctx, int32_t set_id);

/* ------------------------------------------------------------------------
 * Counting
 * ---------------------------------------------------------------------- */

/* Enqueue the count of k candidate sets on `hip_stream` (null = the
 * context's stream).  mode:
 *   EPI_MODE_PLAIN    one launch per set and episode-size class, candidates
 *                     in submission order (asynchronous);
 *   EPI_MODE_BATCHED  all sets (possibly on different streams of one
 *                     timestamp kind) in one captured graph: one persistent
 *                     kernel per launch class (episode size, ring class,
 *                     machine time type) pulls (set, lane block, segment)
 *                     work items from a device queue, then the segmented
 *                     ones are reconciled.  The graph is kept per (sets,
 *                     schedule, options, cost model) and replayed by later
 *                     calls, which are asynchronous; a call that plans a
 *                     new graph synchronises the stream while it plans, and
 *                     episodes with a ring bound above 15 (counted by the
 *                     tracking engine) make the call return when done.
 *   EPI_MODE_INCREMENTAL  after epi_append_stream: only the appended
 *                     events are counted (see epi_append_stream).
 *   EPI_MODE_TRACKING parallel over events instead of episodes, for a few
 *                     long episodes over a long stream (Parallel Local
 *                     Tracking, Sec. IV-C, then the greedy of Alg. 1,
 *                     Sec. IV-A): node by node, every event of the node's
 *                     type finds by binary search the latest start of a
 *                     chain ending at it, the events with a chain are
 *                     compacted in time order (Sec. IV-D/E), and the count
 *                     is the greedy over the (latest start, end) intervals,
 *                     ranked by pointer jumping.  Working memory about
 *                     5*ts + 32 bytes (8*ts + 32 under
 *                     EPI_OPT_STREAM_ORDER) per event of an episode's most
 *                     frequent type, in groups of at most 2 GiB, kept with
 *                     the set for its next count; no work log; returns when
 *                     done.  The only mode for sets submitted under
 *                     EPI_OPT_STREAM_ORDER.
 * sched (batched mode): EPI_SCHED_RR keeps submission order;
 * EPI_SCHED_LEARNED orders each class's episodes by the cost model's
 * predicted work (see epi_costmodel_train; without a trained model it falls
 * back to EPI_SCHED_RR), cuts costly lane blocks into more time segments and
 * queues items longest first; EPI_SCHED_HEURISTIC does the same with the
 * sum of the types' event counts as the cost; EPI_SCHED_MEASURED with the
 * work each episode logged in the set's latest count that kept a work log
 * (events visited + records + queries; EPI_ESTATE for a set that never
 * logged): the schedule an exact cost model would give, for comparison.
 * The counts never depend on mode or sched. */
epi_status epi_count(epi_ctx *ctx, const int32_t *set_ids, int32_t k, int mode, int sched,
                     void *hip_stream);

/* Streaming (the streaming direction of the paper's Future Work section,
 * here exact): append n events to a loaded stream.  Same checks as
 * epi_load_stream, and the first appended time must not precede the
 * stream's last one (EPI_EUNSORTED).  The per-type index is rebuilt;
 * synchronous (the device is idle when it returns).  Sets on the stream keep
 * their counts, which then cover the events before the append, until they
 * are counted again: fully (EPI_MODE_PLAIN / EPI_MODE_BATCHED) or
 * incrementally (EPI_MODE_INCREMENTAL).
 *
 * EPI_MODE_INCREMENTAL in epi_count: a set never counted is counted fully
 * (as EPI_MODE_PLAIN); a set counted before one or more appends only adds
 * the occurrences completed by the appended events.  Each episode keeps its
 * last completion tau from every count, and its machine resumes from the
 * state right after max(tau, B - H - 1) (B = the first appended time, H =
 * the episode's longest span): an occurrence ending at or after B starts at
 * or after B - H, so nothing before that point can still complete (the
 * reasoning of the segment reconciliation).  The counts equal a full count
 * of the whole stream.  Sets from level-wise discovery cannot be counted
 * this way (EPI_EINVAL). */
epi_status epi_append_stream(epi_ctx *ctx, int32_t stream_id, const int32_t *types, const void *times, int64_t n);

/* Engine options (per context), used by tests and by tuning:
 *   EPI_OPT_SEGMENTS      0 = automatic (default); k >= 1 = cut the stream
 *                         into k time segments counted in parallel and
 *                         reconciled exactly (1 = no segmentation)
 *   EPI_OPT_LANES         0 = automatic (default); else the largest number
 *                         of episodes per workgroup (64, 128 or 256); the
 *                         engine uses the widest one whose state fits LDS
 *   EPI_OPT_TARGET_LANES  automatic segmentation aims at this many
 *                         (episode, segment) work lanes (default 262144)
 *   EPI_OPT_PAIR_FILTER   1 (default) / 0: in level-wise discovery with the
 *                         state-machine engine, precompute for each event,
 *                         event type and menu interval whether a constrained
 *                         neighbour exists before and after it (the tracking
 *                         step of Sec. IV-C, for all pairs at once) and skip
 *                         events with none
 *   EPI_OPT_MINE_ENGINE   level-wise discovery engine: 1 (default) extends the
 *                         previous level's chain lists (decomposition of
 *                         Sec. IV-A: one walk over the stream windows that
 *                         follow each frequent episode's end events serves
 *                         all of its extensions; menus of up to 8 intervals,
 *                         longer menus use engine 0); 0 counts every
 *                         candidate with the state machines of epi_count
 *   EPI_OPT_WORKLOG       1 / 0 (default): counts also record, per episode,
 *                         kWork = 5 int32 counters (events visited, partial
 *                         occurrences recorded, predecessor queries,
 *                         completions, deepest interval ring) and, in batched
 *                         mode, a wall-clock start/end per work item
 *   EPI_OPT_TARGET_ITEMS  accepted for compatibility; the batched scheduler
 *                         cuts every lane block of a launch group into the
 *                         same segments (EPI_OPT_TARGET_LANES) and orders
 *                         the items on the device, so it has no effect
 *   EPI_OPT_MINE_LIST_BYTES  level-wise discovery, extension engine: device
 *                         bytes that the end-event lists of every candidate
 *                         of a level may take (default 8 GiB); a level with
 *                         few frequent parent episodes is counted from those
 *                         lists, listed by walks cut into pieces, when they
 *                         fit; else one walk per parent counts it and a
 *                         second writes its chain lists (0 = always the
 *                         latter)
 *   EPI_OPT_MINE_LIST_ALPHAS  level-wise discovery, extension engine: levels
 *                         with fewer frequent parent episodes than this
 *                         (default 65536) take the list path when it fits;
 *                         the others count with one walk per parent, and
 *                         write their chain lists with walks cut into pieces
 *                         (a size walk, then a list walk, over the frequent
 *                         extensions) when the parents with frequent
 *                         extensions are few and the list budget is not 0,
 *                         else with one walk per such parent
 *   EPI_OPT_ALLOW_REPEATS 0 (default) / 1: epi_submit_candidates accepts
 *                         episodes in which a type occurs at several nodes
 *                         (Def. 2 does not exclude them; e.g. A -> B -> A).
 *                         An occurrence still takes one event per node with
 *                         strictly increasing times (every lower bound is
 *                         >= 0 and strict), so one event never fills two
 *                         nodes of an occurrence; the state machines take
 *                         each event at every node of its type.
 *   EPI_OPT_STREAM_ORDER  0 (default) / 1: candidate sets submitted while
 *                         it is 1 decide overlap in stream order, the reset
 *                         of the serial state machine of Sec. III-A taken
 *                         literally: after a completion, any event later in
 *                         the stream may start an occurrence, so two
 *                         occurrences are non-overlapped iff one's last
 *                         event precedes the other's first event in the
 *                         stream (a one-node episode counts every event of
 *                         its type).  Equal to the default (time) semantics
 *                         on streams without equal timestamps.  Such sets
 *                         are counted by EPI_MODE_TRACKING only (other
 *                         modes: EPI_EINVAL).
 *   EPI_OPT_LANE_ENGINE   1 (default) / 0: the state machines keep their
 *                         bookkeeping in registers and, per node, a ring of
 *                         exactly that interval's bound in LDS (lane
 *                         machines), wherever the stream's tiles allow int32
 *                         times relative to the tile; 0 = every group on the
 *                         machines with all their state in LDS (each ring as
 *                         deep as the episode's deepest)
 *   EPI_OPT_RING_CLASSES  batched mode: how episodes of one size form launch
 *                         groups (each group's episodes are ordered by cost
 *                         and cut into lane blocks, and its interval rings
 *                         take the group's largest): 0 (default) = the
 *                         submission groups (size x ring-entries class of
 *                         1, 2, ... 112 entries), 1 = one group per size,
 *                         2 = three per size (ring entries per interval on
 *                         average <= 2, <= 3, more); fewer groups let the
 *                         cost order pack lanes of closer work into a wave
 *                         at a larger LDS footprint
 * EPI_EINVAL for an unknown option or value.  Counts never depend on the
 * engine options (EPI_OPT_ALLOW_REPEATS only widens what is accepted;
 * EPI_OPT_STREAM_ORDER selects the other overlap semantics). */
enum { EPI_OPT_SEGMENTS = 1, EPI_OPT_LANES = 2, EPI_OPT_TARGET_LANES = 3, EPI_OPT_PAIR_FILTER = 4,
       EPI_OPT_MINE_ENGINE = 5, EPI_OPT_WORKLOG = 6, EPI_OPT_TARGET_ITEMS = 7, EPI_OPT_MINE_LIST_BYTES = 8,
       EPI_OPT_ALLOW_REPEATS = 9, EPI_OPT_MINE_LIST_ALPHAS = 10, EPI_OPT_STREAM_ORDER = 11,
       EPI_OPT_LANE_ENGINE = 12, EPI_OPT_RING_CLASSES = 13 };
epi_status epi_set_option(epi_ctx *ctx, int option, int64_t value);

/* Autotune the batched engine for these sets and schedule by coordinate
 * descent from the defaults, one knob at a time: the streams' tile size
 * (largest events per tile: the default 2048, then {4096, 1024, 512}; the
 * streams are re-tiled), the
 * launch groups (EPI_OPT_RING_CLASSES {0, 1, 2}), lanes per workgroup
 * (EPI_OPT_LANES {automatic, 128, 64}) and the segment target
 * (EPI_OPT_TARGET_LANES {131072, 524288, 1048576}), and once more over the
 * four when the first pass moved.  Each trial builds the
 * batched plan, then times two replays with hipEvents (the faster counts);
 * the counts do not
 * depend on the setting.  The fastest is kept: the streams stay re-tiled and
 * the options are set on the context.  With cache_path (may be null) the
 * choice is appended to that text file under a key of the workload's shape
 * (timestamp kind, schedule, K, log2 sizes of events, candidates and
 * candidates per episode size); a later call with the same key applies it
 * without timing (unreadable or malformed entries are ignored).  chosen[4]
 * (may be null) receives tile size, ring classes, lanes (0 = automatic) and
 * segment target.  Sets from level-wise discovery or with stream-order
 * overlap: EPI_EINVAL. */
epi_status epi_autotune(epi_ctx *ctx, const int32_t *set_ids, int32_t k, int sched, const char *cache_path,
                        int64_t *chosen);

/* Wait for all work of the context and report device-side check failures. */
epi_status epi_sync(epi_ctx *ctx);

/* Blocking copy of a set's counts (int32, candidate order of submission) to
 * host memory counts[m]; m must equal the set's size.  EPI_ESTATE if the set
 * was never counted. */
epi_status epi_read_counts(epi_ctx *ctx, int32_t set_id, int32_t *counts, int64_t m);

/* Work log of the set's last count (EPI_OPT_WORKLOG): work[m][5] int32,
 * submission order.  EPI_ESTATE when the last count did not record one. */
epi_status epi_read_worklog(epi_ctx *ctx, int32_t set_id, int32_t *work, int64_t m);

/* Wall-clock (constant-rate device counter) start and end of every work item
 * of the last batched count that included this set (cycles[n_items][2]);
 * with cycles = null only *n_out receives the number of items. */
epi_status epi_read_item_cycles(epi_ctx *ctx, int32_t set_id, int64_t *cycles, int64_t n_items, int64_t *n_out);

/* epi_count in EPI_MODE_PLAIN for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same counts, written to the set's counts buffer, with
 * `segments` time segments per launch group (0: automatic, as
 * EPI_OPT_SEGMENTS = 0), and the per-(segment, episode) records of the
 * segment-parallel count kept in the library's static device scratch of
 * 64 MiB (held per device until the process ends).  Calls no hipMalloc,
 * hipFree or host synchronisation; asynchronous on hip_stream (null: the
 * context's stream); the work log is not recorded.  Every call on one GPU
 * shares that scratch: calls that overlap on one GPU (other streams or other
 * contexts) race; calls on one stream are ordered and safe.  Errors:
 * EPI_ESIZE when a launch group's records exceed the scratch (fewer
 * segments fit), EPI_EINVAL for sets with stream-order overlap or with
 * episodes deeper than the rings (both need the tracking engine's working
 * memory), EPI_ESTATE for an unknown set. */
epi_status epi_count_noalloc(epi_ctx *ctx, int32_t set_id, int64_t segments, void *hip_stream);

/* Batched plans of the context: *plans_built = plans captured and
 * instantiated so far, *replays = batched counts that launched a kept plan
 * again (no capture, no instantiation, no host scheduling), *plans_kept =
 * plans held now (at most 8, least recently used dropped first).  A plan is
 * kept per (set list, schedule, options, cost model); releasing a set drops
 * the plans that count it, appending to or releasing a stream drops all.
 * Any pointer may be null. */
epi_status epi_batched_stats(epi_ctx *ctx, int64_t *plans_built, int64_t *replays, int64_t *plans_kept);

/* The lane order of the set's last batched count (while its plan is kept;
 * EPI_ESTATE otherwise): order[i] = submission index of the episode counted
 * in lane slot i, block[i] = the workgroup-sized lane block of slot i (blocks
 * numbered per set; lanes 64 at a time form the waves of a block; -1: the
 * slot is counted by the tracking engine).  Blocks the scheduler ordered by
 * cost hold episodes of similar predicted work, the divergence of Sec. V-C
 * that the schedule attacks.  order and block are host arrays of m. */
epi_status epi_read_schedule(epi_ctx *ctx, int32_t set_id, int32_t *order, int32_t *block, int64_t m);

/* Device pointer to a set's counts (int32[m], submission order), valid until
 * the set is released; contents are defined once the count's stream work is
 * complete. */
epi_status epi_counts_device(epi_ctx *ctx, int32_t set_id, const int32_t **d_counts);

/* ------------------------------------------------------------------------
 * Cost model of the scheduler: a perceptron with two hidden ReLU layers of
 * 64 units (FP32), y = relu(relu(x W1 + b1) W2 + b2) w3 + b3, trained on the
 * mean squared error with Adam (b1 0.9, b2 0.999, eps 1e-8) by the
 * library's own HIP kernels.  Parameters are one flat FP32 vector:
 * W1[F][64], b1[64], W2[64][64], b2[64], w3[64], b3[1].  The model only
 * orders work; counts never depend on it.
 * ---------------------------------------------------------------------- */

/* Create the context's model for n_features inputs (1..4096): He-uniform
 * weights from a SplitMix64 stream seeded by `seed`, zero biases, Adam state
 * cleared. */
epi_status epi_mlp_init(epi_ctx *ctx, int32_t n_features, uint64_t seed);

/* Number of inputs and parameters of the model (EPI_ESTATE before init). */
epi_status epi_mlp_params(epi_ctx *ctx, int32_t *n_features, int64_t *n_params);

/* Copy the parameters out / in (n = number of parameters); setting them
 * clears the Adam state. */
epi_status epi_mlp_get_params(epi_ctx *ctx, float *p, int64_t n);
epi_status epi_mlp_set_params(epi_ctx *ctx, const float *p, int64_t n);

/* Forward pass on B host samples X[B][F] -> y[B] (host). */
epi_status epi_mlp_forward(epi_ctx *ctx, const float *X, int64_t B, float *y);

/* Loss mean_i (y_i - t_i)^2 and its gradient g[n_params] (host), for host
 * samples X[B][F] and targets t[B]. */
epi_status epi_mlp_grad(epi_ctx *ctx, const float *X, const float *t, int64_t B, float *loss, float *g);

/* One Adam step with gradient g (host) and learning rate lr. */
epi_status epi_mlp_adam_step(epi_ctx *ctx, const float *g, float lr);

/* Train on B host samples for `epochs` passes of consecutive mini-batches
 * of `batch` samples (order as given); losses[epochs] (may be null)
 * receives each epoch's mean loss. */
epi_status epi_mlp_train(epi_ctx *ctx, const float *X, const float *t, int64_t B, int32_t epochs, int32_t batch,
                         float lr, float *losses);

/* Train the cost model on sets counted with the work log on (best without
 * time segments, EPI_OPT_SEGMENTS = 1, so each episode's logged work is its
 * own): features x of each episode -> t = log1p(events visited + records +
 * queries) - x[23], the correction of log work relative to the log of the
 * summed event counts of the episode's types (feature 23, the event-count
 * heuristic).  Features and target are standardised on the training set
 * (x' = (x - x_mu) * x_isd with x_isd = 1 / standard deviation, 0 for a
 * constant feature; t' = (t - y_mu) / y_sd), shuffled once, and a fresh model
 * seeded by `seed` is trained on (x', t') for `epochs` passes of Adam
 * (lr 3e-3, mini-batches of 512); losses[epochs] (may be null) receives the
 * epoch losses in standardised units (1 = the target's variance).  The
 * cost model's prediction of log1p(work) is then x[23] + y_sd * net(x') + y_mu. */
epi_status epi_costmodel_train(epi_ctx *ctx, const int32_t *set_ids, int32_t k, int32_t epochs, uint64_t seed,
                               float *losses);

/* The cost model's standardisation: x_mu[F], x_isd[F] and y_mu_sd[2] =
 * {y_mu, y_sd} (identity after epi_mlp_init; any pointer may be null). */
epi_status epi_costmodel_scaling(epi_ctx *ctx, float *x_mu, float *x_isd, float *y_mu_sd);

/* Save the cost model (parameters and standardisation) to a file / load it
 * into the context (replacing any model; Adam state cleared).  The file is
 * binary: "EPICR001", int32 F, int64 n_params, float params[n_params],
 * float x_mu[F], float x_isd[F], float y_mu, float y_sd, host byte order.
 * EPI_ESTATE when saving without a model; EPI_EINVAL for a path that cannot
 * be opened or a file that is not exactly this layout. */
epi_status epi_costmodel_save(epi_ctx *ctx, const char *path);
epi_status epi_costmodel_load(epi_ctx *ctx, const char *path);

/* The cost model's predicted log1p(work) of every candidate of a set
 * (submission order, y[m]); the model must take the 24 features below.
 * The learned schedule orders work by exp of this prediction. */
epi_status epi_costmodel_predict(epi_ctx *ctx, int32_t set_id, float *y, int64_t m);

/* The model's 24 input features of every candidate of a set (submission
 * order, X[m][24]): log1p of the event count of each node's type (8, zero
 * padded), log1p(hi - lo) and log1p(hi) of each constraint (7 + 7), N, and
 * log1p of the sum of the nodes' type event counts. */
epi_status epi_costmodel_features(epi_ctx *ctx, int32_t set_id, float *X, int64_t m);

/* ------------------------------------------------------------------------
 * Level-wise discovery (Sec. II-C: candidates of size N are generated from
 * the frequent episodes of size N-1 and counted in one pass per level; an
 * episode is frequent when its count is greater than the threshold)
 * ---------------------------------------------------------------------- */

/* Mine the loaded stream level by level, up to episodes of max_size nodes
 * (1..8), with inter-event intervals drawn from a menu of n_menu (1..255)
 * intervals (menu_lo[i], menu_hi[i]].
 *   level 1: every type as a 1-node episode;
 *   level 2: ordered pairs of distinct frequent types x every menu interval;
 *   level N+1: alpha + (last node of beta) for frequent N-node alpha, beta
 *     whose nodes 2..N of alpha equal nodes 1..N-1 of beta, intervals
 *     included, when the new type is not alpha's first.
 * Stops early when a level has no frequent episode.  Synchronous: returns
 * when every level is counted; *mine_id receives a handle.  The levels run
 * on the context's stream, after the work queued on hip_stream so far (null:
 * none).  Their device memory comes from a cache of the context, which
 * keeps released blocks for reuse by later runs until epi_destroy (and gives
 * them back to the device when an allocation would otherwise fail).
 * Errors: EPI_EINTERVAL / EPI_EOVERFLOW for a bad menu, EPI_ESIZE for a bad
 * max_size, plus those of counting. */
epi_status epi_mine(epi_ctx *ctx, int32_t stream_id, int32_t n_menu, const int64_t *menu_lo,
                    const int64_t *menu_hi, int32_t max_size, int64_t threshold, void *hip_stream,
                    int32_t *mine_id);

/* Number of levels counted by a mining run (level numbers are 1..n). */
epi_status epi_mine_levels(epi_ctx *ctx, int32_t mine_id, int32_t *n_levels);

/* Candidates and frequent episodes of a level; times_ms (may be null)
 * receives 3 doubles: candidate generation, count incl. transfers, and
 * counting kernels alone (HIP events), in milliseconds. */
epi_status epi_mine_level_info(epi_ctx *ctx, int32_t mine_id, int32_t level, int64_t *n_candidates,
                               int64_t *n_frequent, double *times_ms);

/* Copy a level's candidates (frequent_only = 0) or frequent episodes (1) with
 * their counts, in the layout of epi_submit_candidates; m must equal the
 * level's candidate or frequent count.  Unused type slots are -1. */
epi_status epi_mine_read(epi_ctx *ctx, int32_t mine_id, int32_t level, int frequent_only, int64_t m,
                         uint8_t *N, int32_t *types, int64_t *lo, int64_t *hi, int32_t *counts);

/* Copy k candidates of a level chosen by index (0 <= idx[r] < candidates). */
epi_status epi_mine_read_at(epi_ctx *ctx, int32_t mine_id, int32_t level, int64_t k, const int64_t *idx,
                            uint8_t *N, int32_t *types, int64_t *lo, int64_t *hi, int32_t *counts);

/* Bytes the level's counting method must read and write (inputs per
 * candidate plus its outputs), for bandwidth accounting. */
epi_status epi_mine_level_bytes(epi_ctx *ctx, int32_t mine_id, int32_t level, int64_t *alg_bytes);

epi_status epi_mine_release(epi_ctx *ctx, int32_t mine_id);

#ifdef __cplusplus
}
#endif

#endif /* EPI_H */
