/*
 * hist.h -- C ABI of the MI355X (gfx950) histogram-filling library.
 *
 * The library fills ROOT-style histograms on the GPU: for every event it finds
 * the bin on each axis, adds the event weight and its square to that bin, and
 * updates the statistics sums.  This is the Fill operation of arXiv:2401.13310
 * Sec. 3.1 (find bin with underflow/overflow bins, increment by a weight,
 * update the sums behind mean and standard deviation), with the statistics as
 * the transform-reduce sums of Sec. 3.2 and sums that accumulate across
 * bulks as required in Sec. 3.3.  A histogram object owns its device
 * allocations and takes bulks of events, and the result is copied back only
 * when it is read (Sec. 3.2).
 *
 * Conventions (shared with every entry point):
 *   - Bins: on an axis with n bins, bin 0 is underflow, bins 1..n are the
 *     in-range bins and bin n+1 is overflow.  Bins include their lower edge.
 *     Fixed-width axes use 1 + floor(n (x - xmin) / (xmax - xmin)) evaluated
 *     in IEEE binary64 left to right, clamped to n; variable axes return the
 *     number of edges e_i with !(x < e_i) (upper_bound).  NaN goes to
 *     overflow.  FP32 coordinates are widened exactly to binary64 first.
 *   - Global bin: g = b0 + (n0+2) * (b1 + (n1+2) * b2), x fastest; the total
 *     bin count is T = prod(n_a + 2), at most 2^31 - 1.
 *   - Statistics (events inside the range on every axis only):
 *       d=1 [Sw, Sw2, Swx, Swx2]
 *       d=2 [Sw, Sw2, Swx, Swx2, Swy, Swy2, Swxy]
 *       d=3 [Sw, Sw2, Swx, Swx2, Swy, Swy2, Swxy, Swz, Swz2, Swxz, Swyz]
 *     S = 2 + 2d + d(d-1)/2 values.  entries counts every event.
 *   - Streams are hipStream_t values passed as void* (NULL = null stream).
 *     Calls marked "asynchronous" enqueue work on the stream and return; the
 *     caller keeps every input buffer alive and unmodified until the stream
 *     has passed the call.  They never synchronize the device (hist_fill only
 *     when it must grow its scratch, see there).
 *   - Device pointers are plain HIP device addresses (e.g. a torch tensor's
 *     data_ptr()).  Host pointers are ordinary process memory.
 *   - Every function returns a hist_status; on error the handle is left as it
 *     was and hist_last_error() holds a message for the calling thread.
 *   - A handle may be used from one stream at a time.
 */
#ifndef HIST_H
#define HIST_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define HIST_API __attribute__((visibility("default")))
#else
#define HIST_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hist_s hist_t;
typedef struct hist_batch_s hist_batch_t;
typedef struct hist_multi_s hist_multi_t;

typedef enum {
    HIST_OK = 0,
    HIST_EINVAL = 1,    /* invalid argument                                 */
    HIST_ENOMEM = 2,    /* device or host allocation failed                 */
    HIST_EDEVICE = 3,   /* a HIP call failed (message in hist_last_error)   */
    HIST_ECAPTURE = 4,  /* a synchronizing call during stream capture       */
    HIST_ENOTSUP = 5    /* combination not supported                         */
} hist_status;

typedef enum { HIST_F64 = 0, HIST_F32 = 1 } hist_dtype;

/* One axis.  edges == NULL: nbins fixed-width bins on [xmin, xmax), both
 * finite, xmin < xmax.  Otherwise edges is a HOST pointer to nbins+1 finite,
 * strictly increasing values (copied by hist_create); xmin/xmax are ignored. */
typedef struct {
    int32_t nbins;
    double xmin, xmax;
    const double *edges;
} hist_axis;

/* hist_create flags */
#define HIST_F_ACC_F32C   (1u << 0)  /* FP32 fills accumulate in compensated FP32 LDS
                                        sums (TwoSum error terms for w and w^2),
                                        merged in FP64; otherwise FP32 inputs are
                                        accumulated in FP64 like FP64 inputs        */
#define HIST_F_LEARNED    (1u << 1)  /* train the learned find-bin index of every
                                        variable axis at creation (hist_train_index) */
#define HIST_F_NO_ALLOC   (1u << 2)  /* fills never allocate: a fill whose plan needs
                                        more scratch than hist_reserve set aside fails
                                        with HIST_ENOMEM instead of growing it       */

/* Accumulation strategies (hist_set_strategy / hist_plan_info).  */
typedef enum {
    HIST_STRAT_AUTO = 0,    /* heuristic, or the autotuner's choice after hist_tune   */
    HIST_STRAT_LDS = 1,     /* LDS-privatized window of bins, out-of-window events use
                               global atomics                                          */
    HIST_STRAT_GLOBAL = 2,  /* global atomics only                                     */
    HIST_STRAT_TILED = 3,   /* bins computed once into a scratch array, then bin-range
                               tiles accumulated in LDS                                */
    HIST_STRAT_PART = 4     /* bins computed once into a scratch array, events then
                               partitioned by bin range (a counting sort) so that one
                               workgroup accumulates each range in LDS and owns its
                               bins: no atomics on the histogram.  For histograms far
                               larger than LDS (about 1e5 bins and up).  Weights are
                               accumulated in FP64, also for HIST_F_ACC_F32C.          */
} hist_strategy;

/* Search used on a variable axis. */
typedef enum {
    HIST_SEARCH_BINARY = 0,   /* binary search over the edges (always available)  */
    HIST_SEARCH_LEARNED = 1   /* learned index + exact bounded search (needs
                                 hist_train_index)                                 */
} hist_search;

/* ---- lifecycle ---------------------------------------------------------- */

/* Creates a histogram on the current HIP device.  dims in 1..3, axes[dims].
 * Allocates and zeroes the device bin arrays, statistics and entry count
 * (scratch comes from hist_reserve or the first fill that needs it).
 * Errors: HIST_EINVAL (bad axes, T > 2^31-1, out == NULL), HIST_ENOMEM,
 * HIST_EDEVICE.  Synchronizes the device once (creation is not a hot call). */
HIST_API hist_status hist_create(int dims, const hist_axis *axes, uint32_t flags, hist_t **out);

/* Frees everything the handle owns.  NULL is accepted.  Synchronizes.
 * HIST_EINVAL, and nothing freed, while a live batch (hist_batch_create) or
 * multi-fill set (hist_multi_create) holds the handle: destroy those first. */
HIST_API hist_status hist_destroy(hist_t *h);

/* ---- the hot path ---------------------------------------------------------- */

/* Fill n events (Sec. 3.1 steps 1-3), adding to earlier fills (Sec. 3.3).
 * coords: HOST array of dims DEVICE pointers; coords[a][i] is coordinate a of
 * event i, n contiguous values of `dtype` each.  weights: DEVICE pointer to n
 * values of `dtype`, or NULL for unit weights.  n == 0 is a no-op.  The entry
 * count is kept on the device and grows by n when the fill runs, so fills
 * captured into a graph count once per replay.
 * Asynchronous on `stream`, launches kernels only (no memset, no copy).
 * Scratch: plans for histograms larger than LDS use the handle's scratch
 * memory (the staging slots of a merged LDS window, the bin array and tables
 * of the tiled and partitioned strategies).  When it is smaller than the plan
 * needs, the fill first grows it -- hipMalloc, and a synchronization of
 * `stream` before the old buffer is freed -- except during stream capture
 * (HIST_ECAPTURE) and for handles created with HIST_F_NO_ALLOC (HIST_ENOMEM).
 * After hist_reserve(n_max, ...) fills of up to n_max events allocate and
 * synchronize nothing and are capture-safe.
 * Errors: HIST_EINVAL (NULL handle, n < 0, NULL coordinate with n > 0;
 * HIST_F_ACC_F32C with FP64 inputs is not an error -- FP64 inputs always
 * accumulate in FP64), HIST_ENOMEM, HIST_ECAPTURE (scratch too small, see
 * above), HIST_EDEVICE (launch failure). */
HIST_API hist_status hist_fill(hist_t *h, const void *const *coords, const void *weights,
                      int64_t n, hist_dtype dtype, void *stream);

/* hist_fill for callers that cannot allocate (code under graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same fill, but every
 * scratch buffer the plan needs comes from one fixed region of
 * hist_static_scratch_bytes() (64 MiB) that the library holds in each GPU's
 * memory for the life of the process; it never calls hipMalloc, hipFree or a
 * synchronization, and never touches the handle's own scratch.  The staging
 * slots of a merged LDS window must fit the region (else HIST_ENOMEM, nothing
 * launched); the tiled and partitioned strategies process the events in
 * chunks whose bin array and tables fit it.  Scratch contents are not kept
 * between calls (whatever must start at zero is cleared by a kernel).  Every
 * call on a GPU shares that GPU's region: calls that overlap in time on one
 * GPU (on different streams, or from different threads) race and give wrong
 * results; serialize them on one stream.  Asynchronous on `stream`; same
 * arguments and errors as hist_fill (HIST_ENOMEM as above, HIST_ENOTSUP for a
 * device ordinal of 64 or more). */
HIST_API hist_status hist_fill_static(hist_t *h, const void *const *coords, const void *weights,
                                      int64_t n, hist_dtype dtype, void *stream);

/* Size in bytes of hist_fill_static's per-GPU scratch region. */
HIST_API int64_t hist_static_scratch_bytes(void);

/* Sizes the handle's scratch for fills of 1..n_max events of `dtype`, with
 * weights (weighted != 0) or without, under the plan choice in force (forced
 * strategy, tuned plan or heuristic): afterwards such fills allocate nothing.
 * A later hist_set_strategy, hist_set_window, hist_set_threads or hist_tune
 * may select plans that need more.  Allocates, synchronizes `stream`;
 * HIST_ECAPTURE while capturing.  Errors: HIST_EINVAL (n_max < 0),
 * HIST_ENOMEM. */
HIST_API hist_status hist_reserve(hist_t *h, int64_t n_max, hist_dtype dtype, int weighted,
                                  void *stream);

/* Find-bin only (Sec. 3.1 step 1 plus the global-bin linearization): writes
 * the global bin of each event to bins_dev (DEVICE, n int32).  Same search
 * and arithmetic as hist_fill.  Asynchronous; allocates nothing. */
HIST_API hist_status hist_findbin(hist_t *h, const void *const *coords, int64_t n, hist_dtype dtype,
                         int32_t *bins_dev, void *stream);

/* ---- events in host memory -------------------------------------------------- */

/* hist_fill_host flag: the coordinate and weight arrays are page-locked
 * (hipHostMalloc) and are copied to the device directly. */
#define HIST_HOST_PINNED  (1u << 0)

/* Fill n events whose columns are in HOST memory, as the paper's histogram
 * does for every bulk (Sec. 3.2: copy the bulk to the device, then fill), but
 * pipelined (the overlap Sec. 6 leaves as future work): the events go through
 * the device in chunks of `chunk` events (0 = 4,194,304) over two slots, so
 * the host->device copy of one chunk runs on a copy stream of the handle while
 * the fill of the previous one runs on `stream`.  Pageable input is first
 * copied by host threads into page-locked staging buffers of the handle;
 * with HIST_HOST_PINNED the copy engine reads the caller's arrays directly.
 * A staging buffer or device slot is reused only after the copy or fill that
 * last used it has run, so a refill never races a copy still reading it (the
 * host-buffer race of Sec. 3.3).
 * coords: HOST array of dims HOST pointers to n contiguous values of `dtype`;
 * weights: HOST pointer or NULL (unit weights).  Same result as hist_fill of
 * the same events (entries grow by n).
 * Returns once the caller's arrays have been read completely (they may then
 * be reused or freed); the fills may still be running on `stream`.
 * Allocates the slots on first use or growth (page-locked host and device
 * memory, kept by the handle) and the fill scratch of a chunk; waits on host
 * for copies of earlier chunks.  HIST_ECAPTURE while `stream` is capturing.
 * Errors: HIST_EINVAL (n < 0, chunk < 0, NULL pointers, unknown flags),
 * HIST_ENOMEM, HIST_EDEVICE. */
HIST_API hist_status hist_fill_host(hist_t *h, const void *const *coords, const void *weights,
                                    int64_t n, hist_dtype dtype, int64_t chunk, uint32_t flags,
                                    void *stream);

/* ---- reading (the only synchronizing calls) -------------------------------- */

/* Statistics (layout above) into HOST out[cap]; *count = S.  cap < S:
 * nothing is written, *count = S, HIST_EINVAL.  Synchronizes `stream`;
 * HIST_ECAPTURE while the stream is capturing. */
HIST_API hist_status hist_stats(hist_t *h, double *out, int cap, int *count, void *stream);

/* Bin sums of weights and of squared weights (HOST, T doubles each, either may
 * be NULL) and the entry count (HOST, may be NULL; the device counter of every
 * fill that has run).  Synchronizes `stream`; HIST_ECAPTURE while capturing. */
HIST_API hist_status hist_read(hist_t *h, double *sumw, double *sumw2, int64_t *entries, void *stream);

/* Zero bins, statistics and entries.  Asynchronous (fill kernels, no memset). */
HIST_API hist_status hist_reset(hist_t *h, void *stream);

/* ---- learned find-bin index --------------------------------------------- */

/* Trains the learned index of variable axis `axis` on the GPU: pairs
 * (x, bin) made from the edge array by the find-bin rule (each edge e_i and
 * each bin midpoint), a per-segment quadratic least-squares model of the bin
 * position over an order-preserving feature of x, and per-segment error
 * bounds measured at every edge.  The bounds make the bounded search exact:
 * after training, hist_fill and hist_findbin on this axis give the same bins
 * as binary search, bit for bit.  Switches the axis to HIST_SEARCH_LEARNED.
 * Synchronizes `stream`.  Errors: HIST_EINVAL (axis not variable). */
HIST_API hist_status hist_train_index(hist_t *h, int axis, void *stream);

/* Selects the search of a variable axis (HIST_SEARCH_LEARNED needs a trained
 * index, else HIST_EINVAL). */
HIST_API hist_status hist_set_search(hist_t *h, int axis, hist_search mode);

/* Describes a trained index: segments, feature kind (0 key bits, 1 linear),
 * mean and max candidate-window width over segments (bins). */
HIST_API hist_status hist_index_info(hist_t *h, int axis, int *segments, int *feature,
                            double *mean_window, double *max_window);

/* ---- plans and autotuning ------------------------------------------------- */

/* Forces a plan for later fills: strategy (hist_strategy), blocks (0 = auto),
 * subhists = LDS copies per block for small histograms (0 = auto).  Used by
 * tests to show every strategy gives the same result. */
HIST_API hist_status hist_set_strategy(hist_t *h, int strategy, int blocks, int subhists);

/* Autotuner: times the candidate plans on the given sample with HIP events on
 * `stream` (strategy, threads per workgroup, workgroups per CU, merge), then
 * refines the chosen one a knob at a time (interleaved LDS copies 1..64 of a
 * whole-histogram window, events per thread 1, 2, 4, 8 where a shape variant
 * exists), keeps the fastest for this histogram shape and remembers it in a
 * process-wide cache keyed by the shape; hist_batch_create applies it to
 * members of that shape.  It also picks the LDS window of bins with the
 * largest sample mass.  The histogram contents are restored to what they
 * were before the call.  Synchronizes; HIST_ECAPTURE while capturing. */
HIST_API hist_status hist_tune(hist_t *h, const void *const *coords, const void *weights, int64_t n,
                      hist_dtype dtype, void *stream);

/* Plan the next fill of n events would use: strategy, blocks, LDS copies,
 * window start and size (bins), accumulator (0 u32, 1 u16, 2 f64, 3 f32c). */
HIST_API hist_status hist_plan_info(hist_t *h, int64_t n, hist_dtype dtype, int weighted,
                           int *strategy, int *blocks, int *subhists, int64_t *window_lo,
                           int64_t *window_len, int *accumulator);

/* Fixes, for later fills, the first bin of the LDS window (-1 = the
 * autotuner's or heuristic choice) and the merge of LDS windows (-1 auto,
 * 0 coalesced global atomics, 1 staging buffer plus reduction kernel).  Used
 * by tests and benchmarks to pin a plan. */
HIST_API hist_status hist_set_window(hist_t *h, int64_t window_lo, int merge);

/* Fixes the threads per workgroup of later fills (0 = heuristic; 256, 512 or
 * 1024), also over a plan hist_tune chose.  Used by tests and benchmarks to
 * pin a plan. */
HIST_API hist_status hist_set_threads(hist_t *h, int threads);

/* Launch shape of later fills (the paper's tuning study, Sec. 4.3, varies the
 * elements each work-item reduces and fuses the statistics reductions):
 * unroll = events per thread and loop iteration of the fill kernel (0 =
 * heuristic, or 1, 2, 4, 8); stats_ept = 0 keeps the statistics fused into
 * the fill pass, 1, 4 or 16 computes them instead with one reduction kernel
 * per statistic that re-reads the columns, with that many events per thread.
 * Variants exist for one binary64 axis (fixed-width or learned index with
 * unit weights, edges staged in LDS, fixed-width with weights) under the LDS
 * and global strategies; other fills keep their heuristic shape.  Results
 * are the same within the tolerance of the summation order. */
HIST_API hist_status hist_set_shape(hist_t *h, int unroll, int stats_ept);

/* Shape the next fill of n events would use: events per thread, statistics
 * kernels' events per thread (0 = fused), threads per workgroup. */
HIST_API hist_status hist_plan_shape(hist_t *h, int64_t n, hist_dtype dtype, int weighted,
                                     int *unroll, int *stats_ept, int *threads);

/* Kernel timing for benchmarks: while enabled, hist_fill records HIP events on
 * its stream around the fill kernel and around the merge-reduction kernel.
 * Enabling (or disabling) clears what was recorded. */
HIST_API hist_status hist_timing(hist_t *h, int enable);

/* Sums of the recorded fill-kernel and merge-kernel durations (ms) and the
 * number of fill launches since the last read or hist_timing call; clears
 * them.  Waits for the recorded events. */
HIST_API hist_status hist_timing_read(hist_t *h, double *fill_ms, double *merge_ms,
                                      int64_t *launches);

/* ---- batched filling ------------------------------------------------------- */

/* One member of a batch: coordinates/weights as for hist_fill. */
typedef struct {
    const void *coords[3];   /* DEVICE pointers, first dims used */
    const void *weights;     /* DEVICE pointer or NULL */
    int64_t n;
    hist_dtype dtype;
} hist_fill_desc;

/* Builds a batch over k handles (distinct, all on this device): a tile list
 * over every member's events and a per-member plan, uploaded once, and a HIP
 * graph that holds one persistent fill launch for all members (plus the
 * partition passes of members far larger than LDS; members of more than 2^25
 * events use global atomics instead).  The batched fill of many histograms
 * in one launch is the paper's future work (Sec. 6); it is split into this
 * set-up call and hist_batch_launch so that the set-up (tile lists, plans,
 * scratch, graph instantiation) is paid once and every launch is one graph
 * replay.  The inputs named in descs are bound into the graph: every
 * hist_batch_launch reads the same device buffers, and they must stay
 * allocated while the batch lives; the k handles are held by the batch
 * (hist_destroy refuses them until hist_batch_destroy).  Allocates and
 * synchronizes.  Errors: HIST_EINVAL, HIST_ENOMEM, HIST_ECAPTURE. */
HIST_API hist_status hist_batch_create(int k, hist_t *const *hs, const hist_fill_desc *descs,
                              hist_batch_t **out, void *stream);

/* Replays the batch graph on `stream`: fills every member once (adding to its
 * sums and entry count, Sec. 3.3).  Asynchronous; allocates nothing. */
HIST_API hist_status hist_batch_launch(hist_batch_t *b, void *stream);

/* Same work as one replay, launched directly without the graph. */
HIST_API hist_status hist_batch_launch_eager(hist_batch_t *b, void *stream);

/* Frees the batch and releases its handles (synchronizes the device).  NULL
 * is accepted. */
HIST_API hist_status hist_batch_destroy(hist_batch_t *b);

/* ---- event filters, computed columns, several histograms per pass ----------- */

/* Operations of the postfix programs of hist_define.  Values are binary64
 * (FP32 columns are widened exactly); every operation is exactly rounded
 * (IEEE 754), no contraction into fused multiply-adds, so results are
 * bit-reproducible.  Comparisons and logic give 1.0 or 0.0; a value is true
 * when it is nonzero (NaN is true).
 *   COL c: push column c          CONST v: push v
 *   NEG ABS SQRT NOT: replace the top value a by -a, |a|, sqrt(a), (a == 0)
 *   ADD SUB MUL DIV: a op b of the two top values (b on top)
 *   MIN: (b < a ? b : a)    MAX: (a < b ? b : a)
 *   LT LE GT GE EQ NE: a op b       AND OR: logical of (a != 0), (b != 0)
 *   SELECT: c a b -> (c != 0 ? a : b) */
typedef enum {
    HIST_OP_COL = 0, HIST_OP_CONST = 1, HIST_OP_ADD = 2, HIST_OP_SUB = 3, HIST_OP_MUL = 4,
    HIST_OP_DIV = 5, HIST_OP_NEG = 6, HIST_OP_ABS = 7, HIST_OP_SQRT = 8, HIST_OP_MIN = 9,
    HIST_OP_MAX = 10, HIST_OP_LT = 11, HIST_OP_LE = 12, HIST_OP_GT = 13, HIST_OP_GE = 14,
    HIST_OP_EQ = 15, HIST_OP_NE = 16, HIST_OP_AND = 17, HIST_OP_OR = 18, HIST_OP_NOT = 19,
    HIST_OP_SELECT = 20
} hist_opcode;

typedef struct {
    int32_t op;      /* hist_opcode */
    int32_t col;     /* HIST_OP_COL: column index */
    double value;    /* HIST_OP_CONST */
} hist_op;

/* A postfix program of 1..32 operations leaving one value, stack depth at
 * most 6; nops == 0 means absent. */
typedef struct {
    const hist_op *ops;
    int32_t nops;
} hist_expr;

/* What one histogram takes from the shared columns: the Filter and Define
 * steps in front of a histogram fill in the paper's RDataFrame usage (Sec. 3,
 * Listing 1; its CUDA kernel skips events marked invalid, Sec. 3.2).
 *   filter:   the event is filled only where the program is nonzero; a
 *             filtered-out event changes nothing (no bin, statistics or
 *             entry).  Absent: every event.
 *   coord[a]: the coordinate on axis a.  Absent: column a.
 *   weight:   the event weight.  Absent: unit weight. */
typedef struct {
    hist_expr filter;
    hist_expr coord[3];
    hist_expr weight;
} hist_define;

/* Prepares one pass that fills k (1..16) distinct histograms (all on this
 * device) from ncols (1..8) shared columns of `dtype`: the paper's future
 * work of several histograms per event loop (Sec. 6).  defs[k] (NULL: every
 * member takes columns 0..dims-1 as coordinates, unit weights, no filter).
 * Programs are checked here (operations, column indices, stack depth).  The
 * plan keeps each member's statistics, learned models and edge arrays of at
 * most 4,096 edges in LDS, then whole-histogram copies of the smallest members
 * while LDS lasts; other members take global atomics.  The handles are held
 * by the plan (hist_destroy refuses them until hist_multi_destroy); they may
 * still be filled on their own.  Allocates and copies the
 * plan to the device (synchronous).  Errors: HIST_EINVAL, HIST_ENOMEM,
 * HIST_EDEVICE. */
HIST_API hist_status hist_multi_create(int k, hist_t *const *hs, const hist_define *defs, int ncols,
                                       hist_dtype dtype, hist_multi_t **out);

/* One pass over n events: columns is a HOST array of ncols DEVICE pointers
 * to n contiguous values each.  Every member adds the events its filter keeps
 * (bins, statistics, entries), as hist_fill of its defined coordinates and
 * weights would.  Asynchronous on `stream`; allocates nothing (capture-safe).
 * Weights accumulate in binary64 (also for handles made with HIST_F_ACC_F32C).
 * Errors: HIST_EINVAL (NULL plan or column, n < 0), HIST_EDEVICE. */
HIST_API hist_status hist_multi_fill(hist_multi_t *m, const void *const *columns, int64_t n,
                                     void *stream);

/* Where member `member` accumulates: in_lds = 1 for an LDS copy (with
 * `copies` interleaved copies), 0 for global atomics; lds_bytes = dynamic LDS
 * of the pass. */
HIST_API hist_status hist_multi_info(const hist_multi_t *m, int member, int *in_lds, int *copies,
                                     int *lds_bytes);

/* Frees the plan (synchronizes the device).  NULL is accepted. */
HIST_API hist_status hist_multi_destroy(hist_multi_t *m);

/* ---- measurement probes ------------------------------------------------------ */

/* What hist_probe measures (the ceilings of the fill's roofline):
 *   HIST_PROBE_READ        streaming read of `bytes` of `buf` (16-byte
 *                          non-temporal loads): bytes/s
 *   HIST_PROBE_LDS_U32     32-bit LDS atomic adds, one 1024-thread workgroup
 *                          per CU, hashed addresses in 64 KB: lane operations/s
 *   HIST_PROBE_LDS_F64     the same with binary64 LDS atomic adds
 *   HIST_PROBE_GLOBAL_U64  device-scope 64-bit atomic adds without return to
 *                          hashed addresses of `buf` (overwritten): operations/s
 *   HIST_PROBE_GLOBAL_F64  the same with binary64 atomic adds */
#define HIST_PROBE_READ       0
#define HIST_PROBE_LDS_U32    1
#define HIST_PROBE_LDS_F64    2
#define HIST_PROBE_GLOBAL_U64 3
#define HIST_PROBE_GLOBAL_F64 4

/* Runs probe `kind` once to warm up, then `reps` times between HIP events on
 * `stream`; *rate = work per second, *ms = mean milliseconds per run (may be
 * NULL).  buf: DEVICE buffer of `bytes` (>= 4096) for the read and global
 * probes, ignored by the LDS probes.  Synchronizes.  Errors: HIST_EINVAL,
 * HIST_EDEVICE. */
HIST_API hist_status hist_probe(int kind, const void *buf, int64_t bytes, int reps, void *stream,
                                double *rate, double *ms);

/* ---- introspection -------------------------------------------------------- */

HIST_API int64_t hist_nbins_total(const hist_t *h);   /* T, or -1 for NULL */
HIST_API int hist_nstats(const hist_t *h);             /* S, or -1 for NULL */
HIST_API const char *hist_strerror(hist_status s);
HIST_API const char *hist_last_error(void);          /* thread-local, never NULL */
HIST_API const char *hist_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HIST_H */
