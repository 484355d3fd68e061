/*
 * lms.h -- C ABI of the MI355X (gfx950) micro-batch stream operator library.
 *
 * LMStream (Lee & Park, arXiv 2111.04289) runs a streaming query as a chain of
 * operations over each admitted micro-batch (Sec. III-A, Fig. 3; problem
 * statement Sec. III-B, Eq. 1-5).  The operations whose GPU functions this
 * library provides are the rows of Table II that touch the data of a single
 * micro-batch: Filtering, Projection, Aggregation (Hash) over tumbling or
 * sliding event-time windows (window slide semantics of Table I, SlideTime,
 * with 0 meaning a tumbling window; Expand is realised by pane
 * decomposition) and Join (Hash) of the stream against a static table.
 * lms_plan implements the MapDevice placement (Algorithm 2) with the device
 * cost model of Eq. 7-9.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Column data pointers in lms_col are DEVICE pointers (hipMalloc'd or
 *    torch CUDA tensors); every other pointer argument is a HOST pointer unless
 *    its name starts with d_.  All buffers are owned by the caller; the library
 *    keeps no pointer after a call returns, except the opaque lms_join_table,
 *    which it owns until lms_join_free.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are stream-ordered and asynchronous: they validate arguments on the
 *    host, enqueue kernels and return.  Results and device counts are valid
 *    once the caller has synchronised the stream.
 *  - Return value: LMS_OK (0) or a negative LMS_E* code for errors detected on
 *    the host (nothing is enqueued then).  lms_last_error() gives a
 *    thread-local message for the last failing call on this thread.
 *  - d_count arguments point to a DEVICE array of 2 int64: [0] receives the
 *    number of result rows the operation produced (also when it exceeds the
 *    capacity: then only `cap` rows are written and the caller may retry with a
 *    larger capacity), [1] receives a device-detected status (0 or a negative
 *    LMS_E* code, e.g. LMS_ECAPACITY).  Results are valid only if [1] == 0.
 *  - Workspace: scratch device memory supplied by the caller, at least the
 *    size that the matching *_workspace() query returns.  The library performs
 *    no device allocation on the per-batch path.  Two calls that overlap in
 *    time must not share a workspace.
 *  - Re-entrancy: calls on different streams with different workspaces may
 *    run concurrently.
 */
#ifndef LMS_H
#define LMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LMS_ABI_VERSION 1

/* Status codes. */
#define LMS_OK 0
#define LMS_EINVAL -1    /* bad argument: null pointer, bad dtype/column index, slide > len, cap too small ... */
#define LMS_EHIP -2      /* a HIP runtime call or kernel launch failed */
#define LMS_ENOMEM -3    /* workspace too small or a library allocation failed */
#define LMS_ECAPACITY -4 /* device: a table is too small (e.g. one window of one key spans more panes than a workgroup table holds) */
#define LMS_ERANGE -5    /* device: an event time lies about 2^30 panes or more from the batch's first row */

typedef void* lms_stream; /* hipStream_t */

typedef enum { LMS_I32 = 0, LMS_I64 = 1, LMS_F32 = 2, LMS_F64 = 3 } lms_dtype;

/* Comparison of a predicate.  Integer columns compare as int64 against ival;
 * floating columns compare as double against fval with IEEE semantics (a NaN
 * row satisfies only LMS_NE). */
typedef enum { LMS_LT = 0, LMS_LE = 1, LMS_GT = 2, LMS_GE = 3, LMS_EQ = 4, LMS_NE = 5 } lms_cmp;

/* Aggregate functions of the hash aggregation (Table II "Aggregation (Hash)";
 * the query shapes of Table III use SUM and AVG).  COUNT counts the rows of the
 * group; SUM/MIN/MAX need an integer input and give int64 (SUM wraps modulo
 * 2^64); AVG accepts any numeric input and gives the double quotient of the
 * double sum by the count. */
typedef enum { LMS_COUNT = 0, LMS_SUM = 1, LMS_MIN = 2, LMS_MAX = 3, LMS_AVG = 4 } lms_aggfn;

/* One column: `data` is a device pointer to nrows values of `dtype`. */
typedef struct {
  void* data;
  int32_t dtype;
  int32_t reserved;
} lms_col;

/* A micro-batch, or one partition of it (Table I: Part_(i,j)), as columns of
 * equal length (structure of arrays). */
typedef struct {
  const lms_col* cols; /* host array of ncols column descriptors */
  int32_t ncols;
  int32_t reserved;
  int64_t nrows;
} lms_batch;

/* Predicate `cols[col] op constant`; a list of predicates is a conjunction. */
typedef struct {
  int32_t col;
  int32_t op; /* lms_cmp */
  int64_t ival;
  double fval;
} lms_pred;

/* Projection: a new integer column v = src * mul + add, evaluated in 64-bit
 * two's complement and truncated to the source column's width (int32 sources
 * wrap modulo 2^32).  Only integer sources are accepted. */
typedef struct {
  int32_t src;
  int32_t reserved;
  int64_t mul;
  int64_t add;
} lms_proj;

/* Event-time window (Table I SlideTime; CQL [range len slide slide] of
 * Table III).  Window starts are origin + k*slide for every integer k; a row
 * with event time ts belongs to each window with start <= ts < start + len.
 * slide == 0 means a tumbling window (slide = len).  Requires
 * 0 < slide <= len and both < 2^31.  Event times must lie within +-2^62. */
typedef struct {
  int32_t ts_col; /* integer column holding the event time */
  int32_t reserved;
  int64_t len;
  int64_t slide;
  int64_t origin;
} lms_window;

/* One aggregate: fn over column `col`, where col indexes the input columns
 * followed by the projected columns (ncols + j is projection j).  col is
 * ignored for LMS_COUNT. */
typedef struct {
  int32_t fn; /* lms_aggfn */
  int32_t col;
} lms_agg;

/* Output of lms_window_agg: one row per (key, window) holding >= 1 row that
 * passed the predicates.  Device columns of capacity `cap`: key (int64, the
 * key column's value widened), window start (int64), then aggs[a] is int64 for
 * COUNT/SUM/MIN/MAX and double for AVG.  Row order is unspecified. */
typedef struct {
  int64_t* key;
  int64_t* wstart;
  void* const* aggs; /* host array of nagg device pointers */
  int64_t cap;
} lms_groups;

/* Library and ABI information. */
int lms_abi_version(void);
const char* lms_last_error(void);

/* ---- Filtering + Projection (Table II rows "Filtering" and "Projection";
 * the select-project query of Sec. II-C / III-D) --------------------------
 * Keeps the rows of `in` for which every predicate holds, in input order, and
 * writes for each kept row the input columns listed in keep[0..nkeep) followed
 * by the projections projs[0..nproj).  out->ncols must equal nkeep + nproj,
 * out column j must have the dtype of its source and room for in->nrows rows
 * (the provable bound; no device-side capacity check is needed).
 * d_count[0] receives the number of kept rows.
 * Workspace: lms_filter_project_workspace(in->nrows) bytes. */
size_t lms_filter_project_workspace(int64_t nrows);
int lms_filter_project(const lms_batch* in, const lms_pred* preds, int32_t npred, const int32_t* keep,
                       int32_t nkeep, const lms_proj* projs, int32_t nproj, const lms_batch* out,
                       int64_t* d_count, void* workspace, size_t ws_bytes, lms_stream stream);

/* Allocation-free variant of lms_filter_project, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, semantics and results as
 * lms_filter_project, without the workspace: its per-tile counts live in a
 * fixed 1 MiB array in the library's device memory, one per GPU, held until
 * the process ends.  in->nrows must not exceed
 * lms_filter_project_noalloc_max_rows() (2^28), else LMS_EINVAL.  The first
 * call on a device looks up that device's copy of the array (a host-side
 * HIP query; it may fail with LMS_EHIP); no call allocates.  Every call on a
 * GPU shares that GPU's array, so calls that overlap in time on one GPU (on
 * different streams, or from different threads) race and give wrong results:
 * order them on one stream or by events. */
int64_t lms_filter_project_noalloc_max_rows(void);
int lms_filter_project_noalloc(const lms_batch* in, const lms_pred* preds, int32_t npred, const int32_t* keep,
                               int32_t nkeep, const lms_proj* projs, int32_t nproj, const lms_batch* out,
                               int64_t* d_count, lms_stream stream);

/* ---- Windowed hash group-by (Table II "Aggregation (Hash)" and "Expand";
 * windows per Table I SlideTime and the range/slide clauses of Table III) ---
 * Groups the rows that pass the predicates by (cols[key_col], window) and
 * computes aggs[0..nagg) per group.  The key column must be integer.  Output
 * rows go to `out` (see lms_groups); d_count[0] receives the number of groups,
 * of which min(count, out->cap) are written.  d_count[1] is LMS_ECAPACITY
 * only if the passing rows of one key fill more distinct panes (pane =
 * gcd(len, slide)) inside a single window than one workgroup table holds
 * (lms_window_agg_pane_limit; a key with more panes than that in all is
 * aggregated in several passes over ranges of its windows), LMS_ERANGE if an
 * event time is 2^30 - slide/pane panes or more before, or 2^30 panes or more
 * after, the first row's pane.
 * Workspace: lms_window_agg_workspace() with the same arguments.  After the
 * call completes the workspace still holds the rows it staged and their
 * partial aggregates; lms_window_agg_emit can then write the same groups
 * again. */
size_t lms_window_agg_workspace(const lms_batch* in, int32_t key_col, const lms_window* w, const lms_agg* aggs,
                                int32_t nagg);
/* Most non-empty panes one key may hold inside a single window for nagg
 * aggregates (the (key, pane) slots of one workgroup table). */
int64_t lms_window_agg_pane_limit(int32_t nagg);
int lms_window_agg(const lms_batch* in, const lms_pred* preds, int32_t npred, const lms_proj* projs, int32_t nproj,
                   int32_t key_col, const lms_window* w, const lms_agg* aggs, int32_t nagg, const lms_groups* out,
                   int64_t* d_count, void* workspace, size_t ws_bytes, lms_stream stream);

/* Re-emission (same operation: Table II "Aggregation (Hash)"): writes the
 * groups of the last lms_window_agg call that used `workspace` into `out`
 * again, from the staged rows and partial aggregates that call left in the
 * workspace -- the input columns are not read (they may already be freed).
 * This is how a caller whose first output capacity was below d_count[0]
 * obtains every group without re-running the scan: allocate d_count[0] rows
 * and emit again.  `out` must hold nagg aggregate columns of the original
 * call's types, in its order; d_count as for lms_window_agg ([1] carries the
 * original call's device status).  The workspace must be untouched since
 * that call, and neither that call nor another use of the workspace may still
 * run (stream order or events).  Returns LMS_EINVAL for bad arguments; a
 * workspace that no call filled, another nagg or a moved workspace set
 * d_count[1] = LMS_EINVAL on the device.  Asynchronous and stream-ordered;
 * performs no allocation.  Row order is unspecified and may differ from the
 * first emission. */
int lms_window_agg_emit(const lms_groups* out, int32_t nagg, int64_t* d_count, void* workspace, size_t ws_bytes,
                        lms_stream stream);

/* ---- Table III query shapes: composite keys, HAVING, ORDER BY ------------------
 * The windowed group-by of lms_window_agg with
 *  - a composite group key: the tuple of nkey integer columns (LR2S groups by
 *    highway, direction and segment).  For nkey > 1 each part declares the
 *    value domain [lo, hi] of its column (a schema property: every passing
 *    row's value must lie in it, else d_count[1] = LMS_ERANGE); the domains'
 *    product must not exceed 2^62 tuples.  For nkey == 1, lo and hi are
 *    ignored;
 *  - HAVING (optional): only groups with aggs[having->agg] op value are kept
 *    (ival for integer aggregates, fval for AVG; LR2S keeps avgSpeed < 40);
 *  - ORDER BY (optional; Table II "Sorting", CM1 orders by SUM(cpu)): rows
 *    ordered by window start, then by aggs[order->agg] (descending if asked),
 *    then by the key tuple; without it, row order is unspecified.
 * Output: out->keys[j] (int64, the key part widened), out->wstart, out->aggs
 * as in lms_groups, capacity out->cap.  out->cap must hold every (key tuple,
 * window) group before HAVING: else d_count[1] = LMS_ECAPACITY and nothing
 * is valid.  d_count[0] = rows written (after HAVING).
 * Workspace: lms_window_query_workspace() with the same key parts, window,
 * aggregates, whether ORDER BY is given, and the capacity. */
typedef struct {
  int32_t col;
  int32_t reserved;
  int64_t lo, hi; /* value domain of the key column (nkey > 1) */
} lms_keypart;
typedef struct {
  int32_t agg; /* index into aggs */
  int32_t op;  /* lms_cmp */
  int64_t ival;
  double fval;
} lms_having;
typedef struct {
  int32_t agg;
  int32_t descending;
} lms_order;
typedef struct {
  int64_t* const* keys; /* host array of nkey device columns */
  int64_t* wstart;
  void* const* aggs;
  int64_t cap;
} lms_qgroups;
size_t lms_window_query_workspace(const lms_batch* in, const lms_keypart* keys, int32_t nkey, const lms_window* w,
                                  const lms_agg* aggs, int32_t nagg, int32_t ordered, int64_t cap);
int lms_window_query(const lms_batch* in, const lms_pred* preds, int32_t npred, const lms_proj* projs, int32_t nproj,
                     const lms_keypart* keys, int32_t nkey, const lms_window* w, const lms_agg* aggs, int32_t nagg,
                     const lms_having* having, const lms_order* order, const lms_qgroups* out, int64_t* d_count,
                     void* workspace, size_t ws_bytes, lms_stream stream);

/* ---- Windowed self-join (Table III LR1: the stream joined with the rows of
 * its own range/slide window on equal keys, A.vehicle == L.vehicle) ---------
 * For every window and every ordered pair (l, a) of rows that both pass the
 * predicates, both lie in the window and have equal keys (l == a included),
 * one output (window start, l, a), l and a being row indices of `in`.  Rows
 * are written in unspecified order; d_count[0] = the number of pairs, of
 * which min(count, cap) are written (re-run with a larger cap to get all).
 * d_count[1] = LMS_ERANGE if event times span 2^30 panes or more.
 * Workspace: lms_window_self_join_workspace(in->nrows). */
size_t lms_window_self_join_workspace(int64_t nrows);
int lms_window_self_join(const lms_batch* in, const lms_pred* preds, int32_t npred, int32_t key_col,
                         const lms_window* w, int64_t* out_wstart, uint32_t* out_l, uint32_t* out_a, int64_t cap,
                         int64_t* d_count, void* workspace, size_t ws_bytes, lms_stream stream);

/* ---- Many micro-batches per launch -------------------------------------------
 * The same windowed group-by over nbatch micro-batches of one schema, with
 * every stage run as one persistent launch over all batches (a fixed grid
 * whose workgroups loop over (batch, chunk), (batch, partition) and
 * (batch, item) work).  lms_window_agg_multi_prepare validates the batches and
 * writes per-batch descriptors into the workspace (an upload ordered on
 * `stream` from the library's pinned staging; the caller's host arrays may be
 * reused as soon as it returns; not capturable) and fills *cfg;
 * lms_window_agg_multi_launch enqueues the seven launches, which read
 * everything from the workspace, so a graph captured around it can be
 * replayed after another prepare into the same workspace (new batches, sizes
 * or outputs).  The kernels compare the prepared job with the limits the
 * launch was configured for (LDS of cfg->max_nparts partitions and
 * cfg->agg_lds bytes, cfg->ma aggregates); a job beyond them does nothing but
 * set status LMS_EINVAL in every d_counts pair.  outs[b] and
 * d_counts[2b..2b+1] receive batch b's result exactly as lms_window_agg would
 * (same groups and values; the order of rows may differ).  The workspace
 * must stay untouched until the launch completes. */
typedef struct {
  int32_t nbatch;
  int32_t ma;         /* aggregate unroll bound of the kernels (2, 4, 6 or 8) */
  int32_t max_nparts; /* largest partition count of a batch */
  int32_t grid_scan;  /* persistent workgroups of the scan stages */
  int32_t grid_agg;   /* persistent workgroups of the aggregation stages */
  int32_t reserved;
  uint64_t agg_lds; /* dynamic LDS bytes of an aggregation workgroup */
} lms_multi_config;
size_t lms_window_agg_multi_workspace(const lms_batch* batches, int32_t nbatch, int32_t key_col, const lms_window* w,
                                      const lms_agg* aggs, int32_t nagg);
int lms_window_agg_multi_prepare(const lms_batch* batches, int32_t nbatch, const lms_pred* preds, int32_t npred,
                                 const lms_proj* projs, int32_t nproj, int32_t key_col, const lms_window* w,
                                 const lms_agg* aggs, int32_t nagg, const lms_groups* outs, int64_t* d_counts,
                                 void* workspace, size_t ws_bytes, lms_multi_config* cfg, lms_stream stream);
int lms_window_agg_multi_launch(const lms_multi_config* cfg, void* workspace, lms_stream stream);

/* Tile and schedule parameters of the windowed group-by (process-wide; NULL
 * or 0 fields select the defaults): rows per scan chunk (rounded up to a
 * power of two, at most 65536), target rows per
 * partition, rows per aggregation piece (>= 1024), persistent scan workgroups
 * per CU, and (key, pane) slots of an aggregation workgroup's LDS table (1024
 * or 2048, the default; the smaller table fits two workgroups' LDS in a CU
 * and lowers the panes one key may hold, lms_window_agg_pane_limit).  Unset partition and piece sizes default to 8
 * and 4 rows per table slot, except that a batch of fewer than 8 x 32 rows per
 * slot targets 1/32 of its rows per partition (at least 2048), so that it
 * spreads over 32 partitions.  Chosen by the project's autotuner; results never
 * depend on them. */
typedef struct {
  int32_t chunk_rows;
  int32_t part_rows;
  int32_t piece_rows;
  int32_t grid_per_cu;
  int32_t lds_groups;
  int32_t reserved;
} lms_tuning;
int lms_set_tuning(const lms_tuning* t);
int lms_get_tuning(lms_tuning* t);

/* ---- Window state across micro-batches ----------------------------------------
 * The windowed group-by of a stream that arrives as a sequence of
 * micro-batches (Sec. II-A window semantics, Sec. III: every micro-batch is a
 * query execution over the newly admitted datasets): partial aggregates of
 * windows still open are kept on the device between micro-batches, per
 * (key, pane) with pane = gcd(len, slide), and each window is emitted once,
 * after the watermark passes its end.  The handle owns one device allocation
 * of lms_wstate_bytes(max_keys, ring_panes, nagg) bytes (what a caller
 * admitting work by free HBM reserves).
 *
 * lms_wstate_create: window (ts_col must be an int64 input column at update
 *   time), aggregates as in lms_window_agg (SUM/MIN/MAX over integer columns,
 *   AVG over any; columns index the update's inputs followed by its
 *   projections), max_keys distinct keys over the stream's life (the key
 *   dictionary never shrinks), ring_panes >= the panes between the oldest
 *   window not yet emitted and the newest row (rounded up to a power of two,
 *   at least len/pane + slide/pane).  Initialisation is enqueued on `stream`.
 * lms_wstate_update: adds the passing rows of a micro-batch.  Rows whose pane
 *   lies only in already-emitted windows are late: dropped and counted.  Rows
 *   that find the dictionary full or their pane's ring entry held by another
 *   live pane are dropped and counted, and set status LMS_ECAPACITY.
 * lms_wstate_emit: writes every window not yet emitted whose end
 *   (start + len) is <= watermark -- or, with flush != 0, every remaining
 *   window holding data -- at most max_windows window starts per call, in
 *   order; then clears the panes no later window needs.  Output as
 *   lms_window_agg: d_count[0] = groups (written up to out->cap; more sets
 *   d_count[1] = LMS_ECAPACITY).  Repeated flush calls drain the rest.
 * lms_wstate_info: copies 8 int64 control words to device memory d_info:
 *   late rows, capacity drops, min pane, max pane, next window index, last
 *   emitted window range [lo, hi], status.
 * Calls on one state must be ordered (one stream, or events); different
 * states are independent. */
typedef struct lms_wstate lms_wstate;
size_t lms_wstate_bytes(int64_t max_keys, int32_t ring_panes, int32_t nagg);
int lms_wstate_create(const lms_window* w, const lms_agg* aggs, int32_t nagg, int64_t max_keys, int32_t ring_panes,
                      lms_wstate** out, lms_stream stream);
int lms_wstate_update(lms_wstate* st, const lms_batch* in, const lms_pred* preds, int32_t npred,
                      const lms_proj* projs, int32_t nproj, int32_t key_col, lms_stream stream);
int lms_wstate_emit(lms_wstate* st, int64_t watermark, int32_t flush, int32_t max_windows, const lms_groups* out,
                    int64_t* d_count, lms_stream stream);
int lms_wstate_info(lms_wstate* st, int64_t* d_info, lms_stream stream);
void lms_wstate_free(lms_wstate* st);

/* ---- Micro-batch admission (ConstructMicroBatch) ---------------------------------
 * Host-only controller of Algorithm 1: datasets arriving from the stream are
 * buffered until the estimated maximum latency of the micro-batch they would
 * form (Eq. 6: oldest buffering time + rows / AvgThPut of Eq. 4) plus one poll
 * period reaches the deadline: SlideTime for sliding windows (Eq. 2), the
 * mean MaxLat (Eq. 5) of the completed batches for tumbling ones (Eq. 3), or
 * an explicit deadline.  The caller polls every poll_ms with the datasets that
 * arrived since its last call and reports each finished batch with
 * lms_admit_done.  Times are in ms on any one clock. */
typedef struct {
  double slide_ms;     /* SlideTime; 0 for a tumbling window */
  double deadline_ms;  /* > 0: explicit latency bound, replacing the window rule */
  double poll_ms;      /* polling period (10 ms in the paper) */
  int32_t poll_idle;   /* 1: also test on polls without new data; 0: only when data arrived */
  int32_t reserved;
} lms_admit_params;
typedef struct {
  int32_t admit;             /* 1: the buffered datasets form the next micro-batch */
  int32_t reserved;
  int64_t datasets, rows;    /* size of the admitted micro-batch (0 if not admitted) */
  double oldest_arrival_ms;  /* creation time of its oldest dataset */
  double est_maxlat_ms;      /* EstMaxLat of the buffered datasets at this poll */
  int64_t buffered_datasets, buffered_rows; /* buffer before the decision */
} lms_admit_decision;
typedef struct {
  int64_t batches_done, admitted, rows_done, buffered_rows;
  double avg_thput_rows_per_ms, mean_maxlat_ms;
} lms_admit_stats;
typedef struct lms_admit lms_admit;
typedef struct lms_mlp_model lms_mlp_model;
typedef struct lms_op_desc lms_op_desc;
typedef struct lms_batch_stats lms_batch_stats;
int lms_admit_create(const lms_admit_params* p, lms_admit** out);
/* arrival_ms/rows: host arrays of the n_new datasets that arrived since the
 * last poll (any order).  On admission the buffer is handed over whole, in
 * creation order, and emptied. */
int lms_admit_poll(lms_admit* a, double now_ms, int64_t n_new, const double* arrival_ms, const int64_t* rows,
                   lms_admit_decision* out);
int lms_admit_done(lms_admit* a, int64_t rows, double proc_ms, double maxlat_ms);
/* Learned micro-batch sizing (Algorithm 1 with a learned Eq. 6 processing
 * term).  After this call the processing term of `rows` buffered rows is the
 * predicted time of the query's operation chain ops[0..nops) on a micro-batch
 * of that many rows -- each operation on the device lms_plan picks in
 * LMS_PLAN_LEARNED mode, with per_batch's statistics and rows and
 * batch_bytes = bytes_per_row * rows (distinct_keys capped at rows) -- times
 * the ratio of measured to predicted processing time over the batches
 * reported since (1 before the first).  model, ops and per_batch are copied.
 * model == NULL returns to Eq. 4's AvgThPut.  Host-only. */
int lms_admit_set_model(lms_admit* a, const lms_mlp_model* model, const lms_op_desc* ops, int32_t nops,
                        const lms_batch_stats* per_batch, double bytes_per_row);
/* The processing term (ms) the controller would use for `rows` buffered rows
 * now (0 while it is unknown: analytic sizing before the first completed
 * batch); -1 for bad arguments. */
double lms_admit_predict_ms(const lms_admit* a, int64_t rows);
int lms_admit_get_stats(const lms_admit* a, lms_admit_stats* out);
void lms_admit_free(lms_admit* a);

/* ---- Stream-static hash join (Table II "Join (Hash)"; the join of LR1 in
 * Table III) ---------------------------------------------------------------
 * lms_join_build hashes the static table `tbl` on integer column key_col and
 * keeps the int32 column payload_col; it allocates the table (device memory
 * owned by the library) and enqueues the build on `stream`.
 * lms_hash_join emits, for every probe row i and every build row j with equal
 * key, the pair (i, payload_j): out_probe_idx[r] = i, out_payload[r] =
 * payload_j, grouped by ascending i (pairs of one probe row in unspecified
 * order).  probe->nrows must be < 2^32.  d_count[0] receives the number of
 * pairs, of which min(count, cap) are written.  cap >= probe->nrows *
 * lms_join_max_mult(t) is always enough.
 * lms_join_max_mult returns the largest number of build rows sharing one key
 * (it synchronises the build stream).  Workspace:
 * lms_hash_join_workspace(probe->nrows). */
typedef struct lms_join_table lms_join_table;
int lms_join_build(const lms_batch* tbl, int32_t key_col, int32_t payload_col, lms_join_table** out,
                   lms_stream stream);
int64_t lms_join_max_mult(lms_join_table* t);
int64_t lms_join_build_rows(const lms_join_table* t);
void lms_join_free(lms_join_table* t);
size_t lms_hash_join_workspace(int64_t nprobe);
int lms_hash_join(const lms_join_table* t, const lms_batch* probe, int32_t key_col, uint32_t* out_probe_idx,
                  int32_t* out_payload, int64_t cap, int64_t* d_count, void* workspace, size_t ws_bytes,
                  lms_stream stream);

/* ---- CPU execution functions ---------------------------------------------
 * The CPU side of MapDevice (Algorithm 2): the same operations on HOST
 * columns (lms_col.data and every output pointer are host pointers), run
 * synchronously on `nthreads` cores, the way an executor splits a micro-batch
 * into NumCores partitions (Table I).  Semantics, dtypes and error codes are
 * those of the GPU entry points above; `count` is a host int64 receiving the
 * number of result rows (of which min(count, capacity) are written).  Window
 * output rows come grouped by key partition, join pairs in probe order. */
int lms_cpu_filter_project(const lms_batch* in, const lms_pred* preds, int32_t npred, const int32_t* keep,
                           int32_t nkeep, const lms_proj* projs, int32_t nproj, const lms_batch* out, int64_t* count,
                           int32_t nthreads);
int lms_cpu_window_agg(const lms_batch* in, const lms_pred* preds, int32_t npred, const lms_proj* projs, int32_t nproj,
                       int32_t key_col, const lms_window* w, const lms_agg* aggs, int32_t nagg, const lms_groups* out,
                       int64_t* count, int32_t nthreads);
int lms_cpu_hash_join(const lms_batch* tbl, int32_t key_col, int32_t payload_col, const lms_batch* probe,
                      int32_t probe_key_col, uint32_t* out_probe_idx, int32_t* out_payload, int64_t cap,
                      int64_t* count, int32_t nthreads);

/* ---- Kernel tracing ---------------------------------------------------------
 * Per-launch timing for profiling and for the timing records of the placement
 * model.  While enabled, every kernel the library launches is bracketed by a
 * pair of hipEvents recorded on its stream.  lms_trace_read waits for the
 * recorded events, aggregates them per kernel name into out[0..max_out) and
 * clears the record; it returns the number of distinct kernels (or a negative
 * LMS_E* code).  Tracing is process-wide. */
typedef struct {
  char name[48];
  int64_t launches;
  double total_ms;
  double min_ms;
  double max_ms;
} lms_trace_stat;
int lms_trace_enable(int32_t on);
int lms_trace_read(lms_trace_stat* out, int32_t max_out);

/* ---- Device placement (MapDevice, Algorithm 2; cost model Eq. 7-9) -------
 * Host-only and synchronous.  ops[0..nops) is the operation chain in
 * execution order (the traversal of the operation DAG, leaf first).  For each
 * operation o with x = Part / InfPT, Part = batch_bytes / num_cores (Sec.
 * III-D: the per-core partition size):
 *   CPU_o = base_o * x (Eq. 7), GPU_o = base_o / x (Eq. 8),
 *   Trans_o = base_trans * x (Eq. 9);
 *   Trans is added to GPU_o if o is the first or the last operation or o-1 was
 *   placed on the CPU, to CPU_o otherwise; o goes to the CPU iff GPU_o > CPU_o.
 * base_cost <= 0 selects the Table II default of the operation's kind.
 * out_dev[o] receives LMS_DEV_CPU or LMS_DEV_GPU, out_cost[o] (may be NULL)
 * the cost of the chosen device including Trans where it was charged.
 * mode LMS_PLAN_LEARNED uses the learned model `model` (lms_mlp_model) and
 * falls back to the analytic rule if model is NULL. */
typedef enum {
  LMS_OP_AGG = 0,     /* Aggregation (Hash): CPU / 1.0 */
  LMS_OP_FILTER = 1,  /* Filtering: CPU / 1.0 */
  LMS_OP_SHUFFLE = 2, /* Shuffling: CPU / 1.0 */
  LMS_OP_PROJECT = 3, /* Projection: Neutral / 0.9 */
  LMS_OP_JOIN = 4,    /* Join (Hash): Neutral / 0.9 */
  LMS_OP_EXPAND = 5,  /* Expand: Neutral / 0.9 */
  LMS_OP_SCAN = 6,    /* Scan (CSV file): GPU / 0.8 */
  LMS_OP_SORT = 7     /* Sorting: GPU / 0.8 */
} lms_opkind;
typedef enum { LMS_DEV_CPU = 0, LMS_DEV_GPU = 1 } lms_device;
typedef enum { LMS_PLAN_ANALYTIC = 0, LMS_PLAN_LEARNED = 1 } lms_plan_mode;

typedef struct lms_op_desc {
  int32_t kind;     /* lms_opkind */
  int32_t ncols;    /* columns the operation reads (learned mode) */
  double base_cost; /* <= 0: Table II default */
  double window_s;  /* window length in seconds, 0 if not windowed (learned mode) */
  double slide_s;   /* window slide in seconds, 0 = tumbling (learned mode) */
} lms_op_desc;

typedef struct lms_batch_stats {
  int64_t batch_bytes; /* size of the micro-batch in bytes */
  int32_t num_cores;   /* NumCores (Table I): number of data partitions */
  int32_t reserved;
  int64_t rows;          /* rows of the micro-batch */
  double selectivity;    /* fraction of rows passing the filter */
  int64_t distinct_keys; /* estimated distinct group keys */
  double interval_s;     /* seconds since the previous micro-batch */
} lms_batch_stats;

typedef struct {
  double infpt_bytes; /* InfPT, the inflection point (Sec. III-D; initial 150 KB = 153600) */
  double base_trans;  /* baseTransCost of Eq. 9 (initial 0.1) */
  int32_t mode;       /* lms_plan_mode */
  int32_t reserved;
  const void* model; /* LMS_PLAN_LEARNED: a const lms_mlp_model*, else NULL */
} lms_cost_params;

double lms_table2_base_cost(int32_t kind);

/* Online inflection-point regression (Sec. III-E, Eq. 10), the tuner of the
 * analytic cost model: after each micro-batch, lms_infpt_record stores the
 * InfPT it ran with, its throughput (rows per ms of processing) and its
 * MaxLat (Eq. 5).  lms_infpt_next fits InfPT = b0 + b1 * Throughput +
 * b2 * Latency by least squares over the last `history` records (0: all),
 * evaluates it at the target throughput (the largest seen) and the target
 * latency (target_latency, or the mean past MaxLat if <= 0), and returns the
 * result times 1 + jitter * u, u uniform in [-1, 1] from SplitMix64 seeded
 * with `seed` (one draw per call; the exploration that keeps the fit
 * identifiable).  With fewer than three records, collinear regressors or a
 * prediction that is not positive, the previous InfPT (init_bytes at first)
 * is kept.  Host-only; returns -1 for a NULL handle. */
typedef struct lms_infpt lms_infpt;
int lms_infpt_create(double init_bytes, int32_t history, double jitter, uint64_t seed, lms_infpt** out);
int lms_infpt_record(lms_infpt* t, double infpt_used, double thput, double maxlat);
double lms_infpt_next(lms_infpt* t, double target_latency);
void lms_infpt_free(lms_infpt* t);
int lms_plan(const lms_op_desc* ops, int32_t nops, const lms_batch_stats* st, const lms_cost_params* cp,
             int32_t* out_dev, double* out_cost);

/* ---- Learned placement model --------------------------------------------------
 * A 12 -> 64 -> 64 -> 2 ReLU MLP predicting (log CPU ms, log GPU ms) of one
 * operation; in LMS_PLAN_LEARNED mode lms_plan places each operation of the
 * chain (Algorithm 2's walk) on the device with the smaller prediction, with
 * Algorithm 2's transfer condition as an input feature instead of Eq. 9.
 * Parameters (FP32, this order): W1[64][12], b1[64], W2[64][64], b2[64],
 * W3[2][64], b3[2].  Features (lms_mlp_features):
 *   x0 log2(rows+1)/24, x1 ncols/8, x2 selectivity, x3 log2(distinct+1)/20,
 *   x4..x7 one-hot class {filter/project/scan, tumbling aggregation, sliding
 *   aggregation, join}, x8 window_s/60, x9 slide_s/60, x10 interval_s/10,
 *   x11 transfer flag (1 if the operation is first or last or follows a CPU
 *   operation).
 * Training (device, stream-ordered): lms_mlp_loss_grad computes the gradient
 * of L = (1/n) sum_s sum_o mask[s][o] (y[s][o] - t[s][o])^2 over n samples
 * (x: n x 12, t and mask: n x 2, row-major device arrays) into d_grad[NPARAMS]
 * and d_loss[1]; lms_mlp_adam_step applies Adam.  lms_mlp_forward writes
 * y (n x 2) with FP32 weights or, if use_bf16, weights rounded to BF16. */
#define LMS_MLP_IN 12
#define LMS_MLP_HIDDEN 64
#define LMS_MLP_OUT 2
#define LMS_MLP_NPARAMS (64 * 12 + 64 + 64 * 64 + 64 + 2 * 64 + 2)
typedef struct lms_mlp lms_mlp;
typedef struct lms_mlp_model {
  float params[LMS_MLP_NPARAMS];
} lms_mlp_model;
int lms_mlp_create(uint64_t seed, lms_mlp** out);
void lms_mlp_free(lms_mlp* m);
int lms_mlp_set_params(lms_mlp* m, const float* host_params);
int lms_mlp_get_params(const lms_mlp* m, float* host_params);
size_t lms_mlp_workspace(int64_t n);
int lms_mlp_loss_grad(const lms_mlp* m, const float* d_x, const float* d_t, const float* d_mask, int64_t n,
                      float* d_grad, float* d_loss, void* workspace, size_t ws_bytes, lms_stream stream);
int lms_mlp_adam_step(lms_mlp* m, const float* d_grad, float lr, float beta1, float beta2, float eps,
                      lms_stream stream);
int lms_mlp_forward(const lms_mlp* m, const float* d_x, int64_t n, float* d_y, int32_t use_bf16, lms_stream stream);
void lms_mlp_host_forward(const float* host_params, const float* x, float* y);
void lms_mlp_features(const lms_op_desc* op, const lms_batch_stats* st, int32_t transfer, float* x);
float lms_bf16_round(float f);

#ifdef __cplusplus
}
#endif

#endif /* LMS_H */
