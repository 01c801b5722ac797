/*
 * sss.h -- speculative segmented sum CSR SpMV on AMD MI355X (gfx950).
 *
 * Computes y = A x for an m x n CSR matrix A (Section 1 states the problem;
 * Section 2.1 defines the CSR arrays): row_ptr (m+1 int32 offsets, row_ptr[0]
 * = 0, non-decreasing, row_ptr[m] = nnz), col (nnz int32 column indices in
 * [0, n)) and val (nnz values).  Rows may be empty; columns need not be sorted
 * or unique within a row.
 *
 * The method is the two-stage speculative segmented sum (Section 3): nnz is cut
 * into tiles of W*T nonzeros (T = 64, the wavefront width), each wavefront
 * ("thread-bunch") handles S consecutive tiles, a search of row_ptr
 * (rightmost match) gives each tile's first row, a segment descriptor built on chip marks row
 * heads, a segmented sum produces compact partial sums that are stored to y at
 * speculated positions, and tiles that contain empty rows are labelled dirty.
 * The second stage -- which the paper runs on a CPU core -- runs here as a
 * device fixup kernel: it adds the carries that cross thread-bunches (the
 * synchronizer) and moves the dirty tiles' partial sums to their rows.
 *
 * Memory and ownership
 *   All matrix and vector pointers passed to execute calls are caller-owned
 *   DEVICE pointers on the current HIP device; the library never frees or
 *   retains them past the call.  col and val must be 16-byte aligned (any
 *   hipMalloc / PyTorch allocation is).  A plan's auxiliary device arrays
 *   (synchronizer, bunch tails, per-bunch dirty masks, speculator) live
 *   from create to destroy, in its own allocation or in a workspace the
 *   caller provides (e.g. a PyTorch tensor).
 *   y is overwritten (not accumulated into).
 *
 * Streams
 *   `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   Execute calls only enqueue work: no allocation, no host synchronisation,
 *   so they can be captured in a HIP graph.  Calls that share a plan must be
 *   ordered on one stream: a plan's auxiliary buffers serve one call at a time.
 *
 * Errors
 *   Every call returns an sss_status.  SSS_ERR_HIP keeps the HIP error, which
 *   sss_last_hip_error() describes (thread-local).
 */
#ifndef SSS_H
#define SSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SSS_OK = 0,
  SSS_ERR_INVALID_VALUE = -1,  /* negative size, null pointer with nonzero size, bad option, misaligned */
  SSS_ERR_UNSUPPORTED = -2,    /* dtype or parameter combination not built */
  SSS_ERR_PLAN_MISMATCH = -3,  /* plan used on another device, or a bind_rows plan with another row_ptr */
  SSS_ERR_HIP = -4,            /* a HIP runtime call failed */
  SSS_ERR_INVALID_CSR = -5,    /* sss_validate_csr found a malformed matrix */
  SSS_ERR_TOO_LARGE = -6       /* sss_csr_spmv_noalloc: the matrix needs more than its static scratch */
} sss_status;

/* Value type.  SSS_F64: val, x, y are double.  SSS_F32: val, x, y are float.
 * SSS_BF16: val is bfloat16 (uint16 bit patterns), x and y are float.  The
 * reduced-precision types multiply in float, sum segments with compensated
 * (TwoSum) float arithmetic, and keep the carries between tiles and between
 * thread-bunches, and the fixup sums, in double. */
typedef enum { SSS_F64 = 0, SSS_F32 = 1, SSS_BF16 = 2 } sss_dtype;

/* How a plan chooses (W, S): FIXED takes opts.W/S/B; SELECTOR computes the
 * matrix features from row_ptr on the device and asks the selector network
 * loaded with sss_selector_set (the defaults when none is loaded).  The grid
 * search (GRID) needs the whole matrix and x, so it has a call of its own,
 * sss_csr_spmv_plan_create_grid; plan_create rejects GRID. */
typedef enum { SSS_MODE_SELECTOR = 0, SSS_MODE_GRID = 1, SSS_MODE_FIXED = 2 } sss_mode;

/* The parameter grid: class c has W = {4, 8, 16}[c / 4], S = {1, 2, 4, 8}[c % 4]
 * (T = 64 and B = 2).  Section 3.4 / Table 3 choose W and S per processor
 * empirically; here they are chosen per matrix. */
/* Largest m, n or nnz a plan accepts: 2^31 - 4097.  The kernels index rows
 * and nonzeros in 32-bit; the margin keeps "a tile boundary plus one tile"
 * and "a row chunk plus one wavefront" inside int32. */
#define SSS_MAX_INDEX 2147479551

#define SSS_N_CLASSES 12
#define SSS_N_FEATURES 8
#define SSS_MLP_HIDDEN 64
#define SSS_MLP_PARAMS 5516

typedef struct {
  int mode;  /* sss_mode */
  int W;     /* nonzeros per lane: 4, 8 or 16 (0 = default for the dtype) */
  int S;     /* tiles per wavefront, 1..16 (0 = default) */
  int B;     /* wavefronts per workgroup, 1..4 (0 = default) */
  int debug; /* nonzero: stage 1 also records tile start rows, segment
                descriptors and dirty flags for sss_plan_debug_dump */
  int bind_rows; /* nonzero: plan_create runs the tile boundary search of
                    Section 3.2 once, for every thread-bunch's first row, on
                    row_ptr (required); execute then reads those rows instead
                    of searching; the plan then serves only that row_ptr
                    array (SSS_ERR_PLAN_MISMATCH for another).  plan_create
                    also lists the thread-bunches that hold a dirty tile
                    (Section 3.2: an empty row r with row_ptr[r] > 0 lies in
                    the tile), and stage 2 gives only those a re-arrangement
                    wavefront instead of one per bunch */
  int batch_persistent; /* batch plans only.  0 (default): stage 1 launches one
                           wavefront per thread-bunch of every matrix.  Nonzero:
                           stage 1 is a persistent grid (as many workgroups as
                           stay resident) whose wavefronts loop over the
                           bunches.  Same results; the default measured faster. */
  void *workspace;        /* single-matrix plans: caller-owned DEVICE memory for the
                             plan's auxiliary arrays, 256-byte aligned, at least
                             sss_csr_spmv_plan_workspace_size bytes, kept alive and
                             unused by others until sss_plan_destroy.  NULL: the
                             plan allocates its own (hipMalloc) and frees it. */
  size_t workspace_bytes; /* size of `workspace` (0 when it is NULL) */
} sss_plan_opts;

typedef struct sss_plan_s *sss_plan;

/* Create a plan for an m x n matrix with nnz nonzeros of value type dt.
 * Section 3.3 sizes the auxiliary arrays it holds: the synchronizer has one
 * entry per thread-bunch, ceil(nnz / (S W T)); the speculator one per tile,
 * ceil(nnz / (W T)), here laid out as S slots per thread-bunch with a
 * per-bunch dirty mask in place of the single global dirty counter; beside
 * the synchronizer each bunch keeps its tail (the part of the row it ends
 * in, when that row goes on into the next bunch) in double, so that a row's
 * parts from several bunches meet in double and y is rounded once.
 * The arrays live in opts->workspace when given (nothing is allocated), else
 * in one hipMalloc owned by the plan.  They are cleared on `stream`.
 * m, n and nnz must not exceed SSS_MAX_INDEX (else SSS_ERR_INVALID_VALUE);
 * a workspace that is too small or not 256-byte aligned is
 * SSS_ERR_INVALID_VALUE.  row_ptr (device, may be NULL in FIXED mode without
 * bind_rows) is read only by the SELECTOR mode and by bind_rows.  Work is
 * enqueued on `stream`, which this call synchronises before it returns (no
 * device-wide synchronisation).  opts may be NULL (FIXED with the defaults).
 * Returns the plan in *out. */
int sss_csr_spmv_plan_create(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr,
                             sss_dtype dt, const sss_plan_opts *opts, void *stream,
                             sss_plan *out);

/* Bytes of device workspace a plan with these arguments needs (host call, no
 * device work): FIXED mode the exact size for its (W, S); SELECTOR mode the
 * largest over the parameter grid and the type's defaults, since the choice
 * is made in plan_create.  opts->workspace is ignored.  SSS_ERR_INVALID_VALUE
 * / SSS_ERR_UNSUPPORTED as for plan_create. */
int sss_csr_spmv_plan_workspace_size(int64_t m, int64_t n, int64_t nnz, sss_dtype dt,
                                     const sss_plan_opts *opts, size_t *bytes);

/* y = A x with a plan (both stages of Section 3.2, enqueued on `stream`).
 * The sizes are the plan's; val/x/y types follow the plan's dtype.  m = 0 is a
 * no-op; nnz = 0 zeroes y.  SSS_ERR_INVALID_VALUE for a NULL plan, a NULL
 * pointer whose array is non-empty, or misaligned col/val.  SSS_ERR_PLAN_MISMATCH
 * if the plan was created on another device, or if it binds rows (bind_rows)
 * and row_ptr is not the array it was made for.  A bound plan's stage 1 also
 * checks each thread-bunch's stored first row against row_ptr's contents
 * (rp[r] <= b < rp[r + 1]) and searches again where it no longer holds, so
 * rewriting that array in place (same m and nnz) gives a correct y, at the
 * search's cost; a dirty tile in a bunch the plan did not list then marks
 * the plan stale, and from that call on stage 2 also re-arranges the
 * unlisted dirty bunches (one after another per 64 bunches: correct, slower;
 * make a new plan for the new structure). */
int sss_csr_spmv_execute(sss_plan p, const int32_t *row_ptr, const int32_t *col,
                         const void *val, const void *x, void *y, void *stream);

/* The two stages of execute, separately (same arguments, same stream order
 * required: stage 2 must follow stage 1 of the same plan on the same stream,
 * with no other call on that plan in between).
 * Stage 1, speculative execution (Section 3.2 and the appendix algorithm's
 * first-stage function): writes y at speculated positions, the synchronizer,
 * the dirty masks and the speculator.  Stage 2, checking prediction
 * (Section 3.2; the appendix's synchronization function plus the
 * re-arrangement): adds the cross-bunch carries, moves the dirty tiles' partial
 * sums to their rows and zeroes leading empty rows.  Every buffer stage 1
 * reads is rewritten by it, so nothing needs resetting between calls.
 * They exist so that a caller can time or overlap the stages. */
int sss_csr_spmv_stage1(sss_plan p, const int32_t *row_ptr, const int32_t *col, const void *val,
                        const void *x, void *y, void *stream);
int sss_csr_spmv_stage2(sss_plan p, const int32_t *row_ptr, void *y, void *stream);

/* Stage 2 on a host core, as the paper runs it on its heterogeneous
 * processors (Section 3.2, Section 3.4), for comparison with the device
 * fixup: waits for the device, copies the plan's synchronizer, dirty masks
 * and speculator to host memory, then performs the carries, the dirty-tile
 * re-arrangement and the zeroing of leading empty rows in one host thread.
 * row_ptr and y are HOST pointers (y holds stage 1's output, e.g. pinned
 * host memory that stage 1 wrote directly).  Not for performance: the
 * device stage 2 is the product path. */
int sss_csr_spmv_stage2_host(sss_plan p, const int32_t *row_ptr, void *y);

/* The one-call form of the method in double precision: y = A x with the
 * default parameters.  Keeps an internal plan per (device, stream, m, n, nnz)
 * that it allocates on first use (so the first call for a new size on a
 * stream is not graph-capturable; later calls are) and keeps until the
 * process ends or sss_csr_spmv_cache_clear.  Calls on one stream run in
 * order; calls of the same size on
 * different streams use different plans and may overlap. */
int sss_csr_spmv(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr,
                 const int32_t *col, const double *val, const double *x, double *y,
                 void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as sss_csr_spmv (double precision, the default parameters, the same
 * kernels, so the same y bit for bit) with the plan's auxiliary arrays in a
 * static device array of 16 MiB that the library holds on each device until
 * the process ends, instead of a cached plan.  Allocates nothing and never
 * synchronises; on a device's first call it looks up that array's address
 * (hipGetSymbolAddress).  Limit: the arrays take about 104 bytes per 2,560
 * nonzeros, so nnz up to about 412 million (beyond: SSS_ERR_TOO_LARGE, before
 * any device work).  Every call on a device shares that one array: calls that
 * overlap on one device (two streams, or two host threads) race and give
 * wrong results; order them on one stream.  Each call leaves the array
 * holding its own intermediate state, which the next call overwrites (nothing
 * needs clearing).  Other arguments and errors as for sss_csr_spmv. */
int sss_csr_spmv_noalloc(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr,
                         const int32_t *col, const double *val, const double *x, double *y,
                         void *stream);

/* Free every plan sss_csr_spmv has cached, on every device and stream (a
 * process that sees many sizes can bound its memory this way).  Waits for
 * the devices the plans live on; the next sss_csr_spmv of a size plans it
 * again.  Must not run while another thread is inside sss_csr_spmv or while
 * a stream is capturing one of its calls.  Returns the first error met, after
 * freeing what it could. */
int sss_csr_spmv_cache_clear(void);

/* One matrix of a batch: device pointers (caller-owned, as for execute), its
 * sizes, and optionally its own S (tiles per wavefront; 0 = the batch's). */
typedef struct {
  int64_t m, n, nnz;
  const int32_t *row_ptr;
  const int32_t *col;
  const void *val;
  const void *x;
  void *y;
  int S;
  int reserved;
} sss_csr_desc;

/* A batch plan: y_i = A_i x_i for `count` matrices in one launch per stage.
 * The thread-bunches of all matrices form one nnz-balanced index space
 * (Section 3.1's decomposition applied to the concatenation); the plan finds
 * each bunch's matrix with the same rightmost-match search the method uses
 * for rows (Section 3.2).  Stage 1 runs one wavefront per bunch, each XCD
 * taking a contiguous run of the bunch space (opts->batch_persistent: a
 * persistent grid instead); stage 2 is a persistent grid.  All matrices
 * share dtype and W; each may have its own S.
 * FIXED mode (opts NULL or mode FIXED): W = opts->W (0: the type's default),
 * each matrix's S = its descriptor's S, else opts->S, else the default.
 * SELECTOR mode: the tile schedule comes from the loaded selector network
 * (sss_selector_set; the type's defaults when none is loaded): each matrix's
 * features (sss_csr_features), with the three size features (rows, columns,
 * nonzeros) replaced by the batch's totals -- one grid runs the bunches of
 * all matrices, so how well a schedule fills the device depends on the whole
 * launch -- are scored (sss_selector_scores); W is
 * opts->W if given, else the W of the class picked for most nonzeros of the
 * batch; each matrix then takes the S of its best-scored class with that W
 * (descriptors' S are ignored).  The descriptors' pointers are bound to the
 * plan: the plan must be recreated if a matrix or vector moves.  Different
 * matrices must not share y storage.  Allocates (the descriptors, prefix
 * arrays and every matrix's synchronizer/speculator) and synchronises. */
int sss_batch_plan_create(int count, const sss_csr_desc *mats, sss_dtype dt, const sss_plan_opts *opts,
                          void *stream, sss_plan *out);

/* Batched GRID plan: the autotuner's choice of tile schedule for a batch.
 * Builds a batch plan for every class (W, S) of the grid, with that S for
 * every matrix (per-matrix S in `mats` is ignored), times each with the
 * autotuner's protocol (see sss_csr_spmv_autotune; `reps` runs of the whole
 * batch per trial) and returns the fastest in *out (NULL on any error).
 * class_us (host, 12 floats, may be NULL) receives each class's microseconds
 * per batch launch, *best_class (may be NULL) the chosen class.  Every y is
 * overwritten.  Allocates and synchronises. */
int sss_batch_plan_create_grid(int count, const sss_csr_desc *mats, sss_dtype dt, int reps, void *stream,
                               float *class_us, int *best_class, sss_plan *out);

/* A batch plan's tile schedule (host call): its W, and each matrix's S in
 * HOST S[count] (count must be the plan's matrix count).  Either may be
 * NULL. */
int sss_batch_plan_schedule(sss_plan p, int count, int *W, int *S);

/* Run a batch plan on `stream`: two launches (stage 1, stage 2), no
 * allocation, no host synchronisation. */
int sss_batch_execute(sss_plan p, void *stream);

/* The same two launches captured once into a HIP graph (on the first call,
 * on a private stream) and replayed on `stream` by every call. */
int sss_batch_graph_launch(sss_plan p, void *stream);

/* Free a plan.  Its own device buffer (no workspace given) goes with hipFree,
 * which waits for the device's outstanding work; a caller-provided workspace
 * is left to the caller and nothing waits.  NULL is OK. */
int sss_plan_destroy(sss_plan p);

/* The plan's chosen parameters and sizes (host integers, any may be NULL). */
int sss_plan_info(sss_plan p, int *W, int *S, int *B, int64_t *n_tiles, int64_t *n_bunches);

/* The sizes and value type a single-matrix plan was made for (host values,
 * any pointer may be NULL).  SSS_ERR_INVALID_VALUE for NULL or a batch plan. */
int sss_plan_shape(sss_plan p, int64_t *m, int64_t *n, int64_t *nnz, sss_dtype *dt);

/* Debug: check row_ptr[0] = 0, monotone row_ptr, row_ptr[m] = nnz and every
 * column in [0, n), on the device.  Synchronises `stream`.  Returns SSS_OK or
 * SSS_ERR_INVALID_CSR. */
int sss_validate_csr(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr,
                     const int32_t *col, void *stream);

/* The thread-bunches a bind_rows plan found, at plan time, to hold a dirty
 * tile (Section 3.2's dirty condition on row_ptr), in increasing order: the
 * first min(*n, cap) of them are copied to host_out (host, int32, may be NULL
 * when cap = 0) and *n receives their number.  Stage 2 gives each listed
 * bunch one re-arrangement wavefront.  A plan with no thread-bunch (m = 0 or
 * nnz = 0) lists none.  SSS_ERR_INVALID_VALUE for a NULL plan or n, a batch
 * plan, or a plan with bunches made without bind_rows. */
int sss_plan_dirty_list(sss_plan p, int32_t *host_out, int64_t cap, int64_t *n);

/* Debug: bytes needed by sss_plan_debug_dump for this plan. */
int sss_plan_debug_size(sss_plan p, size_t *bytes);

/* Debug: copy the last execute's intermediate state to host memory (waits for
 * the device).  Layout, all little-endian:
 *   int64 header[4] = {n_tiles, n_bunches, dirty_count, words_per_tile}
 *   int32 tile_start[n_tiles]          (debug plans only, else zeros)
 *   int32 tile_dirty[n_tiles]          (debug plans only, else zeros)
 *   uint32 heads[n_tiles * words_per_tile]  segment descriptor bits, bit k of
 *          word w = entry 32w+k of the tile, forced first bit included
 *          (debug plans only, else zeros)
 *   int32 speculator[n_tiles * 4]      {start, stop, tile, 0} of every dirty
 *          tile, in tile order; the first dirty_count entries are valid
 *   int32 sync_idx[n_bunches]
 *   double sync_val[n_bunches]
 *   double tail_val[n_bunches]         the bunch's last partial where it ends
 *          inside a row that is not its first row and continues into the
 *          next bunch (else the value a previous call left, or 0)
 * Section 3.2 and the appendix algorithm define these arrays (the tail is
 * this implementation's: the paper stores that partial to y). */
int sss_plan_debug_dump(sss_plan p, void *host_buf, size_t bytes);

/* ---------------------------------------------------------------------------
 * Parameter selection
 * ------------------------------------------------------------------------- */

/* (W, S) of grid class cls (host integers). */
int sss_class_params(int cls, int *W, int *S);

/* Matrix features from row_ptr (device), one pass on `stream`, which this call
 * synchronises; feats is HOST float[8]:
 *   log2(m+1), log2(n+1), log2(nnz+1), log2(1+mean row length),
 *   log2(1+row-length variance), log2(1+max row length), empty-row fraction,
 *   bytes per stored value (8, 4 or 2 for F64, F32, BF16). */
int sss_csr_features(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr, sss_dtype dt, void *stream,
                     float *feats);

/* Grid autotuner: times y = A x for every class, with plans that bind the
 * rows (bind_rows) as a plan made for this one matrix would (after two warm-up runs of
 * each class, five rounds over the classes in turn, each a trial of `reps`
 * back-to-back runs between HIP events on `stream`; per class the median
 * trial's mean), writes microseconds per run for each class to HOST
 * class_us[12] (may be NULL) and the fastest class to *best_class.
 * Device arguments as for execute; y is overwritten.  Allocates plans and
 * synchronises. */
int sss_csr_spmv_autotune(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col,
                          const void *val, const void *x, void *y, sss_dtype dt, int reps, void *stream,
                          float *class_us, int *best_class);

/* Row-wise comparator, NOT the speculative method: the row-based GPU
 * kernels the paper measures against (Section 4.3, CSR-scalar and
 * CSR-vector; Section 2.1 explains their load imbalance on irregular
 * matrices), written for gfx950.  lanes_per_row = 1 is CSR-scalar (a thread
 * per row), 64 is CSR-vector (a wavefront per row), powers of two between
 * give sub-wavefront groups; a row's lanes stride over it and reduce by
 * shuffles.  Plain sums (double for SSS_F64, float otherwise), no plan, no
 * allocation; y is overwritten.  Arguments as for execute; dt as for plans.
 * SSS_ERR_INVALID_VALUE for m, n or nnz negative or above SSS_MAX_INDEX;
 * SSS_ERR_UNSUPPORTED for any other lanes_per_row. */
int sss_csr_rowwise(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col, const void *val,
                    const void *x, void *y, sss_dtype dt, int lanes_per_row, void *stream);
const char *sss_rowwise_last_hip_error(void);

/* Conjugate gradients for a symmetric positive definite A, the iterative use
 * the paper names as the reason to keep CSR (Section 1: a matrix multiplied a
 * few hundred times, where a format conversion would cost as much as the
 * solve).  The iteration is Hestenes and Stiefel's: with q = A p,
 * alpha = (r.r) / (p.q), x += alpha p, r -= alpha q, beta = (r.r)_new / (r.r),
 * p = r + beta p.  Every product goes through the FP64 plan p
 * (sss_csr_spmv_execute, so its checks and errors apply); every vector step
 * and dot product runs in this library's kernels; the step scalars stay on
 * the device, so the calls only enqueue work on `stream` (no host
 * synchronisation, no allocation).  Dot products are plain double sums,
 * per workgroup in a fixed order and then over the workgroups in a fixed
 * order, so a run repeats bit for bit.  A zero p.q or r.r gives alpha or beta
 * = 0 instead of a division by zero (b = 0 from x = 0 stays at 0).
 *
 * Arrays: x, r, dir (the search direction p), q are caller-owned DEVICE
 * double arrays of m entries (the plan's m; the plan must be square, n = m),
 * b likewise (read only); work is caller-owned DEVICE memory of
 * sss_cg_workspace_size bytes, 8-byte aligned, whose first three doubles hold
 * after every call: [0] r.r of the current residual, [1] r.r before the last
 * step, [2] b.b (set by sss_cg_start).  A host reads [0] and [2] for the
 * relative residual sqrt(r.r / b.b).  The five vectors and work must not
 * overlap.  Calls that share work, or any of the vectors, must be ordered on
 * one stream.
 * SSS_ERR_INVALID_VALUE for a NULL or misaligned argument, a batch plan, a
 * non-square plan or iterations < 0; SSS_ERR_UNSUPPORTED for a plan that is
 * not SSS_F64. */
int sss_cg_workspace_size(size_t *bytes);
/* The start: q = A x, r = b - q, dir = r, work = (r.r, r.r, b.b). */
int sss_cg_start(sss_plan p, const int32_t *row_ptr, const int32_t *col, const double *val, const double *b,
                 const double *x, double *r, double *dir, double *q, void *work, void *stream);
/* `iterations` steps of the iteration from the state that sss_cg_start or the
 * previous sss_cg_iterate left in x, r, dir and work (q is scratch). */
int sss_cg_iterate(sss_plan p, const int32_t *row_ptr, const int32_t *col, const double *val, double *x,
                   double *r, double *dir, double *q, void *work, int iterations, void *stream);
const char *sss_cg_last_hip_error(void);

/* Measurement aid, not part of the method: the memory floor of stage 1's
 * access pattern under plan p's tiling (W, S, B).  Streams col and val once,
 * tile by tile, with the same loads and the same one-tile-ahead prefetch as
 * stage 1; with gather != 0 each value is multiplied by x[col] as in the
 * products, else x is not read.  No row structure is read, nothing is
 * segmented, and each lane writes one sum: out[b*64 + lane] for thread-bunch
 * b, so `out` (device, y type of the plan) holds n_bunches*64 elements
 * (n_bunches from sss_plan_info).  Comparing stage 1's time with this one
 * separates the method's own work from the cost of reading the matrix and
 * gathering x.  Same pointer rules as execute; asynchronous on `stream`. */
int sss_floor_probe(sss_plan p, const int32_t *col, const void *val, const void *x, void *out, int gather,
                    void *stream);

/* The same measurement for a batch plan: the batched stage 1's launch (one
 * wavefront per thread-bunch, the same mapping of workgroups to XCDs and
 * the same per-bunch lookup of matrix and bunch) running the probe's loads
 * on each matrix's own col, val and x from the plan's descriptors.  out
 * (device, y type of the plan) holds 64 elements per global thread-bunch:
 * out[g*64 + lane] for bunch g of the concatenated bunch space
 * (n_bunches from sss_plan_info).  SSS_ERR_UNSUPPORTED for a
 * batch_persistent plan.  Asynchronous on `stream`. */
int sss_batch_floor_probe(sss_plan p, void *out, int gather, void *stream);

/* Measurement aid, not part of the method: how fast the device serves random
 * gathers x[col[k]] at all, with none of stage 1's choices (Section 4.4 measures
 * the method by bandwidth utilisation; this is the ceiling the gathers put on
 * it).  A grid-stride loop gives every lane one nonzero per iteration
 * (k = thread + i * threads: col and val read coalesced) and keeps `unroll`
 * (1, 2, 4, 8 or 16) gathers in flight before using any; with_val also
 * streams val and multiplies (all the reads of a CSR SpMV, without its row
 * structure).  mode 0: plain vector loads; 1: non-temporal loads; 2: direct-
 * to-LDS loads (a gather in flight holds no VGPR); 3: buffer loads at device
 * scope (not kept in the CU's L1); plus 4: every wavefront sweeps its own
 * contiguous chunk of the nonzeros (64 at a time) instead of the whole grid
 * sweeping them as one front.  waves_per_simd (1, 2, 4 or 8) caps the
 * occupancy by reserving LDS; the registers may cap it lower, and
 * *resident_per_cu receives the workgroups (of 4 wavefronts) per CU actually
 * launched.  dt is SSS_F64 (x, val double) or SSS_F32 (float); every column
 * must be in [0, n).  out (device, the x type) receives one sum per thread:
 * *threads entries, at most out_len.  Asynchronous on `stream`. */
int sss_gather_probe(const int32_t *col, const void *val, const void *x, int64_t nnz, int64_t n, sss_dtype dt,
                     int mode, int unroll, int waves_per_simd, int with_val, void *out, int64_t out_len,
                     int64_t *threads, int *resident_per_cu, void *stream);
/* The same probe plus the row part of a CSR SpMV's bytes: with row_ptr
 * non-NULL it also reads row_ptr[0..m] (device int32, m + 1 entries) and
 * writes y[r] = row_ptr[r] for r < m (device, the x type), both coalesced in
 * a grid-stride loop, so the probe moves every byte the product moves (col,
 * val, x, row_ptr, y).  The rows go in batches of 4 per thread (loads before
 * stores), spread over the gather loop; mode plus 8 puts them all after it
 * instead.  row_ptr NULL is sss_gather_probe.  INVALID for m < 0, m above
 * SSS_MAX_INDEX, or m > 0 with y NULL. */
int sss_gather_probe_rows(const int32_t *col, const void *val, const void *x, int64_t nnz, int64_t n, sss_dtype dt,
                          int mode, int unroll, int waves_per_simd, int with_val, void *out, int64_t out_len,
                          int64_t *threads, int *resident_per_cu, const int32_t *row_ptr, int64_t m, void *y,
                          void *stream);
const char *sss_probe_last_hip_error(void);

/* GRID-mode plan (the selector's fallback, and the yardstick of its regret):
 * runs sss_csr_spmv_autotune on the caller's matrix and returns in *out a
 * plan with the fastest class's (W, S), the default B and the rows bound
 * (bind_rows) to this row_ptr.  Arguments as for
 * sss_csr_spmv_autotune; y is overwritten; *out is NULL on any error.
 * Allocates and synchronises (a planning call, not for a timed loop). */
int sss_csr_spmv_plan_create_grid(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col,
                                  const void *val, const void *x, void *y, sss_dtype dt, int reps, void *stream,
                                  sss_plan *out);

/* Selector network 8 -> 64 -> 64 -> 12 (ReLU), FP32 parameters packed as
 * W1[8][64], b1[64], W2[64][64], b2[64], W3[64][12], b3[12] (W[i][o]: input i
 * to output o).  All arrays DEVICE float unless stated; N samples, row-major.
 *   forward:  H1 = relu(X W1 + b1), H2 = relu(H1 W2 + b2), Z = H2 W3 + b3
 *   backward: softmax cross-entropy of Z against target distributions Q
 *             [N][12], mean over samples: the gradient (packed like params)
 *             and optionally the per-sample loss [N]; work holds N*140 floats
 *   adam:     one Adam step (bias-corrected, step >= 1) on n parameters
 * Each only enqueues on `stream`.  These train the selector (on the
 * autotuner's timings) and run its inference. */
int sss_mlp_forward(const float *params, const float *X, int N, float *H1, float *H2, float *Z, void *stream);
int sss_mlp_backward(const float *params, const float *X, const float *H1, const float *H2, const float *Z,
                     const float *Q, int N, float *grad, float *loss, float *work, void *stream);
int sss_mlp_adam(float *params, const float *grad, float *m1, float *m2, int n, int step, float lr, float beta1,
                 float beta2, float eps, void *stream);

/* Load a trained selector for the current device: HOST params[5516] and the
 * feature normalisation (x - mean) / std, HOST float[8] each.  Copies them;
 * allocates on first use and keeps the device copy until the process ends. */
int sss_selector_set(const float *params, const float *mean, const float *stdv);

/* Class the loaded selector picks for HOST features[8] (forward kernels on the
 * device, synchronous).  SSS_ERR_UNSUPPORTED if no selector is loaded. */
int sss_selector_predict(const float *feats, int *cls);

/* The loaded selector's 12 class scores (logits, HOST float[12]) for HOST
 * features[8]; the class it picks is the largest.  Batch plans in SELECTOR
 * mode use them to pick each matrix's S among the classes of the batch's W.
 * SSS_ERR_UNSUPPORTED if no selector is loaded. */
int sss_selector_scores(const float *feats, float *logits);

/* 1 if a selector is loaded on the current device. */
int sss_selector_loaded(void);

/* Human-readable status; sss_last_hip_error the last HIP failure (thread). */
const char *sss_status_string(int status);
const char *sss_last_hip_error(void);

/* Library version string. */
const char *sss_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SSS_H */
