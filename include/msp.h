/*
 * msp.h -- C ABI of the MI355X (gfx950) sparse general matrix-matrix product.
 *
 * The library computes C = A * B for sparse A (m x k) and B (k x n) stored in
 * CSR (FSpGEMM Sec. II-A: values, column indices and row pointers), by the
 * row-wise Gustavson method (FSpGEMM Sec. II-B, Fig. 1):
 *
 *     C(i,:) = sum over stored A(i,k) of  A(i,k) * B(k,:)
 *
 * where adding sparse rows merges equal column indices by adding their values
 * (Sec. II-B, "sort and merge"; Algorithm 1).  The merge never tests a sum
 * for zero, so C's structure is the structural union of the B rows that
 * A(i,:) selects: an entry whose terms cancel to 0.0 is still stored.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers inside msp_csr / msp_csr_out are DEVICE pointers on the
 *    handle's device.  Scalar sizes are host values.
 *  - row_ptr is int64 with nrows + 1 entries; its values index col and val
 *    directly and never exceed nnz, the length of those arrays (row_ptr[0]
 *    may be > 0, e.g. for one matrix's rows inside a larger array); col is int32
 *    (so ncols <= 2^31 - 1); nrows <= 2^31 - 8193 (MSP_ERR_INDEX_OVERFLOW
 *    above: launch grids are rounded up from it in 32-bit arithmetic), and
 *    the same bound holds for a batch's total rows; values are FP32 or FP64,
 *    the same type for A, B and C.
 *  - Inputs must be canonical CSR: row_ptr non-decreasing, columns strictly
 *    increasing inside each row and in [0, ncols).  With opts->validate = 1
 *    the library checks this on the device and returns
 *    MSP_ERR_UNSORTED_OR_DUP (or MSP_ERR_INVALID_ARG for out-of-range
 *    indices) instead of computing.
 *  - The output is canonical CSR with strictly increasing columns in a row.
 *  - Inputs are borrowed: they must stay valid until the work queued on the
 *    handle's stream has completed.  The handle owns its workspace and frees
 *    it in msp_destroy.  Output arrays obtained through the allocator belong
 *    to the caller.
 *  - Every call is asynchronous on the handle's stream except for the points
 *    named per entry point where the host must read a size back.  Within a
 *    call, bins with few rows may run on the handle's own side streams
 *    (default priority): they are forked from the handle's stream by an
 *    event and joined back into it before the call queues anything after
 *    them, so every call's work is still ordered after earlier work on the
 *    handle's stream and before later work there.
 *  - No entry point throws, aborts or exits.  On error the return value says
 *    what failed and msp_last_error() gives a message (thread-local); output
 *    arrays already obtained from the allocator are released through its
 *    free function.
 *  - A handle is not thread-safe: calls on one handle must not overlap.
 */
#ifndef MSP_H
#define MSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MSP_OK = 0,
    MSP_ERR_INVALID_ARG = 1,     /* null pointer, negative size, bad option   */
    MSP_ERR_SHAPE = 2,           /* A.ncols != B.nrows, or C shape mismatch    */
    MSP_ERR_DTYPE = 3,           /* value types differ or are not FP32/FP64    */
    MSP_ERR_UNSORTED_OR_DUP = 4, /* input rows not strictly increasing         */
    MSP_ERR_OOM = 5,             /* allocator or workspace allocation failed   */
    MSP_ERR_HIP = 6,             /* a HIP runtime call failed                  */
    MSP_ERR_INDEX_OVERFLOW = 7,  /* a size does not fit the index types        */
    MSP_ERR_UNSUPPORTED = 8      /* a feature not built for this device        */
} msp_status;

typedef enum { MSP_F32 = 0, MSP_F64 = 1 } msp_dtype;

/* A read-only CSR operand (device pointers). */
typedef struct {
    int64_t nrows, ncols, nnz;
    const int64_t* row_ptr;      /* nrows + 1 */
    const int32_t* col;          /* nnz       */
    const void* val;             /* nnz values of type dtype */
    msp_dtype dtype;
} msp_csr;

/* The CSR result.  On input the caller sets row_ptr to a device buffer of
 * nrows + 1 int64 (nrows = A.nrows) or leaves it NULL to have it allocated;
 * col and val are always allocated by the library through the handle's
 * allocator once nnz(C) is known.  On return all fields are filled in. */
typedef struct {
    int64_t nrows, ncols, nnz;
    int64_t* row_ptr;
    int32_t* col;
    void* val;
    msp_dtype dtype;
} msp_csr_out;

/* Device allocator used for outputs.  alloc returns a device pointer of at
 * least `bytes` bytes usable on `stream` (NULL on failure); free releases
 * it.  Python passes callbacks that create and drop torch tensors.  With no
 * allocator set the library uses hipMalloc / hipFree. */
typedef void* (*msp_alloc_fn)(void* ctx, size_t bytes, void* stream);
typedef void (*msp_free_fn)(void* ctx, void* ptr, void* stream);

/* Tuning of the per-bin accumulators.  Zero-initialised fields mean "use the
 * library default".  See msp_autotune. */
typedef struct {
    int32_t hash_scale;     /* table slots = nextpow2(bound) << hash_scale (1..2) */
    int32_t group_scale;    /* lanes per row = default << group_scale (0..2)      */
    int32_t spill_nnz;      /* numeric rows with more nnz use the global path
                               (a power of two, 256..4096)                       */
    int32_t block_rows;     /* rows with bound above this (a power of two,
                               32..1024) use one workgroup per row; below it,
                               merges, lane groups or one wave per row (the
                               wave tables stop at 2048 symbolic keys and 512
                               numeric slots, beyond which workgroups take
                               over)                                            */
    int32_t merge_k;        /* rows with bound <= 32 and at most merge_k A
                               entries use the per-lane merge (4 or 8; -1: off) */
    int32_t share_g;        /* B-row sharing in the numeric merge (Sec. IV-A):
                               a wave takes at most share_g rows (8..64) and
                               stages every distinct B row they reference once
                               in LDS when they fit (-1: off, the default)    */
} msp_tuning;

typedef struct {
    int32_t validate;       /* 1: check inputs on the device first            */
    int32_t force_spill;    /* 1: every nonempty row takes the global path    */
    msp_tuning tuning;      /* zero: defaults (or the handle's tuned values)  */
    int32_t queue_rows;     /* batches: the numeric merge's rows reach the
                               waves as tickets of queue_rows consecutive rows
                               from one shared atomic counter (0: 1024; a
                               multiple of 64 up to 65536; -1: one static row
                               range per wave instead).  Plain calls: unused */
} msp_opts;

typedef struct msp_handle msp_handle;

/* ---- handle -------------------------------------------------------------- */

/* Create a handle on `device` that queues all work on `hip_stream` (a
 * hipStream_t; NULL means the device's null stream), forking bins onto three
 * side streams the handle creates and destroys itself.  Selects the device,
 * checks that it is gfx950 (MSP_ERR_UNSUPPORTED otherwise). */
msp_status msp_create(msp_handle** h, int device, void* hip_stream);
msp_status msp_destroy(msp_handle* h);
/* Queue the handle's later work on `hip_stream`.  The handle's workspaces
 * are shared by its calls, so work queued on the new stream first waits for
 * everything already queued on the old one (an event, no host wait). */
msp_status msp_set_stream(msp_handle* h, void* hip_stream);
msp_status msp_set_allocator(msp_handle* h, msp_alloc_fn alloc, msp_free_fn free_fn, void* ctx);
/* Tuning used when a call's opts->tuning is all zero. */
msp_status msp_set_tuning(msp_handle* h, const msp_tuning* t);
msp_status msp_get_tuning(const msp_handle* h, msp_tuning* t);

/* ---- the plain two-phase product ---------------------------------------- */

/*
 * C = A * B by row-wise Gustavson (FSpGEMM Sec. II-B), two phases:
 *   1. per-row statistics: intermediate products prod_i = sum over A(i,k)
 *      of nnz(B(k,:)), bound u_i = min(prod_i, n);
 *   2. binning of rows by u_i;
 *   3. symbolic pass: per-row structural union size row_nnz_i, with a
 *      per-bin LDS hash of keys, an LDS bitmap, or a global bitmap;
 *   4. device prefix sum -> C.row_ptr, nnz(C);
 *   5. re-binning by row_nnz_i and the numeric pass: LDS hash accumulators
 *      (FP64 sums for both value types) with an in-row column sort; rows
 *      too large for LDS are cut into column slices, each with an LDS
 *      bitmap and an FP64 accumulator indexed by the column's rank, and go
 *      out in column order from the bitmap (the slices are sized from the
 *      symbolic pass's per-window output counts).
 * Host synchronisation: two small device-to-host reads (bin counts, then
 * nnz(C) with the numeric bin counts).  The numeric pass is only queued:
 * it completes on the handle's stream after the call returns.  Its internal
 * consistency checks (a row count that differs from the symbolic count, a
 * hash probe bound) are reported by the next call on the handle or by
 * msp_sync.  Values of C are rounded once from FP64 sums; they satisfy
 * |c - exact| <= k * eps64 * sum|a||b| for a row with k terms.
 * C.col and C.val share one allocation from the allocator: C.col is its
 * start (release that pointer) and C.val follows at the next 256-byte
 * boundary.
 */
msp_status msp_spgemm(msp_handle* h, const msp_csr* A, const msp_csr* B,
                      msp_csr_out* C, const msp_opts* opts);

/* Wait for the work queued on the handle's stream; report any internal
 * error the numeric kernels of earlier calls flagged. */
msp_status msp_sync(msp_handle* h);

/*
 * msp_spgemm for callers that cannot allocate device memory: code under
 * stream or graph capture, serving loops and harnesses that forbid
 * allocation.  It calls no hipMalloc, hipFree or allocator callback.
 *   - Workspace: every per-call workspace of msp_spgemm is carved from one
 *     fixed device array of MSP_NOALLOC_SCRATCH_BYTES bytes per GPU, set up
 *     when the library's first handle on that GPU is created and held until
 *     the process ends.  All handles and calls on a GPU share it, and it keeps
 *     the last call's contents: calls on one GPU whose work overlaps (two
 *     handles, two streams, two threads) race; serialise them.  Products
 *     whose workspace does not fit are refused with MSP_ERR_INVALID_ARG (more
 *     than about (MSP_NOALLOC_SCRATCH_BYTES - 1 MiB) / 24 rows, checked
 *     before anything runs) or MSP_ERR_OOM (a larger workspace found later,
 *     after some kernels ran: C's contents are then undefined).
 *   - Output: the caller sets C->row_ptr (A.nrows + 1 int64), C->col
 *     (capacity int32) and C->val (capacity values of the operands' type),
 *     device buffers; on return C->nnz is nnz(C) and C->col / C->val are the
 *     caller's buffers.  When nnz(C) > capacity the call returns
 *     MSP_ERR_INVALID_ARG with C->nnz set to the count needed and C->row_ptr
 *     holding C's row pointers (the numeric pass has not run).
 *   - Otherwise as msp_spgemm: the same kernels and results, the same host
 *     reads, and the numeric pass only queued on the handle's stream.
 *     Profiling is suspended during the call.
 */
#define MSP_NOALLOC_SCRATCH_BYTES (64LL << 20)
msp_status msp_spgemm_noalloc(msp_handle* h, const msp_csr* A, const msp_csr* B, msp_csr_out* C,
                              int64_t capacity, const msp_opts* opts);

/*
 * Autotuner for one product (it replaces the paper's analytic choice of its
 * hardware parameters, Sec. IV-B4, Eqs. 2-3, by measurement): runs
 * msp_spgemm(A, B) with each of the ncand tunings, one warm call and then
 * `reps` timed calls each (HIP events around the whole call on the
 * handle's stream, the result waited for and released through the
 * allocator), and returns in *best the tuning with the smallest median time;
 * times_ms (ncand doubles, may be NULL) receives each median, or infinity
 * for a candidate the library rejects.  The handle's own tuning is not
 * changed (pass *best to msp_set_tuning).  Synchronises.  Errors: a bad
 * argument; MSP_ERR_HIP at once if the device reports an error; otherwise
 * the last candidate's error when none ran.
 */
msp_status msp_autotune(msp_handle* h, const msp_csr* A, const msp_csr* B, const msp_tuning* cand, int ncand,
                        int reps, msp_tuning* best, double* times_ms);

/* ---- B-row sharing (Sec. IV-A) ------------------------------------------- */

/* The count behind OMAR (Eq. 1).  With A's rows taken in groups of `group`
 * consecutive rows (the last group may be shorter), a row of B is read once
 * per distinct (group, column) pair of A rather than once per entry; this
 * writes that number of pairs to *distinct (host memory), so that
 * OMAR = (nnz(A) - *distinct) / nnz(A).  A is a device CSR (canonical);
 * group in 1..4096 (MSP_ERR_INVALID_ARG otherwise).  Synchronises the
 * handle's stream. */
msp_status msp_omar(msp_handle* h, const msp_csr* A, int64_t group, int64_t* distinct);

typedef struct {
    int64_t batches;      /* merge batches that read B from the LDS stage     */
    int64_t a_entries;    /* A entries of those batches' merge rows: the B-row
                             reads they would make without sharing           */
    int64_t b_rows;       /* distinct B rows they staged, each read once      */
} msp_share_stats;

/* B-row sharing figures of the handle's last call (msp_spgemm with
 * tuning.share_g on; zero otherwise).  Synchronises the handle's stream. */
msp_status msp_share_stats_get(msp_handle* h, msp_share_stats* out);

/* Only the symbolic part: row_nnz (device, A.nrows int32) and the total.
 * Used to produce training targets for the predictor. */
msp_status msp_spgemm_symbolic(msp_handle* h, const msp_csr* A, const msp_csr* B,
                               int32_t* row_nnz, int64_t* nnz_total,
                               const msp_opts* opts);

/* Per-row features of A*B (device outputs, A.nrows rows each; any pointer
 * may be NULL): prod (int64), and the 8 FP32 predictor inputs per row
 * (row-major m x 8): log2(1+x)/16 of nnz(A(i,:)), prod_i, min/mean/max
 * nnz(B(k,:)) and ncols(B), then min(1, prod_i/n) and span_i/n, where
 * span_i is the largest minus the smallest column index over the B rows
 * A(i,:) selects. */
msp_status msp_row_features(msp_handle* h, const msp_csr* A, const msp_csr* B,
                            int64_t* prod, float* features);

/* ---- learned output-size predictor -------------------------------------- */

/*
 * An FP32 multilayer perceptron 8 -> 64 -> 64 -> 1 (ReLU) that maps the 8
 * per-row inputs of msp_row_features to an estimate y of log2(1+row_nnz)/16.
 * Parameters are one flat array of 4801 floats:
 *     W1[64][8] b1[64] W2[64][64] b2[64] W3[64] b3[1]
 * (hidden unit h of layer 1 is relu(sum_f W1[h][f] x[f] + b1[h])).
 * The predictor is not part of the paper; it sizes the accumulators and the
 * output of msp_spgemm_learned.
 */
typedef struct msp_predictor msp_predictor;

typedef struct {
    float lr, beta1, beta2, eps;   /* Adam; 0 selects 1e-3, 0.9, 0.999, 1e-8 */
} msp_train_opts;

typedef struct {
    int64_t overflow_rows;   /* rows whose output outgrew their capacity and
                                were recomputed on the exact path           */
    int64_t sum_cap;         /* total predicted capacity (padded entries)   */
    int64_t nnz;             /* nnz(C)                                      */
    int64_t exact_rows;      /* rows whose capacity fell in the global bin,
                                sent to the exact path without a padded try;
                                all rows (and sum_cap 0) when the upper
                                bounds of those rows exceed the predicted
                                rows' total capacity, in which case the whole
                                product runs on the two-phase path          */
} msp_learned_stats;

/* Create on the handle's device from 4801 host floats (copied). */
msp_status msp_predictor_create(msp_handle* h, const float* init_params, msp_predictor** p);
msp_status msp_predictor_destroy(msp_predictor* p);
/* Copy the parameters to the host (params may be NULL) and the capacity
 * margin delta; set them from the host (params NULL keeps them). */
msp_status msp_predictor_get(msp_handle* h, const msp_predictor* p, float* params, float* delta);
msp_status msp_predictor_set(msp_handle* h, msp_predictor* p, const float* params, float delta);
/*
 * Checkpoint and restore of a predictor as a versioned byte blob of
 * MSP_PREDICTOR_BLOB_BYTES bytes (little-endian):
 *     offset 0   "MSPP"                       magic
 *            4   uint32 version (1)
 *            8   uint32 parameter count (4801)
 *           12   float  delta (capacity margin)
 *           16   int64  Adam steps taken
 *           24   float  parameters[4801]      (msp_predictor_create order)
 *                float  Adam first moments[4801]
 *                float  Adam second moments[4801]
 *       end - 8  uint64 FNV-1a hash of every byte before it
 * so that training can resume where it stopped.  msp_predictor_save
 * writes the blob into the caller's host buffer (cap bytes; *size, when not
 * NULL, receives the blob size; blob NULL only queries the size) after
 * copying the state from the device (synchronises).  msp_predictor_load
 * replaces p's state from a blob: a wrong magic, count, size or hash gives
 * MSP_ERR_INVALID_ARG, another version MSP_ERR_UNSUPPORTED, and p is left
 * unchanged on error.  The _pack / _unpack pair does the same on host
 * arrays only (any of adam_m, adam_v, delta, step may be NULL: packed as
 * zeros, or not returned) and needs no device.
 */
#define MSP_PREDICTOR_BLOB_BYTES 57644
msp_status msp_predictor_save(msp_handle* h, const msp_predictor* p, void* blob, size_t cap, size_t* size);
msp_status msp_predictor_load(msp_handle* h, msp_predictor* p, const void* blob, size_t size);
msp_status msp_predictor_blob_pack(const float* params, const float* adam_m, const float* adam_v, float delta,
                                   int64_t step, void* blob, size_t cap, size_t* size);
msp_status msp_predictor_blob_unpack(const void* blob, size_t size, float* params, float* adam_m, float* adam_v,
                                     float* delta, int64_t* step);
/* Train with Adam on the mean squared error, `steps` mini-batches of
 * `batch` rows: batch_idx (device, steps x batch int32) names rows of
 * feats (device, n x 8) and targets (device, n).  losses_host (steps
 * floats) receives each step's loss when not NULL.  Synchronises. */
msp_status msp_predictor_train(msp_handle* h, msp_predictor* p, const float* feats, const float* targets,
                               int64_t n, const int32_t* batch_idx, int steps, int batch,
                               const msp_train_opts* o, float* losses_host);
/* Gradient of the mean squared error on one batch at the current
 * parameters: idx (device, batch int32) names rows of feats (device, n x 8)
 * and targets (device, n); host outputs: 4801 floats and the loss.
 * Synchronises.  Indices outside [0, n) give MSP_ERR_INVALID_ARG (also in
 * msp_predictor_train, whose parameters are then already updated). */
msp_status msp_predictor_grad(msp_handle* h, msp_predictor* p, const float* feats, const float* targets,
                              int64_t n, const int32_t* idx, int batch, float* grad_host, float* loss_host);
/* Training rows of A*B: the 8 inputs of msp_row_features and the target
 * log2(1 + row_nnz_i) / 16 from the symbolic pass (device outputs, A.nrows
 * rows).  Synchronises. */
msp_status msp_training_rows(msp_handle* h, const msp_csr* A, const msp_csr* B, float* features,
                             float* targets);
/* y (device, n floats) = network output for feats (device, n x 8). */
msp_status msp_predictor_infer(msp_handle* h, const msp_predictor* p, const float* feats, int64_t n, float* y);
/* delta = the q-quantile of 16 (target - y) over the given rows. */
msp_status msp_predictor_calibrate(msp_handle* h, msp_predictor* p, const float* feats, const float* targets,
                                   int64_t n, double q);

/*
 * C = A * B in one pass: per-row capacities
 *     cap_i = clamp(ceil(2^(16 y_i + delta)), max_k nnz(B(k,:)), min(prod_i, n))
 * (when the margin delta alone lifts cap_i past the bound of the numeric
 * bin of the point prediction ceil(2^(16 y_i)), cap_i is that bound; rows
 * with min(prod_i, n) <= 32 take that bound without the network, and so does
 * every row whose bound falls in the same numeric bin as cap_i (same
 * kernel, no risk of overflow) or is at most 2 cap_i (at most twice the
 * room, no risk of overflow)), rows binned by capacity (a row whose
 * capacity falls in the global bin goes straight to the exact path, unless
 * opts->force_spill), numeric kernels writing into a padded buffer,
 * the rows that did not fit recomputed exactly (two-phase path on their
 * sub-matrix), and a compaction into tight CSR.  The result equals
 * msp_spgemm's (identical structure) for any predictor.  Two host reads in
 * the common case, four when rows overflow.  `st` may be NULL.
 */
msp_status msp_spgemm_learned(msp_handle* h, const msp_predictor* p, const msp_csr* A, const msp_csr* B,
                              msp_csr_out* C, const msp_opts* opts, msp_learned_stats* st);

/* ---- batches of products in one graph launch ----------------------------- */

/*
 * A batch of sparse matrices in packed form.  Problem p owns the rows
 * [row_start[p], row_start[p+1]) of one row_ptr array whose entries are
 * offsets into one col/val array (row_ptr[0] need not be 0); its column
 * indices are local to the problem, 0 <= col < ncols[p], sorted and unique
 * within each row.  row_start and ncols are host arrays (nprob + 1 and nprob
 * entries); row_ptr, col and val are device arrays.  A problem's view
 * {rows, ncols[p], nnz, row_ptr + row_start[p], col, val} is a valid
 * msp_csr for the single-product calls.
 */
typedef struct {
    int32_t nprob;
    const int64_t* row_start;   /* host, nprob + 1, row_start[0] = 0 */
    const int64_t* ncols;       /* host, nprob */
    int64_t nnz;                /* entries of col/val */
    const int64_t* row_ptr;     /* device, row_start[nprob] + 1 */
    const int32_t* col;         /* device */
    const void* val;            /* device */
    msp_dtype dtype;
} msp_batch_csr;

typedef struct msp_batch msp_batch;

typedef struct {
    int32_t nstage;             /* 1: C_p = A_p P_p; 2: C_p = R_p (A_p P_p)       */
    int64_t rows[2];            /* rows of each stage (all problems)            */
    int64_t nnz[2];             /* nnz of each stage's product at plan time     */
    int32_t sym_bins[2];        /* bin kernels of each stage's symbolic pass    */
    int32_t num_bins[2];        /* bin kernels of each stage's numeric pass     */
} msp_batch_stats;

/*
 * Plan a batch: C_p = A_p * P_p for every problem p, or, with R not NULL,
 * the Galerkin products C_p = R_p * (A_p * P_p) (two dependent stages, the
 * intermediate A_p P_p kept in the plan).  Shapes: A.ncols[p] = rows of
 * P_p; R.ncols[p] = rows of A_p.  Values of R, A and P have one dtype.
 * Runs the batch once eagerly to size the plan's workspace and output
 * arenas and to pick the bin kernels, then captures every pass of every
 * stage into one hipGraph on a private stream.  The inputs are borrowed:
 * each replay reads them again, so their values may change between
 * replays; their structure must not (a replay that detects a change
 * reports an error and produces nothing).  opts->tuning selects the bin
 * thresholds (zero: the handle's) and opts->queue_rows the work queue of
 * the numeric merge; validate and force_spill are not supported.
 * Synchronises.
 */
msp_status msp_batch_create(msp_handle* h, const msp_batch_csr* R, const msp_batch_csr* A,
                            const msp_batch_csr* P, const msp_opts* opts, msp_batch** plan);
msp_status msp_batch_destroy(msp_batch* plan);
/* Replay the plan's graph on the handle's stream (one graph launch and two
 * small device-to-host copies; no wait).  The results of the previous
 * replay are collected first. */
msp_status msp_batch_execute(msp_handle* h, msp_batch* plan);
/* Wait for the last replay; report a structure change or an internal error
 * it detected. */
msp_status msp_batch_sync(msp_handle* h, msp_batch* plan);
/* Problem p's result of the last replay as a canonical CSR view into the
 * plan's arena (valid until the next replay or msp_batch_destroy; the
 * caller does not free it).  Waits for the replay. */
msp_status msp_batch_result(msp_handle* h, msp_batch* plan, int p, msp_csr* C);
/* Problem p's result copied out: C->row_ptr as in msp_spgemm (caller's,
 * or allocated when NULL), col and val in one allocation from the handle's
 * allocator, owned by the caller.  Queued on the handle's stream. */
msp_status msp_batch_copy_result(msp_handle* h, msp_batch* plan, int p, msp_csr_out* C);
msp_status msp_batch_info(const msp_batch* plan, msp_batch_stats* st);
/*
 * Autotuner: plan the batch with each of the ncand tunings, replay it
 * `reps` times after one warm replay, and return in *best the tuning with
 * the smallest median replay time (times_ms, if not NULL, receives each
 * candidate's median, or infinity where the candidate failed).
 */
msp_status msp_batch_autotune(msp_handle* h, const msp_batch_csr* R, const msp_batch_csr* A,
                              const msp_batch_csr* P, const msp_tuning* cand, int ncand, int reps,
                              msp_tuning* best, double* times_ms);
/* A tuning as a flat JSON object of its fields; returns the length
 * written (snprintf semantics), or -1 when t is NULL.  When parsing, share_g
 * may be absent (the default). */
int msp_tuning_to_json(const msp_tuning* t, char* buf, size_t n);
/* Parse that object (field order and spacing free); checks the values as
 * msp_set_tuning does. */
msp_status msp_tuning_from_json(const char* json, msp_tuning* t);

/* ---- timing ------------------------------------------------------------- */

/* Phases timed with HIP events on the handle's stream when profiling is on. */
enum {
    MSP_PHASE_ROW_STATS = 0,   /* statistics + binning histogram          */
    MSP_PHASE_SYMBOLIC = 1,    /* scatter + symbolic kernels              */
    MSP_PHASE_SCAN = 2,        /* prefix sum + numeric binning histogram  */
    MSP_PHASE_NUMERIC = 3,     /* scatter + numeric kernels               */
    MSP_PHASE_PREDICT = 4,     /* predictor inference (learned form)      */
    MSP_PHASE_FALLBACK = 5,    /* exact fallback rows (learned form)      */
    MSP_PHASE_COMPACT = 6,     /* compaction (learned form)               */
    MSP_PHASE_BATCH = 7,       /* one batched graph launch                */
    MSP_PHASE_GLOBAL_BIN = 8,  /* the global bin's windowed numeric kernel
                                  (an interval inside MSP_PHASE_NUMERIC)   */
    MSP_NUM_PHASES = 9
};

typedef struct {
    double ms[MSP_NUM_PHASES];       /* accumulated event time per phase     */
    int64_t count[MSP_NUM_PHASES];   /* number of timed intervals per phase  */
} msp_profile;

/* Per-phase event timing: bit p of phase_mask times phase p (-1: every
 * phase, 0: off); either way the accumulators are reset.  Each timed
 * phase adds two event records to the stream. */
msp_status msp_profile_enable(msp_handle* h, int phase_mask);
/* Accumulated times of the intervals that have completed so far. */
msp_status msp_profile_get(msp_handle* h, msp_profile* out);

const char* msp_status_string(msp_status s);
const char* msp_last_error(void);
int msp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MSP_H */
