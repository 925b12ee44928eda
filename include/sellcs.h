/*
 * sellcs.h -- C ABI of the SELL-C-sigma sparse matrix-vector library for
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Kreutzer, Hager, Wellein, Fehske, Bishop, "A unified sparse matrix
 * data format for efficient general sparse matrix-vector multiply on modern
 * processors with wide SIMD units" (arXiv:1307.6209).
 *
 * Conventions for every entry point
 *   - Pointers named "device" refer to GPU memory of the current HIP device;
 *     "host" pointers refer to CPU memory. Sizes are element counts unless
 *     stated otherwise.
 *   - A stream argument is a hipStream_t passed as void*; NULL is the null
 *     stream. Calls documented as asynchronous only enqueue work on it.
 *   - Every call returns a sell_status. Nothing is printed and nothing is
 *     thrown across the ABI. On failure, sell_last_error() returns a
 *     thread-local message with the detail (for SELL_ERR_HIP: the HIP error
 *     string). Faults inside kernels surface at the caller's next
 *     synchronisation, as for any HIP call.
 *   - Index types: row pointers int64, column indices int32, chunk offsets
 *     int64, permutation and chunk widths int32. nrows and ncols must be
 *     below 2^31.
 */
#ifndef SELLCS_H
#define SELLCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SELL_OK = 0,
  SELL_ERR_INVALID_ARG = 1, /* null pointer, negative size, k < 1, ... */
  SELL_ERR_BAD_CRS = 2,     /* malformed CRS input (see sell_build) */
  SELL_ERR_OOM = 3,         /* device (or allocator callback) allocation failed */
  SELL_ERR_UNSUPPORTED = 4, /* C, dtype combination or size outside what the kernels take */
  SELL_ERR_HIP = 5          /* a HIP runtime call failed; text in sell_last_error() */
} sell_status;

typedef enum { SELL_F64 = 0, SELL_F32 = 1, SELL_BF16 = 2 } sell_dtype;

typedef struct sell_matrix *sell_handle;
typedef struct sell_batch_s *sell_batch;

/* Optional device allocator. alloc returns NULL on failure (reported as
 * SELL_ERR_OOM). When absent the library uses hipMalloc/hipFree. */
typedef struct {
  void *(*alloc)(size_t bytes, void *ctx);
  void (*free)(void *ptr, void *ctx);
  void *ctx;
} sell_allocator;

/* A general sparse matrix in CRS form (Sect. 3.1 of the paper): row i holds
 * val[rpt[i] .. rpt[i+1]-1] at columns col[rpt[i] .. rpt[i+1]-1]. All three
 * arrays are device pointers, borrowed for the duration of sell_build only.
 * Columns need not be sorted; repeated (row, column) pairs are kept as
 * separate terms. */
typedef struct {
  int64_t nrows, ncols, nnz;
  const int64_t *rpt; /* device, nrows + 1 */
  const int32_t *col; /* device, nnz */
  const double *val;  /* device, nnz */
} sell_crs;

/* Build options; a zeroed struct (or NULL) selects FP64 values, FP64
 * accumulation and automatic kernel parameters. */
typedef struct {
  sell_dtype val_dtype; /* storage of the matrix values: F64, F32 or BF16 */
  sell_dtype acc_dtype; /* accumulation and y: F64 or F32 (F64 values need F64) */
  int32_t unroll;       /* matrix slots in flight per lane: 0 auto (16 for the x-window
                           product with two or four slots per lane, else 8), or 4, 8
                           or 16 (16 applies to the x-window product with two or four
                           slots per lane; elsewhere it is taken as 8) */
  int32_t vec;          /* consecutive slots (rows) each lane loads at once: 0 auto
                           (2 for F64 values with >= 8 nonzeros per row on average,
                           and for F32/BF16 values when the x window is used; else
                           1), else 1, 2 or 4 (2 and 4 need C <= 64 and vec <= C) */
  int32_t seg_cols;     /* widest chunk one work unit covers, in chunk columns,
                           before the chunk is split across waves (rounded up to
                           a multiple of 64): 0 auto, < 0 never split */
  int32_t ktile;        /* right-hand sides per pass in sell_spmmv: 0 auto, else a
                           power of two <= 64. Auto with k = 16, 32 or 64
                           (C >= 16, X and Y aligned to 16 bytes) runs one
                           pass with 8 lanes per row (4 for k = 16), each
                           reading 4 or 8 right-hand sides */
  int32_t kmax;         /* largest k sell_spmmv will be called with on matrices
                           whose chunks are split (sizes the partial-sum buffer):
                           0 means 32 */
  int32_t permute_columns; /* 0: column ids stay the caller's (x, y in original
                           order). 1: columns are renumbered with the row order
                           too (square matrices only), i.e. the matrix stored is
                           P A P^T and x, y live in sorted order -- the form the
                           paper recommends for iterative solvers (Sect. 3.4);
                           see sell_permute / sell_unpermute */
  int32_t xwindow;      /* x window in LDS for sell_spmv: the distinct columns of
                           each group of G consecutive chunks (one workgroup, one
                           wave per chunk) are staged in LDS once and the slots
                           also store their 16-bit position in it (2 bytes
                           streamed instead of 4, x read from LDS; same result
                           bit for bit). 0: used when it fits and the matrix has
                           at least two groups of 4 chunks per compute unit (C in
                           8..64, vec 1 or 2 -- or 4 with FP32/BF16 values and
                           C >= 16 -- no split chunks, at most 8192
                           slots and 1024 runs of consecutive columns per group,
                           window <= 4 KiB times G); -1: never; 1: required
                           (SELL_ERR_UNSUPPORTED when it cannot be built, window
                           up to 16 KiB times G). The global column indices are
                           kept for sell_export, sell_spmmv and the batch. */
  const sell_allocator *alloc; /* NULL: hipMalloc/hipFree */
  int32_t xwindow_chunks; /* G, chunks per x-window group: 0 auto (8 at C = 32
                           when those windows fit and leave two groups per
                           compute unit, else 4), or 4 or 8 (that size only) */
  int32_t row_lengths;  /* 1: also keep the length of every row in sorted order
                           (4 bytes per row of the padded chunks), and sell_spmv
                           runs each row's lanes only to the row's own length --
                           the GPU form of the kernel that Sect. 3.4 describes:
                           the value and index loads of padding are skipped
                           (the plain kernel skips only their x gathers); same
                           result bit for bit (the padding still multiplies
                           zero by zero). The lanes of a short row still wait
                           for the chunk's longest one, so the gain is small:
                           a few per cent on low-beta layouts, none near
                           beta = 1. Needs C in 8..64 (SELL_ERR_UNSUPPORTED
                           otherwise). Used by the global-index sell_spmv only:
                           not by the x-window product (a layout with a window
                           runs that), sell_spmmv or the batch. 0: off. */
} sell_build_opts;

typedef struct {
  int64_t nrows, ncols, nnz;
  int32_t C;             /* chunk height */
  int64_t sigma;         /* sorting scope as requested */
  int64_t nchunks;       /* N_c = ceil(nrows / C) */
  int64_t padded;        /* stored slots cs[N_c] = sum_i C * cl[i] */
  double beta;           /* chunk occupancy nnz / padded (1 when padded == 0) */
  double zeta;           /* coefficient of variation of the row lengths */
  int64_t max_row_len;
  sell_dtype val_dtype, x_dtype, acc_dtype;
  int32_t lanes_per_row; /* lanes of one wavefront that share a row (64 / C, or 1) */
  int32_t unroll;        /* slots in flight per lane of the product that runs */
  int32_t vec;
  int32_t seg_cols;      /* split threshold in chunk columns */
  int64_t nunits;        /* work units of one sell_spmv launch */
  int64_t nsplit;        /* row slices whose chunk is split over several waves */
  int32_t has_perm;      /* 0 when the row order is the identity (sigma == 1) */
  int32_t permuted_columns; /* 1 when built with permute_columns */
  int64_t device_bytes;  /* device memory held by the handle */
  int32_t xwindow;       /* 1 when sell_spmv stages x windows in LDS */
  int32_t xwindow_max;   /* largest window, in x elements */
  int64_t xsegments;     /* runs of consecutive columns over all windows */
  int32_t xwindow_group_chunks; /* chunks that share one x window (a workgroup): 4 or 8; 0 without window */
  int32_t row_lengths;   /* 1 when built with row_lengths */
} sell_info_t;

/*
 * sell_build -- convert CRS to SELL-C-sigma on the device (Sects. 3.3, 3.4).
 *
 * Rows are sorted by descending length within windows of sigma consecutive
 * rows (ties keep the original order; sigma = 1 keeps the original order,
 * sigma >= nrows sorts globally). Rows are then grouped into chunks of C,
 * each chunk padded to its longest row (padding: value 0, column 0) and
 * stored column by column; chunk i starts at cs[i] and is cl[i] columns wide
 * (Eqs. (nc), (max); Listing "SELL-4-sigma spMVM kernel" for the layout
 * val[cs[i] + j*C + r]). Column indices stay the caller's, so x and y keep
 * the original numbering; y is written through the permutation.
 *
 * A:      CRS input, device arrays (borrowed).
 * C:      1, 2, 4, 8, 16, 32, 64 or 128; otherwise SELL_ERR_UNSUPPORTED.
 * sigma:  >= 1; otherwise SELL_ERR_INVALID_ARG.
 * opts:   NULL for defaults. Supported (val, acc) pairs: (F64, F64),
 *         (F32, F32), (F32, F64), (BF16, F32), (BF16, F64); x is F64 for F64
 *         values and F32 otherwise. Values are rounded to nearest-even.
 * stream: all device work runs on it; the call synchronises it once to read
 *         the padded size and the validation flags.
 * out:    receives the new handle; it owns every device array it holds.
 * Errors: SELL_ERR_BAD_CRS when rpt[0] != 0, rpt decreases, rpt[nrows] !=
 *         nnz, a row is longer than 2^31 - 1, or a column lies outside
 *         [0, ncols). SELL_ERR_OOM on allocation failure. No handle is
 *         returned on failure.
 */
sell_status sell_build(const sell_crs *A, int32_t C, int64_t sigma,
                       const sell_build_opts *opts, void *stream,
                       sell_handle *out);

/*
 * sell_spmv -- y = A x (Sect. 3.3, Listing "SELL-4-sigma spMVM kernel"),
 * asynchronous on stream.
 *
 * x: device, ncols elements of the handle's x dtype (F64 or F32).
 * y: device, nrows elements of the accumulation dtype; fully overwritten,
 *    never read. x must not overlap y.
 * Padding slots (value 0, column 0) either multiply x[0] by zero or, on
 * padding-heavy layouts (beta < 0.9), skip their gather -- as do explicit
 * zero entries there -- so x must be finite.
 * Calls on one handle must not overlap in time (they share the handle's
 * partial-sum buffer for split chunks): order them on one stream or
 * synchronise between streams.
 * The call only enqueues kernels (no allocation, copy, memset or
 * synchronisation), so it may be captured into a HIP graph.
 */
sell_status sell_spmv(sell_handle h, const void *x, void *y, void *stream);

/*
 * sell_spmmv -- Y = A X for k right-hand sides at once, asynchronous.
 * (Block form; the paper treats k = 1 only. Column v of Y is mathematically
 * sell_spmv applied to column v of X; the summation order differs, so the
 * two agree within rounding, each within the FP64 bound of the oracle.)
 * FP64 handles only. Each row's products are added in column order; the
 * kernel (pass width, lanes per row) follows the ktile build option.
 *
 * X: device, row-major ncols x k (X[c*k + v]); Y: device, row-major
 * nrows x k, fully overwritten. k >= 1; on handles with split chunks k must
 * not exceed the kmax given at build. Same overlap rule as sell_spmv.
 * X must be finite: for k > 1 every slot holding value 0 -- padding and
 * explicit zero entries alike -- skips its gather of X, so an Inf or NaN in
 * a row of X that only zero slots name does not reach Y (0 * Inf would give
 * NaN); k = 1 follows sell_spmv.
 */
sell_status sell_spmmv(sell_handle h, const void *X, void *Y, int32_t k,
                       void *stream);

/*
 * sell_spmmv_noalloc -- sell_spmmv for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and the same result bit for bit, but
 * the segment sums of split chunks go to a statically allocated scratch
 * array of 64 MiB per device (held until the process ends) instead of the
 * handle's buffer, so k is not limited by the kmax given at build. The call
 * allocates nothing and calls no allocating routine; the first call on a
 * device looks up that device's address of the array.
 *
 * Arguments, layouts, ownership and the finite-X precondition as in
 * sell_spmmv (k = 1 runs the sell_spmv kernels). The handle's device must be
 * the current device (else SELL_ERR_INVALID_ARG). SELL_ERR_UNSUPPORTED,
 * naming the bytes needed, when the segment sums exceed the 64 MiB: for a
 * handle with split chunks they take (rows of split slices) x k doubles
 * (pass kernel: k rounded up to its pass width); handles without split
 * chunks use no scratch. Every call on one device shares that device's
 * array and leaves its contents there (nothing in it needs clearing: each
 * call writes every sum before reading it), so calls that overlap in time
 * on one device -- on different streams, or from different threads -- race
 * and must be serialised by the caller.
 */
sell_status sell_spmmv_noalloc(sell_handle h, const void *X, void *Y, int32_t k,
                               void *stream);

/* sell_info -- host copy of the handle's sizes and parameters. */
sell_status sell_info(sell_handle h, sell_info_t *info);

/*
 * sell_export -- copy the device arrays to host buffers (synchronous).
 * perm: nrows int32 (perm[p] = original row at sorted position p; identity
 * when sigma == 1); cl: nchunks int32; cs: nchunks + 1 int64; col: padded
 * int32; val: padded elements of the value dtype (bfloat16 as raw uint16).
 * Any pointer may be NULL to skip that array.
 */
sell_status sell_export(sell_handle h, int32_t *perm, int32_t *cl, int64_t *cs,
                        int32_t *col, void *val);

/*
 * sell_export_xwindow -- copy the x-window tables of a handle built with the
 * x window (sell_info_t.xwindow == 1) to host buffers (synchronous). Group g
 * is chunks g*G .. g*G+G-1 (G = xwindow_group_chunks, the last group may be
 * short); its window is the sorted list of the distinct column indices its
 * slots hold (padding slots hold column 0), stored as runs of consecutive
 * columns.
 *   segoff: ngroups + 1 int64, ngroups = ceil(nchunks / G); the runs of group
 *           g are segoff[g] .. segoff[g+1]-1.
 *   seg:    3 * xsegments int32; run s is (first column, window position of
 *           that column, length).
 *   lcol:   padded uint16; the window position of the column of every slot
 *           (slot order of sell_export's col).
 * Any pointer may be NULL to skip that array. Errors: SELL_ERR_INVALID_ARG
 * for a null handle, SELL_ERR_UNSUPPORTED when the handle has no x window.
 * (An inspection call: the window is an addition of this library to the
 * paper's layout, Sect. 3.3, which the paper's format does not hold.)
 */
sell_status sell_export_xwindow(sell_handle h, int64_t *segoff, int32_t *seg, uint16_t *lcol);

/* sell_destroy -- release the handle and its device memory (synchronises
 * the device first). NULL is accepted. */
sell_status sell_destroy(sell_handle h);

/*
 * sell_batch_create -- prepare one launch that multiplies count matrices
 * with their own vectors. All handles must share C and dtypes; they are
 * borrowed and must outlive the batch. The work units of all matrices
 * (chunk row slices, long chunks split into segments, the segments first)
 * are concatenated, one wavefront per unit, and the launch is captured once
 * in a hipGraph.
 */
sell_status sell_batch_create(const sell_handle *hs, int32_t count,
                              sell_batch *out);

/*
 * sell_batch_create_persistent -- the same batch as one persistent launch:
 * the grid is the number of wavefronts the device holds at once, and each
 * wavefront runs a list of units back to back: the units placed on an XCD
 * are dealt, in order, to that XCD's wavefronts, each to the one with the
 * least estimated cost so far (wave steps plus a fixed charge per unit). Same
 * arguments, ownership, errors and results as sell_batch_create; use it with
 * sell_batch_spmv and sell_batch_destroy. (One wavefront per unit, the
 * sell_batch_create form, measured faster on uneven power-law batches: the
 * hardware dispatcher balances better than the static estimate.)
 */
sell_status sell_batch_create_persistent(const sell_handle *hs, int32_t count,
                                         sell_batch *out);

/*
 * sell_batch_spmv -- ys[b] = A_b xs[b] for every matrix of the batch, as one
 * graph launch on stream (asynchronous). xs and ys are host arrays of count
 * device pointers (x and y dtypes of the handles; each ys[b] fully
 * overwritten, no xs[b] may overlap a ys[c]). When they differ from the
 * previous call, the device copy of the pointer table is rewritten first,
 * after a device-wide synchronisation (earlier launches of the batch may
 * still read it); with unchanged pointers the call only launches the graph.
 * Calls on one batch must not overlap in time (they share the pointer table
 * and the partial-sum buffer of split chunks).
 */
sell_status sell_batch_spmv(sell_batch b, const void *const *xs,
                            void *const *ys, void *stream);

sell_status sell_batch_destroy(sell_batch b);

/*
 * sell_permute -- xp[p] = x[perm[p]] for p < nrows: a vector in the caller's
 * order to sorted order (square handles; x dtype of the handle).
 * sell_unpermute -- y[perm[p]] = yp[p]: back to the caller's order
 * (accumulation dtype). Both asynchronous on stream; in and out must not
 * overlap. With permute_columns, sell_spmv maps a sorted-order x to a
 * sorted-order y, so a solver can stay in sorted order and convert once.
 */
sell_status sell_permute(sell_handle h, const void *x, void *xp, void *stream);
sell_status sell_unpermute(sell_handle h, const void *yp, void *y, void *stream);

/*
 * sell_crs_spmv -- y = A x straight from CRS (Sect. 3.1, Listing "CRS spMVM
 * kernel"; y is overwritten), FP64, for comparison with SELL-C-sigma on the
 * same device (Sects. 3.2, 5.1). lanes_per_row: 1 = one lane per row (scalar
 * CRS), 2..64 = that many lanes walk a row and add their sums across lanes,
 * 0 = chosen from the mean row length. The CRS arrays are not validated (use
 * sell_build for that). Asynchronous on stream.
 */
sell_status sell_crs_spmv(const sell_crs *A, int32_t lanes_per_row, const double *x,
                          double *y, void *stream);

/* Autotuner search space (zero-length lists fall back to defaults). */
typedef struct {
  const int32_t *C;       int32_t nC;       /* chunk heights */
  const int64_t *sigma;   int32_t nsigma;   /* sorting scopes */
  const int32_t *unroll;  int32_t nunroll;  /* default 4, 8, 16 (16: x-window builds with
                                               two slots per lane only) */
  const int32_t *ktile;   int32_t nktile;   /* used when k > 1 */
  const int32_t *vec;     int32_t nvec;     /* slots per lane (0 = default); with C this sets
                                               the lanes per row, 64 * vec / C */
  const int32_t *seg_cols; int32_t nseg_cols; /* split width of long chunks (0 = automatic):
                                               how many waves share a long row */
  sell_dtype val_dtype, acc_dtype;
  int32_t reps;           /* timed repetitions per candidate (0: 20) */
  int32_t model_guided;   /* 0: time every (C, sigma). K > 0: rank all (C, sigma) by
                             the bytes the code-balance model (Sect. 4, ideal alpha)
                             assigns one product, from a layout-only build (row
                             order, chunk widths; no values), and time only the K
                             best */
  const int32_t *xwindow; int32_t nxwindow; /* x path: the xwindow build option (0 = LDS
                                               window when it fits, -1 = L2 gathers) */
  const int32_t *xwindow_chunks; int32_t nxwindow_chunks; /* waves per workgroup of the window
                                               product: the xwindow_chunks build option
                                               (0 = automatic, 4, 8); NULL/0: {0} */
  const int32_t *row_lengths; int32_t nrow_lengths; /* the row_lengths build option (0, 1);
                                               1 is skipped for C outside 8..64 and where
                                               the layout runs the x-window product;
                                               NULL/0: {0} */
} sell_tune_space;

typedef struct {
  int32_t C;
  int64_t sigma;
  int32_t unroll;
  int32_t ktile;
  int32_t vec;
  int32_t seg_cols;
  double gflops;        /* useful 2 * nnz * k flops per second / 1e9 */
  double us_per_call;
  double beta;
  int32_t candidates;   /* configurations measured */
  int32_t predicted;    /* configurations ranked by the model (model_guided > 0) */
  int32_t xwindow;      /* 1 when the fastest product staged x windows in LDS */
  int32_t xwindow_chunks; /* its chunks (waves) per window workgroup; 0 without window */
  int32_t row_lengths;  /* 1 when the fastest product stopped its lanes at their rows' ends */
} sell_tuned;

/*
 * sell_autotune -- build and time every configuration of the search space on
 * A (device CRS, borrowed) with k right-hand sides and return the fastest by
 * useful GF/s. Synchronous on stream; uses temporary device memory.
 */
sell_status sell_autotune(const sell_crs *A, int32_t k,
                          const sell_tune_space *space, void *stream,
                          sell_tuned *best);

/* Result of sell_batch_autotune. */
typedef struct {
  int32_t C;            /* chunk height of the fastest batch */
  int32_t candidates;   /* batches timed (one per C that every matrix supports) */
  double gflops;        /* useful GF/s of the batch: 2 * (sum of nnz) / time */
  double us_per_call;   /* one batched launch (sell_batch_create form) */
} sell_batch_tuned;

/*
 * sell_batch_autotune -- choose one chunk height for a batch of count
 * matrices (As: host array of device CRS descriptions, borrowed) and a
 * sigma for each matrix. For every C of space->C (default 16, 32, 64) each
 * matrix takes the sigma of space->sigma (default 1, 1024 and one window
 * over all rows) whose layout moves the fewest bytes under the code-balance
 * model (Sect. 4, alpha at its ideal value: padded matrix plus the
 * permutation read when sigma > 1), found by layout-only builds; the batch of
 * those matrices is then built, launched reps times (space->reps, default 20)
 * and timed. Uses space->val_dtype and space->acc_dtype; the other fields of
 * space are ignored. *best receives the fastest C and sigma_out (host,
 * count entries) the sigma each matrix had in that batch. Synchronous on
 * stream; temporary device memory for the vectors and the trial builds.
 * Errors: SELL_ERR_INVALID_ARG for null arguments or count < 1; the errors
 * of sell_build for a malformed matrix; SELL_ERR_UNSUPPORTED when no C of the
 * space suits every matrix.
 */
sell_status sell_batch_autotune(const sell_crs *As, int32_t count,
                                const sell_tune_space *space, void *stream,
                                sell_batch_tuned *best, int64_t *sigma_out);

/*
 * sell_probe_bandwidth -- achievable device memory bandwidth b of the
 * roofline model (Sect. 2.1): kind 0 streams bytes through a read-only sum
 * (the "reduction" benchmark), kind 1 copies bytes/2 to another bytes/2
 * buffer (the "copy" benchmark; no write-allocate factor on this device).
 * kind 2 is the random-gather rate: 2^27 loads of 8 bytes at hashed
 * positions of an array of the largest power-of-two size <= bytes (the
 * x-vector accesses of a matrix without column locality); *gbs is then
 * 8 bytes x gathers / time, so gathers per second = *gbs / 8 x 1e9.
 * kinds 3, 4, 5 are the random-row rate of the block form (sell_spmmv reads
 * the k right-hand sides of a column as one row of 8k bytes): rows of 128,
 * 256 or 512 bytes (k = 16, 32, 64) at hashed row positions of an array of
 * the largest power-of-two row count that fits in bytes, 16 bytes per lane;
 * *gbs is then row bytes x rows / time (rows per second = *gbs / row bytes
 * x 1e9). kind 6 writes bytes with 16-byte non-temporal stores (the store
 * kind of the products' results): the write-only rate. kinds 7, 8, 9 mix
 * both as the block form does: P rows of 128, 256 or 512 bytes are written
 * in order (non-temporal), each the sum of four rows read at hashed row
 * positions of an input of P rows (P the largest power of two with
 * P x row bytes <= bytes; a second buffer of bytes holds the output); *gbs
 * is then 5 x P x row bytes / time.
 * Runs reps timed passes after one warm-up on stream; *gbs receives the mean
 * bandwidth in GB/s (1e9 bytes). Allocates and frees its own buffers.
 * Errors: SELL_ERR_INVALID_ARG for kind outside 0..9, reps < 1 or bytes
 * below 1 MiB; SELL_ERR_OOM when the buffers cannot be allocated.
 */
sell_status sell_probe_bandwidth(int32_t kind, size_t bytes, int32_t reps,
                                 void *stream, double *gbs);

const char *sell_status_string(sell_status s);
const char *sell_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SELLCS_H */
