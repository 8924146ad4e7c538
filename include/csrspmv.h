/*
 * csrspmv — matrix-adaptive CSR sparse matrix-vector multiplication y = A x
 * for AMD Instinct MI355X (gfx950).
 *
 * The method is that of Elafrou, Goumas & Koziris, "Performance Analysis and
 * Optimization of Sparse Matrix-Vector Multiplication on Modern Multi- and
 * Many-Core Processors" (ICPP 2017): find the bottleneck classes of a matrix
 * (memory bandwidth MB, memory latency ML, thread imbalance IMB, computation
 * CMP; Sec. III-A), either by profiling micro-benchmarks against per-class
 * performance bounds (Sec. III-B/C) or from cheap structural features
 * (Sec. III-D), then apply the CSR-based remedies of the optimization pool
 * jointly (Sec. III-E, Table II). The API follows the paper's problem
 * statement: a square (or rectangular) matrix in CSR (Sec. II), FP64 values
 * (Sec. IV-A), y overwritten by A x (Sec. II, Fig. 2), the same A reused for
 * many products so that inspection and selection are paid once
 * (Sec. IV-D) — an inspector/executor split.
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device pointers (hipMalloc'ed or torch CUDA
 *     tensors); pointers named h_* or out are host pointers.
 *   - `stream` is a hipStream_t passed as void*; NULL means the legacy default
 *     stream of the current device.
 *   - The current HIP device when a handle is created is the device the
 *     handle lives on; later calls switch to it themselves.
 *   - Every call returns a csr_status_t; nothing is thrown or aborted across
 *     this boundary. csr_last_error() returns a message for the most recent
 *     failure on the calling thread.
 *   - A handle may be used from one stream at a time; calls on one handle are
 *     not thread-safe.
 */
#ifndef CSRSPMV_H
#define CSRSPMV_H

#ifndef __HIPCC_RTC__  /* the run-time kernel compiler defines these types itself */
#include <stddef.h>
#include <stdint.h>
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct csr_matrix_s *csr_matrix_t;

typedef enum {
    CSR_OK = 0,
    CSR_ERR_INVALID_ARG = 1,     /* bad argument: NULL, negative size, aliasing */
    CSR_ERR_INVALID_MATRIX = 2,  /* the CSR arrays violate the format */
    CSR_ERR_OUT_OF_MEMORY = 3,   /* a device or host allocation failed */
    CSR_ERR_DEVICE = 4,          /* a HIP runtime call failed */
    CSR_ERR_UNSUPPORTED = 5,     /* e.g. nnz > 2^31 - 4096, delta codes on unsorted rows */
    CSR_ERR_NOT_READY = 6        /* e.g. learned selection without loaded weights */
} csr_status_t;

/* Precision of the stored values (BASELINE precision sweep). FP64 storage
 * computes in FP64 with FP64 x and y. FP32 and BF16 storage accumulate in
 * FP32, with x and y in FP32 (x is rounded once by the caller). */
typedef enum { CSR_VAL_F64 = 0, CSR_VAL_F32 = 1, CSR_VAL_BF16 = 2 } csr_val_t;

/* Optimizations of the pool (Sec. III-E, Table II), combinable as a mask. */
enum {
    CSR_OPT_DELTA = 1,     /* MB:  delta-coded column indices (8 or 16 bit) + wide loads */
    CSR_OPT_PREFETCH = 2,  /* ML:  streamed val/col with the x gathers issued ahead */
    CSR_OPT_DECOMP = 4,    /* IMB: long rows split off and computed cooperatively */
    CSR_OPT_MERGE = 8,     /* IMB: nnz-balanced merge-path split */
    CSR_OPT_UNROLL = 16    /* CMP: unrolled independent accumulators, several rows per wave */
};

/* Bottleneck classes (Sec. III-A), as a mask. */
enum { CSR_CLS_MB = 1, CSR_CLS_ML = 2, CSR_CLS_IMB = 4, CSR_CLS_CMP = 8 };

/* Selection modes for csr_select. */
typedef enum {
    CSR_SEL_PLAIN = 0,       /* the baseline row-split kernel, no remedy */
    CSR_SEL_PROFILE = 1,     /* micro-benchmarks + the rule of Sec. III-C, Fig. 4 */
    CSR_SEL_LEARNED = 2,     /* features + the loaded MLP (falls back to PROFILE) */
    CSR_SEL_EXHAUSTIVE = 3,  /* time every catalogue variant, keep the fastest */
    CSR_SEL_FORCED = 4,      /* use cfg->forced_opts / cfg parameters as given */
    CSR_SEL_TREE = 5         /* features + the loaded decision tree (the paper's feature-guided
                                classifier): predicted classes -> Table II remedies (falls
                                back to PROFILE without a tree) */
} csr_sel_t;

/* Tunables; csr_config_default() fills the defaults. */
typedef struct {
    double t_ml;             /* ML threshold on P_ML / P_CSR (paper, on KNC: 1.25; default
                                1.0, from the grid search over the suite on MI355X) */
    double t_imb;            /* IMB threshold on P_IMB / P_CSR (paper, on KNC: 1.24;
                                default 1.0, from the same grid search) */
    double t_mb;             /* MB: P_CSR >= t_mb * P_MB reads "P_CSR ~ P_MB" (default 0.5,
                                from the same grid search) */
    double long_row_factor;  /* a row is long if nnz_i > max(factor*nnz_avg, long_row_floor) */
    int32_t long_row_floor;
    int32_t forced_opts;     /* CSR_SEL_FORCED: mask of CSR_OPT_* */
    int32_t rows_per_group;  /* 0 = auto: lanes per row G in {1,2,4,...,64} */
    int32_t merge_items;     /* 0 = auto (512): merge-path items per tile L, a multiple of 256
                                up to 2048 (256, 512 and 1024 prebuilt, the others compiled
                                at run time on first use) */
    int32_t autotune;        /* 1 = time a small parameter grid for the chosen remedies */
    int32_t timing_calls;    /* SpMV calls per timing run inside selection (default 32) */
    int32_t rows_in_flight;  /* 0 = auto: rows per lane group loaded at once (1, 2 or 4) */
    int32_t exhaustive_set;  /* CSR_SEL_EXHAUSTIVE: 0 = the 16-entry catalogue (the "trivial
                                combined" optimizer of Sec. IV-D), 1 = the baseline and the
                                5 single remedies ("trivial single") */
    int32_t dynamic_rows;    /* row-split plans: 0 = static schedule (one block of rows per
                                workgroup), 1 = dynamic chunks (resident workgroups take
                                blocks of rows from a counter); the autotuner also tries 1
                                for imbalanced matrices */
    int32_t ml_partitions;   /* PROFILE: 0 = the ML test of Fig. 4 on the whole matrix only;
                                Q in 1..4096 = also the partition-aware ML test (the
                                extension the paper proposes in Sec. IV-C): the instrumented
                                baseline and the instrumented P_ML probe are each run 3 times,
                                every row block keeps its shortest time, the row blocks are
                                cut into Q contiguous partitions of about nnz/Q nonzeros, and
                                ML is also set when some partition's summed baseline time
                                exceeds t_ml_part times its summed probe time */
    double t_ml_part;        /* partition-aware ML threshold (used when ml_partitions > 0) */
    int32_t jit_tiles;       /* 1 = the autotuner also tries merge tiles of 768 and 1536 items,
                                compiled at run time (merge_items also accepts any multiple of
                                256 up to 2048; sizes other than 256, 512 and 1024 are compiled
                                on first use) */
    int32_t window_runs;     /* 1 = window-coded merge plans replace the per-tile dictionary
                                by a 64-byte record of at most 14 runs of consecutive
                                columns when every tile's window fits one (the same bits;
                                0, the default, keeps the dictionary; the autotuner tries
                                both) */
    int32_t remedy_map;      /* classes -> optimizations: 0 = the paper's Table II (MB delta
                                codes, ML prefetch, IMB decomposition or merge path, CMP
                                unrolling); 1 (default) = as they pay on MI355X (measured over
                                the synthetic suite): MB delta codes, ML and IMB the merge
                                path with compressed codes (IMB: decomposition when long rows
                                exist), CMP nothing */
    int32_t split_row_blocks; /* 1 (default) = column blocks (x above one XCD's L2, rows
                                whose columns spread over it) also on merge tiles that are
                                not row-aligned: each block carries its split rows through
                                the fixup, and the blocks after the first walk only the rows
                                with nonzeros in them; 0 = only on row-aligned tiles. The
                                autotuner times both where they apply */
    double ood_z;            /* LEARNED: a matrix whose standardized features (log2(1 + f)
                                - mu) / sigma, with the loaded model's mu and sigma, reach
                                beyond ood_z in absolute value lies outside what the model
                                was trained on, and selection falls back to PROFILE (default
                                4.0: the 2,000 training-suite matrices stay below 3; 0 turns
                                the test off) */
} csr_config_t;

/* What csr_select decided and what it cost. */
typedef struct {
    int32_t opts;            /* CSR_OPT_* mask in use */
    int32_t classes;         /* CSR_CLS_* mask (PROFILE), -1 if not computed */
    int32_t variant_id;      /* index into the 16-entry catalogue, -1 if outside it */
    int32_t lanes_per_row;   /* G of the row-split kernels */
    int32_t merge_items;     /* L of the merge-path kernel */
    int32_t delta_bits;      /* 8, 16, or 32 (plain int32 indices) */
    int32_t n_long_rows;     /* rows taken out by the decomposition */
    int32_t fallback;        /* 1 if LEARNED had no model and used PROFILE */
    int32_t merge_slack;     /* > 0: merge tiles cut at row ends (cuts every L - slack items
                                moved to the end of the row in progress; no row spans two
                                tiles); 0: plain cuts every L items */
    int32_t window_codes;    /* 1: the merge path's column codes are window ranks (delta_bits
                                8): each row-aligned tile stores its distinct columns as
                                16-bit offsets from its smallest one, each nonzero the 8-bit
                                rank of its column among them; 2: the same ranks, with each
                                tile's distinct columns stored as at most 14 runs of
                                consecutive columns (a 64-byte record per tile); 3: 9-bit
                                ranks (delta_bits 9) on tiles of 1,024 items, windows of up
                                to 512 columns: the code is the rank's low byte, the ninth
                                bits sit in a 132-byte record per tile */
    int32_t column_blocks;   /* > 1: the merge path runs once per column slab of at most
                                2 MiB of x, each pass adding into y (merge plans without
                                codes, when x outgrows one XCD's L2, rows are short and
                                their columns spread over x) */
    int32_t dynamic_rows;    /* 1: the row-split kernel runs with dynamic chunks */
    int32_t ml_partitions;   /* non-empty partitions of the partition-aware ML test (0: off) */
    int32_t ml_parts_flagged;/* partitions whose time ratio exceeded t_ml_part */
    int32_t jit;             /* 1: the plan's merge kernel was compiled at run time */
    int32_t reserved;
    double p_csr, p_mb, p_ml, p_imb, p_cmp, p_peak;  /* flop/s (PROFILE) */
    double b_max;            /* B/s used for the bounds */
    double t_select_ms;      /* features/probes + decision */
    double t_prep_ms;        /* format conversion for the chosen plan */
    double format_bytes;     /* algorithmic bytes of one SpMV with this plan */
    double ml_part_max;      /* largest partition ratio of the partition-aware ML test */
    double feature_z_max;    /* LEARNED: the largest |standardized feature| the model saw
                                (compared with ood_z); 0 for the other modes */
} csr_plan_info_t;

/* The 16 features of Sec. III-D, Table I (plus two project-defined ones):
 * N, nnz_min, nnz_max, nnz_avg, nnz_sd, bw_min, bw_max, bw_avg, bw_sd,
 * scatter_avg, scatter_sd, clustering_avg, misses_avg, size, mean_col_gap,
 * x_reuse. isum holds the exact integer sums they come from: sum nnz,
 * sum nnz^2, sum bw, sum bw^2, sum misses, sum groups, x-reuse shared and
 * distinct line counts. */
typedef struct {
    double f[16];
    int64_t isum[8];
    int32_t rows_sorted;     /* 1 if every row is strictly increasing */
    int32_t reserved;
} csr_features_t;

/* Fill *cfg with the defaults (t_ml 1.0, t_imb 1.0, t_mb 0.5, remedy_map 1, split_row_blocks 1,
 * long_row_factor 32, long_row_floor 4096, autotune 1, timing_calls 32,
 * ml_partitions 0, t_ml_part 1.5, jit_tiles 0, ood_z 4.0). */
void csr_config_default(csr_config_t *cfg);

/*
 * Ingest (Sec. II: the CSR format). Copies the caller's CSR arrays into
 * device memory owned by the new handle, validates them on the device
 * (row_ptr[0] = 0, row_ptr non-decreasing, row_ptr[n_rows] = nnz,
 * 0 <= col_idx < n_cols), records whether every row is strictly increasing,
 * and converts the values to `storage` (FP32: IEEE round-to-nearest-even;
 * BF16: one round-to-nearest-even step from FP64).
 *   d_row_ptr  int32[n_rows + 1]   device
 *   d_col_idx  int32[nnz]          device
 *   d_val      double[nnz]         device
 * Synchronizes `stream` before returning, so the caller may free its arrays.
 * The plan starts as CSR_SEL_PLAIN. Errors: CSR_ERR_INVALID_ARG (NULL out,
 * negative sizes, NULL arrays with nnz > 0), CSR_ERR_UNSUPPORTED
 * (nnz > 2^31 - 4096: indices are int32 and loop indices step past the last
 * nonzero by up to a workgroup), CSR_ERR_INVALID_MATRIX (no handle is created),
 * CSR_ERR_OUT_OF_MEMORY, CSR_ERR_DEVICE. On error *out is NULL.
 */
csr_status_t csr_create(csr_matrix_t *out, int32_t n_rows, int32_t n_cols, int64_t nnz,
                        const int32_t *d_row_ptr, const int32_t *d_col_idx,
                        const double *d_val, int32_t storage, void *stream);

/* Frees everything the handle owns. NULL is accepted and ignored. */
void csr_destroy(csr_matrix_t A);

/*
 * Feature extraction (Sec. III-D, Table I): one pass over row_ptr and
 * col_idx on the device; integer sums are exact, the FP64 features are
 * formed from them on the host. Synchronizes `stream`.
 */
csr_status_t csr_inspect(csr_matrix_t A, csr_features_t *out, void *stream);

/*
 * Variant selection (Sec. III-C to III-E) and preprocessing of the chosen
 * plan (delta codes, merge-path tiles, long-row list). cfg may be NULL for
 * the defaults; out may be NULL. Synchronizes `stream`. PROFILE and
 * EXHAUSTIVE launch SpMV kernels that write into internal scratch vectors.
 * A matrix without rows keeps the plain plan whatever the mode (nothing is
 * inspected, timed or built).
 */
csr_status_t csr_select(csr_matrix_t A, int32_t mode, const csr_config_t *cfg,
                        csr_plan_info_t *out, void *stream);

/*
 * y = A x (Sec. II, Fig. 2) with the current plan. Asynchronous on `stream`.
 *   d_x  n_cols elements, d_y  n_rows elements, device; FP64 for FP64
 *   storage, FP32 for FP32/BF16 storage. x and y must not overlap
 *   (CSR_ERR_INVALID_ARG).
 */
csr_status_t csr_spmv(csr_matrix_t A, const void *d_x, void *d_y, void *stream);

/*
 * count independent products y_k = A_k x_k in one persistent launch.
 * Every handle must live on the current device and share one storage type.
 * h_A, h_x, h_y are host arrays of count handles / device pointers. The
 * first call for a given handle list builds a device work queue (cached);
 * asynchronous on `stream` after that.
 */
csr_status_t csr_spmv_batched(int32_t count, const csr_matrix_t *h_A,
                              const void *const *h_x, void *const *h_y, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): y = A x
 * for an FP64 CSR matrix given directly as device arrays, with no handle,
 * no allocation and no memset. It runs the kernel of csr_spmv's plain plan
 * with dynamic row chunks (the result is bit-identical to csr_spmv after
 * csr_select(CSR_SEL_FORCED, forced_opts = 0, dynamic_rows = 1)); the
 * chunk counters live in a 256-byte device array of the library, one per
 * GPU, held until the process ends and cleared by a kernel at the start of
 * every call.
 *   d_row_ptr int32[n_rows + 1], d_col_idx int32[nnz], d_val double[nnz],
 *   d_x double[n_cols], d_y double[n_rows]: device, owned by the caller.
 * The arrays must form a valid CSR matrix (what csr_create checks); this
 * call does not check them. Every input size csr_create accepts fits the
 * fixed array (it holds two counters whatever the size). Calls that overlap
 * on one GPU (e.g. on two streams) share the array and race: order them.
 * Asynchronous on `stream`. Errors: CSR_ERR_INVALID_ARG (negative sizes,
 * NULL arrays, x and y overlapping), CSR_ERR_UNSUPPORTED (nnz > 2^31 - 4096),
 * CSR_ERR_DEVICE.
 */
csr_status_t csr_spmv_noalloc(int32_t n_rows, int32_t n_cols, int64_t nnz,
                              const int32_t *d_row_ptr, const int32_t *d_col_idx,
                              const double *d_val, const double *d_x, double *d_y, void *stream);

/* Human-readable name of a status code (static storage); any int is
 * accepted ("CSR_ERR_UNKNOWN" outside the enumeration). */
const char *csr_status_str(int32_t s);

/* Message describing the most recent failure on the calling thread. */
const char *csr_last_error(void);

/* Basic facts about a handle. */
csr_status_t csr_query(csr_matrix_t A, int32_t *n_rows, int32_t *n_cols, int64_t *nnz,
                       int32_t *storage, int32_t *rows_sorted);

/*
 * Run-time specialization (the paper's just-in-time code generation,
 * Sec. IV-D): compiles the merge-path kernel for value storage `storage`,
 * tile size `merge_items` (a multiple of 256 from 256 to 2048), index mode
 * `index_mode` (0 int32 columns, 1 16-bit and 2 8-bit merge codes, 3 window
 * codes, 4 window codes with run records; 9-bit window ranks exist only on the
 * prebuilt 1,024-item tiles and are refused here), non-temporal loads (`streaming`, int32 columns only) and row-aligned
 * tiles (`row_aligned`; required by window codes) with hipRTC for gfx950, from
 * the kernel sources built into the library, and copies the code object (an
 * AMDGPU ELF) to host memory `code` of `bytes` bytes (*needed receives its
 * size; code = NULL only sizes it). Needs no GPU. Launches compile and load
 * their instances themselves; this entry point exists to inspect what they
 * run. CSR_ERR_INVALID_ARG for arguments outside these ranges,
 * CSR_ERR_UNSUPPORTED when codes of that width do not form whole loads at that
 * tile size or the compilation fails (the compiler log is in
 * csr_last_error()).
 */
csr_status_t csr_jit_compile(int32_t storage, int32_t merge_items, int32_t index_mode,
                             int32_t streaming, int32_t row_aligned, void *code, size_t bytes,
                             size_t *needed);

/*
 * Test support: copies an internal device array of the handle to host
 * memory so that encodings and partitions can be compared bit for bit.
 *   what: 0 stored values (nnz elements of the storage type),
 *         1 delta codes (nnz bytes or uint16), 2 merge tile rows int32[T+1],
 *         3 merge tile nonzero offsets int32[T+1], 4 long-row list int32[n],
 *         5 plan info (csr_plan_info_t), 6 merge codes (nnz uint8 or uint16:
 *         column - smallest column of the nonzero's merge tile), 7 merge tile
 *         bases int32[T] (the smallest column of each tile), 8 window
 *         dictionaries uint16[T][256] (the tile's distinct columns, ascending,
 *         minus its base; zero past the window; [T][512] with 9-bit ranks),
 *         9 window lengths int32[T] (9-bit ranks, on tiles of 1,024 items:
 *         records int32[T][33], the length, then 64 uint16 masks: lane l's
 *         bit it * v + e is the ninth rank bit of tile element
 *         it * 64 v + l v + e, v = 2 for FP64 values and 4 otherwise),
 *         10 window codes uint8[nnz] (rank of the column in its tile's window;
 *         its low byte with 9-bit ranks),
 *         11 column-block row pointers int32[B][n_rows + 1] (each from 0),
 *         12 column-block columns int32[nnz] and 13 values (storage type,
 *         nnz): the blocks' nonzeros one block after the other, rows in
 *         order, storage order inside a row; from the last PROFILE selection
 *         with ml_partitions = Q > 0: 14 partition bounds int32[Q+1] (first
 *         row block of each partition; a row block is the baseline's
 *         workgroup of 256/G rows), 15 per-block shortest times int64[2][nblk]
 *         (baseline, then P_ML probe; 100 MHz ticks), 16 partition ratios
 *         double[Q] (0 for a partition without blocks); from the last
 *         PROFILE selection: 17 P_IMB's busy span of every compute unit that
 *         ran work in the instrumented baseline int64[n_cu] (wall-clock
 *         ticks, by compute-unit id), 18 double[3]: the HBM and the cache
 *         triad bandwidth (B/s; B_max is the second when the plan's bytes
 *         fit in the 256 MB Infinity Cache) and the span clock (ticks/s);
 *         19 run-window records int32[T][16] (per tile: smallest column,
 *         window entries | runs << 16, then per run its first column minus
 *         the smallest | its length << 16, zero past the last run);
 *         column blocks on tiles that are not row-aligned, blocks 1 .. B-1
 *         one after the other: 20 the rows with nonzeros in the block,
 *         ascending, int32, and 21 their row pointers int32[n_b + 1] (each
 *         from 0)
 * Returns CSR_ERR_INVALID_ARG if `bytes` differs from the array's size
 * (*needed receives that size when non-NULL) or the array does not exist.
 * Synchronizes `stream`.
 */
csr_status_t csr_debug_copy(csr_matrix_t A, int32_t what, void *h_dst, size_t bytes,
                            size_t *needed, void *stream);

/*
 * Test support for the out-of-memory paths. Reports the device buffers the
 * library holds (*live_buffers, *live_bytes) and the device allocations it
 * attempted since the last arming (*attempts); any output may be NULL. With
 * arm != 0 it then re-arms the failure injector: counting attempts from 0
 * again, those numbered fail_from .. fail_from + fail_count - 1 fail with
 * CSR_ERR_OUT_OF_MEMORY without reaching hipMalloc (fail_count = 0: none
 * fail). Process-wide; not for use while other threads call the library.
 */
csr_status_t csr_debug_alloc(int32_t arm, int64_t fail_from, int64_t fail_count,
                             int64_t *live_buffers, int64_t *live_bytes, int64_t *attempts);

/*
 * Measurement support: `calls` back-to-back SpMVs with the current plan on
 * the caller's vectors (after one warm call), between two HIP events on
 * `stream`: *call_ms = their elapsed time / calls. *kernel_ms = the mean
 * duration of the plan's dominant kernel: for a plan that launches one
 * kernel per call the same figure as *call_ms (so it never exceeds it);
 * otherwise a second pass of `calls` calls with events recorded immediately
 * before and after the dominant kernel, averaged (this includes the
 * events' own overhead). kernel_name (may be NULL) receives the dominant
 * kernel's name as a kernel trace shows it, truncated to name_bytes.
 * Synchronizes.
 */
csr_status_t csr_time_spmv(csr_matrix_t A, const void *d_x, void *d_y, int32_t calls,
                           double *kernel_ms, double *call_ms, char *kernel_name,
                           size_t name_bytes, void *stream);

/*
 * Test support: runs one micro-benchmark of the profile-guided classifier
 * (Sec. III-B) on the caller's vectors so its arithmetic can be checked:
 *   which = 1  P_ML probe: the baseline kernel with every column index
 *              replaced by its own row index (clamped to n_cols - 1)
 *   which = 2  P_CMP probe: the baseline kernel without the column-index
 *              stream, reading x at the row index (clamped likewise)
 * Either way y_i = x_min(i, n_cols-1) * (sum of row i's values). Vector types
 * and ownership as for csr_spmv. Asynchronous on `stream`.
 */
csr_status_t csr_debug_probe(csr_matrix_t A, int32_t which, const void *d_x, void *d_y,
                             void *stream);

/*
 * B_max probe (Sec. III-B; Sec. IV-A, Table III: STREAM triad). Runs
 * a[i] = b[i] + s * c[i] over three FP64 arrays of `bytes_per_array` bytes
 * each (allocated and freed inside, non-temporal loads and stores) and
 * returns the sustained bandwidth in bytes/s counting 3 * bytes_per_array
 * per pass (best of `reps` passes).
 */
csr_status_t csr_triad(size_t bytes_per_array, int32_t reps, double *gbytes_per_s, void *stream);

/*
 * The profile-guided classifier on given bounds (Sec. III-C, Fig. 4) and the
 * remedies of the classes it finds (Sec. III-E, Table II), exactly as
 * csr_select(CSR_SEL_PROFILE) applies them: p[6] = {P_CSR, P_MB, P_ML,
 * P_IMB, P_CMP, P_peak} in flop/s (finite, > 0), the thresholds of cfg
 * (NULL: the defaults), has_long_rows != 0 when the matrix has rows longer
 * than the decomposition threshold. *classes receives the CSR_CLS_* mask,
 * *opts the CSR_OPT_* mask (before autotuning). Host only; used to tune the
 * thresholds by grid search over recorded bounds.
 */
csr_status_t csr_classify(const double *p, const csr_config_t *cfg, int32_t has_long_rows,
                          int32_t *classes, int32_t *opts);

/*
 * The two bandwidths PROFILE selection takes B_max from (Sec. III-B and its
 * footnote: B is raised for working sets that fit in the cache hierarchy),
 * measured on the current device on first use and cached for the process:
 * *hbm from the streaming triad over 3 x 1 GiB, *cache from a triad with
 * ordinary loads and stores over 3 x 48 MiB (inside the 256 MB Infinity
 * Cache), never below *hbm. Bytes/s. Synchronizes `stream`.
 */
csr_status_t csr_device_bandwidth(double *hbm, double *cache, void *stream);

/*
 * Test support: one pass of the B_max triad kernel on caller arrays,
 * d_a[i] = d_b[i] + scalar * d_c[i] as one fused multiply-add, i < n
 * (device arrays of n doubles, n even, 16-byte aligned; d_a must not
 * overlap d_b or d_c). streaming = 1: the non-temporal accesses of the HBM
 * probe, 0: ordinary ones (the cache probe). Asynchronous on `stream`.
 */
csr_status_t csr_debug_triad(double *d_a, const double *d_b, const double *d_c, int64_t n,
                             double scalar, int32_t streaming, void *stream);

/* ---------------------------------------------------------------------------
 * Learned selector (replaces the decision tree of Sec. III-D): an MLP
 * 16-64-64-K, ReLU, softmax over the K catalogue variants (K = 16: baseline,
 * 5 single optimizations, 10 pairs, in the order of csr_plan_info_t's
 * variant_id). Parameters are FP32, laid out W1[64][16], b1[64], W2[64][64],
 * b2[64], W3[K][64], b3[K] (6,288 floats for K = 16). Features are fed as
 * (log2(1 + f) - mu) / sigma.
 * ------------------------------------------------------------------------- */

/* Install a trained model for CSR_SEL_LEARNED on the current device (host
 * arrays: params, 16 mu, 16 sigma > 0; copied). Rejects non-finite values. */
csr_status_t csr_mlp_load(const float *h_params, int32_t K, const double *h_mu,
                          const double *h_sigma);
/* Remove the current device's model (LEARNED then falls back to PROFILE). */
csr_status_t csr_mlp_unload(void);
/* logits[B][K] = MLP(X[B][16]) for B <= 64 normalized rows (device arrays). */
csr_status_t csr_mlp_forward(const float *d_params, int32_t K, const float *d_X, int32_t B,
                             float *d_logits, void *stream);
/* Mean softmax cross-entropy of one batch and its gradient (same layout as
 * params) for B <= 64 rows with labels in [0, K) (device arrays). */
csr_status_t csr_mlp_grad(const float *d_params, int32_t K, const float *d_X,
                          const int32_t *d_labels, int32_t B, float *d_grad, float *d_loss,
                          void *stream);
/* `steps` Adam steps (Kingma & Ba 2015, bias-corrected, step counter
 * t0+1, t0+2, ...) on mini-batches of B rows; d_order holds steps*B row
 * indices into d_X / d_labels (the caller's shuffle). Updates d_params,
 * d_m, d_v in place; d_losses[steps] receives each batch's loss. One
 * workgroup, fixed summation order: bit-reproducible. Synchronizes. */
csr_status_t csr_mlp_train(float *d_params, float *d_m, float *d_v, int32_t K, const float *d_X,
                           const int32_t *d_labels, const int32_t *d_order, int32_t B,
                           int32_t steps, int32_t t0, float lr, float beta1, float beta2,
                           float eps, float *d_losses, void *stream);
/* d_out[n][16] = (log2(1 + d_f) - d_mu) / d_sigma (FP64 in, FP32 out). */
csr_status_t csr_mlp_normalize(const double *d_f, const double *d_mu, const double *d_sigma,
                               int64_t n, float *d_out, void *stream);

/* ---------------------------------------------------------------------------
 * Feature-guided classifier of Sec. III-D: a CART decision tree over the 16
 * features of csr_features_t that predicts the bottleneck classes the
 * profile-guided rule would assign (a CSR_CLS_* mask; 0 = the paper's dummy
 * class, nothing worth optimizing). Node k: feature[k] in [0, 16) with
 * children left[k], right[k] (both > k; go left when f[feature] <=
 * threshold[k]), or feature[k] = -1 for a leaf whose value[k] in [0, 16) is
 * the mask. The root is node 0. Host arrays, copied; one tree per process.
 * ------------------------------------------------------------------------- */
csr_status_t csr_tree_load(int32_t n_nodes, const int32_t *feature, const double *threshold,
                           const int32_t *left, const int32_t *right, const int32_t *value);
/* Remove the tree (TREE then falls back to PROFILE). */
csr_status_t csr_tree_unload(void);

#ifdef __cplusplus
}
#endif
#endif /* CSRSPMV_H */
