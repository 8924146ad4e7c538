// Internal declarations shared by the HIP sources of libcsrspmv.
// Not installed; the public interface is include/csrspmv.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "csrspmv.h"
#include "kdefs.h"

namespace csr {

constexpr int kWave = 64;
constexpr int kMaxResidentGroups = 256 * 8;  // 256-thread workgroups resident at once (256 CUs)
constexpr size_t kPadBytes = 64;  // tail padding of val/col: vector loads may read past nnz

// Error plumbing -------------------------------------------------------------
void set_error(const std::string &msg);
csr_status_t fail(csr_status_t s, const std::string &msg);
csr_status_t hip_fail(hipError_t e, const char *what);

#define CSR_HIP(call)                                                  \
    do {                                                               \
        hipError_t _e = (call);                                        \
        if (_e != hipSuccess) return ::csr::hip_fail(_e, #call);       \
    } while (0)

// Device memory owned by a handle (freed in the destructor).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release();
    csr_status_t alloc(size_t n);
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Pinned host memory owned by a handle (freed in the destructor): staging
// for small device-to-host reads that are waited on at once.
struct HostBuf {
    void *p = nullptr;
    size_t bytes = 0;
    HostBuf() = default;
    HostBuf(const HostBuf &) = delete;
    HostBuf &operator=(const HostBuf &) = delete;
    ~HostBuf() {
        if (p) (void)hipHostFree(p);
    }
    csr_status_t alloc(size_t n);
};

// Grid shape of a static-partition launch: `nblk` logical workgroups, padded to
// a multiple of 8 so that logical block l = (b % 8) * per_xcd + b / 8 gives
// every XCD one contiguous range of logical blocks (workgroups are dispatched
// to the XCDs round-robin).
struct XcdGrid {
    int64_t nblk = 0;     // logical blocks that carry work
    int64_t per_xcd = 0;  // ceil(nblk / 8)
    int64_t launched = 0; // 8 * per_xcd
};
XcdGrid xcd_grid(int64_t nblk);


// Execution plan of one handle -------------------------------------------------
struct Plan {
    int32_t opts = 0;        // CSR_OPT_* mask
    int32_t G = 1;           // lanes per row (row-split kernels)
    int32_t U = 1;           // independent accumulators per lane
    int32_t R = 1;           // rows per lane group in flight at once
    int32_t probe = 0;       // 1: P_CMP micro-benchmark (no column stream, x[row])
    int32_t L = 0;           // merge-path items per tile
    int32_t idx = IDX_I32;   // index encoding
    int32_t nt = 0;          // non-temporal val/col stream
    int32_t jit = 0;         // merge kernel compiled at run time (tile size not prebuilt)
    int32_t long_rows = 0;   // decomposition active
    int32_t cblocks = 0;     // column blocks of the merge path (0: one pass over all columns)
    int32_t dyn = 0;         // row-split: dynamic chunks instead of the static schedule
    int32_t variant_id = 0;
};

}  // namespace csr

struct csr_matrix_s {
    uint64_t id = 0;               // unique per handle (process lifetime)
    uint64_t version = 0;          // incremented by every csr_select
    int device = 0;
    int32_t n_rows = 0, n_cols = 0;
    int32_t max_row_nnz = 0;  // longest row (from validation)
    int64_t nnz = 0;
    int32_t storage = CSR_VAL_F64;
    int32_t rows_sorted = 0;
    csr::DevBuf rp, col, val;      // CSR arrays (values in storage precision)
    csr::DevBuf codes;             // delta codes (uint8 or uint16)
    int32_t code_bits = 32;        // 8 / 16 when `codes` holds a valid encoding
    csr::DevBuf tile_i, tile_j;    // merge-path tile table, T+1 entries each
    csr::DevBuf tile_base;         // merge codes: smallest column of each tile, T entries
    csr::DevBuf mcodes;            // merge codes: per-nonzero offset from its tile's base
    int32_t mcode_bits = 0;        // 8 / 16 when mcodes is valid, 32 = not eligible, 0 = not built
    int32_t mcodes_L = 0;          // tile size the merge codes were built for
    int32_t mcodes_encoded = 0;    // mcodes holds the codes (not only the bases and width)
    csr::DevBuf wdict;             // window codes: per tile kWindowMax (9-bit ranks:
                                   // kWideWindowMax) uint16 column offsets
    csr::DevBuf wlen;              // window codes: window entries of each tile, T int32
    csr::DevBuf wcodes;            // window codes: per-nonzero rank in its tile's window
                                   // (uint8; 9-bit ranks: the low byte)
    int32_t wcode_state = 0;       // 1 valid, -1 not eligible, 0 not built
    int32_t wcode_wide = 0;        // 1: 9-bit ranks (IDX_W9): dictionaries of kWideWindowMax
                                   // entries, wlen holds kWideWords-word records
    int32_t wcodes_L = 0;          // tile size the window codes were built for
    csr::DevBuf wruns;             // run windows: per tile kRunWords int32 (IDX_R8)
    int32_t wruns_state = 0;       // 1 valid, -1 not eligible, 0 not built
    int32_t wruns_L = 0;           // tile size the run windows were built for
    int64_t wdict_entries = 0;     // sum of the window lengths
    // column blocks (ML remedy on the merge path): cb_B slabs of cb_width columns
    int32_t cb_B = 0;              // 0: not built
    int32_t cb_width = 0;
    int32_t cb_L = 0;              // tile size of their tile tables
    csr::DevBuf cb_rp;             // cb_B x (n_rows + 1) row pointers, each from 0
    csr::DevBuf cb_col, cb_val;    // the blocks' nonzeros, one block after the other (+ padding)
    csr::DevBuf cb_tile_i, cb_tile_j;   // per block T_b + 1 entries, one block after the other
    std::vector<int64_t> cb_nnz_off;    // cb_B + 1: first nonzero of each block
    std::vector<int64_t> cb_tile_off;   // cb_B + 1: first tile-table entry of each block
    std::vector<int64_t> cb_tiles;      // T_b
    // tiles that are not row-aligned: blocks b >= 1 run over the rows with
    // nonzeros in them (block 0 over every row, so that it writes all of y)
    int32_t cb_split = 0;
    csr::DevBuf cb_rid;                 // those rows, block after block
    csr::DevBuf cb_rrp;                 // their row pointers (n_b + 1 each, from 0)
    std::vector<int64_t> cb_rows;       // n_b (block 0: n_rows)
    std::vector<int64_t> cb_rid_off;    // first row-list entry of each block (block 0: unused)
    std::vector<int64_t> cb_rrp_off;    // first row pointer of each block (block 0: unused)
    csr::DevBuf carry;             // per-tile carry of the merge-path kernel
    int64_t n_tiles = 0;
    int32_t tiles_L = 0;
    int64_t tiles_slack = 0;   // row-aligned tiles when > 0 (no cross-tile rows)
    int32_t tiles_fixup = 1;   // the cross-tile fixup has work for this tile table
    csr::DevBuf long_list;         // decomposition: long rows (ascending)
    csr::DevBuf long_chunks;       // decomposition: (begin, end) nonzero range per chunk
    csr::DevBuf long_row_chunk;    // decomposition: first chunk of each long row, n_long+1
    csr::DevBuf long_part;         // decomposition: per-chunk partial sums
    int32_t n_long = 0;
    int64_t long_tau = -1;         // threshold the current list was built for
    int64_t n_long_chunks = 0;
    csr::Plan plan;
    csr_config_t plan_cfg{};       // the configuration `plan` was realized with
    csr_plan_info_t info{};
    int has_features = 0;
    csr_features_t feat{};
    csr::DevBuf scratch_x, scratch_y, scratch_col;  // selection probes
    // P_IMB of the last PROFILE selection: busy span of every compute unit
    // that ran work in the instrumented baseline (wall-clock ticks, by CU id),
    // the tick rate, and the device's two triad bandwidths
    std::vector<int64_t> imb_spans;
    double imb_clock_hz = 0.0;
    double bw_hbm = 0.0, bw_cache = 0.0;
    std::vector<int32_t> mlp_bounds;  // partition-aware ML test of the last PROFILE selection
    std::vector<int64_t> mlp_times;
    std::vector<double> mlp_ratios;
    csr::DevBuf dyn_ctr;           // the row-split dynamic schedule's two counters (zeroed once)
    csr::DevBuf feat_parts, feat_reuse, feat_long;  // feature-extraction partials, long rows
    csr::DevBuf feat_bits;         // one bit per row: the rows the sweep left to the long pass
    csr::HostBuf feat_host;        // pinned copy of feat_reuse (the sweep's results)
    double t_inspect_ms = 0.0;
};

namespace csr {

// Launchers (device code lives in the k_*.hip files) ----------------------------
hipError_t launch_validate(const int32_t *rp, const int32_t *col, int32_t n_rows,
                           int32_t n_cols, int64_t nnz, int32_t *d_flags, hipStream_t s);
hipError_t launch_delta_encode(const int32_t *rp, const int32_t *col, int32_t n_rows, int bits,
                               void *codes, int32_t *d_flags, hipStream_t s);
// arr = {rp, col, codes, val, x, y, instrumentation records (probe 2),
//        dynamic-schedule counters (nullptr: static)}
hipError_t launch_rowsplit_s0(int G, int idx, bool nt, int U, int R, int probe,
                              const void *const *arr, int32_t skip_above, int32_t n_rows,
                              int32_t n_cols, hipStream_t s);
hipError_t launch_rowsplit_s1(int G, int idx, bool nt, int U, int R, int probe,
                              const void *const *arr, int32_t skip_above, int32_t n_rows,
                              int32_t n_cols, hipStream_t s);
hipError_t launch_rowsplit_s2(int G, int idx, bool nt, int U, int R, int probe,
                              const void *const *arr, int32_t skip_above, int32_t n_rows,
                              int32_t n_cols, hipStream_t s);
hipError_t launch_merge_partition(const int32_t *rp, int32_t n_rows, int64_t nnz, int64_t L,
                                  int64_t slack, int64_t n_tiles, int32_t *tile_i, int32_t *tile_j,
                                  hipStream_t s);
// Merge codes: base[t] = smallest column of tile t, *max_range = largest
// (max - min) column range over the tiles; then codes[j] = col[j] - base[t].
hipError_t launch_merge_tile_range(const int32_t *col, const int32_t *tile_j, int64_t n_tiles,
                                   int32_t *base, int32_t *max_range, hipStream_t s);
hipError_t launch_merge_encode(const int32_t *col, const int32_t *tile_j, int64_t n_tiles,
                               const int32_t *base, int bits, void *codes, hipStream_t s);
// Window codes: dict[t * kWindowMax + k] = k-th distinct column of tile t -
// base[t], wlen[t] = distinct columns, codes[j] = rank of col[j]; *max_m =
// the largest window (tiles over kWindowMax write nothing). Every tile's
// column range must be below 2^16.
// Run windows: rec[t * kRunWords ...] = tile t's window (dict, wlen, base)
// as runs of consecutive columns; *max_runs = the most runs of any tile
// (records of tiles over kRunsMax hold their first kRunsMax runs).
hipError_t launch_window_runs(const uint16_t *dict, const int32_t *wlen, const int32_t *base,
                              int64_t n_tiles, int32_t *rec, int32_t *max_runs, hipStream_t s);
// wide_vec > 0: 9-bit ranks (windows of up to kWideWindowMax entries; wlen
// receives the per-tile records, masks laid out for `wide_vec` elements per
// lane and load block)
hipError_t launch_window_encode(const int32_t *col, const int32_t *tile_j, const int32_t *base,
                                int64_t n_tiles, uint16_t *dict, int32_t *wlen, uint8_t *codes,
                                int32_t *max_m, hipStream_t s, int wide_vec = 0);
// Column blocks: cnt[b * n_rows + i] = nonzeros of row i in column block b
// (columns [b width, (b+1) width)); then every nonzero is copied to its
// block, rows in order and storage order inside a row, at pos[b] = off[b] +
// rpb[b * (n_rows + 1) + i] (rpb counting from 0 in each block). B <= 16.
constexpr int kMaxColBlocks = 16;
hipError_t launch_colblock_count(const int32_t *rp, const int32_t *col, int32_t n_rows, int32_t B,
                                 int32_t width, int32_t *cnt, hipStream_t s);
hipError_t launch_colblock_scatter(const int32_t *rp, const int32_t *col, const void *val,
                                   int32_t vbytes, int32_t n_rows, int32_t B, int32_t width,
                                   const int32_t *rpb, const int64_t *off, int32_t *colb,
                                   void *valb, hipStream_t s);
// Merge tiles are cut at row ends (slack = longest row + 1) when every row is
// shorter than this; otherwise slack = 0 and rows may span tiles.
constexpr int32_t kMergeRowAlignMax = 64;

// arr = {rp, col, codes, val, x, y, window dict, window lengths}; L = 64 *
// ipt; x32: x spans < 4 GiB; fixup: run the cross-tile fixup pass (tiles not
// row-aligned); idx != IDX_I32: arr[2] holds the merge codes (or the window
// ranks, IDX_W8, row-aligned tiles only) and tile_base the tile bases; acc
// (row-aligned tiles only): y += A x instead of y = A x
hipError_t launch_merge_s0(int ipt, bool nt, bool x32, bool fixup, int idx,
                           const int32_t *tile_base, int32_t n_cols, const void *const *arr,
                           const int32_t *tile_i, const int32_t *tile_j, void *carry, int32_t n_rows, int64_t n_tiles,
                           hipEvent_t after_main, hipStream_t s, bool acc = false,
                           const int32_t *rowid = nullptr);
hipError_t launch_merge_s1(int ipt, bool nt, bool x32, bool fixup, int idx,
                           const int32_t *tile_base, int32_t n_cols, const void *const *arr,
                           const int32_t *tile_i, const int32_t *tile_j, void *carry, int32_t n_rows, int64_t n_tiles,
                           hipEvent_t after_main, hipStream_t s, bool acc = false,
                           const int32_t *rowid = nullptr);
hipError_t launch_merge_s2(int ipt, bool nt, bool x32, bool fixup, int idx,
                           const int32_t *tile_base, int32_t n_cols, const void *const *arr,
                           const int32_t *tile_i, const int32_t *tile_j, void *carry, int32_t n_rows, int64_t n_tiles,
                           hipEvent_t after_main, hipStream_t s, bool acc = false,
                           const int32_t *rowid = nullptr);
hipError_t launch_fill_row_index(const int32_t *rp, int32_t n_rows, int32_t n_cols, int32_t *out,
                                 hipStream_t s);
hipError_t launch_convert_values(const double *src, void *dst, int64_t n, int storage,
                                 hipStream_t s);
// y = A x under plan P. If `before`/`after` are given, they are recorded on
// `s` immediately around the plan's dominant (first) kernel.
hipError_t launch_spmv(const csr_matrix_s *A, const Plan &P, const void *x, void *y,
                       hipStream_t s, hipEvent_t before = nullptr, hipEvent_t after = nullptr);
// Name of the plan's dominant kernel (as in a kernel trace).
// Merge-path tile sizes: prebuilt (256, 512, 1024) or compiled at run time
// (any multiple of 256 up to 2048); merge or window codes of code_bytes per
// nonzero need a lane's codes to form whole loads at tile size L.
bool merge_items_prebuilt(int64_t L);
bool merge_items_supported(int64_t L);
bool merge_codes_fit(int64_t L, int code_bytes);
// The merge kernel instance compiled at run time (hipRTC) and loaded on
// `device`; cached for the life of the process.
csr_status_t jit_merge_kernel(int device, int storage, int ipt, bool nt, bool x32, int idx,
                              bool aln, hipFunction_t *out);
// x of this matrix spans < 4 GiB, so gathers may use 32-bit byte offsets
bool x_fits_32(const csr_matrix_s *A);
// slack of the row-aligned merge partition at tile size L (0: plain cuts),
// and the number of tiles it gives
int64_t merge_slack(const csr_matrix_s *A, int64_t L);
int64_t merge_tile_count(const csr_matrix_s *A, int64_t L);
std::string dominant_kernel(const csr_matrix_s *A, const Plan &P);
// kernels one call of plan P launches
int plan_kernel_count(const csr_matrix_s *A, const Plan &P);
// a[i] = b[i] + scalar * c[i] (one FMA) over n doubles (n even); streaming:
// non-temporal loads and stores (the HBM probe), else ordinary ones (the
// cache-resident probe)
hipError_t launch_triad(double *a, const double *b, const double *c, double scalar,
                        int64_t n, bool streaming, hipStream_t s);
// B_max probe at one footprint: best of `reps` triad passes over three
// arrays of bytes_per_array bytes (allocated and freed inside), in B/s
csr_status_t triad_bandwidth(size_t bytes_per_array, int reps, bool streaming, hipStream_t s,
                             double *bytes_per_s);
// wall_clock64() ticks per second on `device`
double device_wall_clock_hz(int device);

// Partial feature sums of one workgroup (folded in a fixed order).
struct FeatPart {
    int64_t s_nnz2, s_bw, s_bw2, s_miss, s_grp, s_len1;
    int32_t nnz_min, nnz_max, bw_min, bw_max;
    double sc_n, sc_mean, sc_m2;  // Welford state of scatter_i
    double s_cl;                  // sum of clustering_i
};
int32_t features_partials(int32_t n_rows, int G);
int32_t xreuse_samples(int32_t n_rows);
// Rows longer than this are reduced by a whole workgroup each (not by the
// G lanes of the sweep); at most this many of them fit in nnz entries.
int32_t features_long_row(int G);
int64_t features_long_capacity(int64_t nnz, int G);
// Allocate the feature sweep's workspace of a handle (no-op when present).
csr_status_t feature_buffers(csr_matrix_s *A);
// The sweep's results, read back in one copy: the folded partials, the
// number of long rows, then (at kFeatHeader bytes) the x-reuse samples.
constexpr size_t kFeatHeader = 128;
static_assert(sizeof(FeatPart) + sizeof(int32_t) <= kFeatHeader, "feature header");
// The sweep, its fold and the x-reuse samples, enqueued on s; `out` receives
// the results laid out as above (the long rows are not in the fold yet).
// parts: n_parts + long capacity entries; long_list: long capacity + 1 ints
// ([0] the long-row count); long_bits: ceil(n_rows / 32) words, one bit per
// row the sweep leaves to the long pass.
hipError_t launch_features(const int32_t *rp, const int32_t *col, int32_t n_rows, int G,
                           FeatPart *parts, int32_t n_parts, int32_t *long_list,
                           uint32_t *long_bits, void *out, hipStream_t s);
// With n_long > 0 long rows (the count launch_features left): the long rows
// listed in row order from their bits (on the device), their partials, and
// the fold over all partials into `out`; enqueued on s.
hipError_t features_long_rows(const int32_t *rp, const int32_t *col, int32_t n_rows, int64_t nnz,
                              int G, FeatPart *parts, int32_t n_parts, int32_t *long_list,
                              const uint32_t *long_bits, int32_t n_long, void *out,
                              hipStream_t s);

hipError_t launch_long_s0(const int32_t *col, const void *val, const void *x, void *y,
                          const int32_t *chunk_beg, void *part, int64_t n_chunks,
                          const int32_t *long_rows, const int32_t *row_chunk, int32_t n_long,
                          hipStream_t s);
hipError_t launch_long_s1(const int32_t *col, const void *val, const void *x, void *y,
                          const int32_t *chunk_beg, void *part, int64_t n_chunks,
                          const int32_t *long_rows, const int32_t *row_chunk, int32_t n_long,
                          hipStream_t s);
hipError_t launch_long_s2(const int32_t *col, const void *val, const void *x, void *y,
                          const int32_t *chunk_beg, void *part, int64_t n_chunks,
                          const int32_t *long_rows, const int32_t *row_chunk, int32_t n_long,
                          hipStream_t s);

// Learned selector (k_mlp.hip, learn.hip) -------------------------------------------
int mlp_param_count(int K);
int mlp_max_batch();
int mlp_max_classes();
hipError_t launch_mlp_forward(const float *p, int K, const float *X, int B, float *logits,
                              hipStream_t s);
hipError_t launch_mlp_grad(const float *p, int K, const float *X, const int32_t *labels, int B,
                           float *g, float *loss, hipStream_t s);
hipError_t launch_mlp_train(float *p, float *m, float *v, float *g, int K, const float *X,
                            const int32_t *y, const int32_t *order, int B, int steps, int t0,
                            float lr, float b1, float b2, float eps, float *losses,
                            hipStream_t s);
hipError_t launch_mlp_normalize(const double *f, const double *mu, const double *sigma,
                                int64_t n, float *out, hipStream_t s);
hipError_t launch_mlp_select(const float *p, int K, const double *f, const double *mu,
                             const double *sigma, int32_t *out, hipStream_t s);
csr_status_t learned_pick(csr_matrix_s *A, hipStream_t s, double ood_z, int32_t *variant,
                          double *z_max);

// Plans and selection (select.hip) -----------------------------------------------
double plan_bytes(const csr_matrix_s *A, const Plan &P);
// the derived tables plan P reads (tile table, codes, column blocks, long-row
// list, schedule counters) are the ones the handle holds
bool plan_tables_ok(const csr_matrix_s *A, const Plan &P);
csr_status_t realize(csr_matrix_s *A, int32_t opts, const csr_config_t &cfg, Plan *out,
                     hipStream_t s);
void fill_info(const csr_matrix_s *A, const Plan &P, csr_plan_info_t *info);

// Host helpers -------------------------------------------------------------------
int default_lanes_per_row(double nnz_avg);
int device_cu_count(int device);
size_t storage_bytes(int storage);

}  // namespace csr
