// Batched SpMV: device descriptors and the class kernels of a persistent
// batched launch. Every matrix of a batch runs its own plan: the matrices
// whose plans launch the same kernel instance form one class, and each class
// is one persistent kernel over the concatenated work items of its matrices
// (merge-path tiles, row blocks, or long-row chunks), running exactly the
// per-item code of the single-matrix kernel, so each matrix gets the same
// bits as from its own csr_spmv.
#pragma once

#include "internal.h"

namespace csr {

struct BatchMat {
    const int32_t *rp;
    const int32_t *col;         // int32 columns (row split: also with delta codes unused)
    const void *codes;          // merge codes, window ranks, or the row split's delta codes
    const void *val;
    const void *x;
    void *y;
    const int32_t *tile_i;      // merge path: the matrix's (or column block's) tile table
    const int32_t *tile_j;
    const int32_t *tile_base;   // merge and window codes: each tile's smallest column
    const uint16_t *wdict;      // window codes: per-tile dictionaries
    const int32_t *wlen;
    void *carry;                // merge path: per-tile carries; long rows: per-chunk partials
    const int32_t *long_rows;   // long-row pass: the rows, their first chunks, the chunks
    const int32_t *row_chunk;
    const int32_t *chunks;
    int32_t n_rows;
    int32_t n_cols;
    int32_t skip_above;         // row split: longer rows belong to the long-row pass
    int32_t acc;                // merge path, column blocks after the first: y += A x
    const int32_t *rowid;       // merge path, a column block over its rows: y's row of each
    int64_t item_base;          // first item of this matrix in its class's queue
    int64_t item_base2;         // long-row pass: first long row in the second queue
};

// Merge-path class: item g is tile g - item_base of matrix item_mat[g]; the
// carry fixup follows when the tiles are not row-aligned.
hipError_t launch_bmerge_s0(int ipt, bool nt, bool x32, int idx, bool aln, const BatchMat *mats,
                            const int32_t *item_mat, int64_t n_items, int n_cu, hipStream_t s);
hipError_t launch_bmerge_s1(int ipt, bool nt, bool x32, int idx, bool aln, const BatchMat *mats,
                            const int32_t *item_mat, int64_t n_items, int n_cu, hipStream_t s);
hipError_t launch_bmerge_s2(int ipt, bool nt, bool x32, int idx, bool aln, const BatchMat *mats,
                            const int32_t *item_mat, int64_t n_items, int n_cu, hipStream_t s);
// Row-split class: item g is logical row block g - item_base of matrix
// item_mat[g].
hipError_t launch_brows_s0(int G, int idx, bool nt, int U, int R, const BatchMat *mats,
                           const int32_t *item_mat, int64_t n_items, int n_cu, hipStream_t s);
hipError_t launch_brows_s1(int G, int idx, bool nt, int U, int R, const BatchMat *mats,
                           const int32_t *item_mat, int64_t n_items, int n_cu, hipStream_t s);
hipError_t launch_brows_s2(int G, int idx, bool nt, int U, int R, const BatchMat *mats,
                           const int32_t *item_mat, int64_t n_items, int n_cu, hipStream_t s);
// Long-row pass of the decomposition plans: chunk g (item_mat[g]'s chunk
// g - item_base), then long row q (row_mat[q]'s long row q - item_base2).
hipError_t launch_blong_s0(const BatchMat *mats, const int32_t *item_mat, int64_t n_chunks,
                           const int32_t *row_mat, int64_t n_long, int n_cu, hipStream_t s);
hipError_t launch_blong_s1(const BatchMat *mats, const int32_t *item_mat, int64_t n_chunks,
                           const int32_t *row_mat, int64_t n_long, int n_cu, hipStream_t s);
hipError_t launch_blong_s2(const BatchMat *mats, const int32_t *item_mat, int64_t n_chunks,
                           const int32_t *row_mat, int64_t n_long, int n_cu, hipStream_t s);

// Drop every cached batch plan that refers to handle `id` (called on destroy).
void batch_forget(uint64_t id);

}  // namespace csr
