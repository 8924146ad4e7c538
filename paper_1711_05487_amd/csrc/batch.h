// Batched SpMV: device descriptor of one matrix in a persistent launch.
#pragma once

#include "internal.h"

namespace csr {

struct BatchMat {
    const int32_t *rp;
    const int32_t *col;
    const void *val;
    const void *x;
    void *y;
    const int32_t *tile_i;  // this matrix's merge-path tile table (T+1 entries)
    const int32_t *tile_j;
    void *carry;            // T tile carries
    int32_t n_rows;
    int32_t ipt;            // L = 64 * ipt (4, 8 or 16)
    int32_t aligned;        // 1: tiles cut at row ends (no carries, rows reduced by lane groups)
    int32_t reserved;
    int64_t tile_base;      // index of this matrix's first tile in the work queue
};

hipError_t launch_batch_s0(const BatchMat *mats, const int32_t *item_mat, int64_t n_items,
                           int n_cu, hipStream_t s);
hipError_t launch_batch_s1(const BatchMat *mats, const int32_t *item_mat, int64_t n_items,
                           int n_cu, hipStream_t s);
hipError_t launch_batch_s2(const BatchMat *mats, const int32_t *item_mat, int64_t n_items,
                           int n_cu, hipStream_t s);

// Drop every cached batch plan that refers to handle `id` (called on destroy).
void batch_forget(uint64_t id);

}  // namespace csr
