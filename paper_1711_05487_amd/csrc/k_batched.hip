// Batched SpMV: many independent y_k = A_k x_k in one persistent launch.
// The work queue is the concatenation of every matrix's merge-path tiles
// (each matrix with its own tile size L_k = 64 * ipt_k); workgroup b takes
// items b, b + nblk, b + 2 nblk, ... (tiles are equal-sized, so the static
// assignment is balanced and no counter has to be reset between replays).
// Every tile runs exactly the single-matrix tile code, so a matrix's result
// in the batch is bit-identical to its own merge-path SpMV with the same L.
//
// Compiled once per storage type (-DCSR_STORAGE=0/1/2).
#include "batch.h"
#include "merge_tile.h"

#ifndef CSR_STORAGE
#error "CSR_STORAGE must be defined"
#endif

namespace csr {
namespace {

constexpr int S = CSR_STORAGE;
using V = typename St<S>::V;
using X = typename St<S>::X;
using A = typename St<S>::A;

union BatchLds {
    MergeLds<S, 4> l4;
    MergeLds<S, 8> l8;
    MergeLds<S, 16> l16;
};

template <int IPT, bool ALN>
__device__ __forceinline__ void tile(const BatchMat &M, int64_t t, MergeLds<S, IPT> &lds) {
    merge_tile<S, IPT, true, MergeLds<S, IPT>, false, IDX_I32, ALN>(
        t, M.rp, M.col, (const V *)M.val, (const X *)M.x, (X *)M.y, M.tile_i, M.tile_j,
        (A *)M.carry, M.n_rows, lds);
}

__global__ __launch_bounds__(kMergeBlock) void k_batch(const BatchMat *__restrict__ mats,
                                                  const int32_t *__restrict__ item_mat,
                                                  int64_t n_items, int64_t per_xcd, int64_t nblk) {
    __shared__ BatchLds lds;
    const int64_t lb = xcd_logical_block(per_xcd);
    if (lb >= nblk) return;
    for (int64_t g = lb; g < n_items; g += nblk) {
        const BatchMat &M = mats[item_mat[g]];
        const int64_t t = g - M.tile_base;
        if (M.aligned) {
            if (M.ipt == 4)
                tile<4, true>(M, t, lds.l4);
            else if (M.ipt == 8)
                tile<8, true>(M, t, lds.l8);
            else
                tile<16, true>(M, t, lds.l16);
        } else {
            if (M.ipt == 4)
                tile<4, false>(M, t, lds.l4);
            else if (M.ipt == 8)
                tile<8, false>(M, t, lds.l8);
            else
                tile<16, false>(M, t, lds.l16);
        }
        wave_lds_sync();  // LDS is reused by the next item
    }
}

__global__ __launch_bounds__(kBlock) void k_batch_fixup(const BatchMat *__restrict__ mats,
                                                        const int32_t *__restrict__ item_mat,
                                                        int64_t n_items) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= n_items) return;
    const BatchMat &M = mats[item_mat[g]];
    if (M.aligned) return;  // no row spans two tiles
    merge_fixup_tile<S>(g - M.tile_base, M.rp, M.tile_i, M.tile_j, (const A *)M.carry, (X *)M.y,
                        M.n_rows);
}

int blocks_per_cu() {
    static int v = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch, kMergeBlock, 0) != hipSuccess ||
            n < 1)
            n = 1;
        return n;
    }();
    return v;
}

}  // namespace

#define CSR_CAT2(a, b) a##b
#define CSR_CAT(a, b) CSR_CAT2(a, b)
hipError_t CSR_CAT(launch_batch_s, CSR_STORAGE)(const BatchMat *mats, const int32_t *item_mat,
                                                int64_t n_items, int n_cu, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    int64_t nb = (int64_t)n_cu * blocks_per_cu();
    if (nb > n_items) nb = n_items;
    const XcdGrid g = xcd_grid(nb);
    hipLaunchKernelGGL(k_batch, dim3((unsigned)g.launched), dim3(kMergeBlock), 0, s, mats, item_mat,
                       n_items, g.per_xcd, g.nblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_fixup, dim3((unsigned)((n_items + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, mats, item_mat, n_items);
    return hipGetLastError();
}

}  // namespace csr
