// Batched SpMV, merge-path and long-row classes: many independent
// y_k = A_k x_k in persistent launches over the concatenated work items of
// every matrix of a class. Workgroup b takes items b, b + nblk, b + 2 nblk,
// ... (the items of a class are of equal size, so the static assignment is
// balanced and no counter has to be reset between graph replays). Every item
// runs exactly the per-item code of the single-matrix kernel with the
// matrix's own tables, so a matrix's result in the batch is bit-identical to
// its own csr_spmv.
//
// Compiled once per storage type (-DCSR_STORAGE=0/1/2).
#include <type_traits>

#include "batch.h"
#include "long_rows.h"
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

template <int IPT, bool NT, bool X32, int IDX, bool ALN>
__global__ __launch_bounds__(kMergeBlock) void k_bmerge(const BatchMat *__restrict__ mats,
                                                   const int32_t *__restrict__ item_mat,
                                                   int64_t n_items, int64_t per_xcd, int64_t nblk) {
    using Lds = std::conditional_t<ALN, MergeLdsRows<S, IPT>, MergeLds<S, IPT>>;
    __shared__ Lds lds;
    const int64_t lb = xcd_logical_block(per_xcd);
    if (lb >= nblk) return;
    for (int64_t g = lb; g < n_items; g += nblk) {
        const BatchMat &M = mats[item_mat[g]];
        const void *cols = IDX == IDX_I32 ? (const void *)M.col : M.codes;
        merge_tile<S, IPT, NT, Lds, X32, IDX, ALN>(
            g - M.item_base, M.rp, cols, (const V *)M.val, (const X *)M.x, (X *)M.y, M.tile_i,
            M.tile_j, (A *)M.carry, M.n_rows, lds, M.tile_base, M.n_cols, M.wdict, M.wlen,
            M.acc != 0, M.rowid);
        wave_lds_sync();  // LDS is reused by the next item
    }
}

__global__ __launch_bounds__(kBlock) void k_bmerge_fixup(const BatchMat *__restrict__ mats,
                                                         const int32_t *__restrict__ item_mat,
                                                         int64_t n_items) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= n_items) return;
    const BatchMat &M = mats[item_mat[g]];
    merge_fixup_tile<S>(g - M.item_base, M.rp, M.tile_i, M.tile_j, (const A *)M.carry, (X *)M.y,
                        M.n_rows, M.rowid);
}

__global__ __launch_bounds__(kBlock) void k_blong_partial(const BatchMat *__restrict__ mats,
                                                          const int32_t *__restrict__ item_mat,
                                                          int64_t n_chunks) {
    __shared__ A s[kBlock];
    for (int64_t g = blockIdx.x; g < n_chunks; g += gridDim.x) {
        const BatchMat &M = mats[item_mat[g]];
        long_chunk_partial<S>(g - M.item_base, M.col, (const V *)M.val, (const X *)M.x, M.chunks,
                              (A *)M.carry, s);
        __syncthreads();  // s is reused by the next chunk
    }
}

__global__ __launch_bounds__(kBlock) void k_blong_final(const BatchMat *__restrict__ mats,
                                                        const int32_t *__restrict__ row_mat,
                                                        int64_t n_long) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= n_long) return;
    const BatchMat &M = mats[row_mat[q]];
    long_row_final<S>((int32_t)(q - M.item_base2), M.long_rows, M.row_chunk, (const A *)M.carry,
                      (X *)M.y);
}

template <class K>
int64_t persistent_grid(K kernel, int block, int64_t n_items, int n_cu) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return std::min<int64_t>(n_items, (int64_t)n_cu * per_cu);
}

template <int IPT, bool NT, bool X32, int IDX, bool ALN>
hipError_t go(const BatchMat *mats, const int32_t *item_mat, int64_t n_items, int n_cu,
              hipStream_t s) {
    auto kern = k_bmerge<IPT, NT, X32, IDX, ALN>;
    const XcdGrid g = xcd_grid(persistent_grid(kern, kMergeBlock, n_items, n_cu));
    hipLaunchKernelGGL(kern, dim3((unsigned)g.launched), dim3(kMergeBlock), 0, s, mats, item_mat,
                       n_items, g.per_xcd, g.nblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || ALN) return e;
    hipLaunchKernelGGL(k_bmerge_fixup, dim3((unsigned)((n_items + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, mats, item_mat, n_items);
    return hipGetLastError();
}

// the single-matrix path's instance choice: codes always stream and gather
// through the tile's x range; int32 columns pick streaming and 32-bit
// offsets at run time
template <int IPT, bool ALN>
hipError_t go_ipt(bool nt, bool x32, int idx, const BatchMat *mats, const int32_t *item_mat,
                  int64_t n_items, int n_cu, hipStream_t s) {
    switch (idx) {
    case IDX_D16: return go<IPT, true, false, IDX_D16, ALN>(mats, item_mat, n_items, n_cu, s);
    case IDX_D8: return go<IPT, true, false, IDX_D8, ALN>(mats, item_mat, n_items, n_cu, s);
    case IDX_W8:
        if constexpr (ALN) return go<IPT, true, false, IDX_W8, true>(mats, item_mat, n_items, n_cu, s);
        else return hipErrorInvalidValue;
    case IDX_R8:
        if constexpr (ALN) return go<IPT, true, false, IDX_R8, true>(mats, item_mat, n_items, n_cu, s);
        else return hipErrorInvalidValue;
    case IDX_W9:
        if constexpr (ALN && IPT == 16)
            return go<IPT, true, false, IDX_W9, true>(mats, item_mat, n_items, n_cu, s);
        else return hipErrorInvalidValue;
    default: break;
    }
    if (nt)
        return x32 ? go<IPT, true, true, IDX_I32, ALN>(mats, item_mat, n_items, n_cu, s)
                   : go<IPT, true, false, IDX_I32, ALN>(mats, item_mat, n_items, n_cu, s);
    return x32 ? go<IPT, false, true, IDX_I32, ALN>(mats, item_mat, n_items, n_cu, s)
               : go<IPT, false, false, IDX_I32, ALN>(mats, item_mat, n_items, n_cu, s);
}

}  // namespace

#define CSR_CAT2(a, b) a##b
#define CSR_CAT(a, b) CSR_CAT2(a, b)
hipError_t CSR_CAT(launch_bmerge_s, CSR_STORAGE)(int ipt, bool nt, bool x32, int idx, bool aln,
                                                 const BatchMat *mats, const int32_t *item_mat,
                                                 int64_t n_items, int n_cu, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    switch (ipt) {
    case 4:
        return aln ? go_ipt<4, true>(nt, x32, idx, mats, item_mat, n_items, n_cu, s)
                   : go_ipt<4, false>(nt, x32, idx, mats, item_mat, n_items, n_cu, s);
    case 8:
        return aln ? go_ipt<8, true>(nt, x32, idx, mats, item_mat, n_items, n_cu, s)
                   : go_ipt<8, false>(nt, x32, idx, mats, item_mat, n_items, n_cu, s);
    case 16:
        return aln ? go_ipt<16, true>(nt, x32, idx, mats, item_mat, n_items, n_cu, s)
                   : go_ipt<16, false>(nt, x32, idx, mats, item_mat, n_items, n_cu, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t CSR_CAT(launch_blong_s, CSR_STORAGE)(const BatchMat *mats, const int32_t *item_mat,
                                                int64_t n_chunks, const int32_t *row_mat,
                                                int64_t n_long, int n_cu, hipStream_t s) {
    if (n_long == 0) return hipSuccess;
    const int64_t gp = persistent_grid(k_blong_partial, kBlock, n_chunks, n_cu);
    hipLaunchKernelGGL(k_blong_partial, dim3((unsigned)gp), dim3(kBlock), 0, s, mats, item_mat,
                       n_chunks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_blong_final, dim3((unsigned)((n_long + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, mats, row_mat, n_long);
    return hipGetLastError();
}

}  // namespace csr
