// The merge-path tile kernel: one wave64 workgroup per tile of L = 64 * IPT
// path items (merge_tile). The library holds the instances of IPT 4, 8 and
// 16 (k_merge.hip, one object per value storage, so those kernels have
// internal linkage); other tile sizes are compiled at run time from this
// same header (jit.hip), where the module exports the one kernel it holds.
// CSR_STORAGE selects the value storage (0 FP64, 1 FP32, 2 BF16).
#pragma once

#include "merge_tile.h"

#ifndef CSR_STORAGE
#error "CSR_STORAGE must be defined"
#endif

namespace csr {
#ifndef __HIPCC_RTC__
namespace {
#endif

template <int IPT, bool NT, bool X32, int IDX, bool ALN>
__global__ __launch_bounds__(kMergeBlock) void k_merge(
    const int32_t *__restrict__ rp, const void *__restrict__ cols,
    const typename St<CSR_STORAGE>::V *__restrict__ val,
    const typename St<CSR_STORAGE>::X *__restrict__ x, typename St<CSR_STORAGE>::X *__restrict__ y,
    const int32_t *__restrict__ tile_i, const int32_t *__restrict__ tile_j,
    const int32_t *__restrict__ tile_base, typename St<CSR_STORAGE>::A *__restrict__ carry,
    int32_t n_rows, int32_t n_cols, int64_t per_xcd, int64_t n_tiles,
    const uint16_t *__restrict__ wdict, const int32_t *__restrict__ wlen, int32_t acc,
    const int32_t *__restrict__ rowid) {
    constexpr int S = CSR_STORAGE;
    using Lds = std::conditional_t<ALN, MergeLdsRows<S, IPT>, MergeLds<S, IPT>>;
    __shared__ Lds lds;
    const int64_t t = xcd_logical_block(per_xcd);
    if (t >= n_tiles) return;
    merge_tile<S, IPT, NT, Lds, X32, IDX, ALN>(t, rp, cols, val, x, y, tile_i, tile_j, carry,
                                                n_rows, lds, tile_base, n_cols, wdict, wlen,
                                                acc != 0, rowid);
}

#ifndef __HIPCC_RTC__
}  // namespace
#endif
}  // namespace csr
