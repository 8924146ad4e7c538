// nnz-balanced merge-path SpMV: the GPU counterpart of the runtime-chosen
// schedule that the optimization pool applies to thread imbalance (Sec. III-E,
// Table II, IMB). The path merges the row ends rp[1..N] with the nonzero
// indices 0..NNZ-1 (a nonzero j is taken before row end i while j < rp[i+1]);
// tile t covers L = 64 * IPT consecutive path items, so every workgroup gets
// the same amount of work whatever the row lengths.
//
// A tile is one wave64 workgroup: small workgroups keep many independent
// tiles resident per CU, which hides the gather latency of irregular
// matrices far better than 256-thread tiles of the same L (and the
// workgroup barriers reduce to wave-level ones).
//
// Per tile:
//  1. row ends of the rows finishing in the tile -> LDS (tile-local offsets);
//  2. the tile's nonzeros are streamed with aligned vector loads, x gathered,
//     products rounded and stored in LDS (so every global load is coalesced);
//  3. each thread walks IPT path items of the tile (its own merge-path
//     diagonal, found by binary search in LDS), summing products and emitting
//     rows as their ends go by;
//  4. rows split across threads are completed from the per-thread carries in
//     thread order; the row still open at the tile end leaves one carry per
//     tile, and rows split across tiles are finished by k_merge_fixup, which
//     adds the carries in tile order. Every sum has a fixed order, so results
//     are deterministic.
//
// Compiled once per storage type (-DCSR_STORAGE=0/1/2).
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

template <int IPT, bool NT>
__global__ __launch_bounds__(kMergeBlock) void k_merge(
    const int32_t *__restrict__ rp, const int32_t *__restrict__ col, const V *__restrict__ val,
    const X *__restrict__ x, X *__restrict__ y, const int32_t *__restrict__ tile_i,
    const int32_t *__restrict__ tile_j, A *__restrict__ carry, int32_t n_rows, int64_t per_xcd,
    int64_t n_tiles) {
    __shared__ MergeLds<S, IPT> lds;
    const int64_t t = xcd_logical_block(per_xcd);
    if (t >= n_tiles) return;
    merge_tile<S, IPT, NT>(t, rp, col, val, x, y, tile_i, tile_j, carry, n_rows, lds);
}

__global__ __launch_bounds__(kBlock) void k_merge_fixup(const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ tile_i,
                                                        const int32_t *__restrict__ tile_j,
                                                        const A *__restrict__ carry,
                                                        X *__restrict__ y, int32_t n_rows,
                                                        int64_t n_tiles) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < n_tiles) merge_fixup_tile<S>(t, rp, tile_i, tile_j, carry, y, n_rows);
}

template <int IPT, bool NT>
hipError_t go(const void *const *arr, const int32_t *tile_i, const int32_t *tile_j, void *carry,
              int32_t n_rows, int64_t n_tiles, hipEvent_t after_main, hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    const XcdGrid g = xcd_grid(n_tiles);
    hipLaunchKernelGGL((k_merge<IPT, NT>), dim3((unsigned)g.launched), dim3(kMergeBlock), 0, s,
                       (const int32_t *)arr[0], (const int32_t *)arr[1], (const V *)arr[3],
                       (const X *)arr[4], (X *)arr[5], tile_i, tile_j, (A *)carry, n_rows,
                       g.per_xcd, n_tiles);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && after_main) e = hipEventRecord(after_main, s);
    if (e != hipSuccess || n_tiles < 2) return e;
    const unsigned fb = (unsigned)((n_tiles + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_merge_fixup, dim3(fb), dim3(kBlock), 0, s, (const int32_t *)arr[0],
                       tile_i, tile_j, (const A *)carry, (X *)arr[5], n_rows, n_tiles);
    return hipGetLastError();
}

}  // namespace

#define CSR_CAT2(a, b) a##b
#define CSR_CAT(a, b) CSR_CAT2(a, b)
// arr = {rp, col, codes, val, x, y}; L = 64 * ipt
hipError_t CSR_CAT(launch_merge_s, CSR_STORAGE)(int ipt, bool nt, const void *const *arr,
                                                const int32_t *tile_i, const int32_t *tile_j,
                                                void *carry, int32_t n_rows, int64_t n_tiles,
                                                hipEvent_t after_main, hipStream_t s) {
    switch (ipt) {
    case 4: return nt ? go<4, true>(arr, tile_i, tile_j, carry, n_rows, n_tiles, after_main, s)
                      : go<4, false>(arr, tile_i, tile_j, carry, n_rows, n_tiles, after_main, s);
    case 8: return nt ? go<8, true>(arr, tile_i, tile_j, carry, n_rows, n_tiles, after_main, s)
                      : go<8, false>(arr, tile_i, tile_j, carry, n_rows, n_tiles, after_main, s);
    case 16: return nt ? go<16, true>(arr, tile_i, tile_j, carry, n_rows, n_tiles, after_main, s)
                       : go<16, false>(arr, tile_i, tile_j, carry, n_rows, n_tiles, after_main, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace csr
