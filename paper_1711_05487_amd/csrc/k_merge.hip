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
// Per tile (merge_tile): the nonzeros are streamed with coalesced vector
// loads and their products staged in LDS; the tile is then reduced as one
// segmented scan across the wave, with a segment starting at every row end
// inside the tile, and each row reads its sum at its last nonzero. The row
// still open at the tile end leaves one carry per tile; rows split across
// tiles are finished by k_merge_fixup, which adds the carries in tile order.
// When every row has fewer than 64 nonzeros the tiles are cut at row ends
// (the partition's slack): no row is split, the fixup is not launched, and
// each row is summed from LDS by its own group of lanes instead of the scan.
// Every sum has a fixed order, so results are deterministic.
//
// Compiled once per storage type (-DCSR_STORAGE=0/1/2).
#include "merge_kernel.h"
#include "internal.h"

#ifndef CSR_STORAGE
#error "CSR_STORAGE must be defined"
#endif

namespace csr {
namespace {

constexpr int S = CSR_STORAGE;
using V = typename St<S>::V;
using X = typename St<S>::X;
using A = typename St<S>::A;

__global__ __launch_bounds__(kBlock) void k_merge_fixup(const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ tile_i,
                                                        const int32_t *__restrict__ tile_j,
                                                        const A *__restrict__ carry,
                                                        X *__restrict__ y, int32_t n_rows,
                                                        int64_t n_tiles,
                                                        const int32_t *__restrict__ rowid) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < n_tiles) merge_fixup_tile<S>(t, rp, tile_i, tile_j, carry, y, n_rows, rowid);
}

struct MergeArgs {
    const void *const *arr;  // {rp, cols or codes, -, val, x, y}
    const int32_t *tile_i, *tile_j, *tile_base;
    void *carry;
    int32_t n_rows, n_cols;
    int64_t n_tiles;
    bool fixup;
    hipEvent_t after_main;
    bool acc;
    const int32_t *rowid;  // rows as a list (column block over its rows), or null
};

// After the main kernel: the caller's event, then (tiles not row-aligned)
// the fixup pass that adds the carries of rows split across tiles.
hipError_t after_main(hipError_t e, bool aln, const MergeArgs &a, hipStream_t s) {
    if (e == hipSuccess && a.after_main) e = hipEventRecord(a.after_main, s);
    if (e != hipSuccess || a.n_tiles < 2 || aln) return e;
    const unsigned fb = (unsigned)((a.n_tiles + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_merge_fixup, dim3(fb), dim3(kBlock), 0, s, (const int32_t *)a.arr[0],
                       a.tile_i, a.tile_j, (const A *)a.carry, (X *)a.arr[5], a.n_rows, a.n_tiles,
                       a.rowid);
    return hipGetLastError();
}

template <int IPT, bool NT, bool X32, int IDX, bool ALN>
hipError_t go(const MergeArgs &a, hipStream_t s) {
    if (a.n_tiles == 0) return hipSuccess;
    const void *cols = IDX == IDX_I32 ? a.arr[1] : a.arr[2];
    const XcdGrid g = xcd_grid(a.n_tiles);
    hipLaunchKernelGGL((k_merge<IPT, NT, X32, IDX, ALN>), dim3((unsigned)g.launched), dim3(kMergeBlock),
                       0, s, (const int32_t *)a.arr[0], cols, (const V *)a.arr[3],
                       (const X *)a.arr[4], (X *)a.arr[5], a.tile_i, a.tile_j, a.tile_base,
                       (A *)a.carry, a.n_rows, a.n_cols, g.per_xcd, a.n_tiles,
                       (const uint16_t *)a.arr[6], (const int32_t *)a.arr[7], (int32_t)a.acc,
                       a.rowid);
    return after_main(hipGetLastError(), ALN, a, s);
}

// Tile sizes outside the prebuilt set: the same kernel template compiled at
// run time (the fixup pass is the prebuilt one; it does not depend on L).
hipError_t go_jit(int ipt, bool nt, bool x32, int idx, bool aln, const MergeArgs &a,
                  hipStream_t s) {
    if (a.n_tiles == 0) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    hipFunction_t f;
    if (jit_merge_kernel(dev, S, ipt, nt, x32, idx, aln, &f) != CSR_OK) return hipErrorInvalidValue;
    const XcdGrid g = xcd_grid(a.n_tiles);
    const int32_t *rp = (const int32_t *)a.arr[0];
    const void *cols = idx == IDX_I32 ? a.arr[1] : a.arr[2];
    const V *val = (const V *)a.arr[3];
    const X *x = (const X *)a.arr[4];
    X *y = (X *)a.arr[5];
    const int32_t *ti = a.tile_i, *tj = a.tile_j, *tb = a.tile_base;
    A *carry = (A *)a.carry;
    int32_t n_rows = a.n_rows, n_cols = a.n_cols, acc = a.acc;
    int64_t per_xcd = g.per_xcd, n_tiles = a.n_tiles;
    const uint16_t *wdict = (const uint16_t *)a.arr[6];
    const int32_t *wlen = (const int32_t *)a.arr[7];
    const int32_t *rowid = a.rowid;
    void *args[] = {&rp,     &cols,    &val,    &x,     &y,     &ti,   &tj,   &tb,
                    &carry,  &n_rows,  &n_cols, &per_xcd, &n_tiles, &wdict, &wlen, &acc,
                    &rowid};
    e = hipModuleLaunchKernel(f, (unsigned)g.launched, 1, 1, kMergeBlock, 1, 1, 0, s, args,
                              nullptr);
    return after_main(e, aln, a, s);
}

// int32 columns: streaming and 32-bit gathers chosen at run time; merge
// codes and window codes always stream (they are the MB remedy's compressed
// arrays) and gather through the tile's x range
template <int IPT, bool ALN>
hipError_t go_ipt(bool nt, bool x32, int idx, const MergeArgs &a, hipStream_t s) {
    switch (idx) {
    case IDX_D16: return go<IPT, true, false, IDX_D16, ALN>(a, s);
    case IDX_D8: return go<IPT, true, false, IDX_D8, ALN>(a, s);
    case IDX_W8:
        if constexpr (ALN) return go<IPT, true, false, IDX_W8, true>(a, s);
        else return hipErrorInvalidValue;  // window codes need row-aligned tiles
    case IDX_R8:
        if constexpr (ALN) return go<IPT, true, false, IDX_R8, true>(a, s);
        else return hipErrorInvalidValue;
    case IDX_W9:  // 9-bit window ranks: tiles of 1,024 items only
        if constexpr (ALN && IPT == 16) return go<IPT, true, false, IDX_W9, true>(a, s);
        else return hipErrorInvalidValue;
    default: break;
    }
    if (nt)
        return x32 ? go<IPT, true, true, IDX_I32, ALN>(a, s) : go<IPT, true, false, IDX_I32, ALN>(a, s);
    return x32 ? go<IPT, false, true, IDX_I32, ALN>(a, s) : go<IPT, false, false, IDX_I32, ALN>(a, s);
}

}  // namespace

#define CSR_CAT2(a, b) a##b
#define CSR_CAT(a, b) CSR_CAT2(a, b)
// arr = {rp, col, codes, val, x, y}; L = 64 * ipt; x32: x spans < 4 GiB
hipError_t CSR_CAT(launch_merge_s, CSR_STORAGE)(int ipt, bool nt, bool x32, bool fixup, int idx,
                                                const int32_t *tile_base, int32_t n_cols,
                                                const void *const *arr, const int32_t *tile_i,
                                                const int32_t *tile_j, void *carry, int32_t n_rows,
                                                int64_t n_tiles, hipEvent_t after_main,
                                                hipStream_t s, bool acc, const int32_t *rowid) {
    if (rowid && !fixup) return hipErrorInvalidValue;  // row lists only on split rows
    const MergeArgs a{arr, tile_i, tile_j, tile_base, carry, n_rows, n_cols, n_tiles, fixup,
                      after_main, acc, rowid};
    // row-aligned tiles (no fixup) reduce by rows, the others by a
    // segmented scan with carries
    switch (ipt) {
    case 4: return fixup ? go_ipt<4, false>(nt, x32, idx, a, s) : go_ipt<4, true>(nt, x32, idx, a, s);
    case 8: return fixup ? go_ipt<8, false>(nt, x32, idx, a, s) : go_ipt<8, true>(nt, x32, idx, a, s);
    case 16:
        return fixup ? go_ipt<16, false>(nt, x32, idx, a, s) : go_ipt<16, true>(nt, x32, idx, a, s);
    default: return go_jit(ipt, nt, x32, idx, !fixup, a, s);
    }
}

}  // namespace csr
