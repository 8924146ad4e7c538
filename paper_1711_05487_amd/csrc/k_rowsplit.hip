// Row-split CSR SpMV (Sec. II, Fig. 2 and the static row partitioning of
// Sec. IV-A), the baseline of the method and the carrier of three remedies of
// Sec. III-E, Table II: delta-decoded column indices (MB), streamed val/col
// (ML) and unrolled independent accumulators with several rows per wave (CMP).
//
// G lanes of a wave64 share one row (G in 1..64, so 64/G rows per wave). A
// lane group owns R rows at once: the first G*U entries of all R rows are
// loaded before any of them is used (R*U independent loads in flight per
// lane), longer rows finish in a tail loop, and the G partial sums of each row
// are combined by a fixed butterfly. A workgroup of 256 threads owns R chunks
// of 256/G consecutive rows; workgroups are remapped so each XCD's L2 sees a
// contiguous block of rows.
//
// PROBE = 1 is the P_CMP micro-benchmark of Sec. III-B: the same kernel with
// the column-index stream removed and x read at the row index (unit stride).
// PROBE = 2 is the plain kernel instrumented for P_IMB: each workgroup
// records its start and end times (100 MHz constant clock) and the compute
// unit it ran on.
//
// This file is compiled once per storage type (-DCSR_STORAGE=0/1/2).
#include "device.h"
#include "internal.h"
#include "rowsplit_block.h"

#ifndef CSR_STORAGE
#error "CSR_STORAGE must be defined"
#endif

namespace csr {
namespace {

constexpr int S = CSR_STORAGE;
using V = typename St<S>::V;
using X = typename St<S>::X;
using A = typename St<S>::A;

// Static schedule (ctr == nullptr): workgroup b owns logical block
// xcd_logical_block(b). Dynamic chunks (ctr != nullptr, the "dynamic"
// schedule of the row-parallel kernel): workgroups take `per_fetch`
// logical blocks at a time from ctr[0] until none is left; the last
// workgroup out resets both counters for the next launch, so no host-side
// reset is needed (and the launch can be captured in a graph). Every row is
// summed by one lane group in a fixed order: both schedules give the same
// bits. The P_IMB probe (PROBE == 2) is static.
template <int G, int IDX, bool NT, int U, int R, int PROBE>
__global__ __launch_bounds__(kBlock) void k_rowsplit(
    const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const void *__restrict__ codes, const V *__restrict__ val, const X *__restrict__ x,
    X *__restrict__ y, int32_t skip_above, int32_t n_rows, int32_t n_cols, int64_t per_xcd,
    int64_t nblk, int64_t *__restrict__ rec, int32_t *__restrict__ ctr, int32_t per_fetch) {
    if (PROBE != 0 || ctr == nullptr) {
        const int64_t lb = xcd_logical_block(per_xcd);
        if (lb >= nblk) return;
        int64_t t_start = 0;
        if constexpr (PROBE == 2) {
            if (threadIdx.x == 0) t_start = (int64_t)wall_clock64();
        }
        rowsplit_block<S, G, IDX, NT, U, R, PROBE>(lb, rp, col, codes, val, x, y, skip_above,
                                                n_rows, n_cols);
        if constexpr (PROBE == 2) {
            __syncthreads();
            if (threadIdx.x == 0) {
                rec[3 * lb] = t_start;
                rec[3 * lb + 1] = (int64_t)wall_clock64();
                rec[3 * lb + 2] = (int64_t)__smid();
            }
        }
        return;
    }
    __shared__ int32_t s_first;
    for (;;) {
        if (threadIdx.x == 0) s_first = atomicAdd(ctr, per_fetch);
        __syncthreads();
        const int64_t first = s_first;
        __syncthreads();  // s_first is written again by the next fetch
        if (first >= nblk) break;
        const int64_t last = min(first + (int64_t)per_fetch, nblk);
        for (int64_t lb = first; lb < last; ++lb)
            rowsplit_block<S, G, IDX, NT, U, R, PROBE>(lb, rp, col, codes, val, x, y, skip_above,
                                                    n_rows, n_cols);
    }
    if (threadIdx.x == 0 && atomicAdd(ctr + 1, 1) == (int32_t)gridDim.x - 1) {
        atomicExch(ctr, 0);
        atomicExch(ctr + 1, 0);
    }
}

// arr[7]: the dynamic schedule's two counters (nullptr: static schedule)
template <int G, int IDX, bool NT, int U, int R, int PROBE>
hipError_t go(const void *const *arr, int32_t skip_above, int32_t n_rows, int32_t n_cols,
              hipStream_t s) {
    constexpr int NG = kBlock / G;
    const int64_t rows_per_blk = (int64_t)NG * R;
    const int64_t nblk = (n_rows + rows_per_blk - 1) / rows_per_blk;
    if (nblk == 0) return hipSuccess;
    int32_t *ctr = PROBE == 0 ? (int32_t *)arr[7] : nullptr;
    if (ctr) {
        // a resident grid (8 workgroups of 256 per CU) fetching ~8 times each
        const int64_t grid = std::min<int64_t>(nblk, (int64_t)kMaxResidentGroups);
        const int32_t per_fetch = (int32_t)std::max<int64_t>(1, nblk / (grid * 8));
        hipLaunchKernelGGL((k_rowsplit<G, IDX, NT, U, R, PROBE>), dim3((unsigned)grid),
                           dim3(kBlock), 0, s, (const int32_t *)arr[0], (const int32_t *)arr[1],
                           arr[2], (const V *)arr[3], (const X *)arr[4], (X *)arr[5], skip_above,
                           n_rows, n_cols, (int64_t)0, nblk, (int64_t *)arr[6], ctr, per_fetch);
        return hipGetLastError();
    }
    const XcdGrid g = xcd_grid(nblk);
    hipLaunchKernelGGL((k_rowsplit<G, IDX, NT, U, R, PROBE>), dim3((unsigned)g.launched),
                       dim3(kBlock), 0, s, (const int32_t *)arr[0], (const int32_t *)arr[1],
                       arr[2], (const V *)arr[3], (const X *)arr[4], (X *)arr[5], skip_above,
                       n_rows, n_cols, g.per_xcd, g.nblk, (int64_t *)arr[6], (int32_t *)nullptr,
                       (int32_t)1);
    return hipGetLastError();
}

template <int G, bool NT, int U>
hipError_t pick_r(int R, const void *const *arr, int32_t skip, int32_t n_rows, int32_t n_cols,
                  hipStream_t s) {
    if (R >= 4) return go<G, IDX_I32, NT, U, 4, 0>(arr, skip, n_rows, n_cols, s);
    if (R == 2) return go<G, IDX_I32, NT, U, 2, 0>(arr, skip, n_rows, n_cols, s);
    return go<G, IDX_I32, NT, U, 1, 0>(arr, skip, n_rows, n_cols, s);
}

template <int G>
hipError_t pick(int idx, bool nt, int U, int R, int probe, const void *const *arr,
                int32_t skip, int32_t n_rows, int32_t n_cols, hipStream_t s) {
    if (probe == 1) return go<G, IDX_I32, false, 4, 1, 1>(arr, skip, n_rows, n_cols, s);
    if (probe == 2) return go<G, IDX_I32, false, 1, 1, 2>(arr, skip, n_rows, n_cols, s);
    if (idx == IDX_I32) {
        if (nt) return U >= 4 ? pick_r<G, true, 4>(R, arr, skip, n_rows, n_cols, s)
                              : pick_r<G, true, 1>(R, arr, skip, n_rows, n_cols, s);
        return U >= 4 ? pick_r<G, false, 4>(R, arr, skip, n_rows, n_cols, s)
                      : pick_r<G, false, 1>(R, arr, skip, n_rows, n_cols, s);
    }
    if (idx == IDX_D16)
        return nt ? go<G, IDX_D16, true, 1, 1, 0>(arr, skip, n_rows, n_cols, s)
                  : go<G, IDX_D16, false, 1, 1, 0>(arr, skip, n_rows, n_cols, s);
    return nt ? go<G, IDX_D8, true, 1, 1, 0>(arr, skip, n_rows, n_cols, s)
              : go<G, IDX_D8, false, 1, 1, 0>(arr, skip, n_rows, n_cols, s);
}

}  // namespace

// arr = {rp, col, codes, val, x, y, instrumentation records, dynamic counters}
#define CSR_CAT2(a, b) a##b
#define CSR_CAT(a, b) CSR_CAT2(a, b)
hipError_t CSR_CAT(launch_rowsplit_s, CSR_STORAGE)(int G, int idx, bool nt, int U, int R,
                                                   int probe, const void *const *arr,
                                                   int32_t skip_above, int32_t n_rows,
                                                   int32_t n_cols, hipStream_t s) {
    switch (G) {
    case 1: return pick<1>(idx, nt, U, R, probe, arr, skip_above, n_rows, n_cols, s);
    case 2: return pick<2>(idx, nt, U, R, probe, arr, skip_above, n_rows, n_cols, s);
    case 4: return pick<4>(idx, nt, U, R, probe, arr, skip_above, n_rows, n_cols, s);
    case 8: return pick<8>(idx, nt, U, R, probe, arr, skip_above, n_rows, n_cols, s);
    case 16: return pick<16>(idx, nt, U, R, probe, arr, skip_above, n_rows, n_cols, s);
    case 32: return pick<32>(idx, nt, U, R, probe, arr, skip_above, n_rows, n_cols, s);
    case 64: return pick<64>(idx, nt, U, R, probe, arr, skip_above, n_rows, n_cols, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace csr
