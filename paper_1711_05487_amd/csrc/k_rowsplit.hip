// Row-split CSR SpMV (Sec. II, Fig. 2 and the static row partitioning of
// Sec. IV-A), the baseline of the method and the carrier of three remedies of
// Sec. III-E, Table II: delta-decoded column indices (MB), streamed val/col
// (ML) and unrolled independent accumulators with several rows per wave (CMP).
//
// G lanes of a wave64 share one row (G in 1..64, so 64/G rows per wave). Each
// lane walks the row with stride G (U independent accumulators, stride G*U),
// then the G partial sums are combined by a fixed butterfly. A workgroup of
// 256 threads owns `rows_iter` consecutive chunks of 256/G rows; workgroups
// are remapped so each XCD's L2 sees a contiguous block of rows.
//
// This file is compiled once per storage type (-DCSR_STORAGE=0/1/2).
#include "device.h"

#ifndef CSR_STORAGE
#error "CSR_STORAGE must be defined"
#endif

namespace csr {
namespace {

constexpr int S = CSR_STORAGE;
using V = typename St<S>::V;
using X = typename St<S>::X;
using A = typename St<S>::A;

template <int G, int IDX, bool NT, int U>
__global__ __launch_bounds__(kBlock) void k_rowsplit(
    const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const void *__restrict__ codes, const V *__restrict__ val, const X *__restrict__ x,
    X *__restrict__ y, int32_t skip_above, int32_t n_rows, int32_t rows_iter,
    int64_t per_xcd, int64_t nblk) {
    const int64_t lb = xcd_logical_block(per_xcd);
    if (lb >= nblk) return;
    constexpr int NG = kBlock / G;
    const int lane = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    const int64_t first = lb * (int64_t)NG * rows_iter;
    for (int k = 0; k < rows_iter; ++k) {
        const int64_t slot = first + (int64_t)k * NG + grp;
        const bool live = slot < n_rows;
        const int32_t row = (int32_t)slot;
        int32_t b = 0, e = 0;
        if (live) {
            b = rp[row];
            e = rp[row + 1];
        }
        // Decomposition: rows longer than skip_above belong to the long-row
        // pass, which writes their y.
        const bool mine = live && (e - b) <= skip_above;
        if (!mine) e = b;
        A acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = A(0);
        if constexpr (IDX == IDX_I32) {
            for (int32_t j = b + lane; j < e; j += G * U) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int32_t jj = j + u * G;
                    if (jj < e) {
                        const int32_t c = ld<NT>(col + jj);
                        const V v = ld<NT>(val + jj);
                        acc[u] = fma_acc(St<S>::cvt(v), (A)x[c], acc[u]);
                    }
                }
            }
        } else {
            // Delta decode: per chunk of G entries, an inclusive scan of the
            // codes inside the lane group, added to the last column of the
            // previous chunk. The chunk loop bound is uniform in the group.
            int32_t base = 0;
            for (int32_t j0 = b; j0 < e; j0 += G) {
                const int32_t j = j0 + lane;
                const bool ok = j < e;
                int32_t v = 0;
                if (ok) {
                    v = load_code<IDX>(codes, j, j == b);
                    if (j == b) v += row;
                }
                const int32_t s = group_scan<G>(v, lane);
                const int32_t c = base + s;
                base += __shfl(s, G - 1, G);
                if (ok) {
                    const V vv = ld<NT>(val + j);
                    acc[0] = fma_acc(St<S>::cvt(vv), (A)x[c], acc[0]);
                }
            }
        }
        A t = acc[0];
#pragma unroll
        for (int u = 1; u < U; ++u) t += acc[u];
        t = group_sum<G>(t);
        if (mine && lane == 0) y[row] = (X)t;
    }
}

template <int G, int IDX, bool NT, int U>
hipError_t go(const void *const *arr, int32_t skip_above, int32_t n_rows, int32_t rows_iter,
              hipStream_t s) {
    constexpr int NG = kBlock / G;
    const int64_t rows_per_blk = (int64_t)NG * rows_iter;
    const XcdGrid g = xcd_grid((n_rows + rows_per_blk - 1) / rows_per_blk);
    if (g.nblk == 0) return hipSuccess;
    hipLaunchKernelGGL((k_rowsplit<G, IDX, NT, U>), dim3((unsigned)g.launched), dim3(kBlock), 0, s,
                       (const int32_t *)arr[0], (const int32_t *)arr[1], arr[2],
                       (const V *)arr[3], (const X *)arr[4], (X *)arr[5], skip_above, n_rows,
                       rows_iter, g.per_xcd, g.nblk);
    return hipGetLastError();
}

template <int G>
hipError_t pick(int idx, bool nt, int U, const void *const *arr, int32_t skip_above,
                int32_t n_rows, int32_t rows_iter, hipStream_t s) {
    if (idx == IDX_I32) {
        if (nt) return U >= 4 ? go<G, IDX_I32, true, 4>(arr, skip_above, n_rows, rows_iter, s)
                              : go<G, IDX_I32, true, 1>(arr, skip_above, n_rows, rows_iter, s);
        return U >= 4 ? go<G, IDX_I32, false, 4>(arr, skip_above, n_rows, rows_iter, s)
                      : go<G, IDX_I32, false, 1>(arr, skip_above, n_rows, rows_iter, s);
    }
    if (idx == IDX_D16)
        return nt ? go<G, IDX_D16, true, 1>(arr, skip_above, n_rows, rows_iter, s)
                  : go<G, IDX_D16, false, 1>(arr, skip_above, n_rows, rows_iter, s);
    return nt ? go<G, IDX_D8, true, 1>(arr, skip_above, n_rows, rows_iter, s)
              : go<G, IDX_D8, false, 1>(arr, skip_above, n_rows, rows_iter, s);
}

}  // namespace

// arr = {rp, col, codes, val, x, y}
#define CSR_CAT2(a, b) a##b
#define CSR_CAT(a, b) CSR_CAT2(a, b)
hipError_t CSR_CAT(launch_rowsplit_s, CSR_STORAGE)(int G, int idx, bool nt, int U,
                                                   const void *const *arr,
                                                   int32_t skip_above, int32_t n_rows,
                                                   int32_t rows_iter, hipStream_t s) {
    switch (G) {
    case 1: return pick<1>(idx, nt, U, arr, skip_above, n_rows, rows_iter, s);
    case 2: return pick<2>(idx, nt, U, arr, skip_above, n_rows, rows_iter, s);
    case 4: return pick<4>(idx, nt, U, arr, skip_above, n_rows, rows_iter, s);
    case 8: return pick<8>(idx, nt, U, arr, skip_above, n_rows, rows_iter, s);
    case 16: return pick<16>(idx, nt, U, arr, skip_above, n_rows, rows_iter, s);
    case 32: return pick<32>(idx, nt, U, arr, skip_above, n_rows, rows_iter, s);
    case 64: return pick<64>(idx, nt, U, arr, skip_above, n_rows, rows_iter, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace csr
