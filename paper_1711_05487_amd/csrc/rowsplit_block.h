// The row-split CSR SpMV of one logical block of rows (Sec. II, Fig. 2;
// the static row partitioning of Sec. IV-A), shared by the single-matrix
// kernel and the batched one so that a matrix gets the same bits either way.
//
// G lanes of a wave64 share one row (G in 1..64, so 64/G rows per wave). A
// lane group owns R rows at once: the first G*U entries of all R rows are
// loaded before any of them is used (R*U independent loads in flight per
// lane), longer rows finish in a tail loop, and the G partial sums of each row
// are combined by a fixed butterfly. A logical block is R chunks of 256/G
// consecutive rows (one 256-thread workgroup). Rows longer than skip_above
// are left to the long-row pass of the decomposition. PROBE = 1: the P_CMP
// micro-benchmark (no column stream, x read at the row index).
#pragma once

#include "device.h"

namespace csr {

template <int S, int G, int IDX, bool NT, int U, int R, int PROBE>
__device__ __forceinline__ void rowsplit_block(int64_t lb, const int32_t *__restrict__ rp,
                                               const int32_t *__restrict__ col,
                                               const void *__restrict__ codes,
                                               const typename St<S>::V *__restrict__ val,
                                               const typename St<S>::X *__restrict__ x,
                                               typename St<S>::X *__restrict__ y,
                                               int32_t skip_above, int32_t n_rows,
                                               int32_t n_cols) {
    using V = typename St<S>::V;
    using X = typename St<S>::X;
    using A = typename St<S>::A;
    constexpr int NG = kBlock / G;
    const int lane = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    const int64_t first = lb * (int64_t)NG * R;

    int32_t row[R], b[R], e[R];
    bool mine[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int64_t slot = first + (int64_t)k * NG + grp;
        const bool live = slot < n_rows;
        row[k] = live ? (int32_t)slot : 0;
        b[k] = live ? rp[row[k]] : 0;
        e[k] = live ? rp[row[k] + 1] : 0;
        // Decomposition: rows longer than skip_above belong to the long-row
        // pass, which writes their y.
        mine[k] = live && (e[k] - b[k]) <= skip_above;
        if (!mine[k]) e[k] = b[k];
    }
    A acc[R][U];
#pragma unroll
    for (int k = 0; k < R; ++k)
#pragma unroll
        for (int u = 0; u < U; ++u) acc[k][u] = A(0);

    if constexpr (IDX == IDX_I32) {
        // first G*U entries of every row: all loads issued before any use
        int32_t c[R][U];
        V v[R][U];
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t jj = b[k] + lane + u * G;
                const bool ok = jj < e[k];
                if constexpr (PROBE == 1) c[k][u] = min(row[k], n_cols - 1);
                else c[k][u] = ok ? ld<NT>(col + jj) : 0;
                v[k][u] = ok ? ld<NT>(val + jj) : V(0);
            }
        X xv[R][U];
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool ok = b[k] + lane + u * G < e[k];
                xv[k][u] = ok ? x[c[k][u]] : X(0);
            }
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
            for (int u = 0; u < U; ++u)
                acc[k][u] = fma_acc(St<S>::cvt(v[k][u]), (A)xv[k][u], acc[k][u]);
        // tails of rows longer than G*U
#pragma unroll
        for (int k = 0; k < R; ++k) {
            for (int32_t j = b[k] + lane + G * U; j < e[k]; j += G * U) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int32_t jj = j + u * G;
                    if (jj < e[k]) {
                        const int32_t cc = PROBE == 1 ? min(row[k], n_cols - 1) : ld<NT>(col + jj);
                        acc[k][u] = fma_acc(St<S>::cvt(ld<NT>(val + jj)), (A)x[cc], acc[k][u]);
                    }
                }
            }
        }
    } else {
        // Delta decode: per chunk of G entries, an inclusive scan of the codes
        // inside the lane group, added to the last column of the previous
        // chunk. The chunk loop bound is uniform in the group.
#pragma unroll
        for (int k = 0; k < R; ++k) {
            int32_t base = 0;
            for (int32_t j0 = b[k]; j0 < e[k]; j0 += G) {
                const int32_t j = j0 + lane;
                const bool ok = j < e[k];
                int32_t v = 0;
                if (ok) {
                    v = load_code<IDX>(codes, j, j == b[k]);
                    if (j == b[k]) v += row[k];
                }
                const int32_t s = group_scan<G>(v, lane);
                const int32_t c = base + s;
                base += __shfl(s, G - 1, G);
                if (ok) {
                    const V vv = ld<NT>(val + j);
                    acc[k][0] = fma_acc(St<S>::cvt(vv), (A)x[c], acc[k][0]);
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        A t = acc[k][0];
#pragma unroll
        for (int u = 1; u < U; ++u) t += acc[k][u];
        t = group_sum<G>(t);
        if (mine[k] && lane == 0) y[row[k]] = (X)t;
    }
}

}  // namespace csr
