// The long-row pass of the matrix decomposition (IMB remedy, Sec. III-E,
// Figs. 5-6), shared by the single-matrix kernels and the batched ones so
// that a matrix gets the same bits either way. Each long row is cut into
// chunks of consecutive nonzeros; one 256-thread workgroup reduces a chunk in
// a fixed tree order into a partial sum (long_chunk_partial), and the
// partials of a row are added in chunk order (long_row_final). No
// floating-point atomics, so results are deterministic.
#pragma once

#include "device.h"

namespace csr {

// chunk c covers nonzeros [chunk_beg[2c], chunk_beg[2c + 1]) of one long row;
// s: kBlock accumulators in LDS
template <int S>
__device__ __forceinline__ void long_chunk_partial(int64_t c, const int32_t *__restrict__ col,
                                                   const typename St<S>::V *__restrict__ val,
                                                   const typename St<S>::X *__restrict__ x,
                                                   const int32_t *__restrict__ chunk_beg,
                                                   typename St<S>::A *__restrict__ part,
                                                   typename St<S>::A *s) {
    using A = typename St<S>::A;
    const int32_t b = chunk_beg[2 * c], e = chunk_beg[2 * c + 1];
    A acc = A(0);
    for (int32_t j = b + threadIdx.x; j < e; j += kBlock)
        acc = fma_acc(St<S>::cvt(__builtin_nontemporal_load(val + j)),
                      (A)x[__builtin_nontemporal_load(col + j)], acc);
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[c] = s[0];
}

// long row k owns chunks [row_chunk[k], row_chunk[k + 1])
template <int S>
__device__ __forceinline__ void long_row_final(int32_t k, const int32_t *__restrict__ long_rows,
                                               const int32_t *__restrict__ row_chunk,
                                               const typename St<S>::A *__restrict__ part,
                                               typename St<S>::X *__restrict__ y) {
    using A = typename St<S>::A;
    using X = typename St<S>::X;
    A sum = A(0);
    for (int32_t c = row_chunk[k]; c < row_chunk[k + 1]; ++c) sum += part[c];
    y[long_rows[k]] = (X)sum;
}

}  // namespace csr
