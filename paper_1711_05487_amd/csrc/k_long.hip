// Long-row pass of the matrix decomposition (IMB remedy, Sec. III-E, Figs. 5-6):
// rows with more than tau nonzeros are skipped by the row-split pass and
// computed here by many workgroups at once. Each long row is cut into chunks
// of C consecutive nonzeros; one workgroup reduces a chunk in a fixed tree
// order into a partial sum, and a second kernel adds a row's partials in chunk
// order. No floating-point atomics, so results are deterministic.
//
// Compiled once per storage type (-DCSR_STORAGE=0/1/2).
#include "device.h"
#include "internal.h"
#include "long_rows.h"

#ifndef CSR_STORAGE
#error "CSR_STORAGE must be defined"
#endif

namespace csr {
namespace {

constexpr int S = CSR_STORAGE;
using V = typename St<S>::V;
using X = typename St<S>::X;
using A = typename St<S>::A;

// chunk c covers nonzeros [chunk_beg[2c], chunk_beg[2c + 1]) of one long row
__global__ __launch_bounds__(kBlock) void k_long_partial(const int32_t *__restrict__ col,
                                                         const V *__restrict__ val,
                                                         const X *__restrict__ x,
                                                         const int32_t *__restrict__ chunk_beg,
                                                         A *__restrict__ part, int64_t n_chunks) {
    __shared__ A s[kBlock];
    const int64_t c = blockIdx.x;
    if (c >= n_chunks) return;
    long_chunk_partial<S>(c, col, val, x, chunk_beg, part, s);
}

// long row k owns chunks [row_chunk[k], row_chunk[k+1])
__global__ __launch_bounds__(kBlock) void k_long_final(const int32_t *__restrict__ long_rows,
                                                       const int32_t *__restrict__ row_chunk,
                                                       const A *__restrict__ part,
                                                       X *__restrict__ y, int32_t n_long) {
    const int32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n_long) return;
    long_row_final<S>(k, long_rows, row_chunk, part, y);
}

}  // namespace

#define CSR_CAT2(a, b) a##b
#define CSR_CAT(a, b) CSR_CAT2(a, b)
hipError_t CSR_CAT(launch_long_s, CSR_STORAGE)(const int32_t *col, const void *val, const void *x,
                                               void *y, const int32_t *chunk_beg, void *part,
                                               int64_t n_chunks, const int32_t *long_rows,
                                               const int32_t *row_chunk, int32_t n_long,
                                               hipStream_t s) {
    if (n_long == 0) return hipSuccess;
    hipLaunchKernelGGL(k_long_partial, dim3((unsigned)n_chunks), dim3(kBlock), 0, s, col,
                       (const V *)val, (const X *)x, chunk_beg, (A *)part, n_chunks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_long_final, dim3((unsigned)((n_long + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, long_rows, row_chunk, (const A *)part, (X *)y, n_long);
    return hipGetLastError();
}

}  // namespace csr
