// Batched SpMV, row-split classes: the row blocks of every matrix whose plan
// is the same row-split instance (lanes per row G, index encoding,
// streaming, accumulators U, rows in flight R), in one persistent launch.
// Workgroup b takes items b, b + nblk, ...; every item is one logical block
// of its matrix run by the single-matrix kernel's block code, so the result
// is bit-identical to the matrix's own csr_spmv (whose static and dynamic
// schedules give the same bits too).
//
// Compiled once per storage type (-DCSR_STORAGE=0/1/2).
#include "batch.h"
#include "rowsplit_block.h"

#ifndef CSR_STORAGE
#error "CSR_STORAGE must be defined"
#endif

namespace csr {
namespace {

constexpr int S = CSR_STORAGE;
using V = typename St<S>::V;
using X = typename St<S>::X;

template <int G, int IDX, bool NT, int U, int R>
__global__ __launch_bounds__(kBlock) void k_brows(const BatchMat *__restrict__ mats,
                                                  const int32_t *__restrict__ item_mat,
                                                  int64_t n_items, int64_t per_xcd, int64_t nblk) {
    const int64_t lb = xcd_logical_block(per_xcd);
    if (lb >= nblk) return;
    for (int64_t g = lb; g < n_items; g += nblk) {
        const BatchMat &M = mats[item_mat[g]];
        rowsplit_block<S, G, IDX, NT, U, R, 0>(g - M.item_base, M.rp, M.col, M.codes,
                                               (const V *)M.val, (const X *)M.x, (X *)M.y,
                                               M.skip_above, M.n_rows, M.n_cols);
    }
}

template <int G, int IDX, bool NT, int U, int R>
hipError_t go(const BatchMat *mats, const int32_t *item_mat, int64_t n_items, int n_cu,
              hipStream_t s) {
    auto kern = k_brows<G, IDX, NT, U, R>;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const XcdGrid g = xcd_grid(std::min<int64_t>(n_items, (int64_t)n_cu * per_cu));
    hipLaunchKernelGGL(kern, dim3((unsigned)g.launched), dim3(kBlock), 0, s, mats, item_mat,
                       n_items, g.per_xcd, g.nblk);
    return hipGetLastError();
}

// the single-matrix path's instance choice (R >= 4 -> 4, R == 2 -> 2, else
// 1; U >= 4 -> 4, else 1; delta codes with U = R = 1)
template <int G, bool NT, int U>
hipError_t pick_r(int R, const BatchMat *m, const int32_t *im, int64_t n, int n_cu, hipStream_t s) {
    if (R >= 4) return go<G, IDX_I32, NT, U, 4>(m, im, n, n_cu, s);
    if (R == 2) return go<G, IDX_I32, NT, U, 2>(m, im, n, n_cu, s);
    return go<G, IDX_I32, NT, U, 1>(m, im, n, n_cu, s);
}

template <int G>
hipError_t pick(int idx, bool nt, int U, int R, const BatchMat *m, const int32_t *im, int64_t n,
                int n_cu, hipStream_t s) {
    if (idx == IDX_I32) {
        if (nt) return U >= 4 ? pick_r<G, true, 4>(R, m, im, n, n_cu, s)
                              : pick_r<G, true, 1>(R, m, im, n, n_cu, s);
        return U >= 4 ? pick_r<G, false, 4>(R, m, im, n, n_cu, s)
                      : pick_r<G, false, 1>(R, m, im, n, n_cu, s);
    }
    if (idx == IDX_D16)
        return nt ? go<G, IDX_D16, true, 1, 1>(m, im, n, n_cu, s)
                  : go<G, IDX_D16, false, 1, 1>(m, im, n, n_cu, s);
    if (idx == IDX_D8)
        return nt ? go<G, IDX_D8, true, 1, 1>(m, im, n, n_cu, s)
                  : go<G, IDX_D8, false, 1, 1>(m, im, n, n_cu, s);
    return hipErrorInvalidValue;
}

}  // namespace

#define CSR_CAT2(a, b) a##b
#define CSR_CAT(a, b) CSR_CAT2(a, b)
hipError_t CSR_CAT(launch_brows_s, CSR_STORAGE)(int G, int idx, bool nt, int U, int R,
                                                const BatchMat *mats, const int32_t *item_mat,
                                                int64_t n_items, int n_cu, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    switch (G) {
    case 1: return pick<1>(idx, nt, U, R, mats, item_mat, n_items, n_cu, s);
    case 2: return pick<2>(idx, nt, U, R, mats, item_mat, n_items, n_cu, s);
    case 4: return pick<4>(idx, nt, U, R, mats, item_mat, n_items, n_cu, s);
    case 8: return pick<8>(idx, nt, U, R, mats, item_mat, n_items, n_cu, s);
    case 16: return pick<16>(idx, nt, U, R, mats, item_mat, n_items, n_cu, s);
    case 32: return pick<32>(idx, nt, U, R, mats, item_mat, n_items, n_cu, s);
    case 64: return pick<64>(idx, nt, U, R, mats, item_mat, n_items, n_cu, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace csr
