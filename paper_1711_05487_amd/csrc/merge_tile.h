// One merge-path tile of y = A x (one wave64 workgroup, L = 64 * IPT path
// items) and the cross-tile fixup of one tile. Shared by the single-matrix merge kernel
// and the batched persistent kernel, so both perform the same arithmetic in
// the same order.
#pragma once

#include "device.h"

namespace csr {

template <class T, int N> struct VecOf { typedef T type __attribute__((ext_vector_type(N))); };

template <int S, int IPT> struct MergeLds {
    using A = typename St<S>::A;
    static constexpr int BS = kMergeBlock;
    int32_t end[BS * IPT];  // tile-local row ends
    A prod[BS * IPT];       // rounded products of the tile's nonzeros
    int32_t crow[BS];       // per-thread carry row
    A cval[BS];             // per-thread carry value
};

// Tile t: rows i0 = tile_i[t] .. i1 = tile_i[t+1] end inside it; nonzeros
// j0 = tile_j[t] .. j1 = tile_j[t+1] - 1 belong to it. BS = 64 threads,
// L = BS * IPT.
template <int S, int IPT, bool NT, class LDS>
__device__ __forceinline__ void merge_tile(int64_t t, const int32_t *__restrict__ rp,
                                           const int32_t *__restrict__ col,
                                           const typename St<S>::V *__restrict__ val,
                                           const typename St<S>::X *__restrict__ x,
                                           typename St<S>::X *__restrict__ y,
                                           const int32_t *__restrict__ tile_i,
                                           const int32_t *__restrict__ tile_j,
                                           typename St<S>::A *__restrict__ carry, int32_t n_rows,
                                           LDS &lds) {
    using V = typename St<S>::V;
    using X = typename St<S>::X;
    using A = typename St<S>::A;
    constexpr int VEC = (S == CSR_VAL_F64) ? 2 : 4;  // elements per vector load (8..16 bytes)
    using VV = typename VecOf<V, VEC>::type;
    using IV = typename VecOf<int32_t, VEC>::type;
    constexpr int BS = kMergeBlock;
    constexpr int L = BS * IPT;
    int32_t *s_end = lds.end;
    A *s_prod = lds.prod;
    int32_t *s_crow = lds.crow;
    A *s_cval = lds.cval;

    const int tid = threadIdx.x;
    const int32_t i0 = tile_i[t], i1 = tile_i[t + 1];
    const int32_t j0 = tile_j[t], j1 = tile_j[t + 1];
    const int nre = i1 - i0;   // rows whose end lies in this tile
    const int nnz_t = j1 - j0; // nonzeros of this tile

    // 1. the row ends of the rows finishing in the tile (k < nre <= L, so
    //    IPT per thread) and the start of the first row: loads issued now,
    //    written to LDS only after the nonzero loads below are in flight
    int32_t re[IPT];
#pragma unroll
    for (int q = 0; q < IPT; ++q) re[q] = rp[min(i0 + tid + q * BS + 1, i1)];
    const int32_t rs_first = rp[i0] - j0;  // start of row i0 (local), <= 0

    // 2. products, with aligned vector loads covering [j0, j1). Addresses are
    //    clamped to the last needed vector so that every load can be issued
    //    unconditionally (all of them in flight before the first use); lanes
    //    outside [j0, j1) gather x[0] and discard the product.
    if (nnz_t > 0) {
        constexpr int STEP = BS * VEC;
        constexpr int NIT = L / STEP + 1;
        const int32_t a = j0 & ~(VEC - 1);
        const int32_t alast = (j1 - 1) & ~(VEC - 1);
        VV vv[NIT];
        IV cv[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int32_t kc = min(a + it * STEP + tid * VEC, alast);
            vv[it] = ld<NT>(reinterpret_cast<const VV *>(val + kc));
            cv[it] = ld<NT>(reinterpret_cast<const IV *>(col + kc));
        }
        X xs[NIT][VEC];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const int32_t k = a + it * STEP + tid * VEC + e;
                const bool ok = k >= j0 && k < j1;
                xs[it][e] = x[ok ? cv[it][e] : 0];
            }
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const int32_t k = a + it * STEP + tid * VEC + e;
                if (k >= j0 && k < j1) s_prod[k - j0] = St<S>::cvt(vv[it][e]) * (A)xs[it][e];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int k = tid + q * BS;
        if (k < nre) s_end[k] = re[q] - j0;
    }
    __syncthreads();

    // 3. walk this thread's IPT path items
    const int total = nre + nnz_t;
    const int d0 = min(tid * IPT, total);
    const int d1 = min(d0 + IPT, total);
    int lo = max(0, d0 - nnz_t), hi = min(d0, nre);
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s_end[mid] + mid < d0) lo = mid + 1;
        else hi = mid;
    }
    int ri = lo, nj = d0 - lo;
    const int ri0 = ri, nj0 = nj;
    A acc = A(0);
    bool open = false;  // first emitted row started before this thread
    A open_val = A(0);
    for (int d = d0; d < d1; ++d) {
        if (ri < nre && nj >= s_end[ri]) {
            const int rs = ri == 0 ? rs_first : s_end[ri - 1];  // row start (local)
            if (ri == ri0 && rs < nj0) {
                open = true;
                open_val = acc;
            } else {
                y[i0 + ri] = (X)acc;
            }
            acc = A(0);
            ++ri;
        } else {
            acc += s_prod[nj];
            ++nj;
        }
    }
    s_crow[tid] = ri;
    s_cval[tid] = acc;
    __syncthreads();

    // 4a. a row opened by earlier threads: their carries (in thread order), then ours
    if (open) {
        int ta = tid;
        while (ta > 0 && s_crow[ta - 1] == ri0) --ta;
        A sum = A(0);
        for (int q = ta; q < tid; ++q) sum += s_cval[q];
        sum += open_val;
        // For the tile's first row begun in an earlier tile this is only the
        // tile's part; the fixup adds the earlier tiles' carries.
        y[i0 + ri0] = (X)sum;
    }
    // 4b. the row still open at the tile end leaves a carry for later tiles
    if (tid == BS - 1 && i1 < n_rows) {
        int tb = BS;
        while (tb > 0 && s_crow[tb - 1] == nre) --tb;
        A sum = A(0);
        for (int q = tb; q < BS; ++q) sum += s_cval[q];
        carry[t] = sum;
    }
}

// Rows spanning tiles: y[r] = (carries of the tiles that ended inside row r,
// in tile order) + the part computed by the tile where row r ends. One call
// per tile t >= 1 (tile 0 never needs it).
template <int S>
__device__ __forceinline__ void merge_fixup_tile(int64_t t, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ tile_i,
                                                 const int32_t *__restrict__ tile_j,
                                                 const typename St<S>::A *__restrict__ carry,
                                                 typename St<S>::X *__restrict__ y,
                                                 int32_t n_rows) {
    using X = typename St<S>::X;
    using A = typename St<S>::A;
    if (t < 1) return;
    const int32_t r = tile_i[t];
    if (r >= n_rows || tile_i[t + 1] == r || rp[r] >= tile_j[t]) return;
    int64_t ta = t - 1;
    while (ta > 0 && tile_i[ta] == r) --ta;  // tile ta ended inside row r, so did ta+1..t-1
    A sum = A(0);
    for (int64_t q = ta; q < t; ++q) sum += carry[q];
    y[r] = (X)(sum + (A)y[r]);
}

}  // namespace csr
