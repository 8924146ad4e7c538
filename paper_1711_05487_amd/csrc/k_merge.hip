// nnz-balanced merge-path SpMV: the GPU counterpart of the runtime-chosen
// schedule that the optimization pool applies to thread imbalance (Sec. III-E,
// Table II, IMB). The path merges the row ends rp[1..N] with the nonzero
// indices 0..NNZ-1 (a nonzero j is taken before row end i while j < rp[i+1]);
// tile t covers L = 256 * IPT consecutive path items, so every workgroup gets
// the same amount of work whatever the row lengths.
//
// Per tile (one 256-thread workgroup):
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
constexpr int VEC = (S == CSR_VAL_F64) ? 2 : 4;  // elements per vector load (8..16 bytes)

template <class T, int N> struct VecOf { typedef T type __attribute__((ext_vector_type(N))); };
using VV = typename VecOf<V, VEC>::type;
using IV = typename VecOf<int32_t, VEC>::type;

template <int IPT, bool NT, int BS>
__global__ __launch_bounds__(BS) void k_merge(
    const int32_t *__restrict__ rp, const int32_t *__restrict__ col, const V *__restrict__ val,
    const X *__restrict__ x, X *__restrict__ y, const int32_t *__restrict__ tile_i,
    const int32_t *__restrict__ tile_j, A *__restrict__ carry, int32_t n_rows, int64_t per_xcd,
    int64_t n_tiles) {
    constexpr int L = BS * IPT;
    __shared__ int32_t s_end[L];
    __shared__ A s_prod[L];
    __shared__ int32_t s_crow[BS];
    __shared__ A s_cval[BS];

    const int64_t t = xcd_logical_block(per_xcd);
    if (t >= n_tiles) return;
    const int tid = threadIdx.x;
    const int32_t i0 = tile_i[t], i1 = tile_i[t + 1];
    const int32_t j0 = tile_j[t], j1 = tile_j[t + 1];
    const int nre = i1 - i0;   // rows whose end lies in this tile
    const int nnz_t = j1 - j0; // nonzeros of this tile

    // 1. tile-local row ends
    for (int k = tid; k < nre; k += BS) s_end[k] = rp[i0 + k + 1] - j0;

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
            const int rs = ri == 0 ? rp[i0] - j0 : s_end[ri - 1];  // row start (local)
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
        // tile's part; k_merge_fixup adds the earlier tiles' carries.
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
// in tile order) + the part computed by the tile where row r ends.
__global__ __launch_bounds__(kBlock) void k_merge_fixup(const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ tile_i,
                                                        const int32_t *__restrict__ tile_j,
                                                        const A *__restrict__ carry,
                                                        X *__restrict__ y, int32_t n_rows,
                                                        int64_t n_tiles) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < 1 || t >= n_tiles) return;
    const int32_t r = tile_i[t];
    if (r >= n_rows || tile_i[t + 1] == r || rp[r] >= tile_j[t]) return;
    int64_t ta = t - 1;
    while (ta > 0 && tile_i[ta] == r) --ta;  // tile ta ended inside row r, so did ta+1..t-1
    A sum = A(0);
    for (int64_t q = ta; q < t; ++q) sum += carry[q];
    y[r] = (X)(sum + (A)y[r]);
}

template <int IPT, bool NT, int BS>
hipError_t go(const void *const *arr, const int32_t *tile_i, const int32_t *tile_j, void *carry,
              int32_t n_rows, int64_t n_tiles, hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    const XcdGrid g = xcd_grid(n_tiles);
    hipLaunchKernelGGL((k_merge<IPT, NT, BS>), dim3((unsigned)g.launched), dim3(BS), 0, s,
                       (const int32_t *)arr[0], (const int32_t *)arr[1], (const V *)arr[3],
                       (const X *)arr[4], (X *)arr[5], tile_i, tile_j, (A *)carry, n_rows,
                       g.per_xcd, n_tiles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_tiles < 2) return e;
    const unsigned fb = (unsigned)((n_tiles + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_merge_fixup, dim3(fb), dim3(kBlock), 0, s, (const int32_t *)arr[0],
                       tile_i, tile_j, (const A *)carry, (X *)arr[5], n_rows, n_tiles);
    return hipGetLastError();
}

}  // namespace

#define CSR_CAT2(a, b) a##b
#define CSR_CAT(a, b) CSR_CAT2(a, b)
// arr = {rp, col, codes, val, x, y}; L = 256 * ipt
hipError_t CSR_CAT(launch_merge_s, CSR_STORAGE)(int ipt, bool nt, const void *const *arr,
                                                const int32_t *tile_i, const int32_t *tile_j,
                                                void *carry, int32_t n_rows, int64_t n_tiles,
                                                hipStream_t s) {
    switch (ipt) {
    case 4: return nt ? go<4, true, kBlock>(arr, tile_i, tile_j, carry, n_rows, n_tiles, s)
                      : go<4, false, kBlock>(arr, tile_i, tile_j, carry, n_rows, n_tiles, s);
    case 8: return nt ? go<8, true, kBlock>(arr, tile_i, tile_j, carry, n_rows, n_tiles, s)
                      : go<8, false, kBlock>(arr, tile_i, tile_j, carry, n_rows, n_tiles, s);
    case 16: return nt ? go<16, true, kBlock>(arr, tile_i, tile_j, carry, n_rows, n_tiles, s)
                       : go<16, false, kBlock>(arr, tile_i, tile_j, carry, n_rows, n_tiles, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace csr
