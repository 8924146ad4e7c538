// One merge-path tile of y = A x (one wave64 workgroup, L = 64 * IPT path
// items) and the cross-tile fixup of one tile. Shared by the single-matrix
// merge kernel and the batched persistent kernel, so both perform the same
// arithmetic in the same order.
#pragma once

#include "device.h"

namespace csr {

template <class T, int N> struct VecOf { typedef T type __attribute__((ext_vector_type(N))); };
// The same vector with only the element's alignment (for loads at any
// element index; the device runs in unaligned-access mode).
template <class T, int N> struct VecOfU {
    typedef T type __attribute__((ext_vector_type(N), aligned(sizeof(T))));
};

// Orders the LDS accesses of the lanes of one wave. A wave's LDS operations
// complete in issue order, so no wait is needed: only fences that keep the
// compiler from moving memory accesses across this point. Valid because a
// merge tile is exactly one wave.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// DPP lane moves (GFX9 controls). Lanes whose source is outside the row, or
// whose row is masked off, read 0, the identity of the segmented sum below.
enum : int {
    kDppRowShr = 0x110,   // + n: from lane - n within a row of 16
    kDppWaveShr1 = 0x138, // from lane - 1 across the wave
    kDppRowBcast15 = 0x142,
    kDppRowBcast31 = 0x143,
};
template <int CTRL, int ROWS> __device__ __forceinline__ int dpp_move(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, true);
}
template <int CTRL, int ROWS> __device__ __forceinline__ float dpp_move(float v) {
    return __int_as_float(dpp_move<CTRL, ROWS>(__float_as_int(v)));
}
template <int CTRL, int ROWS> __device__ __forceinline__ double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_move<CTRL, ROWS>((int)(uint32_t)b);
    const int hi = dpp_move<CTRL, ROWS>((int)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// One step of the inclusive segmented scan across the wave: combine with the
// (v, h) pair that the DPP move brings, (v1, h1) then (v2, h2) ->
// (h2 ? v2 : v1 + v2, h1 | h2).
template <int CTRL, int ROWS, class A> __device__ __forceinline__ void seg_step(A &v, int &h) {
    const A vu = dpp_move<CTRL, ROWS>(v);
    const int hu = dpp_move<CTRL, ROWS>(h);
    if (!h) v = vu + v;
    h |= hu;
}

// Raw buffer loads through a per-tile range: a lane whose offset lies past
// the range reads zeros and makes no memory access, so windows need no
// address clamping, and constant block offsets fold into the instruction.
constexpr int kBufferWord3 = 0x00020000;  // raw buffer, 32-bit dwords (GFX9 family)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_range(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             kBufferWord3);
}
template <class T, bool NT>
__device__ __forceinline__ T buffer_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    constexpr int aux = NT ? 2 : 0;  // non-temporal
    if constexpr (sizeof(T) == 16)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, aux));
    else if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, aux));
    else if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, aux));
    else {
        static_assert(sizeof(T) == 2, "2, 4, 8 or 16 bytes");
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, aux));
    }
}



// Elements per vector load of the value stream (8..16 bytes per lane).
template <int S> constexpr int merge_vec() { return S == CSR_VAL_F64 ? 2 : 4; }

template <int S, int IPT> struct MergeLds {
    using A = typename St<S>::A;
    static constexpr int BS = kMergeBlock;
    static constexpr int L = BS * IPT;
    static constexpr int STEP = BS * merge_vec<S>();
    static_assert(L % STEP == 0, "a tile is a whole number of load blocks");
    alignas(16) A prod[L];            // products, then their segmented prefix sums
    alignas(16) uint8_t head[L + BS]; // 1 where a row starts inside the tile; [L, L+BS) dummies
};
// Row-aligned tiles need only the products (the x window of window-coded
// tiles and the staged codes share the same buffer, one after the other).
template <int S, int IPT> struct MergeLdsRows {
    alignas(16) typename St<S>::A prod[kMergeBlock * IPT];
};

// Tile t: rows i0 = tile_i[t] .. i1 = tile_i[t+1] end inside it; nonzeros
// j0 = tile_j[t] .. j1 = tile_j[t+1] - 1 belong to it. One wave of BS = 64
// lanes, L = BS * IPT path items.
//
// The tile is reduced as a segmented scan over its nonzeros, with a segment
// starting at every row end that falls inside the tile:
//  1. (merge_issue) the tile's nonzeros are streamed with vector
//     loads, and the row ends of its rows are loaded; every load is issued
//     before the first use;
//  2. (merge_gather) x is gathered at the loaded columns;
//  3. (merge_finish) the products are written to LDS at their position in
//     the tile's window; the row ends mark segment heads in a byte map;
//     lane l scans positions [l*IPT, (l+1)*IPT) in registers, the lanes are
//     joined by a segmented scan across the wave, and the inclusive segment
//     sums go back to LDS; row r of the tile reads the sum at its last
//     nonzero (coalesced y stores), and the segment still open at the tile
//     end is the tile's carry.
// Every sum has a fixed order, so results are deterministic. The first row
// of the tile may have begun in an earlier tile: it gets this tile's part
// here, and merge_fixup_tile adds the earlier tiles' carries.
//
// Row-aligned tiles (the partition cut every tile at a row end) need no
// scan and no carry: the products go to LDS and merge_row_sums gives every
// row a group of lanes that sums it there. Their column codes, if any, are
// either tile-base offsets gathered in window order (merge_issue_rows,
// merge_gather_rows) or window ranks whose x comes from an LDS copy of the
// tile's distinct columns (merge_gather_window).

// Column type of the window: int32 columns, or the w-bit offsets of the
// merge codes (columns = base of the tile + code).
template <int IDX> struct MergeCol { using type = int32_t; };
template <> struct MergeCol<IDX_D16> { using type = uint16_t; };
template <> struct MergeCol<IDX_D8> { using type = uint8_t; };
template <> struct MergeCol<IDX_W8> { using type = uint8_t; };
template <> struct MergeCol<IDX_R8> { using type = uint8_t; };
template <> struct MergeCol<IDX_W9> { using type = uint8_t; };

// Window entries each lane loads (entries lane + 64 k).
template <int IDX> constexpr int window_per_lane() { return IDX == IDX_W9 ? 8 : 4; }

// What a lane holds for one tile between issuing its loads and reducing it.
template <int S, int IPT, int IDX = IDX_I32> struct MergeTileRegs {
    using V = typename St<S>::V;
    using C = typename MergeCol<IDX>::type;
    static constexpr int VEC = merge_vec<S>();
    static constexpr int NIT = IPT / VEC;  // load blocks of STEP = BS * VEC elements
    using VV = typename VecOfU<V, VEC>::type;
    using CV = typename VecOfU<C, VEC>::type;
    int32_t i0, i1, j0, j1;  // the tile's bounds (wave-uniform)
    int32_t last_end;        // rp[i1]: end of the last row ending in the tile
    int32_t base;            // merge codes: the tile's smallest column
    int32_t re[IPT];         // rp[i0 + r + 1] for rows r = lane + q * BS (0 past the
                             // tile's rows; only ceil((i1 - i0) / BS) entries loaded)
    VV vv[NIT];              // values of the tile's window
    CV cv[NIT];              // columns (or codes) of the tile's window
    int32_t wl;              // window codes: entries of the tile's x window
    uint16_t dv[window_per_lane<IDX>()];  // window codes: entries lane + 64 k
    uint32_t hi;             // 9-bit ranks: the lane's ninth-bit mask
    typename VecOf<typename St<S>::X, 4>::type wx;  // run windows: x at entries lane + 64 k
};

// Stage 1: issue the tile's loads. The window [j0, j0 + L) starts at the
// tile's first nonzero and is read in NIT blocks of BS vectors (at element
// alignment) through a buffer range that ends with the last vector holding
// tile nonzeros: lanes past it read zeros (column or code 0, value 0)
// without a memory access, and the last vector reads at most VEC - 1
// elements past j1, a neighbouring tile's or the tail padding. Row ends are
// read through a range holding exactly the tile's rows. Row ends first
// (their count depends on the tile), then columns (needed first), then
// values, so that the wait for each column vector is a fixed count.
// `cols` is the int32 column array, or the merge codes for IDX_D16/D8.
template <int S, int IPT, bool NT, int IDX = IDX_I32>
__device__ __forceinline__ void merge_issue(int64_t t, const int32_t *__restrict__ rp,
                                            const void *__restrict__ cols,
                                            const typename St<S>::V *__restrict__ val,
                                            const int32_t *__restrict__ tile_i,
                                            const int32_t *__restrict__ tile_j,
                                            const int32_t *__restrict__ tile_base,
                                            MergeTileRegs<S, IPT, IDX> &R,
                                            const uint16_t *__restrict__ wdict = nullptr,
                                            const int32_t *__restrict__ wlen = nullptr) {
    using Rg = MergeTileRegs<S, IPT, IDX>;
    using V = typename St<S>::V;
    using C = typename Rg::C;
    constexpr int VEC = Rg::VEC, NIT = Rg::NIT;
    constexpr int BS = kMergeBlock;
    constexpr int STEP = BS * VEC;
    const uint32_t tid = threadIdx.x;
    R.i0 = tile_i[t];
    R.i1 = tile_i[t + 1];
    R.j0 = tile_j[t];
    R.j1 = tile_j[t + 1];
    R.base = IDX == IDX_I32 ? 0 : tile_base[t];
    // elements of the window up to the end of the last vector holding tile
    // nonzeros (a multiple of VEC; 0 for a tile without nonzeros)
    const uint32_t nwin = R.j1 > R.j0 ? ((uint32_t)(R.j1 - 1 - R.j0) & ~(uint32_t)(VEC - 1)) + VEC : 0u;
    // row ends rp[i0 + 1 .. i1]: one load per lane when the tile ends at
    // most BS rows (the common case), else IPT (zeros past the tile's rows)
    const uint32_t nre = (uint32_t)(R.i1 - R.i0);
    const auto rr = buffer_range(rp + R.i0 + 1, nre * (uint32_t)sizeof(int32_t));
    // 9-bit ranks: only the first 64 row ends are held from here (the row
    // sums read the others when a tile ends more than 64 rows), which keeps
    // the kernel's registers, and so its occupancy, down
    if (IDX == IDX_W9 || nre <= (uint32_t)BS) {
        R.re[0] = buffer_load<int32_t, false>(rr, tid * 4u, 0u);
#pragma unroll
        for (int q = 1; q < IPT; ++q) R.re[q] = 0;
    } else {
#pragma unroll
        for (int q = 0; q < IPT; ++q)
            R.re[q] = buffer_load<int32_t, false>(rr, tid * 4u, (uint32_t)(q * BS * 4));
    }
    if constexpr (IDX == IDX_W8 || IDX == IDX_W9) {
        // the window's dictionary entries lane + 64 k: each load reads 64
        // consecutive entries (entries past the window read zero); 9-bit
        // ranks: `wlen` holds the per-tile records (count, then the lanes'
        // ninth-bit masks)
        constexpr int NDV = window_per_lane<IDX>();
        constexpr int WM = IDX == IDX_W9 ? kWideWindowMax : kWindowMax;
        if constexpr (IDX == IDX_W9) {
            R.wl = wlen[t * kWideWords];
            R.hi = reinterpret_cast<const uint16_t *>(wlen + t * kWideWords + 1)[tid];
        } else {
            R.wl = wlen[t];
        }
        const auto rd = buffer_range(wdict + t * WM, (uint32_t)R.wl * 2u);
#pragma unroll
        for (int k = 0; k < NDV; ++k)
            R.dv[k] = buffer_load<uint16_t, NT>(rd, tid * 2u, (uint32_t)(k * kMergeBlock * 2));
    }
    const auto rc = buffer_range(static_cast<const C *>(cols) + R.j0, nwin * (uint32_t)sizeof(C));
    const auto rv = buffer_range(val + R.j0, nwin * (uint32_t)sizeof(V));
#pragma unroll
    for (int it = 0; it < NIT; ++it)
        R.cv[it] = buffer_load<typename Rg::CV, NT>(rc, tid * (uint32_t)(VEC * sizeof(C)),
                                                   (uint32_t)(it * STEP * sizeof(C)));
#pragma unroll
    for (int it = 0; it < NIT; ++it)
        R.vv[it] = buffer_load<typename Rg::VV, NT>(rv, tid * (uint32_t)(VEC * sizeof(V)),
                                                   (uint32_t)(it * STEP * sizeof(V)));
    R.last_end = rp[R.i1];
}

// Stage 2: gather x at the window's columns (all valid: the window holds
// real nonzeros of this tile or its neighbours, or zeroed padding). With
// merge codes, x is read through the range [x + base, x + n_cols): a code
// that is not this tile's (the window's tail) cannot leave x.
template <int S, int IPT, bool X32, int IDX = IDX_I32>
__device__ __forceinline__ void merge_gather(const MergeTileRegs<S, IPT, IDX> &R,
                                             const typename St<S>::X *__restrict__ x,
                                             int32_t n_cols,
                                             typename St<S>::X (&xs)[MergeTileRegs<S, IPT, IDX>::NIT]
                                                                   [MergeTileRegs<S, IPT, IDX>::VEC]) {
    using X = typename St<S>::X;
    constexpr int VEC = MergeTileRegs<S, IPT, IDX>::VEC, NIT = MergeTileRegs<S, IPT, IDX>::NIT;
    if constexpr (IDX != IDX_I32) {
        // a code reaches at most 2^16 - 1 past the base: the range never
        // needs more than 2^16 elements (and stays far below 4 GiB)
        const uint32_t nx = (uint32_t)min(n_cols - R.base, 1 << 16);
        const auto rx = buffer_range(x + R.base, nx * (uint32_t)sizeof(X));
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                xs[it][e] = buffer_load<X, false>(rx, (uint32_t)R.cv[it][e] * (uint32_t)sizeof(X), 0u);
        }
    } else {
        (void)n_cols;
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                if constexpr (X32)  // x spans < 4 GiB: 32-bit byte offsets
                    xs[it][e] = *reinterpret_cast<const X *>(
                        reinterpret_cast<const char *>(x) + (uint32_t)R.cv[it][e] * (uint32_t)sizeof(X));
                else
                    xs[it][e] = x[R.cv[it][e]];
            }
        }
    }
}

// Stage 3: products, segmented scan, rows and carry. With `acc` (a column
// block after the first) the tile's part of each row ending in it is added
// to y, and a row without nonzeros here keeps y; the fixup pass then adds
// the carries as without `acc`. With `rowid` the rows are a list (a column
// block over the rows with nonzeros in it): row r of the list is y's row
// rowid[r].
template <int S, int IPT, class LDS, int IDX = IDX_I32>
__device__ __forceinline__ void merge_finish(int64_t t, MergeTileRegs<S, IPT, IDX> &R,
                                             const typename St<S>::X (&xs)[MergeTileRegs<S, IPT, IDX>::NIT]
                                                                          [MergeTileRegs<S, IPT, IDX>::VEC],
                                             typename St<S>::X *__restrict__ y,
                                             typename St<S>::A *__restrict__ carry,
                                             int32_t n_rows, LDS &lds, bool acc = false,
                                             const int32_t *__restrict__ rowid = nullptr) {
    using X = typename St<S>::X;
    using A = typename St<S>::A;
    constexpr int VEC = MergeTileRegs<S, IPT, IDX>::VEC, NIT = MergeTileRegs<S, IPT, IDX>::NIT;
    using AV = typename VecOf<A, VEC>::type;
    constexpr int BS = kMergeBlock;
    constexpr int L = BS * IPT;
    constexpr int STEP = BS * VEC;
    static_assert(IPT % 4 == 0, "head bytes are cleared and read as 32-bit words");
    A *s_prod = lds.prod;
    uint8_t *s_head = lds.head;
    const int tid = threadIdx.x;
    const int32_t i0 = R.i0, j0 = R.j0;
    const int nre = R.i1 - i0;     // rows whose end lies in this tile (<= L)
    const int nnz_t = R.j1 - j0;   // nonzeros of this tile (<= L)
    constexpr int off = 0;  // window position of the tile's first nonzero
    const int32_t last_end = R.last_end - j0;  // <= 0 if no row ends in the tile

    // 1. products to LDS (positions outside [j0, j1) are never read into a
    //    row or carry sum, so they need no masking; a tile without nonzeros
    //    writes products nobody reads)
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        AV pv;
#pragma unroll
        for (int e = 0; e < VEC; ++e) pv[e] = St<S>::cvt(R.vv[it][e]) * (A)xs[it][e];
        *reinterpret_cast<AV *>(s_prod + it * STEP + tid * VEC) = pv;
    }
    int32_t re[IPT];  // tile-local row ends
#pragma unroll
    for (int q = 0; q < IPT; ++q) re[q] = R.re[q] - j0;

    // 2. segment heads: clear, then mark the end of every row ending inside
    //    the nonzero range (lanes with nothing to mark write their dummy)
#pragma unroll
    for (int w = 0; w < IPT / 4; ++w) reinterpret_cast<uint32_t *>(s_head)[tid * (IPT / 4) + w] = 0;
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q * BS < nre) {
            const bool mark = tid + q * BS < nre && re[q] < nnz_t;
            s_head[mark ? re[q] : L + tid] = 1;
        }
    }
    wave_lds_sync();

    // 3. segmented inclusive scan of positions [tid*IPT, (tid+1)*IPT)
    const int base = tid * IPT;
    A run = A(0);
    bool seen = false;
    A loc[IPT];
    bool pre[IPT];  // position lies before the lane's first head
#pragma unroll
    for (int w = 0; w < IPT / 4; ++w) {
        const uint32_t hw = reinterpret_cast<const uint32_t *>(s_head)[tid * (IPT / 4) + w];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int q = w * 4 + b;
            const A p = s_prod[off + base + q];
            const bool h = (hw >> (8 * b)) & 0xFFu;
            run = h ? p : run + p;
            seen = seen || h;
            loc[q] = run;
            pre[q] = !seen;
        }
    }
    // join the lanes: inclusive segmented scan of the lanes' (tail, head)
    // pairs, within rows of 16 lanes, then across rows; cin = the exclusive
    // value (lane 0 gets 0)
    A v = run;
    int hv = seen;
    seg_step<kDppRowShr + 1, 0xF>(v, hv);
    seg_step<kDppRowShr + 2, 0xF>(v, hv);
    seg_step<kDppRowShr + 4, 0xF>(v, hv);
    seg_step<kDppRowShr + 8, 0xF>(v, hv);
    seg_step<kDppRowBcast15, 0xA>(v, hv);
    seg_step<kDppRowBcast31, 0xC>(v, hv);
    const A cin = dpp_move<kDppWaveShr1, 0xF>(v);
#pragma unroll
    for (int q = 0; q < IPT; ++q) s_prod[off + base + q] = pre[q] ? cin + loc[q] : loc[q];
    wave_lds_sync();

    // 4. rows: y = segment sum at the row's last nonzero, 0 for a row with no
    //    nonzeros in this tile
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q * BS < nre) {
            const int r = tid + q * BS;
            int32_t prev = dpp_move<kDppWaveShr1, 0xF>(re[q]);  // end of row r - 1
            if (q > 0) {
                const int32_t wrap = __builtin_amdgcn_readlane(re[q - 1], BS - 1);
                if (tid == 0) prev = wrap;
            }
            const int32_t start = r == 0 ? 0 : prev;
            const A sum = s_prod[off + max(re[q] - 1, 0)];
            if (r < nre) {
                X *yr = y + (rowid ? rowid[i0 + r] : i0 + r);
                if (re[q] > start) *yr = acc ? (X)((A)*yr + sum) : (X)sum;
                else if (!acc) *yr = X(0);
            }
        }
    }
    // the segment open at the tile end leaves a carry for later tiles
    if (tid == 0 && R.i1 < n_rows)
        carry[t] = nnz_t > max(last_end, 0) ? s_prod[off + nnz_t - 1] : A(0);
}

// Window codes (row-aligned tiles): the tile's x window (its distinct
// columns, at most kWindowMax, or kWideWindowMax with 9-bit ranks) is read
// with four (eight) loads per lane (lane l:
// entries l + 64 k, so that one load covers 64 consecutive entries, which
// are consecutive columns on banded rows and share few cache lines), staged
// in LDS, and every nonzero reads its x there by its rank. The window
// occupies the front of the product buffer, which is overwritten only after
// the last rank has been read.
template <int S, int IPT, int IDX = IDX_W8>
__device__ __forceinline__ typename VecOf<typename St<S>::X, window_per_lane<IDX>()>::type
merge_window_load(const MergeTileRegs<S, IPT, IDX> &R, const typename St<S>::X *__restrict__ x,
                  int32_t n_cols) {
    using X = typename St<S>::X;
    constexpr int NDV = window_per_lane<IDX>();
    static_assert(kWindowMax == 4 * kMergeBlock && kWideWindowMax == 8 * kMergeBlock,
                  "four (eight) window entries per lane");
    // an entry is below 2^16: the range never needs more than 2^16 elements
    const uint32_t nx = (uint32_t)min(n_cols - R.base, 1 << 16);
    const auto rx = buffer_range(x + R.base, nx * (uint32_t)sizeof(X));
    typename VecOf<X, NDV>::type w;
#pragma unroll
    for (int k = 0; k < NDV; ++k) {
        // entries past the window read nothing (an offset past the range)
        const bool in = (int)threadIdx.x + k * kMergeBlock < R.wl;
        w[k] = buffer_load<X, false>(rx, in ? (uint32_t)R.dv[k] * (uint32_t)sizeof(X) : 0x80000000u, 0u);
    }
    return w;
}

template <int S, int IPT, class LDS, int IDX = IDX_W8>
__device__ __forceinline__ void merge_window_stage(
    const MergeTileRegs<S, IPT, IDX> &R,
    const typename VecOf<typename St<S>::X, window_per_lane<IDX>()>::type &w, LDS &lds,
    typename St<S>::X (&xs)[MergeTileRegs<S, IPT, IDX>::NIT][MergeTileRegs<S, IPT, IDX>::VEC]) {
    using X = typename St<S>::X;
    constexpr int VEC = MergeTileRegs<S, IPT, IDX>::VEC, NIT = MergeTileRegs<S, IPT, IDX>::NIT;
    constexpr int NDV = window_per_lane<IDX>();
    static_assert(NDV * kMergeBlock * sizeof(X) <= sizeof(lds.prod),
                  "the window fits the product buffer");
    static_assert(IDX != IDX_W9 || NIT * VEC == 16, "9-bit ranks: 16 elements per lane");
    X *s_win = reinterpret_cast<X *>(lds.prod);
#pragma unroll
    for (int k = 0; k < NDV; ++k) s_win[threadIdx.x + k * kMergeBlock] = w[k];
    wave_lds_sync();
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            uint32_t r = R.cv[it][e];
            if constexpr (IDX == IDX_W9) r |= ((R.hi >> (it * VEC + e)) & 1u) << 8;
            xs[it][e] = s_win[r];
        }
    }
    wave_lds_sync();
}

template <int S, int IPT, class LDS, int IDX = IDX_W8>
__device__ __forceinline__ void merge_gather_window(const MergeTileRegs<S, IPT, IDX> &R,
                                                    const typename St<S>::X *__restrict__ x,
                                                    int32_t n_cols, LDS &lds,
                                                    typename St<S>::X (&xs)[MergeTileRegs<S, IPT, IDX>::NIT]
                                                                          [MergeTileRegs<S, IPT, IDX>::VEC]) {
    merge_window_stage<S, IPT, LDS, IDX>(R, merge_window_load<S, IPT, IDX>(R, x, n_cols), lds, xs);
}

// Run windows (row-aligned tiles, IDX_R8): the tile's record (its smallest
// column, window length, runs of consecutive columns) is read with scalar
// loads first; then every vector load of the tile is issued at once: row
// ends, rank codes, the x window (lane l: entries l + 64 k, each located in
// its run by the wave-uniform run table), values. The x window goes to
// LDS as for window codes, and every nonzero reads x there by its rank.
template <int S, int IPT>
__device__ __forceinline__ void merge_issue_runs(int64_t t, const int32_t *__restrict__ rp,
                                                 const uint8_t *__restrict__ codes,
                                                 const typename St<S>::V *__restrict__ val,
                                                 const typename St<S>::X *__restrict__ x,
                                                 int32_t n_cols, const int32_t *__restrict__ tile_i,
                                                 const int32_t *__restrict__ tile_j,
                                                 const int32_t *__restrict__ runs,
                                                 MergeTileRegs<S, IPT, IDX_R8> &R) {
    using Rg = MergeTileRegs<S, IPT, IDX_R8>;
    using V = typename St<S>::V;
    using X = typename St<S>::X;
    constexpr int VEC = Rg::VEC, NIT = Rg::NIT;
    constexpr int BS = kMergeBlock;
    constexpr int STEP = BS * VEC;
    static_assert(kWindowMax == 4 * kMergeBlock, "four window entries per lane");
    const uint32_t tid = threadIdx.x;
    // the whole record at once (one 64-byte scalar load; records are 64-byte
    // aligned), so no load waits inside the run loop below
    using I4 = typename VecOf<int32_t, 4>::type;
    const I4 *r4 = reinterpret_cast<const I4 *>(runs + t * kRunWords);
    const I4 q0 = r4[0], q1 = r4[1], q2 = r4[2], q3 = r4[3];
    const int32_t rec[kRunWords] = {q0[0], q0[1], q0[2], q0[3], q1[0], q1[1], q1[2], q1[3],
                                    q2[0], q2[1], q2[2], q2[3], q3[0], q3[1], q3[2], q3[3]};
    static_assert(kRunWords == 16, "four 16-byte words per record");
    R.i0 = tile_i[t];
    R.i1 = tile_i[t + 1];
    R.j0 = tile_j[t];
    R.j1 = tile_j[t + 1];
    R.base = rec[0];
    R.wl = rec[1] & 0xFFFF;
    const uint32_t nwin = R.j1 > R.j0 ? ((uint32_t)(R.j1 - 1 - R.j0) & ~(uint32_t)(VEC - 1)) + VEC : 0u;
    const uint32_t nre = (uint32_t)(R.i1 - R.i0);
    const auto rr = buffer_range(rp + R.i0 + 1, nre * (uint32_t)sizeof(int32_t));
    if (nre <= (uint32_t)BS) {
        R.re[0] = buffer_load<int32_t, false>(rr, tid * 4u, 0u);
#pragma unroll
        for (int q = 1; q < IPT; ++q) R.re[q] = 0;
    } else {
#pragma unroll
        for (int q = 0; q < IPT; ++q)
            R.re[q] = buffer_load<int32_t, false>(rr, tid * 4u, (uint32_t)(q * BS * 4));
    }
    const auto rc = buffer_range(codes + R.j0, nwin);
#pragma unroll
    for (int it = 0; it < NIT; ++it)
        R.cv[it] = buffer_load<typename Rg::CV, true>(rc, tid * (uint32_t)VEC, (uint32_t)(it * STEP));
    // window entry k = tid + 64 q lies in run r when k - (entries of runs
    // before r) < length of r; the words past the last run are zero (length
    // 0), so every run slot can be tested; entries past the window read
    // nothing
    uint32_t off[4] = {0x80000000u, 0x80000000u, 0x80000000u, 0x80000000u};
    uint32_t before = 0;
#pragma unroll
    for (int r = 0; r < kRunsMax; ++r) {
        const uint32_t w = (uint32_t)rec[2 + r];
        const uint32_t first = w & 0xFFFFu, len = w >> 16;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t d = tid + (uint32_t)(q * BS) - before;
            if (d < len) off[q] = (first + d) * (uint32_t)sizeof(X);
        }
        before += len;
    }
    // an entry is below 2^16: the range never needs more than 2^16 elements
    const uint32_t nx = (uint32_t)min(n_cols - R.base, 1 << 16);
    const auto rx = buffer_range(x + R.base, nx * (uint32_t)sizeof(X));
#pragma unroll
    for (int q = 0; q < 4; ++q) R.wx[q] = buffer_load<X, false>(rx, off[q], 0u);
    const auto rv = buffer_range(val + R.j0, nwin * (uint32_t)sizeof(V));
#pragma unroll
    for (int it = 0; it < NIT; ++it)
        R.vv[it] = buffer_load<typename Rg::VV, true>(rv, tid * (uint32_t)(VEC * sizeof(V)),
                                                     (uint32_t)(it * STEP * sizeof(V)));
}

// Sum of s[b .. e) in index order, starting from +0.
template <class A> __device__ __forceinline__ A lds_run_sum(const A *s, int b, int e) {
    A v = A(0);
    int p = b;
    for (; p + 4 <= e; p += 4) {
        v += s[p];
        v += s[p + 1];
        v += s[p + 2];
        v += s[p + 3];
    }
    for (; p < e; ++p) v += s[p];
    return v;
}

// Tile-base codes on row-aligned tiles (the partition cut every tile at a
// row end, so each row of the tile has all of its nonzeros in it and
// nothing is carried). The codes are read as one wide vector per lane (lane
// l: window elements [l IPT, (l+1) IPT)) and passed through LDS so that
// gather k reads element 64 k + l: four neighbouring lanes then gather
// consecutive nonzeros, which share cache lines on banded and stencil rows,
// so a gather instruction touches fewer distinct lines than in the values'
// layout. The gathered x goes back through LDS to meet the values, which
// keep their wide loads.
template <int S, int IPT, int IDX = IDX_I32> struct MergeRowRegs {
    using V = typename St<S>::V;
    using C = typename MergeCol<IDX>::type;
    static constexpr int VEC = merge_vec<S>();
    static constexpr int NIT = IPT / VEC;
    static constexpr int CW = IPT * (int)sizeof(C) >= 16 ? 16 / (int)sizeof(C) : IPT;
    static constexpr int NCC = IPT / CW;  // column vectors per lane
    static_assert(IPT % CW == 0, "a lane's columns are a whole number of vectors");
    using VV = typename VecOfU<V, VEC>::type;
    using CC = typename VecOfU<C, CW>::type;
    int32_t i0, i1, j0, j1;  // the tile's bounds (wave-uniform)
    int32_t base;            // merge codes: the tile's smallest column
    int32_t re[IPT];         // rp[i0 + r + 1] for rows r = lane + q * BS, as in MergeTileRegs
    VV vv[NIT];              // values: blocks of BS vectors, as in MergeTileRegs
    CC cc[NCC];              // columns (or codes) of window elements [lane IPT, (lane+1) IPT)
};

template <int S, int IPT, bool NT, int IDX = IDX_I32>
__device__ __forceinline__ void merge_issue_rows(int64_t t, const int32_t *__restrict__ rp,
                                                 const void *__restrict__ cols,
                                                 const typename St<S>::V *__restrict__ val,
                                                 const int32_t *__restrict__ tile_i,
                                                 const int32_t *__restrict__ tile_j,
                                                 const int32_t *__restrict__ tile_base,
                                                 MergeRowRegs<S, IPT, IDX> &R) {
    using Rg = MergeRowRegs<S, IPT, IDX>;
    using V = typename St<S>::V;
    using C = typename Rg::C;
    constexpr int VEC = Rg::VEC, NIT = Rg::NIT, CW = Rg::CW, NCC = Rg::NCC;
    constexpr int BS = kMergeBlock;
    constexpr int STEP = BS * VEC;
    const uint32_t tid = threadIdx.x;
    R.i0 = tile_i[t];
    R.i1 = tile_i[t + 1];
    R.j0 = tile_j[t];
    R.j1 = tile_j[t + 1];
    R.base = IDX == IDX_I32 ? 0 : tile_base[t];
    const uint32_t nnz_t = (uint32_t)(R.j1 - R.j0);
    // value window: whole VEC vectors; column window: whole CW vectors (at
    // most CW - 1 elements past j1, a neighbouring tile's or the padding)
    const uint32_t nwin = nnz_t ? ((nnz_t - 1) & ~(uint32_t)(VEC - 1)) + VEC : 0u;
    const uint32_t ncw = nnz_t ? ((nnz_t - 1) / CW + 1) * CW : 0u;
    const uint32_t nre = (uint32_t)(R.i1 - R.i0);
    const auto rr = buffer_range(rp + R.i0 + 1, nre * (uint32_t)sizeof(int32_t));
    if (nre <= (uint32_t)BS) {
        R.re[0] = buffer_load<int32_t, false>(rr, tid * 4u, 0u);
#pragma unroll
        for (int q = 1; q < IPT; ++q) R.re[q] = 0;
    } else {
#pragma unroll
        for (int q = 0; q < IPT; ++q)
            R.re[q] = buffer_load<int32_t, false>(rr, tid * 4u, (uint32_t)(q * BS * 4));
    }
    const auto rc = buffer_range(static_cast<const C *>(cols) + R.j0, ncw * (uint32_t)sizeof(C));
    const auto rv = buffer_range(val + R.j0, nwin * (uint32_t)sizeof(V));
#pragma unroll
    for (int c = 0; c < NCC; ++c)
        R.cc[c] = buffer_load<typename Rg::CC, NT>(rc, tid * (uint32_t)(IPT * sizeof(C)),
                                                   (uint32_t)(c * CW * sizeof(C)));
#pragma unroll
    for (int it = 0; it < NIT; ++it)
        R.vv[it] = buffer_load<typename Rg::VV, NT>(rv, tid * (uint32_t)(VEC * sizeof(V)),
                                                   (uint32_t)(it * STEP * sizeof(V)));
}

// x at window element k * BS + lane, for k < IPT (the columns pass through
// the LDS buffer, which is free again on return).
template <int S, int IPT, bool X32, int IDX, class LDS>
__device__ __forceinline__ void merge_gather_rows(const MergeRowRegs<S, IPT, IDX> &R,
                                                  const typename St<S>::X *__restrict__ x,
                                                  int32_t n_cols, LDS &lds,
                                                  typename St<S>::X (&xv)[IPT]) {
    using Rg = MergeRowRegs<S, IPT, IDX>;
    using X = typename St<S>::X;
    using C = typename Rg::C;
    constexpr int CW = Rg::CW, NCC = Rg::NCC;
    constexpr int BS = kMergeBlock;
    static_assert(sizeof(C) <= sizeof(lds.prod[0]), "columns fit the product buffer");
    C *s_col = reinterpret_cast<C *>(lds.prod);
    const int tid = threadIdx.x;
#pragma unroll
    for (int c = 0; c < NCC; ++c)
        *reinterpret_cast<typename Rg::CC *>(s_col + tid * IPT + c * CW) = R.cc[c];
    wave_lds_sync();
    C cl[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) cl[k] = s_col[k * BS + tid];
    wave_lds_sync();
    if constexpr (IDX != IDX_I32) {
        // a code reaches at most 2^16 - 1 past the base (see merge_gather)
        const uint32_t nx = (uint32_t)min(n_cols - R.base, 1 << 16);
        const auto rx = buffer_range(x + R.base, nx * (uint32_t)sizeof(X));
#pragma unroll
        for (int k = 0; k < IPT; ++k)
            xv[k] = buffer_load<X, false>(rx, (uint32_t)cl[k] * (uint32_t)sizeof(X), 0u);
    } else {
        (void)n_cols;
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            if constexpr (X32)
                xv[k] = *reinterpret_cast<const X *>(reinterpret_cast<const char *>(x) +
                                                     (uint32_t)cl[k] * (uint32_t)sizeof(X));
            else
                xv[k] = x[cl[k]];
        }
    }
}

// Row sums of a row-aligned tile from its products in LDS (window order).
// With at most 64 rows, every row gets a group of g = 2^k lanes (the
// largest g with g * rows <= 64): lane `sub` of the group sums the sub-th
// contiguous chunk of the row in index order, and the group adds its chunks
// pairwise. With more rows than lanes, lane l sums rows l, l + 64, ...
// alone. `re` holds the row ends as MergeTileRegs does (LAZY: only re[0];
// the others are read from `rp` here). With `acc` the row sums are added to
// y (a column block after the first).
template <int IPT, bool LAZY = false, class A, class X>
__device__ __forceinline__ void merge_row_sums(int32_t i0, int32_t i1, int32_t j0,
                                               const int32_t (&re)[IPT], const A *s_prod,
                                               X *__restrict__ y, bool acc,
                                               const int32_t *__restrict__ rp = nullptr) {
    constexpr int BS = kMergeBlock;
    const int tid = threadIdx.x;
    const int nre = i1 - i0;  // rows of the tile
    X *yb = y + i0;
    if (nre > BS) {
        int32_t rq_prev = 0;  // this lane's row end of the previous round
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            if (q * BS < nre) {
                const int r = tid + q * BS;
                int32_t rq = re[q];
                if constexpr (LAZY)
                    if (q > 0) rq = r < nre ? rp[i0 + 1 + r] : 0;
                const int32_t end = rq - j0;
                int32_t prev = dpp_move<kDppWaveShr1, 0xF>(end);  // end of row r - 1
                if (q > 0) {
                    const int32_t wrap = __builtin_amdgcn_readlane(rq_prev, BS - 1) - j0;
                    if (tid == 0) prev = wrap;
                }
                rq_prev = rq;
                const int32_t start = r == 0 ? 0 : prev;
                if (r < nre) {
                    const A v = lds_run_sum(s_prod, start, end);
                    yb[r] = acc ? (X)((A)yb[r] + v) : (X)v;
                }
            }
        }
    } else if (nre > 0) {
        const int lg = 6 - (nre <= 1 ? 0 : 32 - __clz(nre - 1));  // g * nre <= 64
        const int k = tid >> lg, sub = tid & ((1 << lg) - 1);
        const int32_t e0 = re[0] - j0;
        const int32_t end = __shfl(e0, min(k, nre - 1));
        const int32_t start = __shfl(e0, max(min(k - 1, nre - 1), 0));
        const int32_t b = k == 0 ? 0 : start;
        const int32_t chunk = (end - b + (1 << lg) - 1) >> lg;
        const int32_t cb = min(b + sub * chunk, end);
        A v = lds_run_sum(s_prod, cb, min(cb + chunk, end));
        for (int off = (1 << lg) >> 1; off > 0; off >>= 1) v += __shfl_down(v, off);
        if (sub == 0 && k < nre) yb[k] = acc ? (X)((A)yb[k] + v) : (X)v;
    }
}

// Products of a row-aligned tile whose x was gathered in the values' layout.
template <int S, int IPT, class LDS, int IDX>
__device__ __forceinline__ void merge_finish_rows(const MergeTileRegs<S, IPT, IDX> &R,
                                                  const typename St<S>::X (&xs)[MergeTileRegs<S, IPT, IDX>::NIT]
                                                                               [MergeTileRegs<S, IPT, IDX>::VEC],
                                                  typename St<S>::X *__restrict__ y, LDS &lds,
                                                  bool acc = false,
                                                  const int32_t *__restrict__ rp = nullptr) {
    using A = typename St<S>::A;
    constexpr int VEC = MergeTileRegs<S, IPT, IDX>::VEC, NIT = MergeTileRegs<S, IPT, IDX>::NIT;
    using AV = typename VecOf<A, VEC>::type;
    constexpr int STEP = kMergeBlock * VEC;
    const int tid = threadIdx.x;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        AV pv;
#pragma unroll
        for (int e = 0; e < VEC; ++e) pv[e] = St<S>::cvt(R.vv[it][e]) * (A)xs[it][e];
        *reinterpret_cast<AV *>(lds.prod + it * STEP + tid * VEC) = pv;
    }
    wave_lds_sync();
    merge_row_sums<IPT, IDX == IDX_W9>(R.i0, R.i1, R.j0, R.re, lds.prod, y, acc, rp);
}

// Products of a row-aligned tile whose x was gathered in window order
// (element k * 64 + lane): x goes through LDS to meet the values.
template <int S, int IPT, class LDS, int IDX>
__device__ __forceinline__ void merge_finish_rows(const MergeRowRegs<S, IPT, IDX> &R,
                                                  const typename St<S>::X (&xv)[IPT],
                                                  typename St<S>::X *__restrict__ y, LDS &lds,
                                                  bool acc = false) {
    using X = typename St<S>::X;
    using A = typename St<S>::A;
    constexpr int VEC = MergeRowRegs<S, IPT, IDX>::VEC, NIT = MergeRowRegs<S, IPT, IDX>::NIT;
    using AV = typename VecOf<A, VEC>::type;
    using XV = typename VecOf<X, VEC>::type;
    static_assert(sizeof(X) == sizeof(A), "x is staged in the product buffer");
    constexpr int BS = kMergeBlock;
    constexpr int STEP = BS * VEC;
    A *s_prod = lds.prod;
    X *s_x = reinterpret_cast<X *>(lds.prod);
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < IPT; ++k) s_x[k * BS + tid] = xv[k];
    wave_lds_sync();
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const XV xp = *reinterpret_cast<const XV *>(s_x + it * STEP + tid * VEC);
        AV pv;
#pragma unroll
        for (int e = 0; e < VEC; ++e) pv[e] = St<S>::cvt(R.vv[it][e]) * (A)xp[e];
        *reinterpret_cast<AV *>(s_prod + it * STEP + tid * VEC) = pv;
    }
    wave_lds_sync();
    merge_row_sums<IPT>(R.i0, R.i1, R.j0, R.re, s_prod, y, acc);
}

// One tile, start to end. `cols` is the int32 column array, or the merge
// codes with their tile bases for IDX_D16/D8.
template <int S, int IPT, bool NT, class LDS, bool X32 = false, int IDX = IDX_I32, bool ALN = false>
__device__ __forceinline__ void merge_tile(int64_t t, const int32_t *__restrict__ rp,
                                           const void *__restrict__ cols,
                                           const typename St<S>::V *__restrict__ val,
                                           const typename St<S>::X *__restrict__ x,
                                           typename St<S>::X *__restrict__ y,
                                           const int32_t *__restrict__ tile_i,
                                           const int32_t *__restrict__ tile_j,
                                           typename St<S>::A *__restrict__ carry, int32_t n_rows,
                                           LDS &lds, const int32_t *__restrict__ tile_base = nullptr,
                                           int32_t n_cols = 0,
                                           const uint16_t *__restrict__ wdict = nullptr,
                                           const int32_t *__restrict__ wlen = nullptr,
                                           bool acc = false,
                                           const int32_t *__restrict__ rowid = nullptr) {
    static_assert((IDX != IDX_W8 && IDX != IDX_R8 && IDX != IDX_W9) || ALN,
                  "window codes need row-aligned tiles");
    static_assert(IDX != IDX_W9 || IPT == 16, "9-bit window ranks on tiles of 1,024 items");
    // row lists (`rowid`) only on tiles that are not row-aligned
    if constexpr (ALN) (void)rowid;
    if constexpr (IDX == IDX_R8) {
        // `wlen` holds the tiles' run records
        (void)carry;
        (void)n_rows;
        (void)tile_base;
        (void)wdict;
        MergeTileRegs<S, IPT, IDX> R;
        merge_issue_runs<S, IPT>(t, rp, static_cast<const uint8_t *>(cols), val, x, n_cols, tile_i,
                                 tile_j, wlen, R);
        typename St<S>::X xs[MergeTileRegs<S, IPT, IDX>::NIT][MergeTileRegs<S, IPT, IDX>::VEC];
        merge_window_stage<S, IPT, LDS, IDX>(R, R.wx, lds, xs);
        merge_finish_rows<S, IPT, LDS, IDX>(R, xs, y, lds, acc);
    } else if constexpr (IDX == IDX_W8 || IDX == IDX_W9) {
        (void)carry;
        (void)n_rows;
        MergeTileRegs<S, IPT, IDX> R;
        merge_issue<S, IPT, NT, IDX>(t, rp, cols, val, tile_i, tile_j, tile_base, R, wdict, wlen);
        typename St<S>::X xs[MergeTileRegs<S, IPT, IDX>::NIT][MergeTileRegs<S, IPT, IDX>::VEC];
        merge_gather_window<S, IPT, LDS, IDX>(R, x, n_cols, lds, xs);
        merge_finish_rows<S, IPT, LDS, IDX>(R, xs, y, lds, acc, rp);
    } else if constexpr (ALN && IDX != IDX_I32) {
        // codes: one wide load per lane, gathers in window order
        (void)carry;
        (void)n_rows;
        MergeRowRegs<S, IPT, IDX> R;
        merge_issue_rows<S, IPT, NT, IDX>(t, rp, cols, val, tile_i, tile_j, tile_base, R);
        typename St<S>::X xv[IPT];
        merge_gather_rows<S, IPT, X32, IDX>(R, x, n_cols, lds, xv);
        merge_finish_rows<S, IPT, LDS, IDX>(R, xv, y, lds, acc);
    } else if constexpr (ALN) {
        (void)carry;
        (void)n_rows;
        MergeTileRegs<S, IPT, IDX> R;
        merge_issue<S, IPT, NT, IDX>(t, rp, cols, val, tile_i, tile_j, tile_base, R);
        typename St<S>::X xs[MergeTileRegs<S, IPT, IDX>::NIT][MergeTileRegs<S, IPT, IDX>::VEC];
        merge_gather<S, IPT, X32, IDX>(R, x, n_cols, xs);
        merge_finish_rows<S, IPT, LDS, IDX>(R, xs, y, lds, acc);
    } else {
        MergeTileRegs<S, IPT, IDX> R;
        merge_issue<S, IPT, NT, IDX>(t, rp, cols, val, tile_i, tile_j, tile_base, R);
        typename St<S>::X xs[MergeTileRegs<S, IPT, IDX>::NIT][MergeTileRegs<S, IPT, IDX>::VEC];
        merge_gather<S, IPT, X32, IDX>(R, x, n_cols, xs);
        merge_finish<S, IPT, LDS, IDX>(t, R, xs, y, carry, n_rows, lds, acc, rowid);
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
                                                 int32_t n_rows,
                                                 const int32_t *__restrict__ rowid = nullptr) {
    using X = typename St<S>::X;
    using A = typename St<S>::A;
    if (t < 1) return;
    const int32_t r = tile_i[t];
    if (r >= n_rows || tile_i[t + 1] == r || rp[r] >= tile_j[t]) return;
    // tiles ta..t-1 ended inside row r: ta is the last tile that starts
    // before row r (or 0), found by bisection over the non-decreasing tile
    // rows (a row of a skewed matrix can span hundreds of tiles)
    int64_t lo = 0, hi = t;  // first k in [0, t) with tile_i[k] >= r
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (tile_i[mid] < r) lo = mid + 1;
        else hi = mid;
    }
    const int64_t ta = lo > 0 ? lo - 1 : 0;
    // the carries in tile order; eight loads are issued before their adds
    A sum = A(0);
    int64_t q = ta;
    for (; q + 8 <= t; q += 8) {
        A c[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) c[k] = carry[q + k];
#pragma unroll
        for (int k = 0; k < 8; ++k) sum += c[k];
    }
    for (; q < t; ++q) sum += carry[q];
    X *yr = y + (rowid ? rowid[r] : r);
    *yr = (X)(sum + (A)*yr);
}

}  // namespace csr
