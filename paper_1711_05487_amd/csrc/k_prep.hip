// Ingest kernels (CSR validation, value-precision conversion) and the B_max
// probe (a STREAM-style triad, Sec. IV-A, Table III).
#include <type_traits>

#include "device.h"
#include "internal.h"

namespace csr {
namespace {

// One wave per row, grid-stride. Flags (integer atomics only):
//   1 row_ptr[0] != 0 or row_ptr[n_rows] != nnz
//   2 row_ptr decreasing or outside [0, nnz]
//   4 a column outside [0, n_cols)
//   8 a row that is not strictly increasing (a property, not an error)
// A row whose bounds are invalid is not read, so malformed input never sends
// a load out of the arrays' bounds.
__global__ __launch_bounds__(kBlock) void k_validate(const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     int32_t n_rows, int32_t n_cols, int64_t nnz,
                                                     int32_t *__restrict__ flags) {
    const int lane = threadIdx.x % kWave;
    const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kBlock / kWave;
    if (wave == 0 && lane == 0) {
        if (rp[0] != 0 || (int64_t)rp[n_rows] != nnz) atomicOr(flags, 1);
    }
    int32_t longest = 0;  // this wave's longest row; one atomic per wave at the end
    for (int64_t r = wave; r < n_rows; r += nwaves) {
        const int32_t b = rp[r], e = rp[r + 1];
        if (e < b || b < 0 || (int64_t)e > nnz) {
            if (lane == 0) atomicOr(flags, 2);
            continue;
        }
        longest = max(longest, e - b);
        bool bad = false, unsorted = false;
        for (int32_t j = b + lane; j < e; j += kWave) {
            const int32_t c = col[j];
            if (c < 0 || c >= n_cols) bad = true;
            if (j > b && col[j - 1] >= c) unsorted = true;
        }
        const uint64_t mb = __ballot(bad), mu = __ballot(unsorted);
        if (lane == 0 && (mb | mu)) atomicOr(flags, (mb ? 4 : 0) | (mu ? 8 : 0));
    }
    if (lane == 0 && longest > 0) atomicMax(flags + 1, longest);
}

// FP64 -> BF16 with one round-to-nearest-even step, from the IEEE-754 binary64
// fields: keep 8 significant bits (7 stored) at the exponent's BF16 quantum,
// round on the discarded bits (ties to an even kept part), renormalize a carry
// out of the significand, saturate to infinity above the largest finite value.
__device__ __forceinline__ uint16_t f64_to_bf16(double d) {
    const uint64_t b = (uint64_t)__double_as_longlong(d);
    const uint16_t sign = (uint16_t)((b >> 48) & 0x8000u);
    const int E = (int)((b >> 52) & 0x7FF);
    const uint64_t m = b & 0xFFFFFFFFFFFFFull;
    if (E == 0x7FF) return m ? (uint16_t)(sign | 0x7FC0u) : (uint16_t)(sign | 0x7F80u);
    if (E == 0) return sign;  // |d| < 2^-1022: far below half the smallest BF16 step
    const int e = E - 1023;
    const uint64_t sig = m | (1ull << 52);  // 53-bit significand, value sig * 2^(e-52)
    int shift;                              // bits of sig below the BF16 quantum
    int ebias;                              // BF16 exponent field if no carry
    if (e >= -126) {
        shift = 45;                          // keep 8 bits
        ebias = e + 127;
    } else {
        shift = -e - 81;                     // quantum 2^-133: sig * 2^(e+81)
        ebias = 0;
        if (shift > 60) return sign;         // below 2^-134 even before rounding
    }
    uint64_t q = sig >> shift;
    const uint64_t rem = sig & ((1ull << shift) - 1);
    const uint64_t half = 1ull << (shift - 1);
    if (rem > half || (rem == half && (q & 1))) q += 1;
    if (ebias == 0) {
        // subnormal result; q <= 128, and q == 128 is exactly the smallest
        // normal (exponent field 1, fraction 0), which the same bits encode
        return (uint16_t)(sign | (uint16_t)q);
    }
    if (q == 256) {  // rounding carried into the next binade
        q = 128;
        ebias += 1;
    }
    if (ebias >= 255) return (uint16_t)(sign | 0x7F80u);
    return (uint16_t)(sign | (uint16_t)(ebias << 7) | (uint16_t)(q & 0x7F));
}

__global__ __launch_bounds__(kBlock) void k_convert(const double *__restrict__ src,
                                                    void *__restrict__ dst, int64_t n,
                                                    int storage) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const double v = src[i];
        if (storage == CSR_VAL_F64) static_cast<double *>(dst)[i] = v;
        else if (storage == CSR_VAL_F32) static_cast<float *>(dst)[i] = (float)v;
        else static_cast<uint16_t *>(dst)[i] = f64_to_bf16(v);
    }
}

typedef double dvec2 __attribute__((ext_vector_type(2)));

// Delta codes (MB remedy, Sec. III-E): entry j of row r stores col[j] - r
// (signed, first entry) or col[j] - col[j-1] (unsigned, >= 1) in `bits` bits.
// Flag 1 is raised when some entry does not fit; the codes are then unusable.
template <int BITS>
__global__ __launch_bounds__(kBlock) void k_delta_encode(const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ col,
                                                         int32_t n_rows, void *__restrict__ codes,
                                                         int32_t *__restrict__ flags) {
    const int lane = threadIdx.x % kWave;
    const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kBlock / kWave;
    constexpr int64_t smin = -(1ll << (BITS - 1)), smax = (1ll << (BITS - 1)) - 1;
    constexpr int64_t umax = (1ll << BITS) - 1;
    bool bad = false;  // accumulated over all rows of this wave: one atomic at most
    for (int64_t r = wave; r < n_rows; r += nwaves) {
        const int32_t b = rp[r], e = rp[r + 1];
        for (int32_t j = b + lane; j < e; j += kWave) {
            const int64_t d = (j == b) ? (int64_t)col[j] - r : (int64_t)col[j] - col[j - 1];
            if (j == b) bad |= (d < smin || d > smax);
            else bad |= (d < 1 || d > umax);
            if constexpr (BITS == 16) static_cast<uint16_t *>(codes)[j] = (uint16_t)(d & 0xFFFF);
            else static_cast<uint8_t *>(codes)[j] = (uint8_t)(d & 0xFF);
        }
    }
    const uint64_t m = __ballot(bad);
    if (lane == 0 && m) atomicOr(flags, 1);
}

// Merge-path partition: for t = 0..T, d = min(t*L, N+NNZ) and
// i_t = #{ i : rp[i+1] + i < d } (a lower-bound search), j_t = d - i_t.
// Merge-path partition (reading of the IMB "auto" schedule as an
// nnz-balanced split): cut t lies at path step d = min(t (L - slack), N + NNZ),
// i_t = #{i : rp[i+1] + i < d}, j_t = d - i_t. With slack > 0 (every row has
// fewer than slack nonzeros) a cut inside a row moves forward to that row's
// end, so no row spans two tiles and a tile still holds at most L steps.
__global__ __launch_bounds__(kBlock) void k_merge_partition(const int32_t *__restrict__ rp,
                                                            int32_t n_rows, int64_t nnz, int64_t L,
                                                            int64_t slack, int64_t n_tiles,
                                                            int32_t *__restrict__ tile_i,
                                                            int32_t *__restrict__ tile_j) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t > n_tiles) return;
    const int64_t total = (int64_t)n_rows + nnz;
    const int64_t step = L - slack;
    const int64_t d = t * step < total ? t * step : total;
    int64_t lo = d - nnz > 0 ? d - nnz : 0;
    int64_t hi = d < n_rows ? d : n_rows;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)rp[mid + 1] + mid < d) lo = mid + 1;
        else hi = mid;
    }
    int64_t j = d - lo;
    if (slack > 0 && lo < n_rows && j > rp[lo]) {  // row lo in progress: cut after its end
        lo += 1;
        j = rp[lo];
    }
    tile_i[t] = (int32_t)lo;
    tile_j[t] = (int32_t)j;
}

// Merge codes (MB remedy on the merge path): one wave per tile. Pass 1:
// base[t] = smallest column of the tile's nonzeros, *max_range = the largest
// max - min over the tiles. Pass 2: codes[j] = col[j] - base[t].
__global__ __launch_bounds__(kBlock) void k_merge_tile_range(const int32_t *__restrict__ col,
                                                             const int32_t *__restrict__ tile_j,
                                                             int64_t n_tiles,
                                                             int32_t *__restrict__ base,
                                                             int32_t *__restrict__ max_range) {
    const int lane = threadIdx.x % kWave;
    const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kBlock / kWave;
    int32_t widest = 0;  // this wave's largest range; one atomic per wave at the end
    for (int64_t t = wave; t < n_tiles; t += nwaves) {
        const int32_t j0 = tile_j[t], j1 = tile_j[t + 1];
        int32_t mn = INT32_MAX, mx = INT32_MIN;
        for (int32_t j = j0 + lane; j < j1; j += kWave) {
            mn = min(mn, col[j]);
            mx = max(mx, col[j]);
        }
        mn = -group_max<kWave>(-mn);
        mx = group_max<kWave>(mx);
        if (lane == 0) base[t] = j1 > j0 ? mn : 0;
        if (j1 > j0) widest = max(widest, mx - mn);
    }
    if (lane == 0 && widest > 0) atomicMax(max_range, widest);
}

template <int BITS>
__global__ __launch_bounds__(kWave) void k_merge_encode(const int32_t *__restrict__ col,
                                                        const int32_t *__restrict__ tile_j,
                                                        const int32_t *__restrict__ base,
                                                        void *__restrict__ codes) {
    using C = typename std::conditional<BITS == 16, uint16_t, uint8_t>::type;
    const int64_t t = blockIdx.x;
    const int32_t j0 = tile_j[t], j1 = tile_j[t + 1];
    const int32_t b = base[t];
    for (int32_t j = j0 + (int32_t)threadIdx.x; j < j1; j += kWave)
        static_cast<C *>(codes)[j] = (C)(col[j] - b);
}

// Window codes of row-aligned merge tiles (MB + ML remedies on the merge
// path): tile t's distinct columns u_0 < ... < u_{m-1} are its x window,
// stored as offsets from the tile base (dict, WMAX entries per tile, zero
// past m), and each nonzero stores the rank of its column in the window.
// One wave per tile (waves stride over the tiles): the columns mark a
// bitmap of the tile's column range (< 2^16, checked beforehand) in LDS,
// per-word popcount prefixes give every column its rank, and the set bits,
// in order, are the window. The largest m of every wave goes to *max_m
// (one atomic per wave); a tile with m > WMAX writes nothing. With 9-bit
// ranks (WMAX = kWideWindowMax) the code is the rank's low byte and `wrec`
// holds per tile kWideWords words: m, then per lane a 16-bit mask of the
// ranks' ninth bits for the lane's elements (element e of load block it
// of lane l is tile element it * 64 vec + l vec + e; bit it * vec + e).
constexpr int kWindowWords = 65536 / 32;
template <int WMAX>
__global__ __launch_bounds__(kWave) void k_window_encode(const int32_t *__restrict__ col,
                                                         const int32_t *__restrict__ tile_j,
                                                         const int32_t *__restrict__ base,
                                                         int64_t n_tiles,
                                                         uint16_t *__restrict__ dict,
                                                         int32_t *__restrict__ wrec,
                                                         uint8_t *__restrict__ codes,
                                                         int32_t *__restrict__ max_m, int vec) {
    constexpr bool WIDE = WMAX > kWindowMax;
    __shared__ uint32_t bm[kWindowWords];
    __shared__ uint16_t pre[kWindowWords];
    __shared__ uint32_t hm[kWave];
    const int lane = threadIdx.x;
    int32_t most = 0;
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int32_t j0 = tile_j[t], j1 = tile_j[t + 1];
        const int32_t b = base[t];
        int32_t hi = 0;
        for (int32_t j = j0 + lane; j < j1; j += kWave) hi = max(hi, col[j] - b);
        hi = group_max<kWave>(hi);
        if (hi >= 65536) {  // not eligible (the caller checks the ranges first)
            most = INT32_MAX;
            continue;
        }
        const int nw = (hi >> 5) + 1;
        for (int w = lane; w < nw; w += kWave) bm[w] = 0u;
        if (WIDE) hm[lane] = 0u;
        __syncthreads();
        for (int32_t j = j0 + lane; j < j1; j += kWave) {
            const int32_t off = col[j] - b;
            atomicOr(&bm[off >> 5], 1u << (off & 31));
        }
        __syncthreads();
        // lane l owns words [l W, (l + 1) W)
        const int W = (nw + kWave - 1) / kWave;
        const int w0 = min(lane * W, nw), w1 = min(w0 + W, nw);
        int32_t cnt = 0;
        for (int w = w0; w < w1; ++w) cnt += __popc(bm[w]);
        const int32_t incl = group_scan<kWave>(cnt, lane);
        const int32_t m = __shfl(incl, kWave - 1);
        most = max(most, m);
        if (m <= WMAX) {
            int32_t run = incl - cnt;
            for (int w = w0; w < w1; ++w) {
                pre[w] = (uint16_t)run;
                uint32_t bits = bm[w];
                while (bits) {
                    const int q = __ffs(bits) - 1;
                    dict[t * WMAX + run] = (uint16_t)((w << 5) + q);
                    bits &= bits - 1;
                    ++run;
                }
            }
            for (int k = m + lane; k < WMAX; k += kWave) dict[t * WMAX + k] = 0;
            if (lane == 0) wrec[WIDE ? t * kWideWords : t] = m;
        }
        __syncthreads();
        if (m <= WMAX) {
            for (int32_t j = j0 + lane; j < j1; j += kWave) {
                const int32_t off = col[j] - b;
                const int w = off >> 5;
                const uint32_t below = bm[w] & ((1u << (off & 31)) - 1u);
                const int32_t r = pre[w] + __popc(below);
                codes[j] = (uint8_t)r;
                if (WIDE && r >= kWindowMax) {
                    const int32_t p = j - j0, step = kWave * vec;
                    atomicOr(&hm[(p % step) / vec], 1u << ((p / step) * vec + p % vec));
                }
            }
            if (WIDE) {
                __syncthreads();
                reinterpret_cast<uint16_t *>(wrec + t * kWideWords + 1)[lane] = (uint16_t)hm[lane];
            }
        }
        __syncthreads();  // the bitmap is cleared for the next tile
    }
    if (lane == 0 && most > 0) atomicMax(max_m, most);
}

// Column blocks (ML remedy on the merge path): one thread per row counts,
// then copies, its nonzeros block by block; per-thread counters in LDS.
__global__ __launch_bounds__(kBlock) void k_colblock_count(const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ col,
                                                           int32_t n_rows, int32_t B, int32_t width,
                                                           int32_t *__restrict__ cnt) {
    __shared__ int32_t s_cnt[kBlock * kMaxColBlocks];
    int32_t *c = s_cnt + threadIdx.x * kMaxColBlocks;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (int b = 0; b < B; ++b) c[b] = 0;
    if (i >= n_rows) return;
    for (int32_t j = rp[i]; j < rp[i + 1]; ++j) ++c[col[j] / width];
    for (int b = 0; b < B; ++b) cnt[(int64_t)b * n_rows + i] = c[b];
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_colblock_scatter(
    const int32_t *__restrict__ rp, const int32_t *__restrict__ col, const T *__restrict__ val,
    int32_t n_rows, int32_t B, int32_t width, const int32_t *__restrict__ rpb,
    const int64_t *__restrict__ off, int32_t *__restrict__ colb, T *__restrict__ valb) {
    __shared__ int64_t s_pos[kBlock * kMaxColBlocks];
    int64_t *pos = s_pos + threadIdx.x * kMaxColBlocks;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_rows) return;
    for (int b = 0; b < B; ++b) pos[b] = off[b] + rpb[(int64_t)b * (n_rows + 1) + i];
    for (int32_t j = rp[i]; j < rp[i + 1]; ++j) {
        const int32_t c = col[j];
        const int64_t p = pos[c / width]++;
        colb[p] = c;
        valb[p] = val[j];
    }
}

// P_ML probe input (Sec. III-B): a column array holding, for every entry, the
// index of its own row (clamped to the last column), so the probe reads the
// same bytes as CSR but x regularly.
__global__ __launch_bounds__(kBlock) void k_fill_row_index(const int32_t *__restrict__ rp,
                                                           int32_t n_rows, int32_t n_cols,
                                                           int32_t *__restrict__ out) {
    const int lane = threadIdx.x % kWave;
    const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kBlock / kWave;
    for (int64_t r = wave; r < n_rows; r += nwaves) {
        const int32_t b = rp[r], e = rp[r + 1];
        const int32_t v = (int32_t)(r < n_cols ? r : n_cols - 1);
        for (int32_t j = b + lane; j < e; j += kWave) out[j] = v;
    }
}

// Run windows: tile t's window dict[t][0 .. wlen[t]) (ascending offsets from
// its smallest column base[t]) cut into maximal runs of consecutive
// offsets, written as a record of kRunWords words (zero past the last run);
// one thread per tile.
__global__ __launch_bounds__(kBlock) void k_window_runs(const uint16_t *__restrict__ dict,
                                                        const int32_t *__restrict__ wlen,
                                                        const int32_t *__restrict__ base,
                                                        int64_t n_tiles, int32_t *__restrict__ rec,
                                                        int32_t *__restrict__ max_runs) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n_tiles) return;
    const uint16_t *d = dict + t * kWindowMax;
    const int32_t m = wlen[t];
    int32_t *r = rec + t * kRunWords;
    int32_t nr = 0, k0 = 0;
    for (int32_t k = 1; k <= m; ++k) {
        if (k == m || d[k] != d[k - 1] + 1) {  // run [k0, k) ends here
            if (nr < kRunsMax) r[2 + nr] = (int32_t)((uint32_t)d[k0] | ((uint32_t)(k - k0) << 16));
            ++nr;
            k0 = k;
        }
    }
    for (int32_t q = nr < kRunsMax ? nr : kRunsMax; q < kRunsMax; ++q) r[2 + q] = 0;
    r[0] = m > 0 ? base[t] : 0;
    r[1] = (int32_t)((uint32_t)m | ((uint32_t)nr << 16));
    atomicMax(max_runs, nr);
}

// Triad for B_max: one 16-byte vector per array per thread. STREAM: the
// non-temporal loads and stores of the HBM probe; otherwise ordinary
// accesses, which a working set smaller than the Infinity Cache serves from
// there on repeated passes.
template <bool STREAM>
__global__ __launch_bounds__(kBlock) void k_triad1(dvec2 *__restrict__ a,
                                                   const dvec2 *__restrict__ b,
                                                   const dvec2 *__restrict__ c, double s,
                                                   int64_t n2) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n2) {
        dvec2 bb, cc;
        if constexpr (STREAM) {
            bb = __builtin_nontemporal_load(b + i);
            cc = __builtin_nontemporal_load(c + i);
        } else {
            bb = b[i];
            cc = c[i];
        }
        dvec2 r;
        r.x = fma(s, cc.x, bb.x);
        r.y = fma(s, cc.y, bb.y);
        if constexpr (STREAM) __builtin_nontemporal_store(r, a + i);
        else a[i] = r;
    }
}

unsigned grid_for(int64_t n, int64_t per_block_items, unsigned cap) {
    int64_t g = (n + per_block_items - 1) / per_block_items;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_validate(const int32_t *rp, const int32_t *col, int32_t n_rows,
                           int32_t n_cols, int64_t nnz, int32_t *d_flags, hipStream_t s) {
    const unsigned g = grid_for((int64_t)n_rows * kWave, kBlock, 256 * 16);
    hipLaunchKernelGGL(k_validate, dim3(g), dim3(kBlock), 0, s, rp, col, n_rows, n_cols, nnz,
                       d_flags);
    return hipGetLastError();
}

hipError_t launch_delta_encode(const int32_t *rp, const int32_t *col, int32_t n_rows, int bits,
                               void *codes, int32_t *d_flags, hipStream_t s) {
    const unsigned g = grid_for((int64_t)n_rows * kWave, kBlock, 256 * 16);
    if (bits == 16)
        hipLaunchKernelGGL(k_delta_encode<16>, dim3(g), dim3(kBlock), 0, s, rp, col, n_rows, codes,
                           d_flags);
    else
        hipLaunchKernelGGL(k_delta_encode<8>, dim3(g), dim3(kBlock), 0, s, rp, col, n_rows, codes,
                           d_flags);
    return hipGetLastError();
}

hipError_t launch_merge_partition(const int32_t *rp, int32_t n_rows, int64_t nnz, int64_t L,
                                  int64_t slack, int64_t n_tiles, int32_t *tile_i, int32_t *tile_j,
                                  hipStream_t s) {
    const unsigned g = (unsigned)((n_tiles + 1 + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_merge_partition, dim3(g), dim3(kBlock), 0, s, rp, n_rows, nnz, L, slack,
                       n_tiles, tile_i, tile_j);
    return hipGetLastError();
}

hipError_t launch_merge_tile_range(const int32_t *col, const int32_t *tile_j, int64_t n_tiles,
                                   int32_t *base, int32_t *max_range, hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    const unsigned g = grid_for(n_tiles * kWave, kBlock, 256 * 16);
    hipLaunchKernelGGL(k_merge_tile_range, dim3(g), dim3(kBlock), 0, s, col, tile_j, n_tiles, base,
                       max_range);
    return hipGetLastError();
}

hipError_t launch_merge_encode(const int32_t *col, const int32_t *tile_j, int64_t n_tiles,
                               const int32_t *base, int bits, void *codes, hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    if (bits == 16)
        hipLaunchKernelGGL(k_merge_encode<16>, dim3((unsigned)n_tiles), dim3(kWave), 0, s, col,
                           tile_j, base, codes);
    else
        hipLaunchKernelGGL(k_merge_encode<8>, dim3((unsigned)n_tiles), dim3(kWave), 0, s, col,
                           tile_j, base, codes);
    return hipGetLastError();
}

hipError_t launch_window_encode(const int32_t *col, const int32_t *tile_j, const int32_t *base,
                                int64_t n_tiles, uint16_t *dict, int32_t *wlen, uint8_t *codes,
                                int32_t *max_m, hipStream_t s, int wide_vec) {
    if (n_tiles == 0) return hipSuccess;
    // 12 KiB of LDS per wave: about a dozen waves per CU
    const unsigned g = (unsigned)std::min<int64_t>(n_tiles, 256 * 12);
    if (wide_vec > 0)
        hipLaunchKernelGGL(k_window_encode<kWideWindowMax>, dim3(g), dim3(kWave), 0, s, col,
                           tile_j, base, n_tiles, dict, wlen, codes, max_m, wide_vec);
    else
        hipLaunchKernelGGL(k_window_encode<kWindowMax>, dim3(g), dim3(kWave), 0, s, col, tile_j,
                           base, n_tiles, dict, wlen, codes, max_m, 1);
    return hipGetLastError();
}

hipError_t launch_colblock_count(const int32_t *rp, const int32_t *col, int32_t n_rows, int32_t B,
                                 int32_t width, int32_t *cnt, hipStream_t s) {
    if (n_rows == 0) return hipSuccess;
    if (B < 1 || B > kMaxColBlocks || width < 1) return hipErrorInvalidValue;
    const unsigned g = (unsigned)(((int64_t)n_rows + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_colblock_count, dim3(g), dim3(kBlock), 0, s, rp, col, n_rows, B, width,
                       cnt);
    return hipGetLastError();
}

hipError_t launch_colblock_scatter(const int32_t *rp, const int32_t *col, const void *val,
                                   int32_t vbytes, int32_t n_rows, int32_t B, int32_t width,
                                   const int32_t *rpb, const int64_t *off, int32_t *colb,
                                   void *valb, hipStream_t s) {
    if (n_rows == 0) return hipSuccess;
    if (B < 1 || B > kMaxColBlocks || width < 1) return hipErrorInvalidValue;
    const unsigned g = (unsigned)(((int64_t)n_rows + kBlock - 1) / kBlock);
    switch (vbytes) {
    case 8:
        hipLaunchKernelGGL(k_colblock_scatter<uint64_t>, dim3(g), dim3(kBlock), 0, s, rp, col,
                           (const uint64_t *)val, n_rows, B, width, rpb, off, colb, (uint64_t *)valb);
        break;
    case 4:
        hipLaunchKernelGGL(k_colblock_scatter<uint32_t>, dim3(g), dim3(kBlock), 0, s, rp, col,
                           (const uint32_t *)val, n_rows, B, width, rpb, off, colb, (uint32_t *)valb);
        break;
    case 2:
        hipLaunchKernelGGL(k_colblock_scatter<uint16_t>, dim3(g), dim3(kBlock), 0, s, rp, col,
                           (const uint16_t *)val, n_rows, B, width, rpb, off, colb, (uint16_t *)valb);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fill_row_index(const int32_t *rp, int32_t n_rows, int32_t n_cols, int32_t *out,
                                 hipStream_t s) {
    const unsigned g = grid_for((int64_t)n_rows * kWave, kBlock, 256 * 16);
    hipLaunchKernelGGL(k_fill_row_index, dim3(g), dim3(kBlock), 0, s, rp, n_rows, n_cols, out);
    return hipGetLastError();
}

hipError_t launch_convert_values(const double *src, void *dst, int64_t n, int storage,
                                 hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned g = grid_for(n, kBlock * 4, 256 * 32);
    hipLaunchKernelGGL(k_convert, dim3(g), dim3(kBlock), 0, s, src, dst, n, storage);
    return hipGetLastError();
}

hipError_t launch_window_runs(const uint16_t *dict, const int32_t *wlen, const int32_t *base,
                              int64_t n_tiles, int32_t *rec, int32_t *max_runs, hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_window_runs, dim3((unsigned)((n_tiles + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, dict, wlen, base, n_tiles, rec, max_runs);
    return hipGetLastError();
}

hipError_t launch_triad(double *a, const double *b, const double *c, double scalar, int64_t n,
                        bool streaming, hipStream_t s) {
    const int64_t n2 = n / 2;
    const unsigned g = (unsigned)((n2 + kBlock - 1) / kBlock);
    if (streaming)
        hipLaunchKernelGGL(k_triad1<true>, dim3(g), dim3(kBlock), 0, s, (dvec2 *)a,
                           (const dvec2 *)b, (const dvec2 *)c, scalar, n2);
    else
        hipLaunchKernelGGL(k_triad1<false>, dim3(g), dim3(kBlock), 0, s, (dvec2 *)a,
                           (const dvec2 *)b, (const dvec2 *)c, scalar, n2);
    return hipGetLastError();
}

}  // namespace csr
