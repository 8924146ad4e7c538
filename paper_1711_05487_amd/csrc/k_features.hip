// Matrix features (Sec. III-D, Table I) in one sweep over row_ptr and col_idx.
//
// Per row i (entries in storage order): nnz_i; bw_i = max col - min col;
// misses_i = entries whose distance from the previous entry exceeds 16
// columns (one 128-byte line of FP64 x), the first entry counting as a miss;
// ngroups_i = maximal runs of consecutive columns; scatter_i = nnz_i /
// max(bw_i, 1) and clustering_i = ngroups_i / nnz_i (both 0 for an empty row).
//
// G lanes share a row, each taking a contiguous segment (the entry before a
// segment gives its first gap). Rows longer than 64 G entries are left out
// of the sweep and marked in a bitmap, listed in row order from it on the
// device, and each reduced by a whole workgroup, so one long row does not
// serialize a lane group. Integer totals are
// exact int64 sums; the scatter mean and variance use Welford updates per
// thread merged with Chan's pairwise formula in a fixed tree, so the result
// is deterministic. A second small kernel samples row pairs for the x-reuse
// estimate, and a one-block kernel folds the per-block partials in order.
#include <algorithm>

#include "device.h"
#include "internal.h"

namespace csr {

namespace {

constexpr int kFeatE = 16;   // FP64 values per 128-byte cache line
constexpr int kReuseP = 256; // entries per sampled row
constexpr int kReuseS = 4096;
constexpr int kFeatBlocks = 2048;  // workgroups of the sweep (partials to fold)

__device__ __forceinline__ void welford_push(double &n, double &mean, double &m2, double v) {
    n += 1.0;
    const double d = v - mean;
    mean += d / n;
    m2 += d * (v - mean);
}

__device__ __forceinline__ void chan_merge(FeatPart &a, const FeatPart &b) {
    a.s_nnz2 += b.s_nnz2;
    a.s_bw += b.s_bw;
    a.s_bw2 += b.s_bw2;
    a.s_miss += b.s_miss;
    a.s_grp += b.s_grp;
    a.s_len1 += b.s_len1;
    a.nnz_min = min(a.nnz_min, b.nnz_min);
    a.nnz_max = max(a.nnz_max, b.nnz_max);
    a.bw_min = min(a.bw_min, b.bw_min);
    a.bw_max = max(a.bw_max, b.bw_max);
    a.s_cl += b.s_cl;
    if (b.sc_n > 0.0) {
        if (a.sc_n == 0.0) {
            a.sc_n = b.sc_n;
            a.sc_mean = b.sc_mean;
            a.sc_m2 = b.sc_m2;
        } else {
            const double n = a.sc_n + b.sc_n;
            const double d = b.sc_mean - a.sc_mean;
            a.sc_mean += d * (b.sc_n / n);
            a.sc_m2 += b.sc_m2 + d * d * (a.sc_n * b.sc_n / n);
            a.sc_n = n;
        }
    }
}

__device__ __forceinline__ void part_init(FeatPart &p) {
    p.s_nnz2 = p.s_bw = p.s_bw2 = p.s_miss = p.s_grp = p.s_len1 = 0;
    p.nnz_min = INT32_MAX;
    p.nnz_max = INT32_MIN;
    p.bw_min = INT32_MAX;
    p.bw_max = INT32_MIN;
    p.sc_n = p.sc_mean = p.sc_m2 = 0.0;
    p.s_cl = 0.0;
}

// Statistics of the entries [s0, s1) of a row that starts at b (the entry
// before s0, when inside the row, gives the first gap).
struct SegStats {
    int32_t mn, mx, miss, grps;
};
// The segment is read U entries at a time, all U loads issued before any is
// used (one round covers a segment of up to 16 entries; the 64-entry
// segments of a skewed matrix's rows take four).
__device__ __forceinline__ SegStats seg_stats(const int32_t *__restrict__ col, int32_t b,
                                              int32_t e, int32_t s0, int32_t s1) {
    constexpr int U = 16;
    SegStats g{INT32_MAX, INT32_MIN, 0, 0};
    int32_t prev = s0 > b && s0 < e ? col[s0 - 1] : 0;
    for (int32_t j0 = s0; j0 < s1; j0 += U) {
        int32_t c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = j0 + u < s1 ? col[j0 + u] : 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t j = j0 + u;
            if (j < s1) {
                g.mn = min(g.mn, c[u]);
                g.mx = max(g.mx, c[u]);
                if (j == b) {
                    g.miss += 1;
                    g.grps += 1;
                } else {
                    const int64_t d = (int64_t)c[u] - prev;
                    g.miss += (d > kFeatE || d < -kFeatE) ? 1 : 0;
                    g.grps += (d != 1) ? 1 : 0;
                }
                prev = c[u];
            }
        }
    }
    return g;
}

// One row's contribution (k entries, bandwidth bw).
__device__ __forceinline__ void part_push(FeatPart &p, int32_t k, int32_t bw, int32_t miss,
                                          int32_t grps) {
    p.s_nnz2 += (int64_t)k * k;
    p.s_bw += bw;
    p.s_bw2 += (int64_t)bw * bw;
    p.s_miss += miss;
    p.s_grp += grps;
    p.s_len1 += k > 0 ? k - 1 : 0;
    p.nnz_min = min(p.nnz_min, k);
    p.nnz_max = max(p.nnz_max, k);
    p.bw_min = min(p.bw_min, bw);
    p.bw_max = max(p.bw_max, bw);
    const double sc = k > 0 ? (double)k / (double)(bw > 1 ? bw : 1) : 0.0;
    welford_push(p.sc_n, p.sc_mean, p.sc_m2, sc);
    p.s_cl += k > 0 ? (double)grps / (double)k : 0.0;
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_features(const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     int32_t n_rows, FeatPart *__restrict__ out,
                                                     int32_t *__restrict__ long_list,
                                                     uint32_t *__restrict__ long_bits) {
    __shared__ FeatPart s_part[kBlock / G];
    constexpr int NG = kBlock / G;
    const int lane = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    FeatPart p;
    part_init(p);
    // workgroup b sweeps rows b*NG + grp, then + gridDim*NG, ... (fixed order);
    // the next row's bounds are loaded while this row is reduced
    const int64_t stride = (int64_t)gridDim.x * NG;
    int64_t r = (int64_t)blockIdx.x * NG + grp;
    int32_t nb = r < n_rows ? rp[r] : 0, ne = r < n_rows ? rp[r + 1] : 0;
    for (; r < n_rows; r += stride) {
        const int32_t b = nb, e = ne;
        if (r + stride < n_rows) {
            nb = rp[r + stride];
            ne = rp[r + stride + 1];
        }
        const int32_t k = e - b;
        if (k > 64 * G) {  // reduced by its own workgroup later
            if (lane == 0) {
                atomicAdd(long_list, 1);
                atomicOr(long_bits + (r >> 5), 1u << (r & 31));
            }
            continue;
        }
        // lane takes the contiguous segment [s0, s1) of the row
        const int32_t q = (k + G - 1) / G;
        const int32_t s0 = min(b + lane * q, e), s1 = min(s0 + q, e);
        SegStats g = seg_stats(col, b, e, s0, s1);
        const int32_t mn = -group_max<G>(-g.mn);
        const int32_t mx = group_max<G>(g.mx);
        const int32_t miss = group_isum<G>(g.miss);
        const int32_t grps = group_isum<G>(g.grps);
        if (lane == 0) part_push(p, k, k > 0 ? mx - mn : 0, miss, grps);
    }
    if (lane == 0) s_part[grp] = p;
    __syncthreads();
    for (int w = NG / 2; w > 0; w >>= 1) {
        if (lane == 0 && grp < w) chan_merge(s_part[grp], s_part[grp + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = s_part[0];
}

// Long row list[1 + b], reduced by workgroup b (kBlock contiguous segments;
// integer statistics, so the split does not change them): one partial.
__global__ __launch_bounds__(kBlock) void k_features_long(const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ col,
                                                          const int32_t *__restrict__ long_list,
                                                          FeatPart *__restrict__ out) {
    __shared__ int32_t s_mn[kBlock], s_mx[kBlock], s_miss[kBlock], s_grp[kBlock];
    const int32_t r = long_list[1 + blockIdx.x];
    const int32_t b = rp[r], e = rp[r + 1];
    const int32_t k = e - b;
    const int32_t q = (k + kBlock - 1) / kBlock;
    const int32_t s0 = min(b + (int32_t)threadIdx.x * q, e), s1 = min(s0 + q, e);
    const SegStats g = seg_stats(col, b, e, s0, s1);
    s_mn[threadIdx.x] = g.mn;
    s_mx[threadIdx.x] = g.mx;
    s_miss[threadIdx.x] = g.miss;
    s_grp[threadIdx.x] = g.grps;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_mn[threadIdx.x] = min(s_mn[threadIdx.x], s_mn[threadIdx.x + w]);
            s_mx[threadIdx.x] = max(s_mx[threadIdx.x], s_mx[threadIdx.x + w]);
            s_miss[threadIdx.x] += s_miss[threadIdx.x + w];
            s_grp[threadIdx.x] += s_grp[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        FeatPart p;
        part_init(p);
        part_push(p, k, s_mx[0] - s_mn[0], s_miss[0], s_grp[0]);
        out[blockIdx.x] = p;
    }
}

// Fold the per-block partials in block order (one workgroup, fixed tree)
// into the results header: the fold, then the long-row count.
__global__ __launch_bounds__(kBlock) void k_features_fold(const FeatPart *__restrict__ parts,
                                                          int32_t n_parts,
                                                          const int32_t *__restrict__ long_list,
                                                          char *__restrict__ out) {
    __shared__ FeatPart s[kBlock];
    FeatPart p;
    part_init(p);
    // thread t folds parts t*chunk .. (t+1)*chunk-1 in order
    const int32_t chunk = (n_parts + kBlock - 1) / kBlock;
    const int32_t a = threadIdx.x * chunk;
    const int32_t b = min(a + chunk, n_parts);
    for (int32_t q = a; q < b; ++q) chan_merge(p, parts[q]);
    s[threadIdx.x] = p;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) chan_merge(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *reinterpret_cast<FeatPart *>(out) = s[0];
        *reinterpret_cast<int32_t *>(out + sizeof(FeatPart)) = long_list[0];
    }
}

// x-reuse sample s: rows r = 1 + floor(s (N-1) / S) and r-1, first P entries
// each; line ids col >> 4. distinct = run heads of row r's line ids, shared =
// run heads that also occur among row r-1's line ids.
__global__ __launch_bounds__(kWave) void k_xreuse(const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col, int32_t n_rows,
                                                  int32_t n_samples,
                                                  int32_t *__restrict__ out /* 2 per sample */) {
    __shared__ int32_t s_prev[kReuseP];
    const int s = blockIdx.x;
    if (s >= n_samples) return;
    const int64_t r = 1 + ((int64_t)s * (n_rows - 1)) / n_samples;
    const int32_t b1 = rp[r], e1 = min(rp[r + 1], b1 + kReuseP);
    const int32_t b0 = rp[r - 1], e0 = min(rp[r], b0 + kReuseP);
    const int n0 = e0 - b0;
    for (int k = threadIdx.x; k < n0; k += kWave) s_prev[k] = col[b0 + k] >> 4;
    __syncthreads();
    int distinct = 0, shared = 0;
    for (int32_t j = b1 + threadIdx.x; j < e1; j += kWave) {
        const int32_t line = col[j] >> 4;
        if (j > b1 && (col[j - 1] >> 4) == line) continue;
        ++distinct;
        for (int q = 0; q < n0; ++q)
            if (s_prev[q] == line) {
                ++shared;
                break;
            }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        distinct += __shfl_xor(distinct, off);
        shared += __shfl_xor(shared, off);
    }
    if (threadIdx.x == 0) {
        out[2 * s] = shared;
        out[2 * s + 1] = distinct;
    }
}

template <int G>
hipError_t go(const int32_t *rp, const int32_t *col, int32_t n_rows, FeatPart *parts,
              int32_t n_parts, int32_t *long_list, uint32_t *long_bits, hipStream_t s) {
    hipLaunchKernelGGL(k_features<G>, dim3(n_parts), dim3(kBlock), 0, s, rp, col, n_rows, parts,
                       long_list, long_bits);
    return hipGetLastError();
}

// The long rows in row order, from their bits: thread t counts the set bits
// of its contiguous run of words, the counts are scanned, and each thread
// writes its rows at its offset (list[1 + k] = k-th long row), so the long
// pass folds them in row order without a host sort.
__global__ __launch_bounds__(kBlock) void k_long_order(const uint32_t *__restrict__ bits,
                                                       int64_t n_words,
                                                       int32_t *__restrict__ list) {
    __shared__ int32_t s_off[kBlock];
    const int64_t chunk = (n_words + kBlock - 1) / kBlock;
    const int64_t w0 = min((int64_t)threadIdx.x * chunk, n_words);
    const int64_t w1 = min(w0 + chunk, n_words);
    int32_t c = 0;
    for (int64_t w = w0; w < w1; ++w) c += __popc(bits[w]);
    s_off[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {  // exclusive scan of the counts, in order
        int32_t run = 0;
        for (int q = 0; q < kBlock; ++q) {
            const int32_t v = s_off[q];
            s_off[q] = run;
            run += v;
        }
    }
    __syncthreads();
    int32_t k = 1 + s_off[threadIdx.x];
    for (int64_t w = w0; w < w1; ++w) {
        uint32_t m = bits[w];
        while (m) {
            const int b = __ffs(m) - 1;
            list[k++] = (int32_t)(w * 32 + b);
            m &= m - 1;
        }
    }
}

}  // namespace

int32_t features_partials(int32_t n_rows, int G) {
    const int64_t NG = kBlock / G;
    const int64_t need = n_rows > 0 ? (n_rows + NG - 1) / NG : 1;
    return (int32_t)(need < kFeatBlocks ? need : kFeatBlocks);
}

int32_t xreuse_samples(int32_t n_rows) { return n_rows > 1 ? min(n_rows - 1, kReuseS) : 0; }

int32_t features_long_row(int G) { return 64 * G; }

int64_t features_long_capacity(int64_t nnz, int G) {
    return nnz / ((int64_t)features_long_row(G) + 1) + 1;
}

hipError_t launch_features(const int32_t *rp, const int32_t *col, int32_t n_rows, int G,
                           FeatPart *parts, int32_t n_parts, int32_t *long_list,
                           uint32_t *long_bits, void *out, hipStream_t s) {
    char *const out_b = static_cast<char *>(out);
    int32_t *const reuse_out = reinterpret_cast<int32_t *>(out_b + kFeatHeader);
    hipError_t e;
    if ((e = hipMemsetAsync(long_list, 0, sizeof(int32_t), s)) != hipSuccess) return e;
    const size_t n_words = ((size_t)n_rows + 31) / 32;
    if ((e = hipMemsetAsync(long_bits, 0, sizeof(uint32_t) * n_words, s)) != hipSuccess) return e;
    uint32_t *const lb = long_bits;
    switch (G) {
    case 1: e = go<1>(rp, col, n_rows, parts, n_parts, long_list, lb, s); break;
    case 2: e = go<2>(rp, col, n_rows, parts, n_parts, long_list, lb, s); break;
    case 4: e = go<4>(rp, col, n_rows, parts, n_parts, long_list, lb, s); break;
    case 8: e = go<8>(rp, col, n_rows, parts, n_parts, long_list, lb, s); break;
    case 16: e = go<16>(rp, col, n_rows, parts, n_parts, long_list, lb, s); break;
    case 32: e = go<32>(rp, col, n_rows, parts, n_parts, long_list, lb, s); break;
    default: e = go<64>(rp, col, n_rows, parts, n_parts, long_list, lb, s); break;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_features_fold, dim3(1), dim3(kBlock), 0, s, parts, n_parts,
                       (const int32_t *)long_list, out_b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int32_t ns = xreuse_samples(n_rows);
    if (ns > 0) {
        hipLaunchKernelGGL(k_xreuse, dim3(ns), dim3(kWave), 0, s, rp, col, n_rows, ns, reuse_out);
        e = hipGetLastError();
    }
    return e;
}

hipError_t features_long_rows(const int32_t *rp, const int32_t *col, int32_t n_rows, int64_t nnz,
                              int G, FeatPart *parts, int32_t n_parts, int32_t *long_list,
                              const uint32_t *long_bits, int32_t n_long, void *out,
                              hipStream_t s) {
    if (n_long < 0 || n_long > features_long_capacity(nnz, G)) return hipErrorInvalidValue;
    if (n_long == 0) return hipSuccess;
    // listed in row order, so that their partials are folded in row order
    // (deterministic features)
    const int64_t n_words = ((int64_t)n_rows + 31) / 32;
    hipLaunchKernelGGL(k_long_order, dim3(1), dim3(kBlock), 0, s, long_bits, n_words, long_list);
    hipError_t e;
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_features_long, dim3((unsigned)n_long), dim3(kBlock), 0, s, rp, col,
                       long_list, parts + n_parts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_features_fold, dim3(1), dim3(kBlock), 0, s, parts, n_parts + n_long,
                       (const int32_t *)long_list, static_cast<char *>(out));
    return hipGetLastError();
}

}  // namespace csr
