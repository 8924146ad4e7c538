/*
 * CPU oracle for the adaptive CSR SpMV method of Elafrou, Goumas & Koziris,
 * "Performance Analysis and Optimization of Sparse Matrix-Vector
 * Multiplication on Modern Multi- and Many-Core Processors" (ICPP 2017).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain, single-threaded
 * definition of what the GPU library computes. Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it. It shares no code,
 * header, table or constant with the HIP library, and the library never calls
 * it.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction and no
 * reassociation, so every sum below is evaluated exactly in the order the
 * loops state).
 *
 * Indexing is 0-based and row ranges are half-open [row_ptr[i], row_ptr[i+1]).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* SpMV (Sec. II, Fig. 2: the CSR SpMV listing).                             */
/* The listing's inner statement is read as an accumulation into y[i] that   */
/* starts from +0.0 (an empty row yields +0.0); each product is rounded,     */
/* then added, in storage order.                                             */
/* ------------------------------------------------------------------------ */
void or_spmv(int32_t n_rows, const int32_t *rp, const int32_t *col,
             const double *val, const double *x, double *y)
{
    for (int32_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t j = rp[i]; j < rp[i + 1]; ++j) {
            double p = val[j] * x[col[j]];
            s = s + p;
        }
        y[i] = s;
    }
}

/* |A|.|x| per row: the scale of the rounding error of any summation order. */
void or_absax(int32_t n_rows, const int32_t *rp, const int32_t *col,
              const double *val, const double *x, double *out)
{
    for (int32_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t j = rp[i]; j < rp[i + 1]; ++j)
            s = s + fabs(val[j]) * fabs(x[col[j]]);
        out[i] = s;
    }
}

/*
 * Accurate row dot products: algorithm Dot2 of Ogita, Rump & Oishi,
 * "Accurate sum and dot product", SIAM J. Sci. Comput. 26(6), 2005. Each
 * product is split exactly into p + e with an explicit fma (TwoProduct),
 * partial sums are split exactly with Knuth's TwoSum, and the error terms are
 * accumulated on the side. The result is as accurate as if computed in twice
 * the working precision and then rounded; it is the reference against which
 * both or_spmv and the GPU path are held to 1e-12 * |A||x| per row.
 */
void or_spmv_dot2(int32_t n_rows, const int32_t *rp, const int32_t *col,
                  const double *val, const double *x, double *y)
{
    for (int32_t i = 0; i < n_rows; ++i) {
        double s = 0.0, c = 0.0;
        for (int64_t j = rp[i]; j < rp[i + 1]; ++j) {
            double a = val[j], b = x[col[j]];
            double p = a * b;
            double ep = fma(a, b, -p);           /* exact: a*b = p + ep */
            double t = s + p;                    /* TwoSum(s, p) */
            double z = t - s;
            double es = (s - (t - z)) + (p - z); /* exact: s + p = t + es */
            s = t;
            c = c + (ep + es);
        }
        y[i] = s + c;
    }
}

/* Dense reference: y = A x for a dense row-major m-by-n matrix, columns in
 * ascending order, same unfused multiply-then-add as or_spmv. */
void or_dense_matvec(int32_t m, int32_t n, const double *a, const double *x,
                     double *y)
{
    for (int32_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int32_t j = 0; j < n; ++j) {
            if (a[(int64_t)i * n + j] != 0.0) {
                double p = a[(int64_t)i * n + j] * x[j];
                s = s + p;
            }
        }
        y[i] = s;
    }
}

/* CSR validity as the library's ingest step must decide it: row_ptr[0] = 0,
 * row_ptr non-decreasing, row_ptr[n_rows] = nnz, 0 <= col < n_cols.
 * Returns 1 if valid, 0 otherwise. */
int or_csr_valid(int32_t n_rows, int32_t n_cols, int64_t nnz,
                 const int32_t *rp, const int32_t *col)
{
    if (n_rows < 0 || n_cols < 0 || nnz < 0) return 0;
    if (rp[0] != 0 || (int64_t)rp[n_rows] != nnz) return 0;
    for (int32_t i = 0; i < n_rows; ++i)
        if (rp[i + 1] < rp[i]) return 0;
    for (int64_t j = 0; j < nnz; ++j)
        if (col[j] < 0 || col[j] >= n_cols) return 0;
    return 1;
}

/* 1 if every row's columns are strictly increasing. */
int or_rows_sorted(int32_t n_rows, const int32_t *rp, const int32_t *col)
{
    for (int32_t i = 0; i < n_rows; ++i)
        for (int64_t j = (int64_t)rp[i] + 1; j < rp[i + 1]; ++j)
            if (col[j] <= col[j - 1]) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Reduced-precision value storage.                                          */
/* ------------------------------------------------------------------------ */

/* FP64 -> FP32, IEEE round-to-nearest-even (the C conversion in the default
 * rounding mode). */
void or_to_f32(int64_t n, const double *in, float *out)
{
    for (int64_t k = 0; k < n; ++k) out[k] = (float)in[k];
}

/*
 * FP64 -> BF16 with a single IEEE round-to-nearest-even step, straight from
 * the definition: bf16 has 8 significand bits, exponent range like FP32
 * (normal exponents -126..127, subnormal quantum 2^-133). The value is
 * scaled by its bf16 quantum (a power of two, so exactly), rounded to an
 * integer with ties to even, scaled back, and overflow beyond the largest
 * finite bf16 becomes infinity. NaN maps to the quiet NaN with the same sign.
 */
static uint16_t bf16_of(double v)
{
    union { float f; uint32_t u; } w;
    if (isnan(v)) return (uint16_t)(signbit(v) ? 0xFFC0u : 0x7FC0u);
    if (isinf(v)) return (uint16_t)(signbit(v) ? 0xFF80u : 0x7F80u);
    if (v == 0.0) return (uint16_t)(signbit(v) ? 0x8000u : 0x0000u);
    int e2;
    frexp(v, &e2);                /* |v| = m * 2^e2, m in [0.5, 1) */
    int e = e2 - 1;               /* |v| in [2^e, 2^(e+1)) */
    if (e < -126) e = -126;       /* subnormal range: fixed quantum */
    double q = ldexp(1.0, e - 7); /* spacing of bf16 values near v */
    double r = nearbyint(v / q) * q;  /* v/q exact; nearbyint = ties-to-even */
    if (fabs(r) >= 0x1p128) return (uint16_t)(signbit(v) ? 0xFF80u : 0x7F80u);
    w.f = (float)r;               /* exact: r has <= 8 significant bits */
    return (uint16_t)(w.u >> 16);
}

void or_to_bf16(int64_t n, const double *in, uint16_t *out)
{
    for (int64_t k = 0; k < n; ++k) out[k] = bf16_of(in[k]);
}

void or_bf16_to_f64(int64_t n, const uint16_t *in, double *out)
{
    union { float f; uint32_t u; } w;
    for (int64_t k = 0; k < n; ++k) {
        w.u = (uint32_t)in[k] << 16;
        out[k] = (double)w.f;
    }
}

/* ------------------------------------------------------------------------ */
/* MB remedy: delta-encoded column indices (Sec. III-E, Table II).           */
/* A single width w in {8, 16} is used for the whole matrix (the pool never */
/* mixes the two widths).                                                    */
/* Reading: the first entry of row i stores col - i as a signed w-bit value; */
/* every later entry stores col_j - col_{j-1} as an unsigned w-bit value, so */
/* the rows must be strictly increasing. A matrix is eligible for w only if  */
/* every entry fits.                                                          */
/* ------------------------------------------------------------------------ */
int or_delta_eligible(int32_t n_rows, const int32_t *rp, const int32_t *col,
                      int w)
{
    int64_t smin = -((int64_t)1 << (w - 1)), smax = ((int64_t)1 << (w - 1)) - 1;
    int64_t umax = ((int64_t)1 << w) - 1;
    for (int32_t i = 0; i < n_rows; ++i) {
        int64_t b = rp[i], e = rp[i + 1];
        if (b == e) continue;
        int64_t d0 = (int64_t)col[b] - i;
        if (d0 < smin || d0 > smax) return 0;
        for (int64_t j = b + 1; j < e; ++j) {
            int64_t d = (int64_t)col[j] - col[j - 1];
            if (d < 1 || d > umax) return 0;
        }
    }
    return 1;
}

/* Writes w-bit codes (w/8 bytes each, little endian) into out. Returns 1 on
 * success, 0 if the matrix is not eligible (out then undefined). */
int or_delta_encode(int32_t n_rows, const int32_t *rp, const int32_t *col,
                    int w, void *out)
{
    if (!or_delta_eligible(n_rows, rp, col, w)) return 0;
    uint8_t *o8 = (uint8_t *)out;
    uint16_t *o16 = (uint16_t *)out;
    for (int32_t i = 0; i < n_rows; ++i) {
        for (int64_t j = rp[i]; j < rp[i + 1]; ++j) {
            int64_t d = (j == rp[i]) ? (int64_t)col[j] - i
                                     : (int64_t)col[j] - col[j - 1];
            if (w == 8) o8[j] = (uint8_t)(d & 0xFF);
            else o16[j] = (uint16_t)(d & 0xFFFF);
        }
    }
    return 1;
}

void or_delta_decode(int32_t n_rows, const int32_t *rp, const void *codes,
                     int w, int32_t *col)
{
    const uint8_t *c8 = (const uint8_t *)codes;
    const uint16_t *c16 = (const uint16_t *)codes;
    for (int32_t i = 0; i < n_rows; ++i) {
        int64_t c = 0;
        for (int64_t j = rp[i]; j < rp[i + 1]; ++j) {
            uint32_t u = (w == 8) ? c8[j] : c16[j];
            if (j == rp[i]) {
                int64_t s = (w == 8) ? (int64_t)(int8_t)u : (int64_t)(int16_t)u;
                c = (int64_t)i + s;
            } else {
                c = c + (int64_t)u;
            }
            col[j] = (int32_t)c;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* IMB remedy, nnz-balanced split: merge path over the row ends and the      */
/* nonzeros (the GPU counterpart of the "auto" schedule of Sec. III-E).      */
/* The path merges the row-end list rp[1..N] with the nonzero indices       */
/* 0..NNZ-1; a nonzero j is taken before row end i while j < rp[i+1].        */
/* Row end i is therefore the (rp[i+1] + i + 1)-th item of the path, and the */
/* path position after d items is                                            */
/*     i_d = #{ i : rp[i+1] + i < d },   j_d = d - i_d.                      */
/* Tile t covers items (d_t, d_{t+1}] with d_t = min(t*L, N+NNZ); the table  */
/* holds (i_t, j_t) for t = 0..T, T = ceil((N+NNZ)/L).                       */
/* ------------------------------------------------------------------------ */
/* Row-aligned variant (slack s > 0, used when every row has fewer than s  */
/* nonzeros): cut every L - s items, then move each cut forward to the end */
/* of the row in progress there, so no row spans two tiles and a tile      */
/* still holds at most L items. s = 0 gives the plain partition.           */
int64_t or_merge_tiles(int32_t n_rows, const int32_t *rp, int64_t L, int64_t slack,
                       int32_t *ti, int32_t *tj)
{
    int64_t nnz = rp[n_rows];
    int64_t total = (int64_t)n_rows + nnz;
    int64_t Lp = L - slack;
    int64_t T = (total + Lp - 1) / Lp;
    for (int64_t t = 0; t <= T; ++t) {
        int64_t d = t * Lp < total ? t * Lp : total;
        /* lower bound: first i with rp[i+1] + i >= d */
        int64_t lo = 0, hi = n_rows;
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if ((int64_t)rp[mid + 1] + mid < d) lo = mid + 1;
            else hi = mid;
        }
        int64_t j = d - lo;
        if (slack > 0 && lo < n_rows && j > rp[lo]) { /* row lo in progress */
            lo += 1;
            j = rp[lo];
        }
        ti[t] = (int32_t)lo;
        tj[t] = (int32_t)j;
    }
    return T;
}

/* MB remedy on the merge path (Table II, index compression): each merge   */
/* tile t stores base_t = the smallest column among its nonzeros, and each  */
/* nonzero j of the tile the unsigned w-bit offset col[j] - base_t. The     */
/* matrix is eligible for w iff every tile's column range (max - min) fits  */
/* in w bits. Returns 1 and fills base/codes when eligible, else 0.          */
int or_merge_codes(int64_t T, const int32_t *tj, const int32_t *col, int w,
                   int32_t *base, void *codes)
{
    int64_t lim = (int64_t)1 << w;
    for (int64_t t = 0; t < T; ++t) {
        int32_t mn = 0, mx = 0;
        for (int64_t j = tj[t]; j < tj[t + 1]; ++j) {
            if (j == tj[t] || col[j] < mn) mn = col[j];
            if (j == tj[t] || col[j] > mx) mx = col[j];
        }
        if ((int64_t)mx - mn >= lim) return 0;
        base[t] = mn;
        for (int64_t j = tj[t]; j < tj[t + 1]; ++j) {
            if (w == 16) ((uint16_t *)codes)[j] = (uint16_t)(col[j] - mn);
            else ((uint8_t *)codes)[j] = (uint8_t)(col[j] - mn);
        }
    }
    return 1;
}

/* MB and ML remedies together on row-aligned merge tiles (Table II: index  */
/* compression; x brought close before use, the counterpart of prefetching  */
/* x). Tile t's distinct columns, ascending, u_0 < ... < u_{m-1}, form its  */
/* window: base_t = u_0, dict[t][k] = u_k - u_0 (16 bits), and nonzero j    */
/* of the tile stores the rank k of col[j] in the window (8 bits for        */
/* windows of up to 256 entries, 9 for up to 512). Eligible iff every tile  */
/* has m <= maxw and u_{m-1} - u_0 < 2^16.                                   */
/* dict is T rows of maxw entries, zero past wlen[t] = m. Returns 1 and     */
/* fills the outputs when eligible, else 0.                                  */
static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

int or_window_codes(int64_t T, const int32_t *tj, const int32_t *col, int maxw,
                    int32_t *base, int32_t *wlen, uint16_t *dict, uint16_t *codes)
{
    int64_t cap = 0;
    for (int64_t t = 0; t < T; ++t)
        if ((int64_t)tj[t + 1] - tj[t] > cap) cap = (int64_t)tj[t + 1] - tj[t];
    int32_t *u = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
    int ok = 1;
    for (int64_t t = 0; t < T && ok; ++t) {
        int64_t n = (int64_t)tj[t + 1] - tj[t], m = 0;
        for (int64_t k = 0; k < n; ++k) u[k] = col[tj[t] + k];
        qsort(u, (size_t)n, sizeof(int32_t), cmp_i32);
        for (int64_t k = 0; k < n; ++k)
            if (k == 0 || u[k] != u[m - 1]) u[m++] = u[k];
        if (m > maxw || (m > 0 && (int64_t)u[m - 1] - u[0] >= 65536)) {
            ok = 0;
            break;
        }
        base[t] = m > 0 ? u[0] : 0;
        wlen[t] = (int32_t)m;
        for (int64_t k = 0; k < maxw; ++k)
            dict[t * maxw + k] = k < m ? (uint16_t)(u[k] - u[0]) : 0;
        for (int64_t j = tj[t]; j < tj[t + 1]; ++j) {
            int64_t lo = 0, hi = m - 1; /* col[j] is in u[0..m) */
            while (lo < hi) {
                int64_t mid = (lo + hi) / 2;
                if (u[mid] < col[j]) lo = mid + 1;
                else hi = mid;
            }
            codes[j] = (uint16_t)lo;
        }
    }
    free(u);
    return ok;
}

/* ML remedy composed with the merge path (Table II: x is prefetched into    */
/* the cache; on a GPU, each pass keeps its x gathers inside one slab that  */
/* fits a cache): the columns are cut into B blocks of `width` consecutive  */
/* columns, and block b holds, for every row, the row's nonzeros whose      */
/* column lies in [b width, (b + 1) width), in storage order. rpb holds B   */
/* row-pointer arrays of n + 1 entries, each counting from 0 within its     */
/* block; colb/valb hold the blocks' nonzeros one block after the other.    */
void or_column_blocks(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                      int32_t B, int32_t width, int32_t *rpb, int32_t *colb, double *valb)
{
    int64_t off = 0; /* first nonzero of the current block in colb/valb */
    for (int32_t b = 0; b < B; ++b) {
        int32_t *r = rpb + (int64_t)b * (n + 1);
        int64_t lo = (int64_t)b * width, hi = lo + width, k = 0;
        r[0] = 0;
        for (int32_t i = 0; i < n; ++i) {
            for (int32_t j = rp[i]; j < rp[i + 1]; ++j) {
                if (col[j] >= lo && col[j] < hi) {
                    colb[off + k] = col[j];
                    valb[off + k] = val[j];
                    ++k;
                }
            }
            r[i + 1] = (int32_t)k;
        }
        off += k;
    }
}

/* ------------------------------------------------------------------------ */
/* IMB remedy, decomposition (Sec. III-E, Figs. 5-6): rows with more than    */
/* tau nonzeros are taken out of the row-parallel pass and computed          */
/* cooperatively. Reading of the garbled listing: the offset arrays only     */
/* skip long rows inside the shared val/colind arrays, so the list of long   */
/* rows (ascending) is the whole of the decomposition.                       */
/* ------------------------------------------------------------------------ */
int32_t or_long_rows(int32_t n_rows, const int32_t *rp, int64_t tau,
                     int32_t *out)
{
    int32_t k = 0;
    for (int32_t i = 0; i < n_rows; ++i)
        if ((int64_t)rp[i + 1] - rp[i] > tau) out[k++] = i;
    return k;
}

/* ------------------------------------------------------------------------ */
/* Features (Sec. III-D, Table I) plus two project-defined ones.             */
/*   nnz_i        = rp[i+1] - rp[i]                                          */
/*   bw_i         = max col - min col in row i (0 for rows with <= 1 entry)  */
/*   scatter_i    = nnz_i / max(bw_i, 1), 0 for empty rows                   */
/*   ngroups_i    = number of maximal runs of consecutive columns            */
/*                  (col_j == col_{j-1} + 1 continues a run), storage order  */
/*   clustering_i = ngroups_i / nnz_i, 0 for empty rows                      */
/*   misses_i     = entries whose column distance from the previous entry of */
/*                  the row exceeds E = 16 (FP64 values per 128-byte line);  */
/*                  the first entry of a non-empty row counts as a miss      */
/* Averages divide by N (empty rows included); sd is the population sd.      */
/*                                                                            */
/* out[16]: 0 N, 1 nnz_min, 2 nnz_max, 3 nnz_avg, 4 nnz_sd, 5 bw_min,        */
/* 6 bw_max, 7 bw_avg, 8 bw_sd, 9 scatter_avg, 10 scatter_sd,                */
/* 11 clustering_avg, 12 misses_avg, 13 size (1 if the FP64/int32 CSR plus x */
/* and y fits a 256 MiB last-level cache), 14 mean_col_gap =                 */
/* sum bw_i / sum max(nnz_i - 1, 0), 15 x_reuse (below).                     */
/* iout[8]: 0 sum nnz, 1 sum nnz^2, 2 sum bw, 3 sum bw^2, 4 sum misses,      */
/* 5 sum ngroups, 6 x_reuse shared count, 7 x_reuse distinct count.          */
/*                                                                            */
/* x_reuse: S = min(4096, N - 1) sampled rows r_s = 1 + floor(s (N-1) / S);  */
/* for each, take the first P = 256 entries of rows r and r-1, line ids      */
/* col >> 4; "distinct" counts the run heads of row r's line ids, "shared"   */
/* the run heads that occur among row r-1's line ids.                        */
/* x_reuse = shared / distinct (0 if distinct = 0).                          */
/* ------------------------------------------------------------------------ */
#define FEAT_E 16
#define FEAT_P 256
#define FEAT_S 4096

void or_features(int32_t n_rows, int32_t n_cols, const int32_t *rp,
                 const int32_t *col, double *out, int64_t *iout)
{
    int64_t N = n_rows;
    int64_t nnz = N > 0 ? rp[N] : 0;
    int64_t s_nnz = 0, s_nnz2 = 0, s_bw = 0, s_bw2 = 0, s_miss = 0, s_grp = 0;
    int64_t nnz_min = 0, nnz_max = 0, bw_min = 0, bw_max = 0, s_len1 = 0;
    double s_sc = 0.0, s_cl = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        int64_t b = rp[i], e = rp[i + 1], k = e - b;
        int64_t bw = 0, miss = 0, grp = 0;
        if (k > 0) {
            int64_t mn = col[b], mx = col[b];
            miss = 1;
            grp = 1;
            for (int64_t j = b + 1; j < e; ++j) {
                if (col[j] < mn) mn = col[j];
                if (col[j] > mx) mx = col[j];
                int64_t d = (int64_t)col[j] - col[j - 1];
                if (d > FEAT_E || d < -FEAT_E) miss++;
                if (d != 1) grp++;
            }
            bw = mx - mn;
        }
        if (i == 0 || k < nnz_min) nnz_min = k;
        if (i == 0 || k > nnz_max) nnz_max = k;
        if (i == 0 || bw < bw_min) bw_min = bw;
        if (i == 0 || bw > bw_max) bw_max = bw;
        s_nnz += k;
        s_nnz2 += k * k;
        s_bw += bw;
        s_bw2 += bw * bw;
        s_miss += miss;
        s_grp += grp;
        s_len1 += k > 0 ? k - 1 : 0;
        double sc = k > 0 ? (double)k / (double)(bw > 1 ? bw : 1) : 0.0;
        double cl = k > 0 ? (double)grp / (double)k : 0.0;
        s_sc = s_sc + sc;
        s_cl = s_cl + cl;
    }
    double dN = (double)N;
    double nnz_avg = N ? (double)s_nnz / dN : 0.0;
    double bw_avg = N ? (double)s_bw / dN : 0.0;
    double sc_avg = N ? s_sc / dN : 0.0;
    /* second pass: population standard deviations from their definitions */
    double v_nnz = 0.0, v_bw = 0.0, v_sc = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        int64_t b = rp[i], e = rp[i + 1], k = e - b;
        int64_t bw = 0;
        if (k > 0) {
            int64_t mn = col[b], mx = col[b];
            for (int64_t j = b + 1; j < e; ++j) {
                if (col[j] < mn) mn = col[j];
                if (col[j] > mx) mx = col[j];
            }
            bw = mx - mn;
        }
        double sc = k > 0 ? (double)k / (double)(bw > 1 ? bw : 1) : 0.0;
        double a = (double)k - nnz_avg, c = (double)bw - bw_avg, s = sc - sc_avg;
        v_nnz = v_nnz + a * a;
        v_bw = v_bw + c * c;
        v_sc = v_sc + s * s;
    }
    /* x_reuse over sampled row pairs */
    int64_t shared = 0, distinct = 0;
    if (N > 1) {
        int64_t S = N - 1 < FEAT_S ? N - 1 : FEAT_S;
        for (int64_t s = 0; s < S; ++s) {
            int64_t r = 1 + (s * (N - 1)) / S;
            int64_t b1 = rp[r], e1 = rp[r + 1], b0 = rp[r - 1], e0 = rp[r];
            if (e1 - b1 > FEAT_P) e1 = b1 + FEAT_P;
            if (e0 - b0 > FEAT_P) e0 = b0 + FEAT_P;
            for (int64_t j = b1; j < e1; ++j) {
                int64_t line = col[j] >> 4;
                if (j > b1 && (col[j - 1] >> 4) == line) continue; /* not a run head */
                distinct++;
                for (int64_t q = b0; q < e0; ++q)
                    if ((col[q] >> 4) == line) { shared++; break; }
            }
        }
    }
    double bytes = 12.0 * (double)nnz + 4.0 * (double)(N + 1) + 8.0 * (double)n_cols
                 + 8.0 * (double)N;
    out[0] = dN;
    out[1] = (double)nnz_min;
    out[2] = (double)nnz_max;
    out[3] = nnz_avg;
    out[4] = N ? sqrt(v_nnz / dN) : 0.0;
    out[5] = (double)bw_min;
    out[6] = (double)bw_max;
    out[7] = bw_avg;
    out[8] = N ? sqrt(v_bw / dN) : 0.0;
    out[9] = sc_avg;
    out[10] = N ? sqrt(v_sc / dN) : 0.0;
    out[11] = N ? s_cl / dN : 0.0;
    out[12] = N ? (double)s_miss / dN : 0.0;
    out[13] = bytes <= 268435456.0 ? 1.0 : 0.0;
    out[14] = s_len1 ? (double)s_bw / (double)s_len1 : 0.0;
    out[15] = distinct ? (double)shared / (double)distinct : 0.0;
    iout[0] = s_nnz;
    iout[1] = s_nnz2;
    iout[2] = s_bw;
    iout[3] = s_bw2;
    iout[4] = s_miss;
    iout[5] = s_grp;
    iout[6] = shared;
    iout[7] = distinct;
}
