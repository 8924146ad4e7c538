/*
 * Multi-core CPU baseline of the plain CSR SpMV (Sec. IV-A: the paper's CSR
 * kernels run with OpenMP on all cores, rows split into contiguous blocks of
 * equal nonzero counts, one block per thread, threads placed close).
 *
 * MEASUREMENT INFRASTRUCTURE: only the benchmark and the test suite load
 * it; it shares no code with the GPU library or with the oracle.
 * Each row is summed in storage order from +0.0, as in the oracle; the
 * compiler may fuse multiply and add here, so results agree with the oracle
 * to rounding, not bit for bit.
 */
#include <omp.h>
#include <stdint.h>

/* smallest row i in [0, n] with rp[i] >= target */
static int32_t first_row_at(int32_t n, const int32_t *rp, int64_t target)
{
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if ((int64_t)rp[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

void omp_spmv(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
              const double *x, double *y)
{
#pragma omp parallel
    {
        const int t = omp_get_thread_num(), T = omp_get_num_threads();
        const int64_t nnz = rp[n];
        int32_t r0 = t == 0 ? 0 : first_row_at(n, rp, nnz * t / T);
        int32_t r1 = t == T - 1 ? n : first_row_at(n, rp, nnz * (t + 1) / T);
        for (int32_t i = r0; i < r1; ++i) {
            double s = 0.0;
            for (int32_t j = rp[i]; j < rp[i + 1]; ++j) s += val[j] * x[col[j]];
            y[i] = s;
        }
    }
}

/* seconds for `calls` back-to-back products; *threads = team size */
double omp_spmv_time(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                     const double *x, double *y, int32_t calls, int32_t *threads)
{
    *threads = omp_get_max_threads();
    omp_spmv(n, rp, col, val, x, y); /* warm: page-in, thread team */
    const double t0 = omp_get_wtime();
    for (int32_t c = 0; c < calls; ++c) omp_spmv(n, rp, col, val, x, y);
    return omp_get_wtime() - t0;
}
