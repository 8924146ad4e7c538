// y = A x without any allocation, for callers that cannot allocate device
// memory: the row-split CSR SpMV (Sec. II, Fig. 2) with the dynamic row-chunk
// schedule of csr_spmv's row-split plans, run directly on the caller's CSR
// arrays, with the schedule's two chunk counters in a fixed device array of
// the library instead of handle-owned memory.
#include <mutex>

#include "internal.h"

namespace csr {
namespace {

constexpr size_t kNaScratchBytes = 256;

// The dynamic schedule's counters of the calls on one GPU: [0] the next row
// block to hand out, [1] workgroups finished. Each GPU holds its own copy at
// its own address; host code reaches it only through the address
// hipGetSymbolAddress returns.
__device__ __align__(256) int32_t scratch[kNaScratchBytes / sizeof(int32_t)];

__global__ void k_clear_counters(int32_t *ctr) {
    if (threadIdx.x < 2) ctr[threadIdx.x] = 0;
}

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// The scratch array's device address on `device` (the current device),
// looked up on the first call on that device.
csr_status_t scratch_ptr(int device, void **out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(CSR_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch[device] = p;
    }
    *out = g_scratch[device];
    return CSR_OK;
}

}  // namespace
}  // namespace csr

using namespace csr;

extern "C" {

csr_status_t csr_spmv_noalloc(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *d_row_ptr,
                              const int32_t *d_col_idx, const double *d_val, const double *d_x,
                              double *d_y, void *stream) {
    if (n_rows < 0 || n_cols < 0 || nnz < 0) return fail(CSR_ERR_INVALID_ARG, "negative size");
    if (nnz > kMaxNnz) return fail(CSR_ERR_UNSUPPORTED, "nnz > 2^31 - 4096");
    if (!d_row_ptr || (nnz > 0 && (!d_col_idx || !d_val)))
        return fail(CSR_ERR_INVALID_ARG, "NULL array");
    if ((!d_x && n_cols > 0) || (!d_y && n_rows > 0)) return fail(CSR_ERR_INVALID_ARG, "NULL vector");
    const uintptr_t x0 = (uintptr_t)d_x, x1 = x0 + 8 * (size_t)n_cols;
    const uintptr_t y0 = (uintptr_t)d_y, y1 = y0 + 8 * (size_t)n_rows;
    if (n_rows > 0 && n_cols > 0 && x0 < y1 && y0 < x1)
        return fail(CSR_ERR_INVALID_ARG, "x and y overlap");
    if (n_rows == 0) return CSR_OK;
    int dev = 0;
    CSR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CSR_ERR_UNSUPPORTED, "device id out of range");
    void *ctr = nullptr;
    csr_status_t st = scratch_ptr(dev, &ctr);
    if (st != CSR_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // the counters start at zero (a fill kernel, not a memset node, so that
    // the call can be captured in a graph); the last workgroup of the SpMV
    // zeroes them again
    hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(64), 0, s, static_cast<int32_t *>(ctr));
    CSR_HIP(hipGetLastError());
    const int G = default_lanes_per_row((double)nnz / n_rows);
    const void *arr[8] = {d_row_ptr, d_col_idx, nullptr, d_val, d_x, d_y, nullptr, ctr};
    CSR_HIP(launch_rowsplit_s0(G, IDX_I32, false, 1, 1, 0, arr, INT32_MAX, n_rows, n_cols, s));
    return CSR_OK;
}

}  // extern "C"
