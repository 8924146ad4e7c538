// Host side of csr_spmv_batched: the work queue of every matrix's merge-path
// tiles, a batch-level autotuner over the tile size, and a captured HIP graph
// that later calls replay.
#include <algorithm>
#include <memory>
#include <mutex>
#include <vector>

#include "batch.h"

namespace csr {

namespace {

struct BatchPlan {
    std::vector<uint64_t> key;  // handle id, plan version, ... per matrix
    int storage = 0;
    int device = 0;
    std::vector<BatchMat> mats_h;
    DevBuf mats, item_mat, tile_i, tile_j, carry;
    int64_t n_items = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~BatchPlan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

std::mutex g_mu;
// Never destroyed at exit (no HIP calls after the runtime shuts down); the
// cache keeps the few most recent batches.
std::vector<std::unique_ptr<BatchPlan>> *const g_plans = new std::vector<std::unique_ptr<BatchPlan>>;
constexpr size_t kMaxPlans = 8;

hipError_t launch(const BatchPlan &B, hipStream_t s) {
    const int n_cu = device_cu_count(B.device);
    const BatchMat *m = B.mats.as<BatchMat>();
    const int32_t *im = B.item_mat.as<int32_t>();
    switch (B.storage) {
    case CSR_VAL_F64: return launch_batch_s0(m, im, B.n_items, n_cu, s);
    case CSR_VAL_F32: return launch_batch_s1(m, im, B.n_items, n_cu, s);
    default: return launch_batch_s2(m, im, B.n_items, n_cu, s);
    }
}

// Tile tables for every matrix with tile size 64 * ipt[k]; descriptors and
// the item -> matrix table.
csr_status_t build(BatchPlan &B, int32_t count, const csr_matrix_t *A, const void *const *x,
                   void *const *y, const std::vector<int> &ipt, hipStream_t s) {
    std::vector<int64_t> T(count), base(count + 1, 0), tbase(count + 1, 0);
    for (int k = 0; k < count; ++k) {
        T[k] = merge_tile_count(A[k], (int64_t)kMergeBlock * ipt[k]);
        base[k + 1] = base[k] + T[k];       // work items (tiles)
        tbase[k + 1] = tbase[k] + T[k] + 1; // tile-table entries
    }
    B.n_items = base[count];
    const size_t ab = B.storage == CSR_VAL_F64 ? 8 : 4;
    csr_status_t st;
    if ((st = B.tile_i.alloc(sizeof(int32_t) * tbase[count])) != CSR_OK) return st;
    if ((st = B.tile_j.alloc(sizeof(int32_t) * tbase[count])) != CSR_OK) return st;
    if ((st = B.carry.alloc(ab * (size_t)std::max<int64_t>(B.n_items, 1))) != CSR_OK) return st;
    if ((st = B.mats.alloc(sizeof(BatchMat) * count)) != CSR_OK) return st;
    if ((st = B.item_mat.alloc(sizeof(int32_t) * std::max<int64_t>(B.n_items, 1))) != CSR_OK)
        return st;
    B.mats_h.resize(count);
    std::vector<int32_t> im((size_t)B.n_items);
    for (int k = 0; k < count; ++k) {
        int32_t *ti = B.tile_i.as<int32_t>() + tbase[k];
        int32_t *tj = B.tile_j.as<int32_t>() + tbase[k];
        const int64_t L = (int64_t)kMergeBlock * ipt[k];
        CSR_HIP(launch_merge_partition(A[k]->rp.as<int32_t>(), A[k]->n_rows, A[k]->nnz, L,
                                       merge_slack(A[k], L), T[k], ti, tj, s));
        BatchMat &M = B.mats_h[k];
        M.rp = A[k]->rp.as<int32_t>();
        M.col = A[k]->col.as<int32_t>();
        M.val = A[k]->val.p;
        M.x = x[k];
        M.y = y[k];
        M.tile_i = ti;
        M.tile_j = tj;
        M.carry = B.carry.as<char>() + ab * base[k];
        M.n_rows = A[k]->n_rows;
        M.ipt = ipt[k];
        M.aligned = merge_slack(A[k], L) > 0;
        M.reserved = 0;
        M.tile_base = base[k];
        std::fill(im.begin() + base[k], im.begin() + base[k + 1], k);
    }
    CSR_HIP(hipMemcpyAsync(B.mats.p, B.mats_h.data(), sizeof(BatchMat) * count,
                           hipMemcpyHostToDevice, s));
    if (B.n_items > 0)
        CSR_HIP(hipMemcpyAsync(B.item_mat.p, im.data(), sizeof(int32_t) * im.size(),
                               hipMemcpyHostToDevice, s));
    CSR_HIP(hipStreamSynchronize(s));
    return CSR_OK;
}

csr_status_t time_batch(const BatchPlan &B, hipStream_t s, double *ms) {
    hipEvent_t e0, e1;
    CSR_HIP(hipEventCreate(&e0));
    CSR_HIP(hipEventCreate(&e1));
    hipError_t e = launch(B, s);
    double best = 1e300;
    for (int r = 0; r < 3 && e == hipSuccess; ++r) {
        e = hipEventRecord(e0, s);
        for (int c = 0; c < 5 && e == hipSuccess; ++c) e = launch(B, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float f = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
        best = std::min(best, (double)f / 5);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "batched timing");
    *ms = best;
    return CSR_OK;
}

csr_status_t capture(BatchPlan &B) {
    hipStream_t cs;
    CSR_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t le = launch(B, cs);
        e = hipStreamEndCapture(cs, &B.graph);
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    return CSR_OK;
}

}  // namespace

void batch_forget(uint64_t id) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto &v = *g_plans;
    v.erase(std::remove_if(v.begin(), v.end(),
                           [&](const std::unique_ptr<BatchPlan> &p) {
                               for (size_t q = 0; q < p->key.size(); q += 2)
                                   if (p->key[q] == id) return true;
                               return false;
                           }),
            v.end());
}

}  // namespace csr

using namespace csr;

extern "C" csr_status_t csr_spmv_batched(int32_t count, const csr_matrix_t *h_A,
                                         const void *const *h_x, void *const *h_y, void *stream) {
    if (count < 0 || (count > 0 && (!h_A || !h_x || !h_y)))
        return fail(CSR_ERR_INVALID_ARG, "bad batch arguments");
    if (count == 0) return CSR_OK;
    int dev = 0;
    CSR_HIP(hipGetDevice(&dev));
    const int storage = h_A[0] ? h_A[0]->storage : -1;
    std::vector<uint64_t> key;
    for (int k = 0; k < count; ++k) {
        const csr_matrix_s *A = h_A[k];
        if (!A) return fail(CSR_ERR_INVALID_ARG, "NULL handle in batch");
        if (A->device != dev) return fail(CSR_ERR_INVALID_ARG, "handle on another device");
        if (A->storage != storage) return fail(CSR_ERR_INVALID_ARG, "mixed storage types");
        if ((!h_x[k] && A->n_cols > 0) || (!h_y[k] && A->n_rows > 0))
            return fail(CSR_ERR_INVALID_ARG, "NULL vector in batch");
        key.push_back(A->id);
        key.push_back(A->version);
    }
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_mu);
    auto &plans = *g_plans;
    BatchPlan *B = nullptr;
    for (auto &p : plans)
        if (p->key == key && p->device == dev) B = p.get();
    if (!B) {
        // Per-matrix tile size: a matrix whose own plan is the merge path
        // keeps its L; the others take the tile size the batch autotuner
        // picks (all 256, all 512, or 256 below the median nnz).
        std::vector<int64_t> nnz(count);
        for (int k = 0; k < count; ++k) nnz[k] = h_A[k]->nnz;
        std::vector<int64_t> sorted = nnz;
        std::nth_element(sorted.begin(), sorted.begin() + count / 2, sorted.end());
        const int64_t median = sorted[count / 2];
        std::unique_ptr<BatchPlan> best;
        double best_ms = 1e300;
        for (int mode = 0; mode < 3; ++mode) {
            std::vector<int> ipt(count);
            for (int k = 0; k < count; ++k) {
                const Plan &P = h_A[k]->plan;
                // (tile sizes compiled at run time have no batched instance)
                if ((P.opts & CSR_OPT_MERGE) && merge_items_prebuilt(P.L)) ipt[k] = P.L / kMergeBlock;
                else ipt[k] = mode == 0 ? 4 : mode == 1 ? 8 : (nnz[k] < median ? 4 : 8);
            }
            auto cand = std::make_unique<BatchPlan>();
            cand->key = key;
            cand->storage = storage;
            cand->device = dev;
            csr_status_t st = build(*cand, count, h_A, h_x, h_y, ipt, s);
            if (st != CSR_OK) return st;
            double ms = 0;
            if ((st = time_batch(*cand, s, &ms)) != CSR_OK) return st;
            if (ms < best_ms) {
                best_ms = ms;
                best = std::move(cand);
            }
        }
        csr_status_t st = capture(*best);
        if (st != CSR_OK) return st;
        if (plans.size() >= kMaxPlans) plans.erase(plans.begin());
        plans.push_back(std::move(best));
        B = plans.back().get();
    }
    // new vector pointers: refresh the descriptors (outside the graph)
    bool moved = false;
    for (int k = 0; k < count; ++k) {
        if (B->mats_h[k].x != h_x[k] || B->mats_h[k].y != h_y[k]) {
            B->mats_h[k].x = h_x[k];
            B->mats_h[k].y = h_y[k];
            moved = true;
        }
    }
    if (moved)
        CSR_HIP(hipMemcpyAsync(B->mats.p, B->mats_h.data(), sizeof(BatchMat) * count,
                               hipMemcpyHostToDevice, s));
    CSR_HIP(hipGraphLaunch(B->exec, s));
    return CSR_OK;
}
