// Host side of csr_spmv_batched: every matrix runs its own plan. The
// matrices are grouped into classes by the kernel instance their plan
// launches (merge-path tiles per tile size, index encoding and alignment;
// row-split blocks per lanes, encoding, accumulators and rows in flight; the
// long-row pass of decomposition plans; each column-block pass of a merge
// plan on its own, so that the passes of one matrix run in order); each class
// is one persistent kernel over the concatenated items of its matrices, and
// the classes are captured once into a HIP graph that later calls replay
// (the classes of one pass as parallel branches). A
// plan without a batched instance (a merge tile size compiled at run time)
// has its own launches captured in the same graph.
#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "batch.h"

namespace csr {

namespace {

enum ClassKind { K_MERGE = 0, K_ROWS = 1, K_LONG = 2, K_OWN = 3 };

// (pass, kind, ipt or G, idx, nt, x32, aln, U, R): the kernel instance of a
// class; `pass` orders the column-block passes
using ClassKey = std::tuple<int, int, int, int, int, int, int, int, int>;

struct ClassRun {
    ClassKey key;
    std::vector<int> descs;   // descriptors of the class (indices into BatchPlan::desc_h)
    int64_t n_items = 0;      // tiles, row blocks, or long-row chunks
    int64_t n_items2 = 0;     // long rows
    int64_t item_off = 0;     // offset of the class's item table in BatchPlan::items
    int64_t item_off2 = 0;
    int matrix = -1;          // K_OWN: the batch index of the matrix
};

struct BatchPlan {
    std::vector<uint64_t> key;  // handle id, plan version per matrix
    int storage = 0;
    int device = 0;
    int count = 0;
    std::vector<BatchMat> desc_h;     // every descriptor of every class
    std::vector<int> desc_matrix;     // the batch index each descriptor belongs to
    std::vector<ClassRun> runs;       // in launch order
    std::vector<const void *> xs;     // the vectors the descriptors and the graph hold
    std::vector<void *> ys;
    std::vector<const csr_matrix_s *> mats;
    bool has_own = false;
    DevBuf desc, items;
    HostBuf desc_pin;                 // staging of descriptor refreshes
    hipEvent_t refreshed = nullptr;   // the last refresh copy has read desc_pin
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~BatchPlan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (refreshed) (void)hipEventDestroy(refreshed);
    }
};

std::mutex g_mu;
// Never destroyed at exit (no HIP calls after the runtime shuts down); the
// cache keeps the few most recent batches.
std::vector<std::unique_ptr<BatchPlan>> *const g_plans = new std::vector<std::unique_ptr<BatchPlan>>;
constexpr size_t kMaxPlans = 8;

// the instance choices of the single-matrix launchers
int rows_eff_R(const Plan &P) { return P.idx != IDX_I32 ? 1 : P.R >= 4 ? 4 : P.R == 2 ? 2 : 1; }
int rows_eff_U(const Plan &P) { return P.idx != IDX_I32 ? 1 : P.U >= 4 ? 4 : 1; }

BatchMat base_desc(const csr_matrix_s *A, const void *x, void *y) {
    BatchMat M{};
    M.rp = A->rp.as<int32_t>();
    M.col = A->col.as<int32_t>();
    M.val = A->val.p;
    M.x = x;
    M.y = y;
    M.n_rows = A->n_rows;
    M.n_cols = A->n_cols;
    M.skip_above = INT32_MAX;
    return M;
}

// Group the matrices into classes and fill the descriptors and item counts.
void plan_classes(BatchPlan &B, const csr_matrix_t *h_A, const void *const *x, void *const *y) {
    std::map<ClassKey, ClassRun> cls;
    auto add = [&](const ClassKey &key, const BatchMat &M, int k, int64_t items, int64_t items2) {
        ClassRun &r = cls[key];
        r.key = key;
        BatchMat D = M;
        D.item_base = r.n_items;
        D.item_base2 = r.n_items2;
        r.n_items += items;
        r.n_items2 += items2;
        r.descs.push_back((int)B.desc_h.size());
        B.desc_h.push_back(D);
        B.desc_matrix.push_back(k);
    };
    int own = 0;
    for (int k = 0; k < B.count; ++k) {
        const csr_matrix_s *A = h_A[k];
        const Plan &P = A->plan;
        if (A->n_rows == 0) continue;
        const bool x32 = x_fits_32(A);
        if ((P.opts & CSR_OPT_MERGE) && P.cblocks > 0 && merge_items_prebuilt(P.L)) {
            // one class per pass: pass b adds into the y that pass b - 1 wrote
            const size_t vb = storage_bytes(A->storage);
            for (int b = 0; b < P.cblocks; ++b) {
                BatchMat M = base_desc(A, x[k], y[k]);
                const int64_t o = A->cb_nnz_off[b];
                M.rp = A->cb_rp.as<int32_t>() + (size_t)b * (A->n_rows + 1);
                if (A->cb_split && b > 0) {  // split rows: the block's row list
                    M.rp = A->cb_rrp.as<int32_t>() + A->cb_rrp_off[b];
                    M.rowid = A->cb_rid.as<int32_t>() + A->cb_rid_off[b];
                    M.n_rows = (int32_t)A->cb_rows[b];
                }
                M.col = A->cb_col.as<int32_t>() + o;
                M.val = A->cb_val.as<char>() + vb * (size_t)o;
                M.tile_i = A->cb_tile_i.as<int32_t>() + A->cb_tile_off[b];
                M.tile_j = A->cb_tile_j.as<int32_t>() + A->cb_tile_off[b];
                M.acc = b > 0;
                M.carry = A->carry.p;  // tiles not row-aligned: the pass's carries
                add(ClassKey{b, K_MERGE, P.L / kMergeBlock, IDX_I32, 0, x32, A->tiles_fixup == 0, 0,
                             0},
                    M, k, A->cb_tiles[b], 0);
            }
        } else if ((P.opts & CSR_OPT_MERGE) && merge_items_prebuilt(P.L)) {
            BatchMat M = base_desc(A, x[k], y[k]);
            M.tile_i = A->tile_i.as<int32_t>();
            M.tile_j = A->tile_j.as<int32_t>();
            M.carry = A->carry.p;
            if (P.idx == IDX_W8 || P.idx == IDX_W9) {
                M.codes = A->wcodes.p;
                M.wdict = A->wdict.as<uint16_t>();
                M.wlen = A->wlen.as<int32_t>();
            } else if (P.idx == IDX_R8) {
                M.codes = A->wcodes.p;
                M.wlen = A->wruns.as<int32_t>();  // the tiles' run records
            } else if (P.idx != IDX_I32) {
                M.codes = A->mcodes.p;
            }
            if (P.idx != IDX_I32) M.tile_base = A->tile_base.as<int32_t>();
            const bool aln = A->tiles_fixup == 0;
            const bool nt = P.idx != IDX_I32 || P.nt;
            const bool xx = P.idx == IDX_I32 && x32;
            add(ClassKey{0, K_MERGE, P.L / kMergeBlock, P.idx, nt, xx, aln, 0, 0}, M, k,
                A->n_tiles, 0);
        } else if (P.opts & CSR_OPT_MERGE) {
            ClassRun r;  // a tile size compiled at run time: its own launches
            r.key = ClassKey{0, K_OWN, own++, 0, 0, 0, 0, 0, 0};
            r.matrix = k;
            cls[r.key] = r;
            B.has_own = true;
        } else {
            BatchMat M = base_desc(A, x[k], y[k]);
            M.codes = P.idx != IDX_I32 ? A->codes.p : nullptr;
            if (P.long_rows) M.skip_above = (int32_t)A->long_tau;
            const int R = rows_eff_R(P), U = rows_eff_U(P);
            const int64_t per = (int64_t)(kBlock / P.G) * R;
            add(ClassKey{0, K_ROWS, P.G, P.idx, P.nt, 0, 0, U, R}, M, k,
                (A->n_rows + per - 1) / per, 0);
            if (P.long_rows && A->n_long > 0) {
                BatchMat L = base_desc(A, x[k], y[k]);
                L.long_rows = A->long_list.as<int32_t>();
                L.row_chunk = A->long_row_chunk.as<int32_t>();
                L.chunks = A->long_chunks.as<int32_t>();
                L.carry = A->long_part.p;
                add(ClassKey{0, K_LONG, 0, 0, 0, 0, 0, 0, 0}, L, k, A->n_long_chunks, A->n_long);
            }
        }
    }
    // launch order: the key's order (column-block pass first, so every pass
    // of a matrix follows the previous one)
    int64_t off = 0;
    for (auto &kv : cls) {
        ClassRun r = kv.second;
        r.item_off = off;
        off += r.n_items;
        r.item_off2 = off;
        off += r.n_items2;
        B.runs.push_back(std::move(r));
    }
}

hipError_t launch_run(const BatchPlan &B, const ClassRun &r, hipStream_t s) {
    const int n_cu = device_cu_count(B.device);
    if (std::get<1>(r.key) == K_OWN) {
        const csr_matrix_s *A = B.mats[r.matrix];
        return launch_spmv(A, A->plan, B.xs[r.matrix], B.ys[r.matrix], s);
    }
    const BatchMat *m = B.desc.as<BatchMat>();
    const int32_t *im = B.items.as<int32_t>() + r.item_off;
    const int32_t *im2 = B.items.as<int32_t>() + r.item_off2;
    const int kind = std::get<1>(r.key), a = std::get<2>(r.key), idx = std::get<3>(r.key);
    const bool nt = std::get<4>(r.key), x32 = std::get<5>(r.key), aln = std::get<6>(r.key);
    const int U = std::get<7>(r.key), R = std::get<8>(r.key);
    switch (kind) {
    case K_MERGE:
        switch (B.storage) {
        case CSR_VAL_F64: return launch_bmerge_s0(a, nt, x32, idx, aln, m, im, r.n_items, n_cu, s);
        case CSR_VAL_F32: return launch_bmerge_s1(a, nt, x32, idx, aln, m, im, r.n_items, n_cu, s);
        default: return launch_bmerge_s2(a, nt, x32, idx, aln, m, im, r.n_items, n_cu, s);
        }
    case K_ROWS:
        switch (B.storage) {
        case CSR_VAL_F64: return launch_brows_s0(a, idx, nt, U, R, m, im, r.n_items, n_cu, s);
        case CSR_VAL_F32: return launch_brows_s1(a, idx, nt, U, R, m, im, r.n_items, n_cu, s);
        default: return launch_brows_s2(a, idx, nt, U, R, m, im, r.n_items, n_cu, s);
        }
    default:
        switch (B.storage) {
        case CSR_VAL_F64: return launch_blong_s0(m, im, r.n_items, im2, r.n_items2, n_cu, s);
        case CSR_VAL_F32: return launch_blong_s1(m, im, r.n_items, im2, r.n_items2, n_cu, s);
        default: return launch_blong_s2(m, im, r.n_items, im2, r.n_items2, n_cu, s);
        }
    }
}

// Descriptors and item tables on the device.
csr_status_t upload(BatchPlan &B, hipStream_t s) {
    int64_t n_items = 0;
    for (const ClassRun &r : B.runs) n_items = std::max(n_items, r.item_off2 + r.n_items2);
    std::vector<int32_t> im((size_t)n_items, 0);
    for (const ClassRun &r : B.runs) {
        // a descriptor's items run up to the next descriptor's first ones
        for (size_t q = 0; q < r.descs.size(); ++q) {
            const int d = r.descs[q];
            const BatchMat &M = B.desc_h[d];
            const bool last = q + 1 == r.descs.size();
            const int64_t e1 = last ? r.n_items : B.desc_h[r.descs[q + 1]].item_base;
            const int64_t e2 = last ? r.n_items2 : B.desc_h[r.descs[q + 1]].item_base2;
            std::fill(im.begin() + r.item_off + M.item_base, im.begin() + r.item_off + e1, d);
            std::fill(im.begin() + r.item_off2 + M.item_base2, im.begin() + r.item_off2 + e2, d);
        }
    }
    const size_t db = sizeof(BatchMat) * std::max<size_t>(B.desc_h.size(), 1);
    csr_status_t st;
    if ((st = B.desc.alloc(db)) != CSR_OK) return st;
    if ((st = B.items.alloc(sizeof(int32_t) * std::max<int64_t>(n_items, 1))) != CSR_OK) return st;
    if ((st = B.desc_pin.alloc(db)) != CSR_OK) return st;
    CSR_HIP(hipEventCreateWithFlags(&B.refreshed, hipEventDisableTiming));
    if (!B.desc_h.empty()) {
        std::memcpy(B.desc_pin.p, B.desc_h.data(), sizeof(BatchMat) * B.desc_h.size());
        CSR_HIP(hipMemcpyAsync(B.desc.p, B.desc_pin.p, sizeof(BatchMat) * B.desc_h.size(),
                               hipMemcpyHostToDevice, s));
    }
    if (n_items > 0)
        CSR_HIP(hipMemcpyAsync(B.items.p, im.data(), sizeof(int32_t) * im.size(),
                               hipMemcpyHostToDevice, s));
    CSR_HIP(hipStreamSynchronize(s));
    return CSR_OK;
}

// Streams and events of one capture, released on every path.
struct CaptureRes {
    hipStream_t cs = nullptr;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev;
    ~CaptureRes() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        for (hipStream_t s : side) (void)hipStreamDestroy(s);
        if (cs) (void)hipStreamDestroy(cs);
    }
    hipError_t event(hipEvent_t *out) {
        hipError_t e = hipEventCreateWithFlags(out, hipEventDisableTiming);
        if (e == hipSuccess) ev.push_back(*out);
        return e;
    }
};

// The classes of one column-block pass touch disjoint rows (every matrix
// is in one class per pass; a decomposition plan's row blocks skip the
// long rows its long-row class writes), so they are captured as parallel
// branches (fork on an event, one side stream per class up to
// kCaptureStreams, join before the next pass); small classes then share
// the GPU instead of running one after another.
constexpr int kCaptureStreams = 8;

hipError_t capture_runs(const BatchPlan &B, CaptureRes &R) {
    hipError_t e = hipSuccess;
    size_t q = 0;
    while (q < B.runs.size() && e == hipSuccess) {
        const int pass = std::get<0>(B.runs[q].key);
        size_t q1 = q;
        while (q1 < B.runs.size() && std::get<0>(B.runs[q1].key) == pass) ++q1;
        hipEvent_t fork;
        if ((e = R.event(&fork)) != hipSuccess || (e = hipEventRecord(fork, R.cs)) != hipSuccess)
            break;
        const int nside = (int)std::min<size_t>(q1 - q, (size_t)kCaptureStreams);
        for (int k = 0; k < nside && e == hipSuccess; ++k)
            e = hipStreamWaitEvent(R.side[k], fork, 0);
        for (size_t r = q; r < q1 && e == hipSuccess; ++r)
            e = launch_run(B, B.runs[r], R.side[(r - q) % nside]);
        for (int k = 0; k < nside && e == hipSuccess; ++k) {
            hipEvent_t done;
            if ((e = R.event(&done)) == hipSuccess && (e = hipEventRecord(done, R.side[k])) == hipSuccess)
                e = hipStreamWaitEvent(R.cs, done, 0);
        }
        q = q1;
    }
    return e;
}

csr_status_t capture(BatchPlan &B) {
    if (B.exec) (void)hipGraphExecDestroy(B.exec);
    if (B.graph) (void)hipGraphDestroy(B.graph);
    B.exec = nullptr;
    B.graph = nullptr;
    CaptureRes R;
    CSR_HIP(hipStreamCreateWithFlags(&R.cs, hipStreamNonBlocking));
    for (int k = 0; k < kCaptureStreams; ++k) {
        hipStream_t s2;
        CSR_HIP(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
        R.side.push_back(s2);
    }
    hipError_t e = hipStreamBeginCapture(R.cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t le = capture_runs(B, R);
        e = hipStreamEndCapture(R.cs, &B.graph);
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0);
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
        if (!plan_tables_ok(A, A->plan))
            return fail(CSR_ERR_NOT_READY, "a plan's tables are not in place");
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
        auto fresh = std::make_unique<BatchPlan>();
        fresh->key = key;
        fresh->storage = storage;
        fresh->device = dev;
        fresh->count = count;
        fresh->mats.assign(h_A, h_A + count);
        fresh->xs.assign(h_x, h_x + count);
        fresh->ys.assign(h_y, h_y + count);
        plan_classes(*fresh, h_A, h_x, h_y);
        csr_status_t st;
        if ((st = upload(*fresh, s)) != CSR_OK) return st;
        if ((st = capture(*fresh)) != CSR_OK) return st;
        if (plans.size() >= kMaxPlans) plans.erase(plans.begin());
        plans.push_back(std::move(fresh));
        B = plans.back().get();
    } else {
        // new vector pointers: refresh the descriptors through the pinned
        // staging buffer, once the previous refresh copy has read it (the
        // copy and the graph's kernels are ordered on the stream); launches
        // captured with their vectors are captured again
        bool moved = false;
        for (int k = 0; k < count; ++k)
            moved = moved || B->xs[k] != h_x[k] || B->ys[k] != h_y[k];
        if (moved) {
            B->xs.assign(h_x, h_x + count);
            B->ys.assign(h_y, h_y + count);
            for (size_t d = 0; d < B->desc_h.size(); ++d) {
                B->desc_h[d].x = h_x[B->desc_matrix[d]];
                B->desc_h[d].y = h_y[B->desc_matrix[d]];
            }
            CSR_HIP(hipEventSynchronize(B->refreshed));
            if (!B->desc_h.empty()) {
                std::memcpy(B->desc_pin.p, B->desc_h.data(), sizeof(BatchMat) * B->desc_h.size());
                CSR_HIP(hipMemcpyAsync(B->desc.p, B->desc_pin.p,
                                       sizeof(BatchMat) * B->desc_h.size(),
                                       hipMemcpyHostToDevice, s));
            }
            CSR_HIP(hipEventRecord(B->refreshed, s));
            if (B->has_own) {
                csr_status_t st = capture(*B);
                if (st != CSR_OK) return st;
            }
        }
    }
    CSR_HIP(hipGraphLaunch(B->exec, s));
    return CSR_OK;
}
