// Run-time specialization of the merge-path kernel: the counterpart of the
// paper's just-in-time code generation for the selected optimizations
// (Sec. IV-D). The library holds k_merge for tile sizes L = 256, 512 and
// 1024 ahead of time; any other L = 64 * IPT (IPT a multiple of 4 up to 32)
// is compiled on first use with hipRTC from the same headers (embedded at
// build time), with the same code-generation flags, and the module is kept
// for the life of the process (one per device and instance).
#include <hip/hiprtc.h>

#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"
#include "jit_sources.inc"

namespace csr {
namespace {

struct JitKey {
    int device, storage, ipt, nt, x32, idx, aln;
    bool operator<(const JitKey &o) const {
        return std::tie(device, storage, ipt, nt, x32, idx, aln) <
               std::tie(o.device, o.storage, o.ipt, o.nt, o.x32, o.idx, o.aln);
    }
};

std::mutex g_jit_mu;
// Loaded kernels; their modules are never unloaded (launches may be in
// flight or captured in graphs until the process ends).
std::map<JitKey, hipFunction_t> *const g_jit = new std::map<JitKey, hipFunction_t>;

// The instance a launch uses: merge codes and window codes always stream and
// gather with 64-bit offsets (as the ahead-of-time dispatch does).
JitKey normalize(int device, int storage, int ipt, bool nt, bool x32, int idx, bool aln) {
    const bool codes = idx != IDX_I32;
    return JitKey{device, storage, ipt, codes ? 1 : (int)nt, codes ? 0 : (int)x32, idx, (int)aln};
}

std::string kernel_expr(const JitKey &k) {
    auto b = [](int v) { return v ? "true" : "false"; };
    return "csr::k_merge<" + std::to_string(k.ipt) + ", " + b(k.nt) + ", " + b(k.x32) + ", " +
           std::to_string(k.idx) + ", " + b(k.aln) + ">";
}

csr_status_t check_instance(int storage, int ipt, int idx, bool aln) {
    if (storage < CSR_VAL_F64 || storage > CSR_VAL_BF16)
        return fail(CSR_ERR_INVALID_ARG, "unknown value storage");
    if (!merge_items_supported(64 * ipt))
        return fail(CSR_ERR_INVALID_ARG, "merge tile size must be 64 * IPT, IPT = 4, 8, ..., 32");
    if (idx < IDX_I32 || idx > IDX_R8) return fail(CSR_ERR_INVALID_ARG, "unknown index mode");
    if ((idx == IDX_W8 || idx == IDX_R8) && !aln)
        return fail(CSR_ERR_INVALID_ARG, "window codes need row-aligned tiles");
    if (idx != IDX_I32 && !merge_codes_fit(64 * ipt, idx == IDX_D16 ? 2 : 1))
        return fail(CSR_ERR_UNSUPPORTED, "merge codes do not form whole loads at this tile size");
    return CSR_OK;
}

#define RTC_CHECK(call, what)                                                              \
    do {                                                                                   \
        const hiprtcResult _r = (call);                                                    \
        if (_r != HIPRTC_SUCCESS)                                                          \
            return fail(CSR_ERR_DEVICE, std::string(what) + ": " + hiprtcGetErrorString(_r)); \
    } while (0)

// Compile one instance; the code object and the kernel's symbol on success.
csr_status_t compile(const JitKey &k, std::vector<char> *code, std::string *symbol) {
    const std::string expr = kernel_expr(k);
    hiprtcProgram prog;
    RTC_CHECK(hiprtcCreateProgram(&prog, "#include \"merge_kernel.h\"\n", "k_merge_jit.hip",
                                  kJitHeaderCount, kJitHeaders, kJitHeaderNames),
              "hiprtcCreateProgram");
    struct Destroy {
        hiprtcProgram *p;
        ~Destroy() { (void)hiprtcDestroyProgram(p); }
    } destroy{&prog};
    RTC_CHECK(hiprtcAddNameExpression(prog, expr.c_str()), "hiprtcAddNameExpression");
    const std::string storage_def = "-DCSR_STORAGE=" + std::to_string(k.storage);
    // the ahead-of-time flags: gfx950, -O3, C++17, no packed FP32 instructions
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", storage_def.c_str(),
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        std::string log;
        if (hiprtcGetProgramLogSize(prog, &n) == HIPRTC_SUCCESS && n > 1) {
            log.resize(n);
            (void)hiprtcGetProgramLog(prog, &log[0]);
            if (log.size() > 2000) log.resize(2000);
        }
        return fail(CSR_ERR_UNSUPPORTED, "run-time compilation of " + expr + " failed: " + log);
    }
    const char *lowered = nullptr;
    RTC_CHECK(hiprtcGetLoweredName(prog, expr.c_str(), &lowered), "hiprtcGetLoweredName");
    size_t n = 0;
    RTC_CHECK(hiprtcGetCodeSize(prog, &n), "hiprtcGetCodeSize");
    code->resize(n);
    RTC_CHECK(hiprtcGetCode(prog, code->data()), "hiprtcGetCode");
    *symbol = lowered;
    return CSR_OK;
}

}  // namespace

bool merge_items_prebuilt(int64_t L) { return L == 256 || L == 512 || L == 1024; }

bool merge_items_supported(int64_t L) {
    return L >= 256 && L <= 2048 && L % 256 == 0;
}

bool merge_codes_fit(int64_t L, int code_bytes) {
    // a lane's IPT codes are loaded as whole vectors of at most 16 bytes
    const int64_t b = L / kMergeBlock * code_bytes;
    return b < 16 ? (b == 2 || b == 4 || b == 8) : b % 16 == 0;
}

csr_status_t jit_merge_kernel(int device, int storage, int ipt, bool nt, bool x32, int idx,
                              bool aln, hipFunction_t *out) {
    csr_status_t st;
    if ((st = check_instance(storage, ipt, idx, aln)) != CSR_OK) return st;
    const JitKey k = normalize(device, storage, ipt, nt, x32, idx, aln);
    std::lock_guard<std::mutex> lk(g_jit_mu);
    auto it = g_jit->find(k);
    if (it != g_jit->end()) {
        *out = it->second;
        return CSR_OK;
    }
    std::vector<char> code;
    std::string symbol;
    if ((st = compile(k, &code, &symbol)) != CSR_OK) return st;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != device) CSR_HIP(hipSetDevice(device));
    hipModule_t mod;
    hipFunction_t f;
    hipError_t e = hipModuleLoadData(&mod, code.data());
    if (e == hipSuccess) e = hipModuleGetFunction(&f, mod, symbol.c_str());
    if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return hip_fail(e, "loading the run-time compiled merge kernel");
    (*g_jit)[k] = f;
    *out = f;
    return CSR_OK;
}

}  // namespace csr

using namespace csr;

extern "C" csr_status_t csr_jit_compile(int32_t storage, int32_t merge_items, int32_t index_mode,
                                        int32_t streaming, int32_t row_aligned, void *code,
                                        size_t bytes, size_t *needed) {
    if (merge_items % kMergeBlock != 0)
        return fail(CSR_ERR_INVALID_ARG, "merge tile size must be a multiple of 64");
    const int ipt = merge_items / kMergeBlock;
    csr_status_t st;
    if ((st = check_instance(storage, ipt, index_mode, row_aligned != 0)) != CSR_OK) return st;
    const JitKey k = normalize(-1, storage, ipt, streaming != 0, false, index_mode, row_aligned != 0);
    std::vector<char> obj;
    std::string symbol;
    if ((st = compile(k, &obj, &symbol)) != CSR_OK) return st;
    if (needed) *needed = obj.size();
    if (!code) return CSR_OK;
    if (bytes != obj.size()) return fail(CSR_ERR_INVALID_ARG, "size mismatch");
    std::memcpy(code, obj.data(), obj.size());
    return CSR_OK;
}
