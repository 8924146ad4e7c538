// C ABI of the learned selector: MLP training and inference kernels exposed
// for the training driver and the parity tests, and the per-device model used
// by CSR_SEL_LEARNED.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "internal.h"

namespace csr {

namespace {

struct Model {
    DevBuf params, mu, sigma, feat, pick;
    HostBuf io;  // pinned staging: 16 features in, the pick out
    double h_mu[16] = {}, h_sigma[16] = {};  // the normalization, for the range test
    int K = 0;
    bool ready = false;
};

std::mutex g_model_mu;
// Never freed: device memory is released with the process, and no destructor
// may call into the HIP runtime after it has shut down.
Model *const g_models = new Model[64];

csr_status_t check_model_args(int K) {
    if (K < 2 || K > mlp_max_classes()) return fail(CSR_ERR_INVALID_ARG, "K out of range");
    return CSR_OK;
}

}  // namespace

// Runs the loaded model on the handle's features; *variant = argmax.
// *z_max = the largest |standardized feature| (the model's input). Returns
// CSR_ERR_NOT_READY, so that selection falls back to the profile-guided
// rule, when no model is loaded on the device, when a feature is not
// finite, or when z_max exceeds ood_z > 0 (a matrix outside the range the
// model was trained on).
csr_status_t learned_pick(csr_matrix_s *A, hipStream_t s, double ood_z, int32_t *variant,
                          double *z_max) {
    std::lock_guard<std::mutex> lk(g_model_mu);
    *z_max = 0.0;
    if (A->device < 0 || A->device >= 64 || !g_models[A->device].ready)
        return fail(CSR_ERR_NOT_READY, "no model loaded");
    Model &M = g_models[A->device];
    for (int i = 0; i < 16; ++i)
        if (!std::isfinite(A->feat.f[i])) return fail(CSR_ERR_NOT_READY, "non-finite feature");
    double zm = 0.0;
    for (int i = 0; i < 16; ++i)
        zm = std::max(zm, std::fabs((std::log2(1.0 + A->feat.f[i]) - M.h_mu[i]) / M.h_sigma[i]));
    *z_max = zm;
    if (ood_z > 0.0 && !(zm <= ood_z))
        return fail(CSR_ERR_NOT_READY, "features outside the model's training range");
    double *const hf = static_cast<double *>(M.io.p);
    int32_t *const hp = reinterpret_cast<int32_t *>(hf + 16);
    std::memcpy(hf, A->feat.f, sizeof(double) * 16);
    CSR_HIP(hipMemcpyAsync(M.feat.p, hf, sizeof(double) * 16, hipMemcpyHostToDevice, s));
    CSR_HIP(launch_mlp_select(M.params.as<float>(), M.K, M.feat.as<double>(), M.mu.as<double>(),
                              M.sigma.as<double>(), M.pick.as<int32_t>(), s));
    CSR_HIP(hipMemcpyAsync(hp, M.pick.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    CSR_HIP(hipStreamSynchronize(s));
    *variant = *hp;
    return CSR_OK;
}

}  // namespace csr

using namespace csr;

extern "C" {

csr_status_t csr_mlp_load(const float *h_params, int32_t K, const double *h_mu,
                          const double *h_sigma) {
    if (!h_params || !h_mu || !h_sigma) return fail(CSR_ERR_INVALID_ARG, "NULL model array");
    csr_status_t st = check_model_args(K);
    if (st != CSR_OK) return st;
    for (int i = 0; i < 16; ++i)
        if (!(h_sigma[i] > 0.0) || !std::isfinite(h_mu[i]))
            return fail(CSR_ERR_INVALID_ARG, "normalization must be finite with sigma > 0");
    const int n = mlp_param_count(K);
    for (int q = 0; q < n; ++q)
        if (!std::isfinite(h_params[q])) return fail(CSR_ERR_INVALID_ARG, "non-finite weight");
    int dev = 0;
    CSR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(CSR_ERR_UNSUPPORTED, "device index");
    std::lock_guard<std::mutex> lk(g_model_mu);
    Model &M = g_models[dev];
    M.ready = false;
    if ((st = M.params.alloc(sizeof(float) * n)) != CSR_OK) return st;
    if ((st = M.mu.alloc(sizeof(double) * 16)) != CSR_OK) return st;
    if ((st = M.sigma.alloc(sizeof(double) * 16)) != CSR_OK) return st;
    if ((st = M.feat.alloc(sizeof(double) * 16)) != CSR_OK) return st;
    if ((st = M.pick.alloc(sizeof(int32_t))) != CSR_OK) return st;
    if (!M.io.p && (st = M.io.alloc(sizeof(double) * 16 + sizeof(int32_t) * 2)) != CSR_OK)
        return st;
    CSR_HIP(hipMemcpy(M.params.p, h_params, sizeof(float) * n, hipMemcpyHostToDevice));
    CSR_HIP(hipMemcpy(M.mu.p, h_mu, sizeof(double) * 16, hipMemcpyHostToDevice));
    CSR_HIP(hipMemcpy(M.sigma.p, h_sigma, sizeof(double) * 16, hipMemcpyHostToDevice));
    std::memcpy(M.h_mu, h_mu, sizeof(M.h_mu));
    std::memcpy(M.h_sigma, h_sigma, sizeof(M.h_sigma));
    M.K = K;
    M.ready = true;
    return CSR_OK;
}

csr_status_t csr_mlp_unload(void) {
    int dev = 0;
    CSR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(CSR_ERR_UNSUPPORTED, "device index");
    std::lock_guard<std::mutex> lk(g_model_mu);
    g_models[dev].ready = false;
    return CSR_OK;
}

csr_status_t csr_mlp_forward(const float *d_params, int32_t K, const float *d_X, int32_t B,
                             float *d_logits, void *stream) {
    csr_status_t st = check_model_args(K);
    if (st != CSR_OK) return st;
    if (!d_params || !d_X || !d_logits || B < 1 || B > mlp_max_batch())
        return fail(CSR_ERR_INVALID_ARG, "bad forward arguments");
    CSR_HIP(launch_mlp_forward(d_params, K, d_X, B, d_logits, (hipStream_t)stream));
    return CSR_OK;
}

csr_status_t csr_mlp_grad(const float *d_params, int32_t K, const float *d_X,
                          const int32_t *d_labels, int32_t B, float *d_grad, float *d_loss,
                          void *stream) {
    csr_status_t st = check_model_args(K);
    if (st != CSR_OK) return st;
    if (!d_params || !d_X || !d_labels || !d_grad || !d_loss || B < 1 || B > mlp_max_batch())
        return fail(CSR_ERR_INVALID_ARG, "bad gradient arguments");
    CSR_HIP(launch_mlp_grad(d_params, K, d_X, d_labels, B, d_grad, d_loss, (hipStream_t)stream));
    return CSR_OK;
}

csr_status_t csr_mlp_train(float *d_params, float *d_m, float *d_v, int32_t K, const float *d_X,
                           const int32_t *d_labels, const int32_t *d_order, int32_t B,
                           int32_t steps, int32_t t0, float lr, float beta1, float beta2,
                           float eps, float *d_losses, void *stream) {
    csr_status_t st = check_model_args(K);
    if (st != CSR_OK) return st;
    if (!d_params || !d_m || !d_v || !d_X || !d_labels || !d_order || !d_losses || B < 1 ||
        B > mlp_max_batch() || steps < 0 || t0 < 0 || !(lr > 0.f))
        return fail(CSR_ERR_INVALID_ARG, "bad training arguments");
    if (steps == 0) return CSR_OK;
    DevBuf g;
    if ((st = g.alloc(sizeof(float) * mlp_param_count(K))) != CSR_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    CSR_HIP(launch_mlp_train(d_params, d_m, d_v, g.as<float>(), K, d_X, d_labels, d_order, B,
                             steps, t0, lr, beta1, beta2, eps, d_losses, s));
    CSR_HIP(hipStreamSynchronize(s));  // the gradient scratch is freed on return
    return CSR_OK;
}

csr_status_t csr_mlp_normalize(const double *d_f, const double *d_mu, const double *d_sigma,
                               int64_t n, float *d_out, void *stream) {
    if (n < 0 || (n > 0 && (!d_f || !d_mu || !d_sigma || !d_out)))
        return fail(CSR_ERR_INVALID_ARG, "bad normalize arguments");
    CSR_HIP(launch_mlp_normalize(d_f, d_mu, d_sigma, n, d_out, (hipStream_t)stream));
    return CSR_OK;
}

}  // extern "C"
