// The learned selector: an MLP 16-64-64-K (ReLU hidden layers, softmax
// cross-entropy on timed-best variant labels) that replaces the decision tree
// of the feature-guided classifier (Sec. III-D). Inference, gradients and
// Adam (Kingma & Ba 2015) are hand-written FP32 kernels; one 256-thread
// workgroup holds a whole mini-batch in LDS. Every sum runs in a fixed order,
// so training is bit-reproducible.
//
// Parameter layout (floats): W1[64][16], b1[64], W2[64][64], b2[64],
// W3[K][64], b3[K]  (6,288 values for K = 16).
#include "device.h"
#include "internal.h"

namespace csr {

namespace {

constexpr int kIn = 16, kH = 64, kMaxK = 16, kMaxB = 64;
constexpr int kParams(int K) { return kH * kIn + kH + kH * kH + kH + K * kH + K; }

struct Offs {
    int w1, b1, w2, b2, w3, b3, n;
    __host__ __device__ explicit Offs(int K) {
        w1 = 0;
        b1 = w1 + kH * kIn;
        w2 = b1 + kH;
        b2 = w2 + kH * kH;
        w3 = b2 + kH;
        b3 = w3 + K * kH;
        n = b3 + K;
    }
};

struct Act {
    float x[kMaxB][kIn];
    float h1[kMaxB][kH];
    float h2[kMaxB][kH];
    float z[kMaxB][kMaxK];   // logits, then dL/dlogits
    float g2[kMaxB][kH];     // dL/dh2 (pre-activation)
};  // 56 KiB; dL/dh1 reuses h2 once h2 is no longer needed

// forward pass of B rows of act.x; logits in act.z
__device__ void mlp_forward(const float *__restrict__ p, int K, int B, Act &a) {
    const Offs o(K);
    const int tid = threadIdx.x;
    for (int q = tid; q < B * kH; q += kBlock) {
        const int b = q / kH, j = q % kH;
        float s = p[o.b1 + j];
        for (int i = 0; i < kIn; ++i) s = fmaf(p[o.w1 + j * kIn + i], a.x[b][i], s);
        a.h1[b][j] = s > 0.f ? s : 0.f;
    }
    __syncthreads();
    for (int q = tid; q < B * kH; q += kBlock) {
        const int b = q / kH, j = q % kH;
        float s = p[o.b2 + j];
        for (int i = 0; i < kH; ++i) s = fmaf(p[o.w2 + j * kH + i], a.h1[b][i], s);
        a.h2[b][j] = s > 0.f ? s : 0.f;
    }
    __syncthreads();
    for (int q = tid; q < B * K; q += kBlock) {
        const int b = q / K, j = q % K;
        float s = p[o.b3 + j];
        for (int i = 0; i < kH; ++i) s = fmaf(p[o.w3 + j * kH + i], a.h2[b][i], s);
        a.z[b][j] = s;
    }
    __syncthreads();
}

// loss (mean softmax cross-entropy) and gradients (mean over the batch) into g
__device__ float mlp_backward(const float *__restrict__ p, float *__restrict__ g,
                              const int32_t *__restrict__ labels, int K, int B, Act &a,
                              float *s_loss) {
    const Offs o(K);
    const int tid = threadIdx.x;
    const float invB = 1.0f / (float)B;
    // dL/dz = (softmax - onehot) / B, per row
    if (tid < B) {
        const int b = tid;
        float m = a.z[b][0];
        for (int j = 1; j < K; ++j) m = fmaxf(m, a.z[b][j]);
        float den = 0.f;
        for (int j = 0; j < K; ++j) den += expf(a.z[b][j] - m);
        const int y = labels[b];
        s_loss[b] = -((a.z[b][y] - m) - logf(den));
        for (int j = 0; j < K; ++j) {
            const float pj = expf(a.z[b][j] - m) / den;
            a.z[b][j] = (pj - (j == y ? 1.f : 0.f)) * invB;
        }
    }
    __syncthreads();
    // dW3, db3
    for (int q = tid; q < K * kH; q += kBlock) {
        const int j = q / kH, i = q % kH;
        float s = 0.f;
        for (int b = 0; b < B; ++b) s = fmaf(a.z[b][j], a.h2[b][i], s);
        g[o.w3 + q] = s;
    }
    for (int j = tid; j < K; j += kBlock) {
        float s = 0.f;
        for (int b = 0; b < B; ++b) s += a.z[b][j];
        g[o.b3 + j] = s;
    }
    // dh2 (through ReLU)
    for (int q = tid; q < B * kH; q += kBlock) {
        const int b = q / kH, i = q % kH;
        float s = 0.f;
        for (int j = 0; j < K; ++j) s = fmaf(a.z[b][j], p[o.w3 + j * kH + i], s);
        a.g2[b][i] = a.h2[b][i] > 0.f ? s : 0.f;
    }
    __syncthreads();
    for (int q = tid; q < kH * kH; q += kBlock) {
        const int j = q / kH, i = q % kH;
        float s = 0.f;
        for (int b = 0; b < B; ++b) s = fmaf(a.g2[b][j], a.h1[b][i], s);
        g[o.w2 + q] = s;
    }
    for (int j = tid; j < kH; j += kBlock) {
        float s = 0.f;
        for (int b = 0; b < B; ++b) s += a.g2[b][j];
        g[o.b2 + j] = s;
    }
    float(*g1)[kH] = a.h2;  // h2 was last read before the barrier above
    for (int q = tid; q < B * kH; q += kBlock) {
        const int b = q / kH, i = q % kH;
        float s = 0.f;
        for (int j = 0; j < kH; ++j) s = fmaf(a.g2[b][j], p[o.w2 + j * kH + i], s);
        g1[b][i] = a.h1[b][i] > 0.f ? s : 0.f;
    }
    __syncthreads();
    for (int q = tid; q < kH * kIn; q += kBlock) {
        const int j = q / kIn, i = q % kIn;
        float s = 0.f;
        for (int b = 0; b < B; ++b) s = fmaf(g1[b][j], a.x[b][i], s);
        g[o.w1 + q] = s;
    }
    for (int j = tid; j < kH; j += kBlock) {
        float s = 0.f;
        for (int b = 0; b < B; ++b) s += g1[b][j];
        g[o.b1 + j] = s;
    }
    __syncthreads();
    float l = 0.f;
    if (tid == 0)
        for (int b = 0; b < B; ++b) l += s_loss[b];
    return l * invB;
}

__device__ void load_batch(Act &a, const float *__restrict__ X, const int32_t *__restrict__ idx,
                           int B) {
    for (int q = threadIdx.x; q < B * kIn; q += kBlock) {
        const int b = q / kIn, i = q % kIn;
        a.x[b][i] = X[(int64_t)(idx ? idx[b] : b) * kIn + i];
    }
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_mlp_forward(const float *__restrict__ p, int K,
                                                        const float *__restrict__ X, int B,
                                                        float *__restrict__ logits) {
    __shared__ Act a;
    load_batch(a, X, nullptr, B);
    mlp_forward(p, K, B, a);
    for (int q = threadIdx.x; q < B * K; q += kBlock) logits[q] = a.z[q / K][q % K];
}

__global__ __launch_bounds__(kBlock) void k_mlp_grad(const float *__restrict__ p, int K,
                                                     const float *__restrict__ X,
                                                     const int32_t *__restrict__ labels, int B,
                                                     float *__restrict__ g,
                                                     float *__restrict__ loss) {
    __shared__ Act a;
    __shared__ float s_loss[kMaxB];
    load_batch(a, X, nullptr, B);
    mlp_forward(p, K, B, a);
    const float l = mlp_backward(p, g, labels, K, B, a, s_loss);
    if (threadIdx.x == 0) *loss = l;
}

// Whole training run: `steps` Adam steps over mini-batches whose rows come
// from `order` (steps * B indices into X), bias-corrected Adam with step
// counter t = t0+1, t0+2, ...; loss of every step written to losses.
__global__ __launch_bounds__(kBlock) void k_mlp_train(float *__restrict__ p, float *__restrict__ m,
                                                      float *__restrict__ v, float *__restrict__ g,
                                                      int K, const float *__restrict__ X,
                                                      const int32_t *__restrict__ y,
                                                      const int32_t *__restrict__ order, int B,
                                                      int steps, int t0, float lr, float b1,
                                                      float b2, float eps,
                                                      float *__restrict__ losses) {
    __shared__ Act a;
    __shared__ float s_loss[kMaxB];
    __shared__ int32_t s_lab[kMaxB];
    const Offs o(K);
    for (int st = 0; st < steps; ++st) {
        const int32_t *idx = order + (int64_t)st * B;
        if ((int)threadIdx.x < B) s_lab[threadIdx.x] = y[idx[threadIdx.x]];
        load_batch(a, X, idx, B);
        mlp_forward(p, K, B, a);
        const float l = mlp_backward(p, g, s_lab, K, B, a, s_loss);
        if (threadIdx.x == 0) losses[st] = l;
        const int t = t0 + st + 1;
        const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
        for (int q = threadIdx.x; q < o.n; q += kBlock) {
            const float gq = g[q];
            const float mq = b1 * m[q] + (1.f - b1) * gq;
            const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
            m[q] = mq;
            v[q] = vq;
            p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
        }
        __syncthreads();
    }
}

// f' = (log2(1 + f) - mu) / sigma for n feature rows
__global__ __launch_bounds__(kBlock) void k_mlp_normalize(const double *__restrict__ f,
                                                          const double *__restrict__ mu,
                                                          const double *__restrict__ sigma,
                                                          int64_t n, float *__restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= n * kIn) return;
    const int i = (int)(q % kIn);
    out[q] = (float)((log2(1.0 + f[q]) - mu[i]) / sigma[i]);
}

// One selection: normalize one feature row, forward, argmax (ties -> lower id)
__global__ __launch_bounds__(kBlock) void k_mlp_select(const float *__restrict__ p, int K,
                                                       const double *__restrict__ f,
                                                       const double *__restrict__ mu,
                                                       const double *__restrict__ sigma,
                                                       int32_t *__restrict__ out) {
    __shared__ Act a;
    if (threadIdx.x < kIn)
        a.x[0][threadIdx.x] =
            (float)((log2(1.0 + f[threadIdx.x]) - mu[threadIdx.x]) / sigma[threadIdx.x]);
    __syncthreads();
    mlp_forward(p, K, 1, a);
    if (threadIdx.x == 0) {
        int best = 0;
        for (int j = 1; j < K; ++j)
            if (a.z[0][j] > a.z[0][best]) best = j;
        *out = best;
    }
}

}  // namespace

int mlp_param_count(int K) { return kParams(K); }
int mlp_max_batch() { return kMaxB; }
int mlp_max_classes() { return kMaxK; }

hipError_t launch_mlp_forward(const float *p, int K, const float *X, int B, float *logits,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_forward, dim3(1), dim3(kBlock), 0, s, p, K, X, B, logits);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *p, int K, const float *X, const int32_t *labels, int B,
                           float *g, float *loss, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_grad, dim3(1), dim3(kBlock), 0, s, p, K, X, labels, B, g, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_train(float *p, float *m, float *v, float *g, int K, const float *X,
                            const int32_t *y, const int32_t *order, int B, int steps, int t0,
                            float lr, float b1, float b2, float eps, float *losses,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(kBlock), 0, s, p, m, v, g, K, X, y, order, B,
                       steps, t0, lr, b1, b2, eps, losses);
    return hipGetLastError();
}

hipError_t launch_mlp_normalize(const double *f, const double *mu, const double *sigma,
                                int64_t n, float *out, hipStream_t s) {
    const unsigned g = (unsigned)((n * kIn + kBlock - 1) / kBlock);
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_normalize, dim3(g), dim3(kBlock), 0, s, f, mu, sigma, n, out);
    return hipGetLastError();
}

hipError_t launch_mlp_select(const float *p, int K, const double *f, const double *mu,
                             const double *sigma, int32_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_select, dim3(1), dim3(kBlock), 0, s, p, K, f, mu, sigma, out);
    return hipGetLastError();
}

}  // namespace csr
