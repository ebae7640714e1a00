// The learned grid picker's network: a 2 x 64 FP32 multilayer perceptron
//   h1 = relu(W1 xn + b1),  h2 = relu(W2 h1 + b2),  y = W3 h2 + b3,
// xn = (x - mu) / sd, with hand-written forward, backward, loss and Adam
// kernels.  The paper picks the grid size with a rule of thumb (Sec. 4.3.3);
// the network is this library's learned replacement for it and never
// changes the join result, only K and the dense-tile split threshold.
//
// The sizes are tiny (one sample is ~0.26 MFLOP) and latency-bound, so the
// kernels run on FP32 VALU with fixed reduction orders: every result is
// deterministic for a given batch.  Parameters are one flat array:
//   [W1 (64 x D, row-major), b1 (64), W2 (64 x 64), b2 (64), W3 (2 x 64), b3 (2)].
#include "sj_internal.hpp"

namespace sj {
namespace {

constexpr int kH = 64;   // hidden width
constexpr int kOut = 2;  // (log2 K, log2 tau), standardised
constexpr int kMaxD = 4096;
constexpr int kSmallBatch = 16;  // up to this batch, the spread layer-1 kernel

struct Layout {
    int64_t w1, b1, w2, b2, w3, b3, total;
};

__host__ __device__ inline Layout layout(int D) {
    Layout L;
    L.w1 = 0;
    L.b1 = L.w1 + (int64_t)kH * D;
    L.w2 = L.b1 + kH;
    L.b2 = L.w2 + kH * kH;
    L.w3 = L.b2 + kH;
    L.b3 = L.w3 + kOut * kH;
    L.total = L.b3 + kOut;
    return L;
}

__device__ __forceinline__ float norm_in(const float* x, const float* mu, const float* sd, int i) {
    float v = x[i];
    if (mu) v = v - mu[i];
    if (sd) v = v / sd[i];
    return v;
}

// One workgroup of 256 threads per sample.  Layer 1: each wave owns 16 of
// the 64 outputs; lanes take strided inputs and the wave reduces with a
// fixed butterfly.  act (optional) receives [h1, h2] per sample.
__global__ __launch_bounds__(256) void k_mlp_fwd(const float* __restrict__ P, int D,
                                                 const float* __restrict__ X,
                                                 const float* __restrict__ mu,
                                                 const float* __restrict__ sd, int B,
                                                 float* __restrict__ Y, float* __restrict__ act) {
    __shared__ float xs[kMaxD];
    __shared__ float h1[kH], h2[kH];
    const int b = blockIdx.x;
    if (b >= B) return;
    const Layout L = layout(D);
    const float* x = X + (int64_t)b * D;
    for (int i = threadIdx.x; i < D; i += blockDim.x) xs[i] = norm_in(x, mu, sd, i);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = 0; k < kH / 4; ++k) {
        const int o = w * (kH / 4) + k;
        const float* row = P + L.w1 + (int64_t)o * D;
        float acc = 0.f;
        for (int i = lane; i < D; i += 64) acc = fmaf(row[i], xs[i], acc);
        for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
        if (lane == 0) h1[o] = fmaxf(acc + P[L.b1 + o], 0.f);
    }
    __syncthreads();
    if (threadIdx.x < kH) {
        const int o = threadIdx.x;
        float acc = P[L.b2 + o];
        for (int j = 0; j < kH; ++j) acc = fmaf(P[L.w2 + o * kH + j], h1[j], acc);
        h2[o] = fmaxf(acc, 0.f);
    }
    __syncthreads();
    if (threadIdx.x < kOut) {
        const int o = threadIdx.x;
        float acc = P[L.b3 + o];
        for (int j = 0; j < kH; ++j) acc = fmaf(P[L.w3 + o * kH + j], h2[j], acc);
        Y[(int64_t)b * kOut + o] = acc;
    }
    if (act && threadIdx.x < kH) {
        act[(int64_t)b * 2 * kH + threadIdx.x] = h1[threadIdx.x];
        act[(int64_t)b * 2 * kH + kH + threadIdx.x] = h2[threadIdx.x];
    }
}

// Small batches (inference): layer 1 spread over one workgroup per
// (hidden unit, sample), so the 64 x D weight matrix streams through many
// CUs at once, then layers 2 and 3 per sample.  Each dot product is reduced
// in a fixed order within its workgroup (deterministic; its rounding may
// differ from the per-sample kernel's in the last bits).
__global__ __launch_bounds__(256) void k_mlp_fwd_l1(const float* __restrict__ P, int D,
                                                    const float* __restrict__ X,
                                                    const float* __restrict__ mu,
                                                    const float* __restrict__ sd,
                                                    float* __restrict__ H1) {
    __shared__ float red[256 / 64];
    const int o = blockIdx.x, b = blockIdx.y;
    const Layout L = layout(D);
    const float* row = P + L.w1 + (int64_t)o * D;
    const float* x = X + (int64_t)b * D;
    float acc = 0.f;
    for (int i = threadIdx.x; i < D; i += blockDim.x) acc = fmaf(row[i], norm_in(x, mu, sd, i), acc);
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int w = 0; w < 4; ++w) t += red[w];
        H1[(int64_t)b * kH + o] = fmaxf(t + P[L.b1 + o], 0.f);
    }
}

__global__ __launch_bounds__(64) void k_mlp_fwd_l23(const float* __restrict__ P, int D,
                                                    const float* __restrict__ H1, int B,
                                                    float* __restrict__ Y, float* __restrict__ act) {
    __shared__ float h1[kH], h2[kH];
    const int b = blockIdx.x, o = threadIdx.x;
    if (b >= B) return;
    const Layout L = layout(D);
    h1[o] = H1[(int64_t)b * kH + o];
    __syncthreads();
    float acc = P[L.b2 + o];
    for (int j = 0; j < kH; ++j) acc = fmaf(P[L.w2 + o * kH + j], h1[j], acc);
    h2[o] = fmaxf(acc, 0.f);
    __syncthreads();
    if (o < kOut) {
        float y = P[L.b3 + o];
        for (int j = 0; j < kH; ++j) y = fmaf(P[L.w3 + o * kH + j], h2[j], y);
        Y[(int64_t)b * kOut + o] = y;
    }
    if (act) {
        act[(int64_t)b * 2 * kH + o] = h1[o];
        act[(int64_t)b * 2 * kH + kH + o] = h2[o];
    }
}

// Loss L = 1/(2B) sum_b sum_o (y - t)^2 and dL/dy = (y - t) / B.
__global__ __launch_bounds__(256) void k_mlp_loss(const float* __restrict__ Y,
                                                  const float* __restrict__ T, int B,
                                                  float* __restrict__ dY, float* __restrict__ loss) {
    __shared__ float part[256];
    float acc = 0.f;
    for (int i = threadIdx.x; i < B * kOut; i += blockDim.x) {
        const float e = Y[i] - T[i];
        dY[i] = e / (float)B;
        acc = fmaf(e, e, acc);
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) *loss = part[0] / (2.f * (float)B);
}

// Backward, step 1 (one workgroup of 64 per sample):
//   dh2 = (h2 > 0) * W3^T dy,  dh1 = (h1 > 0) * W2^T dh2   -> dact = [dh1, dh2]
__global__ __launch_bounds__(64) void k_mlp_bwd_act(const float* __restrict__ P, int D,
                                                    const float* __restrict__ act,
                                                    const float* __restrict__ dY, int B,
                                                    float* __restrict__ dact) {
    __shared__ float g2[kH];
    const int b = blockIdx.x, j = threadIdx.x;
    if (b >= B) return;
    const Layout L = layout(D);
    const float* a = act + (int64_t)b * 2 * kH;
    float s = 0.f;
    for (int o = 0; o < kOut; ++o) s = fmaf(P[L.w3 + o * kH + j], dY[(int64_t)b * kOut + o], s);
    const float d2 = a[kH + j] > 0.f ? s : 0.f;
    g2[j] = d2;
    __syncthreads();
    float t = 0.f;
    for (int o = 0; o < kH; ++o) t = fmaf(P[L.w2 + o * kH + j], g2[o], t);
    const float d1 = a[j] > 0.f ? t : 0.f;
    dact[(int64_t)b * 2 * kH + j] = d1;
    dact[(int64_t)b * 2 * kH + kH + j] = d2;
}

// Backward, step 2: one thread per parameter, summing over the batch in
// sample order.
__global__ __launch_bounds__(256) void k_mlp_bwd_w(int D, const float* __restrict__ X,
                                                   const float* __restrict__ mu,
                                                   const float* __restrict__ sd,
                                                   const float* __restrict__ act,
                                                   const float* __restrict__ dact,
                                                   const float* __restrict__ dY, int B,
                                                   float* __restrict__ G) {
    const Layout L = layout(D);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= L.total) return;
    float acc = 0.f;
    if (p < L.b1) {  // W1[o][i]
        const int o = (int)(p / D), i = (int)(p % D);
        for (int b = 0; b < B; ++b)
            acc = fmaf(dact[(int64_t)b * 2 * kH + o], norm_in(X + (int64_t)b * D, mu, sd, i), acc);
    } else if (p < L.w2) {  // b1[o]
        const int o = (int)(p - L.b1);
        for (int b = 0; b < B; ++b) acc += dact[(int64_t)b * 2 * kH + o];
    } else if (p < L.b2) {  // W2[o][j]
        const int o = (int)((p - L.w2) / kH), j = (int)((p - L.w2) % kH);
        for (int b = 0; b < B; ++b)
            acc = fmaf(dact[(int64_t)b * 2 * kH + kH + o], act[(int64_t)b * 2 * kH + j], acc);
    } else if (p < L.w3) {  // b2[o]
        const int o = (int)(p - L.b2);
        for (int b = 0; b < B; ++b) acc += dact[(int64_t)b * 2 * kH + kH + o];
    } else if (p < L.b3) {  // W3[o][j]
        const int o = (int)((p - L.w3) / kH), j = (int)((p - L.w3) % kH);
        for (int b = 0; b < B; ++b)
            acc = fmaf(dY[(int64_t)b * kOut + o], act[(int64_t)b * 2 * kH + kH + j], acc);
    } else {  // b3[o]
        const int o = (int)(p - L.b3);
        for (int b = 0; b < B; ++b) acc += dY[(int64_t)b * kOut + o];
    }
    G[p] = acc;
}

// Adam (Kingma and Ba, 2015) with bias correction; t is the 1-based step.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ P, float* __restrict__ M,
                                              float* __restrict__ V, const float* __restrict__ G,
                                              int64_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = G[i];
    const float m = b1 * M[i] + (1.f - b1) * g;
    const float v = b2 * V[i] + (1.f - b2) * g * g;
    M[i] = m;
    V[i] = v;
    const float mh = m / c1, vh = v / c2;
    P[i] = P[i] - lr * mh / (sqrtf(vh) + eps);
}

}  // namespace

int64_t mlp_params(int D) { return layout(D).total; }

hipError_t mlp_forward(const float* P, int D, const float* X, const float* mu, const float* sd,
                       int B, float* Y, float* act, hipStream_t s, float* h1_scratch) {
    if (B <= 0) return hipSuccess;
    if (h1_scratch && B <= kSmallBatch) {
        hipLaunchKernelGGL(k_mlp_fwd_l1, dim3(kH, (unsigned)B), dim3(256), 0, s, P, D, X, mu, sd,
                           h1_scratch);
        hipLaunchKernelGGL(k_mlp_fwd_l23, dim3((unsigned)B), dim3(kH), 0, s, P, D, h1_scratch, B, Y,
                           act);
    } else {
        hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)B), dim3(256), 0, s, P, D, X, mu, sd, B, Y, act);
    }
    return hipGetLastError();
}

}  // namespace sj

using namespace sj;

extern "C" {

int64_t sj_mlp_param_count(int32_t d_in) {
    if (d_in < 1 || d_in > kMaxD) return -1;
    return layout(d_in).total;
}

sj_status sj_mlp_forward(const float* params, int32_t d_in, const float* mu, const float* sd,
                         const float* X, int32_t batch, float* Y, float* act, void* stream) {
    if (d_in < 1 || d_in > kMaxD || batch < 0 || (batch > 0 && (!params || !X || !Y)))
        return SJ_ERR_ARG;
    return mlp_forward(params, d_in, X, mu, sd, batch, Y, act, (hipStream_t)stream, nullptr) ==
                   hipSuccess
               ? SJ_OK
               : SJ_ERR_DEVICE;
}

sj_status sj_mlp_loss(const float* Y, const float* T, int32_t batch, float* dY, float* loss,
                      void* stream) {
    if (batch < 1 || !Y || !T || !dY) return SJ_ERR_ARG;
    hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, (hipStream_t)stream, Y, T, batch, dY,
                       loss);
    return hipGetLastError() == hipSuccess ? SJ_OK : SJ_ERR_DEVICE;
}

sj_status sj_mlp_backward(const float* params, int32_t d_in, const float* mu, const float* sd,
                          const float* X, int32_t batch, const float* act, const float* dY,
                          float* dact, float* grad, void* stream) {
    if (d_in < 1 || d_in > kMaxD || batch < 1 || !params || !X || !act || !dY || !dact || !grad)
        return SJ_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_bwd_act, dim3((unsigned)batch), dim3(64), 0, s, params, d_in, act, dY,
                       batch, dact);
    const int64_t n = layout(d_in).total;
    hipLaunchKernelGGL(k_mlp_bwd_w, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d_in, X,
                       mu, sd, act, dact, dY, batch, grad);
    return hipGetLastError() == hipSuccess ? SJ_OK : SJ_ERR_DEVICE;
}

sj_status sj_mlp_adam(float* params, float* m, float* v, const float* grad, int64_t n, float lr,
                      float beta1, float beta2, float eps, int32_t step, void* stream) {
    if (n < 0 || step < 1 || (n > 0 && (!params || !m || !v || !grad))) return SJ_ERR_ARG;
    if (n == 0) return SJ_OK;
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       params, m, v, grad, n, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? SJ_OK : SJ_ERR_DEVICE;
}

}  // extern "C"
