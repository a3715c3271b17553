// Learned m-selector: a 32 -> 64 -> 64 -> 1 multilayer perceptron with ReLU
// hidden layers that maps sketch statistics of a data block to log(gamma), the
// compression factor the block needs to meet a target covariance error.  It is
// not part of the paper's method; the method itself generates its training
// labels.  Training runs in FP32 (forward, backward, Adam); inference reads
// BF16 weights and accumulates in FP32.
//
// Parameters, packed FP32: W1[64][32], b1[64], W2[64][64], b2[64], W3[64], b3.
// Inputs are standardized with fixed per-feature (mean, scale) first.
// Loss: expectile regression at level tau on r = target - prediction,
//   L = mean_b |tau - [r_b < 0]| r_b^2,
// which is smooth and, for tau > 1/2, penalizes predicting too small a gamma
// more than too large a one.
#include "pds_device.hpp"
#include "pds_internal.hpp"

namespace pds {

constexpr int kIn = 32, kH = 64;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH, oB3 = oW3 + kH;
constexpr int kParams = oB3 + 1;  // 6337

int mlp_param_count() { return kParams; }

// one thread per (sample, hidden unit): h[b][o] = relu(sum_k W[o][k] in[b][k] + bias[o]);
// four samples per workgroup, exchanged through LDS, stored for the backward pass
__global__ __launch_bounds__(256) void k_mlp_fwd(const float* __restrict__ P, const float* __restrict__ feats,
                                                 const float* __restrict__ mu, const float* __restrict__ sd, int B,
                                                 float* __restrict__ acts, float* __restrict__ out)
{
    __shared__ float xs[4][kIn], h1s[4][kH], h2s[4][kH];
    // every thread reaches every barrier; rows past B compute nothing
    const int w = threadIdx.x >> 6;
    const int b = blockIdx.x * 4 + w;
    const int o = threadIdx.x & 63;
    const bool live = b < B;
    if (live && o < kIn) xs[w][o] = (feats[(int64_t)b * kIn + o] - mu[o]) / sd[o];
    __syncthreads();
    float s = P[oB1 + o];
    for (int k = 0; k < kIn; ++k) s = fmaf(P[oW1 + o * kIn + k], xs[w][k], s);
    h1s[w][o] = s > 0.0f ? s : 0.0f;
    __syncthreads();
    s = P[oB2 + o];
    for (int k = 0; k < kH; ++k) s = fmaf(P[oW2 + o * kH + k], h1s[w][k], s);
    h2s[w][o] = s > 0.0f ? s : 0.0f;
    __syncthreads();
    if (!live) return;
    // acts per sample: xn[32], h1[64], h2[64]
    float* a = acts + (int64_t)b * (kIn + 2 * kH);
    if (o < kIn) a[o] = xs[w][o];
    a[kIn + o] = h1s[w][o];
    a[kIn + kH + o] = h2s[w][o];
    if (o == 0) {
        float y = P[oB3];
        for (int k = 0; k < kH; ++k) y = fmaf(P[oW3 + k], h2s[w][k], y);
        out[b] = y;
    }
}

// per-sample backward: dL/dy, then the hidden-layer error signals
__global__ __launch_bounds__(256) void k_mlp_bwd_signals(const float* __restrict__ P, const float* __restrict__ acts,
                                                         const float* __restrict__ pred,
                                                         const float* __restrict__ target, int B, float tau,
                                                         float* __restrict__ sig, float* __restrict__ lossb)
{
    __shared__ float g2s[4][kH];
    const int w = threadIdx.x >> 6;
    const int b = blockIdx.x * 4 + w;
    const int o = threadIdx.x & 63;
    const bool live = b < B;
    const int bb = live ? b : 0;
    const float* a = acts + (int64_t)bb * (kIn + 2 * kH);
    const float r = target[bb] - pred[bb];
    const float wt = (r < 0.0f) ? (1.0f - tau) : tau;
    const float gy = -2.0f * wt * r / (float)B;
    g2s[w][o] = (a[kIn + kH + o] > 0.0f) ? gy * P[oW3 + o] : 0.0f;
    __syncthreads();
    if (!live) return;
    // sig per sample: gy, g2[64], g1[64]
    float* g = sig + (int64_t)b * (1 + 2 * kH);
    if (o == 0) {
        g[0] = gy;
        lossb[b] = wt * r * r / (float)B;
    }
    g[1 + o] = g2s[w][o];
    float s = 0.0f;
    for (int k = 0; k < kH; ++k) s = fmaf(P[oW2 + k * kH + o], g2s[w][k], s);
    g[1 + kH + o] = (a[kIn + o] > 0.0f) ? s : 0.0f;
}

// parameter gradients: one thread per parameter, a fixed-order sum over the batch
__global__ __launch_bounds__(256) void k_mlp_bwd_params(const float* __restrict__ acts, const float* __restrict__ sig,
                                                        int B, float* __restrict__ grad)
{
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= kParams) return;
    float s = 0.0f;
    for (int b = 0; b < B; ++b) {
        const float* a = acts + (int64_t)b * (kIn + 2 * kH);
        const float* g = sig + (int64_t)b * (1 + 2 * kH);
        float t;
        if (q < oB1) {
            const int o = q / kIn, k = q % kIn;
            t = g[1 + kH + o] * a[k];
        } else if (q < oW2) {
            t = g[1 + kH + (q - oB1)];
        } else if (q < oB2) {
            const int o = (q - oW2) / kH, k = (q - oW2) % kH;
            t = g[1 + o] * a[kIn + k];
        } else if (q < oW3) {
            t = g[1 + (q - oB2)];
        } else if (q < oB3) {
            t = g[0] * a[kIn + kH + (q - oW3)];
        } else {
            t = g[0];
        }
        s += t;
    }
    grad[q] = s;
}

__global__ __launch_bounds__(256) void k_sum_f32(const float* __restrict__ x, int n, float* __restrict__ out)
{
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) s += x[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// P -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ P, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                                              float c1, float c2)
{
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.0f - b1) * gq;
    const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    P[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

__global__ __launch_bounds__(256) void k_pack_bf16(const float* __restrict__ P, int n, unsigned short* __restrict__ Pb)
{
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    __bf16 h = (__bf16)P[q];
    Pb[q] = __builtin_bit_cast(unsigned short, h);
}

__device__ inline float bf(const unsigned short* Pb, int q) { return __uint_as_float(((uint32_t)Pb[q]) << 16); }

// BF16 inference: gamma = clamp(exp(prediction), gmin, gmax); non-finite
// features or prediction give the fallback gamma.
__global__ __launch_bounds__(256) void k_mlp_predict_bf16(const unsigned short* __restrict__ Pb,
                                                          const float* __restrict__ feats, const float* __restrict__ mu,
                                                          const float* __restrict__ sd, int B, float gmin, float gmax,
                                                          float fallback, float* __restrict__ gamma)
{
    __shared__ unsigned short xn[4][kIn];
    __shared__ unsigned short h1[4][kH];
    __shared__ float h2[4][kH];
    __shared__ int bad[4];
    const int w = threadIdx.x >> 6;
    const int b = blockIdx.x * 4 + w;
    const int o = threadIdx.x & 63;
    const bool live = b < B;
    if (o == 0) bad[w] = 0;
    __syncthreads();
    if (live && o < kIn) {
        const float f = feats[(int64_t)b * kIn + o];
        if (!isfinite(f)) atomicOr(&bad[w], 1);
        __bf16 t = (__bf16)((f - mu[o]) / sd[o]);
        xn[w][o] = __builtin_bit_cast(unsigned short, t);
    }
    __syncthreads();
    float s = bf(Pb, oB1 + o);
    for (int k = 0; k < kIn; ++k) s = fmaf(bf(Pb, oW1 + o * kIn + k), __uint_as_float(((uint32_t)xn[w][k]) << 16), s);
    {
        __bf16 t = (__bf16)(s > 0.0f ? s : 0.0f);
        h1[w][o] = __builtin_bit_cast(unsigned short, t);
    }
    __syncthreads();
    s = bf(Pb, oB2 + o);
    for (int k = 0; k < kH; ++k) s = fmaf(bf(Pb, oW2 + o * kH + k), __uint_as_float(((uint32_t)h1[w][k]) << 16), s);
    h2[w][o] = s > 0.0f ? s : 0.0f;
    __syncthreads();
    if (live && o == 0) {
        float y = bf(Pb, oB3);
        for (int k = 0; k < kH; ++k) y = fmaf(bf(Pb, oW3 + k), h2[w][k], y);
        float g = expf(y);
        if (bad[w] || !isfinite(g)) g = fallback;
        gamma[b] = fminf(fmaxf(g, gmin), gmax);
    }
}

hipError_t launch_mlp_forward(const float* P, const float* feats, const float* mu, const float* sd, int B, float* acts,
                              float* out, hipStream_t s)
{
    ProfScope ps_("mlp_forward", s);
    hipLaunchKernelGGL(k_mlp_fwd, dim3((B + 3) / 4), dim3(256), 0, s, P, feats, mu, sd, B, acts, out);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const float* P, const float* acts, const float* pred, const float* target, int B,
                               float tau, float* sig, float* lossb, float* grad, float* loss, hipStream_t s)
{
    ProfScope ps_("mlp_backward", s);
    hipLaunchKernelGGL(k_mlp_bwd_signals, dim3((B + 3) / 4), dim3(256), 0, s, P, acts, pred, target, B, tau, sig,
                       lossb);
    hipLaunchKernelGGL(k_mlp_bwd_params, dim3((kParams + 255) / 256), dim3(256), 0, s, acts, sig, B, grad);
    hipLaunchKernelGGL(k_sum_f32, dim3(1), dim3(256), 0, s, lossb, B, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float* P, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s)
{
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    ProfScope ps_("adam", s);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, P, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_pack_bf16(const float* P, int n, unsigned short* Pb, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_bf16, dim3((n + 255) / 256), dim3(256), 0, s, P, n, Pb);
    return hipGetLastError();
}

hipError_t launch_mlp_predict_bf16(const unsigned short* Pb, const float* feats, const float* mu, const float* sd,
                                   int B, float gmin, float gmax, float fallback, float* gamma, hipStream_t s)
{
    ProfScope ps_("mlp_predict_bf16", s);
    hipLaunchKernelGGL(k_mlp_predict_bf16, dim3((B + 3) / 4), dim3(256), 0, s, Pb, feats, mu, sd, B, gmin, gmax,
                       fallback, gamma);
    return hipGetLastError();
}

}  // namespace pds
