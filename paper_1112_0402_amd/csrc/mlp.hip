// Small multilayer perceptron for the kernel selector: x -> relu(x W1 + b1) -> relu(. W2 + b2)
// -> . W3 + b3, FP32, trained on the GPU with these forward, backward, loss and Adam kernels.
// The network is tiny (a few inputs, 64-wide hidden layers, one output per candidate
// launch), so every kernel is one thread per output value with a short inner loop.
//
// Parameter block (one flat FP32 array): W1 [in][h], b1 [h], W2 [h][h], b2 [h], W3 [h][out],
// b3 [out].  Activation workspace: H1 [batch][h], H2 [batch][h] (after ReLU).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mlp.h"

namespace ffc {

namespace {

// Y[b][o] = act(sum_i X[b][i] W[i][o] + bias[o])
__global__ void linear_fwd(int64_t batch, int n_in, int n_out, const float* __restrict__ X, const float* __restrict__ W,
                           const float* __restrict__ bias, float* __restrict__ Y, int relu) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= batch * n_out) return;
    const int64_t b = idx / n_out;
    const int o = static_cast<int>(idx - b * n_out);
    float s = bias[o];
    for (int i = 0; i < n_in; ++i) s += X[b * n_in + i] * W[static_cast<int64_t>(i) * n_out + o];
    Y[idx] = (relu && s < 0.f) ? 0.f : s;
}

// dW[i][o] = sum_b X[b][i] dY[b][o];  db[o] = sum_b dY[b][o]   (one thread per (i, o) and o)
__global__ void linear_bwd_w(int64_t batch, int n_in, int n_out, const float* __restrict__ X,
                             const float* __restrict__ dY, float* __restrict__ dW, float* __restrict__ db) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n_in * n_out) {
        const int i = idx / n_out, o = idx - (idx / n_out) * n_out;
        float s = 0.f;
        for (int64_t b = 0; b < batch; ++b) s += X[b * n_in + i] * dY[b * n_out + o];
        dW[idx] = s;
    } else if (idx < n_in * n_out + n_out) {
        const int o = idx - n_in * n_out;
        float s = 0.f;
        for (int64_t b = 0; b < batch; ++b) s += dY[b * n_out + o];
        db[o] = s;
    }
}

// dX[b][i] = (sum_o dY[b][o] W[i][o]) * (X[b][i] > 0 if relu_of_x)   (X = the layer's input)
__global__ void linear_bwd_x(int64_t batch, int n_in, int n_out, const float* __restrict__ dY,
                             const float* __restrict__ W, const float* __restrict__ X, float* __restrict__ dX,
                             int relu_of_x) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= batch * n_in) return;
    const int64_t b = idx / n_in;
    const int i = static_cast<int>(idx - b * n_in);
    float s = 0.f;
    for (int o = 0; o < n_out; ++o) s += dY[b * n_out + o] * W[static_cast<int64_t>(i) * n_out + o];
    if (relu_of_x && !(X[idx] > 0.f)) s = 0.f;
    dX[idx] = s;
}

// masked mean squared error: loss = sum m (y - t)^2 / sum m, dY = 2 m (y - t) / sum m.
// One workgroup; the mask count is reduced first.
__global__ void mse_kernel(int64_t n, const float* __restrict__ Y, const float* __restrict__ T,
                           const float* __restrict__ M, float* __restrict__ dY, float* __restrict__ loss) {
    __shared__ float red[256];
    __shared__ float cnt_s;
    float c = 0.f;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) c += M[i];
    red[threadIdx.x] = c;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt_s = red[0] > 0.f ? red[0] : 1.f;
    __syncthreads();
    const float inv = 1.f / cnt_s;
    float l = 0.f;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const float d = (Y[i] - T[i]) * M[i];
        dY[i] = 2.f * d * inv;
        l += d * d;
    }
    __syncthreads();
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] * inv;
}

__global__ void adam_kernel(int64_t n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float wd, float c1,
                            float c2) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i] + wd * p[i];  // L2 term
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

unsigned blocks(int64_t n) { return static_cast<unsigned>((n + 255) / 256); }

struct Offsets {
    int64_t w1, b1, w2, b2, w3, b3, total;
};

Offsets offsets(int in, int h, int out) {
    Offsets o{};
    o.w1 = 0;
    o.b1 = o.w1 + static_cast<int64_t>(in) * h;
    o.w2 = o.b1 + h;
    o.b2 = o.w2 + static_cast<int64_t>(h) * h;
    o.w3 = o.b2 + h;
    o.b3 = o.w3 + static_cast<int64_t>(h) * out;
    o.total = o.b3 + out;
    return o;
}

}  // namespace

int64_t mlp_param_count(int in, int h, int out) { return offsets(in, h, out).total; }

hipError_t mlp_forward(int in, int h, int out, int64_t batch, const float* params, const float* x, float* act,
                       float* y, hipStream_t s) {
    const Offsets o = offsets(in, h, out);
    float* h1 = act;
    float* h2 = act + batch * h;
    linear_fwd<<<blocks(batch * h), 256, 0, s>>>(batch, in, h, x, params + o.w1, params + o.b1, h1, 1);
    linear_fwd<<<blocks(batch * h), 256, 0, s>>>(batch, h, h, h1, params + o.w2, params + o.b2, h2, 1);
    linear_fwd<<<blocks(batch * out), 256, 0, s>>>(batch, h, out, h2, params + o.w3, params + o.b3, y, 0);
    return hipGetLastError();
}

hipError_t mlp_backward(int in, int h, int out, int64_t batch, const float* params, const float* x, const float* act,
                        const float* dy, float* grad, float* work, hipStream_t s) {
    const Offsets o = offsets(in, h, out);
    const float* h1 = act;
    const float* h2 = act + batch * h;
    float* d2 = work;              // dL/d(pre-activation of layer 2 output) via relu mask
    float* d1 = work + batch * h;  // the same for layer 1
    linear_bwd_w<<<blocks(static_cast<int64_t>(h) * out + out), 256, 0, s>>>(batch, h, out, h2, dy, grad + o.w3,
                                                                               grad + o.b3);
    linear_bwd_x<<<blocks(batch * h), 256, 0, s>>>(batch, h, out, dy, params + o.w3, h2, d2, 1);
    linear_bwd_w<<<blocks(static_cast<int64_t>(h) * h + h), 256, 0, s>>>(batch, h, h, h1, d2, grad + o.w2, grad + o.b2);
    linear_bwd_x<<<blocks(batch * h), 256, 0, s>>>(batch, h, h, d2, params + o.w2, h1, d1, 1);
    linear_bwd_w<<<blocks(static_cast<int64_t>(in) * h + h), 256, 0, s>>>(batch, in, h, x, d1, grad + o.w1, grad + o.b1);
    return hipGetLastError();
}

hipError_t mlp_mse(int64_t n, const float* y, const float* t, const float* m, float* dy, float* loss, hipStream_t s) {
    mse_kernel<<<1, 256, 0, s>>>(n, y, t, m, dy, loss);
    return hipGetLastError();
}

hipError_t adam_step(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                     float wd, int step, hipStream_t s) {
    const float c1 = 1.f - powf(b1, static_cast<float>(step));
    const float c2 = 1.f - powf(b2, static_cast<float>(step));
    adam_kernel<<<blocks(n), 256, 0, s>>>(n, p, g, m, v, lr, b1, b2, eps, wd, c1, c2);
    return hipGetLastError();
}

}  // namespace ffc
