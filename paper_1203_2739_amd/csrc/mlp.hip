// Selector network kernels (binary32): a 40 -> 64 -> 64 -> 24 perceptron
// with ReLU hidden layers and softmax cross-entropy, forward and backward,
// and the Adam update.  The layers are a few thousand multiply-adds per
// sample, so every output element is one thread's dot product; sums run in
// a fixed order, so results are reproducible.
#include <hip/hip_runtime.h>

#include <mutex>

#include <cstdint>

#include "mlp.h"

namespace spx {

namespace {

constexpr int kWG = 256;

inline unsigned groups(int64_t n) { return (unsigned)((n + kWG - 1) / kWG); }

// out[b, o] = b_o + sum_k in[b, k] W[o, k]; act = ReLU(out) when relu
__global__ void dense_fwd_kernel(const float *__restrict__ in, int K, const float *__restrict__ W,
                                 const float *__restrict__ bias, int N, int B, float *__restrict__ pre,
                                 float *__restrict__ act, int relu) {
    const int64_t idx = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (idx >= (int64_t)B * N) return;
    const int bi = (int)(idx / N), o = (int)(idx - (int64_t)bi * N);
    float s = bias[o];
    for (int k = 0; k < K; ++k) s += in[(int64_t)bi * K + k] * W[o * K + k];
    pre[idx] = s;
    if (act) act[idx] = relu ? fmaxf(s, 0.0f) : s;
}

// softmax cross-entropy of the labels: d = (softmax - onehot) / B and the
// mean loss; one workgroup, samples strided over threads
__global__ __launch_bounds__(kWG) void softmax_ce_kernel(const float *__restrict__ z, const int32_t *__restrict__ labels,
                                                         int B, int C, float *__restrict__ d, float *__restrict__ loss) {
    __shared__ float part[kWG];
    float acc = 0.0f;
    for (int bi = threadIdx.x; bi < B; bi += kWG) {
        const float *zr = z + (int64_t)bi * C;
        float mx = zr[0];
        for (int c = 1; c < C; ++c) mx = fmaxf(mx, zr[c]);
        float se = 0.0f;
        for (int c = 0; c < C; ++c) se += expf(zr[c] - mx);
        const int y = labels[bi];
        // a label outside 0..C-1 reads nothing: its loss and gradient are NaN
        const bool ok = y >= 0 && y < C;
        acc += ok ? logf(se) - (zr[y] - mx) : __builtin_nanf("");
        for (int c = 0; c < C; ++c)
            d[(int64_t)bi * C + c] =
                ok ? (expf(zr[c] - mx) / se - (c == y ? 1.0f : 0.0f)) / (float)B : __builtin_nanf("");
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int t = 0; t < kWG; ++t) s += part[t];
        *loss = s / (float)B;
    }
}

// gW[o, k] = sum_b d[b, o] act[b, k]; gb[o] = sum_b d[b, o]
__global__ void dense_bwd_w_kernel(const float *__restrict__ d, int N, const float *__restrict__ act, int K, int B,
                                   float *__restrict__ gW, float *__restrict__ gb) {
    const int64_t idx = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (idx < (int64_t)N * K) {
        const int o = (int)(idx / K), k = (int)(idx - (int64_t)o * K);
        float s = 0.0f;
        for (int bi = 0; bi < B; ++bi) s += d[(int64_t)bi * N + o] * act[(int64_t)bi * K + k];
        gW[idx] = s;
    } else if (idx < (int64_t)N * K + N) {
        const int o = (int)(idx - (int64_t)N * K);
        float s = 0.0f;
        for (int bi = 0; bi < B; ++bi) s += d[(int64_t)bi * N + o];
        gb[o] = s;
    }
}

// dprev[b, k] = (sum_o d[b, o] W[o, k]) * (pre[b, k] > 0)
__global__ void dense_bwd_x_kernel(const float *__restrict__ d, int N, const float *__restrict__ W, int K,
                                   const float *__restrict__ pre, int B, float *__restrict__ dprev) {
    const int64_t idx = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (idx >= (int64_t)B * K) return;
    const int bi = (int)(idx / K), k = (int)(idx - (int64_t)bi * K);
    float s = 0.0f;
    for (int o = 0; o < N; ++o) s += d[(int64_t)bi * N + o] * W[o * K + k];
    dprev[idx] = pre[idx] > 0.0f ? s : 0.0f;
}

__global__ void adam_kernel(float *__restrict__ theta, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * kWG + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

// Parameter blocks inside the flat vector, in the order W1, b1, W2, b2, W3, b3.
struct Layout {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
};
static Layout layout(const float *t) {
    Layout L;
    L.W1 = t;
    L.b1 = L.W1 + kMlpHid * kMlpIn;
    L.W2 = L.b1 + kMlpHid;
    L.b2 = L.W2 + kMlpHid * kMlpHid;
    L.W3 = L.b2 + kMlpHid;
    L.b3 = L.W3 + kMlpOut * kMlpHid;
    return L;
}

size_t mlp_workspace_floats(int B) { return (size_t)B * (6 * kMlpHid + 2 * kMlpOut) + 64; }

hipError_t mlp_forward(const float *theta, const float *X, int B, float *logits, float *ws, hipStream_t s) {
    const Layout L = layout(theta);
    float *z1 = ws, *h1 = z1 + (size_t)B * kMlpHid, *z2 = h1 + (size_t)B * kMlpHid, *h2 = z2 + (size_t)B * kMlpHid;
    hipLaunchKernelGGL(dense_fwd_kernel, dim3(groups((int64_t)B * kMlpHid)), dim3(kWG), 0, s, X, kMlpIn, L.W1, L.b1,
                       kMlpHid, B, z1, h1, 1);
    hipLaunchKernelGGL(dense_fwd_kernel, dim3(groups((int64_t)B * kMlpHid)), dim3(kWG), 0, s, h1, kMlpHid, L.W2, L.b2,
                       kMlpHid, B, z2, h2, 1);
    hipLaunchKernelGGL(dense_fwd_kernel, dim3(groups((int64_t)B * kMlpOut)), dim3(kWG), 0, s, h2, kMlpHid, L.W3, L.b3,
                       kMlpOut, B, logits, (float *)nullptr, 0);
    return hipGetLastError();
}

hipError_t mlp_loss_grad(const float *theta, const float *X, const int32_t *labels, int B, float *loss, float *grad,
                         float *ws, hipStream_t s) {
    const Layout L = layout(theta);
    float *z1 = ws, *h1 = z1 + (size_t)B * kMlpHid, *z2 = h1 + (size_t)B * kMlpHid, *h2 = z2 + (size_t)B * kMlpHid;
    float *z3 = h2 + (size_t)B * kMlpHid, *d3 = z3 + (size_t)B * kMlpOut, *d2 = d3 + (size_t)B * kMlpOut,
          *d1 = d2 + (size_t)B * kMlpHid;
    hipError_t e = mlp_forward(theta, X, B, z3, ws, s);
    if (e != hipSuccess) return e;
    float *gW1 = grad, *gb1 = gW1 + kMlpHid * kMlpIn, *gW2 = gb1 + kMlpHid, *gb2 = gW2 + kMlpHid * kMlpHid,
          *gW3 = gb2 + kMlpHid, *gb3 = gW3 + kMlpOut * kMlpHid;
    hipLaunchKernelGGL(softmax_ce_kernel, dim3(1), dim3(kWG), 0, s, z3, labels, B, kMlpOut, d3, loss);
    hipLaunchKernelGGL(dense_bwd_w_kernel, dim3(groups(kMlpOut * kMlpHid + kMlpOut)), dim3(kWG), 0, s, d3, kMlpOut, h2,
                       kMlpHid, B, gW3, gb3);
    hipLaunchKernelGGL(dense_bwd_x_kernel, dim3(groups((int64_t)B * kMlpHid)), dim3(kWG), 0, s, d3, kMlpOut, L.W3,
                       kMlpHid, z2, B, d2);
    hipLaunchKernelGGL(dense_bwd_w_kernel, dim3(groups(kMlpHid * kMlpHid + kMlpHid)), dim3(kWG), 0, s, d2, kMlpHid, h1,
                       kMlpHid, B, gW2, gb2);
    hipLaunchKernelGGL(dense_bwd_x_kernel, dim3(groups((int64_t)B * kMlpHid)), dim3(kWG), 0, s, d2, kMlpHid, L.W2,
                       kMlpHid, z1, B, d1);
    hipLaunchKernelGGL(dense_bwd_w_kernel, dim3(groups(kMlpHid * kMlpIn + kMlpHid)), dim3(kWG), 0, s, d1, kMlpHid, X,
                       kMlpIn, B, gW1, gb1);
    return hipGetLastError();
}

// ------------------------------------------------- no-allocation entry point
// Workspace of spx_mlp_loss_grad_noalloc: a file-scope device array sized
// for batches of up to kNoAllocMaxBatch samples.  Every GPU the library runs
// on holds its own copy until the process ends.  In host code the array's
// name is only a host-side stand-in: its device address on each GPU comes
// from hipGetSymbolAddress, taken once per device with that device current.
constexpr int kNoAllocMaxBatch = 512;
constexpr size_t kNoAllocFloats = (size_t)kNoAllocMaxBatch * (6 * kMlpHid + 2 * kMlpOut) + 64;
static __device__ __align__(256) float scratch[kNoAllocFloats];

static_assert(kNoAllocFloats >= (size_t)kNoAllocMaxBatch * (6 * kMlpHid + 2 * kMlpOut) + 64,
              "scratch must hold the workspace of the largest batch");

hipError_t mlp_noalloc_scratch(float **out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static float *ptr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[dev] = (float *)p;
    }
    *out = ptr[dev];
    return hipSuccess;
}

int mlp_noalloc_max_batch() { return kNoAllocMaxBatch; }

hipError_t mlp_adam(float *theta, const float *grad, float *m, float *v, int t, float lr, float b1, float b2,
                    float eps, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3(groups(kMlpParams)), dim3(kWG), 0, s, theta, grad, m, v, kMlpParams, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

}  // namespace spx
