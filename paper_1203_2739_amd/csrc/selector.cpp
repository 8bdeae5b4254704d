// Learned choice of the product form: matrix features (host) and the C
// interface of the selector network's kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "api_internal.h"
#include "mlp.h"

using namespace spx;

namespace {

int degree_bin(int64_t d) {
    if (d <= 0) return 0;
    int b = 64 - __builtin_clzll((unsigned long long)d);  // floor(log2 d) + 1
    return b < 15 ? b : 15;
}

// Workspace of the network kernels, kept per thread and grown on demand.
float *mlp_ws(int B) {
    thread_local DevPtr ws;
    size_t need = mlp_workspace_floats(B) * sizeof(float);
    if (!ws || ws->bytes < need) ws = dev_alloc(need);
    return (float *)ws->ptr;
}

}  // namespace

extern "C" {

spx_status spx_features(spx_mat A, float *out) {
    return guarded([&] {
        if (!A || !out) fail(SPX_EINVAL, "NULL argument");
        const CsrHost &h = A->h;
        const int64_t m = h.m, n = h.n, nnz = h.nnz;
        double f[SPX_NFEATURES] = {0.0};
        f[0] = std::log1p((double)n);
        f[1] = std::log1p((double)nnz);
        std::vector<int64_t> cdeg((size_t)n, 0);
        for (int64_t q = 0; q < nnz; ++q) cdeg[h.colidx[q]]++;
        std::vector<int64_t> rh(16, 0), ch(16, 0);
        double dsum = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            const int64_t d = (int64_t)h.rowptr[i + 1] - h.rowptr[i];
            rh[degree_bin(d)]++;
            dsum += (double)d;
        }
        for (int64_t j = 0; j < n; ++j) ch[degree_bin(cdeg[j])]++;
        for (int b = 0; b < 16; ++b) {
            if (m) f[2 + b] = (double)rh[b] / (double)m;
            if (n) f[18 + b] = (double)ch[b] / (double)n;
        }
        if (nnz) {
            double usum = 0.0, umax = 0.0, span = 0.0;
            int64_t near = 0, diag = 0, nonempty = 0;
            for (int64_t i = 0; i < m; ++i) {
                const int64_t a0 = h.rowptr[i], a1 = h.rowptr[i + 1];
                if (a1 > a0) {
                    span += (double)(h.colidx[a1 - 1] - h.colidx[a0]) / (double)n;
                    ++nonempty;
                }
                for (int64_t q = a0; q < a1; ++q) {
                    const int64_t j = h.colidx[q];
                    const double u = std::fabs((double)i / (double)m - (double)j / (double)n);
                    usum += u;
                    umax = std::max(umax, u);
                    near += u <= 1.0 / 64.0;
                    diag += (8 * i) / m == (8 * j) / n;
                }
            }
            f[34] = usum / (double)nnz;
            f[35] = umax;
            f[36] = (double)near / (double)nnz;
            f[37] = (double)diag / (double)nnz;
            f[38] = span / (double)nonempty;
        }
        if (m && dsum > 0) {
            const double mean = dsum / (double)m;
            double var = 0.0;
            for (int64_t i = 0; i < m; ++i) {
                const double d = (double)((int64_t)h.rowptr[i + 1] - h.rowptr[i]) - mean;
                var += d * d;
            }
            f[39] = std::sqrt(var / (double)m) / mean;
        }
        for (int t = 0; t < SPX_NFEATURES; ++t) out[t] = (float)f[t];
    });
}

spx_status spx_mlp_forward(const float *theta, const float *X, int32_t B, float *logits, void *stream) {
    return guarded([&] {
        if (B < 1 || !theta || !X || !logits) fail(SPX_EINVAL, "bad arguments");
        hip_check(mlp_forward(theta, X, B, logits, mlp_ws(B), (hipStream_t)stream), "mlp forward");
    });
}

spx_status spx_mlp_loss_grad(const float *theta, const float *X, const int32_t *labels, int32_t B, float *loss,
                             float *grad, void *stream) {
    return guarded([&] {
        if (B < 1 || !theta || !X || !labels || !loss || !grad) fail(SPX_EINVAL, "bad arguments");
        hip_check(mlp_loss_grad(theta, X, labels, B, loss, grad, mlp_ws(B), (hipStream_t)stream), "mlp backward");
    });
}

spx_status spx_mlp_adam(float *theta, const float *grad, float *m, float *v, int32_t t, float lr, float beta1,
                        float beta2, float eps, void *stream) {
    return guarded([&] {
        if (t < 1 || !theta || !grad || !m || !v) fail(SPX_EINVAL, "bad arguments");
        hip_check(mlp_adam(theta, grad, m, v, t, lr, beta1, beta2, eps, (hipStream_t)stream), "adam");
    });
}

}  // extern "C"
