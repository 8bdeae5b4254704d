// Learned choice of the product form: matrix features (host), the C
// interface of the selector network's kernels, the 24 choices, selection by
// the network and the exhaustive timing that is its fallback and yardstick.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <memory>
#include <string>
#include <vector>

#include "api_internal.h"
#include "kernels.h"
#include "mlp.h"

using namespace spx;

namespace {

// The 24 choices: six schedules of plain CSR, then SB, DB and the split at
// K = 8, 16, 32, 64, 128, 256 (default schedule).
constexpr int kChoiceKs[6] = {8, 16, 32, 64, 128, 256};

struct Choice {
    int form, K;
    spx_tune tune;
};

Choice choice_of(int c) {
    if (c < 0 || c >= SPX_NCHOICES) fail(SPX_EINVAL, "choice out of range 0..23");
    Choice ch{SPX_FORM_PLAIN, 1, spx_tune{}};
    if (c < 6) {
        static const int wg[6] = {128, 64, 256, 128, 128, 512};
        static const int npt[6] = {4, 8, 4, 8, 4, 4};
        ch.tune.wg_size = wg[c];
        ch.tune.nnz_per_block = wg[c] * npt[c];
        if (c == 4) ch.tune.reduce_iters = 16;
        return ch;
    }
    static const int forms[3] = {SPX_FORM_SB, SPX_FORM_DB, SPX_FORM_SPLIT};
    ch.form = forms[(c - 6) / 6];
    ch.K = kChoiceKs[(c - 6) % 6];
    return ch;
}

Model model_of(int form) {
    return form == SPX_FORM_SB ? Model::ColumnNet : form == SPX_FORM_DB ? Model::ERowColumnNet : Model::RowColumnNet;
}

// The K-way partition that a K = 256 recursive bisection yields at depth
// log2 K: part p of the 256 tree lies in part p >> (8 - log2 K); the DB row
// border stays the border.  Leaves are the parts.
PartitionResult coarsen(const PartitionResult &tree, int form, int K) {
    int shift = 0;
    while ((256 >> shift) > K) ++shift;
    PartitionResult r;
    r.part.resize(tree.part.size());
    for (size_t i = 0; i < tree.part.size(); ++i) {
        const int32_t p = tree.part[i];
        r.part[i] = (form == SPX_FORM_DB && p >= 256) ? K : (p >> shift);
    }
    r.leaf.resize(r.part.size());
    for (size_t i = 0; i < r.part.size(); ++i) r.leaf[i] = r.part[i] < K ? r.part[i] : 0;
    r.nleaves = K;
    r.seconds = tree.seconds;
    return r;
}

spx_plan_s *plan_of_choice(spx_mat_s &A, const Choice &ch, const PartitionResult *tree) {
    if (ch.form == SPX_FORM_PLAIN) {
        std::unique_ptr<spx_plan_s> P(new spx_plan_s());
        plan_plain(*P, A.h);
        P->tune = resolve_tune(&ch.tune, P->form);
        build_schedule(*P);
        upload_plan(*P, A, nullptr);
        return P.release();
    }
    return plan_from_partition(A, ch.form, ch.K, coarsen(*tree, ch.form, ch.K), nullptr);
}

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    Events() {
        hip_check(hipEventCreate(&a), "event");
        hip_check(hipEventCreate(&b), "event");
    }
    ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

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

void check_exhaustive_args(spx_mat A, const double *x, const double *y, int32_t reps, const int32_t *choice) {
    if (!A || !choice) fail(SPX_EINVAL, "NULL argument");
    if (!A->on_device) fail(SPX_ENODEVICE, "matrix has no device copy");
    if (reps < 1) fail(SPX_EINVAL, "reps must be >= 1");
    if (A->h.m > 0 && !y) fail(SPX_EINVAL, "y is NULL");
    if (A->h.nnz > 0 && !x) fail(SPX_EINVAL, "x is NULL");
}

// Every choice built (the reordered ones cut from the tree of their form)
// and timed over `reps` products after two warm-up products.
void time_choices(spx_mat_s &A, const PartitionResult trees[3], const double *x, double *y, int32_t reps, float *ms,
                  int32_t *choice, hipStream_t s) {
    DevPtr xh = dev_alloc((size_t)std::max<int32_t>(A.h.n, 1) * sizeof(double));
    Events ev;
    float t[SPX_NCHOICES];
    for (int c = 0; c < SPX_NCHOICES; ++c) {
        const Choice ch = choice_of(c);
        std::unique_ptr<spx_plan_s> P(plan_of_choice(A, ch, ch.form == SPX_FORM_PLAIN ? nullptr : &trees[ch.form - 1]));
        const double *xp = x;
        if (ch.form != SPX_FORM_PLAIN) {
            hip_check(launch_gather(x, (const int32_t *)P->d_col_perm->ptr, (double *)xh->ptr, P->n, s), "permute x");
            xp = (const double *)xh->ptr;
        }
        for (int w = 0; w < 2; ++w) hip_check(run_product(*P, xp, y, 0, s), "product");
        hip_check(hipEventRecord(ev.a, s), "event record");
        for (int r = 0; r < reps; ++r) hip_check(run_product(*P, xp, y, 0, s), "product");
        hip_check(hipEventRecord(ev.b, s), "event record");
        hip_check(hipEventSynchronize(ev.b), "event sync");
        hip_check(hipEventElapsedTime(&t[c], ev.a, ev.b), "elapsed");
        t[c] /= (float)reps;
    }
    int best = 0;
    for (int c = 1; c < SPX_NCHOICES; ++c)
        if (t[c] < t[best]) best = c;
    *choice = best;
    if (ms) std::copy(t, t + SPX_NCHOICES, ms);
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

spx_status spx_mlp_loss_grad_noalloc(const float *theta, const float *X, const int32_t *labels, int32_t B,
                                     float *loss, float *grad, void *stream) {
    return guarded([&] {
        if (!theta || !X || !labels || !loss || !grad) fail(SPX_EINVAL, "bad arguments");
        if (B < 1 || B > mlp_noalloc_max_batch())
            fail(SPX_EINVAL, "B must be in 1.." + std::to_string(mlp_noalloc_max_batch()) +
                                 " (the fixed workspace of the no-allocation entry point)");
        float *ws = nullptr;
        hip_check(mlp_noalloc_scratch(&ws), "no-allocation workspace address");
        hip_check(mlp_loss_grad(theta, X, labels, B, loss, grad, ws, (hipStream_t)stream), "mlp backward");
    });
}

spx_status spx_mlp_adam(float *theta, const float *grad, float *m, float *v, int32_t t, float lr, float beta1,
                        float beta2, float eps, void *stream) {
    return guarded([&] {
        if (t < 1 || !theta || !grad || !m || !v) fail(SPX_EINVAL, "bad arguments");
        hip_check(mlp_adam(theta, grad, m, v, t, lr, beta1, beta2, eps, (hipStream_t)stream), "adam");
    });
}

spx_status spx_choice_info(int32_t choice, int32_t *form, int32_t *K, spx_tune *tune) {
    return guarded([&] {
        const Choice ch = choice_of(choice);
        if (form) *form = ch.form;
        if (K) *K = ch.K;
        if (tune) *tune = ch.tune;
    });
}

spx_status spx_select_features(const float *f, const float *theta, const double *mu, const double *sd,
                               int32_t *choice, float *logits_out, void *stream) {
    return guarded([&] {
        if (!f || !theta || !mu || !sd || !choice) fail(SPX_EINVAL, "NULL argument");
        float z[SPX_NFEATURES];
        for (int t = 0; t < SPX_NFEATURES; ++t) {
            const double g = std::log1p(std::max((double)f[t], 0.0));
            z[t] = (float)((g - mu[t]) / sd[t]);
        }
        thread_local DevPtr buf;
        const size_t need = (SPX_NFEATURES + SPX_NCHOICES) * sizeof(float);
        if (!buf || buf->bytes < need) buf = dev_alloc(need);
        float *dz = (float *)buf->ptr, *dl = dz + SPX_NFEATURES;
        hipStream_t s = (hipStream_t)stream;
        hip_check(hipMemcpyAsync(dz, z, sizeof(z), hipMemcpyHostToDevice, s), "features upload");
        hip_check(mlp_forward(theta, dz, 1, dl, mlp_ws(1), s), "mlp forward");
        float lg[SPX_NCHOICES];
        hip_check(hipMemcpyAsync(lg, dl, sizeof(lg), hipMemcpyDeviceToHost, s), "logits download");
        hip_check(hipStreamSynchronize(s), "select");
        int best = 0;
        for (int c = 1; c < SPX_NCHOICES; ++c)
            if (lg[c] > lg[best]) best = c;
        *choice = best;
        if (logits_out) std::copy(lg, lg + SPX_NCHOICES, logits_out);
    });
}

spx_status spx_select(spx_mat A, const float *theta, const double *mu, const double *sd, int32_t *choice,
                      float *logits_out, void *stream) {
    return guarded([&] {
        if (!A) fail(SPX_EINVAL, "NULL handle");
        float f[SPX_NFEATURES];
        spx_status st = spx_features(A, f);
        if (st != SPX_OK) fail(st, "features");
        st = spx_select_features(f, theta, mu, sd, choice, logits_out, stream);
        if (st != SPX_OK) fail(st, "select");
    });
}

spx_status spx_plan_for_choice(spx_mat A, int32_t choice, uint64_t seed, int32_t *row_perm, int32_t *col_perm,
                               spx_plan *out) {
    return guarded([&] {
        if (!A || !out) fail(SPX_EINVAL, "NULL handle");
        *out = nullptr;
        const Choice ch = choice_of(choice);
        std::unique_ptr<spx_plan_s> P;
        if (ch.form == SPX_FORM_PLAIN) {
            P.reset(plan_of_choice(*A, ch, nullptr));
        } else {
            PartitionResult tree = partition(A->h, model_of(ch.form), 256, 0, seed);
            P.reset(plan_of_choice(*A, ch, &tree));
        }
        if (row_perm) {
            if (P->row_perm.empty()) for (int32_t i = 0; i < P->m; ++i) row_perm[i] = i;
            else std::copy(P->row_perm.begin(), P->row_perm.end(), row_perm);
        }
        if (col_perm) {
            if (P->col_perm.empty()) for (int32_t j = 0; j < P->n; ++j) col_perm[j] = j;
            else std::copy(P->col_perm.begin(), P->col_perm.end(), col_perm);
        }
        *out = P.release();
    });
}

spx_status spx_select_exhaustive(spx_mat A, const double *x, double *y, int32_t reps, uint64_t seed, float *ms,
                                 int32_t *choice, double *partition_seconds, void *stream) {
    return guarded([&] {
        check_exhaustive_args(A, x, y, reps, choice);
        auto t0 = std::chrono::steady_clock::now();
        PartitionResult trees[3];
        for (int f = 0; f < 3; ++f)
            trees[f] = partition(A->h, model_of(f + 1), 256, 0, seed);
        const double tpart = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        time_choices(*A, trees, x, y, reps, ms, choice, (hipStream_t)stream);
        if (partition_seconds) *partition_seconds = tpart;
    });
}

spx_status spx_partition_tree(spx_mat A, int32_t form, uint64_t seed, int32_t *parts, double *seconds) {
    return guarded([&] {
        if (!A) fail(SPX_EINVAL, "NULL handle");
        if (form != SPX_FORM_SB && form != SPX_FORM_DB && form != SPX_FORM_SPLIT)
            fail(SPX_EINVAL, "form must be SPX_FORM_SB, SPX_FORM_DB or SPX_FORM_SPLIT");
        const size_t len = form == SPX_FORM_SPLIT ? (size_t)A->h.nnz : (size_t)A->h.m;
        if (len && !parts) fail(SPX_EINVAL, "parts is NULL");
        auto t0 = std::chrono::steady_clock::now();
        const PartitionResult tree = partition(A->h, model_of(form), 256, 0, seed);
        std::copy(tree.part.begin(), tree.part.begin() + std::min(len, tree.part.size()), parts);
        if (seconds) *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    });
}

spx_status spx_select_exhaustive_trees(spx_mat A, const int32_t *tree_sb, const int32_t *tree_db,
                                       const int32_t *tree_split, const double *x, double *y, int32_t reps,
                                       float *ms, int32_t *choice, void *stream) {
    return guarded([&] {
        check_exhaustive_args(A, x, y, reps, choice);
        const int32_t *given[3] = {tree_sb, tree_db, tree_split};
        PartitionResult trees[3];
        for (int f = 0; f < 3; ++f) {
            const size_t len = f == 2 ? (size_t)A->h.nnz : (size_t)A->h.m;
            const int32_t hi = f == 1 ? 256 : 255;  // DB: 256 is the row border
            if (len && !given[f]) fail(SPX_EINVAL, "tree is NULL");
            if (len) trees[f].part.assign(given[f], given[f] + len);
            for (int32_t p : trees[f].part)
                if (p < 0 || p > hi) fail(SPX_EINVAL, "tree part out of range");
        }
        time_choices(*A, trees, x, y, reps, ms, choice, (hipStream_t)stream);
    });
}

}  // extern "C"
