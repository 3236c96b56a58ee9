// sp2_learned.hip -- the learned recursive expansion: a composition of trained
// quadratic maps of the matrix, X_{k+1} = a_k X_k^2 + b_k X_k + c_k I, in the
// form of a deep network whose layers are low-order polynomials of the
// previous layer (the recursive polynomial expansion of the paper's Section
// "GPU friendly algorithms").  One fixed map cannot place its step at a
// Fermi level that differs between Hamiltonians, so every layer is steered by
// the trace like SP2: the map itself when tr X > n_occ, its particle-hole form
// I - f(I - X) otherwise.  (a, b, c) = (1, 0, 0) is exactly SP2.
//
// Training (sp2_learned_fit) works on spectra: every layer is a polynomial of
// H, so the network's D is V diag(p(x_i)) V^T and its error against the
// projector is sum_i (p(x_i) - theta_i)^2 with theta_i = 1 for the n_occ
// lowest levels.  k_learned_grad runs the forward pass (with the trace
// decisions) and the backward pass through the recorded branches for one
// sample per workgroup; the host sums the per-sample gradients in sample
// order and takes an Adam step.  The loss is the mean over samples of
// log(mean squared eigenvalue error), so every sample's error is pushed down
// in proportion.  The coefficients are kept in FP32 (rounded after each
// step).
//
// Inference (sp2_learned_density) is the batched plan with the trained
// coefficients in the step kernel's epilogue, followed by an SP2 check step
// whose idempotency (and trace error) decides: accept; or, when the output is
// close to a projector, hand over to plain SP2 steps on the device (the layers
// then act as a faster gap-opening prefix); or solve again from H by plain SP2
// (sp2_density), reported as SP2_E_FALLBACK.  Training clamps values to
// [-4, 5] (a diverging sample then has a large but finite loss) and clips the
// gradient to norm 10.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "sp2_device.h"

struct sp2_learned {
    int n_layers = 0;
    std::vector<double> coef;       // 3 per layer, FP32-representable
    double fit_loss = 0.0;          // mean log-MSE of the last epoch
    // inference cache: one plan per (sizes, occupations, dtype, bar)
    sp2_plan* plan = nullptr;
    int key_batch = 0, key_n = 0;
    std::vector<int> key_nocc;
    sp2_dtype key_dtype = SP2_F64;
    double key_fb = 0.0;
    void* fb_ws = nullptr;          // workspace of the fallback solves
    size_t fb_ws_bytes = 0;
};

namespace sp2 {

constexpr int kLearnMaxLayers = 64;
constexpr int kContinueSteps = 60;   // plain SP2 steps allowed after the layers
constexpr int kLearnMaxN = 1024;

// One sample per workgroup.  lam: spectra (ascending) of all samples,
// concatenated at off[s]; gersh: emin, emax per sample; idx: the samples of
// this minibatch.  grad: 3 L doubles per minibatch entry; loss: one each.
// Dynamic LDS: L * n doubles of layer inputs.
__global__ __launch_bounds__(kThreads) void k_learned_grad(const double* __restrict__ lam,
                                                           const int* __restrict__ off,
                                                           const int* __restrict__ nsz,
                                                           const int* __restrict__ nocc,
                                                           const double* __restrict__ gersh,
                                                           const int* __restrict__ idx,
                                                           const double* __restrict__ coef, int L,
                                                           double* __restrict__ grad,
                                                           double* __restrict__ loss) {
    extern __shared__ double hist[];   // hist[k * n + i] = input of layer k
    __shared__ double red[4];
    __shared__ int ph[kLearnMaxLayers];
    const int s = idx[blockIdx.x];
    const int n = nsz[s], no = nocc[s];
    const double* l = lam + off[s];
    const double emin = gersh[2 * s], emax = gersh[2 * s + 1];
    const int tid = threadIdx.x;
    for (int i = tid; i < n; i += kThreads) hist[i] = (emax - l[i]) / (emax - emin);
    __syncthreads();
    // forward: layer k reads hist[k], writes hist[k + 1] (or the output)
    double xout[kLearnMaxN / kThreads];
    for (int k = 0; k < L; ++k) {
        const double* x = hist + (size_t)k * n;
        double t = 0.0;
        for (int i = tid; i < n; i += kThreads) t += x[i];
        t = block_sum(t, red);
        const int p = (t - (double)no <= 0.0) ? 1 : 0;
        if (tid == 0) ph[k] = p;
        const double a = coef[3 * k], b = coef[3 * k + 1], c = coef[3 * k + 2];
        int q = 0;
        for (int i = tid; i < n; i += kThreads, ++q) {
            const double u = p ? 1.0 - x[i] : x[i];
            const double y = a * u * u + b * u + c;
            // guard: a composition of quadratics overflows once a value leaves
            // the basin; such samples have a large loss anyway
            const double v = fmin(fmax(p ? 1.0 - y : y, -4.0), 5.0);
            if (k + 1 < L) hist[(size_t)(k + 1) * n + i] = v;
            else xout[q] = v;
        }
        __syncthreads();
    }
    // loss = log(mse), mse = mean_i (x_i - theta_i)^2, theta_i = [i < n_occ]
    double se = 0.0;
    {
        int q = 0;
        for (int i = tid; i < n; i += kThreads, ++q) {
            const double d = xout[q] - (i < no ? 1.0 : 0.0);
            se += d * d;
        }
    }
    const double mse = block_sum(se, red) / (double)n + 1e-30;
    // backward through the recorded branches
    double g[kLearnMaxN / kThreads];
    {
        int q = 0;
        for (int i = tid; i < n; i += kThreads, ++q)
            g[q] = 2.0 * (xout[q] - (i < no ? 1.0 : 0.0)) / ((double)n * mse);
    }
    for (int k = L - 1; k >= 0; --k) {
        const double* x = hist + (size_t)k * n;
        const int p = ph[k];
        const double a = coef[3 * k], b = coef[3 * k + 1];
        const double sg = p ? -1.0 : 1.0;
        double ga = 0.0, gb = 0.0, gc = 0.0;
        int q = 0;
        for (int i = tid; i < n; i += kThreads, ++q) {
            const double u = p ? 1.0 - x[i] : x[i];
            ga += g[q] * sg * u * u;
            gb += g[q] * sg * u;
            gc += g[q] * sg;
            g[q] *= 2.0 * a * u + b;
        }
        ga = block_sum(ga, red);
        gb = block_sum(gb, red);
        gc = block_sum(gc, red);
        if (tid == 0) {
            grad[(size_t)blockIdx.x * 3 * L + 3 * k + 0] = ga;
            grad[(size_t)blockIdx.x * 3 * L + 3 * k + 1] = gb;
            grad[(size_t)blockIdx.x * 3 * L + 3 * k + 2] = gc;
        }
    }
    if (tid == 0) loss[blockIdx.x] = log(mse);
}

// Deterministic generator for the minibatch order (splitmix64).
inline uint64_t splitmix64(uint64_t& x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace sp2

namespace {

void model_free(sp2_learned* m) {
    if (!m) return;
    if (m->plan) sp2_plan_destroy(m->plan);
    if (m->fb_ws) (void)hipFree(m->fb_ws);
    delete m;
}

double to_f32(double v) { return (double)(float)v; }

}  // namespace

extern "C" {

int sp2_learned_create(sp2_learned** model, int n_layers, const double* coef) {
    if (!model) return SP2_E_INVALID;
    *model = nullptr;
    if (n_layers < 0 || n_layers > sp2::kLearnMaxLayers || (n_layers > 0 && !coef)) return SP2_E_INVALID;
    sp2_learned* m = new (std::nothrow) sp2_learned;
    if (!m) return SP2_E_HIP;
    m->n_layers = n_layers;
    m->coef.resize((size_t)3 * n_layers);
    for (int i = 0; i < 3 * n_layers; ++i) {
        if (!std::isfinite(coef[i])) {
            delete m;
            return SP2_E_INVALID;
        }
        m->coef[i] = to_f32(coef[i]);
    }
    *model = m;
    return SP2_OK;
}

int sp2_learned_fit(sp2_learned** model, int n_layers, const double* spectra, const int* n,
                    const int* n_occ, int n_samples, const double* gersh, int epochs, uint64_t seed) {
    if (!model) return SP2_E_INVALID;
    *model = nullptr;
    if (n_layers < 1 || n_layers > sp2::kLearnMaxLayers || !spectra || !n || !n_occ || !gersh ||
        n_samples < 1 || epochs < 0)
        return SP2_E_INVALID;
    int nmax = 0;
    std::vector<int> off(n_samples);
    long total = 0;
    for (int s = 0; s < n_samples; ++s) {
        if (n[s] < 1 || n[s] > sp2::kLearnMaxN || n_occ[s] < 0 || n_occ[s] > n[s] ||
            !(gersh[2 * s + 1] > gersh[2 * s]))
            return SP2_E_INVALID;
        off[s] = (int)total;
        total += n[s];
        if (total > (1l << 30)) return SP2_E_INVALID;
        nmax = n[s] > nmax ? n[s] : nmax;
    }
    const size_t lds = (size_t)n_layers * nmax * sizeof(double);
    if (lds > 150 * 1024) return SP2_E_INVALID;   // layer inputs must fit one CU's LDS
    const int L = n_layers;
    const int B = n_samples < 512 ? n_samples : 512;   // minibatch
    // device copies
    char* dmem = nullptr;
    const size_t b_lam = (size_t)total * sizeof(double);
    const size_t b_int = (size_t)n_samples * sizeof(int);
    const size_t b_g = (size_t)n_samples * 2 * sizeof(double);
    const size_t b_coef = (size_t)3 * L * sizeof(double);
    const size_t b_grad = (size_t)B * 3 * L * sizeof(double);
    const size_t b_loss = (size_t)B * sizeof(double);
    const size_t bytes = b_lam + 4 * b_int + b_g + b_coef + b_grad + b_loss + 16 * 256;
    if (hipMalloc(&dmem, bytes) != hipSuccess) return SP2_E_HIP;
    size_t o = 0;
    auto take = [&](size_t b) { char* p = dmem + o; o = (o + b + 255) / 256 * 256; return p; };
    double* d_lam = (double*)take(b_lam);
    int* d_off = (int*)take(b_int);
    int* d_n = (int*)take(b_int);
    int* d_no = (int*)take(b_int);
    int* d_idx = (int*)take(b_int);
    double* d_g = (double*)take(b_g);
    double* d_coef = (double*)take(b_coef);
    double* d_grad = (double*)take(b_grad);
    double* d_loss = (double*)take(b_loss);
    hipError_t e = hipMemcpy(d_lam, spectra, b_lam, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_off, off.data(), b_int, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_n, n, b_int, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_no, n_occ, b_int, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_g, gersh, b_g, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)sp2::k_learned_grad, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
    // start from SP2 (a, b, c) = (1, 0, 0); Adam with a decaying step
    std::vector<double> coef((size_t)3 * L), mom(coef.size(), 0.0), var(coef.size(), 0.0);
    for (int k = 0; k < L; ++k) {
        coef[3 * k] = 1.0;
        coef[3 * k + 1] = 0.0;
        coef[3 * k + 2] = 0.0;
    }
    std::vector<int> perm(n_samples);
    for (int s = 0; s < n_samples; ++s) perm[s] = s;
    std::vector<double> g((size_t)B * 3 * L), lossv(B);
    uint64_t rng = seed;
    long t = 0;
    double lr = 1e-3, last_loss = 0.0;
    const int per_epoch = (n_samples + B - 1) / B;
    for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) {
        for (int s = n_samples - 1; s > 0; --s) {    // Fisher-Yates with splitmix64
            const int j = (int)(sp2::splitmix64(rng) % (uint64_t)(s + 1));
            const int tmp = perm[s];
            perm[s] = perm[j];
            perm[j] = tmp;
        }
        double ep_loss = 0.0;
        int ep_cnt = 0;
        for (int mb = 0; mb < per_epoch && e == hipSuccess; ++mb) {
            const int b0 = mb * B, nb = (b0 + B <= n_samples) ? B : n_samples - b0;
            e = hipMemcpy(d_idx, perm.data() + b0, nb * sizeof(int), hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(d_coef, coef.data(), b_coef, hipMemcpyHostToDevice);
            if (e != hipSuccess) break;
            hipLaunchKernelGGL(sp2::k_learned_grad, dim3(nb), dim3(sp2::kThreads), lds, 0, d_lam, d_off, d_n,
                               d_no, d_g, d_idx, d_coef, L, d_grad, d_loss);
            e = hipGetLastError();
            if (e == hipSuccess) e = hipMemcpy(g.data(), d_grad, (size_t)nb * 3 * L * sizeof(double),
                                               hipMemcpyDeviceToHost);
            if (e == hipSuccess) e = hipMemcpy(lossv.data(), d_loss, nb * sizeof(double), hipMemcpyDeviceToHost);
            if (e != hipSuccess) break;
            ++t;
            std::vector<double> gsum(coef.size(), 0.0);
            double gn = 0.0;
            for (size_t q = 0; q < coef.size(); ++q) {
                for (int b = 0; b < nb; ++b) gsum[q] += g[(size_t)b * 3 * L + q];   // sample order
                gsum[q] /= nb;
                gn += gsum[q] * gsum[q];
            }
            gn = std::sqrt(gn);
            if (!std::isfinite(gn)) continue;                  // skip a step that overflowed
            const double clip = gn > 10.0 ? 10.0 / gn : 1.0;   // global-norm clipping
            for (size_t q = 0; q < coef.size(); ++q) {
                const double gs = gsum[q] * clip;
                mom[q] = 0.9 * mom[q] + 0.1 * gs;
                var[q] = 0.999 * var[q] + 0.001 * gs * gs;
                const double mh = mom[q] / (1.0 - std::pow(0.9, (double)t));
                const double vh = var[q] / (1.0 - std::pow(0.999, (double)t));
                coef[q] = to_f32(coef[q] - lr * mh / (std::sqrt(vh) + 1e-12));
            }
            for (int b = 0; b < nb; ++b) ep_loss += lossv[b];
            ep_cnt += nb;
        }
        last_loss = ep_cnt ? ep_loss / ep_cnt : 0.0;
        if (epochs >= 10 && (ep + 1) % (epochs / 10) == 0) lr *= 0.8;
    }
    (void)hipFree(dmem);
    if (e != hipSuccess) return SP2_E_HIP;
    int st = sp2_learned_create(model, L, coef.data());
    if (st == SP2_OK) (*model)->fit_loss = last_loss;
    return st;
}

int sp2_learned_coefficients(const sp2_learned* model, double* coef, int capacity, double* fit_loss) {
    if (!model) return SP2_E_INVALID;
    const int c = 3 * model->n_layers;
    if (coef)
        for (int i = 0; i < c && i < capacity; ++i) coef[i] = model->coef[i];
    if (fit_loss) *fit_loss = model->fit_loss;
    return model->n_layers;
}

int sp2_learned_save(const sp2_learned* model, const char* path) {
    if (!model || !path) return SP2_E_INVALID;
    FILE* f = std::fopen(path, "w");
    if (!f) return SP2_E_INVALID;
    std::fprintf(f, "sp2_learned 1\nlayers %d\nfit_loss %a\n", model->n_layers, model->fit_loss);
    for (int k = 0; k < model->n_layers; ++k)
        std::fprintf(f, "%a %a %a\n", model->coef[3 * k], model->coef[3 * k + 1], model->coef[3 * k + 2]);
    const bool ok = std::fclose(f) == 0;
    return ok ? SP2_OK : SP2_E_INVALID;
}

int sp2_learned_load(sp2_learned** model, const char* path) {
    if (!model || !path) return SP2_E_INVALID;
    *model = nullptr;
    FILE* f = std::fopen(path, "r");
    if (!f) return SP2_E_INVALID;
    int version = 0, L = -1;
    double loss = 0.0;
    int ok = std::fscanf(f, "sp2_learned %d layers %d fit_loss %la", &version, &L, &loss) == 3 && version == 1 &&
             L >= 0 && L <= sp2::kLearnMaxLayers;
    std::vector<double> c(ok ? (size_t)3 * L : 0);
    for (size_t i = 0; ok && i < c.size(); ++i) ok = std::fscanf(f, "%la", &c[i]) == 1;
    std::fclose(f);
    if (!ok) return SP2_E_INVALID;
    int st = sp2_learned_create(model, L, c.data());
    if (st == SP2_OK) (*model)->fit_loss = loss;
    return st;
}

int sp2_learned_density(sp2_learned* model, int batch, int n, const void* const* H, void* const* D,
                        const int* n_occ, sp2_dtype dtype, sp2_compute compute, double idem_fallback,
                        void* hip_stream, sp2_info* infos) {
    if (!model || batch < 1 || n < 1 || n > SP2_PLAN_MAX_N || !H || !D || !n_occ) return SP2_E_INVALID;
    if (!(idem_fallback > 0.0) || (dtype != SP2_F64 && dtype != SP2_F32)) return SP2_E_INVALID;
    if (compute < SP2_C_F64 || compute > SP2_C_FP8) return SP2_E_INVALID;
    if (compute != SP2_C_F64) return SP2_E_UNSUPPORTED;
    for (int b = 0; b < batch; ++b)
        if (n_occ[b] < 0 || n_occ[b] > n) return SP2_E_INVALID;
    const bool same = model->plan && model->key_batch == batch && model->key_n == n &&
                      model->key_dtype == dtype && model->key_fb == idem_fallback &&
                      std::equal(model->key_nocc.begin(), model->key_nocc.end(), n_occ);
    if (!same) {
        if (model->plan) sp2_plan_destroy(model->plan);
        model->plan = nullptr;
        std::vector<int> ns(batch, n);
        int max_iter = model->n_layers + 1 + sp2::kContinueSteps;
        if (max_iter > SP2_MAX_ITER) max_iter = SP2_MAX_ITER;
        const int st = sp2::plan_create_impl(&model->plan, batch, ns.data(), n_occ, dtype, SP2_C_F64, 1e-10,
                                             max_iter, nullptr, model->coef.data(), model->n_layers,
                                             idem_fallback, 0);
        if (st != SP2_OK) return st;
        model->key_batch = batch;
        model->key_n = n;
        model->key_nocc.assign(n_occ, n_occ + batch);
        model->key_dtype = dtype;
        model->key_fb = idem_fallback;
    }
    std::vector<sp2_info> inf(batch);
    int st = sp2_plan_run(model->plan, H, D, hip_stream, inf.data());
    if (st == SP2_E_HIP) return st;
    // plain SP2 from H for every rejected matrix
    int worst_neg = 0, worst_pos = SP2_OK;
    for (int b = 0; b < batch; ++b) {
        // a continuation or in-run restart that did not converge, or a
        // rejection the run could not restart (refine_steps == 0): solve
        // again from H on the host side of the plan
        if ((inf[b].status == SP2_E_FALLBACK && inf[b].refine_steps == 0) ||
            inf[b].status == SP2_E_NOT_CONVERGED || inf[b].status == SP2_E_STAGNATED) {
            const size_t need = sp2_workspace_size(n, dtype, SP2_C_F64);
            if (model->fb_ws_bytes < need) {
                if (model->fb_ws) (void)hipFree(model->fb_ws);
                model->fb_ws = nullptr;
                model->fb_ws_bytes = 0;
                if (hipMalloc(&model->fb_ws, need) != hipSuccess) return SP2_E_HIP;
                model->fb_ws_bytes = need;
            }
            sp2_info r{};
            const int s2 = sp2_density(H[b], D[b], n, n, n_occ[b], 1e-10, 100, dtype, SP2_C_F64, -1, model->fb_ws,
                                       model->fb_ws_bytes, hip_stream, &r);
            const int layers_done = inf[b].fp64_prefix_iters;
            inf[b] = r;
            inf[b].fp64_prefix_iters = layers_done;   // the rejected learned pass
            inf[b].refine_steps = r.iterations;       // the plain SP2 solve from H
            if (s2 == SP2_OK) inf[b].status = SP2_E_FALLBACK;
        }
        if (inf[b].status < worst_neg) worst_neg = inf[b].status;
        if (inf[b].status > worst_pos) worst_pos = inf[b].status;
    }
    if (infos)
        for (int b = 0; b < batch; ++b) infos[b] = inf[b];
    return worst_neg < 0 ? worst_neg : worst_pos;
}

int sp2_learned_destroy(sp2_learned* model) {
    if (!model) return SP2_E_INVALID;
    model_free(model);
    return SP2_OK;
}

}  // extern "C"
