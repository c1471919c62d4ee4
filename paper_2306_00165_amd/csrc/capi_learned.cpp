// C ABI of the learned extrapolator's building blocks: the BF16 MLP (forward,
// MSE gradient, Adam) and the FP64 POD of snapshot sets.  The proposal step
// that combines them with a pcfv context lives in capi.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pcfv.h"
#include "eigsym.hpp"
#include "learned.hpp"
#include "learned_api.hpp"

using namespace pcfv;

namespace {

constexpr size_t kAlignL = 256;
size_t upl(size_t x) { return (x + kAlignL - 1) / kAlignL * kAlignL; }

bool valid_cfg(const pcfv_mlp_config* c) {
    if (!c || c->n_layers < 1 || c->n_layers > PCFV_MLP_MAX_LAYERS || c->max_batch < 1 || c->max_batch > 65536)
        return false;
    for (int l = 0; l <= c->n_layers; ++l)
        if (c->dims[l] < 1 || c->dims[l] > 16384) return false;
    return true;
}

struct MlpLayout {
    long long P = 0;
    std::vector<long long> woff, boff;
    size_t off_params, off_grads, off_m, off_v, off_pbf, off_act[PCFV_MLP_MAX_LAYERS], off_Y, off_dzf[2],
        off_dzb[PCFV_MLP_MAX_LAYERS], off_part, total;
};

MlpLayout mlp_layout(const pcfv_mlp_config& c) {
    MlpLayout L;
    const int nl = c.n_layers, B = c.max_batch;
    int dmax = 0;
    for (int l = 0; l < nl; ++l) {
        L.woff.push_back(L.P);
        L.P += (long long)c.dims[l] * c.dims[l + 1];
        L.boff.push_back(L.P);
        L.P += c.dims[l + 1];
    }
    for (int l = 0; l <= nl; ++l) dmax = std::max(dmax, c.dims[l]);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += upl(bytes);
        return at;
    };
    L.off_params = take(L.P * 4);
    L.off_grads = take(L.P * 4);
    L.off_m = take(L.P * 4);
    L.off_v = take(L.P * 4);
    L.off_pbf = take(L.P * 2);
    for (int l = 0; l < nl; ++l) L.off_act[l] = take((size_t)B * c.dims[l] * 2);
    L.off_Y = take((size_t)B * c.dims[nl] * 4);
    L.off_dzf[0] = take((size_t)B * dmax * 4);
    L.off_dzf[1] = take((size_t)B * dmax * 4);
    for (int l = 0; l < nl; ++l) L.off_dzb[l] = take((size_t)B * c.dims[l + 1] * 2);
    L.off_part = take(((size_t)B * c.dims[nl] / 256 + 2) * 4);
    L.total = o;
    return L;
}

}  // namespace

struct pcfv_mlp {
    pcfv_mlp_config cfg;
    MlpLayout L;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    float *params, *grads, *m, *v, *Y, *dzf[2], *part;
    bf16_t *pbf, *act[PCFV_MLP_MAX_LAYERS], *dzb[PCFV_MLP_MAX_LAYERS];
    int t = 0;         // Adam steps taken
    int lastB = 0;     // batch of the last forward / gradient
    std::string err;
};

namespace {

pcfv_status mfail(pcfv_mlp* m, pcfv_status s, const std::string& msg) {
    if (m) m->err = msg;
    return s;
}

#define MTRY(expr, what)                                                                                \
    do {                                                                                               \
        hipError_t _e = (expr);                                                                        \
        if (_e != hipSuccess) return mfail(mlp, PCFV_EDEVICE, std::string(what) + ": " + hipGetErrorString(_e)); \
    } while (0)

std::string g_mlp_create_err;

}  // namespace

namespace pcfv {

// Forward pass of B rows of X (device FP32, B x dims[0]) into Y (device FP32,
// B x dims[L]) on stream s; keeps the layer inputs for a gradient.
pcfv_status mlp_forward_on(pcfv_mlp* mlp, hipStream_t s, const float* X, float* Y, int B) {
    const pcfv_mlp_config& c = mlp->cfg;
    const int nl = c.n_layers;
    if (B < 1 || B > c.max_batch) return mfail(mlp, PCFV_EINVAL, "batch out of range");
    MTRY(launch_to_bf16(s, (long long)B * c.dims[0], X, mlp->act[0]), "input conversion");
    for (int l = 0; l < nl; ++l) {
        const bf16_t* W = mlp->pbf + mlp->L.woff[l];
        const float* b = mlp->params + mlp->L.boff[l];
        const int K = c.dims[l], N = c.dims[l + 1];
        if (l + 1 < nl)
            MTRY(launch_gemm_bf16(s, B, N, K, mlp->act[l], K, false, W, N, false, EPI_BIAS_RELU, b, nullptr, nullptr,
                                  mlp->act[l + 1], N),
                 "hidden layer");
        else
            MTRY(launch_gemm_bf16(s, B, N, K, mlp->act[l], K, false, W, N, false, EPI_F32, b, nullptr, Y, nullptr, N),
                 "output layer");
    }
    mlp->lastB = B;
    return PCFV_OK;
}

void mlp_shape(const pcfv_mlp* mlp, int* din, int* dout, int* max_batch) {
    *din = mlp->cfg.dims[0];
    *dout = mlp->cfg.dims[mlp->cfg.n_layers];
    *max_batch = mlp->cfg.max_batch;
}

}  // namespace pcfv

extern "C" {

long long pcfv_mlp_param_count(const pcfv_mlp_config* cfg) {
    if (!valid_cfg(cfg)) return 0;
    return mlp_layout(*cfg).P;
}

size_t pcfv_mlp_workspace_bytes(const pcfv_mlp_config* cfg) {
    if (!valid_cfg(cfg)) return 0;
    return mlp_layout(*cfg).total;
}

pcfv_status pcfv_mlp_create(const pcfv_mlp_config* cfg, void* hip_stream, void* workspace, pcfv_mlp** out) {
    g_mlp_create_err.clear();
    if (!out || !valid_cfg(cfg)) {
        g_mlp_create_err = "invalid MLP configuration";
        return PCFV_EINVAL;
    }
    *out = nullptr;
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlignL) {
        g_mlp_create_err = "workspace NULL or not 256-byte aligned";
        return PCFV_ENOMEM;
    }
    pcfv_mlp* m = new pcfv_mlp();
    m->cfg = *cfg;
    m->L = mlp_layout(*cfg);
    m->stream = reinterpret_cast<hipStream_t>(hip_stream);
    m->ws = reinterpret_cast<char*>(workspace);
    auto F = [&](size_t off) { return reinterpret_cast<float*>(m->ws + off); };
    auto H = [&](size_t off) { return reinterpret_cast<bf16_t*>(m->ws + off); };
    m->params = F(m->L.off_params);
    m->grads = F(m->L.off_grads);
    m->m = F(m->L.off_m);
    m->v = F(m->L.off_v);
    m->pbf = H(m->L.off_pbf);
    for (int l = 0; l < cfg->n_layers; ++l) {
        m->act[l] = H(m->L.off_act[l]);
        m->dzb[l] = H(m->L.off_dzb[l]);
    }
    m->Y = F(m->L.off_Y);
    m->dzf[0] = F(m->L.off_dzf[0]);
    m->dzf[1] = F(m->L.off_dzf[1]);
    m->part = F(m->L.off_part);
    *out = m;
    return PCFV_OK;
}

void pcfv_mlp_destroy(pcfv_mlp* mlp) { delete mlp; }

const char* pcfv_mlp_last_error(const pcfv_mlp* mlp) { return mlp ? mlp->err.c_str() : g_mlp_create_err.c_str(); }

pcfv_status pcfv_mlp_set_params(pcfv_mlp* mlp, const float* params_host) {
    if (!mlp || !params_host) return mfail(mlp, PCFV_EINVAL, "NULL argument");
    const size_t nb = (size_t)mlp->L.P * 4;
    MTRY(hipMemcpyAsync(mlp->params, params_host, nb, hipMemcpyHostToDevice, mlp->stream), "copy parameters");
    MTRY(hipMemsetAsync(mlp->m, 0, nb, mlp->stream), "clear Adam moments");
    MTRY(hipMemsetAsync(mlp->v, 0, nb, mlp->stream), "clear Adam moments");
    MTRY(launch_to_bf16(mlp->stream, mlp->L.P, mlp->params, mlp->pbf), "bf16 weights");
    MTRY(hipStreamSynchronize(mlp->stream), "synchronize");
    mlp->t = 0;
    return PCFV_OK;
}

pcfv_status pcfv_mlp_get_params(pcfv_mlp* mlp, float* params_host) {
    if (!mlp || !params_host) return mfail(mlp, PCFV_EINVAL, "NULL argument");
    MTRY(hipMemcpyAsync(params_host, mlp->params, (size_t)mlp->L.P * 4, hipMemcpyDeviceToHost, mlp->stream),
         "copy parameters");
    MTRY(hipStreamSynchronize(mlp->stream), "synchronize");
    return PCFV_OK;
}

pcfv_status pcfv_mlp_forward(pcfv_mlp* mlp, const float* X, float* Y, int B) {
    if (!mlp || !X || !Y) return mfail(mlp, PCFV_EINVAL, "NULL argument");
    return mlp_forward_on(mlp, mlp->stream, X, Y, B);
}

pcfv_status pcfv_mlp_grad(pcfv_mlp* mlp, const float* X, const float* T, int B, float* loss_host) {
    if (!mlp || !X || !T) return mfail(mlp, PCFV_EINVAL, "NULL argument");
    const pcfv_mlp_config& c = mlp->cfg;
    const int nl = c.n_layers;
    hipStream_t s = mlp->stream;
    pcfv_status st = mlp_forward_on(mlp, s, X, mlp->Y, B);
    if (st != PCFV_OK) return st;
    int nblk = 0;
    MTRY(launch_mse(s, B, c.dims[nl], mlp->Y, T, mlp->dzf[0], mlp->dzb[nl - 1], mlp->part, &nblk), "loss");
    int cur = 0;
    for (int l = nl - 1; l >= 0; --l) {
        const int K = c.dims[l], N = c.dims[l + 1];
        // dW_l = A_l^T dZ_l, db_l = column sums of dZ_l
        MTRY(launch_gemm_bf16(s, K, N, B, mlp->act[l], K, true, mlp->dzb[l], N, false, EPI_F32, nullptr, nullptr,
                              mlp->grads + mlp->L.woff[l], nullptr, N),
             "weight gradient");
        MTRY(launch_colsum(s, B, N, mlp->dzf[cur], mlp->grads + mlp->L.boff[l]), "bias gradient");
        if (l > 0)   // dZ_{l-1} = (dZ_l W_l^T) masked by the ReLU of layer l-1
            MTRY(launch_gemm_bf16(s, B, K, N, mlp->dzb[l], N, false, mlp->pbf + mlp->L.woff[l], N, true, EPI_RELU_MASK,
                                  nullptr, mlp->act[l], mlp->dzf[1 - cur], mlp->dzb[l - 1], K),
                 "input gradient");
        cur = 1 - cur;
    }
    if (loss_host) {
        std::vector<float> part(nblk);
        MTRY(hipMemcpyAsync(part.data(), mlp->part, (size_t)nblk * 4, hipMemcpyDeviceToHost, s), "copy loss");
        MTRY(hipStreamSynchronize(s), "synchronize");
        double tot = 0;
        for (float x : part) tot += x;
        *loss_host = (float)tot;
    }
    return PCFV_OK;
}

pcfv_status pcfv_mlp_adam_step(pcfv_mlp* mlp, float lr, float beta1, float beta2, float eps) {
    if (!mlp || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return mfail(mlp, PCFV_EINVAL, "invalid Adam arguments");
    ++mlp->t;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, mlp->t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, mlp->t)));
    MTRY(launch_adam(mlp->stream, mlp->L.P, mlp->grads, mlp->m, mlp->v, mlp->params, mlp->pbf, lr, beta1, beta2, eps,
                     c1, c2),
         "adam");
    return PCFV_OK;
}

pcfv_status pcfv_mlp_read(pcfv_mlp* mlp, int what, int layer, void* host, size_t cap_bytes) {
    if (!mlp || !host) return mfail(mlp, PCFV_EINVAL, "NULL argument");
    const pcfv_mlp_config& c = mlp->cfg;
    const int B = mlp->lastB;
    const void* src = nullptr;
    size_t nb = 0;
    if ((what == PCFV_MLP_ACT || what == PCFV_MLP_DZ) && (layer < 0 || layer >= c.n_layers))
        return mfail(mlp, PCFV_EINVAL, "layer out of range");
    switch (what) {
        case PCFV_MLP_ACT: src = mlp->act[layer]; nb = (size_t)B * c.dims[layer] * 2; break;
        case PCFV_MLP_OUT: src = mlp->Y; nb = (size_t)B * c.dims[c.n_layers] * 4; break;
        case PCFV_MLP_DZ: src = mlp->dzb[layer]; nb = (size_t)B * c.dims[layer + 1] * 2; break;
        case PCFV_MLP_GRAD: src = mlp->grads; nb = (size_t)mlp->L.P * 4; break;
        default: return mfail(mlp, PCFV_EINVAL, "unknown buffer");
    }
    if (nb > cap_bytes) return mfail(mlp, PCFV_EINVAL, "host buffer too small");
    MTRY(hipMemcpyAsync(host, src, nb, hipMemcpyDeviceToHost, mlp->stream), "copy");
    MTRY(hipStreamSynchronize(mlp->stream), "synchronize");
    return PCFV_OK;
}

// SplitMix64 (Steele, Lea & Flood 2014): the per-epoch permutation source.
static uint64_t splitmix64(uint64_t& x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

pcfv_status pcfv_mlp_fit(pcfv_mlp* mlp, const float* X, const float* T, int N, int batch, int epochs, float lr,
                         unsigned long long seed, int* idx, float* Xb, float* Tb, float* loss_host) {
    if (!mlp || !X || !T || !idx || !Xb || !Tb || N < 1 || batch < 1 || batch > mlp->cfg.max_batch || batch > N ||
        epochs < 0 || !(lr > 0))
        return mfail(mlp, PCFV_EINVAL, "invalid fit arguments");
    const int din = mlp->cfg.dims[0], dout = mlp->cfg.dims[mlp->cfg.n_layers];
    hipStream_t s = mlp->stream;
    uint64_t state = seed;
    std::vector<int> perm(N);
    const int nb = N / batch;
    for (int e = 0; e < epochs; ++e) {
        for (int i = 0; i < N; ++i) perm[i] = i;
        for (int i = N - 1; i > 0; --i) {   // Fisher-Yates
            const int j = (int)(splitmix64(state) % (uint64_t)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        MTRY(hipMemcpyAsync(idx, perm.data(), (size_t)N * 4, hipMemcpyHostToDevice, s), "copy permutation");
        MTRY(hipStreamSynchronize(s), "synchronize");   // perm is reused next epoch
        double tot = 0;
        for (int bi = 0; bi < nb; ++bi) {
            MTRY(launch_gather(s, batch, din, idx + (size_t)bi * batch, X, Xb), "gather");
            MTRY(launch_gather(s, batch, dout, idx + (size_t)bi * batch, T, Tb), "gather");
            float loss = 0;
            pcfv_status st = pcfv_mlp_grad(mlp, Xb, Tb, batch, loss_host ? &loss : nullptr);
            if (st != PCFV_OK) return st;
            tot += loss;
            st = pcfv_mlp_adam_step(mlp, lr, 0.9f, 0.999f, 1e-8f);
            if (st != PCFV_OK) return st;
        }
        if (loss_host) loss_host[e] = nb ? (float)(tot / nb) : 0.f;
    }
    MTRY(hipStreamSynchronize(s), "synchronize");
    return PCFV_OK;
}

pcfv_status pcfv_learned_prepare(void* hip_stream, int W, int B, int r, const double* c, const double* cb,
                                 const double* ct, int fit, float* in_mu, float* in_isd, float* out_mu, float* out_isd,
                                 float* X, float* T) {
    if (W < 1 || B < 1 || r < 1 || !c || !in_mu || !in_isd || !X || (ct && (!out_mu || !out_isd || !T)))
        return PCFV_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const float kFloor = 1e-12f;
    const int F = (W + (cb ? 1 : 0)) * r;
    if (fit) {
        if (launch_features(s, W, B, r, c, cb, nullptr, nullptr, X) != hipSuccess) return PCFV_EDEVICE;
        if (launch_colstats(s, B, F, X, kFloor, in_mu, in_isd) != hipSuccess) return PCFV_EDEVICE;
        if (launch_normalize(s, B, F, X, in_mu, in_isd) != hipSuccess) return PCFV_EDEVICE;
    } else if (launch_features(s, W, B, r, c, cb, in_mu, in_isd, X) != hipSuccess) {
        return PCFV_EDEVICE;
    }
    if (ct) {
        if (launch_targets(s, W, B, r, c, cb, ct, T) != hipSuccess) return PCFV_EDEVICE;
        if (fit && launch_colstats(s, B, r, T, kFloor, out_mu, out_isd) != hipSuccess) return PCFV_EDEVICE;
        if (launch_normalize(s, B, r, T, out_mu, out_isd) != hipSuccess) return PCFV_EDEVICE;
    }
    return PCFV_OK;
}

// ---------------------------------------------------------------------------
// POD
// ---------------------------------------------------------------------------

static int pod_splits(int M, int N, long long K) {
    const long long tiles = (long long)((M + 63) / 64) * ((N + 63) / 64);
    long long s = std::max(1LL, 512 / std::max(1LL, tiles));
    s = std::min(s, std::max(1LL, K / 256));
    return (int)std::min(64LL, s);
}

size_t pcfv_pod_scratch_bytes(int S, long long n, int r) {
    if (S < 2 || n < 1 || r < 1 || r > S) return 0;
    // centred copy, Gram partials, scaled eigenvectors
    return upl((size_t)S * n * 8) + upl((size_t)pod_splits(S, S, n) * S * S * 8) + upl((size_t)S * S * 8) +
           upl((size_t)S * r * 8);
}

pcfv_status pcfv_pod_build(void* hip_stream, const double* X, int S, long long n, int r, double* mean, double* basis,
                           double* sigma_host, void* scratch) {
    if (!X || !mean || !basis || !scratch || S < 2 || n < 1 || r < 1 || r > S) return PCFV_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    char* w = reinterpret_cast<char*>(scratch);
    double* Xc = reinterpret_cast<double*>(w);
    w += upl((size_t)S * n * 8);
    const int sp = pod_splits(S, S, n);
    double* part = reinterpret_cast<double*>(w);
    w += upl((size_t)sp * S * S * 8);
    double* G = reinterpret_cast<double*>(w);
    w += upl((size_t)S * S * 8);
    double* Vs = reinterpret_cast<double*>(w);
    if (launch_rowmean(s, S, n, X, mean) != hipSuccess) return PCFV_EDEVICE;
    if (launch_center(s, S, n, X, mean, Xc) != hipSuccess) return PCFV_EDEVICE;
    // Gram matrix of the centred snapshots (method of snapshots)
    if (launch_gemm_f64(s, S, S, n, Xc, n, false, Xc, n, true, nullptr, nullptr, G, S, sp, part) != hipSuccess)
        return PCFV_EDEVICE;
    std::vector<double> Gh((size_t)S * S), w8;
    if (hipMemcpyAsync(Gh.data(), G, Gh.size() * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return PCFV_EDEVICE;
    for (int i = 0; i < S; ++i)
        for (int j = 0; j < i; ++j) Gh[(size_t)i * S + j] = Gh[(size_t)j * S + i] = 0.5 * (Gh[(size_t)i * S + j] + Gh[(size_t)j * S + i]);
    if (!eig_symmetric(S, Gh, w8)) return PCFV_ENOTCONV;
    if (!(w8[r - 1] > 0)) return PCFV_EINVAL;   // fewer than r independent snapshots
    // basis_i = sum_s V[s][i] Xc[s] / sqrt(lambda_i)
    std::vector<double> vs((size_t)S * r);
    for (int sidx = 0; sidx < S; ++sidx)
        for (int i = 0; i < r; ++i) vs[(size_t)sidx * r + i] = Gh[(size_t)sidx * S + i] / std::sqrt(w8[i]);
    if (hipMemcpyAsync(Vs, vs.data(), vs.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess) return PCFV_EDEVICE;
    if (launch_gemm_f64(s, r, (int)std::min<long long>(n, 1LL << 30), S, Vs, r, true, Xc, n, false, nullptr, nullptr,
                        basis, n, 1, nullptr) != hipSuccess)
        return PCFV_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return PCFV_EDEVICE;
    if (sigma_host)
        for (int i = 0; i < r; ++i) sigma_host[i] = std::sqrt(w8[i]);
    return PCFV_OK;
}

size_t pcfv_pod_project_scratch_bytes(int m, long long n, int r) {
    if (m < 1 || n < 1 || r < 1) return 0;
    return (size_t)pod_splits(m, r, n) * m * r * 8;
}

pcfv_status pcfv_pod_project(void* hip_stream, const double* X, int m, long long n, int r, const double* mean,
                             const double* basis, double* coef, void* scratch) {
    if (!X || !mean || !basis || !coef || m < 1 || n < 1 || r < 1) return PCFV_EINVAL;
    const int sp = pod_splits(m, r, n);
    if (sp > 1 && !scratch) return PCFV_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    return launch_gemm_f64(s, m, r, n, X, n, false, basis, n, true, mean, nullptr, coef, r, sp,
                           reinterpret_cast<double*>(scratch)) == hipSuccess
               ? PCFV_OK
               : PCFV_EDEVICE;
}

pcfv_status pcfv_pod_project_noalloc(void* hip_stream, const double* X, int m, long long n, int r,
                                     const double* mean, const double* basis, double* coef) {
    if (!X || !mean || !basis || !coef || m < 1 || n < 1 || r < 1) {
        set_create_error("pcfv_pod_project_noalloc: NULL pointer or non-positive size");
        return PCFV_EINVAL;
    }
    const int sp = pod_splits(m, r, n);
    const size_t need = pcfv_pod_project_scratch_bytes(m, n, r);
    if (sp > 1 && need > kStaticScratchBytes) {
        set_create_error("pcfv_pod_project_noalloc: the split-K partials need " + std::to_string(need) +
                         " bytes, more than the " + std::to_string(kStaticScratchBytes) +
                         "-byte device-resident scratch; use pcfv_pod_project with a workspace");
        return PCFV_ENOMEM;
    }
    double* part = nullptr;
    if (sp > 1 && static_scratch(&part) != hipSuccess) {
        set_create_error("pcfv_pod_project_noalloc: hipGetSymbolAddress of the scratch array failed");
        return PCFV_EDEVICE;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    return launch_gemm_f64(s, m, r, n, X, n, false, basis, n, true, mean, nullptr, coef, r, sp, part) == hipSuccess
               ? PCFV_OK
               : PCFV_EDEVICE;
}

pcfv_status pcfv_pod_reconstruct(void* hip_stream, const double* coef, int m, long long n, int r, const double* mean,
                                 const double* basis, double* X) {
    if (!coef || !mean || !basis || !X || m < 1 || n < 1 || r < 1 || n > (1LL << 30)) return PCFV_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    return launch_gemm_f64(s, m, (int)n, r, coef, r, false, basis, n, false, nullptr, mean, X, n, 1, nullptr) ==
                   hipSuccess
               ? PCFV_OK
               : PCFV_EDEVICE;
}

}  // extern "C"
