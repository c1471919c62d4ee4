// C ABI of libpcfv (declared in include/pcfv.h): context, workspace layout,
// and the host-side sequencing of the kernels for each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pcfv.h"
#include "dmd.hpp"
#include "kernels.hpp"
#include "learned.hpp"
#include "learned_api.hpp"
#include "tables.hpp"

using namespace pcfv;

namespace {

enum WsSlot {
    W_MATS, W_MINFO, W_DH, W_DP, W_DPROJ, W_VK, W_DVK, W_AINV, W_TWX, W_TWZ, W_YGL, W_INDEP,
    W_Y, W_YV, W_ATIL, W_P3, W_P6, W_A, W_R, W_CK, W_TMP, W_PART, W_SCAL, W_DMDG, W_DMDC, W_DMDPSI,
    W_COUNT
};

struct WsLayout {
    size_t off[W_COUNT];
    size_t total;
};

constexpr size_t kAlign = 256;
constexpr size_t kMaxPlaneLds = 160 * 1024;   // the LDS a gfx950 work group may allocate
constexpr int kMaxDmd = 256;   // largest DMD window

size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool validate(const pcfv_config* c, std::string& e) {
    if (!c) {
        e = "config is NULL";
        return false;
    }
    if (c->precision != PCFV_FP64 && c->precision != PCFV_MIXED) {
        e = "precision must be PCFV_FP64 (0) or PCFV_MIXED (1)";
        return false;
    }
    if (c->batch < 0 || c->batch > 4096) {
        e = "batch must lie in [0, 4096] (0 means 1)";
        return false;
    }
    if (c->Nx < 6 || c->Nz < 6 || c->Nx > 512 || c->Nz > 512) {
        e = "Nx and Nz must lie in [6, 512]";
        return false;
    }
    if (c->Ny < 9 || c->Ny > 128) {
        e = "Ny must lie in [9, 128]";
        return false;
    }
    if (!(c->Lx > 0) || !(c->Lz > 0) || !(c->Re > 0) || !(c->dt_im > 0) ||
        !std::isfinite(c->Lx + c->Lz + c->Re + c->dt_im)) {
        e = "Lx, Lz, Re and dt_im must be positive and finite";
        return false;
    }
    return true;
}

// Default physical-space work-group size for a launch of nmB modes (see base_kp).
static int plane_threads_default(int prec, long long nmB) {
    if (prec == PREC_FP64) return 768;
    return nmB > 1024 ? 512 : 1024;
}

KP base_kp(const pcfv_config& c) {
    KP p{};
    p.N = c.Ny;
    p.Nx = c.Nx;
    p.Nz = c.Nz;
    p.Kx = c.Nx / 3 - 1;
    p.Kz = c.Nz / 3 - 1;
    p.nkx = 2 * p.Kx + 1;
    p.nkz = p.Kz + 1;
    p.nm = p.nkx * p.nkz;
    p.B = c.batch > 0 ? c.batch : 1;
    p.nmB = p.B * p.nm;
    p.np = padded_ny(p.N);
    // widest x slab (a divisor of Nx) whose physical-space kernels fit the LDS
    // budget, at most 12 when a launch holds few modes (the latency-bound
    // case: more work groups) and at most 16 otherwise (fewer slabs, less
    // partial traffic)
    p.XS = 1;
    const int xs_max = (p.nmB <= 1024) ? 12 : 16;
    for (int xs = xs_max; xs >= 1; --xs) {
        if (c.Nx % xs) continue;
        p.XS = xs;
        if (plane_lds_bytes(p, PLANE_ADJ) <= kMaxPlaneLds && plane_lds_bytes(p, PLANE_JVP) <= kMaxPlaneLds)
            break;
    }
    p.NS = c.Nx / p.XS;
    p.prec = c.precision == PCFV_MIXED ? PREC_FP32 : PREC_FP64;
    // Physical-space group size: 768 threads in FP64 (1024 would spill a few
    // registers of the forward kernel); in FP32 1024, or 512 with many modes
    // (more groups resident per CU)
    p.pthreads = plane_threads_default(p.prec, p.nmB);
    // per-mode groups of 256 threads (4 lanes per contraction row): their
    // contractions have no idle waves for Ny up to 64 and several groups share a CU
    p.mthreads = 256;
    return p;
}

// The fixed matrices as the per-mode kernels read them: every N x N slot
// zero-padded to np rows of mat_ld(np) entries, same transposed layout.
std::vector<double> padded_mats(const std::vector<double>& mats, int N, int np) {
    const int ld = mat_ld(np);
    std::vector<double> out((size_t)M_COUNT * np * ld, 0.0);
    for (int id = 0; id < M_COUNT; ++id)
        for (int k = 0; k < N; ++k)
            std::copy_n(mats.data() + ((size_t)id * N + k) * N, N, out.data() + ((size_t)id * np + k) * ld);
    return out;
}

// x-slab widths the autotuner may choose: divisors of Nx up to 16 whose
// physical-space kernels fit the LDS budget, no narrower than half the
// default (so the partial buffers are at most twice the default's).
std::vector<int> xs_candidates(const pcfv_config& c) {
    KP p = base_kp(c);
    p.prec = PREC_FP64;
    const int xs0 = p.XS;
    std::vector<int> out;
    for (int xs = 16; xs >= 1; --xs) {
        if (c.Nx % xs || 2 * xs < xs0) continue;
        p.XS = xs;
        if (plane_lds_bytes(p, PLANE_ADJ) <= kMaxPlaneLds && plane_lds_bytes(p, PLANE_JVP) <= kMaxPlaneLds)
            out.push_back(xs);
    }
    if (out.empty()) out.push_back(xs0);
    return out;
}

WsLayout layout(const pcfv_config& c) {
    const KP p = base_kp(c);
    const std::vector<int> xsc = xs_candidates(c);
    const size_t N = p.N, nm = p.nm, NS = c.Nx / *std::min_element(xsc.begin(), xsc.end()), nmB = p.nmB,
                 B = p.B;
    size_t sz[W_COUNT];
    sz[W_MATS] = (size_t)M_COUNT * p.np * mat_ld(p.np) * 8;
    sz[W_MINFO] = nm * MI_STRIDE * 8;
    sz[W_DH] = sz[W_DP] = sz[W_DPROJ] = nm * N * 8;
    sz[W_VK] = sz[W_DVK] = nm * 4 * N * 8;
    sz[W_AINV] = nm * 16 * 8;
    sz[W_TWX] = (size_t)c.Nx * 16;
    sz[W_TWZ] = (size_t)c.Nz * 16;
    sz[W_YGL] = N * 8;
    sz[W_INDEP] = nm * 4;
    sz[W_Y] = sz[W_YV] = 6 * N * nmB * 16;
    sz[W_ATIL] = 3 * N * nmB * 16;
    sz[W_P3] = NS * 3 * N * nmB * 16;
    sz[W_P6] = NS * 6 * N * nmB * 16;
    sz[W_A] = sz[W_R] = sz[W_CK] = sz[W_TMP] = 3 * nmB * N * 16;
    sz[W_PART] = nmB * 4 * 8;
    sz[W_SCAL] = (64 + 4 * B) * 8;
    const long long nstate = 4LL * (p.Kx + 2LL * p.Kx * p.Kz + p.Kz) * (p.N - 3) + 2LL * (p.N - 2);
    sz[W_DMDG] = B * kMaxDmd * kMaxDmd * 16;
    sz[W_DMDC] = B * kMaxDmd * 8;
    sz[W_DMDPSI] = B * (size_t)nstate * 8;
    WsLayout L;
    size_t o = 0;
    for (int i = 0; i < W_COUNT; ++i) {
        L.off[i] = o;
        o += up(sz[i]);
    }
    L.total = o;
    return L;
}

}  // namespace

struct pcfv_ctx {
    pcfv_config cfg;
    Tables t;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    WsLayout L;
    KP kp;
    double2 *Y, *Yv, *Atil, *P3, *P6, *a, *r, *ck, *tmp;
    double *part, *scal, *dmdG, *dmdC, *dmdPsi;
    std::string err;

    template <class T>
    T* at(int slot) { return reinterpret_cast<T*>(ws + L.off[slot]); }
    long long nfield() const { return 3LL * kp.nmB * kp.N; }  // complex values, all guesses
};

namespace {

thread_local std::string g_create_err;  // reason of the last failed pcfv_create on this thread

}  // namespace

void pcfv::set_create_error(const std::string& msg) { g_create_err = msg; }

namespace {

pcfv_status fail(pcfv_ctx* c, pcfv_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

pcfv_status hip_check(pcfv_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return PCFV_OK;
    return fail(c, PCFV_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define PCFV_TRY(expr, what)                                   \
    do {                                                       \
        pcfv_status _s = hip_check(ctx, (expr), what);         \
        if (_s != PCFV_OK) return _s;                          \
    } while (0)

const double2* cd(const double* p) { return reinterpret_cast<const double2*>(p); }
double2* dd(double* p) { return reinterpret_cast<double2*>(p); }

// Residual of u into r (if r) and per-mode cost partials; Y must hold the
// y-values of u.
pcfv_status residual_core(pcfv_ctx* ctx, const double* u, double* r, bool cost) {
    const KP& p = ctx->kp;
    PCFV_TRY(launch_plane(p, ctx->stream, PLANE_FWD, ctx->Y, nullptr, ctx->P3), "plane fwd");
    int flags = (r ? RES_WRITE_R : 0) | (cost ? RES_COST : 0);
    PCFV_TRY(launch_mode_res(p, ctx->stream, flags, ctx->P3, cd(u), r ? dd(r) : ctx->r, ctx->part,
                             nullptr, nullptr),
             "mode res");
    return PCFV_OK;
}

pcfv_status read_scalars(pcfv_ctx* ctx, int stride, int op, double* host) {
    const KP& p = ctx->kp;
    PCFV_TRY(launch_reduce(ctx->stream, ctx->part, p.B, p.nm, stride, op, ctx->scal), "reduce");
    PCFV_TRY(hipMemcpyAsync(host, ctx->scal, (size_t)p.B * stride * sizeof(double), hipMemcpyDeviceToHost,
                            ctx->stream),
             "copy scalars");
    PCFV_TRY(hipStreamSynchronize(ctx->stream), "synchronize");
    return PCFV_OK;
}

// Per-guess cost J^2 and ||u_b + u||_W of the current state (Y must hold its
// y-values).
pcfv_status cost_and_norm(pcfv_ctx* ctx, const double* u, std::vector<double>& cost,
                          std::vector<double>& ntot) {
    const int B = ctx->kp.B;
    pcfv_status s = residual_core(ctx, u, nullptr, true);
    if (s != PCFV_OK) return s;
    cost.assign(B, 0.0);
    s = read_scalars(ctx, 1, 0, cost.data());
    if (s != PCFV_OK) return s;
    PCFV_TRY(launch_norms(ctx->kp, ctx->stream, cd(u), ctx->part), "norms");
    std::vector<double> nrm(3 * B);
    s = read_scalars(ctx, 3, 0, nrm.data());
    if (s != PCFV_OK) return s;
    ntot.assign(B, 0.0);
    for (int b = 0; b < B; ++b) ntot[b] = std::sqrt(nrm[3 * b + 1]);
    return PCFV_OK;
}

pcfv_status descent_step(pcfv_ctx* ctx, double* u, double dtau) {
    const KP& p = ctx->kp;
    hipStream_t s = ctx->stream;
    PCFV_TRY(launch_plane(p, s, PLANE_FWD, ctx->Y, nullptr, ctx->P3), "plane fwd");
    PCFV_TRY(launch_mode_res(p, s, RES_COST | RES_ADJ, ctx->P3, cd(u), nullptr, ctx->part, ctx->a,
                             ctx->Atil),
             "mode res");
    PCFV_TRY(launch_plane(p, s, PLANE_ADJ, ctx->Y, ctx->Atil, ctx->P6), "plane adj");
    PCFV_TRY(launch_mode_grad(p, s, GRAD_PROJECT | GRAD_UPDATE, ctx->P6, ctx->a, dtau, dd(u), ctx->Y),
             "mode grad");
    return PCFV_OK;
}


// Scratch of the learned proposal: POD coefficients of the window, features,
// MLP output, predicted coefficients, state vectors, projection partials.
struct LearnedScratch {
    size_t c, cb, x, y, cs, psi, part, total;
    int splits;
};

LearnedScratch learned_scratch(const KP& p, int W, int r) {
    LearnedScratch L{};
    const long long n = p.nstate;
    const int rows = W * p.B;
    const long long tiles = (long long)((rows + 63) / 64) * ((r + 63) / 64);
    L.splits = (int)std::min(64LL, std::max(1LL, std::min(512 / std::max(1LL, tiles), n / 256)));
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o += up(b);
        return at;
    };
    L.c = take((size_t)rows * r * 8);
    L.cb = take((size_t)p.B * r * 8);
    L.x = take((size_t)p.B * (W + 1) * r * 4);
    L.y = take((size_t)p.B * r * 4);
    L.cs = take((size_t)p.B * r * 8);
    L.psi = take((size_t)p.B * n * 8);
    L.part = take((size_t)L.splits * rows * r * 8);
    L.total = o;
    return L;
}

// Learned proposal of every guess into u_out (field layout) and its cost.
// base (state vectors [B][n], required iff the model uses a base candidate)
// is the state the predicted POD step starts from; otherwise the last snapshot.
pcfv_status learned_core(pcfv_ctx* ctx, const pcfv_learned_model* md, const double* snaps, const double* base,
                         double* u_out, std::vector<double>& cost) {
    const KP& p = ctx->kp;
    const int W = md->window, r = md->r, B = p.B;
    int din = 0, dout = 0, mb = 0;
    if (!md->mlp || !md->pod_mean || !md->pod_basis || !md->in_mu || !md->in_isd || !md->out_mu || !md->out_isd ||
        !md->scratch || W < 1 || r < 1)
        return fail(ctx, PCFV_EINVAL, "incomplete learned model");
    if (md->use_base && !base) return fail(ctx, PCFV_EINVAL, "the model needs a base candidate");
    mlp_shape(md->mlp, &din, &dout, &mb);
    if (din != (W + (md->use_base ? 1 : 0)) * r || dout != r || mb < B)
        return fail(ctx, PCFV_EINVAL, "MLP shape does not match the model");
    const LearnedScratch L = learned_scratch(p, W, r);
    char* w = reinterpret_cast<char*>(md->scratch);
    double* c = reinterpret_cast<double*>(w + L.c);
    double* cb = md->use_base ? reinterpret_cast<double*>(w + L.cb) : nullptr;
    float* x = reinterpret_cast<float*>(w + L.x);
    float* y = reinterpret_cast<float*>(w + L.y);
    double* cs = reinterpret_cast<double*>(w + L.cs);
    double* psi = reinterpret_cast<double*>(w + L.psi);
    double* part = reinterpret_cast<double*>(w + L.part);
    const long long n = p.nstate;
    hipStream_t s = ctx->stream;
    PCFV_TRY(launch_gemm_f64(s, W * B, r, n, snaps, n, false, md->pod_basis, n, true, md->pod_mean, nullptr, c, r,
                             L.splits, part),
             "POD projection");
    if (cb)
        PCFV_TRY(launch_gemm_f64(s, B, r, n, base, n, false, md->pod_basis, n, true, md->pod_mean, nullptr, cb, r,
                                 L.splits, part),
                 "POD projection of the base");
    PCFV_TRY(launch_features(s, W, B, r, c, cb, md->in_mu, md->in_isd, x), "features");
    pcfv_status st = mlp_forward_on(md->mlp, s, x, y, B);
    if (st != PCFV_OK) return fail(ctx, st, "MLP forward failed");
    // psi = base + dc basis: the step lies in the POD space, the base (last
    // snapshot or candidate) keeps everything the modes do not resolve
    PCFV_TRY(launch_prediction(s, B, r, y, md->out_mu, md->out_isd, cs), "prediction");
    // a short line search along the predicted step, judged by the true cost
    const double* psi0 = cb ? base : snaps + (size_t)(W - 1) * B * n;
    const int ns = std::min(std::max(md->n_scales, 0), PCFV_LEARNED_MAX_SCALES);
    const size_t fbytes1 = (size_t)3 * p.nm * p.N * 16;
    cost.assign(B, HUGE_VAL);
    std::vector<double> ck(B);
    for (int k = 0; k < std::max(ns, 1); ++k) {
        const double a = ns ? md->scales[k] : 1.0;
        double2* trial = (ns > 1) ? ctx->tmp : dd(u_out);
        PCFV_TRY(hipMemcpyAsync(psi, psi0, (size_t)B * n * 8, hipMemcpyDeviceToDevice, s), "base state");
        PCFV_TRY(launch_gemm_f64(s, B, (int)n, r, cs, r, false, md->pod_basis, n, false, nullptr, nullptr, psi, n, 1,
                                 nullptr, true, a),
                 "POD step");
        PCFV_TRY(launch_unpack(p, s, psi, trial), "unpack");
        PCFV_TRY(launch_synth(p, s, trial, ctx->Y), "synth");
        st = residual_core(ctx, reinterpret_cast<const double*>(trial), nullptr, true);
        if (st != PCFV_OK) return st;
        st = read_scalars(ctx, 1, 0, ck.data());
        if (st != PCFV_OK) return st;
        for (int b = 0; b < B; ++b)
            if (ck[b] < cost[b] || !std::isfinite(cost[b])) {
                cost[b] = ck[b];
                if (trial != dd(u_out))
                    PCFV_TRY(hipMemcpyAsync(reinterpret_cast<char*>(u_out) + b * fbytes1,
                                            reinterpret_cast<const char*>(trial) + b * fbytes1, fbytes1,
                                            hipMemcpyDeviceToDevice, s),
                             "keep candidate");
            }
    }
    return PCFV_OK;
}

// DMD extrapolation of the window snaps ([M][B][n_state]): every candidate of
// every guess (ranks r <= r*, the kinds of dmd_candidates) is judged by its true
// cost; writes the cheapest of each guess to u_out (the last snapshot if it has
// none), its cost, rank and kind (0 and -1 for none).  Candidates are
// evaluated slot by slot, slot i holding the i-th candidate of every guess.
pcfv_status dmd_core(pcfv_ctx* ctx, const double* snaps, int M, double dtau, double* u_out,
                     std::vector<double>& best_cost, std::vector<int>& best_rank, std::vector<int>& best_kind) {
    const KP& p = ctx->kp;
    const int B = p.B;
    const long long n = p.nstate;
    const size_t gbytes = (size_t)M * M * 2 * sizeof(double);
    const size_t fbytes1 = (size_t)3 * p.nm * p.N * 16;   // one guess's field
    if (M < 3 || M > kMaxDmd) return fail(ctx, PCFV_EINVAL, "DMD window must hold 3..256 snapshots");
    PCFV_TRY(launch_dmd_gram(ctx->stream, snaps, M, B, n, ctx->dmdG), "dmd gram");
    std::vector<double> G((size_t)B * M * M * 2);
    PCFV_TRY(hipMemcpyAsync(G.data(), ctx->dmdG, (size_t)B * gbytes, hipMemcpyDeviceToHost, ctx->stream),
             "copy gram");
    PCFV_TRY(hipStreamSynchronize(ctx->stream), "synchronize");
    // the guesses' small dense algebra, spread over host threads
    std::vector<std::vector<DmdCandidate>> cands(B);
    std::vector<std::string> errs(B);
    std::vector<int> rs(B, 0);
    auto work = [&](int b) {
        std::vector<long double> Gb((size_t)M * M);
        for (size_t k = 0; k < Gb.size(); ++k)
            Gb[k] = (long double)G[((size_t)b * M * M + k) * 2] + (long double)G[((size_t)b * M * M + k) * 2 + 1];
        rs[b] = dmd_candidates(Gb, M, dtau, cands[b], errs[b]);
    };
    const int nth = std::max(1, std::min<int>(B, (int)std::thread::hardware_concurrency()));
    if (nth == 1) {
        for (int b = 0; b < B; ++b) work(b);
    } else {
        std::atomic<int> next{0};
        std::vector<std::thread> pool;
        for (int t = 0; t < nth; ++t)
            pool.emplace_back([&]() {
                for (int b = next++; b < B; b = next++) work(b);
            });
        for (auto& th : pool) th.join();
    }
    size_t nslots = 0;
    for (int b = 0; b < B; ++b) {
        if (rs[b] < 0) return fail(ctx, PCFV_EINVAL, errs[b]);
        nslots = std::max(nslots, cands[b].size());
    }
    best_cost.assign(B, std::numeric_limits<double>::infinity());
    best_rank.assign(B, 0);
    best_kind.assign(B, -1);
    // fallback: the last snapshot
    PCFV_TRY(launch_unpack(p, ctx->stream, snaps + (size_t)(M - 1) * B * n, dd(u_out)), "unpack");
    std::vector<double> cvec((size_t)B * (M - 1));
    std::vector<double> costs(B);
    for (size_t slot = 0; slot < nslots; ++slot) {
        for (int b = 0; b < B; ++b)
            for (int k = 0; k < M - 1; ++k)
                cvec[(size_t)b * (M - 1) + k] = (slot < cands[b].size()) ? cands[b][slot].coef[k] : 0.0;
        PCFV_TRY(hipMemcpyAsync(ctx->dmdC, cvec.data(), cvec.size() * sizeof(double), hipMemcpyHostToDevice,
                                ctx->stream),
                 "copy coefficients");
        PCFV_TRY(launch_dmd_combine(ctx->stream, snaps, M, B, n, ctx->dmdC, ctx->dmdPsi), "dmd combine");
        PCFV_TRY(launch_unpack(p, ctx->stream, ctx->dmdPsi, ctx->tmp), "unpack");
        PCFV_TRY(launch_synth(p, ctx->stream, ctx->tmp, ctx->Y), "synth");
        pcfv_status st = residual_core(ctx, reinterpret_cast<const double*>(ctx->tmp), nullptr, true);
        if (st != PCFV_OK) return st;
        st = read_scalars(ctx, 1, 0, costs.data());
        if (st != PCFV_OK) return st;
        for (int b = 0; b < B; ++b)
            if (slot < cands[b].size() && std::isfinite(costs[b]) && costs[b] < best_cost[b]) {
                best_cost[b] = costs[b];
                best_rank[b] = cands[b][slot].rank;
                best_kind[b] = cands[b][slot].kind;
                PCFV_TRY(hipMemcpyAsync(u_out + (size_t)b * 3 * p.nm * p.N * 2,
                                        reinterpret_cast<const char*>(ctx->tmp) + b * fbytes1, fbytes1,
                                        hipMemcpyDeviceToDevice, ctx->stream),
                         "copy candidate");
            }
    }
    return PCFV_OK;
}
}  // namespace

extern "C" {

size_t pcfv_workspace_bytes(const pcfv_config* cfg) {
    std::string e;
    if (!validate(cfg, e)) return 0;
    return layout(*cfg).total;
}

pcfv_status pcfv_create(const pcfv_config* cfg, void* hip_stream, void* workspace, pcfv_ctx** out) {
    g_create_err.clear();
    if (!out) {
        g_create_err = "out is NULL";
        return PCFV_EINVAL;
    }
    *out = nullptr;
    std::string e;
    if (!validate(cfg, e)) {
        g_create_err = e;
        return PCFV_EINVAL;
    }
    if (!workspace) {
        g_create_err = "workspace is NULL";
        return PCFV_ENOMEM;
    }
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign) {
        g_create_err = "workspace is not 256-byte aligned";
        return PCFV_EINVAL;
    }
    pcfv_ctx* ctx = new pcfv_ctx();
    ctx->cfg = *cfg;
    ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
    ctx->ws = reinterpret_cast<char*>(workspace);
    if (!build_tables(cfg->Lx, cfg->Lz, cfg->Re, cfg->Nx, cfg->Ny, cfg->Nz, cfg->dt_im, ctx->t, e)) {
        g_create_err = "table construction failed: " + e;
        delete ctx;
        return PCFV_EINVAL;
    }
    ctx->L = layout(*cfg);
    KP p = base_kp(*cfg);
    const Tables& t = ctx->t;
    p.lam = t.lam;
    p.nu = t.nu;
    p.alpha = t.alpha;
    p.beta = t.beta;
    p.M = ctx->at<double>(W_MATS);
    p.minfo = ctx->at<double>(W_MINFO);
    p.dH = ctx->at<double>(W_DH);
    p.dP = ctx->at<double>(W_DP);
    p.dproj = ctx->at<double>(W_DPROJ);
    p.Vk = ctx->at<double>(W_VK);
    p.DVk = ctx->at<double>(W_DVK);
    p.Ainv = ctx->at<double>(W_AINV);
    p.twx = ctx->at<double2>(W_TWX);
    p.twz = ctx->at<double2>(W_TWZ);
    p.ygl = ctx->at<double>(W_YGL);
    p.indep = ctx->at<int>(W_INDEP);
    p.nstate = t.n_state;
    ctx->kp = p;
    ctx->Y = ctx->at<double2>(W_Y);
    ctx->Yv = ctx->at<double2>(W_YV);
    ctx->Atil = ctx->at<double2>(W_ATIL);
    ctx->P3 = ctx->at<double2>(W_P3);
    ctx->P6 = ctx->at<double2>(W_P6);
    ctx->a = ctx->at<double2>(W_A);
    ctx->r = ctx->at<double2>(W_R);
    ctx->ck = ctx->at<double2>(W_CK);
    ctx->tmp = ctx->at<double2>(W_TMP);
    ctx->part = ctx->at<double>(W_PART);
    ctx->scal = ctx->at<double>(W_SCAL);
    ctx->dmdG = ctx->at<double>(W_DMDG);
    ctx->dmdC = ctx->at<double>(W_DMDC);
    ctx->dmdPsi = ctx->at<double>(W_DMDPSI);
    const std::vector<double> pm = padded_mats(t.mats, p.N, p.np);
    struct Up {
        int slot;
        const void* src;
        size_t bytes;
    } ups[] = {
        {W_MATS, pm.data(), pm.size() * 8},           {W_MINFO, t.minfo.data(), t.minfo.size() * 8},
        {W_DH, t.dH.data(), t.dH.size() * 8},         {W_DP, t.dP.data(), t.dP.size() * 8},
        {W_DPROJ, t.dproj.data(), t.dproj.size() * 8}, {W_VK, t.Vk.data(), t.Vk.size() * 8},
        {W_DVK, t.DVk.data(), t.DVk.size() * 8},      {W_AINV, t.Ainv.data(), t.Ainv.size() * 8},
        {W_TWX, t.twx.data(), t.twx.size() * 8},      {W_TWZ, t.twz.data(), t.twz.size() * 8},
        {W_YGL, t.ygl.data(), t.ygl.size() * 8},      {W_INDEP, t.indep.data(), t.indep.size() * 4},
    };
    for (const Up& u : ups) {
        hipError_t he = hipMemcpyAsync(ctx->ws + ctx->L.off[u.slot], u.src, u.bytes, hipMemcpyHostToDevice,
                                       ctx->stream);
        if (he == hipSuccess) he = hipStreamSynchronize(ctx->stream);
        if (he != hipSuccess) {
            g_create_err = std::string("copying tables to the workspace: ") + hipGetErrorString(he);
            delete ctx;
            return PCFV_EDEVICE;
        }
    }
    *out = ctx;
    return PCFV_OK;
}

void pcfv_destroy(pcfv_ctx* ctx) { delete ctx; }

pcfv_status pcfv_get_layout(const pcfv_ctx* ctx, pcfv_layout* out) {
    if (!ctx || !out) return PCFV_EINVAL;
    const KP& p = ctx->kp;
    out->Kx = p.Kx;
    out->Kz = p.Kz;
    out->Ny = p.N;
    out->nkx = p.nkx;
    out->nkz = p.nkz;
    out->n_modes = p.nm;
    out->n_complex = 3LL * p.nm * p.N;
    out->n_state = ctx->t.n_state;
    out->batch = p.B;
    out->stride_kz = p.N;
    out->stride_kx = (long long)p.nkz * p.N;
    out->stride_c = (long long)p.nm * p.N;
    out->stride_b = 3LL * p.nm * p.N;
    return PCFV_OK;
}

pcfv_status pcfv_set_stream(pcfv_ctx* ctx, void* hip_stream) {
    if (!ctx) return PCFV_EINVAL;
    ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return PCFV_OK;
}

pcfv_status pcfv_set_precision(pcfv_ctx* ctx, int precision) {
    if (!ctx) return PCFV_EINVAL;
    if (precision != PCFV_FP64 && precision != PCFV_MIXED)
        return fail(ctx, PCFV_EINVAL, "precision must be PCFV_FP64 (0) or PCFV_MIXED (1)");
    ctx->kp.prec = precision == PCFV_MIXED ? PREC_FP32 : PREC_FP64;
    return PCFV_OK;
}

pcfv_status pcfv_residual(pcfv_ctx* ctx, const double* u, double* r, double* cost_host) {
    if (!ctx || !u) return fail(ctx, PCFV_EINVAL, "NULL argument");
    PCFV_TRY(launch_synth(ctx->kp, ctx->stream, cd(u), ctx->Y), "synth");
    pcfv_status s = residual_core(ctx, u, r, cost_host != nullptr);
    if (s != PCFV_OK || !cost_host) return s;
    return read_scalars(ctx, 1, 0, cost_host);
}

pcfv_status pcfv_cost(pcfv_ctx* ctx, const double* u, double* cost_host) {
    if (!ctx || !u || !cost_host) return fail(ctx, PCFV_EINVAL, "NULL argument");
    return pcfv_residual(ctx, u, nullptr, cost_host);
}

pcfv_status pcfv_jvp(pcfv_ctx* ctx, const double* u, const double* v, double* Jv) {
    if (!ctx || !u || !v || !Jv) return fail(ctx, PCFV_EINVAL, "NULL argument");
    const KP& p = ctx->kp;
    PCFV_TRY(launch_synth(p, ctx->stream, cd(u), ctx->Y), "synth u");
    PCFV_TRY(launch_synth(p, ctx->stream, cd(v), ctx->Yv), "synth v");
    PCFV_TRY(launch_plane(p, ctx->stream, PLANE_JVP, ctx->Y, ctx->Yv, ctx->P3), "plane jvp");
    PCFV_TRY(launch_mode_res(p, ctx->stream, RES_WRITE_R, ctx->P3, cd(v), dd(Jv), ctx->part, nullptr,
                             nullptr),
             "mode res");
    return PCFV_OK;
}

pcfv_status pcfv_adjoint(pcfv_ctx* ctx, const double* u, const double* w, double* out) {
    if (!ctx || !u || !w || !out) return fail(ctx, PCFV_EINVAL, "NULL argument");
    const KP& p = ctx->kp;
    PCFV_TRY(launch_synth(p, ctx->stream, cd(u), ctx->Y), "synth u");
    PCFV_TRY(launch_mode_res(p, ctx->stream, RES_INPUT_W | RES_ADJ, ctx->P3, cd(w), nullptr, ctx->part,
                             ctx->a, ctx->Atil),
             "adjoint solve");
    PCFV_TRY(launch_plane(p, ctx->stream, PLANE_ADJ, ctx->Y, ctx->Atil, ctx->P6), "plane adj");
    PCFV_TRY(launch_mode_grad(p, ctx->stream, 0, ctx->P6, ctx->a, 0.0, dd(out), nullptr), "mode grad");
    return PCFV_OK;
}

pcfv_status pcfv_project(pcfv_ctx* ctx, const double* g, double* Pg) {
    if (!ctx || !g || !Pg) return fail(ctx, PCFV_EINVAL, "NULL argument");
    PCFV_TRY(launch_project(ctx->kp, ctx->stream, cd(g), dd(Pg)), "project");
    return PCFV_OK;
}

pcfv_status pcfv_descend(pcfv_ctx* ctx, double* u, const pcfv_descent_opts* o,
                         pcfv_descent_report* rep) {
    if (!ctx || !u || !o) return fail(ctx, PCFV_EINVAL, "NULL argument");
    if (o->max_steps < 0 || !(o->dtau > 0) || o->check_every < 1 || o->max_halvings < 0 ||
        !(o->rel_tol >= 0))
        return fail(ctx, PCFV_EINVAL, "invalid descent options");
    const bool use_dmd = o->dmd_window > 0;
    if (use_dmd && (o->dmd_window < 3 || o->dmd_window > kMaxDmd || o->dmd_stride < 1 || o->dmd_gap < 0 ||
                    !o->dmd_buffer || !(o->dmd_accept > 0)))
        return fail(ctx, PCFV_EINVAL, "invalid DMD options");
    const KP& p = ctx->kp;
    // the refinement phase switches ctx->kp.prec; every exit restores it
    struct PrecGuard {
        KP& kp;
        int saved;
        ~PrecGuard() { kp.prec = saved; }
    } guard{ctx->kp, ctx->kp.prec};
    const int B = p.B;
    const size_t fbytes = (size_t)ctx->nfield() * 16;
    const size_t fbytes1 = (size_t)3 * p.nm * p.N * 16;
    double dtau = o->dtau, tau = 0;
    long long steps = 0, steps32 = 0;
    // snapshot stride of the current DMD window (grows after weak windows)
    long long stride = o->dmd_stride;
    const bool adaptive = use_dmd && o->dmd_stride_max > o->dmd_stride;
    const double grow_ratio = o->dmd_grow_ratio > 0 ? o->dmd_grow_ratio : 0.5;
    int halvings = 0, n_dmd = 0, n_acc = 0, n_lacc = 0;
    std::vector<double> cost, ntot, cost_prev;
    pcfv_descent_report local{};
    if (!rep) rep = &local;
    auto worst_rel = [&]() {
        double w = 0;
        for (int b = 0; b < B; ++b)
            w = std::max(w, ntot[b] > 0 ? std::sqrt(std::max(cost[b], 0.0)) / ntot[b] : 0.0);
        return w;
    };
    auto max_cost = [&]() { return cost.empty() ? 0.0 : *std::max_element(cost.begin(), cost.end()); };
    auto report = [&](pcfv_status st) {
        rep->steps = steps;
        rep->tau = tau;
        rep->cost = max_cost();
        rep->rel_res = cost.empty() ? 0.0 : worst_rel();
        rep->dtau_final = dtau;
        rep->n_halvings = halvings;
        rep->n_dmd = n_dmd;
        rep->n_dmd_accepted = n_acc;
        rep->steps_fp32 = steps32;
        rep->n_learned_accepted = n_lacc;
        rep->dmd_stride_final = use_dmd ? (int)stride : 0;
        return st;
    };
    // FP32 -> FP64 once every guess is below fp64_below: new y-values and cost
    auto maybe_refine = [&]() -> pcfv_status {
        if (!(o->fp64_below > 0) || ctx->kp.prec != PREC_FP32 || worst_rel() >= o->fp64_below) return PCFV_OK;
        ctx->kp.prec = PREC_FP64;
        PCFV_TRY(launch_synth(p, ctx->stream, cd(u), ctx->Y), "synth");
        pcfv_status st = cost_and_norm(ctx, u, cost, ntot);
        if (st != PCFV_OK) return st;
        cost_prev = cost;
        return PCFV_OK;
    };
    // converged: below rel_tol, and past the FP32 phase if a refinement is asked for
    auto converged = [&]() {
        return o->rel_tol > 0 && worst_rel() < o->rel_tol &&
               (ctx->kp.prec == PREC_FP64 || !(o->fp64_below > 0));
    };
    auto finite = [&]() {
        for (double c : cost)
            if (!std::isfinite(c)) return false;
        return true;
    };
    PCFV_TRY(launch_synth(p, ctx->stream, cd(u), ctx->Y), "synth");
    if (o->no_cost_checks && !(o->rel_tol > 0) && !(o->grow_tol > 0) && !use_dmd && !(o->fp64_below > 0)) {
        // nothing reads the cost: max_steps steps, enqueued without a host sync
        for (; steps < o->max_steps; ++steps) {
            pcfv_status s1 = descent_step(ctx, u, dtau);
            if (s1 != PCFV_OK) return s1;
        }
        tau = steps * dtau;
        if (ctx->kp.prec == PREC_FP32) steps32 = steps;
        report(PCFV_OK);
        rep->cost = rep->rel_res = std::numeric_limits<double>::quiet_NaN();
        return PCFV_OK;
    }
    pcfv_status s = cost_and_norm(ctx, u, cost, ntot);
    if (s != PCFV_OK) return s;
    if (!finite()) return report(fail(ctx, PCFV_ENAN, "cost is not finite"));
    cost_prev = cost;
    s = maybe_refine();
    if (s != PCFV_OK) return s;
    if (converged()) return report(PCFV_OK);
    bool window = false;
    int nsnap = 0;
    long long next_snap = 0, window_start = 0, since_check = 0;
    // checkpoint for the divergence rollback: the state, and the step count,
    // fictitious time and FP32 step count it was taken at
    long long steps_ck = 0, steps32_ck = 0;
    double tau_ck = 0;
    auto checkpoint = [&]() -> pcfv_status {
        steps_ck = steps;
        steps32_ck = steps32;
        tau_ck = tau;
        if (o->grow_tol > 0)
            PCFV_TRY(hipMemcpyAsync(ctx->ck, u, fbytes, hipMemcpyDeviceToDevice, ctx->stream), "checkpoint");
        return PCFV_OK;
    };
    s = checkpoint();
    if (s != PCFV_OK) return s;
    while (steps < o->max_steps) {
        if (use_dmd && !window && steps >= window_start &&
            (o->dmd_start <= 0 || std::sqrt(std::max(max_cost(), 0.0)) < o->dmd_start)) {
            window = true;
            nsnap = 0;
            next_snap = steps;
        }
        if (window && steps == next_snap) {
            PCFV_TRY(launch_pack(p, ctx->stream, cd(u), o->dmd_buffer + (size_t)nsnap * B * p.nstate), "pack");
            ++nsnap;
            next_snap += stride;
            if (nsnap == o->dmd_window) {
                std::vector<double> cnow, nnow, dcost;
                std::vector<int> drank, dkind;
                s = cost_and_norm(ctx, u, cnow, nnow);
                if (s != PCFV_OK) return s;
                double2* cand = ctx->a;   // scratch: recomputed by every step
                s = dmd_core(ctx, o->dmd_buffer, o->dmd_window, stride * dtau,
                             reinterpret_cast<double*>(cand), dcost, drank, dkind);
                if (s != PCFV_OK) return s;
                ++n_dmd;
                std::vector<double> lcost;
                double2* lcand = ctx->r;  // scratch: not written by the steps
                if (o->learned) {
                    const int W = o->learned->window;
                    if (W > o->dmd_window) return report(fail(ctx, PCFV_EINVAL, "learned window exceeds dmd_window"));
                    const double* base = nullptr;
                    if (o->learned->use_base) {   // the DMD candidates (last snapshot where DMD had none)
                        PCFV_TRY(launch_pack(p, ctx->stream, cand, ctx->dmdPsi), "pack");
                        base = ctx->dmdPsi;
                    }
                    s = learned_core(ctx, o->learned, o->dmd_buffer + (size_t)(o->dmd_window - W) * B * p.nstate,
                                     base, reinterpret_cast<double*>(lcand), lcost);
                    if (s != PCFV_OK) return s;
                }
                bool weak = false;   // some guess gained less than grow_ratio
                for (int b = 0; b < B; ++b) {
                    const bool dok = drank[b] > 0 && std::isfinite(dcost[b]);
                    const bool lok = o->learned && std::isfinite(lcost[b]);
                    const bool use_l = lok && (!dok || lcost[b] < dcost[b]);
                    const double best = use_l ? lcost[b] : (dok ? dcost[b] : HUGE_VAL);
                    if (!(best < grow_ratio * cnow[b])) weak = true;
                    if (!(best < o->dmd_accept * cnow[b])) continue;
                    const double2* src = use_l ? lcand : cand;
                    PCFV_TRY(hipMemcpyAsync(reinterpret_cast<char*>(u) + b * fbytes1,
                                            reinterpret_cast<const char*>(src) + b * fbytes1, fbytes1,
                                            hipMemcpyDeviceToDevice, ctx->stream),
                             "accept");
                    ++n_acc;
                    if (use_l) ++n_lacc;
                }
                PCFV_TRY(launch_synth(p, ctx->stream, cd(u), ctx->Y), "synth");
                s = cost_and_norm(ctx, u, cost, ntot);
                if (s != PCFV_OK) return s;
                cost_prev = cost;
                s = maybe_refine();
                if (s != PCFV_OK) return s;
                s = checkpoint();
                if (s != PCFV_OK) return s;
                window = false;
                window_start = steps + o->dmd_gap;
                if (adaptive && weak) stride = std::min<long long>(4 * stride, o->dmd_stride_max);
                since_check = 0;
                if (converged()) return report(PCFV_OK);
                continue;
            }
        }
        long long k = std::min<long long>(o->check_every - since_check, o->max_steps - steps);
        if (window) k = std::min<long long>(k, next_snap - steps);
        for (long long i = 0; i < k; ++i) {
            s = descent_step(ctx, u, dtau);
            if (s != PCFV_OK) return s;
        }
        if (ctx->kp.prec == PREC_FP32) steps32 += k;
        steps += k;
        tau += k * dtau;
        since_check += k;
        if (since_check < o->check_every && steps < o->max_steps) continue;
        since_check = 0;
        s = cost_and_norm(ctx, u, cost, ntot);
        if (s != PCFV_OK) return s;
        if (!finite()) return report(fail(ctx, PCFV_ENAN, "cost is not finite"));
        bool grew = false;
        for (int b = 0; b < B; ++b) grew |= (o->grow_tol > 0 && cost[b] > o->grow_tol * cost_prev[b]);
        if (grew) {
            // back to the last checkpoint: state, steps, fictitious time
            PCFV_TRY(hipMemcpyAsync(u, ctx->ck, fbytes, hipMemcpyDeviceToDevice, ctx->stream), "restore");
            cost = cost_prev;
            steps = steps_ck;
            steps32 = steps32_ck;
            tau = tau_ck;
            window = false;
            if (halvings >= o->max_halvings) {
                PCFV_TRY(hipStreamSynchronize(ctx->stream), "synchronize");
                return report(fail(ctx, PCFV_EDIVERGED, "cost grew beyond grow_tol"));
            }
            PCFV_TRY(launch_synth(p, ctx->stream, cd(u), ctx->Y), "synth");
            dtau *= 0.5;
            ++halvings;
            continue;
        }
        cost_prev = cost;
        s = maybe_refine();
        if (s != PCFV_OK) return s;
        s = checkpoint();
        if (s != PCFV_OK) return s;
        if (converged()) return report(PCFV_OK);
    }
    return report(o->rel_tol > 0 ? fail(ctx, PCFV_ENOTCONV, "max_steps reached above rel_tol") : PCFV_OK);
}

pcfv_status pcfv_dmd_extrapolate(pcfv_ctx* ctx, const double* snaps, int M, double dtau_snap,
                                 double* u_out, double* cost_host, int* rank_host, int* kind_host) {
    if (!ctx || !snaps || !u_out) return fail(ctx, PCFV_EINVAL, "NULL argument");
    std::vector<double> cost;
    std::vector<int> rank, kind;
    pcfv_status s = dmd_core(ctx, snaps, M, dtau_snap, u_out, cost, rank, kind);
    if (s != PCFV_OK) return s;
    for (int b = 0; b < ctx->kp.B; ++b) {
        if (cost_host) cost_host[b] = cost[b];
        if (rank_host) rank_host[b] = rank[b];
        if (kind_host) kind_host[b] = kind[b];
    }
    PCFV_TRY(hipStreamSynchronize(ctx->stream), "synchronize");
    return PCFV_OK;
}

pcfv_status pcfv_norms(pcfv_ctx* ctx, const double* u, double* out_host) {
    if (!ctx || !u || !out_host) return fail(ctx, PCFV_EINVAL, "NULL argument");
    PCFV_TRY(launch_norms(ctx->kp, ctx->stream, cd(u), ctx->part), "norms");
    pcfv_status s = read_scalars(ctx, 3, 0, out_host);
    if (s != PCFV_OK) return s;
    for (int b = 0; b < ctx->kp.B; ++b) {
        out_host[3 * b] = std::sqrt(std::max(out_host[3 * b], 0.0));
        out_host[3 * b + 1] = std::sqrt(std::max(out_host[3 * b + 1], 0.0));
    }
    return PCFV_OK;
}

pcfv_status pcfv_pack_state(pcfv_ctx* ctx, const double* u, double* psi) {
    if (!ctx || !u || !psi) return fail(ctx, PCFV_EINVAL, "NULL argument");
    PCFV_TRY(launch_pack(ctx->kp, ctx->stream, cd(u), psi), "pack");
    return PCFV_OK;
}

pcfv_status pcfv_unpack_state(pcfv_ctx* ctx, const double* psi, double* u) {
    if (!ctx || !u || !psi) return fail(ctx, PCFV_EINVAL, "NULL argument");
    PCFV_TRY(launch_unpack(ctx->kp, ctx->stream, psi, dd(u)), "unpack");
    return PCFV_OK;
}

pcfv_status pcfv_check_state(pcfv_ctx* ctx, const double* u, double* defects_host) {
    if (!ctx || !u || !defects_host) return fail(ctx, PCFV_EINVAL, "NULL argument");
    PCFV_TRY(launch_check(ctx->kp, ctx->stream, cd(u), ctx->part), "check");
    return read_scalars(ctx, 3, 1, defects_host);
}

pcfv_status pcfv_time_kernels(pcfv_ctx* ctx, const double* u, int nrep, double* ms_out, int* n_out) {
    if (!ctx || !u || !ms_out || nrep < 1) return fail(ctx, PCFV_EINVAL, "bad argument");
    const KP& p = ctx->kp;
    hipStream_t s = ctx->stream;
    const size_t fbytes = (size_t)ctx->nfield() * 16;
    PCFV_TRY(hipMemcpyAsync(ctx->tmp, u, fbytes, hipMemcpyDeviceToDevice, s), "copy");
    PCFV_TRY(launch_synth(p, s, ctx->tmp, ctx->Y), "synth");
    PCFV_TRY(launch_plane(p, s, PLANE_FWD, ctx->Y, nullptr, ctx->P3), "plane fwd");
    PCFV_TRY(launch_mode_res(p, s, RES_COST | RES_ADJ, ctx->P3, ctx->tmp, nullptr, ctx->part, ctx->a,
                             ctx->Atil),
             "mode res");
    hipEvent_t e0, e1;
    PCFV_TRY(hipEventCreate(&e0), "event");
    PCFV_TRY(hipEventCreate(&e1), "event");
    for (int k = 0; k < 5; ++k) {
        PCFV_TRY(hipEventRecord(e0, s), "record");
        for (int i = 0; i < nrep; ++i) {
            hipError_t he = hipSuccess;
            switch (k) {
                case 0: he = launch_synth(p, s, ctx->tmp, ctx->Yv); break;
                case 1: he = launch_plane(p, s, PLANE_FWD, ctx->Y, nullptr, ctx->P3); break;
                case 2:
                    he = launch_mode_res(p, s, RES_COST | RES_ADJ, ctx->P3, ctx->tmp, nullptr, ctx->part,
                                         ctx->a, ctx->Atil);
                    break;
                case 3: he = launch_plane(p, s, PLANE_ADJ, ctx->Y, ctx->Atil, ctx->P6); break;
                case 4:
                    he = launch_mode_grad(p, s, GRAD_PROJECT | GRAD_UPDATE, ctx->P6, ctx->a, 0.0, ctx->tmp,
                                          ctx->Yv);
                    break;
            }
            PCFV_TRY(he, "launch");
        }
        PCFV_TRY(hipEventRecord(e1, s), "record");
        PCFV_TRY(hipEventSynchronize(e1), "event sync");
        float ms = 0;
        PCFV_TRY(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        ms_out[k] = ms / nrep;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (n_out) *n_out = 5;
    return PCFV_OK;
}

pcfv_status pcfv_time_descent_kernels(pcfv_ctx* ctx, double* u, double dtau, int nsteps, double* ms_out) {
    if (!ctx || !u || !ms_out || nsteps < 1 || nsteps > 4096) return fail(ctx, PCFV_EINVAL, "bad argument");
    const KP& p = ctx->kp;
    hipStream_t s = ctx->stream;
    std::vector<hipEvent_t> ev((size_t)nsteps * 5, nullptr);
    pcfv_status st = PCFV_OK;
    auto cleanup = [&]() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    for (hipEvent_t& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            cleanup();
            return fail(ctx, PCFV_EDEVICE, "event creation failed");
        }
    hipError_t he = launch_synth(p, s, cd(u), ctx->Y);
    for (int i = 0; i < nsteps && he == hipSuccess; ++i) {   // the kernels of descent_step, bracketed
        hipEvent_t* e = &ev[(size_t)i * 5];
        he = hipEventRecord(e[0], s);
        if (he == hipSuccess) he = launch_plane(p, s, PLANE_FWD, ctx->Y, nullptr, ctx->P3);
        if (he == hipSuccess) he = hipEventRecord(e[1], s);
        if (he == hipSuccess)
            he = launch_mode_res(p, s, RES_COST | RES_ADJ, ctx->P3, cd(u), nullptr, ctx->part, ctx->a, ctx->Atil);
        if (he == hipSuccess) he = hipEventRecord(e[2], s);
        if (he == hipSuccess) he = launch_plane(p, s, PLANE_ADJ, ctx->Y, ctx->Atil, ctx->P6);
        if (he == hipSuccess) he = hipEventRecord(e[3], s);
        if (he == hipSuccess) he = launch_mode_grad(p, s, GRAD_PROJECT | GRAD_UPDATE, ctx->P6, ctx->a, dtau, dd(u), ctx->Y);
        if (he == hipSuccess) he = hipEventRecord(e[4], s);
    }
    if (he == hipSuccess) he = hipEventSynchronize(ev.back());
    double acc[4] = {0, 0, 0, 0};
    for (int i = 0; i < nsteps && he == hipSuccess; ++i)
        for (int k = 0; k < 4 && he == hipSuccess; ++k) {
            float ms = 0;
            he = hipEventElapsedTime(&ms, ev[(size_t)i * 5 + k], ev[(size_t)i * 5 + k + 1]);
            acc[k] += ms;
        }
    cleanup();
    if (he != hipSuccess) st = hip_check(ctx, he, "timed descent");
    if (st != PCFV_OK) return st;
    for (int k = 0; k < 4; ++k) ms_out[k] = acc[k] / nsteps;
    return PCFV_OK;
}

const char* pcfv_last_error(const pcfv_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

pcfv_status pcfv_autotune(pcfv_ctx* ctx, const double* u, int steps, pcfv_tune_entry* entries, int cap,
                          int* n_entries) {
    if (!ctx || !u || steps < 1) return fail(ctx, PCFV_EINVAL, "invalid autotune arguments");
    const size_t fbytes = (size_t)ctx->nfield() * 16;
    const KP saved = ctx->kp;
    std::vector<pcfv_tune_entry> res;
    hipEvent_t e0, e1;
    PCFV_TRY(hipEventCreate(&e0), "event");
    PCFV_TRY(hipEventCreate(&e1), "event");
    double best = std::numeric_limits<double>::infinity();
    KP best_kp = saved;
    pcfv_status st = PCFV_OK;
    for (int xs : xs_candidates(ctx->cfg)) {
        static const int kPlaneThreads[] = {256, 512, 576, 768, 1024};
        for (int cand = 0; cand < 10; ++cand) {
            const int nt = kPlaneThreads[cand % 5], mt = (cand < 5) ? 256 : 512;
            ctx->kp.XS = xs;
            ctx->kp.NS = ctx->cfg.Nx / xs;
            ctx->kp.pthreads = nt;
            ctx->kp.mthreads = mt;
            hipError_t he = hipMemcpyAsync(ctx->tmp, u, fbytes, hipMemcpyDeviceToDevice, ctx->stream);
            if (he == hipSuccess) he = launch_synth(ctx->kp, ctx->stream, ctx->tmp, ctx->Y);
            // one untimed step, then `steps` timed ones (dtau = 0 leaves the copy unchanged)
            for (int i = 0; i <= steps && st == PCFV_OK && he == hipSuccess; ++i) {
                if (i == 1) he = hipEventRecord(e0, ctx->stream);
                if (he == hipSuccess) st = descent_step(ctx, reinterpret_cast<double*>(ctx->tmp), 0.0);
            }
            if (he == hipSuccess) he = hipEventRecord(e1, ctx->stream);
            if (he == hipSuccess) he = hipEventSynchronize(e1);
            float ms = 0;
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            if (he != hipSuccess) st = hip_check(ctx, he, "autotune");
            if (st != PCFV_OK) break;
            pcfv_tune_entry t{xs, nt, mt, ms / steps};
            res.push_back(t);
            if (t.ms_per_step < best) {
                best = t.ms_per_step;
                best_kp = ctx->kp;
            }
        }
        if (st != PCFV_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->kp = (st == PCFV_OK) ? best_kp : saved;
    if (st != PCFV_OK) return st;
    if (n_entries) *n_entries = (int)res.size();
    for (int i = 0; entries && i < (int)res.size() && i < cap; ++i) entries[i] = res[i];
    return PCFV_OK;
}

pcfv_status pcfv_set_tuning(pcfv_ctx* ctx, int xs, int plane_threads, int mode_threads) {
    if (!ctx) return PCFV_EINVAL;
    const std::vector<int> xsc = xs_candidates(ctx->cfg);
    if (std::find(xsc.begin(), xsc.end(), xs) == xsc.end())
        return fail(ctx, PCFV_EINVAL, "slab width is not one of the candidates");
    if (plane_threads != 256 && plane_threads != 512 && plane_threads != 576 && plane_threads != 768 &&
        plane_threads != 1024)
        return fail(ctx, PCFV_EINVAL, "plane_threads must be 256, 512, 576, 768 or 1024");
    if (mode_threads != 256 && mode_threads != 512) return fail(ctx, PCFV_EINVAL, "mode_threads must be 256 or 512");
    ctx->kp.XS = xs;
    ctx->kp.NS = ctx->cfg.Nx / xs;
    ctx->kp.pthreads = plane_threads;
    ctx->kp.mthreads = mode_threads;
    return PCFV_OK;
}

pcfv_status pcfv_get_tuning(const pcfv_ctx* ctx, int* xs, int* plane_threads, int* mode_threads) {
    if (!ctx) return PCFV_EINVAL;
    if (xs) *xs = ctx->kp.XS;
    if (plane_threads) *plane_threads = ctx->kp.pthreads;
    if (mode_threads) *mode_threads = ctx->kp.mthreads;
    return PCFV_OK;
}

// ---------------------------------------------------------------------------
// Groups: several contexts advanced by one launch per stage
// ---------------------------------------------------------------------------

struct pcfv_group {
    std::vector<pcfv_ctx*> members;
    int prec0 = PREC_FP64;             // the members' precision at creation
    std::vector<GroupMember> base;     // per-member records (tables at the group's np)
    GroupMember* dev[2] = {nullptr, nullptr};   // device records per precision (n + 1 each), in the workspace
    std::vector<GroupMember> host[2];
    GroupLaunch gl[2]{};
    hipStream_t stream = nullptr;      // the caller's
    int graph_steps = 0;               // steps captured in `exec` (0: none)
    hipGraphExec_t exec = nullptr;
    std::string err;
};

namespace {

pcfv_status gfail(pcfv_group* g, pcfv_status s, const std::string& msg) {
    if (g) g->err = msg;
    return s;
}

#define PCFV_TRY_G(expr, what) PCFV_GTRY(expr, what)

#define PCFV_GTRY(expr, what)                                                                  \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess) return gfail(g, PCFV_EDEVICE, std::string(what) + ": " + hipGetErrorString(_e)); \
    } while (0)

// Workspace of a group: two record arrays of n + 1 entries (FP32 and FP64
// subsets), then the fixed matrices of every member whose padded Ny differs
// from the group's, re-padded to the group's.
struct GroupWs {
    size_t rec[2], mats_at, total;
    std::vector<size_t> mats;   // per member: offset, or SIZE_MAX if none
    int np, pthreads, mthreads;
    bool many;
};

bool group_ws(pcfv_ctx* const* m, int n, GroupWs& L, std::string& e) {
    if (!m || n < 1) {
        e = "invalid group arguments";
        return false;
    }
    for (int k = 0; k < n; ++k)
        if (!m[k] || m[k]->kp.prec != m[0]->kp.prec) {
            e = "group members must be non-NULL and share one precision";
            return false;
        }
    long long group_modes = 0;
    L.np = 0;
    for (int k = 0; k < n; ++k) {
        group_modes += m[k]->kp.nmB;
        L.np = std::max(L.np, m[k]->kp.np);
    }
    L.many = group_modes > 1024;
    L.pthreads = L.many ? plane_threads_default(m[0]->kp.prec, group_modes)   // the single-context default
                        : m[0]->kp.pthreads;                                   // for many modes
    L.mthreads = m[0]->kp.mthreads;
    size_t o = 0;
    for (int p = 0; p < 2; ++p) {
        L.rec[p] = o;
        o += up(sizeof(GroupMember) * (n + 1));
    }
    L.mats_at = o;
    L.mats.assign(n, SIZE_MAX);
    for (int k = 0; k < n; ++k)
        if (m[k]->kp.np != L.np) {
            L.mats[k] = o;
            o += up((size_t)M_COUNT * L.np * mat_ld(L.np) * 8);
        }
    L.total = o;
    return true;
}

// Device records of the members idx in precision prec (sentinel last).
pcfv_status upload_records(pcfv_group* g, int prec, const std::vector<int>& idx, double* const* u,
                           const double* dtau) {
    const int slot = (prec == PREC_FP32) ? 0 : 1;
    GroupLaunch& gl = g->gl[slot];
    std::vector<GroupMember>& host = g->host[slot];
    host.assign(idx.size() + 1, GroupMember{});
    long long items[2] = {0, 0};
    for (size_t i = 0; i < idx.size(); ++i) {
        GroupMember m = g->base[idx[i]];
        m.kp.prec = prec;
        m.item0[GPH_PLANE] = (int)items[GPH_PLANE];
        m.item0[GPH_MODE] = (int)items[GPH_MODE];
        items[GPH_PLANE] += (long long)m.kp.B * m.kp.NS * m.kp.N;
        items[GPH_MODE] += m.kp.nmB;
        m.u = dd(u[idx[i]]);
        m.dtau = dtau[idx[i]];
        host[i] = m;
    }
    if (items[0] > INT_MAX / 2 || items[1] > INT_MAX / 2) return gfail(g, PCFV_EINVAL, "group too large");
    host.back().item0[GPH_PLANE] = (int)items[GPH_PLANE];
    host.back().item0[GPH_MODE] = (int)items[GPH_MODE];
    gl.n = (int)idx.size();
    gl.prec = prec;
    gl.items[GPH_PLANE] = (int)items[GPH_PLANE];
    gl.items[GPH_MODE] = (int)items[GPH_MODE];
    gl.gm = g->dev[slot];
    PCFV_GTRY(hipMemcpyAsync(g->dev[slot], host.data(), sizeof(GroupMember) * host.size(), hipMemcpyHostToDevice,
                             g->stream),
              "member records");
    return PCFV_OK;
}

pcfv_status group_launch(pcfv_group* g, int slot, int which) {
    if (g->gl[slot].n == 0) return PCFV_OK;
    PCFV_GTRY(launch_group(g->gl[slot], g->stream, which), "grouped launch");
    return PCFV_OK;
}

// One descent step of every member in the record sets of both precisions.
pcfv_status group_step(pcfv_group* g) {
    for (int k : {GK_PLANE_FWD, GK_MODE_RES, GK_PLANE_ADJ, GK_MODE_GRAD})
        for (int slot = 0; slot < 2; ++slot) {
            pcfv_status st = group_launch(g, slot, k);
            if (st != PCFV_OK) return st;
        }
    return PCFV_OK;
}

void drop_graph(pcfv_group* g) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    g->exec = nullptr;
    g->graph_steps = 0;
}

pcfv_status capture(pcfv_group* g, int nsteps) {
    drop_graph(g);
    PCFV_GTRY(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    pcfv_status st = PCFV_OK;
    for (int i = 0; i < nsteps && st == PCFV_OK; ++i) st = group_step(g);
    hipGraph_t graph = nullptr;
    hipError_t he = hipStreamEndCapture(g->stream, &graph);
    if (st != PCFV_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    PCFV_GTRY(he, "end capture");
    he = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    PCFV_GTRY(he, "instantiate graph");
    g->graph_steps = nsteps;
    return PCFV_OK;
}

// Host-side wait for the members' own streams (their fields may still be
// being written there) before group launches on the group's stream.
pcfv_status wait_members(pcfv_group* g) {
    for (pcfv_ctx* c : g->members)
        if (c->stream != g->stream) PCFV_GTRY(hipStreamSynchronize(c->stream), "member stream");
    return PCFV_OK;
}

}  // namespace

size_t pcfv_group_workspace_bytes(pcfv_ctx* const* members, int n) {
    GroupWs L;
    std::string e;
    return group_ws(members, n, L, e) ? L.total : 0;
}

pcfv_status pcfv_group_create(pcfv_ctx* const* members, int n, void* hip_stream, void* workspace,
                              pcfv_group** out) {
    g_create_err.clear();
    if (!out) {
        g_create_err = "out is NULL";
        return PCFV_EINVAL;
    }
    *out = nullptr;
    GroupWs L;
    if (!group_ws(members, n, L, g_create_err)) return PCFV_EINVAL;
    if (!workspace) {
        g_create_err = "workspace is NULL";
        return PCFV_ENOMEM;
    }
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign) {
        g_create_err = "workspace is not 256-byte aligned";
        return PCFV_EINVAL;
    }
    pcfv_group* g = new pcfv_group();
    char* ws = reinterpret_cast<char*>(workspace);
    g->members.assign(members, members + n);
    g->prec0 = members[0]->kp.prec;
    g->stream = reinterpret_cast<hipStream_t>(hip_stream);
    g->dev[0] = reinterpret_cast<GroupMember*>(ws + L.rec[0]);
    g->dev[1] = reinterpret_cast<GroupMember*>(ws + L.rec[1]);
    g->base.resize(n);
    for (int slot = 0; slot < 2; ++slot) {
        GroupLaunch& gl = g->gl[slot];
        gl.n = 0;
        gl.np = L.np;
        gl.pthreads = L.pthreads;
        gl.mthreads = L.mthreads;
    }
    for (int k = 0; k < n; ++k) {
        pcfv_ctx* c = members[k];
        GroupMember& m = g->base[k];
        m = GroupMember{};
        m.kp = c->kp;
        m.kp.pthreads = L.pthreads;
        m.kp.mthreads = L.mthreads;
        if (L.mats[k] != SIZE_MAX) {   // the per-mode kernels read the tables at the group's stride
            const std::vector<double> pm = padded_mats(c->t.mats, c->kp.N, L.np);
            double* d = reinterpret_cast<double*>(ws + L.mats[k]);
            hipError_t he = hipMemcpy(d, pm.data(), pm.size() * 8, hipMemcpyHostToDevice);
            if (he != hipSuccess) {
                g_create_err = std::string("group setup: ") + hipGetErrorString(he);
                delete g;
                return PCFV_EDEVICE;
            }
            m.kp.M = d;
        }
        m.kp.np = L.np;
        if (L.many) {
            // a throughput launch: the widest slab of the member's candidates
            // (the single-context default for many modes; every candidate's
            // partial buffers fit)
            m.kp.XS = xs_candidates(c->cfg).front();   // descending
            m.kp.NS = c->cfg.Nx / m.kp.XS;
        }
        m.Y = c->Y;
        m.P3 = c->P3;
        m.P6 = c->P6;
        m.Atil = c->Atil;
        m.a = c->a;
        m.part = c->part;
        for (int slot = 0; slot < 2; ++slot) {
            KP kp = m.kp;
            kp.prec = slot ? PREC_FP64 : PREC_FP32;
            for (int md : {PLANE_FWD, PLANE_JVP, PLANE_ADJ})
                g->gl[slot].plane_lds[md] = std::max(g->gl[slot].plane_lds[md], plane_lds_bytes(kp, md));
            g->gl[slot].mode_lds = std::max(g->gl[slot].mode_lds, mode_lds_bytes(kp));
        }
    }
    *out = g;
    return PCFV_OK;
}

void pcfv_group_destroy(pcfv_group* g) {
    if (!g) return;
    drop_graph(g);
    delete g;
}

pcfv_status pcfv_group_set_stream(pcfv_group* g, void* hip_stream) {
    if (!g) return PCFV_EINVAL;
    drop_graph(g);
    g->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return PCFV_OK;
}

pcfv_status pcfv_group_descend(pcfv_group* g, double* const* u, const double* dtau, long long steps,
                               int graph_steps) {
    if (!g || !u || !dtau || steps < 0 || graph_steps < 0) return gfail(g, PCFV_EINVAL, "invalid arguments");
    const int n = (int)g->members.size();
    for (int k = 0; k < n; ++k)
        if (!u[k] || !std::isfinite(dtau[k])) return gfail(g, PCFV_EINVAL, "NULL field or non-finite dtau");
    if (graph_steps > 0 && !g->stream)
        return gfail(g, PCFV_EINVAL, "graph capture needs a stream other than the null stream");
    pcfv_status st = wait_members(g);
    if (st != PCFV_OK) return st;
    std::vector<int> all(n);
    for (int k = 0; k < n; ++k) all[k] = k;
    const int slot = (g->prec0 == PREC_FP32) ? 0 : 1;
    g->gl[1 - slot].n = 0;
    st = upload_records(g, g->prec0, all, u, dtau);
    if (st != PCFV_OK) return st;
    st = group_launch(g, slot, GK_SYNTH);
    if (st != PCFV_OK) return st;
    long long done = 0;
    if (graph_steps > 0 && steps >= graph_steps) {
        if (g->graph_steps != graph_steps) {
            st = capture(g, graph_steps);
            if (st != PCFV_OK) return st;
        }
        for (; done + graph_steps <= steps; done += graph_steps)
            PCFV_GTRY(hipGraphLaunch(g->exec, g->stream), "graph launch");
    }
    for (; done < steps; ++done) {
        st = group_step(g);
        if (st != PCFV_OK) return st;
    }
    PCFV_GTRY(hipStreamSynchronize(g->stream), "synchronize");
    return PCFV_OK;
}

pcfv_status pcfv_group_descend_tol(pcfv_group* g, double* const* u, const double* dtau,
                                   const pcfv_group_opts* o, pcfv_descent_report* reports, int* status) {
    if (!g || !u || !dtau || !o || !reports || !status) return gfail(g, PCFV_EINVAL, "NULL argument");
    const int n = (int)g->members.size();
    if (o->max_steps < 0 || o->check_every < 1 || !(o->rel_tol > 0))
        return gfail(g, PCFV_EINVAL, "invalid options (max_steps >= 0, check_every >= 1, rel_tol > 0)");
    const bool use_dmd = o->dmd_window > 0;
    if (use_dmd && (o->dmd_window < 3 || o->dmd_window > kMaxDmd || o->dmd_stride < 1 || !(o->dmd_accept > 0) ||
                    !o->dmd_buffers))
        return gfail(g, PCFV_EINVAL, "invalid DMD options");
    for (int k = 0; k < n; ++k) {
        if (!u[k] || !(dtau[k] > 0)) return gfail(g, PCFV_EINVAL, "NULL field or non-positive dtau");
        if (use_dmd && !o->dmd_buffers[k]) return gfail(g, PCFV_EINVAL, "NULL DMD buffer");
    }
    drop_graph(g);   // the records change below; a captured graph would replay stale ones
    // every exit puts the members back in the group's precision
    struct PrecRestore {
        pcfv_group* g;
        ~PrecRestore() {
            for (pcfv_ctx* c : g->members) c->kp.prec = g->prec0;
        }
    } restore{g};
    pcfv_status st = wait_members(g);
    if (st != PCFV_OK) return st;
    std::vector<int> prec(n, g->prec0), active(n, 1), nsnap(n, 0), stat(n, PCFV_ENOTCONV);
    std::vector<long long> steps(n, 0), steps32(n, 0);
    std::vector<double> cost(n, 0), rel(n, 0);
    std::vector<int> ndmd(n, 0), nacc(n, 0);
    auto measure = [&](int k) -> pcfv_status {   // member k's J^2 and relative residual (y-values current)
        pcfv_ctx* c = g->members[k];
        std::vector<double> ck, nk;
        pcfv_status s2 = cost_and_norm(c, u[k], ck, nk);
        if (s2 != PCFV_OK) return gfail(g, s2, c->err);
        double cw = 0, rw = 0;
        bool finite = true;
        for (size_t b = 0; b < ck.size(); ++b) {
            finite &= std::isfinite(ck[b]);
            cw = std::max(cw, ck[b]);
            rw = std::max(rw, nk[b] > 0 ? std::sqrt(std::max(ck[b], 0.0)) / nk[b] : 0.0);
        }
        cost[k] = finite ? cw : NAN;
        rel[k] = finite ? rw : NAN;
        return PCFV_OK;
    };
    // y-values of every member in its precision, then the first check
    for (int k = 0; k < n; ++k) {
        pcfv_ctx* c = g->members[k];
        c->kp.prec = prec[k];
        PCFV_TRY_G(launch_synth(c->kp, c->stream, cd(u[k]), c->Y), "synth");
        st = measure(k);
        if (st != PCFV_OK) return st;
    }
    long long done = 0;
    for (;;) {
        // members' phase changes: converged, failed, FP32 -> FP64 refinement
        bool changed = false;
        for (int k = 0; k < n; ++k) {
            if (!active[k]) continue;
            pcfv_ctx* c = g->members[k];
            if (!std::isfinite(cost[k])) {
                active[k] = 0;
                stat[k] = PCFV_ENAN;
                changed = true;
                continue;
            }
            if (prec[k] == PREC_FP32 && o->fp64_below > 0 && rel[k] < o->fp64_below) {
                prec[k] = PREC_FP64;
                c->kp.prec = PREC_FP64;
                PCFV_TRY_G(launch_synth(c->kp, c->stream, cd(u[k]), c->Y), "synth");
                st = measure(k);
                if (st != PCFV_OK) return st;
                nsnap[k] = 0;   // a DMD window does not straddle the switch
                changed = true;
            }
            const bool refined = prec[k] == PREC_FP64 || !(o->fp64_below > 0);
            if (rel[k] < o->rel_tol && refined) {
                active[k] = 0;
                stat[k] = PCFV_OK;
                changed = true;
            }
        }
        if (done >= o->max_steps) break;
        std::vector<int> subset[2];
        for (int k = 0; k < n; ++k)
            if (active[k]) subset[prec[k] == PREC_FP32 ? 0 : 1].push_back(k);
        if (subset[0].empty() && subset[1].empty()) break;
        (void)changed;
        for (pcfv_ctx* c : g->members)
            if (c->stream != g->stream) PCFV_GTRY(hipStreamSynchronize(c->stream), "member stream");
        for (int slot = 0; slot < 2; ++slot) {
            g->gl[slot].n = 0;
            if (!subset[slot].empty()) {
                st = upload_records(g, slot ? PREC_FP64 : PREC_FP32, subset[slot], u, dtau);
                if (st != PCFV_OK) return st;
            }
        }
        // steps until the next check or snapshot
        long long kmax = std::min<long long>(o->check_every, o->max_steps - done);
        const long long stride = use_dmd ? o->dmd_stride : LLONG_MAX;
        if (use_dmd) kmax = std::min<long long>(kmax, stride - done % stride);
        for (long long i = 0; i < kmax; ++i) {
            st = group_step(g);
            if (st != PCFV_OK) return st;
        }
        done += kmax;
        for (int k = 0; k < n; ++k)
            if (active[k]) {
                steps[k] += kmax;
                if (prec[k] == PREC_FP32) steps32[k] += kmax;
            }
        PCFV_GTRY(hipStreamSynchronize(g->stream), "synchronize");
        // snapshots and DMD windows (per member, on its own stream)
        if (use_dmd && done % stride == 0) {
            for (int k = 0; k < n; ++k) {
                if (!active[k]) continue;
                pcfv_ctx* c = g->members[k];
                const long long ns = c->kp.nstate * c->kp.B;
                PCFV_TRY_G(launch_pack(c->kp, c->stream, cd(u[k]), o->dmd_buffers[k] + (size_t)nsnap[k] * ns), "pack");
                if (++nsnap[k] < o->dmd_window) continue;
                nsnap[k] = 0;
                std::vector<double> cnow, nnow, dcost;
                std::vector<int> drank, dkind;
                st = cost_and_norm(c, u[k], cnow, nnow);
                if (st != PCFV_OK) return gfail(g, st, c->err);
                st = dmd_core(c, o->dmd_buffers[k], o->dmd_window, o->dmd_stride * dtau[k],
                              reinterpret_cast<double*>(c->a), dcost, drank, dkind);
                if (st != PCFV_OK) return gfail(g, st, c->err);
                ++ndmd[k];
                const size_t fb1 = (size_t)3 * c->kp.nm * c->kp.N * 16;
                for (int b = 0; b < c->kp.B; ++b)
                    if (drank[b] > 0 && std::isfinite(dcost[b]) && dcost[b] < o->dmd_accept * cnow[b]) {
                        PCFV_TRY_G(hipMemcpyAsync(reinterpret_cast<char*>(u[k]) + b * fb1,
                                                  reinterpret_cast<const char*>(c->a) + b * fb1, fb1,
                                                  hipMemcpyDeviceToDevice, c->stream),
                                   "accept");
                        ++nacc[k];
                    }
                PCFV_TRY_G(launch_synth(c->kp, c->stream, cd(u[k]), c->Y), "synth");
            }
        }
        if (done % o->check_every == 0 || done >= o->max_steps)
            for (int k = 0; k < n; ++k)
                if (active[k]) {
                    st = measure(k);
                    if (st != PCFV_OK) return st;
                }
    }
    for (pcfv_ctx* c : g->members) PCFV_GTRY(hipStreamSynchronize(c->stream), "member stream");
    pcfv_status worst = PCFV_OK;
    for (int k = 0; k < n; ++k) {
        pcfv_descent_report& r = reports[k];
        r = pcfv_descent_report{};
        r.steps = steps[k];
        r.tau = steps[k] * dtau[k];
        r.cost = cost[k];
        r.rel_res = rel[k];
        r.dtau_final = dtau[k];
        r.n_dmd = ndmd[k];
        r.n_dmd_accepted = nacc[k];
        r.steps_fp32 = steps32[k];
        status[k] = stat[k];
        if (stat[k] == PCFV_ENAN || (stat[k] != PCFV_OK && worst == PCFV_OK)) worst = (pcfv_status)stat[k];
    }
    return worst;
}

const char* pcfv_group_last_error(const pcfv_group* g) { return g ? g->err.c_str() : g_create_err.c_str(); }

size_t pcfv_learned_scratch_bytes(const pcfv_ctx* ctx, int window, int r) {
    if (!ctx || window < 1 || r < 1) return 0;
    return learned_scratch(ctx->kp, window, r).total;
}

pcfv_status pcfv_learned_propose(pcfv_ctx* ctx, const pcfv_learned_model* model, const double* snaps,
                                 const double* base, double* u_out, double* cost_host) {
    if (!ctx || !model || !snaps || !u_out) return fail(ctx, PCFV_EINVAL, "NULL argument");
    std::vector<double> cost;
    pcfv_status s = learned_core(ctx, model, snaps, base, u_out, cost);
    if (s != PCFV_OK) return s;
    if (cost_host)
        for (int b = 0; b < ctx->kp.B; ++b) cost_host[b] = cost[b];
    return PCFV_OK;
}

int pcfv_host_dmd(const double* Ge_hi, const double* Ge_lo, int M, double dtau, double* coef, int* labels,
                  int cap) {
    if (!Ge_hi || M < 3 || M > kMaxDmd || cap < 0) return -1;
    std::vector<long double> G((size_t)M * M);
    for (size_t k = 0; k < G.size(); ++k)
        G[k] = (long double)Ge_hi[k] + (Ge_lo ? (long double)Ge_lo[k] : 0.0L);
    std::vector<DmdCandidate> c;
    std::string err;
    if (dmd_candidates(G, M, dtau, c, err) < 0) return -1;
    for (int i = 0; i < (int)c.size() && i < cap; ++i) {
        if (coef) std::copy(c[i].coef.begin(), c[i].coef.end(), coef + (size_t)i * (M - 1));
        if (labels) {
            labels[2 * i] = c[i].rank;
            labels[2 * i + 1] = c[i].kind;
        }
    }
    return (int)c.size();
}

size_t pcfv_host_table(const pcfv_config* cfg, int which, double* out, size_t cap) {
    std::string e;
    if (!validate(cfg, e)) return 0;
    Tables t;
    if (!build_tables(cfg->Lx, cfg->Lz, cfg->Re, cfg->Nx, cfg->Ny, cfg->Nz, cfg->dt_im, t, e)) return 0;
    const std::vector<double>* v = nullptr;
    switch (which) {
        case 0: v = &t.mats; break;
        case 1: v = &t.minfo; break;
        case 2: v = &t.dH; break;
        case 3: v = &t.dP; break;
        case 4: v = &t.dproj; break;
        case 5: v = &t.Vk; break;
        case 6: v = &t.DVk; break;
        case 7: v = &t.Ainv; break;
        case 8: v = &t.mu; break;
        default: return 0;
    }
    if (out) std::memcpy(out, v->data(), std::min(cap, v->size()) * sizeof(double));
    return v->size();
}

}  // extern "C"
