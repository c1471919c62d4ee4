// Kernels of the learned extrapolator (see learned.hpp).
//
// BF16 GEMM: each work group computes a 64 x 64 tile of C with four waves
// (2 x 2, 32 x 32 each); every 32-deep slice of K is staged in LDS as
// sA[m][k] and sB[n][k] (k contiguous, rows padded to 40 elements so that a
// lane's eight consecutive k values are one aligned 16-byte read) and fed to
// v_mfma_f32_16x16x32_bf16.  Lane l of that instruction supplies
// A[l % 16][8 (l / 16) .. +7] and B[8 (l / 16) .. +7][l % 16] and receives
// C[4 (l / 16) + r][l % 16], r = 0..3 (checked on the device by the tests).
#include "learned.hpp"

#include <mutex>

namespace pcfv {

// Device-resident scratch of the allocation-free POD projection
// (pcfv_pod_project_noalloc): the split-K partials of its FP64 GEMM.  Every
// GPU the library runs on holds one copy for the life of the process.  In host
// code the array's name is only a stand-in for the symbol; its device address
// comes from hipGetSymbolAddress (static_scratch below).
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int GT = 64;        // C tile edge
constexpr int GK = 32;        // K slice
constexpr int LDK = GK + 8;   // padded LDS row (bf16 elements)

__device__ __forceinline__ bf16_t f2bf(float f) {   // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40u);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}

__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const bf16_t* __restrict__ A, int lda,
                                                   int TA, const bf16_t* __restrict__ B, int ldb, int TB, int epi,
                                                   const float* __restrict__ bias, const bf16_t* __restrict__ mask,
                                                   float* __restrict__ outf, bf16_t* __restrict__ outb, int ldc) {
    __shared__ __align__(16) bf16_t sA[GT * LDK];
    __shared__ __align__(16) bf16_t sB[GT * LDK];
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int lr = lane & 15, lq = lane >> 4;
    v4f acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += GK) {
        for (int e = tid; e < GT * GK; e += 256) {
            const int m = TA ? e % GT : e / GK, k = TA ? e / GT : e % GK;
            const int gm = m0 + m, gk = k0 + k;
            bf16_t v = 0;
            if (gm < M && gk < K) v = TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
            sA[m * LDK + k] = v;
        }
        for (int e = tid; e < GT * GK; e += 256) {
            const int n = TB ? e / GK : e % GT, k = TB ? e % GK : e / GT;
            const int gn = n0 + n, gk = k0 + k;
            bf16_t v = 0;
            if (gn < N && gk < K) v = TB ? B[(size_t)gn * ldb + gk] : B[(size_t)gk * ldb + gn];
            sB[n * LDK + k] = v;
        }
        __syncthreads();
        v8bf a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) __builtin_memcpy(&a[i], &sA[(wm + 16 * i + lr) * LDK + 8 * lq], 16);
#pragma unroll
        for (int j = 0; j < 2; ++j) __builtin_memcpy(&b[j], &sB[(wn + 16 * j + lr) * LDK + 8 * lq], 16);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + 16 * i + 4 * lq + r, col = n0 + wn + 16 * j + lr;
                if (row >= M || col >= N) continue;
                const size_t o = (size_t)row * ldc + col;
                float v = acc[i][j][r];
                if (epi == EPI_F32) {
                    outf[o] = v + (bias ? bias[col] : 0.f);
                } else if (epi == EPI_BIAS_RELU) {
                    outb[o] = f2bf(fmaxf(v + bias[col], 0.f));
                } else {
                    v = (mask[o] != 0) ? v : 0.f;
                    outf[o] = v;
                    outb[o] = f2bf(v);
                }
            }
}

__global__ void k_to_bf16(long long n, const float* __restrict__ src, bf16_t* __restrict__ dst) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = f2bf(src[i]);
}

__global__ __launch_bounds__(256) void k_mse(long long n, float scale, const float* __restrict__ Y,
                                             const float* __restrict__ T, float* __restrict__ dYf,
                                             bf16_t* __restrict__ dYb, float* __restrict__ part) {
    __shared__ float red[256];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    float e2 = 0.f;
    if (i < n) {
        const float d = Y[i] - T[i];
        const float g = 2.f * scale * d;
        dYf[i] = g;
        dYb[i] = f2bf(g);
        e2 = d * d * scale;
    }
    red[threadIdx.x] = e2;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_colsum(int B, int N, const float* __restrict__ G, float* __restrict__ out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int m = 0; m < B; ++m) s += G[(size_t)m * N + n];
    out[n] = s;
}

__global__ void k_adam(long long n, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       float* __restrict__ p, bf16_t* __restrict__ pb, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    p[i] = pi;
    if (pb) pb[i] = f2bf(pi);
}

// FP64 GEMM partials: split z of K, 64 x 64 tile, thread (tx, ty) owns rows
// ty + 16 i and columns tx + 16 j.
constexpr int FT = 64, FK = 16;
// With one split (direct != 0) the tile goes straight to C (+ Cadd).
__global__ __launch_bounds__(256) void k_gemm_f64(int M, int N, long long K, long long kchunk,
                                                  const double* __restrict__ A, long long lda, int TA,
                                                  const double* __restrict__ B, long long ldb, int TB,
                                                  const double* __restrict__ Ashift, double* __restrict__ part,
                                                  int direct, int accumulate, double alpha,
                                                  const double* __restrict__ Cadd, double* __restrict__ C,
                                                  long long ldc) {
    __shared__ double sA[FK][FT + 1];
    __shared__ double sB[FK][FT + 1];
    const int m0 = blockIdx.y * FT, n0 = blockIdx.x * FT, z = blockIdx.z;
    const long long kb = (long long)z * kchunk, ke = (kb + kchunk < K) ? kb + kchunk : K;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    double acc[4][4] = {};
    for (long long k0 = kb; k0 < ke; k0 += FK) {
        for (int e = tid; e < FT * FK; e += 256) {
            const int m = TA ? e % FT : e / FK, k = TA ? e / FT : e % FK;
            const int gm = m0 + m;
            const long long gk = k0 + k;
            double v = 0.0;
            if (gm < M && gk < ke) {
                v = TA ? A[gk * lda + gm] : A[(long long)gm * lda + gk];
                if (Ashift) v -= Ashift[gk];
            }
            sA[k][m] = v;
        }
        for (int e = tid; e < FT * FK; e += 256) {
            const int n = TB ? e / FK : e % FT, k = TB ? e % FK : e / FT;
            const int gn = n0 + n;
            const long long gk = k0 + k;
            double v = 0.0;
            if (gn < N && gk < ke) v = TB ? B[(long long)gn * ldb + gk] : B[gk * ldb + gn];
            sB[k][n] = v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < FK; ++k) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = sA[k][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = sB[k][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = m0 + ty + 16 * i, col = n0 + tx + 16 * j;
            if (row >= M || col >= N) continue;
            if (direct)
                C[row * ldc + col] =
                    (accumulate ? C[row * ldc + col] : 0.0) + alpha * acc[i][j] + (Cadd ? Cadd[col] : 0.0);
            else
                part[((size_t)z * M + row) * N + col] = acc[i][j];
        }
}

__global__ void k_gemm_f64_reduce(int M, int N, int splits, const double* __restrict__ part, int accumulate,
                                  double alpha, const double* __restrict__ Cadd, double* __restrict__ C,
                                  long long ldc) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)M * N) return;
    const int row = (int)(e / N), col = (int)(e - (long long)row * N);
    double s = 0.0;
    for (int z = 0; z < splits; ++z) s += part[(size_t)z * M * N + e];
    C[row * ldc + col] = (accumulate ? C[row * ldc + col] : 0.0) + alpha * s + (Cadd ? Cadd[col] : 0.0);
}

__global__ void k_rowmean(int S, long long n, const double* __restrict__ X, double* __restrict__ mean) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double s = 0.0;
    for (int i = 0; i < S; ++i) s += X[(long long)i * n + k];
    mean[k] = s / S;
}

__global__ void k_center(int S, long long n, const double* __restrict__ X, const double* __restrict__ mean,
                         double* __restrict__ Xc) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)S * n) return;
    Xc[e] = X[e] - mean[e % n];
}

__global__ void k_colstats(int B, int n, const float* __restrict__ F, float floor_, float* __restrict__ mu,
                           float* __restrict__ isd) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += F[(size_t)b * n + j];
    const double m = s / B;
    double q = 0.0;
    for (int b = 0; b < B; ++b) {
        const double d = F[(size_t)b * n + j] - m;
        q += d * d;
    }
    const double sd = sqrt(q / B);
    mu[j] = (float)m;
    isd[j] = (float)(1.0 / (sd > floor_ ? sd : (double)floor_));
}

__global__ void k_features(int W, int B, int r, const double* __restrict__ c, const double* __restrict__ cb,
                           const float* __restrict__ mu, const float* __restrict__ isd, float* __restrict__ x) {
    const int F = (W + (cb ? 1 : 0)) * r;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)B * F) return;
    const int b = (int)(e / F), rem = (int)(e - (long long)b * F), w = rem / r, i = rem - w * r;
    const double last = c[((size_t)(W - 1) * B + b) * r + i];
    double v;
    if (w < W - 1)
        v = c[((size_t)w * B + b) * r + i] - last;
    else if (w == W - 1)
        v = last;
    else
        v = cb[(size_t)b * r + i] - last;
    x[e] = mu ? (float)((v - mu[rem]) * isd[rem]) : (float)v;
}

__global__ void k_targets(int W, int B, int r, const double* __restrict__ c, const double* __restrict__ cb,
                          const double* __restrict__ ct, float* __restrict__ t) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * r) return;
    const int b = e / r, i = e - b * r;
    t[e] = (float)(ct[e] - (cb ? cb[e] : c[((size_t)(W - 1) * B + b) * r + i]));
}

__global__ void k_normalize(int B, int n, float* __restrict__ F, const float* __restrict__ mu,
                            const float* __restrict__ isd) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)B * n) return;
    const int j = (int)(e % n);
    F[e] = (F[e] - mu[j]) * isd[j];
}

__global__ void k_gather(int rows, int n, const int* __restrict__ idx, const float* __restrict__ src,
                         float* __restrict__ dst) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)rows * n) return;
    const int row = (int)(e / n), j = (int)(e - (long long)row * n);
    dst[e] = src[(size_t)idx[row] * n + j];
}

__global__ void k_prediction(int B, int r, const float* __restrict__ y, const float* __restrict__ omu,
                             const float* __restrict__ oisd, double* __restrict__ dc) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * r) return;
    const int i = e % r;
    dc[e] = (double)y[e] / oisd[i] + omu[i];
}

unsigned blocks(long long n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_gemm_bf16(hipStream_t s, int M, int N, int K, const bf16_t* A, int lda, bool TA, const bf16_t* B,
                            int ldb, bool TB, int epi, const float* bias, const bf16_t* mask, float* outf,
                            bf16_t* outb, int ldc) {
    if (M <= 0 || N <= 0 || K <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gemm_bf16, dim3(blocks(N, GT), blocks(M, GT)), dim3(256), 0, s, M, N, K, A, lda, (int)TA, B,
                       ldb, (int)TB, epi, bias, mask, outf, outb, ldc);
    return hipGetLastError();
}

hipError_t launch_to_bf16(hipStream_t s, long long n, const float* src, bf16_t* dst) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks(n, 256)), dim3(256), 0, s, n, src, dst);
    return hipGetLastError();
}

hipError_t launch_mse(hipStream_t s, int B, int n, const float* Y, const float* T, float* dYf, bf16_t* dYb,
                      float* part, int* nblocks) {
    const long long tot = (long long)B * n;
    *nblocks = (int)blocks(tot, 256);
    hipLaunchKernelGGL(k_mse, dim3(*nblocks), dim3(256), 0, s, tot, 1.0f / (float)tot, Y, T, dYf, dYb, part);
    return hipGetLastError();
}

hipError_t launch_colsum(hipStream_t s, int B, int N, const float* G, float* out) {
    hipLaunchKernelGGL(k_colsum, dim3(blocks(N, 256)), dim3(256), 0, s, B, N, G, out);
    return hipGetLastError();
}

hipError_t launch_adam(hipStream_t s, long long n, const float* g, float* m, float* v, float* p, bf16_t* pb, float lr,
                       float beta1, float beta2, float eps, float c1, float c2) {
    hipLaunchKernelGGL(k_adam, dim3(blocks(n, 256)), dim3(256), 0, s, n, g, m, v, p, pb, lr, beta1, beta2, eps, c1,
                       c2);
    return hipGetLastError();
}

hipError_t launch_gemm_f64(hipStream_t s, int M, int N, long long K, const double* A, long long lda, bool TA,
                           const double* B, long long ldb, bool TB, const double* Ashift, const double* Cadd,
                           double* C, long long ldc, int splits, double* part, bool accumulate, double alpha) {
    if (M <= 0 || N <= 0 || K <= 0 || splits < 1) return hipErrorInvalidValue;
    long long kchunk = (K + splits - 1) / splits;
    kchunk = (kchunk + FK - 1) / FK * FK;
    const int z = (int)((K + kchunk - 1) / kchunk);
    const int direct = (z == 1);
    hipLaunchKernelGGL(k_gemm_f64, dim3(blocks(N, FT), blocks(M, FT), z), dim3(256), 0, s, M, N, K, kchunk, A, lda,
                       (int)TA, B, ldb, (int)TB, Ashift, part, direct, (int)accumulate, alpha, Cadd, C, ldc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || direct) return e;
    hipLaunchKernelGGL(k_gemm_f64_reduce, dim3(blocks((long long)M * N, 256)), dim3(256), 0, s, M, N, z, part,
                       (int)accumulate, alpha, Cadd, C, ldc);
    return hipGetLastError();
}

hipError_t launch_rowmean(hipStream_t s, int S, long long n, const double* X, double* mean) {
    hipLaunchKernelGGL(k_rowmean, dim3(blocks(n, 256)), dim3(256), 0, s, S, n, X, mean);
    return hipGetLastError();
}

hipError_t launch_center(hipStream_t s, int S, long long n, const double* X, const double* mean, double* Xc) {
    hipLaunchKernelGGL(k_center, dim3(blocks((long long)S * n, 256)), dim3(256), 0, s, S, n, X, mean, Xc);
    return hipGetLastError();
}

hipError_t launch_colstats(hipStream_t s, int B, int n, const float* F, float floor_, float* mu, float* isd) {
    hipLaunchKernelGGL(k_colstats, dim3(blocks(n, 256)), dim3(256), 0, s, B, n, F, floor_, mu, isd);
    return hipGetLastError();
}

hipError_t launch_features(hipStream_t s, int W, int B, int r, const double* c, const double* cb, const float* mu,
                           const float* isd, float* x) {
    const long long n = (long long)B * (W + (cb ? 1 : 0)) * r;
    hipLaunchKernelGGL(k_features, dim3(blocks(n, 256)), dim3(256), 0, s, W, B, r, c, cb, mu, isd, x);
    return hipGetLastError();
}

hipError_t launch_prediction(hipStream_t s, int B, int r, const float* y, const float* omu, const float* oisd,
                             double* dc) {
    hipLaunchKernelGGL(k_prediction, dim3(blocks((long long)B * r, 256)), dim3(256), 0, s, B, r, y, omu, oisd, dc);
    return hipGetLastError();
}

hipError_t launch_targets(hipStream_t s, int W, int B, int r, const double* c, const double* cb, const double* ct,
                          float* t) {
    hipLaunchKernelGGL(k_targets, dim3(blocks((long long)B * r, 256)), dim3(256), 0, s, W, B, r, c, cb, ct, t);
    return hipGetLastError();
}

hipError_t launch_normalize(hipStream_t s, int B, int n, float* F, const float* mu, const float* isd) {
    hipLaunchKernelGGL(k_normalize, dim3(blocks((long long)B * n, 256)), dim3(256), 0, s, B, n, F, mu, isd);
    return hipGetLastError();
}

hipError_t launch_gather(hipStream_t s, int rows, int n, const int* idx, const float* src, float* dst) {
    hipLaunchKernelGGL(k_gather, dim3(blocks((long long)rows * n, 256)), dim3(256), 0, s, rows, n, idx, src, dst);
    return hipGetLastError();
}

// Device address of `scratch` on the current device: looked up once per device
// (with that device current) and kept, since each GPU holds its own copy at
// its own address.
hipError_t static_scratch(double** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = static_cast<double*>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

}  // namespace pcfv
