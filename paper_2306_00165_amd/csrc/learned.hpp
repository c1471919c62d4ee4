// Kernels of the learned extrapolator: BF16 matrix-core GEMMs for the MLP
// (FP32 accumulation), its elementwise pieces (loss, bias gradients, Adam),
// and FP64 GEMMs for the proper orthogonal decomposition (POD) of snapshots.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/pcfv.h"

namespace pcfv {

typedef uint16_t bf16_t;   // bfloat16 bit pattern

// Epilogues of the BF16 GEMM C = op(A) op(B) (M x N, FP32 accumulation).
enum GemmEpilogue {
    EPI_F32 = 0,         // outf[m][n] = acc + (bias ? bias[n] : 0)
    EPI_BIAS_RELU = 1,   // outb[m][n] = bf16(max(acc + bias[n], 0))
    EPI_RELU_MASK = 2,   // g = acc * (mask[m][n] != 0): outf = g, outb = bf16(g)
};

// op(A)(m, k) = TA ? A[k * lda + m] : A[m * lda + k]; op(B)(k, n) = TB ?
// B[n * ldb + k] : B[k * ldb + n].  Output row stride ldc.  mask (bf16,
// stride ldc) is read by EPI_RELU_MASK.
hipError_t launch_gemm_bf16(hipStream_t s, int M, int N, int K, const bf16_t* A, int lda, bool TA,
                            const bf16_t* B, int ldb, bool TB, int epi, const float* bias,
                            const bf16_t* mask, float* outf, bf16_t* outb, int ldc);

// dst[i] = bf16(src[i]) (round to nearest even).
hipError_t launch_to_bf16(hipStream_t s, long long n, const float* src, bf16_t* dst);

// MSE loss of Y against T (B x n): dY = 2 (Y - T) / (B n) in FP32 and BF16,
// and per-block partial sums of (Y - T)^2 / (B n) into part (nblocks values,
// returned in *nblocks).
hipError_t launch_mse(hipStream_t s, int B, int n, const float* Y, const float* T, float* dYf,
                      bf16_t* dYb, float* part, int* nblocks);

// out[n] = sum_m G[m][n] (G is B x N, FP32), deterministic order.
hipError_t launch_colsum(hipStream_t s, int B, int N, const float* G, float* out);

// Adam (bias-corrected) on n parameters: m, v moments, p master weights; pb
// (if non-NULL) receives bf16(p).
hipError_t launch_adam(hipStream_t s, long long n, const float* g, float* m, float* v, float* p,
                       bf16_t* pb, float lr, float beta1, float beta2, float eps, float c1, float c2);

// FP64 GEMM with split K: C = op(A) op(B) (+ epilogue), M x N, row stride ldc.
// Ashift (length K, or NULL) is subtracted from every row of op(A) along k
// (op(A)(m, k) - Ashift[k]); Cadd (length N, or NULL) is added to every row
// of the result; the product is scaled by alpha and, with accumulate, added
// to C's previous contents.  part: scratch of splits * M * N doubles (unused,
// may be NULL, when K fits one split).
hipError_t launch_gemm_f64(hipStream_t s, int M, int N, long long K, const double* A, long long lda, bool TA,
                           const double* B, long long ldb, bool TB, const double* Ashift, const double* Cadd,
                           double* C, long long ldc, int splits, double* part, bool accumulate = false,
                           double alpha = 1.0);

// mean[k] = (1/S) sum_s X[s][k] (X is S x n, FP64).
hipError_t launch_rowmean(hipStream_t s, int S, long long n, const double* X, double* mean);

// Xc[s][k] = X[s][k] - mean[k] (S x n).
hipError_t launch_center(hipStream_t s, int S, long long n, const double* X, const double* mean, double* Xc);

// Per-column mean and inverse standard deviation of F (B x n, FP32):
// mu[j], isd[j] = 1 / max(std, floor).
hipError_t launch_colstats(hipStream_t s, int B, int n, const float* F, float floor_, float* mu, float* isd);

// Features of the learned extrapolator from POD coefficients c (rows: guess
// b, window position w < W, r coefficients; double, [W][B][r]) and, if cb is
// non-NULL, the coefficients cb ([B][r]) of a base candidate:
//   x[b][w r + i] = c[w][b][i] - c[W-1][b][i] for w < W-1, c[W-1][b][i] for
//   w = W-1, cb[b][i] - c[W-1][b][i] for w = W (with cb), then normalised
//   (x - mu) * isd (raw if mu is NULL), as FP32; (W + [cb]) r per row.
hipError_t launch_features(hipStream_t s, int W, int B, int r, const double* c, const double* cb, const float* mu,
                           const float* isd, float* x);

// Prediction: the step from the last snapshot to the limit in POD
// coefficients, dc[b][i] = y[b][i] / oisd[i] + omu[i].
hipError_t launch_prediction(hipStream_t s, int B, int r, const float* y, const float* omu, const float* oisd,
                             double* dc);

// Raw training targets t[b][i] = ct[b][i] - (cb ? cb[b][i] : c[W-1][b][i]) (FP32).
hipError_t launch_targets(hipStream_t s, int W, int B, int r, const double* c, const double* cb, const double* ct,
                          float* t);
// F[b][j] = (F[b][j] - mu[j]) * isd[j] (B x n, FP32, in place).
hipError_t launch_normalize(hipStream_t s, int B, int n, float* F, const float* mu, const float* isd);
// dst[i][j] = src[idx[i]][j] (rows x n, FP32).
hipError_t launch_gather(hipStream_t s, int rows, int n, const int* idx, const float* src, float* dst);

// Size of the device-resident scratch array of the allocation-free entry point.
constexpr size_t kStaticScratchBytes = PCFV_NOALLOC_SCRATCH_BYTES;
// Device address of that array on the current device (looked up with
// hipGetSymbolAddress on the first call per device, then cached).
hipError_t static_scratch(double** out);

}  // namespace pcfv
