// HIP kernels of the pcfv hot path (gfx950, FP64).
//
// Data layouts (complex128 as double2):
//   spectral  u[c][m][n]      c = component, m = ikx*nkz + kz, n = Chebyshev index
//   y-values  Y[f][j][m]      field f at Gauss-Lobatto point j, Fourier mode m
//   partials  P[s][f][j][m]   x-slab s of a forward transform (summed by the consumer)
//
// One descent step (Sec. 4, five steps, in their exact discrete form):
//   k_plane<FWD>    U = u_b + u and grad U on the grid from the y-values, the
//                   convective term (U.grad)U, forward transform in x and z
//   k_mode_res      per Fourier mode: analysis in y, F = M + nu L u, the
//                   influence-matrix Stokes solve r = lam S F (Sec. 4 steps
//                   (1)-(2)), the cost partial <r,r>, the transposed solve
//                   a = S* r and the y-values of a
//   k_plane<ADJ>    the adjoint products U_j a_i and (d_j U_i) a_i, forward
//                   transform in x and z
//   k_mode_grad     per mode: g = J* r = lam [M'* a + nu L* a] (Sec. 3.3 in
//                   discrete form), f = -P g (Sec. 3.4), u += dtau f (step (5)),
//                   and the y-values of the new u for the next step.
#include <algorithm>
#include <cstdio>
#include <type_traits>

#include "kernels.hpp"

namespace pcfv {
namespace {

constexpr int WAVE = 64;
constexpr int MODE_VECS = 24;                  // LDS vectors (stride NP) used by the mode kernels
constexpr int RED_SLOTS = 16;                  // doubles per wave for block reductions

// Work-group shapes of the per-mode kernels (one Fourier mode per work group):
// MT threads; every output row of a contraction is summed by KS lanes of a
// wave, ROWS rows per wave.  256 threads with KS = 4 (the default) or 512
// threads with KS = 8 (half of each lane's serial chain, twice the waves).
template <int MT> struct MC {
    static constexpr int THREADS = MT, WAVES = MT / WAVE, KS = (MT >= 512) ? 8 : 4, ROWS = WAVE / KS;
};

__device__ __forceinline__ double2 c2(double x, double y) { return make_double2(x, y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return c2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return c2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscl(double s, double2 a) { return c2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return c2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// (i s) z for real s
__device__ __forceinline__ double2 imul(double s, double2 z) { return c2(-s * z.y, s * z.x); }

// The physical-space kernels are instantiated for R = double (FP64 path) and
// R = float (FP32 transforms and products); C<R> is the matching complex type.
// The per-mode kernels always compute in FP64 and read/write the y-value and
// partial arrays in the storage type of the physical-space precision.
template <class R> struct CT;
template <> struct CT<double> { typedef double2 T; };
template <> struct CT<float> { typedef float2 T; };
template <class R> using C = typename CT<R>::T;

// mkc: complex from two reals of either precision (overloads, no int literals).
__device__ __forceinline__ double2 mkc(double x, double y) { return make_double2(x, y); }
__device__ __forceinline__ float2 mkc(float x, float y) { return make_float2(x, y); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return mkc(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return mkc(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscl(float s, float2 a) { return mkc(s * a.x, s * a.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return mkc(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 imul(float s, float2 z) { return mkc(-s * z.y, s * z.x); }

// Fused multiply-add in the precision of its arguments.
__device__ __forceinline__ double fmar(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fmar(float a, float b, float c) { return fmaf(a, b, c); }

// acc + a b for complex a, b as four fused multiply-adds.
__device__ __forceinline__ double2 cmac(double2 acc, double2 a, double2 b) {
    return c2(fmar(-a.y, b.y, fmar(a.x, b.x, acc.x)), fmar(a.y, b.x, fmar(a.x, b.y, acc.y)));
}
__device__ __forceinline__ float2 cmac(float2 acc, float2 a, float2 b) {
    return mkc(fmar(-a.y, b.y, fmar(a.x, b.x, acc.x)), fmar(a.y, b.x, fmar(a.x, b.y, acc.y)));
}

__device__ __forceinline__ double2 widen(double2 v) { return v; }
__device__ __forceinline__ double2 widen(float2 v) { return make_double2(v.x, v.y); }
template <class T> __device__ __forceinline__ T narrow(double2 v);
template <> __device__ __forceinline__ double2 narrow<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 narrow<float2>(double2 v) {
    return make_float2((float)v.x, (float)v.y);
}


// Work groups are dispatched to the 8 XCDs of the chip round-robin.  Launchers
// pad the grid to a multiple of 8 and kernels map their work-group index w to
// the logical work item (w % 8) * (nwg / 8) + w / 8, so each XCD processes one
// contiguous range of work items and neighbouring items, which share cache
// lines of the [field][j][mode] arrays, share one L2.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_item(int w, int nwg) { return (w % NXCD) * (nwg / NXCD) + w / NXCD; }

struct MS {
    double a, b, k2, ik2, sig, wgt;
};
__device__ __forceinline__ MS mscal(const KP& p, int m) {
    const double* mi = p.minfo + (size_t)m * MI_STRIDE;
    return {mi[MI_A], mi[MI_B], mi[MI_K2], mi[MI_INVK2], mi[MI_SIG], mi[MI_WGT]};
}

// Fixed matrix id: an NP x mat_ld(NP) slot, transposed
// (slot[k * mat_ld(NP) + n] = A[n][k]), zero outside the matrix.
template <int NP>
__device__ __forceinline__ const double* mat(const KP& p, int id) {
    return p.M + (size_t)id * NP * mat_ld(NP);
}


// Sums over the lanes that share one output row of a contraction: lanes
// MC<MT>::ROWS apart within the wave (8, 16, 32 apart for ROWS = 8; 16, 32 for
// ROWS = 16).  The exchanges run on the VALU: a DPP rotation by 8 within each
// 16-lane row and the gfx950 permlane16/permlane32 swaps, which exchange the
// odd and even 16-lane rows and the two 32-lane halves.  Every lane of a row
// group receives the same bits (the partners add the same two numbers).
__device__ __forceinline__ double ror8_add(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)__double2loint(v), 0x128, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)__double2hiint(v), 0x128, 0xf, 0xf, false);
    return v + __hiloint2double(hi, lo);
}
__device__ __forceinline__ double swap16_add(double v) {
    const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}
__device__ __forceinline__ double swap32_add(double v) {
    const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}
// A double moved across lanes by a DPP pattern (both halves).
template <int CTRL> __device__ __forceinline__ double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)__double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)__double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// v in the partner lane (lane ^ 1) of a lane pair
template <class R> __device__ __forceinline__ R lane_pair_swap(R v) {
    if constexpr (sizeof(R) == 8)
        return dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    else
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xf, 0xf, false));
}

__device__ __forceinline__ double swap16_max(double v) {
    const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return fmax(__hiloint2double((int)h[0], (int)l[0]), __hiloint2double((int)h[1], (int)l[1]));
}
__device__ __forceinline__ double swap32_max(double v) {
    const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return fmax(__hiloint2double((int)h[0], (int)l[0]), __hiloint2double((int)h[1], (int)l[1]));
}

// Sum (maximum) over the 64 lanes of a wave, on the VALU: quad permutes
// (lane xor 1, xor 2), rotations by 4 and 8 within each 16-lane row, then the
// row swaps.  Every lane of the wave must be active; lane 0 holds the total
// (every lane holds a total, summed in an order that may differ by lane).
__device__ __forceinline__ double wsum(double v) {
    v += dpp_d<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x124>(v);   // row_ror:4
    v += dpp_d<0x128>(v);   // row_ror:8
    v = swap16_add(v);
    return swap32_add(v);
}
__device__ __forceinline__ double wmax(double v) {
    v = fmax(v, dpp_d<0xB1>(v));
    v = fmax(v, dpp_d<0x4E>(v));
    v = fmax(v, dpp_d<0x124>(v));
    v = fmax(v, dpp_d<0x128>(v));
    v = swap16_max(v);
    return swap32_max(v);
}

// Block reduction of NV values per thread (deterministic order): every thread
// receives the block totals.  red: LDS scratch of MC<MT>::WAVES * RED_SLOTS doubles.
template <int MT, int NV>
__device__ void bsum(double (&v)[NV], double* red) {
    static_assert(NV <= RED_SLOTS, "too many values");
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wsum(v[i]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) red[wave * RED_SLOTS + i] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double t = 0;
        for (int w = 0; w < MC<MT>::WAVES; ++w) t += red[w * RED_SLOTS + i];
        v[i] = t;
    }
    __syncthreads();
}

template <int MT, int NV>
__device__ void bmax(double (&v)[NV], double* red) {
    static_assert(NV <= RED_SLOTS, "too many values");
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wmax(v[i]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) red[wave * RED_SLOTS + i] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double t = 0;
        for (int w = 0; w < MC<MT>::WAVES; ++w) t = fmax(t, red[w * RED_SLOTS + i]);
        v[i] = t;
    }
    __syncthreads();
}

template <int MT> __device__ __forceinline__ double row_sum(double v) {
    static_assert(MC<MT>::ROWS == 8 || MC<MT>::ROWS == 16, "row groups of 8 or 16 lanes");
    if constexpr (MC<MT>::ROWS == 8) v = ror8_add(v);
    v = swap16_add(v);
    return swap32_add(v);
}

// Raw buffer view of the fixed-matrix block: every matrix element is fetched
// with one buffer load whose per-lane offset is fixed for the whole kernel
// and whose matrix and step offsets are wave-uniform (scalar operand), so a
// contraction issues no address arithmetic.  Offsets past the block read 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t mat_rsrc(const KP& p, int NP) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p.M), 0, M_COUNT * NP * mat_ld(NP) * 8, 0x00020000);
}
__device__ __forceinline__ double mat_load(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0);
    return __hiloint2double((int)v[1], (int)v[0]);
}

// One contraction's matrix elements as the lanes hold them.  y = A x for
// A = fixed matrix id (nout x nin, zero-padded to NP rows): each output row is
// computed by MC<MT>::KS lanes of one wave, each summing every MC<MT>::KS-th
// term over the padded length NP, then combined across lanes; rows are dealt
// out MC<MT>::ROWS per wave in PASSES passes.  The padding terms multiply
// exact zeros of A by finite entries of x (the LDS vectors start zeroed), so
// no step is predicated, and the loads of every pass are issued before any
// arithmetic, so one contraction waits for memory once.  A wave whose rows
// all lie at or past nout neither loads nor computes.
template <int NP, int MT> struct MatRegs {
    typedef MC<MT> S;
    static constexpr int ROWS_PER_PASS = S::WAVES * S::ROWS;
    static constexpr int PASSES = (NP + ROWS_PER_PASS - 1) / ROWS_PER_PASS;
    static constexpr int PER = NP / S::KS;
    double a[PASSES][PER];
};

template <int NP, int MT>
__device__ __forceinline__ MatRegs<NP, MT> mat_fetch(const KP& p, int id, int nout) {
    typedef MC<MT> S;
    typedef MatRegs<NP, MT> A;
    constexpr int LD = mat_ld(NP);
    const __amdgpu_buffer_rsrc_t rs = mat_rsrc(p, NP);
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    const int r = lane % S::ROWS, q = lane / S::ROWS;
    A m;
#pragma unroll
    for (int ps = 0; ps < A::PASSES; ++ps) {
        const int n0 = ps * A::ROWS_PER_PASS;
        if (n0 + wave * S::ROWS >= nout) break;   // wave-uniform: no rows of this wave are left
        const int voff = (q * LD + min(n0 + wave * S::ROWS + r, NP - 1)) * 8;
#pragma unroll
        for (int i = 0; i < A::PER; ++i) m.a[ps][i] = mat_load(rs, voff, (id * NP + S::KS * i) * LD * 8);
    }
    return m;
}

// y = A x for one complex vector, A = fixed matrix id, x in LDS.  Row n of
// the result goes to ep(n, y_n), called by one lane for every n < nout; the
// row-to-thread map depends only on NP and MT, so an epilogue may read
// entries [n] that the same thread stored in an earlier contraction's
// epilogue without a barrier.  Caller synchronises before other threads read
// what the epilogue stores.
template <int NP, int MT, class EP>
__device__ __forceinline__ void mv_ep(const KP& p, int id, int nout, const double2* x, EP&& ep) {
    typedef MC<MT> S;
    typedef MatRegs<NP, MT> A;
    const A m = mat_fetch<NP, MT>(p, id, nout);
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    const int r = lane % S::ROWS, q = lane / S::ROWS;
#pragma unroll
    for (int ps = 0; ps < A::PASSES; ++ps) {
        const int n0 = ps * A::ROWS_PER_PASS;
        if (n0 + wave * S::ROWS >= nout) break;
        const int n = n0 + wave * S::ROWS + r;
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int i = 0; i < A::PER; ++i) {
            const double2 v = x[q + S::KS * i];
            re = fma(m.a[ps][i], v.x, re);
            im = fma(m.a[ps][i], v.y, im);
        }
        re = row_sum<MT>(re);
        im = row_sum<MT>(im);
        if (q == 0 && n < nout) ep(n, c2(re, im));
    }
}

// The same matrix applied to three vectors; ep(n, y0_n, y1_n, y2_n).
template <int NP, int MT, class EP>
__device__ __forceinline__ void mv3_ep(const KP& p, int id, int nout, const double2* x0, const double2* x1,
                                       const double2* x2, EP&& ep) {
    typedef MC<MT> S;
    typedef MatRegs<NP, MT> A;
    const A m = mat_fetch<NP, MT>(p, id, nout);
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    const int r = lane % S::ROWS, q = lane / S::ROWS;
#pragma unroll
    for (int ps = 0; ps < A::PASSES; ++ps) {
        const int n0 = ps * A::ROWS_PER_PASS;
        if (n0 + wave * S::ROWS >= nout) break;
        const int n = n0 + wave * S::ROWS + r;
        double acc[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < A::PER; ++i) {
            const int k = q + S::KS * i;
            const double2 v0 = x0[k], v1 = x1[k], v2 = x2[k];
            acc[0] = fma(m.a[ps][i], v0.x, acc[0]);
            acc[1] = fma(m.a[ps][i], v0.y, acc[1]);
            acc[2] = fma(m.a[ps][i], v1.x, acc[2]);
            acc[3] = fma(m.a[ps][i], v1.y, acc[3]);
            acc[4] = fma(m.a[ps][i], v2.x, acc[4]);
            acc[5] = fma(m.a[ps][i], v2.y, acc[5]);
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) acc[i] = row_sum<MT>(acc[i]);
        if (q == 0 && n < nout) ep(n, c2(acc[0], acc[1]), c2(acc[2], acc[3]), c2(acc[4], acc[5]));
    }
}

// y = A x into LDS (x and y must not alias; entries [nout, NP) of y untouched).
template <int NP, int MT>
__device__ __forceinline__ void mv(const KP& p, int id, int nout, const double2* x, double2* y) {
    mv_ep<NP, MT>(p, id, nout, x, [&](int n, double2 v) { y[n] = v; });
}
template <int NP, int MT>
__device__ __forceinline__ void mv3(const KP& p, int id, int nout, const double2* x0, const double2* x1,
                                    const double2* x2, double2* y0, double2* y1, double2* y2) {
    mv3_ep<NP, MT>(p, id, nout, x0, x1, x2, [&](int n, double2 a, double2 b, double2 c) {
        y0[n] = a;
        y1[n] = b;
        y2[n] = c;
    });
}

// LDS of the per-mode kernels: MODE_VECS complex vectors at stride NP, then
// the block-reduction scratch.  The vectors start zeroed, so the padded tail
// [Ny, NP) and every entry not yet written hold finite values.
template <int NP, int MT>
__device__ __forceinline__ double2* mode_vectors() {
    extern __shared__ double2 sm[];
    for (int i = threadIdx.x; i < MODE_VECS * NP; i += MT) sm[i] = c2(0.0, 0.0);
    __syncthreads();
    return sm;
}

// Per-mode tables of the solves and the projection, staged in LDS after the
// mode vectors (then the block-reduction scratch): dH, dP (NP each), the
// homogeneous responses Vk, DVk (4 rows of NP), the 4 x 4 inverse influence
// matrix and the projection diagonal dq (NP).  Read from LDS, they cost no
// global round trip in the middle of a solve, where a barrier would keep the
// compiler from loading them early.
constexpr int tab_doubles(int np) { return 11 * np + 16; }
struct ModeTabs {
    const double *dH, *dP, *Vk, *DVk, *Ai, *dq;
};
template <int NP>
__device__ __forceinline__ double* mode_tab(double2* vs) { return reinterpret_cast<double*>(vs + (size_t)MODE_VECS * NP); }
template <int NP>
__device__ __forceinline__ double* mode_red(double2* vs) { return mode_tab<NP>(vs) + tab_doubles(NP); }

// Mode m's tables into LDS (solve: dH, dP, Vk, DVk, Ainv; proj: dq), each
// thread's loads issued together; the caller's next barrier publishes them.
template <int NP, int MT>
__device__ __forceinline__ ModeTabs stage_tabs(const KP& p, int m, double* tab, bool solve, bool proj) {
    const int N = p.N;
    double *dH = tab, *dP = tab + NP, *Vk = tab + 2 * NP, *DVk = tab + 6 * NP, *Ai = tab + 10 * NP,
           *dq = tab + 10 * NP + 16;
    const size_t mN = (size_t)m * N;
    for (int n = threadIdx.x; n < max(N, 16); n += MT) {
        double h = 0, q = 0, r = 0, a = 0, v[4] = {0, 0, 0, 0}, dv[4] = {0, 0, 0, 0};
        if (solve && n < N) {
            h = p.dH[mN + n];
            q = p.dP[mN + n];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                v[k] = p.Vk[4 * mN + (size_t)k * N + n];
                dv[k] = p.DVk[4 * mN + (size_t)k * N + n];
            }
        }
        if (solve && n < 16) a = p.Ainv[(size_t)m * 16 + n];
        if (proj && n < N) r = p.dproj[mN + n];
        if (solve && n < N) {
            dH[n] = h;
            dP[n] = q;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                Vk[k * NP + n] = v[k];
                DVk[k * NP + n] = dv[k];
            }
        }
        if (solve && n < 16) Ai[n] = a;
        if (proj && n < N) dq[n] = r;
    }
    return {dH, dP, Vk, DVk, Ai, dq};
}

// The opening reads of the residual and gradient kernels in one pass: mode m's
// tables (as stage_tabs), the three components of spectral field f at the
// guess offset so (into fd[0..2] at stride NP) and the NS x-slab partials of
// NF fields of work item mB (summed in slab order into pd[0..NF-1] at stride
// NP).  Every load of a thread is issued before its first LDS store, so the
// three groups of reads cost one round trip.  The caller's next barrier
// publishes the results.
template <int NP, int MT, int NF, class YT>
__device__ __forceinline__ ModeTabs open_mode(const KP& p, int m, int mB, size_t so, double* tab, bool solve,
                                              bool proj, const double2* __restrict__ f, double2* fd,
                                              const YT* __restrict__ P, double2* pd) {
    const int N = p.N, NS = p.NS;
    const size_t nm = p.nm, nmB = p.nmB, mN = (size_t)m * N;
    double *dH = tab, *dP = tab + NP, *Vk = tab + 2 * NP, *DVk = tab + 6 * NP, *Ai = tab + 10 * NP,
           *dq = tab + 10 * NP + 16;
    for (int n = threadIdx.x; n < max(N, 16); n += MT) {
        // every load is unconditional at a clamped (in-bounds) index, and only the
        // stores are guarded: a load under a condition would make the compiler
        // wait for it where the condition ends, before the next loads issue
        const int nc = min(n, N - 1);
        const double h = p.dH[mN + nc], q = p.dP[mN + nc], r = p.dproj[mN + nc];
        const double a = p.Ainv[(size_t)m * 16 + min(n, 15)];
        double v[4], dv[4], fx[3], fy[3];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = p.Vk[4 * mN + (size_t)k * N + nc];
            dv[k] = p.DVk[4 * mN + (size_t)k * N + nc];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double2 w = f[so + ((size_t)c * nm + m) * N + nc];
            fx[c] = w.x;
            fy[c] = w.y;
        }
        // slab partials in batches of four, summed in slab order; the first
        // batch is straight-line code, so its loads issue with the ones above
        // (a loop entry would wait for them first)
        double ax[NF], ay[NF];
        YT pv[4][NF];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const size_t sl = (size_t)min(k, NS - 1);
#pragma unroll
            for (int g = 0; g < NF; ++g) pv[k][g] = P[((sl * NF + g) * N + nc) * nmB + mB];
        }
#pragma unroll
        for (int g = 0; g < NF; ++g) ax[g] = ay[g] = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < NS)
#pragma unroll
                for (int g = 0; g < NF; ++g) {
                    const double2 w = widen(pv[k][g]);
                    ax[g] += w.x;
                    ay[g] += w.y;
                }
        for (int s0 = 4; s0 < NS; s0 += 4) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const size_t sl = (size_t)min(s0 + k, NS - 1);
#pragma unroll
                for (int g = 0; g < NF; ++g) pv[k][g] = P[((sl * NF + g) * N + nc) * nmB + mB];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (s0 + k < NS)
#pragma unroll
                    for (int g = 0; g < NF; ++g) {
                        const double2 w = widen(pv[k][g]);
                        ax[g] += w.x;
                        ay[g] += w.y;
                    }
        }
        if (n < N) {
#pragma unroll
            for (int g = 0; g < NF; ++g) pd[g * NP + n] = c2(ax[g], ay[g]);
#pragma unroll
            for (int c = 0; c < 3; ++c) fd[c * NP + n] = c2(fx[c], fy[c]);
            if (solve) {
                dH[n] = h;
                dP[n] = q;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    Vk[k * NP + n] = v[k];
                    DVk[k * NP + n] = dv[k];
                }
            }
            if (proj) dq[n] = r;
        }
        if (solve && n < 16) Ai[n] = a;
    }
    return {dH, dP, Vk, DVk, Ai, dq};
}

// The per-mode kernels read a few values per thread from global memory before
// their first contraction.  The helpers below issue all of a thread's loads
// before the first use, so their latencies overlap instead of adding up.

// The three components of spectral field f at mode m of the guess at offset
// so, into LDS vectors d0, d1, d2.
template <int MT>
__device__ __forceinline__ void read_field3(const KP& p, const double2* __restrict__ f, size_t so, int m,
                                            double2* d0, double2* d1, double2* d2) {
    const int N = p.N;
    const size_t nm = p.nm;
    for (int n = threadIdx.x; n < N; n += MT) {
        const double2 a = f[so + (size_t)m * N + n], b = f[so + (nm + m) * N + n], c = f[so + (2 * nm + m) * N + n];
        d0[n] = a;
        d1[n] = b;
        d2[n] = c;
    }
}


// ---------------------------------------------------------------------------
// Stokes solve S (kappa > 0) by the influence-matrix method in the fixed
// tau eigenbasis.  Writes (ox, oy, oz) = velocity of the Chebyshev-tau
// solution for forcing (Fx, Fy, Fz).  The algorithm:
//   h  = D Fy + i a Fx + i b Fz                  (divergence of the forcing)
//   p0 = Poisson-tau solve (D^2 - k^2) p0 = h, p0(+-1) = 0
//   v0 = Helmholtz-tau solve (sig - nu D^2) v0 = Fy - D p0, v0(+-1) = 0
//   c  = -A^{-1} (Dv0(+1), Dv0(-1), tau residuals of the v equation)
//   v  = v0 + sum_k c_k v_k   (homogeneous responses: Dirichlet data of p
//                              and the tau correction of the Poisson equation)
//   eta = Helmholtz-tau solve of (i b Fx - i a Fz)   (wall-normal vorticity)
//   u_x = (i a Dv - i b eta)/k^2, u_z = (i b Dv + i a eta)/k^2
// Each tau solve is Pl diag(d) Pr; with the precomposed fixed matrices
// PRD = Pr R D, PRDPL = Pr R D Pl and DPL = D Pl the whole solve is three
// contraction phases:
//   A: s1 = Pr Fh, s2 = Pr Fe, s3 = Pr Fy, s4 = PRD Fy
//      t1 = -dP (s4 + s1), te = dH s2
//   B: t2 = dH (s3 - PRDPL t1)           (p0 = Pl t1 is never formed)
//   C: v0 = Pl t2, Dv0 = DPL t2, eta = Pl te, and p0(N-1) = Pl[N-1,:] t1
// w: 10 scratch vectors.
// ---------------------------------------------------------------------------
template <int NP, int MT>
__device__ void stokes(const KP& p, const ModeTabs& T, const MS& c, const double2* Fx, const double2* Fy,
                       const double2* Fz, double2* ox, double2* oy, double2* oz, double2* w,
                       double* red) {
    const int N = p.N, M = N - 2, t = threadIdx.x;
    double2 *Fh = w, *Fe = w + NP, *s1 = w + 2 * NP, *s2 = w + 3 * NP, *s3 = w + 4 * NP,
            *t2 = w + 6 * NP, *v0 = w + 7 * NP, *Dv0 = w + 8 * NP, *eta = w + 9 * NP;
    const double* dH = T.dH;
    const double* dP = T.dP;
    for (int n = t; n < N; n += MT) {
        const double2 fx = Fx[n], fz = Fz[n];
        Fh[n] = cadd(imul(c.a, fx), imul(c.b, fz));
        Fe[n] = csub(imul(c.b, fx), imul(c.a, fz));
    }
    __syncthreads();
    // the diagonal steps run in the epilogues: row n of each contraction is
    // stored by the thread that stored row n of the earlier ones
    mv3<NP, MT>(p, M_PR, M, Fh, Fe, Fy, s1, s2, s3);
    mv_ep<NP, MT>(p, M_PRD, M, Fy, [&](int n, double2 s4) {
        s1[n] = cscl(-dP[n], cadd(s4, s1[n]));   // t1
        s2[n] = cscl(dH[n], s2[n]);              // te
    });
    __syncthreads();
    mv_ep<NP, MT>(p, M_PRDPL, M, s1, [&](int n, double2 v) { t2[n] = cscl(dH[n], csub(s3[n], v)); });
    __syncthreads();
    mv<NP, MT>(p, M_PL, N, t2, v0);
    mv<NP, MT>(p, M_DPL, N, t2, Dv0);
    mv<NP, MT>(p, M_PL, N, s2, eta);
    __syncthreads();
    const double* PLlast = mat<NP>(p, M_PL) + (N - 1);  // row N-1 of Pl: PLlast[k * mat_ld(NP)]
    double sums[6] = {0, 0, 0, 0, 0, 0};
    for (int n = t; n < N; n += MT) {
        const double2 d = Dv0[n];
        sums[0] += d.x;
        sums[1] += d.y;
        sums[2] += (n & 1) ? -d.x : d.x;
        sums[3] += (n & 1) ? -d.y : d.y;
        if (n < M) {
            sums[4] += PLlast[(size_t)n * mat_ld(NP)] * s1[n].x;
            sums[5] += PLlast[(size_t)n * mat_ld(NP)] * s1[n].y;
        }
    }
    bsum<MT>(sums, red);
    const double2 e0 = c2(sums[0], sums[1]), e1 = c2(sums[2], sums[3]), p0last = c2(sums[4], sums[5]);
    const double tn = 2.0 * (N - 1);
    const double2 e2 = csub(cadd(cscl(c.sig, v0[N - 2]), cscl(tn, p0last)), Fy[N - 2]);
    const double2 e3 = csub(cscl(c.sig, v0[N - 1]), Fy[N - 1]);
    const double* Ai = T.Ai;
    double2 cc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double2 sk = cadd(cadd(cscl(Ai[4 * k], e0), cscl(Ai[4 * k + 1], e1)),
                          cadd(cscl(Ai[4 * k + 2], e2), cscl(Ai[4 * k + 3], e3)));
        cc[k] = cscl(-1.0, sk);
    }
    const double* Vk = T.Vk;     // row k at Vk[k * NP]
    const double* DVk = T.DVk;
    for (int n = t; n < N; n += MT) {
        double2 v = v0[n], Dv = Dv0[n];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v = cadd(v, cscl(Vk[k * NP + n], cc[k]));
            Dv = cadd(Dv, cscl(DVk[k * NP + n], cc[k]));
        }
        const double2 e = eta[n];
        ox[n] = cscl(c.ik2, csub(imul(c.a, Dv), imul(c.b, e)));
        oy[n] = v;
        oz[n] = cscl(c.ik2, cadd(imul(c.b, Dv), imul(c.a, e)));
    }
    __syncthreads();
}

// Conjugate transpose of stokes(): (yx, yy, yz) = S^H (xu, xv, xw), the steps
// above run backwards with every matrix transposed (three contraction phases).
// w: 11 scratch vectors.
template <int NP, int MT>
__device__ void stokes_h(const KP& p, const ModeTabs& T, const MS& c, const double2* xu, const double2* xv,
                         const double2* xw, double2* yx, double2* yy, double2* yz,
                         double2* w, double* red) {
    const int N = p.N, M = N - 2, t = threadIdx.x;
    double2 *bDv = w, *beta = w + NP, *bv0 = w + 2 * NP, *bDv0 = w + 3 * NP, *bt2 = w + 4 * NP,
            *tmp = w + 5 * NP, *bte = w + 6 * NP, *bFh = w + 7 * NP, *bFe = w + 8 * NP,
            *bFy = w + 9 * NP, *bFy2 = w + 10 * NP;
    const double* dH = T.dH;
    const double* dP = T.dP;
    const double* Vk = T.Vk;     // row k at Vk[k * NP]
    const double* DVk = T.DVk;
    double dots[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int n = t; n < N; n += MT) {
        const double2 a0 = xu[n], a2 = xw[n], bv = xv[n];
        const double2 bd = cscl(c.ik2, cadd(imul(-c.a, a0), imul(-c.b, a2)));
        bDv[n] = bd;
        beta[n] = cscl(c.ik2, csub(imul(c.b, a0), imul(c.a, a2)));
#pragma unroll
        for (int k = 0; k < 4; ++k) {   // v = v0 + Vk^T c and Dv = Dv0 + DVk^T c
            dots[2 * k] += Vk[k * NP + n] * bv.x + DVk[k * NP + n] * bd.x;
            dots[2 * k + 1] += Vk[k * NP + n] * bv.y + DVk[k * NP + n] * bd.y;
        }
    }
    bsum<MT>(dots, red);
    const double* Ai = T.Ai;
    double2 be[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double2 sj = c2(0, 0);
#pragma unroll
        for (int k = 0; k < 4; ++k) sj = cadd(sj, cscl(Ai[4 * k + j], c2(dots[2 * k], dots[2 * k + 1])));
        be[j] = cscl(-1.0, sj);
    }
    for (int n = t; n < N; n += MT) {
        double2 x = xv[n];
        if (n == N - 2) x = cadd(x, cscl(c.sig, be[2]));
        if (n == N - 1) x = cadd(x, cscl(c.sig, be[3]));
        bv0[n] = x;
        bDv0[n] = cadd(bDv[n], (n & 1) ? csub(be[0], be[1]) : cadd(be[0], be[1]));
    }
    __syncthreads();
    mv<NP, MT>(p, M_PLT, M, bv0, bt2);
    mv_ep<NP, MT>(p, M_DPLT, M, bDv0, [&](int n, double2 v) {
        bt2[n] = cscl(dH[n], cadd(bt2[n], v));   // u2 = dH (PL^T bv0 + DPL^T bDv0)
    });
    mv_ep<NP, MT>(p, M_PLT, M, beta, [&](int n, double2 v) { bte[n] = cscl(dH[n], v); });   // bs2
    __syncthreads();
    const double2 bp0last = cscl(2.0 * (N - 1), be[2]);
    const double* PLlast = mat<NP>(p, M_PL) + (N - 1);
    mv_ep<NP, MT>(p, M_PRDPLT, M, bt2, [&](int n, double2 v) {   // bs1 = -dP (Pl[N-1,:] bp0last - PRDPL^T u2)
        tmp[n] = cscl(-dP[n], csub(cscl(PLlast[(size_t)n * mat_ld(NP)], bp0last), v));
    });
    __syncthreads();
    mv3<NP, MT>(p, M_PRT, M, tmp, bte, bt2, bFh, bFe, bFy);
    mv<NP, MT>(p, M_PRDT, N, tmp, bFy2);
    __syncthreads();
    for (int n = t; n < N; n += MT) {
        const double2 h = (n < M) ? bFh[n] : c2(0, 0), e = (n < M) ? bFe[n] : c2(0, 0);
        double2 y = cadd((n < M) ? bFy[n] : c2(0, 0), bFy2[n]);
        if (n == N - 2) y = csub(y, be[2]);
        if (n == N - 1) y = csub(y, be[3]);
        yx[n] = cadd(imul(-c.a, h), imul(-c.b, e));
        yy[n] = y;
        yz[n] = cadd(imul(-c.b, h), imul(c.a, e));
    }
    __syncthreads();
}

template <int NP, int MT>
__device__ void stokes0(const KP& p, const ModeTabs& T, const double2* Fx, const double2* Fz, double2* ox,
                        double2* oy, double2* oz, double2* w) {
    const int N = p.N, M = N - 2, t = threadIdx.x;
    double2 *t1 = w, *t2 = w + NP;
    const double* dH = T.dH;
    mv<NP, MT>(p, M_PR, M, Fx, t1);
    mv<NP, MT>(p, M_PR, M, Fz, t2);
    __syncthreads();
    for (int n = t; n < M; n += MT) {
        t1[n] = cscl(dH[n], t1[n]);
        t2[n] = cscl(dH[n], t2[n]);
    }
    __syncthreads();
    mv<NP, MT>(p, M_PL, N, t1, ox);
    mv<NP, MT>(p, M_PL, N, t2, oz);
    for (int n = t; n < N; n += MT) oy[n] = c2(0, 0);
    __syncthreads();
}

template <int NP, int MT>
__device__ void stokes0_h(const KP& p, const ModeTabs& T, const double2* xu, const double2* xw, double2* yx,
                          double2* yy, double2* yz, double2* w) {
    const int N = p.N, M = N - 2, t = threadIdx.x;
    double2 *t1 = w, *t2 = w + NP;
    const double* dH = T.dH;
    mv<NP, MT>(p, M_PLT, M, xu, t1);
    mv<NP, MT>(p, M_PLT, M, xw, t2);
    __syncthreads();
    for (int n = t; n < M; n += MT) {
        t1[n] = cscl(dH[n], t1[n]);
        t2[n] = cscl(dH[n], t2[n]);
    }
    __syncthreads();
    mv<NP, MT>(p, M_PRT, M, t1, yx);
    mv<NP, MT>(p, M_PRT, M, t2, yz);
    for (int n = t; n < N; n += MT) {
        yy[n] = c2(0, 0);
        if (n >= M) {
            yx[n] = c2(0, 0);
            yz[n] = c2(0, 0);
        }
    }
    __syncthreads();
}

// W-orthogonal projection onto divergence-free no-slip fields (kappa > 0) in
// the (v, eta) parametrisation: the W-Gram matrix is block diagonal there,
// the eta block is the fixed G-orthogonal Dirichlet projector and the v block
// is diagonalised by fixed vectors X with diagonal 1/(1 + Lambda/kappa^2).
// Three contraction phases.  w: 8 scratch vectors.
template <int NP, int MT>
__device__ void project(const KP& p, const ModeTabs& T, const MS& c, const double2* gx, const double2* gy,
                        const double2* gz, double2* ox, double2* oy, double2* oz, double2* w) {
    const int N = p.N, t = threadIdx.x;
    double2 *gh = w, *ge = w + NP, *t1 = w + 2 * NP, *t2 = w + 3 * NP, *t4 = w + 4 * NP,
            *v = w + 5 * NP, *eta = w + 6 * NP, *Dv = w + 7 * NP;
    const double* dq = T.dq;
    for (int n = t; n < N; n += MT) {
        const double2 x = gx[n], z = gz[n];
        gh[n] = cadd(imul(c.a, x), imul(c.b, z));
        ge[n] = csub(imul(c.b, x), imul(c.a, z));
    }
    __syncthreads();
    mv<NP, MT>(p, M_DTG, N, gh, t1);
    mv_ep<NP, MT>(p, M_G, N, gy, [&](int n, double2 v) { t2[n] = csub(v, cscl(c.ik2, t1[n])); });
    mv<NP, MT>(p, M_PID, N, ge, eta);
    __syncthreads();
    mv_ep<NP, MT>(p, M_PVLT, N - 4, t2, [&](int n, double2 v) { t4[n] = cscl(dq[n], v); });
    __syncthreads();
    mv<NP, MT>(p, M_PVL, N, t4, v);
    mv<NP, MT>(p, M_DPVL, N, t4, Dv);
    __syncthreads();
    for (int n = t; n < N; n += MT) {
        const double2 d = Dv[n], e = eta[n];
        ox[n] = cscl(c.ik2, csub(imul(c.a, d), imul(c.b, e)));
        oy[n] = v[n];
        oz[n] = cscl(c.ik2, cadd(imul(c.b, d), imul(c.a, e)));
    }
    __syncthreads();
}

template <int NP, int MT>
__device__ void project0(const KP& p, const double2* gx, const double2* gz, double2* ox,
                         double2* oy, double2* oz) {
    const int N = p.N;
    mv<NP, MT>(p, M_PID, N, gx, ox);
    mv<NP, MT>(p, M_PID, N, gz, oz);
    for (int n = threadIdx.x; n < N; n += MT) oy[n] = c2(0, 0);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// y-values of u and of du/dy for the three components: Y[c] = C u_c,
// Y[3+c] = C D u_c (Gauss-Lobatto synthesis).
template <int NP, int MT, class YT>
__device__ __forceinline__ void synth_body(const KP& p, int mB, const double2* __restrict__ u,
                                           YT* __restrict__ Y) {
    const int N = p.N, nm = p.nm, nmB = p.nmB, t = threadIdx.x;
    if (mB >= nmB) return;
    const int b = mB / nm, m = mB - b * nm;   // guess, Fourier mode
    const size_t so = (size_t)b * 3 * nm * N; // offset of this guess in spectral arrays
    double2* V = mode_vectors<NP, MT>();
    read_field3<MT>(p, u, so, m, V, V + NP, V + 2 * NP);
    __syncthreads();
    mv3<NP, MT>(p, M_C, N, V, V + NP, V + 2 * NP, V + 3 * NP, V + 4 * NP, V + 5 * NP);
    mv3<NP, MT>(p, M_CD, N, V, V + NP, V + 2 * NP, V + 6 * NP, V + 7 * NP, V + 8 * NP);
    __syncthreads();
    for (int f = 0; f < 6; ++f)
        for (int j = t; j < N; j += MT)
            Y[((size_t)f * N + j) * nmB + mB] = narrow<YT>(V[(3 + f) * NP + j]);
}

template <int MODE, class R, int PLANE_THREADS>
__device__ __forceinline__ void plane_body(const KP& p, int item, const C<R>* __restrict__ Y1,
                                           const C<R>* __restrict__ Y2, C<R>* __restrict__ out) {
    typedef C<R> CR;
    extern __shared__ __align__(16) unsigned char smraw[];
    CR* sm = reinterpret_cast<CR*>(smraw);
    const R zero = 0, two = 2, alpha = (R)p.alpha, beta = (R)p.beta;
    constexpr int NG3 = (MODE == PLANE_JVP) ? 6 : 3;  // velocity fields: (V, i a V, W) groups
    constexpr int NG1 = (MODE == PLANE_ADJ) ? 3 : 0;  // adjoint fields: single outputs
    constexpr int NXF = 3 * NG3 + NG1;
    constexpr int NZF = (MODE == PLANE_ADJ) ? 9 : 3;  // after the forward z stage
    static_assert(NG1 == 0 || NG1 == NG3, "adjoint fields pair with the velocity groups");
    if (item >= p.B * p.NS * p.N) return;
    const int jb = item / p.NS, s = item - jb * p.NS;   // the slabs of a plane run on one XCD
    const int b = jb / p.N, j = jb - b * p.N;          // guess, Gauss-Lobatto plane
    const int N = p.N, Nx = p.Nx, Nz = p.Nz, nkx = p.nkx, nkz = p.nkz, nm = p.nm, XS = p.XS;
    const int nmB = p.nmB, mo = b * nm;                // y-value arrays are [f][j][b * nm + m]
    const int Kx = p.Kx;
    const int tid = threadIdx.x;
    // LDS rows are padded: the kz rows of the spectral buffer xb and of the z
    // twiddles to kz_row(nkz) entries (twice an odd number), the products pb
    // to Nz + 1.  Lanes at neighbouring x or z then start in different banks,
    // also where the two lanes of a pair read neighbouring kz.
    const int per = XS * nkz, tzs = kz_row(nkz);
    const int ldz = kz_row(nkz), pfs = XS * ldz, ldq = Nz + 1, pz = XS * ldq;
    // The slab holds the points x = s + NS xl (xl < XS): since
    //   exp(2 pi i kx x / Nx) = exp(2 pi i kx s / Nx) exp(2 pi i (kx mod XS) xl / XS),
    // its x transforms split into a fold of the retained kx by kx mod XS (with
    // the slab's phase) and an XS-point DFT.
    // Twiddle tables: TS[ikx] = exp(2 pi i kx s / Nx) for every retained kx,
    // TD[xl][q] = exp(2 pi i q xl / XS) (symmetric), TZ[z][kz] =
    // exp(2 pi i kz z / Nz) with padded rows, so that lanes running over kz
    // (forward z transform) and lanes running over z (inverse z transform)
    // both read distinct LDS banks.  With Nz even TZ holds the
    // rows z < Nz/2 only: the twiddles of z + Nz/2 are (-1)^kz times those of z.
    const int nzt = (Nz & 1) ? Nz : Nz / 2;
    CR* TS = sm;
    CR* TD = TS + nkx;
    CR* TZ = TD + XS * XS;
    CR* xb = TZ + nzt * tzs;
    R* pb = reinterpret_cast<R*>(xb + NXF * pfs);
    // The folded arrays (inverse x) and the XS-point DFTs (forward x) use the
    // products buffer, which is not live at those times: array a at
    // zb[a * pfs + q * ldz + kz].
    CR* zb = reinterpret_cast<CR*>(pb);
    // Set-up of the twiddle tables, entry i of each.  Every index is reduced
    // mod Nx or Nz, so the loads are in bounds for any i and only the stores
    // are guarded.  The first pass's loads are issued here and its stores
    // made after the fold below, so the two sets of global reads are in
    // flight together; the tables are published by the fold's barrier (the
    // fold itself reads the slab phases from global memory).
    const int ntd = XS * XS, ntz = nzt * nkz, nset = max(max(nkx, ntd), ntz);
    auto tw_load = [&](int i, double2 (&v)[3]) {
        const int kx = (i <= Kx) ? i : i - nkx;   // kx + Nx > 0 for every i
        const int xl = i / XS, q = i - xl * XS;
        const int z = i / nkz, kz = i - z * nkz;
        v[0] = p.twx[(kx + Nx) * s % Nx];
        v[1] = p.twx[(q * xl) % XS * p.NS];
        v[2] = p.twz[(kz * z) % Nz];
    };
    auto tw_store = [&](int i, const double2 (&v)[3]) {
        const int z = i / nkz, kz = i - z * nkz;
        if (i < nkx) TS[i] = narrow<CR>(v[0]);
        if (i < ntd) TD[i] = narrow<CR>(v[1]);
        if (i < ntz) TZ[z * tzs + kz] = narrow<CR>(v[2]);
    };
    double2 tw0[3];
    tw_load(tid, tw0);

    // Inverse transform in x for the slab's points, all retained kz, in chunks
    // of up to three velocity groups g (fields V, i a V, W; in the adjoint
    // variant the adjoint field g too, NG1 == NG3 there).
    //  fold: work item (g, q, kz) forms, over the retained kx = q (mod XS),
    //        Z[q] = sum Y[kx] exp(2 pi i kx s / Nx) for V, kx V, W (and A);
    //        every y-value of the plane is read once, from global memory;
    //  DFT:  work item (g, xl, kz) forms sum_q Z[q] exp(2 pi i q xl / XS).
    constexpr int NZA = NG1 > 0 ? 4 : 3;     // folded arrays per group
    constexpr int GCH = NG3 < 3 ? NG3 : 3;   // groups per chunk
    // XS-point DFTs (here and in the forward x transform) pair the outputs
    // q and q + XS/2 (points xl and xl + XS/2) when XS is even
    const int npx = (XS & 1) ? 1 : 2, hxs = (XS & 1) ? XS : XS / 2, perx = hxs * nkz;
    for (int g0 = 0; g0 < NG3; g0 += GCH) {
        for (int it = tid; it < GCH * per; it += PLANE_THREADS) {
            const int gc = it / per, rem = it - gc * per, q = rem / nkz, kz = rem - q * nkz;
            const int g = g0 + gc;
            const CR* src = (g < 3) ? Y1 : Y2;
            const int comp = g % 3;
            const CR* Vp = src + ((size_t)comp * N + j) * nmB + mo + kz;
            const CR* Wp = src + ((size_t)(3 + comp) * N + j) * nmB + mo + kz;
            const CR* Ap = (NG1 > 0) ? Y2 + ((size_t)g * N + j) * nmB + mo + kz : nullptr;
            CR zV = mkc(zero, zero), zK = zV, zW = zV, zA = zV;
            // the retained kx = q (mod XS) are kx0 + XS t (t < cnt), with slab
            // phase exp(2 pi i kx s / Nx) at twx[ti], ti stepping by XS s < Nx;
            // the terms go in batches of FB whose loads issue together: past
            // the last term the index is clamped and the phase set to zero, so
            // no use of a load is conditional (the compiler would otherwise
            // sink each load to its use and wait for it there)
            constexpr int FB = 4;
            const int kx0 = -Kx + (q + Kx) % XS;
            const int cnt = (kx0 <= Kx) ? (Kx - kx0) / XS + 1 : 0;
            const int dts = XS * s;
            int ti = (kx0 + Nx) * s % Nx;
            for (int t0 = 0; t0 < cnt; t0 += FB) {
                CR tw[FB], yv[FB], yw[FB], ya[FB];
#pragma unroll
                for (int u = 0; u < FB; ++u) {
                    const int kx = kx0 + XS * min(t0 + u, cnt - 1);
                    const size_t ikx = (size_t)((kx >= 0) ? kx : kx + nkx) * nkz;
                    const CR t = narrow<CR>(p.twx[ti]);
                    const bool live = t0 + u < cnt;
                    tw[u] = mkc(live ? t.x : zero, live ? t.y : zero);
                    ti += dts;
                    if (ti >= Nx) ti -= Nx;
                    yv[u] = Vp[ikx];
                    yw[u] = Wp[ikx];
                    if constexpr (NG1 > 0) ya[u] = Ap[ikx];
                }
#pragma unroll
                for (int u = 0; u < FB; ++u) {
                    const R kx = (R)(kx0 + XS * (t0 + u));
                    const CR vt = cmul(yv[u], tw[u]);
                    zV = cadd(zV, vt);
                    zK = mkc(fmar(kx, vt.x, zK.x), fmar(kx, vt.y, zK.y));
                    zW = cmac(zW, yw[u], tw[u]);
                    if constexpr (NG1 > 0) zA = cmac(zA, ya[u], tw[u]);
                }
            }
            CR* zo = zb + (size_t)(NZA * gc) * pfs + q * ldz + kz;
            zo[0] = zV;
            zo[pfs] = zK;
            zo[2 * pfs] = zW;
            if constexpr (NG1 > 0) zo[3 * pfs] = zA;
        }
        if (g0 == 0) {
            tw_store(tid, tw0);
#pragma unroll 1
            for (int i = tid + PLANE_THREADS; i < nset; i += PLANE_THREADS) {
                double2 v[3];
                tw_load(i, v);
                tw_store(i, v);
            }
        }
        __syncthreads();
        // With XS even an item takes the points xl and xl + XS/2: their
        // twiddles differ by (-1)^q, so the even- and odd-q sums give both.
        for (int it = tid; it < GCH * perx; it += PLANE_THREADS) {
            const int gc = it / perx, rem = it - gc * perx, xl = rem / nkz, kz = rem - xl * nkz;
            const int g = g0 + gc;
            const CR* zi = zb + (size_t)(NZA * gc) * pfs + kz;
            const CR* td = TD + xl * XS;
            CR e[4], o[4];   // V, kx V, W, A: even- and odd-q sums
#pragma unroll
            for (int i = 0; i < 4; ++i) e[i] = o[i] = mkc(zero, zero);
            auto term = [&](int q, CR (&a)[4]) {
                const CR tw = td[q];
#pragma unroll
                for (int i = 0; i < NZA; ++i) a[i] = cmac(a[i], zi[i * pfs + q * ldz], tw);
            };
            for (int q = 0; q + 1 < XS; q += 2) {
                term(q, e);
                term(q + 1, o);
            }
            if (XS & 1) term(XS - 1, e);   // odd XS: unpaired, a single point from e + o
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h >= npx) break;
                const int xo = (xl + h * hxs) * ldz + kz;
                CR a[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = h ? csub(e[i], o[i]) : cadd(e[i], o[i]);
                xb[(3 * g) * pfs + xo] = a[0];
                xb[(3 * g + 1) * pfs + xo] = imul(alpha, a[1]);
                xb[(3 * g + 2) * pfs + xo] = a[2];
                if constexpr (NG1 > 0) xb[(3 * NG3 + g) * pfs + xo] = a[3];
            }
        }
        __syncthreads();
    }

    // inverse (complex-to-real) transform in z, then the products.  Per
    // velocity field the kz sums give U, dU/dx, dU/dy, dU/dz: Re of the sums,
    // the kz > 0 terms doubled (real field), kz weights applied in the loop,
    // beta at the end; one twiddle load per kz serves every field.  With Nz
    // even but not a multiple of 4 (a multiple of 4: mirrored points, below)
    // the lanes 2k and 2k + 1 take the points z and z + Nz/2 of one x,
    // whose twiddles differ by (-1)^kz: the first sums the odd kz, its partner
    // the even kz > 0, and an exchange of the sums between the two lanes gives
    // each its point (even + odd, even - odd).  With Nz odd a lane takes one
    // point and sums every kz.
    const R yj = (R)p.ygl[j];
    constexpr int NA = NG1 > 0 ? NG1 : 1;
    const bool pair = !(Nz & 1);
    const int hz = pair ? Nz / 2 : Nz;   // = nzt: the twiddle rows cover z < hz
    // With Nz a multiple of 4 a lane pair takes the four points z, Nz - z,
    // z + Nz/2 and Nz/2 - z (0 <= z <= Nz/4) of one x.  With
    // w = exp(2 pi i kz z / Nz) their twiddles are w, conj(w), (-1)^kz w and
    // (-1)^kz conj(w), so Re(c w) = c.x cos - c.y sin and its mirror
    // c.x cos + c.y sin share one read of c and of w: lane pc sums the kz of
    // parity pc (0 even, 1 odd) as c.x cos and c.y sin per value field and as
    // kz c.y cos and kz c.x sin per velocity field (dU/dz), and an exchange
    // of the combined sums between the two lanes gives lane 0 the points z
    // and Nz - z, lane 1 the points z + Nz/2 and Nz/2 - z.  For z = 0 and
    // z = Nz/4 the second points repeat first ones and are not stored.
    const bool mirror = !(Nz & 3);
    if (mirror) {
        const int q4 = Nz / 4, nq = q4 + 1;
        for (int it = tid; it < 2 * XS * nq; it += PLANE_THREADS) {
            const int pc = it & 1, qd = it >> 1;
            const int xl = qd / nq, z = qd - xl * nq;
            const CR* c0 = xb + xl * ldz;   // field f at c0[f * pfs + kz]
            const CR* tz = TZ + z * tzs;
            R va[NG3][3], vb[NG3][3], vc[NG3], vd[NG3], aa[NA], ab[NA];
#pragma unroll
            for (int g = 0; g < NG3; ++g) {
                vc[g] = vd[g] = 0;
#pragma unroll
                for (int q = 0; q < 3; ++q) va[g][q] = vb[g][q] = 0;
            }
#pragma unroll
            for (int i = 0; i < NA; ++i) aa[i] = ab[i] = 0;
            for (int kz = 2 - pc; kz < nkz; kz += 2) {
                const CR tw = tz[kz];
                const R kc = (R)kz * tw.x, ks = (R)kz * tw.y;
#pragma unroll
                for (int g = 0; g < NG3; ++g) {
                    const CR cV = c0[(3 * g) * pfs + kz], cA = c0[(3 * g + 1) * pfs + kz], cW = c0[(3 * g + 2) * pfs + kz];
                    va[g][0] = fmar(cV.x, tw.x, va[g][0]);
                    vb[g][0] = fmar(cV.y, tw.y, vb[g][0]);
                    vd[g] = fmar(cV.y, kc, vd[g]);
                    vc[g] = fmar(cV.x, ks, vc[g]);
                    va[g][1] = fmar(cA.x, tw.x, va[g][1]);
                    vb[g][1] = fmar(cA.y, tw.y, vb[g][1]);
                    va[g][2] = fmar(cW.x, tw.x, va[g][2]);
                    vb[g][2] = fmar(cW.y, tw.y, vb[g][2]);
                }
#pragma unroll
                for (int i = 0; i < NG1; ++i) {
                    const CR cc = c0[(3 * NG3 + i) * pfs + kz];
                    aa[i] = fmar(cc.x, tw.x, aa[i]);
                    ab[i] = fmar(cc.y, tw.y, ab[i]);
                }
            }
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {   // first point (z or z + Nz/2), then its mirror
                const R m = h2 ? (R)1 : (R)-1;
                // own parity's sum for this point, then the parities add (lane 0)
                // or subtract (lane 1) with the partner's
                auto tot = [&](R u) {
                    const R y = lane_pair_swap(u);
                    return pc ? y - u : u + y;
                };
                R val[NG3][4], at[NA];
#pragma unroll
                for (int g = 0; g < NG3; ++g) {
                    val[g][0] = c0[(3 * g) * pfs].x + two * tot(fmar(m, vb[g][0], va[g][0]));
                    val[g][1] = c0[(3 * g + 1) * pfs].x + two * tot(fmar(m, vb[g][1], va[g][1]));
                    val[g][2] = c0[(3 * g + 2) * pfs].x + two * tot(fmar(m, vb[g][2], va[g][2]));
                    val[g][3] = -two * beta * tot(fmar(-m, vc[g], vd[g]));
                }
#pragma unroll
                for (int i = 0; i < NG1; ++i) at[i] = c0[(3 * NG3 + i) * pfs].x + two * tot(fmar(m, ab[i], aa[i]));
                val[0][0] += yj;   // base flow u_b = y e_x
                val[0][2] += (R)1; // d(u_b)_x / dy = 1
                // the point z' < Nz/2 of each (z', z' + Nz/2) pair stores the sum
                // of the two products, the other the difference, as the forward
                // z transform reads them
                const bool lower = pc == h2, wr = !(h2 && (z == 0 || z == q4));
                const int zp = pc ? (h2 ? Nz / 2 - z : z + Nz / 2) : (h2 ? Nz - z : z);
                const int pt = xl * ldq + zp;
                auto put = [&](int f, R q) {
                    const R w = lane_pair_swap(q);
                    if (wr) pb[f * pz + pt] = lower ? q + w : w - q;
                };
                if (MODE == PLANE_FWD) {
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        put(i, val[0][0] * val[i][1] + val[1][0] * val[i][2] + val[2][0] * val[i][3]);
                } else if (MODE == PLANE_JVP) {
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        R q = 0;
#pragma unroll
                        for (int jj = 0; jj < 3; ++jj)
                            q += val[jj][0] * val[3 + i][1 + jj] + val[3 + jj][0] * val[i][1 + jj];
                        put(i, q);
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int jj = 0; jj < 3; ++jj) put(3 * i + jj, val[jj][0] * at[i]);
#pragma unroll
                    for (int jj = 0; jj < 3; ++jj)
                        put(9 + jj, val[0][1 + jj] * at[0] + val[1][1 + jj] * at[1] + val[2][1 + jj] * at[2]);
                }
            }
        }
    } else {
        // items XS * Nz (even with Nz even): lane pairs are active together
        for (int it = tid; it < XS * Nz; it += PLANE_THREADS) {
            const int h = pair ? (it & 1) : 0, pr = pair ? (it >> 1) : it;
            const int xl = pr / hz, z = pr - xl * hz;
            const CR* c0 = xb + xl * ldz;   // field f at c0[f * pfs + kz]
            const CR* tz = TZ + z * tzs;
            R v[NG3][4], a[NA];
    #pragma unroll
            for (int g = 0; g < NG3; ++g)
    #pragma unroll
                for (int q = 0; q < 4; ++q) v[g][q] = 0;
    #pragma unroll
            for (int i = 0; i < NA; ++i) a[i] = 0;
            const int kst = pair ? 2 : 1;
            for (int kz = 1 + h; kz < nkz; kz += kst) {
                const CR tw = tz[kz];
                const R kzr = (R)kz;
    #pragma unroll
                for (int g = 0; g < NG3; ++g) {
                    const CR cV = c0[(3 * g) * pfs + kz], cA = c0[(3 * g + 1) * pfs + kz], cW = c0[(3 * g + 2) * pfs + kz];
                    v[g][0] = fmar(-cV.y, tw.y, fmar(cV.x, tw.x, v[g][0]));
                    v[g][3] = fmar(kzr, fmar(cV.y, tw.x, cV.x * tw.y), v[g][3]);
                    v[g][1] = fmar(-cA.y, tw.y, fmar(cA.x, tw.x, v[g][1]));
                    v[g][2] = fmar(-cW.y, tw.y, fmar(cW.x, tw.x, v[g][2]));
                }
    #pragma unroll
                for (int i = 0; i < NG1; ++i) {
                    const CR cc = c0[(3 * NG3 + i) * pfs + kz];
                    a[i] = fmar(-cc.y, tw.y, fmar(cc.x, tw.x, a[i]));
                }
            }
            // own sums S and the partner's P: point z is S + P (h = 0, S odd),
            // point z + Nz/2 is S - P (h = 1, S even)
            const R sg = h ? (R)-1 : (R)1;
            auto tot = [&](R own) { return pair ? own + sg * lane_pair_swap(own) : own; };
            R val[NG3][4], at[NA];
    #pragma unroll
            for (int g = 0; g < NG3; ++g) {
                val[g][0] = c0[(3 * g) * pfs].x + two * tot(v[g][0]);
                val[g][1] = c0[(3 * g + 1) * pfs].x + two * tot(v[g][1]);
                val[g][2] = c0[(3 * g + 2) * pfs].x + two * tot(v[g][2]);
                val[g][3] = -two * beta * tot(v[g][3]);
            }
    #pragma unroll
            for (int i = 0; i < NG1; ++i) at[i] = c0[(3 * NG3 + i) * pfs].x + two * tot(a[i]);
            val[0][0] += yj;   // base flow u_b = y e_x
            val[0][2] += (R)1; // d(u_b)_x / dy = 1
            // product f at this point; a lane pair stores the sum of its two
            // products at z and their difference at z + Nz/2, which the forward z
            // transform reads for even and odd kz respectively
            const int pt = xl * ldq + z + h * hz;
            auto put = [&](int f, R q) {
                if (pair) {
                    const R w = lane_pair_swap(q);
                    pb[f * pz + pt] = h ? w - q : q + w;
                } else {
                    pb[f * pz + pt] = q;
                }
            };
            if (MODE == PLANE_FWD) {
    #pragma unroll
                for (int i = 0; i < 3; ++i)
                    put(i, val[0][0] * val[i][1] + val[1][0] * val[i][2] + val[2][0] * val[i][3]);
            } else if (MODE == PLANE_JVP) {
    #pragma unroll
                for (int i = 0; i < 3; ++i) {
                    R q = 0;
    #pragma unroll
                    for (int jj = 0; jj < 3; ++jj)
                        q += val[jj][0] * val[3 + i][1 + jj] + val[3 + jj][0] * val[i][1 + jj];
                    put(i, q);
                }
            } else {
    #pragma unroll
                for (int i = 0; i < 3; ++i)
    #pragma unroll
                    for (int jj = 0; jj < 3; ++jj) put(3 * i + jj, val[jj][0] * at[i]);
    #pragma unroll
                for (int jj = 0; jj < 3; ++jj)
                    put(9 + jj, val[0][1 + jj] * at[0] + val[1][1 + jj] * at[1] + val[2][1 + jj] * at[2]);
            }
        }
    }
    __syncthreads();

    // forward transform in z (normalised), into xb.  Adjoint variant: work item
    // (i, xl, kz) forms the three outputs of component i, sharing the twiddles.
    // With Nz even the sum runs over z < Nz/2 of q[z] + (-1)^kz q[z + Nz/2],
    // which the products stage stored (at z for even kz, at z + Nz/2 for odd).
    const R invNz = (R)1 / (R)Nz, invNx = (R)1 / (R)Nx;
    constexpr int NZI = (MODE == PLANE_ADJ) ? 3 : NZF;
    for (int it = tid; it < NZI * per; it += PLANE_THREADS) {
        const int o = it / per, rem = it - o * per, xl = rem / nkz, kz = rem - xl * nkz;
        const CR* tzk = TZ + kz;   // tzk[z * tzs] = exp(2 pi i kz z / Nz)
        const int ko = xl * ldq + ((pair && (kz & 1)) ? hz : 0);   // row of the stored sums
        if (MODE != PLANE_ADJ) {
            const R* q = pb + o * pz + ko;
            R ar = 0, ai = 0;
            for (int z = 0; z < nzt; ++z) {
                const CR tw = tzk[z * tzs];
                const R v = q[z];
                ar = fmar(v, tw.x, ar);
                ai = fmar(-v, tw.y, ai);
            }
            xb[o * pfs + xl * ldz + kz] = mkc(ar * invNz, ai * invNz);
        } else {
            const int i = o;
            const R* q1 = pb + (9 + i) * pz + ko;      // Q_i
            const R* q2 = pb + (3 * i + 2) * pz + ko;  // P_{i,z}
            const R* qx = pb + (3 * i) * pz + ko;      // P_{i,x}
            const R* qy = pb + (3 * i + 1) * pz + ko;  // P_{i,y}
            R ar = 0, ai = 0, br = 0, bi = 0, xr = 0, xi = 0, yr = 0, yi = 0;
            for (int z = 0; z < nzt; ++z) {
                const CR tw = tzk[z * tzs];
                const R v1 = q1[z], v2 = q2[z], vx = qx[z], vy = qy[z];
                ar = fmar(v1, tw.x, ar);
                ai = fmar(-v1, tw.y, ai);
                br = fmar(v2, tw.x, br);
                bi = fmar(-v2, tw.y, bi);
                xr = fmar(vx, tw.x, xr);
                xi = fmar(-vx, tw.y, xi);
                yr = fmar(vy, tw.x, yr);
                yi = fmar(-vy, tw.y, yi);
            }
            const int xo = xl * ldz + kz;
            xb[(3 * i) * pfs + xo] = cscl(invNz, csub(mkc(ar, ai), imul(beta * (R)kz, mkc(br, bi))));  // Q_i - i b P_{i,z}
            xb[(3 * i + 1) * pfs + xo] = mkc(xr * invNz, xi * invNz);
            xb[(3 * i + 2) * pfs + xo] = mkc(yr * invNz, yi * invNz);
        }
    }
    __syncthreads();

    // Forward transform in x over this slab (partial sum), retained modes only.
    //  DFT: work item (f, q, kz) forms F[f][q] = sum_xl v[f][xl] exp(-2 pi i q xl / XS);
    //  per mode (kx, kz): F[f][kx mod XS] exp(-2 pi i kx s / Nx) / Nx.
    // The adjoint outputs are X_i = F(A_i) - i a kx F(B_i) and Y_i = F(C_i) from
    // the fields (A_i, B_i, C_i) = xb fields (3 i, 3 i + 1, 3 i + 2).
    constexpr int NOUT = (MODE == PLANE_ADJ) ? 6 : 3;
    constexpr int NIN = (MODE == PLANE_ADJ) ? 9 : 3;
    // With XS even an item forms F[q] and F[q + XS/2] from the even- and
    // odd-xl sums (their twiddles differ by (-1)^xl).
    for (int it = tid; it < NIN * perx; it += PLANE_THREADS) {
        const int f = it / perx, rem = it - f * perx, q = rem / nkz, kz = rem - q * nkz;
        const CR* v = xb + f * pfs + kz;
        const CR* td = TD + q * XS;
        R er = 0, ei = 0, orr = 0, oi = 0;
        auto term = [&](int xl, R& ar, R& ai) {   // (ar, ai) += v conj(tw)
            const CR tw = td[xl], x = v[xl * ldz];
            ar = fmar(x.y, tw.y, fmar(x.x, tw.x, ar));
            ai = fmar(-x.x, tw.y, fmar(x.y, tw.x, ai));
        };
        for (int xl = 0; xl + 1 < XS; xl += 2) {
            term(xl, er, ei);
            term(xl + 1, orr, oi);
        }
        if (XS & 1) term(XS - 1, er, ei);
        zb[f * pfs + q * ldz + kz] = mkc(er + orr, ei + oi);
        if (npx == 2) zb[f * pfs + (q + hxs) * ldz + kz] = mkc(er - orr, ei - oi);
    }
    __syncthreads();
    for (int mm = tid; mm < nm; mm += PLANE_THREADS) {
        const int ikx = mm / nkz, kz = mm - ikx * nkz;
        const int kx = (ikx <= Kx) ? ikx : ikx - nkx;
        const int q = ((kx % XS) + XS) % XS;
        const CR ts = TS[ikx];
        const CR* fi = zb + q * ldz + kz;   // F[f][q] at fi[f * pfs]
        // (x + i y) conj(ts) / Nx
        auto out1 = [&](CR v) {
            return mkc(fmar(v.y, ts.y, v.x * ts.x) * invNx, fmar(-v.x, ts.y, v.y * ts.x) * invNx);
        };
        CR* o0 = out + ((size_t)s * NOUT * N + j) * nmB + mo + mm;   // output o at o0[o * N * nmB]
        const size_t os = (size_t)N * nmB;
        if (MODE != PLANE_ADJ) {
#pragma unroll
            for (int o = 0; o < 3; ++o) o0[o * os] = out1(fi[o * pfs]);
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                o0[i * os] = out1(csub(fi[(3 * i) * pfs], imul(alpha * (R)kx, fi[(3 * i + 1) * pfs])));
                o0[(3 + i) * os] = out1(fi[(3 * i + 2) * pfs]);
            }
        }
    }
}

template <int NP, int MT, class YT>
__device__ __forceinline__ void mode_res_body(
    const KP& p, int mB, int flags, const YT* __restrict__ P3, const double2* __restrict__ u,
    double2* __restrict__ r, double* __restrict__ cost_part, double2* __restrict__ a,
    YT* __restrict__ Atil) {
    const int N = p.N, nm = p.nm, nmB = p.nmB, t = threadIdx.x;
    if (mB >= nmB) return;
    const int b = mB / nm, m = mB - b * nm;   // guess, Fourier mode
    const size_t so = (size_t)b * 3 * nm * N; // offset of this guess in spectral arrays
    double2* const vs = mode_vectors<NP, MT>();
    auto vec = [&](int k) { return vs + (size_t)k * NP; };
    double* red = mode_red<NP>(vs);
    const MS c = mscal(p, m);
    const bool zero = (m == 0);
    double2 *R0 = vec(9), *R1 = vec(10), *R2 = vec(11);
    ModeTabs T;
    if (flags & RES_INPUT_W) {
        T = stage_tabs<NP, MT>(p, m, mode_tab<NP>(vs), true, false);
        read_field3<MT>(p, u, so, m, vec(9), vec(10), vec(11));
        __syncthreads();
    } else {
        T = open_mode<NP, MT, 3>(p, m, mB, so, mode_tab<NP>(vs), true, false, u, vec(3), P3, vec(0));
        __syncthreads();
        mv3<NP, MT>(p, M_CINV, N, vec(0), vec(1), vec(2), vec(6), vec(7), vec(8));
        mv3_ep<NP, MT>(p, M_D2, N, vec(3), vec(4), vec(5), [&](int n, double2 d0, double2 d1, double2 d2) {
            const double2 d[3] = {d0, d1, d2};
#pragma unroll
            for (int i = 0; i < 3; ++i) {   // F = -(advection) + nu L u, L = D^2 - k^2
                const double2 L = csub(d[i], cscl(c.k2, vec(3 + i)[n]));
                vec(6 + i)[n] = cadd(cscl(-1.0, vec(6 + i)[n]), cscl(p.nu, L));
            }
        });
        __syncthreads();
        if (zero)
            stokes0<NP, MT>(p, T, vec(6), vec(8), R0, R1, R2, vec(12));
        else
            stokes<NP, MT>(p, T, c, vec(6), vec(7), vec(8), R0, R1, R2, vec(12), red);
        for (int i = 0; i < 3; ++i)
            for (int n = t; n < N; n += MT) {
                const double2 v = cscl(p.lam, vec(9 + i)[n]);
                vec(9 + i)[n] = v;
                if (flags & RES_WRITE_R) r[so + ((size_t)i * nm + m) * N + n] = v;
            }
        __syncthreads();
    }
    if (!(flags & (RES_COST | RES_ADJ))) return;
    mv3<NP, MT>(p, M_G, N, R0, R1, R2, vec(3), vec(4), vec(5));
    __syncthreads();
    if (flags & RES_COST) {
        double s = 0;
        for (int i = 0; i < 3; ++i)
            for (int n = t; n < N; n += MT) {
                const double2 x = vec(9 + i)[n], y = vec(3 + i)[n];
                s += x.x * y.x + x.y * y.y;
            }
        double tot[1] = {s};
        bsum<MT>(tot, red);
        if (t == 0) cost_part[mB] = c.wgt * tot[0];
    }
    if (!(flags & RES_ADJ)) return;
    if (zero)
        stokes0_h<NP, MT>(p, T, vec(3), vec(5), vec(6), vec(7), vec(8), vec(12));
    else
        stokes_h<NP, MT>(p, T, c, vec(3), vec(4), vec(5), vec(6), vec(7), vec(8), vec(12), red);
    mv3<NP, MT>(p, M_GINV, N, vec(6), vec(7), vec(8), vec(0), vec(1), vec(2));
    mv3<NP, MT>(p, M_CINVT, N, vec(6), vec(7), vec(8), vec(12), vec(13), vec(14));
    __syncthreads();
    for (int i = 0; i < 3; ++i)
        for (int n = t; n < N; n += MT) {
            a[so + ((size_t)i * nm + m) * N + n] = vec(i)[n];
            Atil[((size_t)i * N + n) * nmB + mB] = narrow<YT>(vec(12 + i)[n]);
        }
}

template <int NP, int MT, class YT>
__device__ __forceinline__ void mode_grad_body(const KP& p, int mB, int flags, const YT* __restrict__ P6,
                                               const double2* __restrict__ a, double dtau,
                                               double2* __restrict__ uo, YT* __restrict__ Y) {
    const int N = p.N, nm = p.nm, nmB = p.nmB, t = threadIdx.x;
    if (mB >= nmB) return;
    const int b = mB / nm, m = mB - b * nm;   // guess, Fourier mode
    const size_t so = (size_t)b * 3 * nm * N; // offset of this guess in spectral arrays
    double2* const vs = mode_vectors<NP, MT>();
    auto vec = [&](int k) { return vs + (size_t)k * NP; };
    const MS c = mscal(p, m);
    const bool zero = (m == 0);
    const ModeTabs T = open_mode<NP, MT, 6>(p, m, mB, so, mode_tab<NP>(vs), false, (flags & GRAD_PROJECT) != 0, a,
                                            vec(6), P6, vec(0));
    __syncthreads();
    mv3<NP, MT>(p, M_MA, N, vec(0), vec(1), vec(2), vec(9), vec(10), vec(11));
    mv3<NP, MT>(p, M_MB, N, vec(3), vec(4), vec(5), vec(12), vec(13), vec(14));
    mv3_ep<NP, MT>(p, M_ML, N, vec(6), vec(7), vec(8), [&](int n, double2 l0, double2 l1, double2 l2) {
        const double2 l[3] = {l0, l1, l2};
#pragma unroll
        for (int i = 0; i < 3; ++i) {   // g = lam (nu L* a - M'* a)
            const double2 adv = cadd(vec(9 + i)[n], vec(12 + i)[n]);
            const double2 lap = csub(l[i], cscl(c.k2, vec(6 + i)[n]));
            vec(9 + i)[n] = cscl(p.lam, csub(cscl(p.nu, lap), adv));
        }
    });
    __syncthreads();
    double2 *F0 = vec(9), *F1 = vec(10), *F2 = vec(11);
    if (flags & GRAD_PROJECT) {
        if (zero)
            project0<NP, MT>(p, vec(9), vec(11), vec(0), vec(1), vec(2));
        else
            project<NP, MT>(p, T, c, vec(9), vec(10), vec(11), vec(0), vec(1), vec(2), vec(12));
        for (int i = 0; i < 3; ++i)
            for (int n = t; n < N; n += MT) vec(i)[n] = cscl(-1.0, vec(i)[n]);
        __syncthreads();
        F0 = vec(0);
        F1 = vec(1);
        F2 = vec(2);
    }
    double2* Fs[3] = {F0, F1, F2};
    if (flags & GRAD_UPDATE) {
        for (int n = t; n < N; n += MT) {
            size_t gi[3];
            double2 uv[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                gi[i] = so + ((size_t)i * nm + m) * N + n;
                uv[i] = uo[gi[i]];
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double2 un = cadd(uv[i], cscl(dtau, Fs[i][n]));
                uo[gi[i]] = un;
                vec(3 + i)[n] = un;
            }
        }
        __syncthreads();
        mv3<NP, MT>(p, M_C, N, vec(3), vec(4), vec(5), vec(6), vec(7), vec(8));
        mv3<NP, MT>(p, M_CD, N, vec(3), vec(4), vec(5), vec(12), vec(13), vec(14));
        __syncthreads();
        for (int i = 0; i < 3; ++i)
            for (int n = t; n < N; n += MT) {
                Y[((size_t)i * N + n) * nmB + mB] = narrow<YT>(vec(6 + i)[n]);
                Y[((size_t)(3 + i) * N + n) * nmB + mB] = narrow<YT>(vec(12 + i)[n]);
            }
    } else {
        for (int i = 0; i < 3; ++i)
            for (int n = t; n < N; n += MT) uo[so + ((size_t)i * nm + m) * N + n] = Fs[i][n];
    }
}

// Single-context kernels: one logical work item per work group.
template <int NP, int MT, class YT>
__global__ __launch_bounds__(MT) void k_synth(KP p, const double2* __restrict__ u,
                                                        YT* __restrict__ Y) {
    synth_body<NP, MT, YT>(p, xcd_item(blockIdx.x, gridDim.x), u, Y);
}

template <int MODE, class R, int NT>
__global__ __launch_bounds__(NT) void k_plane(KP p, const C<R>* __restrict__ Y1, const C<R>* __restrict__ Y2,
                                              C<R>* __restrict__ out) {
    plane_body<MODE, R, NT>(p, xcd_item(blockIdx.x, gridDim.x), Y1, Y2, out);
}

// Minimum waves per SIMD the per-mode kernels are compiled for: 4 (at most
// 128 VGPRs) from NP = 72 up, where launches hold thousands of modes and
// occupancy pays; below, the register budget is left free (at one 48^3 guess
// the bound made the kernels spill and run slower).
template <int NP> constexpr int mode_min_waves() { return NP >= 72 ? 4 : 1; }

template <int NP, int MT, class YT>
__global__ __launch_bounds__(MT, mode_min_waves<NP>()) void k_mode_res(KP p, int flags, const YT* __restrict__ P3,
                                                           const double2* __restrict__ u,
                                                           double2* __restrict__ r, double* __restrict__ cost_part,
                                                           double2* __restrict__ a, YT* __restrict__ Atil) {
    mode_res_body<NP, MT, YT>(p, xcd_item(blockIdx.x, gridDim.x), flags, P3, u, r, cost_part, a, Atil);
}

template <int NP, int MT, class YT>
__global__ __launch_bounds__(MT, mode_min_waves<NP>()) void k_mode_grad(KP p, int flags, const YT* __restrict__ P6,
                                                            const double2* __restrict__ a, double dtau,
                                                            double2* __restrict__ uo, YT* __restrict__ Y) {
    mode_grad_body<NP, MT, YT>(p, xcd_item(blockIdx.x, gridDim.x), flags, P6, a, dtau, uo, Y);
}

// Grouped kernels: one launch covers every member of a group (contexts of
// different grids, Re and batch).  The logical items of member k are
// [item0[k], item0[k+1]); each work group finds its member by binary search
// and runs the single-context body with that member's parameters.
__device__ __forceinline__ int group_member(const GroupMember* __restrict__ gm, int n, int it, int phase) {
    int lo = 0, hi = n;  // invariant: gm[lo].item0[phase] <= it < gm[hi].item0[phase] (gm[n] sentinel)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (gm[mid].item0[phase] <= it) lo = mid; else hi = mid;
    }
    return lo;
}

template <int NP, int MT, class YT>
__global__ __launch_bounds__(MT) void kg_synth(const GroupMember* __restrict__ gm, int n) {
    const int it = xcd_item(blockIdx.x, gridDim.x);
    if (it >= gm[n].item0[GPH_MODE]) return;
    const int k = group_member(gm, n, it, GPH_MODE);
    const GroupMember& g = gm[k];
    synth_body<NP, MT, YT>(g.kp, it - g.item0[GPH_MODE], g.u, static_cast<YT*>(g.Y));
}

template <int MODE, class R, int NT>
__global__ __launch_bounds__(NT) void kg_plane(const GroupMember* __restrict__ gm, int n) {
    const int it = xcd_item(blockIdx.x, gridDim.x);
    if (it >= gm[n].item0[GPH_PLANE]) return;
    const int k = group_member(gm, n, it, GPH_PLANE);
    const GroupMember& g = gm[k];
    if (MODE == PLANE_FWD)
        plane_body<MODE, R, NT>(g.kp, it - g.item0[GPH_PLANE], static_cast<const C<R>*>(g.Y), nullptr,
                                static_cast<C<R>*>(g.P3));
    else
        plane_body<MODE, R, NT>(g.kp, it - g.item0[GPH_PLANE], static_cast<const C<R>*>(g.Y),
                                static_cast<const C<R>*>(g.Atil), static_cast<C<R>*>(g.P6));
}

template <int NP, int MT, class YT>
__global__ __launch_bounds__(MT, mode_min_waves<NP>()) void kg_mode_res(const GroupMember* __restrict__ gm, int n) {
    const int it = xcd_item(blockIdx.x, gridDim.x);
    if (it >= gm[n].item0[GPH_MODE]) return;
    const int k = group_member(gm, n, it, GPH_MODE);
    const GroupMember& g = gm[k];
    mode_res_body<NP, MT, YT>(g.kp, it - g.item0[GPH_MODE], RES_COST | RES_ADJ, static_cast<const YT*>(g.P3), g.u,
                          nullptr, g.part, g.a, static_cast<YT*>(g.Atil));
}

template <int NP, int MT, class YT>
__global__ __launch_bounds__(MT, mode_min_waves<NP>()) void kg_mode_grad(const GroupMember* __restrict__ gm, int n) {
    const int it = xcd_item(blockIdx.x, gridDim.x);
    if (it >= gm[n].item0[GPH_MODE]) return;
    const int k = group_member(gm, n, it, GPH_MODE);
    const GroupMember& g = gm[k];
    mode_grad_body<NP, MT, YT>(g.kp, it - g.item0[GPH_MODE], GRAD_PROJECT | GRAD_UPDATE, static_cast<const YT*>(g.P6),
                           g.a, g.dtau, g.u, static_cast<YT*>(g.Y));
}

template <int NP, int MT>
__global__ __launch_bounds__(MT) void k_project(KP p, const double2* __restrict__ g,
                                                          double2* __restrict__ out) {
    const int mB = xcd_item(blockIdx.x, gridDim.x), N = p.N, nm = p.nm, nmB = p.nmB, t = threadIdx.x;
    if (mB >= nmB) return;
    const int b = mB / nm, m = mB - b * nm;   // guess, Fourier mode
    const size_t so = (size_t)b * 3 * nm * N; // offset of this guess in spectral arrays
    double2* const vs = mode_vectors<NP, MT>();
    auto vec = [&](int k) { return vs + (size_t)k * NP; };
    const ModeTabs T = stage_tabs<NP, MT>(p, m, mode_tab<NP>(vs), false, true);
    read_field3<MT>(p, g, so, m, vec(0), vec(1), vec(2));
    __syncthreads();
    if (m == 0)
        project0<NP, MT>(p, vec(0), vec(2), vec(3), vec(4), vec(5));
    else
        project<NP, MT>(p, T, mscal(p, m), vec(0), vec(1), vec(2), vec(3), vec(4), vec(5), vec(12));
    for (int i = 0; i < 3; ++i)
        for (int n = t; n < N; n += MT) out[so + ((size_t)i * nm + m) * N + n] = vec(3 + i)[n];
}

// Deterministic per-guess reductions of per-mode partials: out[g * stride + c]
// = sum (op 0) or max (op 1) over rows i < n of part[(g * n + i) * stride + c].
// One work group per guess g.
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ part, int n, int stride,
                                                int op, double* __restrict__ out) {
    __shared__ double red[256];
    const int g = blockIdx.x;
    part += (size_t)g * n * stride;
    for (int c = 0; c < stride; ++c) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < n; i += 256) {
            const double v = part[(size_t)i * stride + c];
            acc = op ? fmax(acc, v) : acc + v;
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w)
                red[threadIdx.x] = op ? fmax(red[threadIdx.x], red[threadIdx.x + w])
                                      : red[threadIdx.x] + red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[(size_t)g * stride + c] = red[0];
        __syncthreads();
    }
}

// Per-mode partials of ||u||^2, ||u_b + u||^2 and <curl U, curl U> (U = u_b + u).
template <int NP, int MT>
__global__ __launch_bounds__(MT) void k_norms(KP p, const double2* __restrict__ u,
                                                        double* __restrict__ part) {
    const int mB = xcd_item(blockIdx.x, gridDim.x), N = p.N, nm = p.nm, nmB = p.nmB, t = threadIdx.x;
    if (mB >= nmB) return;
    const int b = mB / nm, m = mB - b * nm;   // guess, Fourier mode
    const size_t so = (size_t)b * 3 * nm * N; // offset of this guess in spectral arrays
    double2* const vs = mode_vectors<NP, MT>();
    auto vec = [&](int k) { return vs + (size_t)k * NP; };
    double* red = mode_red<NP>(vs);
    const MS c = mscal(p, m);
    read_field3<MT>(p, u, so, m, vec(0), vec(1), vec(2));
    __syncthreads();
    mv3<NP, MT>(p, M_G, N, vec(0), vec(1), vec(2), vec(3), vec(4), vec(5));
    __syncthreads();
    double s0 = 0;
    for (int i = 0; i < 3; ++i)
        for (int n = t; n < N; n += MT) s0 += vec(i)[n].x * vec(3 + i)[n].x + vec(i)[n].y * vec(3 + i)[n].y;
    {
        double tot[1] = {s0};
        bsum<MT>(tot, red);
        s0 = tot[0];
    }
    if (m == 0 && t == 0) vec(0)[1] = cadd(vec(0)[1], c2(1.0, 0.0));  // + u_b = T_1(y) e_x
    __syncthreads();
    mv3<NP, MT>(p, M_G, N, vec(0), vec(1), vec(2), vec(3), vec(4), vec(5));
    mv<NP, MT>(p, M_D, N, vec(0), vec(6));
    mv<NP, MT>(p, M_D, N, vec(2), vec(7));
    __syncthreads();
    double s1 = 0;
    for (int i = 0; i < 3; ++i)
        for (int n = t; n < N; n += MT) s1 += vec(i)[n].x * vec(3 + i)[n].x + vec(i)[n].y * vec(3 + i)[n].y;
    {
        double tot[1] = {s1};
        bsum<MT>(tot, red);
        s1 = tot[0];
    }
    // vorticity: (D U_z - i b U_y, i b U_x - i a U_z, i a U_y - D U_x)
    for (int n = t; n < N; n += MT) {
        const double2 ux = vec(0)[n], uy = vec(1)[n], uz = vec(2)[n];
        vec(8)[n] = csub(vec(7)[n], imul(c.b, uy));
        vec(9)[n] = csub(imul(c.b, ux), imul(c.a, uz));
        vec(10)[n] = csub(imul(c.a, uy), vec(6)[n]);
    }
    __syncthreads();
    mv3<NP, MT>(p, M_G, N, vec(8), vec(9), vec(10), vec(11), vec(12), vec(13));
    __syncthreads();
    double s2 = 0;
    for (int i = 0; i < 3; ++i)
        for (int n = t; n < N; n += MT)
            s2 += vec(8 + i)[n].x * vec(11 + i)[n].x + vec(8 + i)[n].y * vec(11 + i)[n].y;
    {
        double tot[1] = {s2};
        bsum<MT>(tot, red);
        s2 = tot[0];
    }
    if (t == 0) {
        part[(size_t)mB * 3 + 0] = c.wgt * s0;
        part[(size_t)mB * 3 + 1] = c.wgt * s1;
        part[(size_t)mB * 3 + 2] = c.wgt * s2;
    }
}

// Per-mode admissibility defects: max |div|, max |wall value|, Hermitian defect.
template <int NP, int MT>
__global__ __launch_bounds__(MT) void k_check(KP p, const double2* __restrict__ u,
                                                        double* __restrict__ part) {
    const int mB = xcd_item(blockIdx.x, gridDim.x), N = p.N, nm = p.nm, nmB = p.nmB, t = threadIdx.x;
    if (mB >= nmB) return;
    const int b = mB / nm, m = mB - b * nm;   // guess, Fourier mode
    const size_t so = (size_t)b * 3 * nm * N; // offset of this guess in spectral arrays
    double2* const vs = mode_vectors<NP, MT>();
    auto vec = [&](int k) { return vs + (size_t)k * NP; };
    double* red = mode_red<NP>(vs);
    const MS c = mscal(p, m);
    read_field3<MT>(p, u, so, m, vec(0), vec(1), vec(2));
    __syncthreads();
    mv<NP, MT>(p, M_D, N, vec(1), vec(3));
    __syncthreads();
    double dv = 0, herm = 0;
    double wr[6] = {0, 0, 0, 0, 0, 0}, wi[6] = {0, 0, 0, 0, 0, 0};
    const int ikx = m / p.nkz, kz = m - ikx * p.nkz;
    const int kx = (ikx <= p.Kx) ? ikx : ikx - p.nkx;
    const int mp = ((p.nkx - ikx) % p.nkx) * p.nkz;
    for (int n = t; n < N; n += MT) {
        const double2 d = cadd(cadd(imul(c.a, vec(0)[n]), vec(3)[n]), imul(c.b, vec(2)[n]));
        dv = fmax(dv, hypot(d.x, d.y));
        for (int i = 0; i < 3; ++i) {
            const double2 v = vec(i)[n];
            wr[2 * i] += v.x;
            wi[2 * i] += v.y;
            wr[2 * i + 1] += (n & 1) ? -v.x : v.x;
            wi[2 * i + 1] += (n & 1) ? -v.y : v.y;
            if (m == 0) herm = fmax(herm, fabs(v.y));
            if (kz == 0 && kx > 0) {
                const double2 w = u[so + ((size_t)i * nm + mp) * N + n];
                herm = fmax(herm, hypot(w.x - v.x, w.y + v.y));
            }
        }
    }
    double sums[12];
    for (int q = 0; q < 6; ++q) {
        sums[2 * q] = wr[q];
        sums[2 * q + 1] = wi[q];
    }
    bsum<MT>(sums, red);
    double wall = 0;
    for (int q = 0; q < 6; ++q) wall = fmax(wall, hypot(sums[2 * q], sums[2 * q + 1]));
    double mx[2] = {dv, herm};
    bmax<MT>(mx, red);
    dv = mx[0];
    herm = mx[1];
    if (t == 0) {
        part[(size_t)mB * 3 + 0] = dv;
        part[(size_t)mB * 3 + 1] = wall;
        part[(size_t)mB * 3 + 2] = herm;
    }
}

template <int MT>
__global__ __launch_bounds__(MT) void k_pack(KP p, const double2* __restrict__ u,
                                                       double* __restrict__ psi) {
    const int mB = xcd_item(blockIdx.x, gridDim.x), N = p.N, nm = p.nm, nmB = p.nmB, t = threadIdx.x;
    if (mB >= nmB) return;
    const int b = mB / nm, m = mB - b * nm;   // guess, Fourier mode
    const size_t so = (size_t)b * 3 * nm * N; // offset of this guess in spectral arrays
    const int idx = p.indep[m];
    if (idx < 0) return;
    if (m == 0) {
        for (int n = t; n < N - 2; n += MT) {
            psi[(size_t)b * p.nstate + n] = u[so + (size_t)m * N + n].x;
            psi[(size_t)b * p.nstate + (N - 2) + n] = u[so + ((size_t)2 * nm + m) * N + n].x;
        }
        return;
    }
    const MS c = mscal(p, m);
    double* o = psi + (size_t)b * p.nstate + 2 * (N - 2) + (size_t)idx * (4 * N - 12);
    for (int n = t; n < N; n += MT) {
        const double2 v = u[so + ((size_t)nm + m) * N + n];
        const double2 e = csub(imul(c.b, u[so + (size_t)m * N + n]), imul(c.a, u[so + ((size_t)2 * nm + m) * N + n]));
        if (n < N - 4) {
            o[n] = v.x;
            o[(N - 4) + n] = v.y;
        }
        if (n < N - 2) {
            o[2 * (N - 4) + n] = e.x;
            o[2 * (N - 4) + (N - 2) + n] = e.y;
        }
    }
}

// Sum over lanes of x[n] (n < lim, n = par mod 2), optionally weighted by n^2.
template <int MT>
__device__ double2 par_sum(const double2* x, int lim, int par, bool sq, double* red) {
    double v[2] = {0, 0};
    for (int n = threadIdx.x; n < lim; n += MT)
        if ((n & 1) == par) {
            const double w = sq ? (double)n * n : 1.0;
            v[0] += w * x[n].x;
            v[1] += w * x[n].y;
        }
    bsum<MT>(v, red);
    return c2(v[0], v[1]);
}

template <int NP, int MT>
__global__ __launch_bounds__(MT) void k_unpack(KP p, const double* __restrict__ psi,
                                                         double2* __restrict__ u) {
    const int mB = xcd_item(blockIdx.x, gridDim.x), N = p.N, nm = p.nm, nmB = p.nmB, t = threadIdx.x;
    if (mB >= nmB) return;
    const int b = mB / nm, m = mB - b * nm;   // guess, Fourier mode
    const size_t so = (size_t)b * 3 * nm * N; // offset of this guess in spectral arrays
    const int idx = p.indep[m];
    if (idx < 0) return;
    double2* const vs = mode_vectors<NP, MT>();
    auto vec = [&](int k) { return vs + (size_t)k * NP; };
    double* red = mode_red<NP>(vs);
    if (m == 0) {
        for (int n = t; n < N; n += MT) {
            vec(0)[n] = c2(n < N - 2 ? psi[(size_t)b * p.nstate + n] : 0.0, 0);
            vec(1)[n] = c2(n < N - 2 ? psi[(size_t)b * p.nstate + (N - 2) + n] : 0.0, 0);
        }
        __syncthreads();
        for (int f = 0; f < 2; ++f) {  // Dirichlet: each parity class sums to zero
            const double2 s0 = par_sum<MT>(vec(f), N - 2, (N - 2) & 1, false, red);
            const double2 s1 = par_sum<MT>(vec(f), N - 2, (N - 1) & 1, false, red);
            __syncthreads();
            if (t == 0) {
                vec(f)[N - 2] = cscl(-1.0, s0);
                vec(f)[N - 1] = cscl(-1.0, s1);
            }
            __syncthreads();
        }
        for (int n = t; n < N; n += MT) {
            u[so + (size_t)m * N + n] = vec(0)[n];
            u[so + ((size_t)nm + m) * N + n] = c2(0, 0);
            u[so + ((size_t)2 * nm + m) * N + n] = vec(1)[n];
        }
        return;
    }
    const MS c = mscal(p, m);
    const double* o = psi + (size_t)b * p.nstate + 2 * (N - 2) + (size_t)idx * (4 * N - 12);
    double2 *v = vec(0), *e = vec(1), *Dv = vec(2);
    for (int n = t; n < N; n += MT) {
        v[n] = (n < N - 4) ? c2(o[n], o[(N - 4) + n]) : c2(0, 0);
        e[n] = (n < N - 2) ? c2(o[2 * (N - 4) + n], o[2 * (N - 4) + (N - 2) + n]) : c2(0, 0);
    }
    __syncthreads();
    // clamped v: within each parity class sum v_n = 0 and sum n^2 v_n = 0
    for (int q = N - 2; q < N; ++q) {
        const int pp = q - 2, par = q & 1;
        const double2 s0 = par_sum<MT>(v, pp, par, false, red), s2 = par_sum<MT>(v, pp, par, true, red);
        const double2 vq = cscl(1.0 / ((double)q * q - (double)pp * pp), csub(cscl((double)pp * pp, s0), s2));
        __syncthreads();
        if (t == 0) {
            v[q] = vq;
            v[pp] = csub(cscl(-1.0, s0), vq);
        }
        __syncthreads();
    }
    {
        const double2 s0 = par_sum<MT>(e, N - 2, (N - 2) & 1, false, red);
        const double2 s1 = par_sum<MT>(e, N - 2, (N - 1) & 1, false, red);
        __syncthreads();
        if (t == 0) {
            e[N - 2] = cscl(-1.0, s0);
            e[N - 1] = cscl(-1.0, s1);
        }
        __syncthreads();
    }
    mv<NP, MT>(p, M_D, N, v, Dv);
    __syncthreads();
    const int ikx = m / p.nkz, kz = m - ikx * p.nkz;
    const int mp = ((p.nkx - ikx) % p.nkx) * p.nkz;
    for (int n = t; n < N; n += MT) {
        const double2 ux = cscl(c.ik2, csub(imul(c.a, Dv[n]), imul(c.b, e[n])));
        const double2 uz = cscl(c.ik2, cadd(imul(c.b, Dv[n]), imul(c.a, e[n])));
        const double2 vals[3] = {ux, v[n], uz};
        for (int i = 0; i < 3; ++i) {
            u[so + ((size_t)i * nm + m) * N + n] = vals[i];
            if (kz == 0) u[so + ((size_t)i * nm + mp) * N + n] = c2(vals[i].x, -vals[i].y);
        }
    }
}

// Double-double accumulation (Dekker/Knuth error-free transforms): the DMD
// algebra factors the Gram matrix, whose error the factor inherits times
// cond(E)^2, so the Gram is summed to about 2^-100 relative accuracy.
struct dd {
    double hi, lo;
};

__device__ inline dd dd_add(dd a, dd b) {
    const double s = a.hi + b.hi;
    const double v = s - a.hi;
    double e = (a.hi - (s - v)) + (b.hi - v);
    e += a.lo + b.lo;
    const double h = s + e;
    return dd{h, e - (h - s)};
}

__device__ inline dd dd_fma(double x, double y, dd acc) {
    const double p = x * y;
    return dd_add(acc, dd{p, fma(x, y, -p)});
}

// Gram matrix of the snapshot differences of each guess: with S[k][b][:] the
// minimal state vectors (k < M), e_0 = S[0], e_k = S[k] - S[k-1];
// G[b][i][j] = e_i . e_j as a (hi, lo) pair of doubles.  One work group per
// (b, i <= j), deterministic reduction order.
__global__ __launch_bounds__(256) void k_dmd_gram(const double* __restrict__ S, int M, int B,
                                                  long long n, double* __restrict__ G) {
    __shared__ double rhi[256], rlo[256];
    int w = blockIdx.x;
    const int npair = M * (M + 1) / 2;
    const int b = w / npair;
    w -= b * npair;
    int i = 0;
    while (w >= M - i) {
        w -= M - i;
        ++i;
    }
    const int j = i + w;
    const size_t stride = (size_t)B * n;
    const double* si = S + (size_t)i * stride + (size_t)b * n;
    const double* sj = S + (size_t)j * stride + (size_t)b * n;
    dd acc{0.0, 0.0};
    for (long long t = threadIdx.x; t < n; t += 256) {
        const double ei = (i > 0) ? si[t] - si[t - stride] : si[t];
        const double ej = (j > 0) ? sj[t] - sj[t - stride] : sj[t];
        acc = dd_fma(ei, ej, acc);
    }
    rhi[threadIdx.x] = acc.hi;
    rlo[threadIdx.x] = acc.lo;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            const dd r = dd_add(dd{rhi[threadIdx.x], rlo[threadIdx.x]},
                                dd{rhi[threadIdx.x + h], rlo[threadIdx.x + h]});
            rhi[threadIdx.x] = r.hi;
            rlo[threadIdx.x] = r.lo;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* g = G + (size_t)b * M * M * 2;
        g[((size_t)i * M + j) * 2] = rhi[0];
        g[((size_t)i * M + j) * 2 + 1] = rlo[0];
        g[((size_t)j * M + i) * 2] = rhi[0];
        g[((size_t)j * M + i) * 2 + 1] = rlo[0];
    }
}

// psi[b][t] = sum_k coef[b][k] S[k + 1][b][t], k < M - 1.
__global__ __launch_bounds__(256) void k_dmd_combine(const double* __restrict__ S, int M, int B,
                                                     long long n, const double* __restrict__ coef,
                                                     double* __restrict__ psi) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    const int b = blockIdx.y;
    if (t >= n) return;
    const size_t stride = (size_t)B * n;
    double acc = 0.0;
    for (int k = 0; k < M - 1; ++k) acc = fma(coef[(size_t)b * (M - 1) + k], S[(size_t)(k + 1) * stride + (size_t)b * n + t], acc);
    psi[(size_t)b * n + t] = acc;
}

__global__ void k_axpy(long long n, double a, const double* __restrict__ x, double* __restrict__ y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = fma(a, x[i], y[i]);
}

}  // namespace

size_t plane_lds_bytes(const KP& p, int mode) {
    const int ng3 = (mode == PLANE_JVP) ? 6 : 3, ng1 = (mode == PLANE_ADJ) ? 3 : 0;
    const int npf = (mode == PLANE_ADJ) ? 12 : 3;
    const size_t nxf = 3 * ng3 + ng1, r = p.prec == PREC_FP32 ? 4 : 8;
    const size_t products = (size_t)npf * p.XS * (p.Nz + 1) * r;
    const size_t row = (size_t)p.XS * kz_row(p.nkz) * 2 * r;   // one x-slab array of kz_row(nkz) complex per x
    const size_t folded = (size_t)(ng1 > 0 ? 12 : 9) * row;    // aliases products, as does the x DFT (<= 9 arrays)
    const size_t nzt = (p.Nz & 1) ? p.Nz : p.Nz / 2;   // rows of the z twiddle table
    const size_t twiddles = (size_t)p.nkx + (size_t)p.XS * p.XS + nzt * kz_row(p.nkz);
    return twiddles * 2 * r + nxf * row + std::max(products, folded);
}

size_t mode_lds_bytes(const KP& p) {
    return (size_t)MODE_VECS * p.np * 16 + (size_t)tab_doubles(p.np) * 8 + (size_t)(p.mthreads / WAVE) * RED_SLOTS * 8;
}

static dim3 mode_grid(const KP& p) { return dim3((unsigned)((p.nmB + NXCD - 1) / NXCD * NXCD)); }

// The per-mode kernels are compiled for a fixed set of padded Ny (KP::np, a
// multiple of 8 so that every split of a contraction is whole) and every
// contraction loop is fully unrolled; Ny takes the smallest that holds it.
static const int kPaddedNy[] = {16, 32, 48, 56, 64, 72, 80, 96, 112, 128};
int padded_ny(int N) {
    for (int np : kPaddedNy)
        if (N <= np) return np;
    return 0;
}

#define PCFV_DISPATCH_NP(np, ...)                                 \
    switch (np) {                                                 \
        case 16: { constexpr int NP = 16; __VA_ARGS__; } break;   \
        case 32: { constexpr int NP = 32; __VA_ARGS__; } break;   \
        case 48: { constexpr int NP = 48; __VA_ARGS__; } break;   \
        case 56: { constexpr int NP = 56; __VA_ARGS__; } break;   \
        case 64: { constexpr int NP = 64; __VA_ARGS__; } break;   \
        case 72: { constexpr int NP = 72; __VA_ARGS__; } break;   \
        case 80: { constexpr int NP = 80; __VA_ARGS__; } break;   \
        case 96: { constexpr int NP = 96; __VA_ARGS__; } break;   \
        case 112: { constexpr int NP = 112; __VA_ARGS__; } break; \
        case 128: { constexpr int NP = 128; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;                     \
    }

// Dispatch on the padded Ny (NP) and the per-mode work-group size (MT).
#define PCFV_DISPATCH_MODE(np, mt, ...)                                                  \
    switch (mt) {                                                                        \
        case 256: { constexpr int MT = 256; PCFV_DISPATCH_NP(np, __VA_ARGS__); } break;  \
        case 512: { constexpr int MT = 512; PCFV_DISPATCH_NP(np, __VA_ARGS__); } break;  \
        default: return hipErrorInvalidValue;                                            \
    }

// The y-value and partial arrays are raw storage: FP64 complex for PREC_FP64,
// FP32 complex (half the bytes, same buffers) for PREC_FP32.
template <class YT>
static hipError_t synth_t(const KP& p, hipStream_t s, const double2* u, void* Y) {
    PCFV_DISPATCH_MODE(p.np, p.mthreads, hipLaunchKernelGGL((k_synth<NP, MT, YT>), mode_grid(p), dim3(MT),
                                                      mode_lds_bytes(p), s, p, u, static_cast<YT*>(Y)));
    return hipGetLastError();
}

hipError_t launch_synth(const KP& p, hipStream_t s, const double2* u, void* Y) {
    return p.prec == PREC_FP32 ? synth_t<float2>(p, s, u, Y) : synth_t<double2>(p, s, u, Y);
}

template <class R, int NT>
static hipError_t plane_t(const KP& p, hipStream_t s, int mode, const void* Y1, const void* Y2, void* out) {
    typedef C<R> CR;
    const dim3 grid((unsigned)((p.B * p.NS * p.N + NXCD - 1) / NXCD * NXCD)), block(NT);
    const size_t lds = plane_lds_bytes(p, mode);
    const CR* y1 = static_cast<const CR*>(Y1);
    const CR* y2 = static_cast<const CR*>(Y2);
    CR* o = static_cast<CR*>(out);
    if (mode == PLANE_FWD) {
        hipLaunchKernelGGL((k_plane<PLANE_FWD, R, NT>), grid, block, lds, s, p, y1, y2, o);
    } else if (mode == PLANE_JVP) {
        if constexpr (NT <= 512)
            hipLaunchKernelGGL((k_plane<PLANE_JVP, R, NT>), grid, block, lds, s, p, y1, y2, o);
        else
            return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((k_plane<PLANE_ADJ, R, NT>), grid, block, lds, s, p, y1, y2, o);
    }
    return hipGetLastError();
}

// Work-group sizes of the physical-space kernels.  Their four stages hand out
// (fields x slab points) work items to the threads, so the size that wastes
// the fewest partial passes depends on the slab; the JVP variant carries twice
// the fields (more registers) and runs with at most 512 threads.
#define PCFV_DISPATCH_PT(nt, ...)                                   \
    switch (nt) {                                                   \
        case 256: { constexpr int NT = 256; __VA_ARGS__; } break;   \
        case 512: { constexpr int NT = 512; __VA_ARGS__; } break;   \
        case 576: { constexpr int NT = 576; __VA_ARGS__; } break;   \
        case 768: { constexpr int NT = 768; __VA_ARGS__; } break;   \
        case 1024: { constexpr int NT = 1024; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;                       \
    }

hipError_t launch_plane(const KP& p, hipStream_t s, int mode, const void* Y1, const void* Y2, void* out) {
    const int nt = (mode == PLANE_JVP) ? std::min(p.pthreads, 512) : p.pthreads;
    if (p.prec == PREC_FP32) {
        PCFV_DISPATCH_PT(nt, return plane_t<float, NT>(p, s, mode, Y1, Y2, out));
    } else {
        PCFV_DISPATCH_PT(nt, return plane_t<double, NT>(p, s, mode, Y1, Y2, out));
    }
    return hipErrorInvalidValue;
}

template <class YT>
static hipError_t mode_res_t(const KP& p, hipStream_t s, int flags, const void* P3, const double2* u,
                             double2* r, double* cost_part, double2* a, void* Atil) {
    PCFV_DISPATCH_MODE(p.np, p.mthreads, hipLaunchKernelGGL((k_mode_res<NP, MT, YT>), mode_grid(p), dim3(MT),
                                                      mode_lds_bytes(p), s, p, flags, static_cast<const YT*>(P3),
                                                      u, r, cost_part, a, static_cast<YT*>(Atil)));
    return hipGetLastError();
}

hipError_t launch_mode_res(const KP& p, hipStream_t s, int flags, const void* P3, const double2* u,
                           double2* r, double* cost_part, double2* a, void* Atil) {
    return p.prec == PREC_FP32 ? mode_res_t<float2>(p, s, flags, P3, u, r, cost_part, a, Atil)
                               : mode_res_t<double2>(p, s, flags, P3, u, r, cost_part, a, Atil);
}

template <class YT>
static hipError_t mode_grad_t(const KP& p, hipStream_t s, int flags, const void* P6, const double2* a,
                              double dtau, double2* u_or_out, void* Y) {
    PCFV_DISPATCH_MODE(p.np, p.mthreads, hipLaunchKernelGGL((k_mode_grad<NP, MT, YT>), mode_grid(p), dim3(MT),
                                                      mode_lds_bytes(p), s, p, flags, static_cast<const YT*>(P6),
                                                      a, dtau, u_or_out, static_cast<YT*>(Y)));
    return hipGetLastError();
}

hipError_t launch_mode_grad(const KP& p, hipStream_t s, int flags, const void* P6, const double2* a,
                            double dtau, double2* u_or_out, void* Y) {
    return p.prec == PREC_FP32 ? mode_grad_t<float2>(p, s, flags, P6, a, dtau, u_or_out, Y)
                               : mode_grad_t<double2>(p, s, flags, P6, a, dtau, u_or_out, Y);
}

static dim3 grid8(int items) { return dim3((unsigned)((items + NXCD - 1) / NXCD * NXCD)); }

template <class R, int NT, class YT>
static hipError_t group_t(const GroupLaunch& g, hipStream_t s, int which) {
    const dim3 gp = grid8(g.items[GPH_PLANE]), gmo = grid8(g.items[GPH_MODE]);
    switch (which) {
        case GK_SYNTH:
            PCFV_DISPATCH_MODE(g.np, g.mthreads, hipLaunchKernelGGL((kg_synth<NP, MT, YT>), gmo, dim3(MT), g.mode_lds, s,
                                                      g.gm, g.n));
            break;
        case GK_PLANE_FWD:
            hipLaunchKernelGGL((kg_plane<PLANE_FWD, R, NT>), gp, dim3(NT), g.plane_lds[PLANE_FWD], s, g.gm, g.n);
            break;
        case GK_MODE_RES:
            PCFV_DISPATCH_MODE(g.np, g.mthreads, hipLaunchKernelGGL((kg_mode_res<NP, MT, YT>), gmo, dim3(MT), g.mode_lds,
                                                      s, g.gm, g.n));
            break;
        case GK_PLANE_ADJ:
            hipLaunchKernelGGL((kg_plane<PLANE_ADJ, R, NT>), gp, dim3(NT), g.plane_lds[PLANE_ADJ], s, g.gm, g.n);
            break;
        case GK_MODE_GRAD:
            PCFV_DISPATCH_MODE(g.np, g.mthreads, hipLaunchKernelGGL((kg_mode_grad<NP, MT, YT>), gmo, dim3(MT), g.mode_lds,
                                                      s, g.gm, g.n));
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_group(const GroupLaunch& g, hipStream_t s, int which) {
    if (g.prec == PREC_FP32) {
        PCFV_DISPATCH_PT(g.pthreads, return group_t<float, NT, float2>(g, s, which));
    } else {
        PCFV_DISPATCH_PT(g.pthreads, return group_t<double, NT, double2>(g, s, which));
    }
    return hipErrorInvalidValue;
}

hipError_t launch_project(const KP& p, hipStream_t s, const double2* g, double2* out) {
    PCFV_DISPATCH_MODE(p.np, p.mthreads, hipLaunchKernelGGL((k_project<NP, MT>), mode_grid(p), dim3(MT), mode_lds_bytes(p), s, p, g, out));
    return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t s, const double* part, int ngroups, int n, int stride, int op,
                         double* out) {
    hipLaunchKernelGGL(k_reduce, dim3(ngroups), dim3(256), 0, s, part, n, stride, op, out);
    return hipGetLastError();
}

hipError_t launch_norms(const KP& p, hipStream_t s, const double2* u, double* part) {
    PCFV_DISPATCH_MODE(p.np, p.mthreads, hipLaunchKernelGGL((k_norms<NP, MT>), mode_grid(p), dim3(MT), mode_lds_bytes(p), s, p, u, part));
    return hipGetLastError();
}

hipError_t launch_check(const KP& p, hipStream_t s, const double2* u, double* part) {
    PCFV_DISPATCH_MODE(p.np, p.mthreads, hipLaunchKernelGGL((k_check<NP, MT>), mode_grid(p), dim3(MT), mode_lds_bytes(p), s, p, u, part));
    return hipGetLastError();
}

hipError_t launch_pack(const KP& p, hipStream_t s, const double2* u, double* psi) {
    if (p.mthreads == 512)
        hipLaunchKernelGGL(k_pack<512>, mode_grid(p), dim3(512), 0, s, p, u, psi);
    else
        hipLaunchKernelGGL(k_pack<256>, mode_grid(p), dim3(256), 0, s, p, u, psi);
    return hipGetLastError();
}

hipError_t launch_unpack(const KP& p, hipStream_t s, const double* psi, double2* u) {
    PCFV_DISPATCH_MODE(p.np, p.mthreads, hipLaunchKernelGGL((k_unpack<NP, MT>), mode_grid(p), dim3(MT), mode_lds_bytes(p), s, p, psi, u));
    return hipGetLastError();
}

hipError_t launch_dmd_gram(hipStream_t s, const double* S, int M, int B, long long n, double* G) {
    hipLaunchKernelGGL(k_dmd_gram, dim3((unsigned)(B * M * (M + 1) / 2)), dim3(256), 0, s, S, M, B, n, G);
    return hipGetLastError();
}

hipError_t launch_dmd_combine(hipStream_t s, const double* S, int M, int B, long long n,
                              const double* coef, double* psi) {
    hipLaunchKernelGGL(k_dmd_combine, dim3((unsigned)((n + 255) / 256), (unsigned)B), dim3(256), 0, s, S, M, B,
                       n, coef, psi);
    return hipGetLastError();
}

hipError_t launch_axpy(hipStream_t s, long long n, double a, const double* x, double* y) {
    hipLaunchKernelGGL(k_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a, x, y);
    return hipGetLastError();
}

}  // namespace pcfv
