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
#include <cstdio>

#include "kernels.hpp"

namespace pcfv {
namespace {

constexpr int WAVE = 64;
constexpr int MODE_THREADS = 64;   // one wavefront per Fourier mode
constexpr int PLANE_THREADS = 256;
constexpr int MODE_VECS = 24;      // LDS vectors (length N) used by the mode kernels

__device__ __forceinline__ double2 c2(double x, double y) { return make_double2(x, y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return c2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return c2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscl(double s, double2 a) { return c2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return c2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// (i s) z for real s
__device__ __forceinline__ double2 imul(double s, double2 z) { return c2(-s * z.y, s * z.x); }

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
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

__device__ __forceinline__ const double* mat(const KP& p, int id) {
    return p.M + (size_t)id * p.N * p.N;
}

// y = A x for one complex vector; A (nout x nin) stored transposed (slot[m*N+n]).
// x and y live in LDS and must not alias.  Caller synchronises afterwards.
__device__ void mv(const KP& p, int id, int nin, int nout, const double2* x, double2* y) {
    const double* __restrict__ A = mat(p, id);
    const int N = p.N;
    for (int n = threadIdx.x; n < nout; n += MODE_THREADS) {
        double re = 0.0, im = 0.0;
#pragma unroll 8
        for (int k = 0; k < nin; ++k) {
            const double a = A[k * N + n];
            const double2 v = x[k];
            re = fma(a, v.x, re);
            im = fma(a, v.y, im);
        }
        y[n] = c2(re, im);
    }
}

// The same matrix applied to three vectors.
__device__ void mv3(const KP& p, int id, int nin, int nout, const double2* x0,
                    const double2* x1, const double2* x2, double2* y0, double2* y1,
                    double2* y2) {
    const double* __restrict__ A = mat(p, id);
    const int N = p.N;
    for (int n = threadIdx.x; n < nout; n += MODE_THREADS) {
        double r0 = 0, i0 = 0, r1 = 0, i1 = 0, r2 = 0, i2 = 0;
#pragma unroll 4
        for (int k = 0; k < nin; ++k) {
            const double a = A[k * N + n];
            const double2 v0 = x0[k], v1 = x1[k], v2 = x2[k];
            r0 = fma(a, v0.x, r0);
            i0 = fma(a, v0.y, i0);
            r1 = fma(a, v1.x, r1);
            i1 = fma(a, v1.y, i1);
            r2 = fma(a, v2.x, r2);
            i2 = fma(a, v2.y, i2);
        }
        y0[n] = c2(r0, i0);
        y1[n] = c2(r1, i1);
        y2[n] = c2(r2, i2);
    }
}

// ---------------------------------------------------------------------------
// Stokes solve S (kappa > 0) by the influence-matrix method in the fixed
// tau eigenbasis.  Writes (ox, oy, oz) = velocity of the Chebyshev-tau
// solution for forcing (Fx, Fy, Fz).  w: 10 scratch vectors.
//   h  = D Fy + i a Fx + i b Fz                  (divergence of the forcing)
//   p0 = Poisson-tau solve (D^2 - k^2) p0 = h, p0(+-1) = 0
//   v0 = Helmholtz-tau solve (sig - nu D^2) v0 = Fy - D p0, v0(+-1) = 0
//   c  = -A^{-1} (Dv0(+1), Dv0(-1), tau residuals of the v equation)
//   v  = v0 + sum_k c_k v_k   (homogeneous responses: Dirichlet data of p
//                              and the tau correction of the Poisson equation)
//   eta = Helmholtz-tau solve of (i b Fx - i a Fz)   (wall-normal vorticity)
//   u_x = (i a Dv - i b eta)/k^2, u_z = (i b Dv + i a eta)/k^2
// ---------------------------------------------------------------------------
__device__ void stokes(const KP& p, int m, const MS& c, const double2* Fx, const double2* Fy,
                       const double2* Fz, double2* ox, double2* oy, double2* oz, double2* w) {
    const int N = p.N, M = N - 2, t = threadIdx.x;
    double2 *Fh = w, *Fe = w + N, *h = w + 2 * N, *t1 = w + 3 * N, *t2 = w + 4 * N,
            *p0 = w + 5 * N, *eta = w + 6 * N, *q = w + 7 * N, *v0 = w + 8 * N,
            *Dv0 = w + 9 * N;
    const double* dH = p.dH + (size_t)m * N;
    const double* dP = p.dP + (size_t)m * N;
    for (int n = t; n < N; n += MODE_THREADS) {
        const double2 fx = Fx[n], fz = Fz[n];
        Fh[n] = cadd(imul(c.a, fx), imul(c.b, fz));
        Fe[n] = csub(imul(c.b, fx), imul(c.a, fz));
    }
    __syncthreads();
    mv(p, M_D, N, N, Fy, h);
    __syncthreads();
    for (int n = t; n < M; n += MODE_THREADS) h[n] = cscl(-1.0, cadd(h[n], Fh[n]));
    __syncthreads();
    mv(p, M_PR, M, M, h, t1);
    mv(p, M_PR, M, M, Fe, t2);
    __syncthreads();
    for (int n = t; n < M; n += MODE_THREADS) {
        t1[n] = cscl(dP[n], t1[n]);
        t2[n] = cscl(dH[n], t2[n]);
    }
    __syncthreads();
    mv(p, M_PL, M, N, t1, p0);
    mv(p, M_PL, M, N, t2, eta);
    __syncthreads();
    mv(p, M_D, N, N, p0, q);
    __syncthreads();
    for (int n = t; n < N; n += MODE_THREADS) q[n] = csub(Fy[n], q[n]);
    __syncthreads();
    mv(p, M_PR, M, M, q, t1);
    __syncthreads();
    for (int n = t; n < M; n += MODE_THREADS) t1[n] = cscl(dH[n], t1[n]);
    __syncthreads();
    mv(p, M_PL, M, N, t1, v0);
    __syncthreads();
    mv(p, M_D, N, N, v0, Dv0);
    __syncthreads();
    double spr = 0, spi = 0, smr = 0, smi = 0;
    for (int n = t; n < N; n += MODE_THREADS) {
        const double2 d = Dv0[n];
        spr += d.x;
        spi += d.y;
        smr += (n & 1) ? -d.x : d.x;
        smi += (n & 1) ? -d.y : d.y;
    }
    const double2 e0 = c2(wsum(spr), wsum(spi)), e1 = c2(wsum(smr), wsum(smi));
    const double tn = 2.0 * (N - 1);
    const double2 e2 = csub(cadd(cscl(c.sig, v0[N - 2]), cscl(tn, p0[N - 1])), Fy[N - 2]);
    const double2 e3 = csub(cscl(c.sig, v0[N - 1]), Fy[N - 1]);
    const double* Ai = p.Ainv + (size_t)m * 16;
    double2 cc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double2 s = cadd(cadd(cscl(Ai[4 * k], e0), cscl(Ai[4 * k + 1], e1)),
                         cadd(cscl(Ai[4 * k + 2], e2), cscl(Ai[4 * k + 3], e3)));
        cc[k] = cscl(-1.0, s);
    }
    const double* Vk = p.Vk + (size_t)m * 4 * N;
    const double* DVk = p.DVk + (size_t)m * 4 * N;
    for (int n = t; n < N; n += MODE_THREADS) {
        double2 v = v0[n], Dv = Dv0[n];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v = cadd(v, cscl(Vk[k * N + n], cc[k]));
            Dv = cadd(Dv, cscl(DVk[k * N + n], cc[k]));
        }
        const double2 e = eta[n];
        ox[n] = cscl(c.ik2, csub(imul(c.a, Dv), imul(c.b, e)));
        oy[n] = v;
        oz[n] = cscl(c.ik2, cadd(imul(c.b, Dv), imul(c.a, e)));
    }
    __syncthreads();
}

// Conjugate transpose of stokes(): (yx, yy, yz) = S^H (xu, xv, xw), obtained by
// running the steps above backwards with every matrix transposed.  w: 12 vectors.
__device__ void stokes_h(const KP& p, int m, const MS& c, const double2* xu, const double2* xv,
                         const double2* xw, double2* yx, double2* yy, double2* yz,
                         double2* w) {
    const int N = p.N, M = N - 2, t = threadIdx.x;
    double2 *bDv = w, *beta = w + N, *bv = w + 2 * N, *bDv0 = w + 3 * N, *bv0 = w + 4 * N,
            *bp0 = w + 5 * N, *bFy = w + 6 * N, *bq = w + 7 * N, *bh = w + 8 * N,
            *tt = w + 9 * N, *tu = w + 10 * N, *bFe = w + 11 * N;
    const double* dH = p.dH + (size_t)m * N;
    const double* dP = p.dP + (size_t)m * N;
    for (int n = t; n < N; n += MODE_THREADS) {
        const double2 a0 = xu[n], a2 = xw[n];
        bDv[n] = cscl(c.ik2, cadd(imul(-c.a, a0), imul(-c.b, a2)));
        beta[n] = cscl(c.ik2, csub(imul(c.b, a0), imul(c.a, a2)));
    }
    __syncthreads();
    mv(p, M_DT, N, N, bDv, tt);
    __syncthreads();
    for (int n = t; n < N; n += MODE_THREADS) bv[n] = cadd(xv[n], tt[n]);
    __syncthreads();
    const double* Vk = p.Vk + (size_t)m * 4 * N;
    double2 bc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double sr = 0, si = 0;
        for (int n = t; n < N; n += MODE_THREADS) {
            sr += Vk[k * N + n] * bv[n].x;
            si += Vk[k * N + n] * bv[n].y;
        }
        bc[k] = c2(wsum(sr), wsum(si));
    }
    const double* Ai = p.Ainv + (size_t)m * 16;
    double2 be[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double2 s = cadd(cadd(cscl(Ai[j], bc[0]), cscl(Ai[4 + j], bc[1])),
                         cadd(cscl(Ai[8 + j], bc[2]), cscl(Ai[12 + j], bc[3])));
        be[j] = cscl(-1.0, s);
    }
    for (int n = t; n < N; n += MODE_THREADS) bDv0[n] = (n & 1) ? csub(be[0], be[1]) : cadd(be[0], be[1]);
    __syncthreads();
    mv(p, M_DT, N, N, bDv0, tt);
    __syncthreads();
    const double tn = 2.0 * (N - 1);
    for (int n = t; n < N; n += MODE_THREADS) {
        double2 x = cadd(bv[n], tt[n]);
        if (n == N - 2) x = cadd(x, cscl(c.sig, be[2]));
        if (n == N - 1) x = cadd(x, cscl(c.sig, be[3]));
        bv0[n] = x;
        bp0[n] = (n == N - 1) ? cscl(tn, be[2]) : c2(0, 0);
        bFy[n] = (n == N - 2) ? cscl(-1.0, be[2]) : ((n == N - 1) ? cscl(-1.0, be[3]) : c2(0, 0));
    }
    __syncthreads();
    mv(p, M_PLT, N, M, bv0, tt);
    mv(p, M_PLT, N, M, beta, tu);
    __syncthreads();
    for (int n = t; n < M; n += MODE_THREADS) {
        tt[n] = cscl(dH[n], tt[n]);
        tu[n] = cscl(dH[n], tu[n]);
    }
    __syncthreads();
    mv(p, M_PRT, M, M, tt, bq);
    mv(p, M_PRT, M, M, tu, bFe);
    for (int n = M + t; n < N; n += MODE_THREADS) {
        bq[n] = c2(0, 0);
        bFe[n] = c2(0, 0);
    }
    __syncthreads();
    mv(p, M_DT, N, N, bq, tt);
    __syncthreads();
    for (int n = t; n < N; n += MODE_THREADS) {
        bFy[n] = cadd(bFy[n], bq[n]);
        bp0[n] = csub(bp0[n], tt[n]);
    }
    __syncthreads();
    mv(p, M_PLT, N, M, bp0, tu);
    __syncthreads();
    for (int n = t; n < M; n += MODE_THREADS) tu[n] = cscl(dP[n], tu[n]);
    __syncthreads();
    mv(p, M_PRT, M, M, tu, bh);
    __syncthreads();
    for (int n = t; n < N; n += MODE_THREADS) bh[n] = (n < M) ? cscl(-1.0, bh[n]) : c2(0, 0);
    __syncthreads();
    mv(p, M_DT, N, N, bh, tt);
    __syncthreads();
    for (int n = t; n < N; n += MODE_THREADS) {
        const double2 h = bh[n], e = bFe[n];
        yx[n] = cadd(imul(-c.a, h), imul(-c.b, e));
        yy[n] = cadd(bFy[n], tt[n]);
        yz[n] = cadd(imul(-c.b, h), imul(c.a, e));
    }
    __syncthreads();
}

// (0,0) mode: u_x and u_z solve the Dirichlet tau Helmholtz problem with
// sigma = lam, u_y = 0.  w: 2 scratch vectors.
__device__ void stokes0(const KP& p, const double2* Fx, const double2* Fz, double2* ox,
                        double2* oy, double2* oz, double2* w) {
    const int N = p.N, M = N - 2, t = threadIdx.x;
    double2 *t1 = w, *t2 = w + N;
    const double* dH = p.dH;
    mv(p, M_PR, M, M, Fx, t1);
    mv(p, M_PR, M, M, Fz, t2);
    __syncthreads();
    for (int n = t; n < M; n += MODE_THREADS) {
        t1[n] = cscl(dH[n], t1[n]);
        t2[n] = cscl(dH[n], t2[n]);
    }
    __syncthreads();
    mv(p, M_PL, M, N, t1, ox);
    mv(p, M_PL, M, N, t2, oz);
    for (int n = t; n < N; n += MODE_THREADS) oy[n] = c2(0, 0);
    __syncthreads();
}

__device__ void stokes0_h(const KP& p, const double2* xu, const double2* xw, double2* yx,
                          double2* yy, double2* yz, double2* w) {
    const int N = p.N, M = N - 2, t = threadIdx.x;
    double2 *t1 = w, *t2 = w + N;
    const double* dH = p.dH;
    mv(p, M_PLT, N, M, xu, t1);
    mv(p, M_PLT, N, M, xw, t2);
    __syncthreads();
    for (int n = t; n < M; n += MODE_THREADS) {
        t1[n] = cscl(dH[n], t1[n]);
        t2[n] = cscl(dH[n], t2[n]);
    }
    __syncthreads();
    mv(p, M_PRT, M, M, t1, yx);
    mv(p, M_PRT, M, M, t2, yz);
    for (int n = t; n < N; n += MODE_THREADS) {
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
// w: 9 scratch vectors.
__device__ void project(const KP& p, int m, const MS& c, const double2* gx, const double2* gy,
                        const double2* gz, double2* ox, double2* oy, double2* oz, double2* w) {
    const int N = p.N, t = threadIdx.x;
    double2 *gh = w, *ge = w + N, *t1 = w + 2 * N, *t2 = w + 3 * N, *bv = w + 4 * N,
            *t4 = w + 5 * N, *v = w + 6 * N, *eta = w + 7 * N, *Dv = w + 8 * N;
    const double* dq = p.dproj + (size_t)m * N;
    for (int n = t; n < N; n += MODE_THREADS) {
        const double2 x = gx[n], z = gz[n];
        gh[n] = cadd(imul(c.a, x), imul(c.b, z));
        ge[n] = csub(imul(c.b, x), imul(c.a, z));
    }
    __syncthreads();
    mv(p, M_DTG, N, N, gh, t1);
    mv(p, M_G, N, N, gy, t2);
    mv(p, M_PID, N, N, ge, eta);
    __syncthreads();
    for (int n = t; n < N; n += MODE_THREADS) bv[n] = csub(t2[n], cscl(c.ik2, t1[n]));
    __syncthreads();
    mv(p, M_PVLT, N, N - 4, bv, t4);
    __syncthreads();
    for (int n = t; n < N - 4; n += MODE_THREADS) t4[n] = cscl(dq[n], t4[n]);
    __syncthreads();
    mv(p, M_PVL, N - 4, N, t4, v);
    __syncthreads();
    mv(p, M_D, N, N, v, Dv);
    __syncthreads();
    for (int n = t; n < N; n += MODE_THREADS) {
        const double2 d = Dv[n], e = eta[n];
        ox[n] = cscl(c.ik2, csub(imul(c.a, d), imul(c.b, e)));
        oy[n] = v[n];
        oz[n] = cscl(c.ik2, cadd(imul(c.b, d), imul(c.a, e)));
    }
    __syncthreads();
}

__device__ void project0(const KP& p, const double2* gx, const double2* gz, double2* ox,
                         double2* oy, double2* oz) {
    const int N = p.N;
    mv(p, M_PID, N, N, gx, ox);
    mv(p, M_PID, N, N, gz, oz);
    for (int n = threadIdx.x; n < N; n += MODE_THREADS) oy[n] = c2(0, 0);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// y-values of u and of du/dy for the three components: Y[c] = C u_c,
// Y[3+c] = C D u_c (Gauss-Lobatto synthesis).
__global__ __launch_bounds__(MODE_THREADS) void k_synth(KP p, const double2* __restrict__ u,
                                                        double2* __restrict__ Y) {
    extern __shared__ double2 sm[];
    const int m = xcd_item(blockIdx.x, gridDim.x), N = p.N, nm = p.nm, t = threadIdx.x;
    if (m >= nm) return;
    double2* V = sm;
    for (int i = 0; i < 3; ++i)
        for (int n = t; n < N; n += MODE_THREADS) V[i * N + n] = u[((size_t)i * nm + m) * N + n];
    __syncthreads();
    mv3(p, M_C, N, N, V, V + N, V + 2 * N, V + 3 * N, V + 4 * N, V + 5 * N);
    mv3(p, M_CD, N, N, V, V + N, V + 2 * N, V + 6 * N, V + 7 * N, V + 8 * N);
    __syncthreads();
    for (int f = 0; f < 6; ++f)
        for (int j = t; j < N; j += MODE_THREADS)
            Y[((size_t)f * N + j) * nm + m] = V[(3 + f) * N + j];
}

template <int MODE>
__global__ __launch_bounds__(PLANE_THREADS) void k_plane(KP p, const double2* __restrict__ Y1,
                                                         const double2* __restrict__ Y2,
                                                         double2* __restrict__ out) {
    extern __shared__ double2 sm[];
    constexpr int NG3 = (MODE == PLANE_JVP) ? 6 : 3;  // velocity fields: (V, i a V, W) groups
    constexpr int NG1 = (MODE == PLANE_ADJ) ? 3 : 0;  // adjoint fields: single outputs
    constexpr int NXF = 3 * NG3 + NG1;
    constexpr int NZF = (MODE == PLANE_ADJ) ? 9 : 3;  // after the forward z stage
    const int item = xcd_item(blockIdx.x, gridDim.x);
    if (item >= p.NS * p.N) return;
    const int j = item / p.NS, s = item - j * p.NS;   // the slabs of a plane run on one XCD
    const int N = p.N, Nx = p.Nx, Nz = p.Nz, nkx = p.nkx, nkz = p.nkz, nm = p.nm, XS = p.XS;
    const int Kx = p.Kx;
    const int x0 = s * XS, tid = threadIdx.x;
    const int per = XS * nkz, pz = XS * Nz;
    double2* twx = sm;
    double2* twz = twx + Nx;
    double2* xb = twz + Nz;
    double* pb = reinterpret_cast<double*>(xb + NXF * per);
    for (int i = tid; i < Nx; i += PLANE_THREADS) twx[i] = p.twx[i];
    for (int i = tid; i < Nz; i += PLANE_THREADS) twz[i] = p.twz[i];
    __syncthreads();

    // inverse transform in x for the slab's x positions, all retained kz
    for (int it = tid; it < (NG3 + NG1) * per; it += PLANE_THREADS) {
        const int g = it / per, rem = it - g * per, xl = rem / nkz, kz = rem - xl * nkz;
        const int x = x0 + xl;
        if (g < NG3) {
            const double2* src = (g < 3) ? Y1 : Y2;
            const int comp = g % 3;
            const double2* Vp = src + ((size_t)comp * N + j) * nm + kz;
            const double2* Wp = src + ((size_t)(3 + comp) * N + j) * nm + kz;
            double2 aV = c2(0, 0), aA = c2(0, 0), aW = c2(0, 0);
            const int step = x % Nx;
            int idx = 0;                                   // (kx * x) mod Nx, kx = 0, 1, ..
            for (int ikx = 0; ikx < nkx; ++ikx) {
                if (ikx == Kx + 1) idx = (Nx - (Kx * x) % Nx) % Nx;   // kx = -Kx
                const int kx = (ikx <= Kx) ? ikx : ikx - nkx;
                const double2 tw = twx[idx];
                const double2 vt = cmul(Vp[(size_t)ikx * nkz], tw);
                aV = cadd(aV, vt);
                aA = cadd(aA, imul(p.alpha * kx, vt));
                aW = cadd(aW, cmul(Wp[(size_t)ikx * nkz], tw));
                idx += step;
                if (idx >= Nx) idx -= Nx;
            }
            xb[(3 * g) * per + rem] = aV;
            xb[(3 * g + 1) * per + rem] = aA;
            xb[(3 * g + 2) * per + rem] = aW;
        } else {
            const int comp = g - NG3;
            const double2* Ap = Y2 + ((size_t)comp * N + j) * nm + kz;
            double2 acc = c2(0, 0);
            const int step = x % Nx;
            int idx = 0;
            for (int ikx = 0; ikx < nkx; ++ikx) {
                if (ikx == Kx + 1) idx = (Nx - (Kx * x) % Nx) % Nx;
                acc = cadd(acc, cmul(Ap[(size_t)ikx * nkz], twx[idx]));
                idx += step;
                if (idx >= Nx) idx -= Nx;
            }
            xb[(3 * NG3 + comp) * per + rem] = acc;
        }
    }
    __syncthreads();

    // inverse (complex-to-real) transform in z at each point, then the products
    const double yj = p.ygl[j];
    for (int pt = tid; pt < pz; pt += PLANE_THREADS) {
        const int xl = pt / Nz, z = pt - xl * Nz;
        double val[NG3][4];  // U, dU/dx, dU/dy, dU/dz of each velocity field
#pragma unroll
        for (int g = 0; g < NG3; ++g) {
            const double2* cV = xb + (3 * g) * per + xl * nkz;
            const double2* cA = xb + (3 * g + 1) * per + xl * nkz;
            const double2* cW = xb + (3 * g + 2) * per + xl * nkz;
            double sV = 0, sZ = 0, sA = 0, sW = 0;
            int idx = 0;                                   // (kz * z) mod Nz
            for (int kz = 1; kz < nkz; ++kz) {
                idx += z;
                if (idx >= Nz) idx -= Nz;
                const double2 tw = twz[idx];
                const double2 t = cmul(cV[kz], tw);
                sV += t.x;
                sZ += p.beta * kz * t.y;
                sA += cmul(cA[kz], tw).x;
                sW += cmul(cW[kz], tw).x;
            }
            val[g][0] = cV[0].x + 2.0 * sV;
            val[g][1] = cA[0].x + 2.0 * sA;
            val[g][2] = cW[0].x + 2.0 * sW;
            val[g][3] = -2.0 * sZ;
        }
        val[0][0] += yj;   // base flow u_b = y e_x
        val[0][2] += 1.0;  // d(u_b)_x / dy = 1
        if (MODE == PLANE_FWD) {
#pragma unroll
            for (int i = 0; i < 3; ++i)
                pb[i * pz + pt] = val[0][0] * val[i][1] + val[1][0] * val[i][2] + val[2][0] * val[i][3];
        } else if (MODE == PLANE_JVP) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                double q = 0;
#pragma unroll
                for (int jj = 0; jj < 3; ++jj)
                    q += val[jj][0] * val[3 + i][1 + jj] + val[3 + jj][0] * val[i][1 + jj];
                pb[i * pz + pt] = q;
            }
        } else {
            double at[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double2* cc = xb + (3 * NG3 + i) * per + xl * nkz;
                double sr = 0;
                int idx = 0;
                for (int kz = 1; kz < nkz; ++kz) {
                    idx += z;
                    if (idx >= Nz) idx -= Nz;
                    sr += cmul(cc[kz], twz[idx]).x;
                }
                at[i] = cc[0].x + 2.0 * sr;
            }
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int jj = 0; jj < 3; ++jj) pb[(3 * i + jj) * pz + pt] = val[jj][0] * at[i];
#pragma unroll
            for (int jj = 0; jj < 3; ++jj)
                pb[(9 + jj) * pz + pt] =
                    val[0][1 + jj] * at[0] + val[1][1 + jj] * at[1] + val[2][1 + jj] * at[2];
        }
    }
    __syncthreads();

    // forward transform in z (normalised), into xb
    const double invNz = 1.0 / Nz, invNx = 1.0 / Nx;
    for (int it = tid; it < NZF * per; it += PLANE_THREADS) {
        const int o = it / per, rem = it - o * per, xl = rem / nkz, kz = rem - xl * nkz;
        if (MODE != PLANE_ADJ) {
            const double* q = pb + o * pz + xl * Nz;
            double ar = 0, ai = 0;
            for (int z = 0, idx = 0; z < Nz; ++z, idx = (idx + kz >= Nz) ? idx + kz - Nz : idx + kz) {
                const double2 tw = twz[idx];
                ar += q[z] * tw.x;
                ai -= q[z] * tw.y;
            }
            xb[o * per + rem] = c2(ar * invNz, ai * invNz);
        } else {
            const int i = o / 3, kind = o - 3 * i;
            if (kind == 0) {  // Q_i - i b P_{i,z}
                const double* q1 = pb + (9 + i) * pz + xl * Nz;
                const double* q2 = pb + (3 * i + 2) * pz + xl * Nz;
                double ar = 0, ai = 0, br = 0, bi = 0;
                for (int z = 0, idx = 0; z < Nz; ++z, idx = (idx + kz >= Nz) ? idx + kz - Nz : idx + kz) {
                    const double2 tw = twz[idx];
                    ar += q1[z] * tw.x;
                    ai -= q1[z] * tw.y;
                    br += q2[z] * tw.x;
                    bi -= q2[z] * tw.y;
                }
                const double2 r = csub(c2(ar, ai), imul(p.beta * kz, c2(br, bi)));
                xb[o * per + rem] = cscl(invNz, r);
            } else {  // P_{i,x} (kind 1) or P_{i,y} (kind 2)
                const double* q = pb + (3 * i + (kind - 1)) * pz + xl * Nz;
                double ar = 0, ai = 0;
                for (int z = 0, idx = 0; z < Nz; ++z, idx = (idx + kz >= Nz) ? idx + kz - Nz : idx + kz) {
                    const double2 tw = twz[idx];
                    ar += q[z] * tw.x;
                    ai -= q[z] * tw.y;
                }
                xb[o * per + rem] = c2(ar * invNz, ai * invNz);
            }
        }
    }
    __syncthreads();

    // forward transform in x over this slab (partial sum), retained modes only
    constexpr int NOUT = (MODE == PLANE_ADJ) ? 6 : 3;
    for (int it = tid; it < NOUT * nm; it += PLANE_THREADS) {
        const int o = it / nm, mm = it - o * nm, ikx = mm / nkz, kz = mm - ikx * nkz;
        const int kx = (ikx <= Kx) ? ikx : ikx - nkx;
        const int kstep = ((kx % Nx) + Nx) % Nx;            // kx mod Nx
        const int idx0 = (int)(((long long)kstep * x0) % Nx);  // (kx * x0) mod Nx
        double2 res;
        if (MODE != PLANE_ADJ) {
            double ar = 0, ai = 0;
            for (int xl = 0, idx = idx0; xl < XS; ++xl, idx = (idx + kstep >= Nx) ? idx + kstep - Nx : idx + kstep) {
                const double2 tw = twx[idx], v = xb[o * per + xl * nkz + kz];
                ar += v.x * tw.x + v.y * tw.y;
                ai += v.y * tw.x - v.x * tw.y;
            }
            res = c2(ar * invNx, ai * invNx);
        } else if (o < 3) {  // X_i = F(A_i) - i a F(B_i)
            double ar = 0, ai = 0, br = 0, bi = 0;
            for (int xl = 0, idx = idx0; xl < XS; ++xl, idx = (idx + kstep >= Nx) ? idx + kstep - Nx : idx + kstep) {
                const double2 tw = twx[idx];
                const double2 va = xb[(3 * o) * per + xl * nkz + kz];
                const double2 vb = xb[(3 * o + 1) * per + xl * nkz + kz];
                ar += va.x * tw.x + va.y * tw.y;
                ai += va.y * tw.x - va.x * tw.y;
                br += vb.x * tw.x + vb.y * tw.y;
                bi += vb.y * tw.x - vb.x * tw.y;
            }
            res = cscl(invNx, csub(c2(ar, ai), imul(p.alpha * kx, c2(br, bi))));
        } else {  // Y_i = F(C_i)
            const int i = o - 3;
            double ar = 0, ai = 0;
            for (int xl = 0, idx = idx0; xl < XS; ++xl, idx = (idx + kstep >= Nx) ? idx + kstep - Nx : idx + kstep) {
                const double2 tw = twx[idx], v = xb[(3 * i + 2) * per + xl * nkz + kz];
                ar += v.x * tw.x + v.y * tw.y;
                ai += v.y * tw.x - v.x * tw.y;
            }
            res = c2(ar * invNx, ai * invNx);
        }
        out[(((size_t)s * NOUT + o) * N + j) * nm + mm] = res;
    }
}

__global__ __launch_bounds__(MODE_THREADS) void k_mode_res(
    KP p, int flags, const double2* __restrict__ P3, const double2* __restrict__ u,
    double2* __restrict__ r, double* __restrict__ cost_part, double2* __restrict__ a,
    double2* __restrict__ Atil) {
    extern __shared__ double2 sm[];
    const int m = xcd_item(blockIdx.x, gridDim.x), N = p.N, nm = p.nm, t = threadIdx.x;
    if (m >= nm) return;
    auto vec = [&](int k) { return sm + (size_t)k * N; };
    const MS c = mscal(p, m);
    const bool zero = (m == 0);
    double2 *R0 = vec(9), *R1 = vec(10), *R2 = vec(11);
    if (flags & RES_INPUT_W) {
        for (int i = 0; i < 3; ++i)
            for (int n = t; n < N; n += MODE_THREADS) vec(9 + i)[n] = u[((size_t)i * nm + m) * N + n];
        __syncthreads();
    } else {
        for (int i = 0; i < 3; ++i)
            for (int n = t; n < N; n += MODE_THREADS) {
                double2 acc = c2(0, 0);
                for (int s = 0; s < p.NS; ++s) acc = cadd(acc, P3[(((size_t)s * 3 + i) * N + n) * nm + m]);
                vec(i)[n] = acc;
                vec(3 + i)[n] = u[((size_t)i * nm + m) * N + n];
            }
        __syncthreads();
        mv3(p, M_CINV, N, N, vec(0), vec(1), vec(2), vec(6), vec(7), vec(8));
        __syncthreads();
        mv3(p, M_D2, N, N, vec(3), vec(4), vec(5), vec(0), vec(1), vec(2));
        __syncthreads();
        for (int i = 0; i < 3; ++i)
            for (int n = t; n < N; n += MODE_THREADS) {
                const double2 L = csub(vec(i)[n], cscl(c.k2, vec(3 + i)[n]));
                vec(6 + i)[n] = cadd(cscl(-1.0, vec(6 + i)[n]), cscl(p.nu, L));
            }
        __syncthreads();
        if (zero)
            stokes0(p, vec(6), vec(8), R0, R1, R2, vec(12));
        else
            stokes(p, m, c, vec(6), vec(7), vec(8), R0, R1, R2, vec(12));
        for (int i = 0; i < 3; ++i)
            for (int n = t; n < N; n += MODE_THREADS) {
                const double2 v = cscl(p.lam, vec(9 + i)[n]);
                vec(9 + i)[n] = v;
                if (flags & RES_WRITE_R) r[((size_t)i * nm + m) * N + n] = v;
            }
        __syncthreads();
    }
    if (!(flags & (RES_COST | RES_ADJ))) return;
    mv3(p, M_G, N, N, R0, R1, R2, vec(3), vec(4), vec(5));
    __syncthreads();
    if (flags & RES_COST) {
        double s = 0;
        for (int i = 0; i < 3; ++i)
            for (int n = t; n < N; n += MODE_THREADS) {
                const double2 x = vec(9 + i)[n], y = vec(3 + i)[n];
                s += x.x * y.x + x.y * y.y;
            }
        s = wsum(s);
        if (t == 0) cost_part[m] = c.wgt * s;
    }
    if (!(flags & RES_ADJ)) return;
    if (zero)
        stokes0_h(p, vec(3), vec(5), vec(6), vec(7), vec(8), vec(12));
    else
        stokes_h(p, m, c, vec(3), vec(4), vec(5), vec(6), vec(7), vec(8), vec(12));
    mv3(p, M_GINV, N, N, vec(6), vec(7), vec(8), vec(0), vec(1), vec(2));
    mv3(p, M_CINVT, N, N, vec(6), vec(7), vec(8), vec(12), vec(13), vec(14));
    __syncthreads();
    for (int i = 0; i < 3; ++i)
        for (int n = t; n < N; n += MODE_THREADS) {
            a[((size_t)i * nm + m) * N + n] = vec(i)[n];
            Atil[((size_t)i * N + n) * nm + m] = vec(12 + i)[n];
        }
}

__global__ __launch_bounds__(MODE_THREADS) void k_mode_grad(KP p, int flags,
                                                            const double2* __restrict__ P6,
                                                            const double2* __restrict__ a,
                                                            double dtau, double2* __restrict__ uo,
                                                            double2* __restrict__ Y) {
    extern __shared__ double2 sm[];
    const int m = xcd_item(blockIdx.x, gridDim.x), N = p.N, nm = p.nm, t = threadIdx.x;
    if (m >= nm) return;
    auto vec = [&](int k) { return sm + (size_t)k * N; };
    const MS c = mscal(p, m);
    const bool zero = (m == 0);
    for (int i = 0; i < 3; ++i)
        for (int n = t; n < N; n += MODE_THREADS) {
            double2 sx = c2(0, 0), sy = c2(0, 0);
            for (int s = 0; s < p.NS; ++s) {
                sx = cadd(sx, P6[(((size_t)s * 6 + i) * N + n) * nm + m]);
                sy = cadd(sy, P6[(((size_t)s * 6 + 3 + i) * N + n) * nm + m]);
            }
            vec(i)[n] = sx;
            vec(3 + i)[n] = sy;
            vec(6 + i)[n] = a[((size_t)i * nm + m) * N + n];
        }
    __syncthreads();
    mv3(p, M_MA, N, N, vec(0), vec(1), vec(2), vec(9), vec(10), vec(11));
    __syncthreads();
    mv3(p, M_MB, N, N, vec(3), vec(4), vec(5), vec(0), vec(1), vec(2));
    __syncthreads();
    mv3(p, M_ML, N, N, vec(6), vec(7), vec(8), vec(3), vec(4), vec(5));
    __syncthreads();
    for (int i = 0; i < 3; ++i)
        for (int n = t; n < N; n += MODE_THREADS) {
            const double2 adv = cadd(vec(9 + i)[n], vec(i)[n]);
            const double2 lap = csub(vec(3 + i)[n], cscl(c.k2, vec(6 + i)[n]));
            vec(9 + i)[n] = cscl(p.lam, csub(cscl(p.nu, lap), adv));
        }
    __syncthreads();
    double2 *F0 = vec(9), *F1 = vec(10), *F2 = vec(11);
    if (flags & GRAD_PROJECT) {
        if (zero)
            project0(p, vec(9), vec(11), vec(0), vec(1), vec(2));
        else
            project(p, m, c, vec(9), vec(10), vec(11), vec(0), vec(1), vec(2), vec(12));
        for (int i = 0; i < 3; ++i)
            for (int n = t; n < N; n += MODE_THREADS) vec(i)[n] = cscl(-1.0, vec(i)[n]);
        __syncthreads();
        F0 = vec(0);
        F1 = vec(1);
        F2 = vec(2);
    }
    double2* Fs[3] = {F0, F1, F2};
    if (flags & GRAD_UPDATE) {
        for (int i = 0; i < 3; ++i)
            for (int n = t; n < N; n += MODE_THREADS) {
                const size_t gi = ((size_t)i * nm + m) * N + n;
                const double2 un = cadd(uo[gi], cscl(dtau, Fs[i][n]));
                uo[gi] = un;
                vec(3 + i)[n] = un;
            }
        __syncthreads();
        mv3(p, M_C, N, N, vec(3), vec(4), vec(5), vec(6), vec(7), vec(8));
        mv3(p, M_CD, N, N, vec(3), vec(4), vec(5), vec(12), vec(13), vec(14));
        __syncthreads();
        for (int i = 0; i < 3; ++i)
            for (int n = t; n < N; n += MODE_THREADS) {
                Y[((size_t)i * N + n) * nm + m] = vec(6 + i)[n];
                Y[((size_t)(3 + i) * N + n) * nm + m] = vec(12 + i)[n];
            }
    } else {
        for (int i = 0; i < 3; ++i)
            for (int n = t; n < N; n += MODE_THREADS) uo[((size_t)i * nm + m) * N + n] = Fs[i][n];
    }
}

__global__ __launch_bounds__(MODE_THREADS) void k_project(KP p, const double2* __restrict__ g,
                                                          double2* __restrict__ out) {
    extern __shared__ double2 sm[];
    const int m = xcd_item(blockIdx.x, gridDim.x), N = p.N, nm = p.nm, t = threadIdx.x;
    if (m >= nm) return;
    auto vec = [&](int k) { return sm + (size_t)k * N; };
    for (int i = 0; i < 3; ++i)
        for (int n = t; n < N; n += MODE_THREADS) vec(i)[n] = g[((size_t)i * nm + m) * N + n];
    __syncthreads();
    if (m == 0)
        project0(p, vec(0), vec(2), vec(3), vec(4), vec(5));
    else
        project(p, m, mscal(p, m), vec(0), vec(1), vec(2), vec(3), vec(4), vec(5), vec(12));
    for (int i = 0; i < 3; ++i)
        for (int n = t; n < N; n += MODE_THREADS) out[((size_t)i * nm + m) * N + n] = vec(3 + i)[n];
}

// Deterministic column reductions of per-mode partials: out[c] = sum (op 0) or
// max (op 1) over rows of part[row * stride + c].
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ part, int n, int stride,
                                                int op, double* __restrict__ out) {
    __shared__ double red[256];
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
        if (threadIdx.x == 0) out[c] = red[0];
        __syncthreads();
    }
}

// Per-mode partials of ||u||^2, ||u_b + u||^2 and <curl U, curl U> (U = u_b + u).
__global__ __launch_bounds__(MODE_THREADS) void k_norms(KP p, const double2* __restrict__ u,
                                                        double* __restrict__ part) {
    extern __shared__ double2 sm[];
    const int m = xcd_item(blockIdx.x, gridDim.x), N = p.N, nm = p.nm, t = threadIdx.x;
    if (m >= nm) return;
    auto vec = [&](int k) { return sm + (size_t)k * N; };
    const MS c = mscal(p, m);
    for (int i = 0; i < 3; ++i)
        for (int n = t; n < N; n += MODE_THREADS) vec(i)[n] = u[((size_t)i * nm + m) * N + n];
    __syncthreads();
    mv3(p, M_G, N, N, vec(0), vec(1), vec(2), vec(3), vec(4), vec(5));
    __syncthreads();
    double s0 = 0;
    for (int i = 0; i < 3; ++i)
        for (int n = t; n < N; n += MODE_THREADS) s0 += vec(i)[n].x * vec(3 + i)[n].x + vec(i)[n].y * vec(3 + i)[n].y;
    s0 = wsum(s0);
    __syncthreads();
    if (m == 0 && t == 0) vec(0)[1] = cadd(vec(0)[1], c2(1.0, 0.0));  // + u_b = T_1(y) e_x
    __syncthreads();
    mv3(p, M_G, N, N, vec(0), vec(1), vec(2), vec(3), vec(4), vec(5));
    mv(p, M_D, N, N, vec(0), vec(6));
    mv(p, M_D, N, N, vec(2), vec(7));
    __syncthreads();
    double s1 = 0;
    for (int i = 0; i < 3; ++i)
        for (int n = t; n < N; n += MODE_THREADS) s1 += vec(i)[n].x * vec(3 + i)[n].x + vec(i)[n].y * vec(3 + i)[n].y;
    s1 = wsum(s1);
    // vorticity: (D U_z - i b U_y, i b U_x - i a U_z, i a U_y - D U_x)
    for (int n = t; n < N; n += MODE_THREADS) {
        const double2 ux = vec(0)[n], uy = vec(1)[n], uz = vec(2)[n];
        vec(8)[n] = csub(vec(7)[n], imul(c.b, uy));
        vec(9)[n] = csub(imul(c.b, ux), imul(c.a, uz));
        vec(10)[n] = csub(imul(c.a, uy), vec(6)[n]);
    }
    __syncthreads();
    mv3(p, M_G, N, N, vec(8), vec(9), vec(10), vec(11), vec(12), vec(13));
    __syncthreads();
    double s2 = 0;
    for (int i = 0; i < 3; ++i)
        for (int n = t; n < N; n += MODE_THREADS)
            s2 += vec(8 + i)[n].x * vec(11 + i)[n].x + vec(8 + i)[n].y * vec(11 + i)[n].y;
    s2 = wsum(s2);
    if (t == 0) {
        part[(size_t)m * 3 + 0] = c.wgt * s0;
        part[(size_t)m * 3 + 1] = c.wgt * s1;
        part[(size_t)m * 3 + 2] = c.wgt * s2;
    }
}

// Per-mode admissibility defects: max |div|, max |wall value|, Hermitian defect.
__global__ __launch_bounds__(MODE_THREADS) void k_check(KP p, const double2* __restrict__ u,
                                                        double* __restrict__ part) {
    extern __shared__ double2 sm[];
    const int m = xcd_item(blockIdx.x, gridDim.x), N = p.N, nm = p.nm, t = threadIdx.x;
    if (m >= nm) return;
    auto vec = [&](int k) { return sm + (size_t)k * N; };
    const MS c = mscal(p, m);
    for (int i = 0; i < 3; ++i)
        for (int n = t; n < N; n += MODE_THREADS) vec(i)[n] = u[((size_t)i * nm + m) * N + n];
    __syncthreads();
    mv(p, M_D, N, N, vec(1), vec(3));
    __syncthreads();
    double dv = 0, herm = 0;
    double wr[6] = {0, 0, 0, 0, 0, 0}, wi[6] = {0, 0, 0, 0, 0, 0};
    const int ikx = m / p.nkz, kz = m - ikx * p.nkz;
    const int kx = (ikx <= p.Kx) ? ikx : ikx - p.nkx;
    const int mp = ((p.nkx - ikx) % p.nkx) * p.nkz;
    for (int n = t; n < N; n += MODE_THREADS) {
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
                const double2 w = u[((size_t)i * nm + mp) * N + n];
                herm = fmax(herm, hypot(w.x - v.x, w.y + v.y));
            }
        }
    }
    double wall = 0;
    for (int q = 0; q < 6; ++q) wall = fmax(wall, hypot(wsum(wr[q]), wsum(wi[q])));
    dv = wmax(dv);
    herm = wmax(herm);
    if (t == 0) {
        part[(size_t)m * 3 + 0] = dv;
        part[(size_t)m * 3 + 1] = wall;
        part[(size_t)m * 3 + 2] = herm;
    }
}

__global__ __launch_bounds__(MODE_THREADS) void k_pack(KP p, const double2* __restrict__ u,
                                                       double* __restrict__ psi) {
    const int m = xcd_item(blockIdx.x, gridDim.x), N = p.N, nm = p.nm, t = threadIdx.x;
    if (m >= nm) return;
    const int idx = p.indep[m];
    if (idx < 0) return;
    if (m == 0) {
        for (int n = t; n < N - 2; n += MODE_THREADS) {
            psi[n] = u[(size_t)m * N + n].x;
            psi[(N - 2) + n] = u[((size_t)2 * nm + m) * N + n].x;
        }
        return;
    }
    const MS c = mscal(p, m);
    double* o = psi + 2 * (N - 2) + (size_t)idx * (4 * N - 12);
    for (int n = t; n < N; n += MODE_THREADS) {
        const double2 v = u[((size_t)nm + m) * N + n];
        const double2 e = csub(imul(c.b, u[(size_t)m * N + n]), imul(c.a, u[((size_t)2 * nm + m) * N + n]));
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
__device__ double2 par_sum(const double2* x, int lim, int par, bool sq) {
    double sr = 0, si = 0;
    for (int n = threadIdx.x; n < lim; n += MODE_THREADS)
        if ((n & 1) == par) {
            const double w = sq ? (double)n * n : 1.0;
            sr += w * x[n].x;
            si += w * x[n].y;
        }
    return c2(wsum(sr), wsum(si));
}

__global__ __launch_bounds__(MODE_THREADS) void k_unpack(KP p, const double* __restrict__ psi,
                                                         double2* __restrict__ u) {
    extern __shared__ double2 sm[];
    const int m = xcd_item(blockIdx.x, gridDim.x), N = p.N, nm = p.nm, t = threadIdx.x;
    if (m >= nm) return;
    const int idx = p.indep[m];
    if (idx < 0) return;
    auto vec = [&](int k) { return sm + (size_t)k * N; };
    if (m == 0) {
        for (int n = t; n < N; n += MODE_THREADS) {
            vec(0)[n] = c2(n < N - 2 ? psi[n] : 0.0, 0);
            vec(1)[n] = c2(n < N - 2 ? psi[(N - 2) + n] : 0.0, 0);
        }
        __syncthreads();
        for (int f = 0; f < 2; ++f) {  // Dirichlet: each parity class sums to zero
            const double2 s0 = par_sum(vec(f), N - 2, (N - 2) & 1, false);
            const double2 s1 = par_sum(vec(f), N - 2, (N - 1) & 1, false);
            __syncthreads();
            if (t == 0) {
                vec(f)[N - 2] = cscl(-1.0, s0);
                vec(f)[N - 1] = cscl(-1.0, s1);
            }
            __syncthreads();
        }
        for (int n = t; n < N; n += MODE_THREADS) {
            u[(size_t)m * N + n] = vec(0)[n];
            u[((size_t)nm + m) * N + n] = c2(0, 0);
            u[((size_t)2 * nm + m) * N + n] = vec(1)[n];
        }
        return;
    }
    const MS c = mscal(p, m);
    const double* o = psi + 2 * (N - 2) + (size_t)idx * (4 * N - 12);
    double2 *v = vec(0), *e = vec(1), *Dv = vec(2);
    for (int n = t; n < N; n += MODE_THREADS) {
        v[n] = (n < N - 4) ? c2(o[n], o[(N - 4) + n]) : c2(0, 0);
        e[n] = (n < N - 2) ? c2(o[2 * (N - 4) + n], o[2 * (N - 4) + (N - 2) + n]) : c2(0, 0);
    }
    __syncthreads();
    // clamped v: within each parity class sum v_n = 0 and sum n^2 v_n = 0
    for (int q = N - 2; q < N; ++q) {
        const int pp = q - 2, par = q & 1;
        const double2 s0 = par_sum(v, pp, par, false), s2 = par_sum(v, pp, par, true);
        const double2 vq = cscl(1.0 / ((double)q * q - (double)pp * pp), csub(cscl((double)pp * pp, s0), s2));
        __syncthreads();
        if (t == 0) {
            v[q] = vq;
            v[pp] = csub(cscl(-1.0, s0), vq);
        }
        __syncthreads();
    }
    {
        const double2 s0 = par_sum(e, N - 2, (N - 2) & 1, false);
        const double2 s1 = par_sum(e, N - 2, (N - 1) & 1, false);
        __syncthreads();
        if (t == 0) {
            e[N - 2] = cscl(-1.0, s0);
            e[N - 1] = cscl(-1.0, s1);
        }
        __syncthreads();
    }
    mv(p, M_D, N, N, v, Dv);
    __syncthreads();
    const int ikx = m / p.nkz, kz = m - ikx * p.nkz;
    const int mp = ((p.nkx - ikx) % p.nkx) * p.nkz;
    for (int n = t; n < N; n += MODE_THREADS) {
        const double2 ux = cscl(c.ik2, csub(imul(c.a, Dv[n]), imul(c.b, e[n])));
        const double2 uz = cscl(c.ik2, cadd(imul(c.b, Dv[n]), imul(c.a, e[n])));
        const double2 vals[3] = {ux, v[n], uz};
        for (int i = 0; i < 3; ++i) {
            u[((size_t)i * nm + m) * N + n] = vals[i];
            if (kz == 0) u[((size_t)i * nm + mp) * N + n] = c2(vals[i].x, -vals[i].y);
        }
    }
}

__global__ void k_axpy(long long n, double a, const double* __restrict__ x, double* __restrict__ y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = fma(a, x[i], y[i]);
}

}  // namespace

size_t plane_lds_bytes(const KP& p, int mode) {
    const int ng3 = (mode == PLANE_JVP) ? 6 : 3, ng1 = (mode == PLANE_ADJ) ? 3 : 0;
    const int npf = (mode == PLANE_ADJ) ? 12 : 3;
    const size_t nxf = 3 * ng3 + ng1;
    return (size_t)(p.Nx + p.Nz) * 16 + nxf * p.XS * p.nkz * 16 + (size_t)npf * p.XS * p.Nz * 8;
}

size_t mode_lds_bytes(const KP& p) { return (size_t)MODE_VECS * p.N * 16; }

static dim3 mode_grid(const KP& p) { return dim3((unsigned)((p.nm + NXCD - 1) / NXCD * NXCD)); }

hipError_t launch_synth(const KP& p, hipStream_t s, const double2* u, double2* Y) {
    hipLaunchKernelGGL(k_synth, mode_grid(p), dim3(MODE_THREADS), 9 * p.N * 16, s, p, u, Y);
    return hipGetLastError();
}

hipError_t launch_plane(const KP& p, hipStream_t s, int mode, const double2* Y1, const double2* Y2,
                        double2* out) {
    const dim3 grid((unsigned)((p.NS * p.N + NXCD - 1) / NXCD * NXCD)), block(PLANE_THREADS);
    const size_t lds = plane_lds_bytes(p, mode);
    if (mode == PLANE_FWD)
        hipLaunchKernelGGL(k_plane<PLANE_FWD>, grid, block, lds, s, p, Y1, Y2, out);
    else if (mode == PLANE_JVP)
        hipLaunchKernelGGL(k_plane<PLANE_JVP>, grid, block, lds, s, p, Y1, Y2, out);
    else
        hipLaunchKernelGGL(k_plane<PLANE_ADJ>, grid, block, lds, s, p, Y1, Y2, out);
    return hipGetLastError();
}

hipError_t launch_mode_res(const KP& p, hipStream_t s, int flags, const double2* P3,
                           const double2* u, double2* r, double* cost_part, double2* a,
                           double2* Atil) {
    hipLaunchKernelGGL(k_mode_res, mode_grid(p), dim3(MODE_THREADS), mode_lds_bytes(p), s, p, flags,
                       P3, u, r, cost_part, a, Atil);
    return hipGetLastError();
}

hipError_t launch_mode_grad(const KP& p, hipStream_t s, int flags, const double2* P6,
                            const double2* a, double dtau, double2* u_or_out, double2* Y) {
    hipLaunchKernelGGL(k_mode_grad, mode_grid(p), dim3(MODE_THREADS), mode_lds_bytes(p), s, p, flags,
                       P6, a, dtau, u_or_out, Y);
    return hipGetLastError();
}

hipError_t launch_project(const KP& p, hipStream_t s, const double2* g, double2* out) {
    hipLaunchKernelGGL(k_project, mode_grid(p), dim3(MODE_THREADS), mode_lds_bytes(p), s, p, g, out);
    return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t s, const double* part, int n, int stride, int op,
                         double* out) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, part, n, stride, op, out);
    return hipGetLastError();
}

hipError_t launch_norms(const KP& p, hipStream_t s, const double2* u, double* part) {
    hipLaunchKernelGGL(k_norms, mode_grid(p), dim3(MODE_THREADS), 14 * p.N * 16, s, p, u, part);
    return hipGetLastError();
}

hipError_t launch_check(const KP& p, hipStream_t s, const double2* u, double* part) {
    hipLaunchKernelGGL(k_check, mode_grid(p), dim3(MODE_THREADS), 4 * p.N * 16, s, p, u, part);
    return hipGetLastError();
}

hipError_t launch_pack(const KP& p, hipStream_t s, const double2* u, double* psi) {
    hipLaunchKernelGGL(k_pack, mode_grid(p), dim3(MODE_THREADS), 0, s, p, u, psi);
    return hipGetLastError();
}

hipError_t launch_unpack(const KP& p, hipStream_t s, const double* psi, double2* u) {
    hipLaunchKernelGGL(k_unpack, mode_grid(p), dim3(MODE_THREADS), 3 * p.N * 16, s, p, psi, u);
    return hipGetLastError();
}

hipError_t launch_axpy(hipStream_t s, long long n, double a, const double* x, double* y) {
    hipLaunchKernelGGL(k_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a, x, y);
    return hipGetLastError();
}

}  // namespace pcfv
