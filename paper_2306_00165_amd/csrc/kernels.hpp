// Device-side parameters and launch wrappers of the pcfv kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "tables.hpp"

namespace pcfv {

// Everything a kernel needs about the discretisation; passed by value.
struct KP {
    int N, Nx, Nz, nkx, nkz, nm, Kx, Kz;
    int B, nmB;              // guesses per launch, B * nm
    long long nstate;        // state-vector length of one guess
    int XS, NS;              // x-slab width of the physical-space kernels, number of slabs
    int prec;                // PREC_FP64, or PREC_FP32 for the physical-space transforms and products
    int pthreads;            // threads per work group of the physical-space kernels (256, 512, 576, 768, 1024)
    int mthreads;            // threads per work group of the per-mode kernels (256 or 512)
    int np;                  // padded Ny of the per-mode kernels: stride of M and of their LDS vectors
    double lam, nu, alpha, beta;
    const double* M;         // M_COUNT fixed matrices, np x mat_ld(np) zero-padded slots, transposed
    const double* minfo;     // per-mode scalars (MI_STRIDE each)
    const double* dH;        // per-mode 1/(sigma - nu mu_k)
    const double* dP;        // per-mode 1/(kappa^2 - mu_k)
    const double* dproj;     // per-mode 1/(1 + Lambda_k / kappa^2)
    const double* Vk;        // per-mode homogeneous v responses (4 x N)
    const double* DVk;       // their derivatives
    const double* Ainv;      // per-mode inverse influence matrices (4 x 4)
    const double2* twx;      // exp(2 pi i k/Nx)
    const double2* twz;      // exp(2 pi i k/Nz)
    const double* ygl;       // Gauss-Lobatto points
    const int* indep;        // independent-mode index (state vector)
};

// Precision of the physical-space stage (transforms in x and z, products, and
// the y-value / partial arrays that carry them); per-mode work is always FP64.
enum Precision { PREC_FP64 = 0, PREC_FP32 = 1 };

// Physical-space kernel variants.
enum PlaneMode { PLANE_FWD = 0, PLANE_JVP = 1, PLANE_ADJ = 2 };

// Flags of the residual / transposed-solve mode kernel.
enum ResFlags {
    RES_INPUT_W = 1,   // skip the residual: the input field is taken as r
    RES_WRITE_R = 2,   // write r
    RES_COST = 4,      // write the per-mode cost partial
    RES_ADJ = 8,       // form a = S* r and the synthesis values of a for the adjoint products
};

// Flags of the gradient mode kernel.
enum GradFlags {
    GRAD_PROJECT = 1,  // f = -P g instead of g
    GRAD_UPDATE = 2,   // u += dtau f and synthesise the new u (descent step)
};

// One member of a grouped launch (a context: its parameters and buffers).
// item0[GPH_PLANE] / item0[GPH_MODE]: first logical work item of the member in
// the physical-space / per-mode launches; entry n of the array is a sentinel
// holding the totals.
enum GroupPhase { GPH_PLANE = 0, GPH_MODE = 1 };
struct GroupMember {
    KP kp;
    int item0[2];
    double dtau;
    double2* u;       // the member's fields (updated in place)
    void* Y;          // y-values (storage type per precision)
    void* P3;         // forward-transform partials
    void* P6;
    void* Atil;       // y-values of a = S* r
    double2* a;
    double* part;     // per-mode cost partials
};

// Everything a grouped launch needs besides the member array.
struct GroupLaunch {
    const GroupMember* gm;   // device array of n + 1 entries
    int n;
    int items[2];            // total logical items per phase
    int np;                  // padded Ny (largest over the members)
    int prec;                // common precision
    int pthreads;            // common physical-space work-group size
    int mthreads;            // common per-mode work-group size
    size_t plane_lds[3];     // largest LDS per plane mode over the members
    size_t mode_lds;
};
enum GroupKernel { GK_SYNTH = 0, GK_PLANE_FWD = 1, GK_MODE_RES = 2, GK_PLANE_ADJ = 3, GK_MODE_GRAD = 4 };
hipError_t launch_group(const GroupLaunch& g, hipStream_t s, int which);
int padded_ny(int N);
// Row stride (doubles) of the fixed-matrix slots for padded Ny np: a multiple
// of 16 so that every aligned 8-row chunk a wave loads lies in one 128-byte line.
constexpr int mat_ld(int np) { return (np + 15) / 16 * 16; }
// Row length (complex entries) of the kz rows in the physical-space kernels'
// LDS: the smallest length >= nkz that is twice an odd number, so that rows
// z and z + 1 (or x and x + 1) start 2 mod 4 complex entries apart.
constexpr int kz_row(int nkz) { return nkz + (6 - nkz % 4) % 4; }

size_t plane_lds_bytes(const KP& p, int mode);
size_t mode_lds_bytes(const KP& p);

// All launches are asynchronous on `s`; they return the launch error code.
// Y, Y1, Y2, P3, P6, Atil and out of launch_plane are y-value / partial
// arrays whose element type follows p.prec (double2 or float2).
hipError_t launch_synth(const KP& p, hipStream_t s, const double2* u, void* Y);
hipError_t launch_plane(const KP& p, hipStream_t s, int mode, const void* Y1, const void* Y2,
                        void* out);
hipError_t launch_mode_res(const KP& p, hipStream_t s, int flags, const void* P3,
                           const double2* u, double2* r, double* cost_part, double2* a,
                           void* Atil);
hipError_t launch_mode_grad(const KP& p, hipStream_t s, int flags, const void* P6,
                            const double2* a, double dtau, double2* u_or_out, void* Y);
hipError_t launch_project(const KP& p, hipStream_t s, const double2* g, double2* out);
// Per-guess reductions: out[g * stride + c] = sum (op 0) or max (op 1) over
// rows i < n of part[(g * n + i) * stride + c], for groups g < ngroups.
hipError_t launch_reduce(hipStream_t s, const double* part, int ngroups, int n, int stride, int op,
                         double* out);
hipError_t launch_norms(const KP& p, hipStream_t s, const double2* u, double* part);
hipError_t launch_check(const KP& p, hipStream_t s, const double2* u, double* part);
hipError_t launch_pack(const KP& p, hipStream_t s, const double2* u, double* psi);
hipError_t launch_unpack(const KP& p, hipStream_t s, const double* psi, double2* u);
hipError_t launch_axpy(hipStream_t s, long long n, double a, const double* x, double* y);
// DMD: Gram matrix of snapshot differences ([B][M][M]) and linear combination
// of snapshots 2..M with per-guess coefficients ([B][M-1]).  S is [M][B][n].
hipError_t launch_dmd_gram(hipStream_t s, const double* S, int M, int B, long long n, double* G);
hipError_t launch_dmd_combine(hipStream_t s, const double* S, int M, int B, long long n,
                              const double* coef, double* psi);

}  // namespace pcfv
