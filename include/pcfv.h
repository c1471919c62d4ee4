/*
 * pcfv.h -- C ABI of libpcfv: the hot path of the adjoint-based variational
 * method for equilibria of plane Couette flow (Ashtari & Schneider,
 * arXiv 2306.00165) on AMD MI355X (gfx950).
 *
 * The problem (Sec. 3.1): perturbation u about the laminar base flow
 * u_b = y e_x (Sec. 5) in the box x in [0,Lx), y in [-1,1], z in [0,Lz),
 * periodic in x and z, no-slip walls, Reynolds number Re.  The method
 * (Sec. 2-4) minimises J^2 = <r(u), r(u)> by the forward-Euler descent
 * u <- u + dtau f,  f = -P J*(u) r(u).
 *
 * Discretisation (Sec. 4, Fourier-Chebyshev-Fourier expansion):
 *   Nx, Nz  = collocation points / FFT lengths in x and z;
 *   retained |kx| <= Kx = Nx/3 - 1, 0 <= kz <= Kz = Nz/3 - 1 (2/3 rule);
 *   Ny      = number of Chebyshev coefficients = Gauss-Lobatto points.
 *
 * Spectral field layout (every u, r, v, w, g argument below):
 *   device memory, complex128 stored as interleaved (re, im) doubles,
 *   index [b][c][ikx][kz][n] with b = 0..batch-1 the guess (all guesses of a
 *   context share the discretisation and are advanced together),
 *   c = 0,1,2 the velocity component (x, y, z),
 *   ikx = 0..2Kx in FFT order (kx = 0,1,..,Kx,-Kx,..,-1), kz = 0..Kz and
 *   n = 0..Ny-1 the Chebyshev index (fastest).  Length 3*(2Kx+1)*(Kz+1)*Ny
 *   complex values per guess.  On the kz = 0 plane both signs of kx are stored and
 *   must be complex conjugates; the (0,0) mode is real.
 *
 * Operators (exact discrete definitions, all in FP64):
 *   <a,b>_W   volume-averaged L2 inner product (Sec. 3.2, inner product of
 *             the search space): sum over stored modes of w Re a^H G b, with
 *             G the Chebyshev Gram matrix, w = 1/2 on kz = 0 and 1 otherwise.
 *   r(u)      = lam S(M(u) + nu L u): one first-order IMEX step of size
 *             dt_im of the NSE minus u, divided by dt_im (Sec. 4 steps (1)-(2));
 *             lam = 1/dt_im, nu = 1/Re, L = D^2 - kappa^2, M(u) = -A[(U.grad)U]
 *             with U = u_b + u evaluated on the Nx x Ny x Nz grid and A the
 *             truncating analysis; S = Chebyshev-tau Stokes solve, done with
 *             the influence-matrix method (Sec. 4), keeping div = 0 and
 *             no-slip exact.
 *   J(u)v     directional derivative of r (Sec. 2; App. A.1).
 *   J*(u)w    its exact adjoint in <.,.>_W (Sec. 2 definition; the paper's
 *             continuous form is Sec. 3.3 / App. A.2).
 *   P         W-orthogonal projection onto divergence-free, no-slip fields
 *             (Sec. 3.4).
 *
 * Conventions:
 *   - All array arguments are caller-owned device pointers; the library never
 *     frees them.  Inputs and outputs must not alias unless stated.
 *   - Every call is enqueued on the context's HIP stream and returns without
 *     synchronising, except calls that return a host value (*_host), which
 *     synchronise the stream before returning.
 *   - Errors are reported by return code; nothing is thrown across the ABI.
 *     pcfv_last_error() gives a message for the last failure on a context.
 *   - Inputs are assumed admissible (divergence-free, no-slip, Hermitian)
 *     where stated; pcfv_check_state() measures the defects.
 *   - One context per host thread; a context is not thread-safe.
 */
#ifndef PCFV_H
#define PCFV_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pcfv_ctx pcfv_ctx;
struct pcfv_learned_model;

typedef enum {
    PCFV_OK = 0,
    PCFV_EINVAL = -1,     /* bad configuration or argument                        */
    PCFV_ENOMEM = -2,     /* workspace too small                                  */
    PCFV_EDEVICE = -3,    /* a HIP call failed                                    */
    PCFV_ENAN = -4,       /* cost became NaN or Inf during descent                */
    PCFV_EDIVERGED = -5,  /* cost grew beyond grow_tol and halvings ran out       */
    PCFV_ENOTCONV = -6    /* max_steps reached above rel_tol (a local minimum of
                             J, Sec. 2, or simply not enough steps)               */
} pcfv_status;

/* Problem definition (Sec. 3.1 and Sec. 5.1).  6 <= Nx, Nz <= 512 (any
 * integers), 9 <= Ny <= 128.  batch: number of guesses held and advanced
 * together (0 or 1: one guess; at most 4096).
 * precision: PCFV_FP64 (0), everything in FP64; or PCFV_MIXED (1), the
 * transforms in x and z and the nonlinear products in FP32 while the Stokes
 * solves, the influence matrix, projection, cost and update stay FP64.  The
 * state u and every argument stay FP64 in both. */
enum { PCFV_FP64 = 0, PCFV_MIXED = 1 };
typedef struct {
    double Lx, Lz, Re;
    int Nx, Ny, Nz;
    double dt_im;        /* Delta t of the Stokes step inside r(u); the paper uses 0.25 */
    int precision;       /* PCFV_FP64 or PCFV_MIXED */
    int batch;
} pcfv_config;

/* Layout of the spectral fields of a context: complex value (b, c, ikx, kz, n)
 * at offset b stride_b + c stride_c + ikx stride_kx + kz stride_kz + n
 * (in complex values; n is contiguous). */
typedef struct {
    int Kx, Kz, Ny, nkx, nkz;
    long long n_modes;   /* nkx * nkz                                   */
    long long n_complex; /* 3 * n_modes * Ny: complex values per guess  */
    long long n_state;   /* length of the minimal real state vector of one guess */
    int batch;
    long long stride_b, stride_c, stride_kx, stride_kz;
} pcfv_layout;

/* Bytes of device workspace pcfv_create needs for this configuration;
 * 0 if the configuration is invalid. */
size_t pcfv_workspace_bytes(const pcfv_config* cfg);

/* Build a context.  hip_stream: a hipStream_t (NULL = the default stream).
 * workspace: caller-owned device memory of at least pcfv_workspace_bytes(cfg)
 * bytes, 256-byte aligned; it holds every table and scratch buffer the
 * context uses and must outlive the context.  The context's tables are
 * computed on the host in extended precision and copied in (synchronously).
 * Errors: PCFV_EINVAL (bad cfg or NULL out), PCFV_ENOMEM (NULL workspace),
 * PCFV_EDEVICE. */
pcfv_status pcfv_create(const pcfv_config* cfg, void* hip_stream, void* workspace,
                        pcfv_ctx** out);

/* Release host-side state; never touches caller memory.  Safe on NULL. */
void pcfv_destroy(pcfv_ctx* ctx);

pcfv_status pcfv_get_layout(const pcfv_ctx* ctx, pcfv_layout* out);
pcfv_status pcfv_set_stream(pcfv_ctx* ctx, void* hip_stream);

/* Switch the context between PCFV_FP64 and PCFV_MIXED for later calls (the
 * workspace of either precision serves both).  PCFV_EINVAL otherwise. */
pcfv_status pcfv_set_precision(pcfv_ctx* ctx, int precision);

/* Residual r(u) (Sec. 4 steps (1)-(2), Sec. 3.2 residual).  u admissible.
 * r may be NULL (then only the cost is formed).  cost_host, if non-NULL,
 * receives J^2 = <r,r>_W of each guess (batch values) and the call
 * synchronises. */
pcfv_status pcfv_residual(pcfv_ctx* ctx, const double* u, double* r, double* cost_host);

/* J^2 = <r(u), r(u)>_W (Sec. 2 cost function) per guess; synchronises. */
pcfv_status pcfv_cost(pcfv_ctx* ctx, const double* u, double* cost_host);

/* Jv = J(u) v, the directional derivative of r at u along v (Sec. 2). */
pcfv_status pcfv_jvp(pcfv_ctx* ctx, const double* u, const double* v, double* Jv);

/* out = J*(u) w, the exact W-adjoint of J(u) (not projected).  w may be any
 * Hermitian-consistent field. */
pcfv_status pcfv_adjoint(pcfv_ctx* ctx, const double* u, const double* w, double* out);

/* Pg = P g, the W-orthogonal projection onto divergence-free no-slip fields
 * (Sec. 3.4). g any Hermitian-consistent field.  Pg may equal g (in place). */
pcfv_status pcfv_project(pcfv_ctx* ctx, const double* g, double* Pg);

/* One or more descent steps (Sec. 4 step (5)), optionally accelerated by DMD
 * extrapolation (Sec. 6.2). */
typedef struct {
    long long max_steps;  /* steps to take at most                                  */
    double dtau;          /* forward-Euler step (the paper: 0.03 at 32x31x32)         */
    double rel_tol;       /* stop when ||r||_W / ||u_b + u||_W < rel_tol (0 = never)  */
    int check_every;      /* cost read-back period in steps (>= 1)                    */
    double grow_tol;      /* cost growth factor between checks that counts as
                             divergence (<= 0: disabled)                             */
    int max_halvings;     /* dtau halvings allowed on divergence                      */
    /* DMD (Sec. 6.2): snapshots every dmd_stride steps; after dmd_window of them
     * the window is extrapolated (pcfv_dmd_extrapolate) and each guess whose
     * extrapolated cost is below dmd_accept times its current cost restarts
     * from it; the next window starts dmd_gap steps later.  Windows start only
     * once every guess has J = sqrt(J^2) < dmd_start (<= 0: at once).
     * dmd_window = 0 disables DMD.  dmd_buffer: device memory for
     * dmd_window * batch * n_state doubles, caller-owned. */
    int dmd_window;
    int dmd_stride;
    int dmd_gap;
    double dmd_start;
    double dmd_accept;
    double* dmd_buffer;
    /* Mixed precision: on a PCFV_MIXED context, once every guess has
     * ||r||/||u_b+u|| < fp64_below at a check, the rest of the call runs in
     * FP64 (the refinement phase); <= 0 keeps the context's precision.  The
     * refinement steps equal those of a PCFV_FP64 context with the same launch
     * shape (pcfv_get_tuning) bit for bit. */
    double fp64_below;
    /* Learned extrapolator (may be NULL): at the end of every DMD window its
     * proposal from the window's last model->window snapshots competes with
     * the DMD candidate; each guess takes the cheaper of the two by true
     * cost, under the same dmd_accept rule. */
    const struct pcfv_learned_model* learned;
    /* With no_cost_checks != 0 and nothing above that reads the cost (rel_tol
     * = 0, grow_tol <= 0, no DMD, fp64_below <= 0), the call enqueues
     * max_steps steps and returns without evaluating the cost or
     * synchronising; the report's cost and rel_res are then NaN.  (Every step
     * still forms its per-mode cost partials on the device.) */
    int no_cost_checks;
    /* Adaptive DMD window (Sec. 6.2 leaves the snapshot spacing open): with
     * dmd_stride_max > dmd_stride, a window after which some guess's best
     * candidate costs at least dmd_grow_ratio times its current cost (or has
     * no candidate) makes the next windows' stride four times longer, up to
     * dmd_stride_max steps.  Near a fixed point the slowest directions must
     * move the snapshots enough to be resolved; a longer window does that.
     * dmd_grow_ratio <= 0 means 0.5.  dmd_stride_max <= dmd_stride: fixed
     * stride. */
    int dmd_stride_max;
    double dmd_grow_ratio;
} pcfv_descent_opts;

typedef struct {
    long long steps;      /* steps taken                                             */
    double tau;           /* fictitious time advanced                                */
    double cost;          /* J^2 at the last check (of the final state if converged)  */
    double rel_res;       /* ||r||_W / ||u_b + u||_W at the last check               */
    double dtau_final;
    int n_halvings;
    int n_dmd;            /* DMD extrapolations performed                            */
    int n_dmd_accepted;   /* guesses restarted from an extrapolated state             */
    long long steps_fp32; /* steps taken with the FP32 physical-space stage           */
    int n_learned_accepted; /* restarts from a learned proposal (counted in n_dmd_accepted) */
    int dmd_stride_final; /* snapshot stride of the last DMD window (pcfv_descend)     */
} pcfv_descent_report;

/* Advance every guess of u in place with the same dtau.  Returns PCFV_OK when
 * every guess reached rel_tol (or, with rel_tol = 0, after max_steps),
 * PCFV_ENOTCONV when max_steps ran out above rel_tol, PCFV_ENAN on a
 * non-finite cost, PCFV_EDIVERGED when some guess's cost kept growing after
 * max_halvings halvings.  With grow_tol > 0 the state is checkpointed at every
 * check; when a guess's cost has grown by more than grow_tol since the last
 * check, u, the step count and tau go back to that checkpoint and dtau is
 * halved (u is the checkpointed state on PCFV_EDIVERGED).  The report gives
 * the largest cost and relative residual over the guesses. */
pcfv_status pcfv_descend(pcfv_ctx* ctx, double* u, const pcfv_descent_opts* opts,
                         pcfv_descent_report* report);

/* DMD extrapolation (Sec. 6) of each guess.  snaps: device, [M][batch][n_state]
 * minimal state vectors (pcfv_pack_state), oldest first, consecutive ones
 * dtau_snap apart, 3 <= M <= 256.  Candidates (Sec. 6.1-6.2, and a reading for
 * targets without an omega = 0 mode), for r = 1, 2, ..:
 *   kind 0 (r <= r*, the numerical rank of [psi_1 .. psi_{M-1}], singular
 *     values above 1e-7 of the largest): Re(b_1 phi_1) of the rank-r exact
 *     DMD of the snapshots, the mode with the smallest |omega|, amplitudes
 *     fitted at the last snapshot;
 *   kind 1 (r <= r*_d, the numerical rank of the differences
 *     [d_1 .. d_{M-2}], d_k = psi_{k+1} - psi_k): the fixed point of the
 *     affine model fitted by the rank-r exact DMD of the differences,
 *     psi_M + Re sum_{|lambda_q| < 1} b_q phi_q lambda_q / (1 - lambda_q)
 *     (exact for affine dynamics around any fixed point, the laminar state
 *     included).
 * Each candidate's true cost J^2 is evaluated; the cheapest (earliest in the
 * order rank, kind on ties) is written to u_out (batch fields), its cost to
 * cost_host[b], its rank and kind to rank_host[b] and kind_host[b] (any of the
 * three may be NULL).  A guess whose window has rank 0 gets its last snapshot,
 * rank 0 and kind -1.  Synchronises. */
pcfv_status pcfv_dmd_extrapolate(pcfv_ctx* ctx, const double* snaps, int M, double dtau_snap,
                                 double* u_out, double* cost_host, int* rank_host, int* kind_host);

/* Norms per guess b: out_host[3b] = ||u||_W, out_host[3b+1] = ||u_b + u||_W,
 * out_host[3b+2] = D = <curl U, curl U>_W (so that laminar flow has D = 1,
 * Table 2); out_host holds 3 * batch doubles.  Synchronises. */
pcfv_status pcfv_norms(pcfv_ctx* ctx, const double* u, double* out_host);

/* Minimal real state vector psi (Sec. 6.2), n_state doubles per guess:
 * (0,0) mode: u_x and u_z coefficients n = 0..Ny-3; then for each independent
 * mode (kz > 0, or kz = 0 with kx > 0) in storage order: Re v, Im v for
 * n = 0..Ny-5, Re eta, Im eta for n = 0..Ny-3, with v the wall-normal velocity
 * and eta = i b u_x - i a u_z.  pack needs admissible u; unpack returns an
 * admissible, Hermitian-consistent field. */
pcfv_status pcfv_pack_state(pcfv_ctx* ctx, const double* u, double* psi);
pcfv_status pcfv_unpack_state(pcfv_ctx* ctx, const double* psi, double* u);

/* Admissibility defects of each guess b: defects_host[3b] = max |divergence
 * coefficient|, [3b+1] = max |wall value|, [3b+2] = max Hermitian defect on
 * kz = 0 (3 * batch doubles); synchronises. */
pcfv_status pcfv_check_state(pcfv_ctx* ctx, const double* u, double* defects_host);

/* Measurement hook (used by the benchmark, not part of the method): nsteps
 * plain descent steps of u (in place, step dtau) with HIP events on the
 * context stream around each kernel: ms_out[0..3] = average device time per
 * launch, in milliseconds, of the forward products, the residual/adjoint-solve
 * per mode, the adjoint products and the gradient/projection/update per mode,
 * as they run inside consecutive steps.  1 <= nsteps <= 4096.  Synchronises. */
pcfv_status pcfv_time_descent_kernels(pcfv_ctx* ctx, double* u, double dtau, int nsteps, double* ms_out);

/* Measurement hook (used by the benchmark, not part of the method): average
 * device time per launch, in milliseconds, of each kernel of one descent
 * step, measured with HIP events on the context stream over nrep launches
 * each (u is left unchanged).  ms_out[0..4] = synthesis, forward products,
 * residual/adjoint-solve per mode, adjoint products, gradient/projection/
 * update per mode; *n_out receives the number of entries.  Synchronises. */
pcfv_status pcfv_time_kernels(pcfv_ctx* ctx, const double* u, int nrep, double* ms_out,
                              int* n_out);

/* Message of the last failure on ctx; with ctx = NULL, the reason of the last
 * failed pcfv_create on the calling thread.  Valid until the next call. */
const char* pcfv_last_error(const pcfv_ctx* ctx);

/* Autotuner over the launch shapes: for every candidate x-slab width of the
 * physical-space kernels (divisors of Nx up to 16 whose staging fits the
 * 160 KiB of LDS a work group may use, at least half the default), their work-group size (256, 512, 576, 768,
 * 1024 threads) and the
 * per-mode kernels' work-group size (256 threads with 4 lanes per contraction
 * row, 512 with 8) it times
 * `steps` descent steps (after one untimed step) on a scratch copy of u with
 * dtau = 0, keeps the fastest for every later call, and reports each
 * candidate in entries[0..cap) (n_entries gets the count).  u is not
 * modified.  Synchronises. */
typedef struct {
    int xs;               /* x-slab width */
    int plane_threads;    /* work-group size of the physical-space kernels */
    int mode_threads;     /* work-group size of the per-mode kernels */
    double ms_per_step;   /* measured descent-step time */
} pcfv_tune_entry;
pcfv_status pcfv_autotune(pcfv_ctx* ctx, const double* u, int steps, pcfv_tune_entry* entries, int cap,
                          int* n_entries);
/* The launch shape in use (x-slab width, physical-space and per-mode work-group
 * sizes; any pointer may be NULL).  Without pcfv_autotune: the widest slab
 * that fits, up to 12 (16 when the context holds more than 1024 modes over all
 * guesses), physical-space groups of 768 threads in FP64 and of 1024 in
 * mixed precision (512 for more than 1024 modes), and 256-thread per-mode
 * groups. */
pcfv_status pcfv_get_tuning(const pcfv_ctx* ctx, int* xs, int* plane_threads, int* mode_threads);
/* Sets the launch shape explicitly: xs must be one of the slab widths the
 * autotuner considers, plane_threads one of 256, 512, 576, 768, 1024 and
 * mode_threads 256 or 512; anything else returns PCFV_EINVAL and leaves the
 * shape unchanged.  Results do not depend on the shape beyond rounding. */
pcfv_status pcfv_set_tuning(pcfv_ctx* ctx, int xs, int plane_threads, int mode_threads);

/* Groups (batching over uneven grids): n contexts, each with its own grid,
 * Re, batch and tables but one precision at creation, are advanced together;
 * every descent step is one launch per stage (physical-space forward,
 * residual and transposed solve, physical-space adjoint, gradient/projection/
 * update) over all members (two per stage while some members have switched
 * from FP32 to FP64), so small members share the chip instead of running one
 * after another.  The physical-space work-group size is members[0]'s; the
 * per-mode one, the slab width and the LDS staging follow the single-context
 * default rules applied to the modes of all members together.
 *
 * Memory and streams: the group allocates nothing on the device.  workspace:
 * caller-owned device memory of pcfv_group_workspace_bytes(members, n) bytes,
 * 256-byte aligned, holding the members' device records and, for members
 * whose padded Ny differs from the group's, their tables at the group's
 * stride (copied in synchronously by pcfv_group_create).  hip_stream: the
 * caller's stream (NULL = the default stream) on which every group launch is
 * enqueued; a HIP graph (graph_steps > 0) needs a non-NULL stream.  Members,
 * their workspaces and the group workspace must outlive the group.
 * pcfv_group_workspace_bytes returns 0 for invalid members (NULL, or mixed
 * precisions). */
typedef struct pcfv_group pcfv_group;
size_t pcfv_group_workspace_bytes(pcfv_ctx* const* members, int n);
pcfv_status pcfv_group_create(pcfv_ctx* const* members, int n, void* hip_stream, void* workspace,
                              pcfv_group** out);
void pcfv_group_destroy(pcfv_group* group);   /* never touches caller memory */
pcfv_status pcfv_group_set_stream(pcfv_group* group, void* hip_stream);
/* steps plain descent steps (Sec. 4 step (5)) of every member: u[k] is member
 * k's field array (device, in place), dtau[k] its step.  graph_steps > 0
 * captures that many steps in a HIP graph once (reused across calls, since
 * fields and steps are read from the device records) and replays it; the
 * remainder runs as plain launches.  Waits for the members' streams first
 * and synchronises before returning.  Costs are read with pcfv_cost on each
 * member afterwards. */
pcfv_status pcfv_group_descend(pcfv_group* group, double* const* u, const double* dtau, long long steps,
                               int graph_steps);
/* Descent of every member to a tolerance (Sec. 4 step (5), Sec. 6.2 for the
 * DMD windows).  Every check_every steps each active member's cost and
 * relative residual ||r||_W / ||u_b + u||_W (largest over its guesses) are
 * read back; a member stops once it is below rel_tol (and, on a PCFV_MIXED
 * group with fp64_below > 0, past its FP64 switch), or with PCFV_ENAN on a
 * non-finite cost; the others go on.  With fp64_below > 0 a PCFV_MIXED
 * member switches to FP64 once below fp64_below (its y-values are rebuilt in
 * FP64; from then on its stages run in the FP64 launches).  dmd_window > 0:
 * every dmd_stride steps (fixed: the adaptive stride of pcfv_descend is not
 * used here) each active member's state vector goes into its
 * window (dmd_buffers[k]: device, dmd_window * batch_k * n_state_k doubles,
 * caller-owned); a full window is extrapolated as pcfv_dmd_extrapolate does
 * and each guess whose best candidate costs less than dmd_accept times its
 * current cost restarts from it.  reports[k] and status[k] (n each) give
 * member k's steps, fp32 steps, cost, relative residual, DMD counts and
 * PCFV_OK / PCFV_ENOTCONV (max_steps reached) / PCFV_ENAN.  Returns PCFV_OK
 * if every member converged, else the first failing status (PCFV_ENAN
 * first).  Synchronises. */
typedef struct {
    long long max_steps;   /* group steps at most                                */
    double rel_tol;        /* > 0                                               */
    int check_every;       /* cost read-back period in steps (>= 1)              */
    double fp64_below;     /* FP32 -> FP64 switch (PCFV_MIXED groups; <= 0: none) */
    int dmd_window;        /* snapshots per DMD window (0: no DMD; 3..256)        */
    int dmd_stride;        /* steps between snapshots                            */
    double dmd_accept;     /* accept a candidate below dmd_accept x current cost  */
    double* const* dmd_buffers;   /* n device buffers (see above)                */
} pcfv_group_opts;
pcfv_status pcfv_group_descend_tol(pcfv_group* group, double* const* u, const double* dtau,
                                   const pcfv_group_opts* opts, pcfv_descent_report* reports, int* status);
const char* pcfv_group_last_error(const pcfv_group* group);

/* ---------------------------------------------------------------------------
 * Learned extrapolator (alongside the DMD extrapolation of Sec. 6): a
 * multilayer perceptron maps a window of W snapshots, projected on r POD
 * modes of the state vector, to the POD coefficients of the descent limit.
 * Matrix products run on the matrix cores in BF16 with FP32 accumulation;
 * FP32 master weights are trained with Adam.  Every proposal is judged by
 * the true residual of the method, and DMD stays the fallback.
 * ------------------------------------------------------------------------- */
#define PCFV_MLP_MAX_LAYERS 8
#define PCFV_LEARNED_MAX_SCALES 8

/* dims[0] inputs, dims[n_layers] outputs; ReLU after every layer but the
 * last.  Parameters (FP32, host order): for each layer l, W_l (dims[l] x
 * dims[l+1], row-major: input index major) then b_l (dims[l+1]). */
typedef struct {
    int n_layers;
    int dims[PCFV_MLP_MAX_LAYERS + 1];
    int max_batch;        /* rows per call, at most */
} pcfv_mlp_config;
typedef struct pcfv_mlp pcfv_mlp;

long long pcfv_mlp_param_count(const pcfv_mlp_config* cfg);           /* 0 if cfg is invalid */
size_t pcfv_mlp_workspace_bytes(const pcfv_mlp_config* cfg);           /* 0 if cfg is invalid */
/* workspace: caller-owned device memory, 256-byte aligned, outliving the MLP. */
pcfv_status pcfv_mlp_create(const pcfv_mlp_config* cfg, void* hip_stream, void* workspace, pcfv_mlp** out);
void pcfv_mlp_destroy(pcfv_mlp* mlp);
const char* pcfv_mlp_last_error(const pcfv_mlp* mlp);   /* NULL: the last create error */
/* Load FP32 parameters from the host (and their BF16 copies); resets Adam.  Synchronises. */
pcfv_status pcfv_mlp_set_params(pcfv_mlp* mlp, const float* params_host);
pcfv_status pcfv_mlp_get_params(pcfv_mlp* mlp, float* params_host);    /* synchronises */
/* Y (device FP32, B x dims[L]) from X (device FP32, B x dims[0]), 1 <= B <= max_batch. */
pcfv_status pcfv_mlp_forward(pcfv_mlp* mlp, const float* X, float* Y, int B);
/* Forward pass, loss = mean over all B x dims[L] outputs of (Y - T)^2 and its
 * gradient with respect to every parameter (kept in the MLP); loss_host, if
 * non-NULL, receives the loss and the call synchronises. */
pcfv_status pcfv_mlp_grad(pcfv_mlp* mlp, const float* X, const float* T, int B, float* loss_host);
/* One Adam step (Kingma & Ba, bias-corrected) with the kept gradient. */
pcfv_status pcfv_mlp_adam_step(pcfv_mlp* mlp, float lr, float beta1, float beta2, float eps);
/* Test hook: copy an internal buffer of the last forward / gradient call to
 * the host: PCFV_MLP_ACT the BF16 input of `layer` (B x dims[layer]),
 * PCFV_MLP_OUT the FP32 output of the last gradient call, PCFV_MLP_DZ the BF16
 * gradient with respect to the pre-activation of `layer` (B x dims[layer+1]),
 * PCFV_MLP_GRAD every parameter gradient (FP32).  Synchronises. */
enum { PCFV_MLP_ACT = 0, PCFV_MLP_OUT = 1, PCFV_MLP_DZ = 2, PCFV_MLP_GRAD = 3 };
pcfv_status pcfv_mlp_read(pcfv_mlp* mlp, int what, int layer, void* host, size_t cap_bytes);

/* POD of S snapshots X (device, S x n, row-major) by the method of
 * snapshots: mean (n), the r leading orthonormal modes basis (r x n,
 * row-major) of the centred snapshots and, if non-NULL, their singular values
 * sigma_host (r).  scratch: device, pcfv_pod_scratch_bytes(S, n, r) bytes.
 * 2 <= S, r <= S.  PCFV_EINVAL if fewer than r modes have positive energy,
 * PCFV_ENOTCONV if the eigen-iteration fails.  Synchronises. */
size_t pcfv_pod_scratch_bytes(int S, long long n, int r);
pcfv_status pcfv_pod_build(void* hip_stream, const double* X, int S, long long n, int r, double* mean, double* basis,
                           double* sigma_host, void* scratch);
/* coef (m x r) = (X - mean) basis^T for X (m x n); scratch: device,
 * pcfv_pod_project_scratch_bytes(m, n, r) bytes.  Asynchronous. */
size_t pcfv_pod_project_scratch_bytes(int m, long long n, int r);
pcfv_status pcfv_pod_project(void* hip_stream, const double* X, int m, long long n, int r, const double* mean,
                             const double* basis, double* coef, void* scratch);
/* Allocation-free variant of pcfv_pod_project, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and the same split of the
 * sum over n, so coef equals pcfv_pod_project's bit for bit, but the split-K
 * partials live in a device-resident array of PCFV_NOALLOC_SCRATCH_BYTES
 * (8 MiB) that the library holds on every GPU it runs on until the process
 * ends.  The call allocates nothing and calls no allocating routine; its
 * first call on a device looks up that device's copy of the array (with the
 * device current: hip_stream must belong to the current device).  Every call
 * on one GPU shares that array and leaves its contents behind, so calls that
 * overlap on one GPU (different streams, threads) race; the partials are
 * written in full before they are read, so nothing needs clearing between
 * calls.  Errors: PCFV_EINVAL (bad arguments), PCFV_ENOMEM when the partials
 * (pcfv_pod_project_scratch_bytes(m, n, r) bytes) exceed the array (message
 * from pcfv_last_error(NULL)), PCFV_EDEVICE.  Asynchronous on hip_stream. */
#define PCFV_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
pcfv_status pcfv_pod_project_noalloc(void* hip_stream, const double* X, int m, long long n, int r,
                                     const double* mean, const double* basis, double* coef);
/* X (m x n) = mean + coef basis.  Asynchronous. */
pcfv_status pcfv_pod_reconstruct(void* hip_stream, const double* coef, int m, long long n, int r, const double* mean,
                                 const double* basis, double* X);

/* A trained extrapolator.  Input features of guess b: for w < W-1 the
 * differences c_w - c_{W-1} of the POD coefficients of the window's snapshots,
 * c_{W-1} itself and, if use_base, c_base - c_{W-1} for the POD coefficients
 * of a base candidate ((W + use_base) r values, window position major),
 * normalised as (x - in_mu) * in_isd.  The MLP output y gives a step in POD
 * coefficients, dc = y / out_isd + out_mu, and the proposal is the base plus
 * that step: psi_{W-1} + dc basis, or psi_base + dc basis with use_base (what
 * the r modes do not resolve is kept from the base).  With use_base the
 * descent passes the DMD candidate as the base, so the network learns a
 * correction to DMD.  All pointers are device memory owned by the caller. */
typedef struct pcfv_learned_model {
    int window;               /* W */
    int use_base;             /* 0: step from the last snapshot; 1: from a base candidate */
    int r;                    /* POD modes */
    const double* pod_mean;   /* n_state */
    const double* pod_basis;  /* r x n_state */
    const float* in_mu;       /* (W + use_base) r */
    const float* in_isd;      /* (W + use_base) r */
    const float* out_mu;      /* r */
    const float* out_isd;     /* r */
    pcfv_mlp* mlp;            /* dims[0] = (W + use_base) r, dims[last] = r, max_batch >= the context batch */
    /* Step lengths tried along the predicted step (psi = base + s dc basis);
     * each guess gets the one of least true cost.  n_scales = 0: s = 1 only. */
    int n_scales;
    double scales[PCFV_LEARNED_MAX_SCALES];
    void* scratch;            /* pcfv_learned_scratch_bytes(ctx, window, r) bytes */
} pcfv_learned_model;
size_t pcfv_learned_scratch_bytes(const pcfv_ctx* ctx, int window, int r);

/* Training set of the extrapolator from POD coefficients: c (device, [W][B][r]
 * doubles: W window snapshots of B training windows), cb (device, B x r: the
 * base candidates' coefficients, or NULL for a model without base) and ct
 * (device, B x r: the coefficients of each window's descent limit, or NULL).
 * Writes the features X (device FP32, B x (W + [cb]) r) and, if ct, the
 * targets T (B x r: ct - cb, or ct - c_{W-1}) of the model's definition.  fit != 0 first computes the normalisation from this
 * set (per-column mean and 1/max(std, 1e-12)) into in_mu, in_isd and, if ct,
 * out_mu, out_isd; fit = 0 uses the given ones.  Asynchronous on hip_stream. */
pcfv_status pcfv_learned_prepare(void* hip_stream, int W, int B, int r, const double* c, const double* cb,
                                 const double* ct, int fit, float* in_mu, float* in_isd, float* out_mu, float* out_isd,
                                 float* X, float* T);

/* Minibatch training: `epochs` passes over the N rows of (X, T) (device FP32,
 * N x dims[0] and N x dims[L]) in batches of `batch` rows (a permutation per
 * epoch drawn from `seed` by SplitMix64; a short last batch is dropped), one
 * Adam step (lr, 0.9, 0.999, 1e-8) per batch.  idx: device scratch of N ints;
 * Xb, Tb: device scratch of batch x dims[0] and batch x dims[L] floats.
 * loss_host (if non-NULL) receives the mean loss of every epoch.  Synchronises. */
pcfv_status pcfv_mlp_fit(pcfv_mlp* mlp, const float* X, const float* T, int N, int batch, int epochs, float lr,
                         unsigned long long seed, int* idx, float* Xb, float* Tb, float* loss_host);
/* Proposal for every guess from the window snaps (device, [W][batch][n_state],
 * oldest first, spaced as in training) and, if model->use_base, the base
 * candidates base (device, [batch][n_state]; ignored otherwise): u_out (batch
 * fields) and its cost J^2 per guess in cost_host (may be NULL).  Synchronises. */
pcfv_status pcfv_learned_propose(pcfv_ctx* ctx, const pcfv_learned_model* model, const double* snaps,
                                 const double* base, double* u_out, double* cost_host);

/* Test hook (no device): host-side copy of a constant table for cfg, computed
 * without a device (for tests of the setup arithmetic).  which: 0 fixed matrices (27 slots of
 * Ny x Ny, each matrix stored transposed), 1 per-mode scalars, 2 Helmholtz diagonals,
 * 3 Poisson diagonals, 4 projection diagonals, 5 homogeneous v responses,
 * 6 their derivatives, 7 inverse influence matrices, 8 eigenvalues of the tau
 * second derivative.  Copies min(cap, size) doubles to out (if non-NULL) and
 * returns the table size in doubles, or 0 if cfg or which is invalid. */
size_t pcfv_host_table(const pcfv_config* cfg, int which, double* out, size_t cap);

/* Test hook (no device): the host-side DMD algebra of Sec. 6.1-6.2.  Given
 * the M x M Gram matrix Ge = Ge_hi + Ge_lo (row-major, an unevaluated sum of
 * two doubles per entry; Ge_lo may be NULL) of E = [psi_1, psi_2 - psi_1, ..,
 * psi_M - psi_{M-1}], writes the candidates of pcfv_dmd_extrapolate in their
 * evaluation order: candidate i's M-1 coefficients c (steady state
 * psi_s = sum_k c_k psi_{k+2}) to coef[i (M-1) + k] and its (rank, kind) to
 * labels[2i], labels[2i+1], for i < cap (either array may be NULL).  Returns
 * the number of candidates, or -1 on invalid input.  3 <= M <= 256. */
int pcfv_host_dmd(const double* Ge_hi, const double* Ge_lo, int M, double dtau, double* coef, int* labels,
                  int cap);

#ifdef __cplusplus
}
#endif
#endif /* PCFV_H */
