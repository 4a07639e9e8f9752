/*
 * mpfc.h -- C ABI of libmpfc.so: the implicit time step of the two
 * energy-stable convex-splitting schemes for the modified phase field crystal
 * (MPFC) equation, solved by nonlinear FAS multigrid on one AMD Instinct
 * MI355X (gfx950) GPU.
 *
 * Paper: Baskaran, Zhou, Hu, Wang, Wise, Lowengrub, "Energy stable and
 * efficient finite-difference nonlinear multigrid schemes for the modified
 * phase field crystal equation".
 *
 * The problem (Sec. 3.1, Sec. 3.2, App. B): given phi^k, psi^k (and phi^{k-1}
 * for the second-order scheme) on an m x n cell-centred grid with spacing h
 * (each axis periodic or homogeneous Neumann, App. A), find phi^{k+1}, mu,
 * kappa solving N(u) = S (App. B.1, B.2) and then psi^{k+1} (eq. discrete_1_b
 * or discrete_2_b).
 *
 * Conventions for every entry point:
 *  - Grid functions are contiguous arrays of m*n values, row-major with x
 *    fastest: cell (i, j) at index j*m + i.  m and n are powers of two, or
 *    (mpfc_create, FP64 only) multiples of 4 such as Sec. 4.6's 512 x 400.
 *  - Pointers named d_* are device pointers (hipMalloc'd or from a PyTorch
 *    tensor), owned by the caller, and must stay valid until the call
 *    returns.  Pointers named h_* are host pointers owned by the caller.
 *  - `stream` is a hipStream_t (NULL = default stream) passed as void*;
 *    all device work of a call is ordered on it.
 *  - Return value: 0 (MPFC_OK) or a negative MPFC_E* code; no exception
 *    crosses the ABI.  Argument errors are detected on the host before any
 *    HIP call.  mpfc_strerror() names a code; mpfc_last_error() gives the
 *    detail of the last failure on the calling thread.
 */
#ifndef MPFC_H
#define MPFC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPFC_VERSION 1

enum {
    MPFC_OK = 0,
    MPFC_EINVAL = -1,        /* invalid argument (checked on the host) */
    MPFC_ENOTCONVERGED = -2, /* cycle limit reached; outputs hold the last iterate */
    MPFC_ENONFINITE = -3,    /* NaN/Inf residual; outputs hold the last iterate */
    MPFC_EDIVERGED = -4,     /* residual grew by the divergence factor */
    MPFC_ENOMEM = -5,        /* device allocation failed */
    MPFC_EHIP = -6           /* a HIP runtime call failed */
};

enum { MPFC_FP64 = 0, MPFC_MIXED = 1 };                           /* precision */
enum { MPFC_GUESS_PREV = 0, MPFC_GUESS_EXTRAP = 1,                 /* initial guess */
       MPFC_GUESS_CNN = 2 /* learned, with the extrapolated guess as fallback (mpfc_cnn_load) */ };
enum { MPFC_NEWTON = 0, MPFC_PICARD = 1 };                        /* linearisation */
/* Boundary conditions (App. A): every axis is periodic (eqs. per-bcs) unless
 * its bit is set, then homogeneous Neumann (eqs. h-n-bcs: the ghost cell
 * repeats the boundary cell).  Sec. 4.5 runs periodic in x, Neumann in y. */
enum { MPFC_BC_PERIODIC = 0, MPFC_BC_NEUMANN_X = 1, MPFC_BC_NEUMANN_Y = 2 };

/* Model and discretisation (Sec. 2, Sec. 3): alpha = 1 - eps; dt is the time
 * step s.  scheme 1: first-order convex splitting (Sec. 3.1); scheme 2:
 * second-order scheme (Sec. 3.2).  bc: MPFC_BC_* bits (0 = periodic).
 * Requires h > 0, dt > 0, M > 0, beta >= 0, eps <= 1.  The learned guess
 * (MPFC_GUESS_CNN) needs periodic boundaries. */
typedef struct {
    double eps, beta, M, h, dt;
    int scheme;
    int bc;
} mpfc_params;

/* Solver options.  nu1/nu2: pre/post red-black smoothing passes per level
 * (App. B "l_max"), each in [0, 4]; tol: stop when the finest residual norm
 * sqrt(h^2 sum_c sum_ij r_c^2) <= tol; max_cycles: V-cycle limit;
 * coarsest: smaller side of the coarsest grid, must be 2.  Levels are
 * coarsened while the smaller side exceeds it and both sides of the next
 * level stay even.  Power-of-two grids end at 2x2 or 2x4 cells (so m/n or n/m
 * is at most 2), solved directly by Newton's method.  Other grids (sides
 * multiples of 4; FP64, nu1, nu2 <= 2, no learned guess) end at a larger
 * level (512 x 400: 64 x 50, at most 4096 cells), relaxed by coarse_sweeps
 * red-black sweeps per V-cycle (in [1, 64], default 2); its Poisson problem
 * is solved exactly in the separable eigenbasis.  energy: 1 to compute the energies of Sec. 3 after each
 * step; diverge: factor of residual growth over the initial residual
 * reported as MPFC_EDIVERGED.
 * precision = MPFC_MIXED: FP64 outer defect correction (FP64 finest residual,
 * norm and stopping test; u updated in FP64) around inner_cycles FP32 FAS
 * V-cycles per outer iteration on the correction equation N(u+e) - N(u) = r,
 * whose nonlinear difference is evaluated in factored form; max_cycles then
 * limits the outer iterations.  inner_cycles_next: FP32 V-cycles in each
 * outer iteration after the step's first, in [0, 16] (0: inner_cycles).  The
 * first outer iteration takes the defect of the initial guess down to FP32's
 * floor; the later ones start from that floor and need fewer cycles.
 * inner_nu_coarse: smoothing passes before and after the coarse-grid
 * correction on the levels below the finest in those FP32 cycles, in
 * [0, min(nu1, nu2)]; 0 keeps nu1 and nu2.  Each FP32 cycle only has to
 * reduce the correction equation's residual, which the next FP64 defect
 * measures, so it need not be the finest level's V(nu1, nu2): the levels
 * below the finest are latency bound, and V(1, 1) there costs less per cycle
 * for the same contraction.  Grids with tiled levels only (larger than
 * 32 x 32 cells); others ignore it.
 * omega: relaxation factor of the smoother, in (0, 2): each cell moves by
 * omega times the solution of its local 3x3 system.  1 (the default) is the
 * collective Gauss-Seidel update of App. B.  App. B's update amplifies a band
 * of error modes when s M h^-4 / (beta + q/s) is in an intermediate range
 * (q = 1 or 2 by scheme), where V-cycles can diverge (first-order scheme at
 * h = 0.5: s from about 0.15 to 0.3); under-relaxation near 0.8 converges
 * there.  The solution of the step does not depend on omega.  The 3-D
 * contexts take omega = 1 only.
 * coarse_threshold: cells of the largest level the persistent coarse kernel
 * takes (every smaller level runs there too, in one workgroup; larger ones
 * run as fused tile launches): 0 for the default 1024 (32 x 32), else a power
 * of two in [256, 1024].  Power-of-two grids only (others: 0); a batch takes
 * 0 only.  The iterates do not depend on it. */
typedef struct {
    int nu1, nu2, max_cycles;
    double tol;
    int precision, guess, linearization;
    int coarsest;
    int energy;
    double diverge;
    int inner_cycles;
    int coarse_sweeps;
    double omega;
    int coarse_threshold;
    int inner_cycles_next;
    int inner_nu_coarse;
} mpfc_opts;

/* Per-step report.  residual_history is a caller-owned host array of
 * max_cycles + 1 doubles (may be NULL): entry 0 is the norm of the initial
 * guess's residual, entry k the norm after V-cycle k.  Energies (Sec. 3):
 * energy_F = F(phi^{k+1}) (eq. discrete_energy_PFC), energy_pseudo =
 * F + ||psi^{k+1}||_{-1}^2/(2M) (eq. discrete_energy_MPFC), energy_mod =
 * energy_pseudo + ||grad_h(phi^{k+1} - phi^k)||^2/2 (eq. energy_numer),
 * mass = h^2 sum phi^{k+1}. */
typedef struct {
    double energy_F, energy_pseudo, energy_mod, mass;
    double residual;     /* last residual norm */
    int n_cycles;        /* V-cycles run */
    int status;          /* return code of the step */
    int outer_iters;     /* mixed precision: FP64 defect-correction iterations */
    int energy_status;   /* 0, or MPFC_ENOTCONVERGED when the Poisson solve of the
                            -1 norm stopped at its cycle limit (energy_pseudo and
                            energy_mod are then approximate) */
    double *residual_history;
} mpfc_info;

typedef struct mpfc_ctx mpfc_ctx;

/* Default options: V(2,2), tol 1e-10, 100 cycles, FP64, extrapolated guess,
 * Newton linearisation, coarsest 2, energies on, divergence factor 1e8. */
void mpfc_default_opts(mpfc_opts *o);

/* Host-only validation of a configuration (no HIP call). */
int mpfc_validate(int m, int n, const mpfc_params *p, const mpfc_opts *o);

/* Create a solver context for an m x n grid: allocates the multigrid level
 * hierarchy and all workspace on the current HIP device.  *out receives the
 * context (owned by the caller, released by mpfc_destroy).  `stream` orders
 * all later work of the context. */
int mpfc_create(mpfc_ctx **out, int m, int n, const mpfc_params *p, const mpfc_opts *o,
                void *stream);

/* One time step (Sec. 3.1 / 3.2 with App. B).
 *   d_phi_n    phi^k (read)
 *   d_phi_nm1  phi^{k-1} (read; scheme 2 only; NULL means phi^{k-1} = phi^k,
 *              the start-up rule of Sec. 3.2)
 *   d_psi      psi^k on entry, psi^{k+1} on return (required: for scheme 2
 *              psi carries the history of the run, eq. discrete_2_b; the
 *              first step uses psi^0 = 0; must not alias d_phi_n or
 *              d_phi_nm1)
 *   d_phi_np1  phi^{k+1} (written; must not alias the inputs)
 *   d_mu, d_kappa  optional outputs (NULL to skip): mu^{k+1} (mu^{k+1/2} for
 *              scheme 2) and kappa; distinct arrays that alias none of the
 *              above (else MPFC_EINVAL)
 *   h_info     optional report (NULL to skip).
 * Returns after the final residual readback (the outputs are complete on the
 * context's stream).  On MPFC_ENOTCONVERGED / ENONFINITE / EDIVERGED the
 * outputs hold the last iterate and psi is still updated from it. */
int mpfc_step(mpfc_ctx *ctx, const double *d_phi_n, const double *d_phi_nm1, double *d_psi,
              double *d_phi_np1, double *d_mu, double *d_kappa, mpfc_info *h_info);

/* Energies of a state (Sec. 3; App. A "-1" norm with a mean-zero Poisson
 * solve under the context's boundary conditions): out[0..3] = F(phi), F + ||psi||_{-1}^2/(2M),
 * that + ||grad_h(phi - phi_prev)||^2/2, h^2 sum phi.  d_phi_prev may be NULL
 * (then the last term is 0). */
int mpfc_energies(mpfc_ctx *ctx, const double *d_phi, const double *d_phi_prev,
                  const double *d_psi, double *h_out);

/* Pinning (Sec. 4.6): from the next step on, mu is replaced by
 * mu~ = mu + 2 (phi^{k+1/2} - phi_hat) W with phi^{k+1/2} = (phi^{k+1} + phi^k)/2,
 * i.e. N^(2) gains -W phi and S^(2) gains W (phi^k - 2 phi_hat); the mu that
 * mpfc_step returns is mu~, and energy_F includes h^2 sum W (phi - phi_hat)^2.
 * d_weight (W >= 0) and d_phihat are m x n device arrays, copied during the
 * call (the caller keeps ownership); coarse levels use 2x2 averages of W.
 * d_weight = NULL switches pinning off.  Needs scheme 2, MPFC_FP64 and
 * MPFC_NEWTON (else MPFC_EINVAL); allocates the weight pyramid on first use. */
int mpfc_set_pinning(mpfc_ctx *ctx, const double *d_weight, const double *d_phihat);

/* Three space dimensions.  The paper notes that the schemes extend to three
 * dimensions in a straightforward way; this is that extension: the same
 * equations (Sec. 3.1 / 3.2, App. B.1 / B.2) with the seven-point Laplacian
 * (sum of the six face neighbours - 6 f) / h^2 on an m x n x l cell-centred
 * grid, periodic in every axis, cell (i, j, k) at index (k*n + j)*m + i; the
 * FAS V-cycle uses 2x2x2-average restriction and trilinear prolongation, the
 * coarsest level (smallest side 2) is relaxed by coarse_sweeps red-black sweeps
 * (red = (i+j+k) even); grid sums carry h^3 and the gradient norm is h times
 * the sum of squared face differences.  m, n, l powers of two >= 2, bc = 0,
 * MPFC_FP64, guess MPFC_GUESS_PREV or MPFC_GUESS_EXTRAP; other options as for
 * mpfc_create.  Arguments, ownership, outputs and return codes of
 * mpfc3d_step are those of mpfc_step (arrays of m*n*l doubles). */
typedef struct mpfc3d_ctx mpfc3d_ctx;
int mpfc3d_validate(int m, int n, int l, const mpfc_params *p, const mpfc_opts *o);
int mpfc3d_create(mpfc3d_ctx **out, int m, int n, int l, const mpfc_params *p,
                  const mpfc_opts *o, void *stream);
int mpfc3d_step(mpfc3d_ctx *ctx, const double *d_phi_n, const double *d_phi_nm1, double *d_psi,
                double *d_phi_np1, double *d_mu, double *d_kappa, mpfc_info *h_info);
/* Live timing (HIP events, direct launches while on) of the finest level's
 * red-black half-sweep launches: total ms, launch count, finest cells. */
int mpfc3d_prof_enable(mpfc3d_ctx *ctx, int on);
int mpfc3d_prof_read(mpfc3d_ctx *ctx, double *total_ms, long long *launches, long long *cells,
                     int reset);
void mpfc3d_destroy(mpfc3d_ctx *ctx);

/* Live timing of the two finest-level launches of each V-cycle (the dominant
 * kernels of the step) with HIP events on the context's stream:
 * which = 0: the down launch (nu1 red-black passes of the App. B smoother,
 * residual, restriction); which = 1: the up launch (coarse-grid correction,
 * nu2 passes, residual norm).  what = 1 enables, 0 disables; while enabled
 * the cycles are launched one by one instead of as a captured graph.
 * mpfc_prof_read returns, since the last reset, the summed event-to-event
 * duration in milliseconds, the number of launches timed and the cells of
 * the finest grid each launch covers. */
int mpfc_prof_enable(mpfc_ctx *ctx, int what);
int mpfc_prof_read(mpfc_ctx *ctx, int which, double *h_total_ms, long long *h_launches,
                   long long *h_cells_per_launch, int reset);

/* Tile of the tiled launch `which` (0 down, 1 up, 2 / 3 the FP32 down / up of
 * mixed precision, 4 / 5 the Poisson down / up of the energies) on multigrid
 * level `level` (0 = finest; only levels above 32 x 32 cells are tiled): the
 * interior tile tx x ty and the halo allowance of the kernel variant.  The
 * shapes are chosen when the context is created (timed; MPFC_TILE_SHAPE=<k>
 * forces shape k). */
int mpfc_tile_shape(mpfc_ctx *ctx, int level, int which, int *tx, int *ty, int *halo);

void mpfc_destroy(mpfc_ctx *ctx);
const char *mpfc_strerror(int code);
const char *mpfc_last_error(void);
int mpfc_version(void);

/* ---- Operator-level entry points (one operation of the V-cycle each) ----
 * Same operators as mpfc_step uses, on caller-provided FP64 device arrays of
 * an m x n grid with spacing p->h and boundary conditions p->bc; the library
 * forms the coefficients of eqs. discrete_1_a / discrete_2_a from *p
 * (c = s M/(beta + 1/s) or s M/(beta + 2/s), alpha = 1 - eps); *p is checked
 * as by mpfc_validate.  A coarse level of the multigrid hierarchy is a grid
 * of spacing 2^l h: pass a copy of the parameters with that h.  d_phik is
 * phi^k on this grid (scheme 2; ignored for scheme 1).  m and n are even
 * (any even value: powers of two use the bit-mask kernels, other sides the
 * general-index ones); otherwise MPFC_EINVAL. */

/* `sweeps` red-black nonlinear Gauss-Seidel passes (App. B), red
 * ((i+j) even) first, Newton (MPFC_NEWTON) or Picard (MPFC_PICARD) local
 * linearisation, in place on (d_phi, d_mu, d_kappa); m, n >= 4.  Runs the
 * fused tile kernel of the V-cycle and allocates a scratch copy of u. */
int mpfc_op_smooth(const mpfc_params *p, int linearization, int m, int n, const double *d_phik,
                   double *d_phi, double *d_mu, double *d_kappa, const double *d_f1,
                   const double *d_f2, const double *d_f3, int sweeps, void *stream);

/* mpfc_op_smooth without any allocation, for callers that cannot allocate
 * device memory during a call (code under HIP graph capture, serving loops):
 * same arguments, same result.  Its scratch (a copy of u and the discarded
 * restriction outputs) is a static device array of about 6.8 MB that each
 * GPU the library runs on holds until the process ends, so m n must be at
 * most 512 x 512 = 262144 cells (else MPFC_EINVAL).  Calls that overlap on
 * one GPU (other threads or streams) race on that array; each call waits for
 * its stream before returning, so calls in sequence do not.  The scratch is
 * fully written before it is read; nothing is kept between calls. */
int mpfc_op_smooth_noalloc(const mpfc_params *p, int linearization, int m, int n,
                           const double *d_phik, double *d_phi, double *d_mu, double *d_kappa,
                           const double *d_f1, const double *d_f2, const double *d_f3,
                           int sweeps, void *stream);

/* r = f - N(u) (App. B), three output arrays. */
int mpfc_op_residual(const mpfc_params *p, int m, int n, const double *d_phik,
                     const double *d_phi, const double *d_mu, const double *d_kappa,
                     const double *d_f1, const double *d_f2, const double *d_f3, double *d_r1,
                     double *d_r2, double *d_r3, void *stream);

/* Source S of the step (App. B.1 / B.2) from phi^k, phi^{k-1}, psi^k. */
int mpfc_op_source(const mpfc_params *p, int m, int n, const double *d_phik,
                   const double *d_phikm1, const double *d_psik, double *d_S1, double *d_S2,
                   double *d_S3, void *stream);

/* Average of the 2x2 fine cells under each coarse cell: (m/2) x (n/2) out. */
int mpfc_op_restrict(int m, int n, const double *d_fine, double *d_coarse, void *stream);

/* ---- batched simulations ------------------------------------------------------
 * Many independent simulations, each with its own grid size and parameters
 * (same scheme), advanced one time step at a time by shared launches: each
 * stage of the step (set-up, the tiled levels of one size, the coarse levels,
 * the residual, the psi update) is one launch over the work of every
 * simulation, and each simulation stops on its own residual test (Sec. 4's
 * V-cycle iteration, run per simulation).  A simulation's iterates are those
 * of a single-grid context with the same options. */
#define MPFC_BATCH_MAX 4096

typedef struct {
    int m, n;            /* grid cells in x and y (powers of two, m n > 1024) */
    mpfc_params p;       /* eps, beta, M, h, dt, scheme (scheme equal across the batch) */
} mpfc_sim_desc;

typedef struct mpfc_batch mpfc_batch;

/* Create a batch of `nsim` simulations (1 ... MPFC_BATCH_MAX): every one is
 * validated as by mpfc_validate, and gets its own level hierarchy and
 * workspace on the current device.  The options apply to all of them; the
 * energy option is ignored (a batch computes no energies).  Tile shapes are
 * chosen by timing every launch of the batch at creation.  *out is owned by
 * the caller and released by mpfc_batch_destroy.  `stream` orders all work. */
int mpfc_batch_create(mpfc_batch **out, int nsim, const mpfc_sim_desc *sims,
                      const mpfc_opts *o, void *stream);

/* One time step of every simulation.  Each argument is a host array of nsim
 * device pointers with the meaning of mpfc_step's argument of that name
 * (d_phi_nm1 may be NULL, or hold NULL entries: phi^{k-1} = phi^k).
 * h_infos: NULL, or nsim reports (residual_history honoured per entry;
 * energies are 0).  Returns MPFC_OK when every simulation converged, else the
 * status of the first one that did not (all outputs are still written). */
int mpfc_batch_step(mpfc_batch *b, const double *const *d_phi_n,
                    const double *const *d_phi_nm1, double *const *d_psi,
                    double *const *d_phi_np1, mpfc_info *h_infos);

/* Number of simulations (0 for NULL). */
int mpfc_batch_size(const mpfc_batch *b);

void mpfc_batch_destroy(mpfc_batch *b);

/* ---- learned initial guess -------------------------------------------------------
 * Each step has exactly one solution (Sec. 3, unique solvability), so its
 * initial guess is free; a better one only saves V-cycles.  The learned guess
 * is a periodic convolutional network (four 3x3 layers, 3 -> 32 -> 32 -> 32 -> 1
 * channels, tanh-form GELU after the first three; BF16 weights and
 * activations on the matrix cores, FP32 accumulation):
 *   inputs  x0 = in_scale phi^n, x1 = (phi^n - phi^{n-1}) / sigma1 and
 *           x2 = (dt psi^n - (phi^n - phi^{n-1})) / sigma1, sigma1 the rms of
 *           phi^n - phi^{n-1} (x1 = x2 = 0 when sigma1 = 0); psi^n enters
 *           because the step depends on it and, for scheme 2, it carries the
 *           run's history (eq. discrete_2_b);
 *   output  delta; guess = 2 phi^n - phi^{n-1} + c, c = out_scale sigma1 delta
 *           minus its mean (the guess keeps the mass of the extrapolation).
 * In a step with guess mode MPFC_GUESS_CNN both the learned and the
 * extrapolated guess are completed (mu, kappa as for any guess) and the one
 * with the smaller FP64 residual starts the V-cycles (fallback).
 *
 * Blob (host float32, mpfc_cnn_blob_size() values): header [2, 3, 32, 4,
 * in_scale, out_scale, dt, 0] (dt: the time step the network was trained
 * for; mpfc_cnn_load rejects another), then per layer W[ky][kx][ci][co]
 * (ky, kx = 0..2 for offsets -1..1 in y and x) and b[co]: W1 (3,3,3,32), b1 (32),
 * W2 (3,3,32,32), b2, W3 (3,3,32,32), b3, W4 (3,3,32,1), b4 (1).  Grids must be
 * powers of two of at least 16 x 16. */
int mpfc_cnn_blob_size(void);

/* Copy a network into the context (device memory of its own, freed with the
 * context); also resets the counters below.  EINVAL on a malformed blob. */
int mpfc_cnn_load(mpfc_ctx *ctx, const float *h_blob, size_t count);

/* Steps that started from the learned guess, and fallbacks to extrapolation. */
int mpfc_cnn_counts(mpfc_ctx *ctx, long long *used, long long *fallbacks);

typedef struct {
    float lr, beta1, beta2, eps;   /* Adam (Kingma and Ba, 2015) */
} mpfc_cnn_hparams;

typedef struct mpfc_cnn_trainer mpfc_cnn_trainer;

/* Trainer for batches of `batch` samples of an m x n grid, starting from
 * h_blob (FP32 master weights on the device, BF16 copies for the kernels).
 * Loss: mean over every pixel of the batch of (delta - t)^2 with
 * t = (phi^{n+1} - 2 phi^n + phi^{n-1}) / (out_scale sigma1). */
int mpfc_cnn_trainer_create(mpfc_cnn_trainer **out, int m, int n, int batch,
                            const float *h_blob, size_t count, const mpfc_cnn_hparams *hp,
                            void *stream);

/* Forward and backward pass over one batch (host arrays of `batch` device
 * pointers to m x n FP64 fields: phi^{n-1}, phi^n, psi^n and the solution
 * phi^{n+1}); `update` != 0 then takes one Adam step.
 * h_loss: the loss before the update; h_grad: NULL or mpfc_cnn_blob_size() - 8
 * floats receiving the gradient in blob order. */
int mpfc_cnn_train_step(mpfc_cnn_trainer *t, const double *const *d_phi_nm1,
                        const double *const *d_phi_n, const double *const *d_psi_n,
                        const double *const *d_phi_np1, int update, double *h_loss,
                        float *h_grad);

/* Mean-corrected learned guesses of a batch with the current weights. */
int mpfc_cnn_predict(mpfc_cnn_trainer *t, const double *const *d_phi_nm1,
                     const double *const *d_phi_n, const double *const *d_psi_n,
                     double *const *d_guess);

/* Learning rate of the following Adam steps (a schedule is the caller's). */
int mpfc_cnn_trainer_set_lr(mpfc_cnn_trainer *t, float lr);

/* Current weights as a blob (count = mpfc_cnn_blob_size()). */
int mpfc_cnn_trainer_blob(mpfc_cnn_trainer *t, float *h_blob, size_t count);

void mpfc_cnn_trainer_destroy(mpfc_cnn_trainer *t);

#ifdef __cplusplus
}
#endif
#endif /* MPFC_H */
