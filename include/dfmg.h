/*
 * dfmg -- divergence-free geometric multigrid for isogeometric compatible
 * (divergence-conforming B-spline) discretizations of the generalized Stokes
 * and Oseen problems on MI355X (gfx950).
 *
 * Method: Coley, Benzaken, Evans, "A geometric multigrid method for
 * isogeometric compatible discretizations of the generalized Stokes and Oseen
 * problems" (arXiv:1705.09282).  The problem statement (weak form with Nitsche
 * no-slip and strong no-penetration, block system K U = F) is the paper's
 * section on spatial discretization; the spaces are its compatible B-spline
 * spaces; the solver is its Algorithm 1 (V-cycle) with the additive Schwarz
 * smoother of equation ASM on subdomains that are supports of streamfunction
 * (2D) / vector-potential (3D) basis functions.
 *
 * Conventions (all entry points):
 *  - Return value 0 = success, negative = error (DFMG_E*).  The message of the
 *    last error on the calling thread is returned by dfmg_last_error().
 *    No C++ exception crosses this interface.
 *  - "host" pointers are CPU memory owned by the caller; "device" pointers are
 *    HIP device memory owned by the caller.  The library owns only its context
 *    (host memory) and the internal HIP stream and graph it creates at bind.
 *  - Vectors are FP64 in canonical DOF order [u_0 | u_1 (| u_2) | p]; inside a
 *    block the tensor multi-index runs x fastest.  Velocity component c has
 *    B-spline degree k+1 in direction c and k in the others, with the two end
 *    functions in direction c removed (strong v.n = 0); the pressure block keeps
 *    all (N+k)^d functions of degree k.  Level n_levels-1 is the finest grid.
 *  - Device work is ordered on the stream given to dfmg_bind; calls that
 *    return numbers to the host (solve, norms) synchronize that stream.
 *  - A context is not thread-safe; different contexts are independent.
 */
#ifndef DFMG_H
#define DFMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DFMG_OK 0
#define DFMG_EINVAL (-1)   /* invalid argument or size */
#define DFMG_ENOMEM (-2)   /* workspace too small / host allocation failed */
#define DFMG_EHIP (-3)     /* HIP runtime error; message carries hipGetErrorString */
#define DFMG_ENOTCONV (-4) /* max_cycles reached; U holds the last iterate */
#define DFMG_EDIVERGED (-5)/* NaN/Inf or residual growth; U holds the last iterate */
#define DFMG_ESTATE (-6)   /* call out of order (e.g. vcycle before bind) */

typedef struct dfmg_ctx dfmg_ctx;

/* The parametric unit square (dim 2) or cube (dim 3) split into n_elem^dim
 * equal elements on the finest grid; n_levels nested grids obtained by
 * halving, so n_elem must be divisible by 2^(n_levels-1) (coarsest grid
 * n_elem / 2^(n_levels-1) >= 1).
 *
 * geometry 0: the physical domain is the unit square / cube itself.
 * geometry 1: the quarter annulus of the paper's mapped 2D test (and, in 3D,
 *   the hollow cylinder section: that annulus extruded along z by depth),
 *   x = r (cos theta, sin theta) [, depth xi_3] with r = r_inner + (r_outer -
 *   r_inner) xi_1 and theta(xi_2) the quarter circle from the x axis to the
 *   y axis as a quadratic rational Bezier arc (section on isogeometric
 *   compatible B-splines, equations physical_2D and physical_3D: velocities
 *   by the contravariant Piola map, pressures by q o F = q_hat / det J).  The
 *   coefficient vectors keep the parametric layout; the operators are the
 *   physical ones (the velocity rows couple every component), assembled by
 *   quadrature on the finest grid and by Galerkin products below.  Takes
 *   generalized Stokes problems only (advection kind 0), no time stepping and
 *   no manufactured load (the caller assembles F); the residual runs with
 *   one lane per row and no single-workgroup coarse cycle.  Zero-filled
 *   fields (geometry 0) keep the unit domain. */
typedef struct {
    int dim;
    int n_elem;
    int n_levels;
    int geometry;
    double r_inner, r_outer, depth;  /* geometry 1: 0 < r_inner < r_outer; depth > 0 in 3D */
} dfmg_grid;

/* Advection field of the generalized Oseen problem (paper, weak form).
 * kind 0: none (generalized Stokes).
 * kind 1: rigid rotation about the centre, a = c * (-(y - 1/2), x - 1/2) in
 *         2D, a = c * (-(y - 1/2), x - 1/2, 0) in 3D.
 * kind 2: a = c * u with u the manufactured velocity of
 *         dfmg_manufactured_rhs (the paper's Oseen problems take the
 *         advection equal to the manufactured velocity).
 * kind 3: a = c * w with w the field of the finest velocity space whose
 *         coefficients (n_v values, canonical velocity order, host memory,
 *         copied at setup) are `coeffs`: Guermond's scheme advects with
 *         3/2 u^n - 1/2 u^{n-1}.  Its term is assembled by Gauss quadrature
 *         on the finest grid and Galerkin-projected (R C P) to the coarser
 *         ones; subdomain inverses are not shared.
 * |a| (the network's input |a| h / nu) is max |a|: |c| / sqrt(2) for
 * kind 1, |c| max |u| for kind 2, not defined for kind 3 (0). */
typedef struct {
    int kind;
    double c;
    const double *coeffs;  /* kind 3 only (else ignored, may be NULL) */
} dfmg_advection;

/* Solver options.  dfmg_default_options fills: nu1 = nu2 = 2, eta = 0 (use the
 * stable fixed damping for (dim, k): 0.35 for 2D k=1, 0.2 for 2D k=2, 0.07 for
 * 3D k=1, 0.02 for 3D k=2), precision 0, smoother 0, max_cycles 200,
 * use_graph 1, cycles_per_check 1, share_inverses 1, inner_cycles 1,
 * multiplicative 0, time_stepping 0. */
typedef struct {
    int nu1;              /* pre-smoothing steps per level (Algorithm 1)        */
    int nu2;              /* post-smoothing steps per level                     */
    double eta;           /* fixed additive-Schwarz damping; <= 0: default      */
    int precision;        /* 0: FP64 V-cycles; 1: solve by FP64 iterative
                             refinement around FP32 V-cycles (see dfmg_solve)    */
    int smoother;         /* 0 auto, 1 two-pass gather, 2 coloured scatter, 3 one-pass,
                             4 two-pass with one thread per small subdomain */
    int max_cycles;       /* solve: cycle limit (ENOTCONV beyond)               */
    int use_graph;        /* 1: replay the V-cycle as a captured hipGraph       */
    int cycles_per_check; /* solve: V-cycles launched between host checks       */
    int share_inverses;   /* 1: subdomains with equal local systems (to 1e-14)
                             share one stored inverse; 0: one per subdomain     */
    int inner_cycles;     /* precision 1: FP32 V-cycles per refinement step     */
    int multiplicative;   /* 1: multiplicative Schwarz smoother (equation MSM):
                             each smoothing step solves the subdomains one after
                             another, each on the residual the previous ones
                             left, undamped (eta, the smoother forms and the
                             damping schedule do not apply).  Subdomains are
                             visited colour by colour in the coupling-free
                             colouring (o, a mod (k+2), b mod (k+2)[, c mod
                             (k+2)]) of dfmg_export_sweep_colours, ascending
                             inside a colour (the paper leaves the order open).
                             Needs precision 0. */
    int time_stepping;    /* 1: reserve the quadrature workspace of the
                             Crank-Nicolson / Adams-Bashforth load
                             (dfmg_cnab_rhs, dfmg_cnab_step) */
} dfmg_options;

#define DFMG_MAX_HISTORY 512

typedef struct {
    int cycles;           /* V-cycles applied                                   */
    int converged;        /* 1 if ||F - K U||_2 <= tol ||F||_2                  */
    int status;           /* return code of the solve                           */
    int fallback;         /* 1 if the learned damping was replaced by the fixed one */
    double res0;          /* ||F - K U_0||_2                                    */
    double res_final;     /* residual norm at exit                              */
    double rho;           /* (res_final / res0)^(1/cycles)                      */
    double fnorm;         /* ||F||_2                                            */
    double solve_seconds; /* wall time of the solve (host clock, stream synced) */
    int n_history;
    double history[DFMG_MAX_HISTORY]; /* residual norm at the start of each cycle */
} dfmg_stats;

void dfmg_default_options(dfmg_options *opt);

/* Host-side setup of the whole hierarchy (section on nested complexes and
 * Galerkin coarse operators K_l = R K_{l+1} P, subdomains of the Schwarz
 * smoother, prefactored local saddle-point inverses, coarse-grid inverse).
 * k in {1, 2} is the pressure degree (the paper's p = k + 1), nu > 0,
 * sigma >= 0.  opt may be NULL (defaults).  On success *out owns host memory
 * released by dfmg_destroy.  Errors: EINVAL. */
int dfmg_setup(const dfmg_grid *grid, int k, double nu, double sigma,
               const dfmg_advection *adv, const dfmg_options *opt, dfmg_ctx **out);

/* Batch of nprob independent problems on one mesh (same grid and k), with
 * per-problem nu[p], sigma[p] and adv[p] (adv may be NULL).  Every kernel
 * launch of the batch covers all problems, which share the mesh data (index
 * maps, transfer operators).  Vectors of a batch are nprob blocks of the
 * finest-level length n, problem-major; dfmg_solve, dfmg_vcycle,
 * dfmg_residual_norm, dfmg_div_norm, the level-wise kernels and
 * dfmg_manufactured_rhs act on every problem (stats and norms: nprob
 * entries).  Exports describe the shared mesh data and problem 0's matrix.
 * dfmg_setup is the batch of one.  Errors: EINVAL. */
int dfmg_batch_setup(int nprob, const dfmg_grid *grid, int k, const double *nu, const double *sigma,
                     const dfmg_advection *adv, const dfmg_options *opt, dfmg_ctx **out);
int dfmg_batch_size(const dfmg_ctx *ctx, int *nprob);

void dfmg_destroy(dfmg_ctx *ctx);

/* Device bytes the caller must provide to dfmg_bind. */
int dfmg_workspace_bytes(const dfmg_ctx *ctx, size_t *bytes);

/* Bind caller-owned device memory (>= dfmg_workspace_bytes, 256-byte aligned)
 * and the caller's HIP stream (NULL = default stream); uploads the hierarchy
 * and synchronizes.  The workspace must stay valid until dfmg_destroy.
 * Errors: EINVAL, ENOMEM (too small), EHIP. */
int dfmg_bind(dfmg_ctx *ctx, void *dev_workspace, size_t bytes, void *hip_stream);

/* Sizes of level `level` (0 = coarsest).  Any output pointer may be NULL.
 * n_patch is 0 on level 0 (exact solve there).  nnz counts the non-zero
 * entries of K_level. */
int dfmg_sizes(const dfmg_ctx *ctx, int level, int64_t *n_vel, int64_t *n_pres,
               int64_t *n_patch, int64_t *nnz);

/* Set one damping per smoothed level, finest first: n = n_levels - 1 values in
 * (0, 1) for every problem, or n = nprob * (n_levels - 1) values, problem-major;
 * replaces the fixed damping for later cycles. */
int dfmg_set_eta(dfmg_ctx *ctx, const double *eta_host, int n);

/* ncycles applications of Algorithm 1 on the finest level: U <- MGV(U, F).
 * F_dev, U_dev: device, length n of the finest level; U is read and written.
 * Stream-ordered, no host synchronization.  Errors: ESTATE, EINVAL, EHIP. */
int dfmg_vcycle(dfmg_ctx *ctx, const double *F_dev, double *U_dev, int ncycles);

/* Per-level smoothing steps of Algorithm 1 (nu1 before, nu2 after the coarse
 * correction), n = n_levels - 1 entries each, finest level first, in [0, 16],
 * for every problem of the batch (they share the launch sequence).  Default:
 * the options' nu1, nu2 on every level.  Errors: EINVAL. */
int dfmg_set_smoothing(dfmg_ctx *ctx, const int *nu1_host, const int *nu2_host, int n);
int dfmg_get_smoothing(const dfmg_ctx *ctx, int *nu1_host, int *nu2_host);

/* Repeat V-cycles from U (device, in/out) until ||F - K U||_2 <= tol ||F||_2
 * (numerical-results protocol, relative to ||F||), then shift the pressure to
 * zero mean.  st may be NULL (else nprob entries).  Errors: ENOTCONV,
 * EDIVERGED (worst over the batch), ESTATE, EHIP.
 * With precision 1 each step computes r = F - K U in FP64, applies
 * inner_cycles V-cycles in FP32 (FP32 values, FP32 accumulation, FP64 coarse
 * solve) to K dU = r from dU = 0 that also accumulate the potential
 * coefficients psi of dU's velocity (every local velocity correction is the
 * curl of local streamfunctions (2D) or vector potentials (3D), the reduced
 * subdomain problem; in 3D the minimum-norm local potentials, since the
 * curl has gradients in its kernel near the boundary; prolongation and the
 * coarse solve carry psi along), and updates u += curl psi, p += dU_p in
 * FP64, so u stays divergence-free to FP64 rounding.  The FP32
 * cycle runs smoother form 3 where tuned so and form 4 otherwise.  Stats
 * count refinement steps as cycles. */
int dfmg_solve(dfmg_ctx *ctx, const double *F_dev, double *U_dev, double tol, dfmg_stats *st);

/* Crank-Nicolson / Adams-Bashforth time stepping of the Navier-Stokes
 * equations (section on temporal discretization, equation GS): each step is
 * the generalized Stokes problem of the context (sigma = 2 / dt, no
 * advection) with the load
 *   F_u = F2 - (K U^n)_u + (N_i, 2 sigma u^n - 3 (u^n . grad) u^n
 *                                 + (u^{n-1} . grad) u^{n-1}),   F_p = 0,
 * where F2 is the caller's load vector of 2 f(t_{n+1/2}) (every term of the
 * step is doubled so that its implicit side is the context's operator; the
 * paper's printed f(t_{n+1/2}) lacks that factor 2) and, for the first step
 * (Uold NULL), -2 (u^n . grad) u^n replaces the convective terms (the
 * paper's footnote).  Integrals by Gauss quadrature, k + 3 points per
 * direction per element.  All vectors are device arrays of the finest level
 * (problem-major in a batch).  Needs options.time_stepping = 1 at setup and
 * advection kind 0.
 * dfmg_cnab_rhs: the load into Fout (stream-ordered).
 * dfmg_cnab_step: the load, then dfmg_solve from Unext = U^n to tol; Unext
 * receives U^{n+1} (with zero-mean pressure).  Errors: as dfmg_solve;
 * ESTATE without time_stepping; EINVAL with advection. */
int dfmg_cnab_rhs(dfmg_ctx *ctx, const double *F2_dev, const double *U_dev, const double *Uold_dev, double *Fout_dev);
int dfmg_cnab_step(dfmg_ctx *ctx, const double *F2_dev, const double *Uold_dev, const double *U_dev, double *Unext_dev,
                   double tol, dfmg_stats *st);
/* Guermond's semi-implicit step (equation GO): the operator of the context
 * advects with a^{n+1} = 3/2 u^n - 1/2 u^{n-1} (u^0 at the first step, the
 * paper's footnote; advection kind 3 at setup), sigma = 2 / dt, and the load
 * of the doubled step is F_u = F2 - (K(a) U^n)_u + (N_i, 2 sigma u^n),
 * F_p = 0, F2 the caller's load of 2 f(t_{n+1/2}).  Needs time_stepping = 1.
 * The operator changes every step: a new context per step. */
int dfmg_go_rhs(dfmg_ctx *ctx, const double *F2_dev, const double *U_dev, double *Fout_dev);

/* ||F - K U||_2 on the finest level (device inputs, host output). */
int dfmg_residual_norm(dfmg_ctx *ctx, const double *F_dev, const double *U_dev, double *out);

/* ||div u_h||_{L2(Omega)} of the velocity part of U (lemma of the section on
 * the Stokes complex: zero for an exactly divergence-free field). */
int dfmg_div_norm(dfmg_ctx *ctx, const double *U_dev, double *out);

/* ---- Level-wise kernels (device pointers), for parity checks of each step ----
 * residual:  r = F - K_level U                       (Algorithm 1, residual)
 * smooth:    nsteps x  U <- U + eta_l sum_i E_i^T M_i E_i (F - K_level U)
 *            (equation ASM; M_i the bordered local inverse)
 * restrict:  G = R_level r,   R_level = P_{level-1}^T   (level >= 1)
 * prolong:   U += P_{level-1} dU                       (level >= 1)
 * coarse:    dU = K_0^{-1} G with zero-mean pressure (bordered inverse) */
int dfmg_level_residual(dfmg_ctx *ctx, int level, const double *F_dev, const double *U_dev, double *r_dev);
int dfmg_level_smooth(dfmg_ctx *ctx, int level, const double *F_dev, double *U_dev, int nsteps);
int dfmg_level_restrict(dfmg_ctx *ctx, int level, const double *r_dev, double *G_dev);
int dfmg_level_prolong_add(dfmg_ctx *ctx, int level, const double *dU_dev, double *U_dev);
int dfmg_coarse_solve(dfmg_ctx *ctx, const double *G_dev, double *dU_dev);

/* Average duration in milliseconds of one launch of a V-cycle kernel over
 * `reps` back-to-back launches on the library's stream, timed with HIP events
 * recorded on that stream, on the context's own level vectors (whatever the
 * last cycle left there) for every problem of the batch, in the launch
 * configuration the cycles use.  kernel: 0 = FP64 residual r = F - K_level U,
 * 1 = FP32 residual (precision 1 only), 2 = FP64 smoothing step, 3 = FP32
 * smoothing step (levels >= 1).  Synchronizes; leaves the level vectors
 * changed (a solve reloads them).  Errors: EINVAL. */
int dfmg_time_kernel(dfmg_ctx *ctx, int kernel, int level, int reps, double *ms_out);

/* ---- Kernel variants per level (the autotuner's search space) ----
 * lpr[l]:      lanes of a wavefront per matrix row in the residual kernel of
 *              level l (1, 2 or 4);
 * smoother[l]: 1 = subdomain-parallel local solves + per-DOF gather of the
 *              corrections, 2 = one launch per DOF-disjoint colour with plain
 *              read-modify-write scatter (no atomics), 3 = one pass in which
 *              every DOF recomputes the local-solve rows it receives, 4 =
 *              as 1 with one thread per subdomain of at most 8 DOFs (the
 *              interior ones); 3 and 4 equal 1 bit for bit; ignored on
 *              level 0.  smoother[l] = 5 on levels 1 .. t (t <= n_levels - 2)
 *              runs levels t .. 0 of every V-cycle in one launch with one
 *              workgroup per problem (same sums as 1 with lpr 1); off by
 *              default.
 * Arrays have n_levels entries.  The variants differ only in summation
 * order (lpr splits a row's dot product over lanes). */
int dfmg_get_tuning(const dfmg_ctx *ctx, int *lpr, int *smoother);
int dfmg_set_tuning(dfmg_ctx *ctx, const int *lpr, const int *smoother);
/* Tile shape of the form-4 local solves per level (n_levels entries each):
 * bs threads per workgroup (64, 128, 256, 512: bs interior subdomains, or
 * bs / tb boundary subdomains, per workgroup), ms how a workgroup reads an
 * inverse all its interior subdomains share (0 scalar loads per wavefront,
 * 1 staged in LDS per workgroup, 2 per-thread loads), tb threads per
 * boundary subdomain (32 or 64).  Defaults 256, 0, 64.  All shapes give the
 * same bits; a shape whose LDS would exceed 48 KB runs as the default.
 * Errors: EINVAL. */
int dfmg_get_tile_shape(const dfmg_ctx *ctx, int *bs, int *ms, int *tb);
int dfmg_set_tile_shape(dfmg_ctx *ctx, const int *bs, const int *ms, const int *tb);
/* Average milliseconds of one V-cycle (the kind the solves run: FP64, or the
 * FP32 cycle of the refinement) captured as a hipGraph and replayed reps
 * times, best of three rounds, on the context's level vectors, HIP events on
 * the library stream.  Requires dfmg_bind; synchronizes. */
int dfmg_time_cycle(dfmg_ctx *ctx, int reps, double *ms_out);
/* Time every variant of every level on the device (reps launches each, HIP
 * events on the library stream) and keep the fastest; ms_out (nullable,
 * 2 * n_levels entries) receives the best residual and smoother times.
 * Then times whole V-cycles for every choice of t (levels of at most 16384
 * DOFs) and keeps the fastest.  Last, in context: whole V-cycles captured
 * as one graph and replayed (as the solves run them) for every lanes-per-row
 * variant and smoother form of one level at a time, finest level first, the
 * others as chosen; a change is kept when the cycle gets faster by more than
 * 0.5% (best of three rounds of reps replays); on levels that run form 4,
 * the same for the tile shape (workgroup size, then the reading of shared
 * inverses, then the threads per boundary subdomain).  Requires dfmg_bind.
 * Leaves the solver state unchanged. */
int dfmg_autotune(dfmg_ctx *ctx, int reps, double *ms_out);

/* ---- Learned per-level smoothing parameters ----
 * A perceptron predicts, for every smoothed level, the damping eta in (0, 1)
 * of equation ASM and the number of smoothing steps of Algorithm 1:
 * x = (log10(nu)/2, log10(sigma)/4, |a| h / nu, k - 1.5) with |a| = max|a|
 * and h = 1/n_elem; h1 = tanh(W1 x + b1) (32), h2 = tanh(W2 h1 + b2) (32),
 * z = W3 h2 + b3 (10 outputs); eta_l = 1 / (1 + exp(-z_l)) from outputs 0..4
 * and steps_l = clamp(round(z_{5+l}), 1, 8) from outputs 5..9, finest
 * smoothed level first (deeper hierarchies reuse the last).  Parameters are
 * FP32, packed [W1 (32x4 row-major), b1, W2 (32x32), b2, W3 (10x32), b3].
 * The three kernels below take device arrays and a HIP stream (NULL =
 * default) and do not synchronize. */
#define DFMG_MLP_NPARAM 1546
/* Z (n x 10) = outputs for the features X (n x 4). */
int dfmg_mlp_forward(int n, const float *W_dev, const float *X_dev, float *Z_dev, void *stream);
/* G = gradient and *loss_dev = value of scale * sum M (Z - Y)^2 over the n
 * samples (Y, M: n x 10 targets and weights); work_dev holds
 * n * (DFMG_MLP_NPARAM + 1) floats.  Fixed summation order (deterministic). */
int dfmg_mlp_grad(int n, const float *W_dev, const float *X_dev, const float *Y_dev, const float *M_dev,
                  float scale, float *work_dev, float *G_dev, float *loss_dev, void *stream);
/* dfmg_mlp_grad without the work array, for callers that cannot allocate
 * device memory (code under HIP graph capture, loops that forbid hipMalloc):
 * the per-sample partials live in a static device array of the library
 * (DFMG_MLP_SCRATCH_SAMPLES * (DFMG_MLP_NPARAM + 1) floats, 3.2 MB per GPU,
 * held until the process ends), so n must lie in [1,
 * DFMG_MLP_SCRATCH_SAMPLES] (EINVAL otherwise, nothing launched).  Same
 * kernels and summation order as dfmg_mlp_grad, so the results are equal
 * bit for bit.  Allocates nothing.  Every call on one GPU uses that GPU's
 * one array: calls that overlap on a GPU (other streams, other threads)
 * race and give wrong results; serialize them.  Errors: EINVAL, EHIP. */
#define DFMG_MLP_SCRATCH_SAMPLES 512
int dfmg_mlp_grad_noalloc(int n, const float *W_dev, const float *X_dev, const float *Y_dev, const float *M_dev,
                          float scale, float *G_dev, float *loss_dev, void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, t >= 1). */
int dfmg_mlp_adam(float *W_dev, float *m_dev, float *v_dev, const float *G_dev, int t, float lr, void *stream);
/* Use the network W_host for the dampings of every problem of ctx (computed
 * on the device from each problem's nu, sigma, advection, grid and k) and for
 * the batch's smoothing steps per level (the largest prediction over its
 * problems, pre = post; they share one launch sequence), replacing
 * dfmg_set_smoothing.  With rho_plain_host (nprob entries, nullable) a solve
 * switches a problem back to the fixed damping as soon as one V-cycle after
 * the first contracts its residual by more than 1.05 * rho_plain (a
 * single-cycle ratio of the fixed damping), or any cycle lets it grow by six
 * orders, and reports it in stats.fallback.  The switch happens once per
 * solve; the next solve starts from the learned dampings again; the steps stay.
 * W_host NULL restores the fixed damping and the options' steps.  Requires
 * dfmg_bind. */
int dfmg_set_learned(dfmg_ctx *ctx, const float *W_host, const double *rho_plain_host);
/* Current dampings, nprob * (n_levels - 1) values, finest level first. */
int dfmg_get_eta(dfmg_ctx *ctx, double *eta_host);

/* Chebyshev damping schedule of the additive smoother (each smoothing step is
 * still U <- U + eta_j S^-1 (F - K U), equation ASM with a scalar damping, so
 * every correction stays divergence-free; only eta changes from step to step).
 * The smoother is a polynomial in the preconditioned operator S^-1 K; with
 * dampings 1 / theta_j, theta_j the zeros of the Chebyshev polynomial of
 * degree nu mapped to [b / alpha, b], its error polynomial is the scaled
 * Chebyshev polynomial T_nu((b + a - 2x) / (b - a)) / T_nu((b + a) / (b - a)),
 * a = b / alpha, which has the least maximum over [a, b] among polynomials of
 * degree nu with value 1 at 0 (Chebyshev semi-iteration, as used for
 * multigrid smoothing by Adams, Brezina, Hu and Tuminaro, 2003).  b = 1.05 x
 * the largest |eigenvalue| of S^-1 K of each problem and smoothed level,
 * estimated here by `iters` power-iteration steps with the level's residual
 * and smoother kernels in FP64 (deterministic start vector; host norms;
 * synchronizes the stream).  nu = the level's pre- or post-smoothing count:
 * pre-smoothing takes the zeros theta_0 > theta_1 > ..., post-smoothing the
 * reverse order.  The schedule replaces the per-level dampings (fixed or
 * learned) in every smoothing step of later cycles, in FP64 and FP32 cycles
 * alike, and follows later changes of the step counts (dfmg_set_smoothing,
 * dfmg_set_learned).  The fallback of dfmg_set_learned switches a problem to
 * its fixed damping in every step; the next solve restores the schedule.
 * The single-workgroup coarse cycle is not used while a schedule is on.
 * alpha in (1, 1e6] turns it on, alpha < 0 turns it on with the default
 * ratio of the dimension (10 in 2D, 60 in 3D), alpha 0 off (iters unused
 * then); iters in [1, 1000].  Requires dfmg_bind.  Errors: EINVAL, ESTATE,
 * EHIP. */
int dfmg_set_chebyshev(dfmg_ctx *ctx, double alpha, int iters);
/* Interval ratios alpha of the schedule in use, per smoothed level (finest
 * first): n = n_levels - 1 values for every problem or nprob * (n_levels - 1)
 * problem-major, each in (1, 1e6]; rebuilds the dampings from the existing
 * eigenvalue estimates.  ESTATE without a schedule; EINVAL. */
int dfmg_set_chebyshev_alpha(dfmg_ctx *ctx, const double *alpha_host, int n);
/* Current ratios (host out), nprob * (n_levels - 1), finest level first. */
int dfmg_get_alpha(const dfmg_ctx *ctx, double *alpha_host);
/* Learned Chebyshev schedule: the network W_host (same layout and inference
 * kernel as dfmg_set_learned, inputs log10(nu)/2, log10(sigma)/4, |a|h/nu,
 * k - 1.5) predicts per smoothed level, finest first, the logit of
 * a / b = 1 / alpha (outputs 0..4; levels past the fifth take output 4;
 * alpha clamped to [1.5, 1000]) and the smoothing steps (outputs 5..9,
 * rounded, clamped to [1, 8], the largest over the batch, pre = post).
 * Turns the schedule on with those ratios and steps (eigenvalue estimates by
 * `iters` power iterations unless a previous call made them); the per-level
 * dampings are the fixed ones, which the fallback (rho_plain_host, as in
 * dfmg_set_learned) switches a problem to.  W_host NULL turns the schedule
 * off and restores the options' steps.  Requires dfmg_bind; synchronizes the
 * stream.  Errors: EINVAL, ESTATE, EHIP. */
int dfmg_set_learned_chebyshev(dfmg_ctx *ctx, const float *W_host, const double *rho_plain_host, int iters);
/* The eigenvalue estimates of the last dfmg_set_chebyshev (host out):
 * nprob * (n_levels - 1) values, finest level first.  ESTATE before. */
int dfmg_get_lmax(const dfmg_ctx *ctx, double *lmax_host);
/* The per-step dampings in use (host out): nprob * (n_levels - 1) * 32
 * values, problem-major, finest level first; per level 16 pre-smoothing steps
 * then 16 post-smoothing steps (entries past a step count repeat its last).
 * ESTATE without a schedule. */
int dfmg_get_schedule(dfmg_ctx *ctx, double *out_host);

/* ---- Host exports for bit-exact index-map parity and value parity ----
 * CSR of K_level (explicit zeros dropped): rowptr[n+1], col[nnz], val[nnz]. */
int dfmg_export_matrix(const dfmg_ctx *ctx, int level, int64_t *rowptr, int32_t *col, double *val);
/* Subdomains of level >= 1: ptr[n_patch+1], dofs[ptr[n_patch]] (ascending
 * global DOF indices per subdomain), color[n_patch] (DOF-disjoint colours).
 * dfmg_patch_total gives ptr[n_patch]. */
int dfmg_patch_total(const dfmg_ctx *ctx, int level, int64_t *total);
int dfmg_export_patches(const dfmg_ctx *ctx, int level, int64_t *ptr, int32_t *dofs, int32_t *color);
/* Coupling-free colour of every subdomain of level >= 1 (n_patch entries):
 * the visiting order of the multiplicative sweep (contexts set up with
 * multiplicative = 1 and 0 alike).  Two subdomains of one colour share no
 * DOF and K couples no DOF of one with a DOF of the other. */
int dfmg_export_sweep_colours(const dfmg_ctx *ctx, int level, int32_t *colour);
/* Prolongation P_{level-1} (rows: level, cols: level-1) as CSR; nnz via
 * dfmg_prolongation_nnz. */
int dfmg_prolongation_nnz(const dfmg_ctx *ctx, int level, int64_t *nnz);
int dfmg_export_prolongation(const dfmg_ctx *ctx, int level, int64_t *rowptr, int32_t *col, double *val);

/* Load vector F = [l(N^v_i); 0] (host output, length n of the finest level) for
 * the manufactured solution u = curl psi, psi = sin^2(pi x) sin^2(pi y) (2D) or
 * psi = (g, 0, g), g = sin^2(pi x) sin^2(pi y) sin^2(pi z) (3D), with pressure
 * prod_j sin(2 pi x_j), forcing f = sigma u - nu Lap u + grad p + (a . grad) u,
 * by Gauss quadrature with k+3 points per direction per element. */
int dfmg_manufactured_rhs(const dfmg_ctx *ctx, double *F_host);

/* ---- Batches of problems on different meshes ----
 * nprob independent problems, problem p on grids[p] with pressure degree k[p],
 * nu[p], sigma[p], adv[p] (adv may be NULL).  Problems sharing (dim, n_elem,
 * n_levels, k) form a group that runs as one single-mesh batch (every launch
 * covers the group); a solve step runs the groups on their own streams,
 * forked from and joined back into the batch's stream, and with use_graph the
 * whole step is captured once as one hipGraph with a branch per group.
 * Vectors: problem p's F and U start at offset[p] of one FP64 device array of
 * offset[nprob] entries (caller order; offsets from dfmg_multi_layout).
 * Options apply to every group.  Errors: EINVAL. */
typedef struct dfmg_multi dfmg_multi;
int dfmg_multi_setup(int nprob, const dfmg_grid *grids, const int *k, const double *nu, const double *sigma,
                     const dfmg_advection *adv, const dfmg_options *opt, dfmg_multi **out);
void dfmg_multi_destroy(dfmg_multi *m);
/* offset[nprob + 1] (host, nullable) and the number of groups (nullable). */
int dfmg_multi_layout(const dfmg_multi *m, int64_t *offset, int *n_groups);
int dfmg_multi_workspace_bytes(const dfmg_multi *m, size_t *bytes);
/* As dfmg_bind, for all groups at once (one caller-owned workspace). */
int dfmg_multi_bind(dfmg_multi *m, void *dev_workspace, size_t bytes, void *hip_stream);
/* dfmg_autotune of every group. */
int dfmg_multi_autotune(dfmg_multi *m, int reps);
/* dfmg_set_learned for every problem; rho_plain_host has nprob entries in
 * caller order (nullable). */
int dfmg_multi_set_learned(dfmg_multi *m, const float *W_host, const double *rho_plain_host);
/* dfmg_set_chebyshev for every group (alpha < 0: each group's default ratio
 * for its dimension). */
int dfmg_multi_set_chebyshev(dfmg_multi *m, double alpha, int iters);
/* dfmg_set_learned_chebyshev for every group; rho_plain_host has nprob
 * entries in caller order (nullable). */
int dfmg_multi_set_learned_chebyshev(dfmg_multi *m, const float *W_host, const double *rho_plain_host, int iters);
/* Manufactured load vectors of every problem (host, offset[nprob] entries). */
int dfmg_multi_manufactured_rhs(const dfmg_multi *m, double *F_host);
/* dfmg_solve of every problem (stats: nprob entries, caller order). */
int dfmg_multi_solve(dfmg_multi *m, const double *F_dev, double *U_dev, double tol, dfmg_stats *stats);
int dfmg_multi_residual_norm(dfmg_multi *m, const double *F_dev, const double *U_dev, double *out_host);
int dfmg_multi_div_norm(dfmg_multi *m, const double *U_dev, double *out_host);

const char *dfmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DFMG_H */
