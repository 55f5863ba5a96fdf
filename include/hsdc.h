/*
 * hsdc.h -- C ABI of the MI355X (gfx950) hybrid spectral deferred correction
 * library for the monodomain equation.
 *
 * Method: de Souza, Pezzuto, Krause, "High-order parallel-in-time method for
 * the monodomain equation in cardiac electrophysiology" (arXiv 2405.19994).
 * The semi-discrete problem is y' = f_I + f_E + f_e with y = (V_m, w_a, w_g)
 * (Sec. 2.2, eqs. sd_sys, def_f_IE, def_Lambda); one HSDC step solves the
 * exponential collocation system C(y_n) = 1 (x) y_n (Sec. 3.1.2, eq. def_C) by
 * the preconditioned Picard iteration of eq. prec_picard with the IMEX /
 * exponential-Euler preconditioner of eq. def_P; PFASST couples P steps
 * (Sec. 3.2, eqs. erk_sys, def_D, def_Q, Algorithm 1).
 *
 * Cell model: ten Tusscher-Panfilov 2006 epicardial cell, 19 states per node:
 *   0 V;  1 Ca_i 2 Ca_SR 3 Ca_ss 4 Na_i 5 K_i 6 Rbar (w_a, explicit);
 *   7 m 8 h 9 j 10 xr1 11 xr2 12 xs 13 r 14 s 15 d 16 f 17 f2 18 fCass
 *   (w_g, exponential).
 * Units: ms, mV, cm, mS/cm, uF/cm^2, uA/cm^2, mM.
 *
 * Layout: a state is field-major (structure of arrays): field f of node p at
 * y[f * N + p], nodes numbered x fastest, p = ix + nx (iy + ny iz).  All
 * device arrays passed in are FP64, contiguous, and owned by the caller; the
 * library copies what it keeps.  All device work is enqueued on the caller's
 * HIP stream (hipStream_t passed as void *); calls that return host values
 * synchronise that stream.
 *
 * Errors: every call returns an hsdc_status; nothing throws across the ABI.
 * Argument checks fail with HSDC_EINVAL before any device work;
 * hsdc_last_error() gives a message.  A context is used by one host thread at
 * a time.
 */
#ifndef HSDC_H
#define HSDC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HSDC_NFIELDS 19
#define HSDC_NAUX 6
#define HSDC_NGATES 12
#define HSDC_MAX_M 8

typedef struct hsdc_ctx hsdc_ctx;

typedef enum {
  HSDC_OK = 0,
  HSDC_EINVAL = -1,     /* malformed argument; nothing was enqueued            */
  HSDC_ENOMEM = -2,     /* device allocation failed                            */
  HSDC_EDEVICE = -3,    /* a HIP runtime call failed                           */
  HSDC_ENOCONV = -4,    /* a diffusion solve missed cg_rtol within cg_maxit;   */
                        /* the state was still advanced                        */
  HSDC_ENONFINITE = -5, /* a residual or state norm is NaN or Inf              */
  HSDC_ESTATE = -6      /* call not valid in the context's mode                */
} hsdc_status;

/* Semi-discrete monodomain problem (Sec. 2.1-2.2).  Cell-centred uniform mesh,
 * node p at ((ix + 1/2) dx, ...), no-flux walls (mirror ghost).  The diffusion
 * operator is (A V)_p = sum over faces (p,q) of k_pq (V_q - V_p), with
 * k_pq = sigma_axis / dx^2, or the harmonic mean of sigma_node over the face
 * divided by dx^2 when sigma_node is given; f_I = (chi Cm)^-1 A V. */
typedef struct {
  int32_t dim;               /* 1, 2 or 3                                         */
  int32_t nx, ny, nz;        /* nodes per axis; unused axes must be 1             */
  double dx;                 /* cm                                                */
  double sigma[3];           /* mS/cm, diagonal conductivity tensor (x, y, z)     */
  const double *sigma_node;  /* device [N] per-node sigma (mS/cm) or NULL         */
  double chi;                /* surface-to-volume ratio, 1/cm                     */
  double Cm;                 /* membrane capacitance, uF/cm^2                     */
  double g_scale[3];         /* multipliers of G_Na, G_CaL, G_Kr (1 = published)  */
  const double *stim_w;      /* device [N] stimulus weight per node, or NULL      */
  double stim_amp;           /* uA/cm^2; I_stim = stim_amp * stim_w(x) while      */
  double stim_t0;            /*   stim_t0 < t <= stim_t0 + stim_dur (window open  */
  double stim_dur;           /*   on the left, closed on the right)               */
  int32_t fd_order;          /* finite differences of A: 2 (or 0) the 3/5/7-point */
                             /* stencil above; 4 the fourth-order stencil of      */
                             /* Sec. 2.2, per axis sigma_axis (-V_{p-2} + 16      */
                             /* V_{p-1} - 30 V_p + 16 V_{p+1} - V_{p+2}) /        */
                             /* (12 dx^2) with the same mirror at the walls       */
                             /* (V_{-1} = V_0, V_{-2} = V_1); uniform sigma only  */
} hsdc_problem;

/* Method (Sec. 3, Algorithm 1). */
typedef struct {
  int32_t levels;            /* 1 (serial HSDC), 2 (two-level PFASST) or 3        */
                             /* (three levels, FP64, Sec. 5.1: M = 6, 3, 1)       */
  int32_t M[3];              /* Radau IIA nodes per level, M[0] fine, 1..8        */
  int32_t space_coarsen;     /* 1, or 2: every coarser level on the mesh of the   */
                             /* finer one coarsened 2x                            */
  int32_t P;                 /* time slices per block (1 for serial HSDC)         */
  double dt;                 /* step size per slice, ms                           */
  int32_t max_iter;          /* sweeps per step (levels = 1, P = 1) or maximum    */
                             /* PFASST iterations per block                       */
  double tol;                /* PFASST stop: all ||r_n||_inf < tol ||y_n||_inf;   */
                             /* tol <= 0 runs exactly max_iter iterations         */
  int32_t burn_in;           /* 1: staggered coarse burn-in before a block, P > 1 */
  int32_t solver;            /* diffusion solves on FP64 levels: 0 conjugate      */
                             /* gradients started from a Chebyshev iterate over   */
                             /* the Gershgorin interval of I - a K (steps from    */
                             /* the warm start without inner products, the first  */
                             /* inside the node update: degree 7 on 2D meshes,    */
                             /* in one tiled launch, else 3);                     */
                             /* 1 Chebyshev iteration over that                   */
                             /* interval (no inner products: the iteration count  */
                             /* comes from the residual bound of the Chebyshev    */
                             /* polynomial, the same ||b - A x||_2 <= cg_rtol     */
                             /* ||b||_2); 2 conjugate gradients from the warm     */
                             /* start; 3 direct solve in the DCT-II eigenbasis of */
                             /* A (Sec. 5: the paper's Laplacian solves), exact   */
                             /* up to rounding, for uniform sigma and FP64 levels */
                             /* (required with fd_order 4).  An FP32 coarse level */
                             /* always runs CG from the warm start.               */
  double cg_rtol;            /* diffusion solve: ||b - A x||_2 <= cg_rtol ||b||_2 */
  int32_t cg_maxit;          /* iteration cap per diffusion solve (Chebyshev:     */
                             /* cap on the polynomial degree)                     */
  int32_t coarse_fp32;       /* levels = 2: 1 runs the coarse level's cell model  */
                             /* and stores its reaction terms, Lambda and CG work */
                             /* vectors in FP32; states, K V, right-hand sides,   */
                             /* collocation integrals, phi functions, reductions, */
                             /* tau and the fine level stay FP64, so the fixed    */
                             /* point is the FP64 fine collocation solution       */
  double coarse_cg_rtol;     /* coarse diffusion solves; <= 0: cg_rtol (FP64      */
                             /* coarse level) or 1e-5 (FP32 coarse level, where   */
                             /* it is relative to the warm start's residual)      */
  int32_t residual_norm;     /* relative residual of slice n (stop test, residual */
                             /* calls): 0 ||r_n||_inf / ||y_n||_inf over all      */
                             /* fields and nodes (Algorithm 1); 1 the largest     */
                             /* per-field ratio ||r_{n,f}||_inf / ||y_{n,f}||_inf */
                             /* (fields of very different magnitude: Ca_i is      */
                             /* about 1e-4 mM beside K_i about 136 mM)            */
  int32_t prefix_stop;       /* two levels: 0 every slice iterates until all have */
                             /* converged (Algorithm 1); 1 the slices whose       */
                             /* residual, and that of every earlier slice, is     */
                             /* below tol stop iterating (the variant Sec. 3.2    */
                             /* describes beside Algorithm 1); a stopped slice    */
                             /* keeps its fine and coarse iterates and the first  */
                             /* active slice starts from them                     */
} hsdc_method;

/* Counters since init (host copy). */
typedef struct {
  int64_t steps;             /* time steps completed (blocks x P for PFASST)      */
  int64_t sweeps;            /* sweeps on the fine level                          */
  int64_t coarse_sweeps;     /* sweeps on the coarse level (incl. burn-in)        */
  int64_t cg_solves;         /* diffusion solves                                  */
  int64_t cg_iters;          /* solver iterations over all solves (Chebyshev:    */
                             /* the degree of the residual polynomial)            */
  int64_t cg_unconverged;    /* solves that hit cg_maxit                          */
  int64_t pfasst_iters;      /* PFASST iterations                                 */
  int64_t ionic_evals;       /* node-wise cell-model evaluations (x mesh nodes)   */
  int64_t cg_redo_steps;     /* serial steps, and coarse parts of PFASST          */
                             /* iterations, recomputed because a solve run with   */
                             /* a predicted iteration budget missed its tolerance */
} hsdc_stats;

/* Create a context and its initial state (Sec. 3.1: y(0) = y_0).
 * y0: device [19][N] initial state, or NULL for the TTP06 epicardial rest state
 * on every node.  The first step (serial) or block (PFASST: spread of y0 on every
 * slice, then the burn-in when enabled and P > 1) is prepared, so sweeps and
 * iterations can be applied at once.  *out receives the context; on failure
 * *out is NULL.  hip_stream may be NULL (the null stream). */
hsdc_status hsdc_init_state(const hsdc_problem *prob, const hsdc_method *meth,
                            const double *y0, void *hip_stream, hsdc_ctx **out);

/* A batch of count independent tissues stepped together by serial hybrid SDC
 * (Sec. 3.1; every kernel launch covers every tissue).  probs[n] describes
 * tissue n; the tissues may differ only in nx, ny, nz, sigma_node and stim_w
 * (dim, dx, sigma, chi, Cm, g_scale and the stimulus timing and amplitude are
 * shared; sigma_node and stim_w are given for all tissues or for none).  meth
 * must have levels = 1 and P = 1; count is 1..4096.  y0: host array of count
 * device pointers, y0[n] device [19][N_n], or NULL (or a NULL entry) for the
 * TTP06 rest state.  The context then behaves as a serial context whose slice
 * n is tissue n: hsdc_advance steps every tissue, hsdc_sdc_sweep (slice 0)
 * sweeps every tissue, hsdc_residual returns one residual per tissue, and
 * get/set_state take the tissue as the slice (arrays of N_n nodes).  Device
 * rows are padded to the largest tissue.  Errors as hsdc_init_state, and
 * HSDC_EINVAL naming the first tissue whose shared fields differ. */
hsdc_status hsdc_init_batch(const hsdc_problem *probs, int32_t count, const hsdc_method *meth,
                            const double *const *y0, void *hip_stream, hsdc_ctx **out);

/* Launch tuning of a context (results are unchanged up to the order of the CG
 * reductions): cg_blocks caps the blocks of each CG kernel (1..1024, <= 0
 * keeps the current cap, default 512); cg_margin is the number of spare
 * launches added to a predicted CG budget (0..64, negative keeps the current
 * margin; by default none after the one-launch CG start of 2D meshes, one
 * otherwise).  A budgeted solve gets one CG launch per iteration it is
 * predicted to need plus the margin, none when its start is predicted to meet
 * cg_rtol and the margin is 0; its convergence is checked from the residual's
 * partial sums by the kernel that follows it, and a step with a missed solve
 * is recomputed.  A Chebyshev budget gets one spare launch more, since its
 * iteration count moves in steps of two.  Takes effect from the next solve;
 * call it between steps, not concurrently with work on the context. */
hsdc_status hsdc_tune(hsdc_ctx *ctx, int32_t cg_blocks, int32_t cg_margin);

/* Launch shapes of a context's FP64 levels (an FP32 coarse level keeps the
 * defaults); results are unchanged up to the order of the reductions over
 * blocks and tiles.
 *   node_block:   threads per block of the node update (the cell model and
 *                 the diffusion right-hand side, eq. def_P): 64, 128, 256
 *                 (default) or 512; 0 keeps the current size.
 *   cg_tile:      tile of the one-launch CG start on 2D meshes (solver 0):
 *                 iterates in LDS: 0: 64 x 16 nodes, 1024 threads;
 *                 1: 32 x 32, 1024; 2: 32 x 16, 512; 3: 32 x 8, 256;
 *                 4: 16 x 16, 256; iterates in registers (blocks of 64
 *                 columns, 512 threads): 5: 48 x 16; 6: 48 x 8; 7: 48 x 24;
 *                 8: 48 x 32; -1 keeps.  The default is the tallest register
 *                 tile that gives at least 192 tiles, else 48 x 8.
 *   prolong_tile: tile of the coarse-to-fine correction into the fine level
 *                 (Algorithm 1, space coarsening 2), 256 fine nodes per tile:
 *                 3D 0: 32 x 4 x 2 (default), 1: 64 x 2 x 2, 2: 16 x 8 x 2,
 *                 3: 16 x 4 x 4; 2D 0: 32 x 8 (default), 1: 64 x 4,
 *                 2: 16 x 16, 3: 128 x 2; -1 keeps.
 * HSDC_EINVAL for any other value.  Takes effect from the next launch (a
 * captured step graph is captured again); call it between steps, not
 * concurrently with work on the context. */
hsdc_status hsdc_tune_shapes(hsdc_ctx *ctx, int32_t node_block, int32_t cg_tile,
                             int32_t prolong_tile);

/* Graph replay (contexts created on a non-null stream).  Serial and batch
 * contexts: hsdc_advance then captures one whole step (max_iter
 * sweeps with their CG solves at predicted iteration budgets, y_{n+1} =
 * y_{n,M}, the start of the next step) into a HIP graph and replays it once
 * per step; the step number the kernels use is kept in device memory.  Every
 * replay's solves are still verified; a step with a solve that missed cg_rtol
 * is recomputed from the saved y_n with every solve checked, as without
 * graphs.  Budgets rise at once and are lowered every 16 steps (to the most
 * iterations used since, plus the margin); a step is captured again when they
 * change.  Two-level PFASST contexts: the coarse part of every iteration (the
 * FAS restriction, the coarse evaluations and the Q^seq chain of coarse
 * sweeps, whose solves run at predicted budgets in any case and are verified
 * once at the part's end) is captured once and replayed per iteration; a part
 * with a missed solve runs again with every solve checked; budgets are lowered
 * every 8 iterations.  The fine Q^par sweep, the coarse-grid correction and
 * the residual run as without graphs.  Results equal those without graphs.
 * Kernel timing (hsdc_profile_enable) runs without graphs.  on = 0 releases
 * the graph. */
hsdc_status hsdc_use_graph(hsdc_ctx *ctx, int32_t on);

/* Serial steps of a small 1D mesh in one launch (Sec. 3.1.3, the sweep of eq.
 * prec_picard; on by default).  A serial context on a 1D mesh of at most 256
 * nodes (second-order stencil, solver 0, 1 or 2) advances the steps of an
 * hsdc_advance call in launches of one workgroup (at most 1024 steps a
 * launch): one thread per node, the stencil products and the diffusion
 * solves through LDS, each solve direct (cyclic reduction of the tridiagonal
 * system, exact up to rounding, counted in the stats as a solve with no CG
 * iteration) instead of CG to cg_rtol.
 * The per-launch kernels of other meshes need launches of a few microseconds
 * each, about a hundred per step.  Not taken while graph replay or kernel
 * timing is on, or between the sweeps of a step (hsdc_sdc_sweep).  on = 0
 * keeps every step on the per-launch kernels.  A step that turns a state
 * non-finite ends the call with HSDC_ENONFINITE. */
hsdc_status hsdc_single_block(hsdc_ctx *ctx, int32_t on);

/* Apply nsweeps preconditioned Picard iterations (eq. prec_picard, one forward
 * substitution with P^-1 of eq. def_P each) to the stage vector of one slice of
 * the fine level.  PFASST contexts keep the slice's start value y_{n,0}; serial
 * and batch contexts take slice 0 and sweep every tissue.  level must be 0. */
hsdc_status hsdc_sdc_sweep(hsdc_ctx *ctx, int32_t level, int32_t slice, int32_t nsweeps);

/* Serial mode: nsteps times {max_iter sweeps; y_{n+1} = y_{n,M}; spread y_{n+1}}
 * (the step applies the sweeps the current step has not had yet).
 * PFASST mode: nsteps blocks, each iterated until converged or max_iter
 * (Algorithm 1), then the next block starts from y_{P-1,M}.
 * The status describes this call only: HSDC_ENONFINITE when a solve or the
 * residual met a NaN or Inf (the state is not finite; stepping stops at the
 * step where it was found), else HSDC_ENOCONV when a solve of this call
 * reached cg_maxit (the state was still advanced). */
hsdc_status hsdc_advance(hsdc_ctx *ctx, int32_t nsteps);

/* One iteration of Algorithm 1 on the current block: FAS correction tau,
 * coarse Q^seq sweep, coarse-grid correction, fine Q^par sweep, residual.
 * res_host (host [P], may be NULL) receives ||r_n||_inf / ||y_n||_inf;
 * *all_converged (may be NULL) is 1 when every slice is below tol. */
hsdc_status hsdc_pfasst_iter(hsdc_ctx *ctx, double *res_host, int32_t *all_converged);

/* Relative residual ||r_n||_inf / ||y_n||_inf of every slice of the fine level,
 * r_n = C(y_n) - 1 (x) y_{n-1,M} (rows of D(z) - b in Algorithm 1; y_{-1,M} is
 * the block start value).  res_host: host [P].  level must be 0: Algorithm 1
 * tests convergence on the fine level only, and the coarse level's equations
 * carry the FAS correction tau of the current iteration (its iterate is an
 * intermediate of one iteration, not a solution of C(y) = 1 (x) u).
 * HSDC_ENONFINITE when a residual or state norm is NaN or Inf. */
hsdc_status hsdc_residual(hsdc_ctx *ctx, int32_t level, double *res_host);

/* Copy stage `node` (0..M) of `slice` of `level` to / from device [19][N_level]. */
hsdc_status hsdc_get_state(const hsdc_ctx *ctx, int32_t level, int32_t slice, int32_t node,
                           double *dst);
hsdc_status hsdc_set_state(hsdc_ctx *ctx, int32_t level, int32_t slice, int32_t node,
                           const double *src);

/* Current global step index n of the first slice (time t_n = n dt). */
int64_t hsdc_current_step(const hsdc_ctx *ctx);
hsdc_status hsdc_get_stats(const hsdc_ctx *ctx, hsdc_stats *out);

/* Kernel timing (diagnostics).  While enabled, every kernel the context
 * launches is bracketed by HIP events on the context's stream; per kernel
 * class the launch count, the summed event time and the algorithmic HBM bytes
 * (the distinct bytes the launch must read and write, counted from the sizes)
 * are accumulated.  Enabling adds a small per-launch overhead.  Classes:
 * "node_update", "assemble", "cg_init", "cg_iter", "eval_stages", "spmv",
 * "residual", "transfer", "copy", "fas_integrals", "cheb_iter" (at most 16). */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
  double bytes;
} hsdc_kernel_profile;
hsdc_status hsdc_profile_enable(hsdc_ctx *ctx, int32_t on);
/* Copies up to max class records to out (host), *count receives the number
 * of classes with at least one launch; resets the accumulators. */
hsdc_status hsdc_profile_read(hsdc_ctx *ctx, hsdc_kernel_profile *out, int32_t max,
                              int32_t *count);

void hsdc_destroy(hsdc_ctx *ctx);
/* Message of the last failed call on ctx (or of the last failed context-free
 * call when ctx is NULL).  Never NULL. */
const char *hsdc_last_error(const hsdc_ctx *ctx);

/* ---- exported building blocks (used by the parity tests) ---------------- */

/* Node-wise TTP06 evaluation at n states y (device [19][n]): I_ion (pA/pF,
 * device [n]), h_a (device [6][n]), Lambda_g = -1/tau (device [12][n]) and
 * w_g,inf (device [12][n]) (eqs. monodomain_g_lambda, def_Lambda). */
hsdc_status hsdc_ionic_eval(int64_t n, const double *y, const double *g_scale_host3,
                            double *I_ion, double *h_a, double *lam, double *w_inf,
                            void *hip_stream);

/* phi_k(x) for k = 1..kmax (Appendix A, eq. def_phik): out device [kmax][n]. */
hsdc_status hsdc_phi(int64_t n, const double *x, int32_t kmax, double *out, void *hip_stream);

/* out = (chi Cm)^-1 A v for the operator of *prob (device [N] each), enqueued
 * on hip_stream; the call returns at once for a uniform sigma and after the
 * kernel when it built (and frees) the face coefficients of sigma_node. */
hsdc_status hsdc_apply_diffusion(const hsdc_problem *prob, const double *v, double *out,
                                 void *hip_stream);

/* Solve (I - a (chi Cm)^-1 A) x = b by CG to ||b - A x||_2 <= rtol ||b||_2;
 * x (device [N]) holds the initial guess on entry.  *iters_host receives the
 * iteration count.  Returns HSDC_ENOCONV when maxit is reached. */
hsdc_status hsdc_diffusion_solve(const hsdc_problem *prob, double a, const double *b, double *x,
                                 double rtol, int32_t maxit, int32_t *iters_host,
                                 void *hip_stream);

/* The same solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * arguments, results and errors as hsdc_diffusion_solve, but the CG vectors,
 * the face coefficients of sigma_node, the partial sums and the CG scalars
 * live in one static device array of the library (about 40 MiB, held by
 * every device the library runs on until the process ends), so the call
 * allocates nothing.  Meshes of more than HSDC_NOALLOC_MAX_NODES nodes are
 * rejected with HSDC_EINVAL before any device work.  Every call on a device
 * shares that device's array: calls that overlap on one device (other host
 * threads, or other streams) race and must be serialised by the caller. */
#define HSDC_NOALLOC_MAX_NODES 524288
hsdc_status hsdc_diffusion_solve_noalloc(const hsdc_problem *prob, double a, const double *b,
                                         double *x, double rtol, int32_t maxit,
                                         int32_t *iters_host, void *hip_stream);

/* ---- discrete adjoint of serial hybrid SDC ------------------------------ */

/* The gradient of a probe-voltage misfit through nsteps steps of serial hybrid
 * SDC (Sec. 3.1.3: K = max_iter sweeps of eq. prec_picard with the
 * preconditioner of eq. def_P, exponential collocation of eq. def_C):
 *   L = sum_{s=1..S} sum_{q} (V(probes[q], t = s sample_every dt) - targets[s-1][q])^2,
 * S = nsteps / sample_every, with respect to the per-node conductivity field
 * (problem with sigma_node), the G_Na, G_CaL, G_Kr scalings and the initial
 * state.  The gradient is the exact derivative of the discrete forward map
 * (solves taken as exact: use cg_rtol of 1e-13 or below): the forward keeps
 * y_n before every step, the backward recomputes each step from it and runs
 * the transposed sweep (the cell model's Jacobian transposed: the currents in
 * one reverse pass, the gates by dual numbers; the symmetric diffusion solves;
 * the derivatives of a_ij(z) and of phi_1 through phi_k' = phi_k - k
 * phi_{k+1}).  Its solves run at iteration budgets checked once per step (a
 * step with a missed solve is run again with every solve checked).
 * hsdc_misfit_forward: meth serial (levels = 1, P = 1) with M <= 6; probes
 * device [nprobes] distinct node indices; targets device [S][nprobes] (copied);
 * *loss_host receives L; *out an opaque handle holding the checkpoints
 * (19 N 8 bytes per step and the final state) and the context (released by
 * hsdc_adj_destroy).
 * Errors as hsdc_init_state and hsdc_advance. */
typedef struct hsdc_adj hsdc_adj;
hsdc_status hsdc_misfit_forward(const hsdc_problem *prob, const hsdc_method *meth, const double *y0,
                                int32_t nsteps, int32_t sample_every, int32_t nprobes,
                                const int64_t *probes, const double *targets, double *loss_host,
                                hsdc_adj **out, void *hip_stream);
/* dL/dsigma_node (device [N], or NULL; needs sigma_node), dL/dg_scale (host
 * [3], or NULL) and dL/dy0 (device [19][N], or NULL) of the forward run held by
 * adj.  May be called more than once.  HSDC_ENOCONV when an adjoint solve
 * reaches cg_maxit. */
hsdc_status hsdc_misfit_backward(hsdc_adj *adj, double *grad_sigma, double *grad_gscale_host,
                                 double *grad_y0);
void hsdc_adj_destroy(hsdc_adj *adj);

/* Exponential collocation coefficients a_ij(z) (eq. def_aij), computed on the
 * device as sum_k c_i^k w_j^{k-1} phi_k(c_i z) (eq. def_aij_computable) with
 * the Radau IIA nodes and Fornberg weights of the library: z device [n],
 * out device [n][M][M] (row i, column j); c_host (host [M], may be NULL)
 * receives the nodes c_1..c_M. */
hsdc_status hsdc_colloc_coefficients(int32_t M, int64_t n, const double *z, double *out,
                                     double *c_host, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* HSDC_H */
