/*
 * nkreg.h -- C ABI of the MI355X (gfx950) Gauss-Newton-Krylov registration library.
 *
 * The library solves the optimal-control formulation of diffeomorphic image
 * registration of Mang & Biros, "An inexact Newton-Krylov algorithm for
 * constrained diffeomorphic image registration" (arXiv 1408.6299):
 *
 *   minimise over v:  J[v] = 1/2 ||m_R - m_1||^2_{L2} + beta/2 sum_l <v_l, A v_l>
 *   subject to        dt m + grad m . v = 0,  m(0) = m_T,  gamma div v = 0,
 *
 * on the periodic box [0, 2 pi)^d, d in {2, 3} (objective e:objective with the
 * quadratic regulariser e:quadratic-regularization, constraint e:constraint).
 * Space is Fourier pseudospectral, time is RK2 (Heun) with h_t = 1/nt, and v
 * is expanded in time in nc Chebyshev coefficients (e:expansion).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Pointers named d_* are DEVICE pointers (hipMalloc'd memory, e.g. torch
 *   tensors) owned by the caller. The library reads them during the call (or,
 *   for asynchronous calls, before the stream reaches the call's end) and never
 *   frees or keeps them. Pointers named h_* are host pointers.
 * - Arrays are contiguous, row-major, last axis fastest, axis 0 = x1.
 *   A scalar field has n = N1*N2(*N3) values; x_j = 2 pi j / N_i.
 *   A velocity-shaped array has layout [nc][d][N1][N2](N3).
 * - Element types: scalar fields (images, m_1, the gradient / divergence
 *   building blocks) use the transport precision, float if
 *   config.precision == 32 and double if 64. Velocity-shaped arrays (velocity
 *   coefficients, gradients, Hessian products, Krylov vectors) are double in
 *   both modes: the transport solves run in the transport precision, the
 *   control space (including the spectral operators beta A, K and the
 *   preconditioner applied to it) runs in FP64.
 * - Gradients and Hessian products are the nodal values of the L2-Riesz
 *   representative: dJ[w] = h_d * sum(g * w), h_d = prod(2 pi / N_i). This is
 *   the scaling of the paper's Table t:eigenvalues.
 * - All host scalars are double. Reductions are always accumulated in FP64.
 * - Calls run on the stream given to nkreg_create. Calls returning host scalars
 *   synchronise that stream; the others are asynchronous.
 * - A handle is not thread-safe. No exception crosses the ABI.
 * - The library owns its workspace (trajectory, spectra, Krylov vectors), which
 *   it allocates in nkreg_create and frees in nkreg_destroy. The gradient, the
 *   Hessian matvec, PCG and the Newton and Picard drivers allocate nothing; the
 *   beta search, det(grad y), the Hessian assembly and Lanczos allocate their own
 *   temporaries for the duration of the call, and a batch allocates its argument
 *   tables when it (re)builds its graph.
 */
#ifndef NKREG_H
#define NKREG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NKREG_OK = 0,
  NKREG_EINVAL = -1,     /* bad argument value (beta <= 0, d not 2/3, reg not 1/2, null pointer) */
  NKREG_ESHAPE = -2,     /* grid size not a power of two in [8, 512], or sizes inconsistent */
  NKREG_ENOMEM = -3,     /* device allocation failed */
  NKREG_EHIP = -4,       /* a HIP runtime call failed */
  NKREG_ESTATE = -5,     /* call order: Hessian matvec / PCG without a prior gradient */
  NKREG_ENONFINITE = -6, /* a reduction produced NaN or Inf */
  NKREG_ECFL = -7,       /* the velocity violates the CFL bound config.cfl_max */
  NKREG_ENOCONV = -8,    /* PCG / Newton reached its iteration limit (outputs still written) */
  NKREG_ENOTIMPL = -9    /* feature not available for this configuration */
} nkreg_status;

typedef struct {
  int dim;              /* d: 2 or 3 */
  int n[3];             /* N1, N2, N3 (N3 ignored for d = 2); powers of two in [8, 512] */
  int nt;               /* RK2 time steps, h_t = 1/nt */
  int nc;               /* Chebyshev coefficients in time, 1..16 (1 = stationary) */
  int reg;              /* 1: H1 seminorm, A = -Lap;  2: H2 seminorm, A = Lap^2 */
  int incompressible;   /* gamma: 1 applies the Leray projection K to body forces */
  double beta;          /* regularisation weight, > 0 */
  int precision;        /* 32 or 64: precision of the transport solves, their FFTs and scalar fields */
  int checkpoint_every; /* 0: keep grad m^j, grad m*_j for all j (2 nt d fields); K > 0: keep m at
                           every K-th step and recompute a K-step segment inside each adjoint
                           and incremental sweep (2 K d fields; one extra state solve per sweep) */
  double cfl_max;       /* CFL bound checked by nkreg_objective_gradient; <= 0 disables */
  int trajectory_slots; /* with K > 0: K-step segments of the trajectory kept in memory (2 S K d
                           fields), 0 or 1 = one. Segment s lives in slot s % S; a sweep recomputes
                           a segment only when its slot holds another one, so a matvec recomputes
                           2 (nseg - S) segments (nseg = ceil(nt / K)) and none once S >= nseg.
                           Results do not depend on S. */
} nkreg_config;

typedef struct nkreg_problem nkreg_problem;

/* Options of the outer iteration (Algorithm a:outer-iteration). */
typedef struct {
  int max_outer;        /* relative gradient rule: at most max_outer iterations; C1-C5 rule: n_opt of
                           (C5) k > n_opt, i.e. at most max_outer + 1 iterations */
  double gtol;          /* relative gradient rule ||g_k||_inf <= gtol ||g_0||_inf; <= 0: the paper's
                           rule (C1 and C2 and C3) or C4 or C5 of e:stopping-criteria / e:converged */
  double tau_J;         /* tolerance of C1-C3 */
  int pcg_maxit;        /* cap on PCG iterations per Newton step; <= 0: n (system size) */
  int cfl_guard;        /* 1: halve the step until h_t max|v^i|/h_x^i <= cfl_max before the line search */
  int verbose;          /* 1: print one line per outer iteration to stderr */
  double gref_inf;      /* > 0: ||g_0||_inf of the relative gradient rule (continuation passes the
                           first level's value); <= 0: the gradient at the solve's starting point */
  double* h_history;    /* optional host array of history_cap rows of NKREG_HISTORY_COLS doubles, one
                           row per iterate v_k from k = 0: k, J, J_dist, J_reg, ||g_k||_inf, PCG
                           iterations of the step that produced v_k, its step length alpha, PDE
                           solves so far (n_PDE), the CFL number of v_k, min and max of det F_1 at
                           v_k (NaN unless history_detf). Rows past history_cap are dropped.
                           nkreg_continuation appends every level's rows; nkreg_beta_search
                           ignores it. NULL: no history */
  int history_cap;
  int history_detf;     /* 1: also solve for det F_1 at every iterate (one FP64 deformation-gradient
                           solve per row, e:def-grad as nkreg_det_grad_y); with verbose, the line
                           printed per iteration carries the CFL number and, with this, det F_1 */
} nkreg_solve_opts;

#define NKREG_HISTORY_COLS 11

/* What the outer iteration did (quantities of interest, Table t:quantities-of-interest). */
typedef struct {
  int iterations;       /* outer iterations k* */
  int cg_iterations;    /* total PCG iterations (= Hessian matvecs) */
  int n_pde;            /* hyperbolic PDE solves: 2 per gradient, 2 per matvec, 1 per line-search trial */
  int line_search_failed;
  int converged;
  double J0, J;         /* objective at v = v0 and at the end */
  double J_dist, J_reg; /* data term and regulariser at the end */
  double gnorm0_inf, gnorm_inf;
  double seconds;       /* wall-clock of the whole solve */
  int stop_reason;      /* 1 relative gradient rule, 2 (C1 and C2 and C3), 3 C4, 4 iteration limit
                           (relative rule: max_outer iterations; C1-C5 rule: C5, k > max_outer),
                           5 line search failed, 6 objective stagnation (Picard) */
  int history_rows;     /* rows this solve wrote to opts.h_history */
} nkreg_solve_report;

/* Library version string, e.g. "nkreg 1.0 gfx950". */
const char* nkreg_version(void);
/* Human-readable text of a status code. */
const char* nkreg_status_string(int status);
/* Text of the last error on this thread (HIP error names etc.). */
const char* nkreg_last_error(void);

/* Create a problem handle on a HIP stream (NULL = the null stream). Allocates
 * the workspace. Errors: EINVAL, ESHAPE, ENOMEM, EHIP. */
int nkreg_create(const nkreg_config* cfg, void* hip_stream, nkreg_problem** out);
/* Free the handle and its workspace. NULL is accepted. */
int nkreg_destroy(nkreg_problem* p);
/* Change beta (continuation; Section "Parameter Selection"). Keeps the cached state. */
int nkreg_set_beta(nkreg_problem* p, double beta);

/* Hessian used by nkreg_hessian_matvec, nkreg_pcg and nkreg_newton_solve:
 * mode 0 = Gauss-Newton (e:gauss-newton, the default), 1 = full Newton
 * (e:second-order-opt-cond: the incremental adjoint keeps -div(v~ lam) and the
 * incremental body force keeps lam grad m~). Full Newton keeps lam^{j+1},
 * lam*_j of every gradient evaluation and grad m~ of every matvec (2 nt + 2 nt d
 * fields, also when the state trajectory is checkpointed). Switching modes
 * invalidates the cached state (a new gradient is needed before a matvec). The
 * full-Newton Hessian can be indefinite away from a minimiser: PCG stops at
 * non-positive curvature and, if that happens in its first iteration, returns
 * the preconditioned right-hand side P^-1 rhs (a descent direction). */
int nkreg_set_hessian(nkreg_problem* p, int mode);

/* Hessian matvecs are captured into a HIP graph per (input, output) pointer
 * pair and replayed (the default), and so is the PCG step of a batch item in
 * nkreg_batch_pcg (per solution vector); enable = 0 launches every kernel eagerly.
 * All work runs on the caller's stream; graphs are captured on a stream of the
 * handle's own (capture is not possible on the null stream) and replayed on the
 * caller's. */
int nkreg_use_graphs(nkreg_problem* p, int enable);

/* Writes a JSON object describing the handle's launch configuration (transport
 * precision, graph use, elements per lane of the row and column transforms, whether
 * the control-space multiplier runs fused with its column transforms, and the
 * autotuner's timings, which it records at the first graph capture) into
 * buf (len bytes, NUL-terminated, truncated if needed). */
int nkreg_describe(nkreg_problem* p, char* buf, int len);

/* Copy the template m_T and reference m_R (each n values) into the handle. Both are
 * stored with the template's mean c subtracted: a constant is transported exactly
 * and J, g and H depend only on differences and gradients of the images, so the
 * shift changes nothing but the round-off of the transforms (which scales with a
 * field's norm, mean included); nkreg_forward adds c back to m_1. Synchronises.
 * Errors: ENONFINITE (m_T not finite). */
int nkreg_set_images(nkreg_problem* p, const void* d_mT, const void* d_mR);

/* State equation e:first-order-forward: Heun from m(0) = m_T under velocity
 * coefficients d_v; writes m_1 (n values) to d_m1 (may be NULL) and caches the
 * trajectory (grad m^j and grad m*_j) for later adjoint / Hessian calls. */
int nkreg_forward(nkreg_problem* p, const void* d_v, void* d_m1);

/* Objective and reduced gradient at d_v: forward solve, adjoint solve
 * (e:first-order-adjoint, lambda(1) = m_R - m_1) and
 * g = beta A v + K[f] (e:eliminated-control; K only if incompressible), f the
 * time-integrated body force lambda grad m. Writes g to d_g (nc*d*n values,
 * may be NULL) and J, J_dist, J_reg to host doubles (may be NULL). Caches the
 * state for nkreg_hessian_matvec / nkreg_pcg. Synchronises.
 * Errors: ECFL (velocity above cfl_max), ENONFINITE. */
int nkreg_objective_gradient(nkreg_problem* p, const void* d_v, double* h_J, double* h_J_dist,
                             double* h_J_reg, void* d_g);

/* Objective only (one forward solve); does not touch the cached state. Synchronises. */
int nkreg_objective(nkreg_problem* p, const void* d_v, double* h_J, double* h_J_dist,
                    double* h_J_reg);

/* Gauss-Newton reduced Hessian matvec at the cached state (Algorithm
 * a:hessian-matvec with the GN approximation e:gauss-newton, eliminated form
 * e:eliminated-icontrol): incremental state forward, incremental adjoint
 * backward, H vt = beta A vt + K[f~]. d_vt and d_Hvt hold nc*d*n values and may
 * not alias. Errors: ESTATE if no gradient has been computed since create or
 * the last set_images. Asynchronous. */
int nkreg_hessian_matvec(nkreg_problem* p, const void* d_vt, void* d_Hvt);

/* Spectral preconditioner (beta A)^-1 with the zero mode unscaled (Section
 * "Inversion: Regularization Operators"). Asynchronous. */
int nkreg_precond_apply(nkreg_problem* p, const void* d_r, void* d_z);

/* Apply the Leray projection K (e:eliminated-control) to nc*d*n values. Asynchronous. */
int nkreg_project(nkreg_problem* p, const void* d_f, void* d_out);

/* PCG on H s = rhs at the cached state, x0 = 0, stop when
 * ||r||_2 <= rtol ||rhs||_2 (e:termination-criterion-ksm), at most maxit
 * iterations (<= 0: n). Writes s, the iteration count and ||r||/||rhs||.
 * Returns ENOCONV (with s written) if maxit is reached. Synchronises. */
int nkreg_pcg(nkreg_problem* p, const void* d_rhs, void* d_s, double rtol, int maxit,
              int* h_iters, double* h_relres);

/* Deformation gradient e:def-grad under d_v, computed in FP64 whatever the
 * problem precision; writes det F_1 (n doubles) to d_detF (may be NULL) and
 * (min, max, mean, population std) to h_stats[4]. Synchronises. */
int nkreg_det_grad_y(nkreg_problem* p, const void* d_v, void* d_detF, double* h_stats);

/* Gauss-Newton-Krylov outer iteration (Algorithm a:outer-iteration) from the
 * velocity in d_v (overwritten with the solution). Synchronises. */
int nkreg_newton_solve(nkreg_problem* p, void* d_v, const nkreg_solve_opts* opts,
                       nkreg_solve_report* report);

/* Beta continuation (Section "Parameter Selection"): Newton solves at each
 * beta of h_betas[0..levels) in turn, each warm-started from the previous
 * level's solution in d_v (overwritten with the last level's). The relative
 * gradient rule of every level uses opts->gref_inf if positive, else the first
 * level's ||g_0||_inf (a warm-started level's own g_0 is already small).
 * h_reports receives one report per level. The handle keeps the last beta.
 * Returns ENOCONV if a level did not converge. Synchronises. */
int nkreg_continuation(nkreg_problem* p, void* d_v, const double* h_betas, int levels,
                       const nkreg_solve_opts* opts, nkreg_solve_report* h_reports);

/* Parameter continuation in beta with a lower bound eps_F on det F_1
 * (Section "Parameter Selection", Table t:para-cont). Solves at beta_start
 * and divides beta by ten while min det F_1 >= eps_F; after the first beta
 * that breaks the bound, bisects (arithmetic midpoint) between the last
 * accepted and the breaching beta until half the bracket is below dbeta_rel
 * times the first breaching beta. The descent also stops below beta_min or
 * when ||m_R - m_1|| changes by less than l2_rel_min (relative) between two
 * accepted betas. Every trial is warm-started from the last accepted solution
 * (the first from d_v); the solves use opts->solve, whose gref_inf <= 0 means
 * the first solve's ||g_0||_inf. On return d_v holds the solution at beta*,
 * the smallest accepted beta, and the handle's beta is beta*. Returns ENOCONV
 * if the bound is broken already at beta_start (d_v then holds that solve).
 * Synchronises. */
#define NKREG_MAX_BETA_TRIALS 64
typedef struct {
  double eps_F;         /* lower bound on min det F_1, in (0, 1) */
  double beta_start;    /* first beta; <= 0: 1 */
  double beta_min;      /* lower bound on beta; <= 0: 1e-6 */
  double dbeta_rel;     /* bisection tolerance relative to the first breaching beta; <= 0: 0.05 */
  double l2_rel_min;    /* stagnation bound on the relative change of ||m_R - m_1||; <= 0: 1e-2 */
  int max_steps;        /* Newton solves at most; <= 0 or > NKREG_MAX_BETA_TRIALS: the maximum */
  nkreg_solve_opts solve;
} nkreg_beta_search_opts;

typedef struct {
  int steps;            /* Newton solves (trials) */
  int breached;         /* 1 if some trial broke the bound */
  int reason;           /* 1 bisection converged, 2 L2 distance stagnates, 3 lower bound on beta,
                           4 step limit, 5 bound broken at beta_start */
  double beta_star, min_det_star, l2_rel_star;  /* l2_rel = ||m_R - m_1|| / ||m_R - m_T|| */
  double dbeta_min;     /* dbeta_rel x first breaching beta (0 without a breach) */
  int newton_iterations, cg_iterations;
  double seconds;
  double trial_beta[NKREG_MAX_BETA_TRIALS], trial_min_det[NKREG_MAX_BETA_TRIALS],
      trial_l2_rel[NKREG_MAX_BETA_TRIALS];
  int trial_accepted[NKREG_MAX_BETA_TRIALS];
} nkreg_beta_search_report;
int nkreg_beta_search(nkreg_problem* p, void* d_v, const nkreg_beta_search_opts* opts,
                      nkreg_beta_search_report* report);

/* Globalised Picard iteration (Section "Picard Method", e:picard): the Picard
 * iterate -(beta A)^-1 [gamma grad p + f] minus the current iterate gives the
 * direction s_k = -P^-1 g_k (a preconditioned gradient descent); it is scaled by
 * the step memory alpha~ (memory = 1: alpha~ starts at 1, shrinks by alpha
 * after a backtracking line search and doubles after alpha = 1) and enters the
 * Armijo line search from alpha = 1. Stops on the relative gradient rule of
 * opts (gtol > 0 required; opts->gref_inf as for Newton), after opts->max_outer
 * iterations, or when J changed by at most stagnation_tol (1 + J_0) in each of
 * stagnation_count consecutive iterations (<= 0: never). The report's
 * cg_iterations is 0. popts may be NULL (memory on, 10 iterations, 1e-6).
 * Returns ENOCONV without convergence. Synchronises. */
typedef struct {
  int memory;
  int stagnation_count;
  double stagnation_tol;
} nkreg_picard_opts;
int nkreg_picard_solve(nkreg_problem* p, void* d_v, const nkreg_solve_opts* opts, const nkreg_picard_opts* popts,
                       nkreg_solve_report* report);

/* Hessian analysis at the cached state (Section "Spectral Analysis", Table
 * t:eigenvalues). nkreg_hessian_assemble writes the n x n matrix (n = nc*d*prod N_i,
 * doubles, row j = H e_j; H is symmetric unless the Leray projection is on) by n
 * matvecs with the current Hessian mode. It runs them G at a time (G <= 32, fewer
 * on large grids) as one captured batch group of the handle and G - 1 temporary
 * clones (same configuration, images, velocity and mode; their matvecs are
 * bit-identical to the handle's), so it allocates G - 1 handles' workspace and
 * 2 G n doubles while it runs. nkreg_hessian_lanczos runs up to `steps` (1..512) Lanczos steps on H with
 * full reorthogonalisation from a fixed pseudo-random start and writes the Ritz
 * values in ascending order to h_ritz (capacity >= steps) and their number to
 * h_count; the extreme Ritz values estimate H's extreme eigenvalues and condition
 * number (Section "Parameter Selection", Regularization). Synchronise. */
int nkreg_hessian_assemble(nkreg_problem* p, void* d_H);
int nkreg_hessian_lanczos(nkreg_problem* p, int steps, double* h_ritz, int* h_count);

/* Building blocks exposed for testing the spectral machinery. */
/* d_g (d*n) = spectral gradient of the scalar field d_u (n). */
int nkreg_gradient(nkreg_problem* p, const void* d_u, void* d_g);
/* d_s (n) = spectral divergence of the vector field d_w (d*n). */
int nkreg_divergence(nkreg_problem* p, const void* d_w, void* d_s);
/* d_out = A d_x (nc*d*n values, A = -Lap or Lap^2 per component). */
int nkreg_apply_reg(nkreg_problem* p, const void* d_x, void* d_out);

/* nkreg_gradient without a handle and without any device allocation, for callers
 * that cannot allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). d_g (dim * n values) = spectral gradient of the scalar field
 * d_u (n values) on the grid dim, n[0..dim) (powers of two in [8, 512]) in the given
 * precision (32: float, 64: double), on hip_stream (NULL = the null stream); the
 * result is the same bits as nkreg_gradient's. The row spectra and twiddles live in a
 * fixed device array of the library, 8 MiB + 16 KiB on each GPU that runs the call
 * (held until the process ends): the grid's 2 (d = 2) or 3 (d = 3) spectra of
 * n * sizeof(element) bytes must fit in 8 MiB (every 2D grid; 3D up to 64^3 in FP64),
 * else ESHAPE. Every call on one GPU uses that GPU's one array, so calls that overlap
 * on one GPU (concurrent streams or threads) race; calls ordered on a stream do not.
 * Asynchronous. Errors: EINVAL, ESHAPE, EHIP. */
int nkreg_gradient_noalloc(int dim, const int* n, int precision, const void* d_u, void* d_g, void* hip_stream);

/* Exchange canary of the register FFTs (test instrumentation, Section "Numerical
 * Discretization" transforms): count complex sequences of length m (interleaved re, im
 * in the given precision, m contiguous values each) transformed forward then inverse
 * (unnormalised, so out = m * in up to rounding) with the library's wavefront FFT at
 * `elems` complex values per lane, `lockstep` sequences per lane group (1, or 2 as the
 * row stages transform several sequences together). poison != 0 overwrites the LDS
 * scratch with NaN around every exchange: if a wavefront's exchange read were served
 * before its earlier writes, or a later write overtook a read, NaN would reach d_out;
 * with correct ordering the output equals the unpoisoned run's bit for bit. Forms:
 * (m, elems, lockstep) in {32, 128, 256} x {4} x {1, 2}, {64, 128} x {2} x {1, 2} and
 * {64, 256, 512} x {8} x {1}; others return ENOTIMPL. Allocates and frees a twiddle
 * table. Synchronises. */
int nkreg_exchange_canary(int precision, int m, int elems, int lockstep, int poison, const void* d_in, void* d_out,
                          int count, void* hip_stream);

/* Latency floor of a chain of dependent launches (measurement instrumentation for the
 * launch-bound grids): *h_us_per_node receives the microseconds per node of a HIP graph of
 * `nodes` launches replayed on hip_stream, each reading the FP32 complex rows x cols array
 * the previous one wrote (two arrays allocated and freed here). kind 0: an empty kernel;
 * 1: a row-pattern copy (one wavefront per row, contiguous); 2: a column-pattern copy (one
 * wavefront per column, rows/64 elements per lane, the column pass's workgroup order);
 * 3: row and column copies alternating, as the transport stages and column passes of a
 * matvec do. rows and cols are multiples of 64 in [64, 4096], nodes in [2, 4096]; EINVAL
 * otherwise. Synchronises. */
int nkreg_launch_floor(int kind, int rows, int cols, int nodes, void* hip_stream, double* h_us_per_node);

/* FP64 inner product sum(a*b) of two double arrays of cnt elements. Synchronises. */
int nkreg_dot(nkreg_problem* p, const void* d_a, const void* d_b, long long cnt, double* h_out);

/* Launch timing of one kernel of the library. nkreg_timer_arm selects a kernel
 * (row stages: 0 state stage 1, 1 state stage 2, 2 incremental stage 1,
 * 3 incremental stage 2, 4 adjoint start, 5 adjoint stage 1, 6 adjoint stage 2,
 * 7 R2C, 8 C2R, 9 gradient, 10 divergence; column passes: 20 forward, 21 inverse,
 * 22 derivative) and times each of its next `capacity` launches with a pair of
 * HIP events that the dispatch itself stamps (hipExtLaunchKernelGGL on the
 * caller's stream). nkreg_timer_read synchronises, returns the
 * number of recorded launches, their average duration in milliseconds and the
 * average algorithmic bytes per launch (fields read plus fields written), and
 * disarms the timer. While the timer is armed, Hessian matvecs launch eagerly
 * instead of replaying their HIP graph (graph-recorded events cannot be timed). */
int nkreg_timer_arm(nkreg_problem* p, int kernel_id, int capacity);
/* One Hessian matvec (eager launches) that adds up the algorithmic bytes of all
 * its launches (fields each kernel reads plus fields it writes); divided by a
 * matvec's duration it gives the whole matvec's achieved bandwidth. Synchronises. */
int nkreg_matvec_bytes(nkreg_problem* p, const void* d_vt, void* d_Hvt, double* h_bytes, int* h_launches);
int nkreg_timer_read(nkreg_problem* p, int* launches, double* avg_ms, double* bytes_per_launch);

/* Batches of independent problems of uneven sizes (the batched form of the path:
 * many image pairs, each its own problem of Algorithm a:outer-iteration).
 *
 * nkreg_batch_create makes count problem handles from cfgs[0..count) on one HIP
 * stream (NULL = the null stream), owned by the batch and destroyed with it;
 * nkreg_batch_item returns item i's handle, through which the caller sets its
 * images (nkreg_set_images) and runs any single-problem call. nkreg_batch_wrap
 * makes a batch over existing handles instead (the batch does not own them; they
 * may live on different streams).
 *
 * Batched calls apply one operation to every item as a single HIP-graph launch:
 * - nkreg_batch_objective_gradient: each item's objective and reduced gradient at
 *   d_v[i], exactly as nkreg_objective_gradient (forward sweep keeping the
 *   trajectory, adjoint sweep, g = beta A v + K[f]); g[i] receives the gradient
 *   (g or g[i] NULL: not written), and J, J_dist, J_reg (host arrays of count
 *   doubles, each may be NULL) the objective terms. Each item's CFL bound is
 *   checked first (ECFL). Leaves every item's state ready for Hessian matvecs.
 *   Synchronises.
 * - nkreg_batch_set_state: the same without outputs (each item's forward and
 *   adjoint sweeps at d_v[i]). Synchronises.
 * - nkreg_batch_hessian_matvec: H_i vt_i for every item at its cached state
 *   (ESTATE if an item has none). Asynchronous.
 * Items with the same grid, time steps, scheme and precision form a group: each
 * kernel of the operation runs once for the whole group, reading every item's
 * pointers and scalars (beta included) from a device table, and groups run as
 * independent graph branches. Results are bit-identical to the items' own calls.
 * The graph of each operation and its tables are built on the first call and
 * replayed while the pointer sets and the items' configurations are unchanged.
 * When all items live on one stream the graph replays on it; otherwise on a
 * stream of the batch that waits for every item's stream, and every item's stream
 * waits for the batch. Where the LDS-tiled column pass applies, each group times it
 * against the per-column pass at the group's scale and keeps the faster (both give
 * the same values); groups of small square 2D grids time the persistent small-grid
 * sweep kernel against the launches the same way. nkreg_batch_groups reports the
 * last built matvec graph: the number of groups and, for up to cap groups, their
 * sizes and forms (0 = per-column launches, 1 = tiled column launches, 2 = the
 * persistent small-grid kernel; sizes, form may be NULL). Errors: EINVAL, ESHAPE (a
 * configuration), ENOMEM, EHIP, ESTATE, ECFL, ENONFINITE. */
typedef struct nkreg_batch nkreg_batch;
int nkreg_batch_create(int count, const nkreg_config* cfgs, void* hip_stream, nkreg_batch** out);
int nkreg_batch_wrap(int count, nkreg_problem* const* items, nkreg_batch** out);
int nkreg_batch_item(nkreg_batch* b, int i, nkreg_problem** out);
int nkreg_batch_objective_gradient(nkreg_batch* b, const void* const* d_v, double* h_J, double* h_J_dist,
                                   double* h_J_reg, void* const* d_g);
int nkreg_batch_set_state(nkreg_batch* b, const void* const* d_v);
/* PCG on every item (e:termination-criterion-ksm, as nkreg_pcg: x0 = 0, stop when
 * ||r_i||_2 <= rtol ||rhs_i||_2, at most maxit iterations, <= 0: n) at each item's cached
 * state (ESTATE if an item has none). The items iterate in lockstep: each iteration is
 * one batched matvec graph launch for all items, then every unfinished item's own vector
 * work (its step replayed as a graph while graphs are in use) on one of up to eight
 * streams that the batch owns (ordered after the matvec and after the items' streams,
 * which wait for it in turn), then one wait. Each item's x_i, iteration count and relative residual equal those
 * of its own nkreg_pcg bit for bit. iters and relres (count entries each) may be NULL.
 * Returns ENOCONV (outputs written) if any item reached maxit. Synchronises. */
int nkreg_batch_pcg(nkreg_batch* b, const void* const* d_rhs, void* const* d_x, double rtol, int maxit, int* h_iters,
                    double* h_relres);
int nkreg_batch_hessian_matvec(nkreg_batch* b, const void* const* d_vt, void* const* d_Hvt);
int nkreg_batch_groups(nkreg_batch* b, int* groups, int* sizes, int* form, int cap);
int nkreg_batch_destroy(nkreg_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* NKREG_H */
