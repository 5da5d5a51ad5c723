/*
 * pitmg.h -- parallel-in-time multigrid preconditioned FGMRES for the lifted,
 * time-major augmented system of an optimal-control problem, on gfx950.
 *
 * Method: arXiv 2405.04808 (Vuchkov, Cyr, Javeed, Ridzal).
 *   - augmented system A = [[I, B^T], [B, 0]] with B = dF~ (eq. (augsys),
 *     Sec. 5.1), lifted with virtual interface variables v and multipliers
 *     mu (Fig. 4), permuted to time-major block-tridiagonal form A~ = P A Q^T
 *     (Fig. 5, eq. (augsysp));
 *   - preconditioner: one multigrid V-cycle (Alg. 1, recursed) with weighted
 *     block Jacobi smoothing (eq. (jacobi) with the correction scaled by
 *     omega), injection / linear interpolation in time and averaging /
 *     piecewise-constant transfer of the control (Sec. 5.3.1, the
 *     interface multiplier scaled by mu_scale), and GMRES right-
 *     preconditioned by symmetric block Gauss-Seidel on the coarsest grid,
 *     to a relative tolerance (Sec. 5.3.4);
 *   - outer solver: flexible GMRES (Saad 1993), needed because the coarse
 *     GMRES makes the preconditioner nonlinear (Sec. 5.3.4, Sec. 6).
 *
 * Vectors.  Every vector crossing this interface is a DEVICE pointer to FP64
 * data in type-major order (Fig. 4):
 *     x = [ u_1..u_n | v_1..v_n | z_1..z_n | lambda_1..lambda_n | mu_1..mu_n ]
 * with u_k, v_k, lambda_k, mu_k of length p and z_k of length q, so the
 * length is (4p+q) n.  The library permutes to the time-major blocks of
 * Fig. 5 internally; callers never see the permutation.
 *
 * Blocks.  For level l (n_l = n / c^l steps, l = 0 finest, c the option
 * coarsen, 2 by default) the caller gives
 * the Jacobian blocks of the lifted constraint (Sec. 4.1 eq. (blocks) with
 * the substitutions of Sec. 5.1), row-major FP64:
 *     N[l]: n_l blocks p x p  (N_k)
 *     V[l]: n_l blocks p x p  (V_k; the block of step 1 is never read,
 *                              since v_0 := 0)
 *     Z[l]: n_l blocks p x q  (Z~_k)
 * Block k of level l starts at X[l] + k * X_stride.  A stride of 0 means one
 * block shared by every step (the natural form of V and Z~ for theta = 1).
 * Coarse levels are rediscretisations at step c^l dt (geometric multigrid,
 * Sec. 5.3): the caller supplies them.
 *
 * Streams and ownership.  All device work of a handle is ordered on the HIP
 * stream given at setup (0 = the null stream).  Setup copies host blocks
 * into library memory (blocks_on_device = 0) or borrows device blocks
 * (blocks_on_device = 1: the caller keeps them alive and unchanged until
 * pitmg_refactor or pitmg_destroy).  The handle owns the factors and all
 * work buffers.  Vector arguments are caller-owned.  Entry points that
 * return results to the host synchronise the stream before returning.
 *
 * Errors.  Every call returns a pitmg_status.  A negative value is an error
 * and leaves output vectors unspecified; PITMG_NOT_CONVERGED (1) from the
 * solver leaves the last iterate in x.  pitmg_last_error() gives a message.
 * Argument checks run on the host before any device work.
 */
#ifndef PITMG_H
#define PITMG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pitmg_handle pitmg_handle;

typedef enum {
  PITMG_OK = 0,
  PITMG_NOT_CONVERGED = 1,     /* maxit reached; x holds the last iterate      */
  PITMG_ERR_INVALID = -1,      /* bad argument (sizes, null pointer, level)    */
  PITMG_ERR_SINGULAR = -2,     /* a block S_k = N_k N_k^T + Z~_k Z~_k^T is not
                                  positive definite: the time-step block of
                                  D is singular (Thm. 1's hypothesis fails);
                                  see pitmg_failed_block                       */
  PITMG_ERR_NONFINITE = -3,    /* right-hand side or residual not finite       */
  PITMG_ERR_HIP = -4,          /* HIP runtime error                            */
  PITMG_ERR_OOM = -5,          /* device allocation failed                     */
  PITMG_ERR_UNSUPPORTED = -6   /* sizes beyond what this build handles         */
} pitmg_status;

typedef struct {
  int p;                       /* states per step                              */
  int q;                       /* controls per step                            */
  int n;                       /* steps on the finest grid                     */
  int n_levels;                /* grids l = 0..n_levels-1; n % c^(n_levels-1)
                                  must be 0 (c = options.coarsen, 2 by
                                  default: Sec. 5.3.1)                         */
  const double* const* N;      /* n_levels pointers                            */
  const double* const* V;
  const double* const* Z;
  long long N_stride;          /* p*p (or 0: shared)                           */
  long long V_stride;          /* p*p or 0                                     */
  long long Z_stride;          /* p*q or 0                                     */
  int blocks_on_device;        /* 0: host pointers (copied); 1: device (borrowed) */
} pitmg_problem;

typedef struct {
  int nu_pre;                  /* block Jacobi sweeps before the coarse solve  */
  int nu_post;                 /* and after it                                 */
  double coarse_tol;           /* relative tolerance of the coarse GMRES       */
  int coarse_maxit;            /* coarse GMRES step limit (no restart)         */
  int coarse_fixed_its;        /* >0: exactly this many coarse steps, no
                                  tolerance test (deterministic cycle)         */
  int restart;                 /* FGMRES restart length                        */
  int maxit;                   /* FGMRES total step limit                      */
  int transfer_variant;        /* 0: transfers as printed (coarse step k <->
                                  fine step 2k-1, last even fine step copies the
                                  last coarse value); 1: time-aligned
                                  (coarse k <-> fine 2k)                        */
  int smoother_fp32;           /* k > 0: the k finest levels (all levels above
                                  the coarsest when k >= n_levels-1) factor and
                                  smooth in FP32 from FP32 copies of N, V, Z~;
                                  the finest-level residual, the coarse solve,
                                  FGMRES and Arnoldi stay FP64.  0: all FP64.
                                  Fixed at setup.                               */
  int coarse_mode;             /* 0: GMRES + SGS on the coarsest grid; 1: the
                                  attached network (pitmg_coarse_net_attach)
                                  replaces it until the stall rule falls back
                                  to GMRES + SGS for the rest of the solve      */
  double stall_ratio;          /* stall rule: FGMRES residual-estimate ratio
                                  est_j / est_{j-1} above this ...             */
  int stall_steps;             /* ... on this many consecutive steps           */
  int vcycle_graph;            /* 1: inside FGMRES and pitmg_vcycle, replay the
                                  finest-level V-cycle from a captured HIP
                                  graph (captured on first use, again when the
                                  coarse solve needs more steps than captured).
                                  Needs a stream other than the null stream and
                                  nu_post > 0; not used while profiling,
                                  recording coarse pairs or with coarse_mode 1 */
  int apply_from_sweep;        /* 1: when the preconditioner's last step was an
                                  FP64 block Jacobi sweep z = D^{-1}(b - (L+L^T)
                                  y) on the finest level (nu_post >= 2), FGMRES
                                  forms A~ z as b - (L+L^T)(y - z), equal in
                                  exact arithmetic and free of block reads;
                                  likewise the coarse GMRES forms A~ z of an
                                  SGS result z = a + d (forward sweep a,
                                  backward correction d) as v + L d;
                                  0: always the explicit product             */
  int pair_sweeps;             /* 1: run two consecutive sweeps of a level in
                                  one launch where the level sweeps with the
                                  register-tiled kernels (p = q in {64, 128}:
                                  the one-step kernel, and in FP64 the kernel
                                  for V, Z~ shared by every step).  The
                                  permuted system of Sec. 5.2 is block
                                  tridiagonal, so a block Jacobi sweep of
                                  Sec. 5.3.2 couples block k only to k-1 and
                                  k+1: a work-group takes the second sweep's
                                  couplings from its own first sweep and, at
                                  its edges, from its neighbours'.  The
                                  one-step kernel also keeps N_k and G_k^{-1}
                                  in registers for both sweeps.  Results are
                                  bitwise those of two launches.  Each
                                  neighbour wait is bounded (2 s); one that
                                  runs out marks the handle, and the FGMRES
                                  solve that contains it returns
                                  PITMG_ERR_HIP.  Streams under capture get
                                  one sweep per launch.
                                  2: as 1, and where every level above the
                                  coarsest sweeps with the one-step kernel
                                  (V-cycle, nu 2/2, step ratio 2, block
                                  Jacobi), the pre-smoothing of all those
                                  levels is one launch and their
                                  post-smoothing another: a block of level
                                  l + 1 starts as soon as the blocks of level
                                  l it reads have finished (dataflow flags,
                                  bounded waits as above), so the levels
                                  overlap.  Results are bitwise those of 1.
                                  0: one sweep per launch.                     */
  double omega;                /* weight of the block Jacobi correction on every
                                  level above the coarsest:
                                  y <- y + omega D^{-1}(b - A~ y).  1 is the
                                  undamped sweep printed in eq. (jacobi).  A~
                                  is block tridiagonal (Fig. 5), so the
                                  undamped iteration matrix has a spectrum
                                  symmetric about 0 and leaves the oscillating
                                  twin of every slow smooth error mode as slow
                                  as the mode itself; omega = 1/2 damps those
                                  twins by at least 1/2 per sweep and leaves the
                                  smooth modes to the coarse grid.  (0, 1].   */
  double mu_scale;             /* scale of the interface multiplier mu in the
                                  transfers of Sec. 5.3.1 (which admit
                                  alternatives): interpolation multiplies the
                                  coarse mu by it, restriction weights the mu
                                  residual rows by it.  mu is 1/dt times a
                                  lambda-sized function (the u_k row balances
                                  N_k^T lambda_k + mu_k with N_k ~ M/dt), so
                                  the step ratio 2 keeps its grid functions
                                  consistent; 1 is the printed, unscaled
                                  transfer.  > 0.                             */
  int cycle;                   /* 0: V-cycle (Alg. 1 recursed).  1: W, 2: F
                                  (the variants Sec. 6 reports trying): every
                                  level above the coarsest makes a second
                                  coarse correction from the coarse residual
                                  the first leaves, W recursing with W in
                                  both, F with F then V.                      */
  int smoother;                /* smoothing sweep y <- y + omega M^{-1}(b - A~ y)
                                  with the splittings of Sec. 5.3.4: 0 block
                                  Jacobi (M = D), 1 forward block Gauss-
                                  Seidel (M = D + L), 2 backward (D + L^T),
                                  3 symmetric ((D + L) D^{-1} (D + L^T)).
                                  Gauss-Seidel sweeps are sequential in time
                                  (a chain of n dependent p x p products per
                                  sweep) and run in FP64 (smoother_fp32 must
                                  be 0).  Fixed at setup.                     */
  int unlifted;                /* 1: the handle also solves the augmented system
                                  without virtual variables (Fig. 2, B = dF;
                                  pitmg_unlifted_*).  Its hierarchy is then the
                                  lifted system of the blocks sqrt2 N_k,
                                  sqrt2 V_k, Z~_k (scaled on the device into
                                  the handle's own copies), whose exact solve
                                  read through the lift / project maps is the
                                  unlifted inverse; the lifted entry points
                                  act on that scaled system.  Fixed at
                                  setup.  0: the lifted system only.          */
  int coarsen;                 /* step ratio between consecutive levels: 2 (the
                                  coarsening of Sec. 5.3), or 4, 8, 16 (the
                                  larger factors Sec. 6 reports trying).  Level
                                  l has n / coarsen^l steps, so n must be
                                  divisible by coarsen^(n_levels-1), and the
                                  caller's blocks are rediscretisations at
                                  those steps.  For c != 2: injection of the
                                  first fine step of each coarse step, linear
                                  interpolation over its c fine steps, the
                                  control averaged / copied, the mu block
                                  scaled by mu_scale^(log2 c), transfer
                                  variant 0 only, and stand-alone transfer
                                  kernels instead of the ones folded into the
                                  sweeps.  Fixed at setup.                    */
} pitmg_options;

typedef struct {
  int iters;                   /* FGMRES steps taken                           */
  int converged;               /* 1 if the residual estimate met tol           */
  double relres_est;           /* last residual estimate / ||b||               */
  double relres_true;          /* ||b - A~ x|| / ||b|| recomputed at the end   */
  int coarse_calls;            /* coarse solves in this call                   */
  int coarse_its_total;        /* their GMRES steps, summed                    */
  double ms_solve;             /* wall time of the call, ms                    */
  int net_calls;               /* coarse corrections given by the network      */
  int fallback_at;             /* first FGMRES step (0-based) that used GMRES +
                                  SGS after the stall rule fired, or -1        */
} pitmg_stats;

/* Defaults: nu 2/2, coarse tol 1e-3, coarse maxit 50, restart 30, maxit 300,
 * transfer_variant 0, smoother_fp32 0, coarse_mode 0, stall_ratio 0.9,
 * stall_steps 2, vcycle_graph 0, apply_from_sweep 1, pair_sweeps 2,
 * omega 0.5, mu_scale 2, cycle 0 (V), smoother 0 (block Jacobi), unlifted
 * 0, coarsen 2.  (omega = 1 with mu_scale = 1 is the cycle exactly as
 * printed.) */
void pitmg_default_options(pitmg_options* opt);

/* Create a handle: validate, allocate, take the blocks (copy or borrow) and
 * factor every block of every level (S_k = N_k N_k^T + Z~_k Z~_k^T, its
 * Cholesky factor G_k and G_k^{-1}).  stream: a hipStream_t or NULL.
 * Defined by: the blocks of the scaled constraint Jacobian (Sec. 4.1) with
 * the lifting substitutions (Sec. 5.1); the diagonal blocks D_k of the
 * permuted system (Sec. 5.2, Fig. 5), invertible when N_k is (Thm. 1), which
 * is exactly when S_k is positive definite; the level hierarchy of
 * Sec. 5.3.  PITMG_ERR_SINGULAR on a non-positive pivot of some S_k
 * (pitmg_failed_block names it); PITMG_ERR_INVALID on sizes, strides or
 * options out of range; PITMG_ERR_UNSUPPORTED for p or q above 512 or
 * n >= 2^20; PITMG_ERR_OOM when device memory runs out.  *h is NULL on
 * error. */
int pitmg_setup(pitmg_handle** h, const pitmg_problem* pb,
                const pitmg_options* opt, void* stream);

/* New blocks of the same sizes and strides (a new linearisation point):
 * re-borrow or re-copy and re-factor without allocating.  Defined by: each
 * SQP iteration linearises the constraint at a new iterate and solves its
 * augmented systems with the same preconditioner structure (Sec. 6).
 * Errors as pitmg_setup; on error the handle keeps its sizes but its
 * factors are not valid until a refactor succeeds. */
int pitmg_refactor(pitmg_handle* h, const pitmg_problem* pb);

/* Replace the options (sizes of the Krylov space may only shrink below the
 * values given at setup). */
int pitmg_set_options(pitmg_handle* h, const pitmg_options* opt);

/* y = A~ x on level `level` (type-major device vectors of that level):
 * the lifted augmented operator of eq. (augsysp) (Sec. 5.1, Fig. 4; the
 * time-major blocks of Fig. 5 are internal).  x and y must not overlap.
 * PITMG_ERR_INVALID for a level out of range or a NULL vector. */
int pitmg_apply(pitmg_handle* h, int level, const double* x, double* y);

/* One weighted block Jacobi sweep on level `level` (Sec. 5.3.2, the second
 * form of eq. (jacobi), with the correction scaled by the option omega on
 * every level above the coarsest):
 * y_out = (1 - w) y_in + w D^{-1} (b - (L + L^T) y_in); y_in == NULL means
 * y_in = 0.  y_out must not overlap b or y_in.  PITMG_ERR_INVALID for a
 * level out of range or a NULL b or y_out. */
int pitmg_jacobi_sweep(pitmg_handle* h, int level, const double* b,
                       const double* y_in, double* y_out);

/* The coarsest-level solve on its own (Sec. 5.3.4): GMRES right-
 * preconditioned by symmetric block Gauss-Seidel, from x0 = 0 on level
 * n_levels-1, to the relative tolerance coarse_tol (or exactly
 * coarse_fixed_its steps); *its receives the step count (host int, may be
 * NULL; the stream is synchronised when it is given). */
int pitmg_coarse_solve(pitmg_handle* h, const double* b, double* x, int* its);

/* pitmg_coarse_solve without a device buffer of the handle: for callers that
 * cannot allocate or own device memory around the call (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments and result as pitmg_coarse_solve, the same kernels; the coarse
 * Krylov bases, GMRES state and SGS work vectors live in a static device
 * array of 32 MiB that each GPU the library runs on holds until the process
 * ends.  The scratch of one coarse solve is about (2c + 9)(4p+q) n_c
 * doubles (c = coarse_fixed_its if set, else coarse_maxit; n_c the coarsest
 * step count); a solve that needs more than the array returns
 * PITMG_ERR_UNSUPPORTED.  The call allocates nothing (no hipMalloc, hipFree
 * or allocating library routine); it clears the parts of the array that must
 * start at zero with a kernel.  All calls on one GPU share its array, so
 * calls that overlap in time on one GPU (any handles, any streams) race.
 * its may be NULL; otherwise the stream is synchronised and the step count
 * returned. */
int pitmg_coarse_solve_noalloc(pitmg_handle* h, const double* b, double* x, int* its);

/* e = MG(r): one V-cycle from a zero initial guess on the finest level
 * (Alg. 1, recursed to the coarsest level; Sec. 5.3: smoothing Sec. 5.3.2,
 * transfers Sec. 5.3.1, coarse solve Sec. 5.3.4).  r and e are finest-level
 * device vectors and must not overlap.  PITMG_ERR_HIP if a two-sweep launch
 * reports a timed-out hand-off. */
int pitmg_vcycle(pitmg_handle* h, const double* r, double* e);

/* Solve A~ y = b~ (type-major x) by FGMRES preconditioned with one V-cycle
 * per step, to ||b - A~ x|| estimate <= tol ||b||.  x: in = initial guess if
 * use_x0 != 0 (else ignored), out = solution.  st may be NULL.  Defined by:
 * flexible GMRES (Saad 1993) with the multigrid preconditioner, needed
 * because the coarse GMRES makes that preconditioner vary (Sec. 5.3.4,
 * Sec. 6); the true residual of the returned iterate is recomputed and
 * reported in st->relres_true.  Returns PITMG_NOT_CONVERGED (x = last
 * iterate) when maxit steps do not reach tol, PITMG_ERR_NONFINITE on a
 * non-finite residual. */
int pitmg_fgmres_solve(pitmg_handle* h, const double* rhs, double* x,
                       double tol, int use_x0, pitmg_stats* st);

/* The augmented system without virtual variables (Sec. 5, Fig. 2: the
 * constraint Jacobian B = dF of the theta-method steps, blocks K_k = N_k,
 * C_k = V_k, B_k = Z~_k of the lifted system at v = u), on type-major device
 * vectors [u_1..u_n | z_1..z_n | lambda_1..lambda_n] of length (2p+q) n.
 * Both need a handle set up with options.unlifted = 1 (else
 * PITMG_ERR_INVALID).  y = A x (x and y must not overlap). */
int pitmg_unlifted_apply(pitmg_handle* h, const double* x, double* y);
/* FGMRES on A x = rhs preconditioned by one lifted cycle carried through
 * the maps E r = (u/sqrt2, u/sqrt2, z, lambda, 0) and E^T y = ((u+v)/sqrt2,
 * z, lambda): M r = E^T MG(E r), which is A^{-1} when the cycle is exact
 * (the paper names lift / project preconditioning without giving maps;
 * these are the exact ones for the scaled hierarchy).  Arguments, stopping
 * rule, stats and return codes as pitmg_fgmres_solve. */
int pitmg_unlifted_fgmres_solve(pitmg_handle* h, const double* rhs, double* x, double tol,
                                int use_x0, pitmg_stats* st);

/* Solve count independent systems, one handle each (distinct handles; give
 * each its own stream at setup for the solves to overlap on the device).
 * Every solve runs the same FGMRES as pitmg_fgmres_solve, and with the same
 * handle, options and inputs it produces the same iterates; the host
 * interleaves their phases, so each solve's kernels are in flight while the
 * host waits on the others.  rhs[i], x[i]: device vectors of system i (x[i]
 * as in pitmg_fgmres_solve).  st, status: arrays of count (may be NULL);
 * status[i] is system i's return code.  Returns the first error code of any
 * system, else PITMG_NOT_CONVERGED if any did not converge, else PITMG_OK. */
int pitmg_fgmres_solve_batch(pitmg_handle* const* h, int count, const double* const* rhs,
                             double* const* x, double tol, int use_x0, pitmg_stats* st,
                             int* status);

/* Choose, per level above the coarsest, the block Jacobi sweep's launch
 * shape by timing the candidates on this device: the number of consecutive
 * time steps one work-group takes (1..4) where V and Z~ are shared by every
 * step, and the one-step-per-group kernel.  cfg (host, n_levels entries, may
 * be NULL) receives the choice per level: k >= 1 steps per group, -1 the
 * one-step kernel, 0 the built-in rule (no candidates).  The results of a
 * sweep do not depend on the choice beyond rounding.  Synchronises. */
int pitmg_autotune(pitmg_handle* h, int* cfg);

/* Bound of each neighbour wait of the two-sweep launches (pair_sweeps), in
 * seconds; default 2.  For callers that test the error path: a bound of 0
 * makes a wait fail as soon as its neighbour is not already done, so that
 * FGMRES solves return PITMG_ERR_HIP ("a hand-off wait timed out") while
 * every kernel still exits.  Results after a failed wait are not valid.
 * PITMG_ERR_INVALID outside [0, 60]. */
int pitmg_set_handoff_wait(pitmg_handle* h, double seconds);

/* Set the sweep launch shapes directly (host array of n_levels entries, same
 * meaning as pitmg_autotune's output; the coarsest entry must be 0): to reuse
 * a tuned choice on another handle of the same shape, or to fix the launch
 * mix of a profiled run.  A shape the level cannot use is an error. */
int pitmg_set_sweep_shapes(pitmg_handle* h, const int* cfg);

/* Kernel timing: on = 1 brackets every launch with HIP events on the
 * handle's stream and accumulates per-kernel-class time; on = 2 times only
 * the block Jacobi sweep (class 1), whose kernels record their own start and
 * end, and leaves every other launch unbracketed; 0 turns timing off.
 * Classes: 0 factor, 1 jacobi, 2 apply, 3 transfer, 4 coarse, 5 krylov. */
int pitmg_profile_enable(pitmg_handle* h, int on);
/* Time the sweeps of every `every`-th finest-level V-cycle only (default 1):
 * every V-cycle launches the same sweeps, so a sample gives the same average
 * launch duration at a fraction of the event cost. */
int pitmg_profile_sample(pitmg_handle* h, int every);
int pitmg_profile_read(pitmg_handle* h, int cls, int* launches, double* ms,
                       double* bytes);
int pitmg_profile_reset(pitmg_handle* h);

/* After PITMG_ERR_SINGULAR: the (level, step k, 1-based) of the first
 * failing block. */
int pitmg_failed_block(const pitmg_handle* h, int* level, int* k);

/* ------------------------------------------------------------------------
 * Learned coarse-grid correction (a project extension: the paper has no
 * learned component; FGMRES admits a preconditioner that changes from step
 * to step, Sec. 5.3.4, which is what makes replacing the coarse solve safe).
 *
 * Network over the T coarse steps, C = 4p+q channels, H hidden channels:
 *     x = r_c / s,  s = ||r_c||_2 / sqrt(T C)        (s = 0 gives e_c = 0)
 *     h1 = tanh(conv(W1,b1,x)), h2 = tanh(conv(W2,b2,h1)), y = conv(W3,b3,h2)
 *     e_c = s y
 * conv(W,b,x)[t][o] = b[o] + sum_{c,d} W[o][c][d] x[t+d-1][c], zero padded in
 * time; W1 [H][C][3], W2 [H][H][3], W3 [C][H][3].  Samples are node-major FP32
 * [T][C] rows (u_t, v_t, z_t, lambda_t, mu_t).  Parameters: one flat FP32
 * vector [W1, b1, W2, b2, W3, b3] (pitmg_net_param_count entries), the master
 * copy; products run on bfloat16 operands (weights, layer inputs, layer
 * output gradients, rounded to nearest even) with FP32 accumulation.
 * Training: mean squared error over all entries, Adam (beta1 0.9, beta2
 * 0.999, eps 1e-8, bias-corrected).  All pointers below are DEVICE pointers
 * unless marked host.  A network runs on its own stream for training and on
 * the handle's stream when attached; do not train a network while a handle
 * it is attached to is solving.
 * ---------------------------------------------------------------------- */
typedef struct pitmg_net pitmg_net;

long long pitmg_net_param_count(int C, int H);

/* Create a network for C channels over T steps with H hidden channels that
 * trains on batches of up to max_batch samples.  Parameters start at zero:
 * set them with pitmg_net_set_params. */
int pitmg_net_create(pitmg_net** net, int C, int T, int H, int max_batch, void* stream);

/* Copy the FP32 master parameters in (device pointer if on_device, else
 * host) and reset the Adam state. */
int pitmg_net_set_params(pitmg_net* net, const float* theta, int on_device);
/* Copy the FP32 master parameters out to host memory. */
int pitmg_net_get_params(pitmg_net* net, float* theta_host);

/* y = net(x) for batch samples: x, y [batch][T][C] FP32. */
int pitmg_net_forward(pitmg_net* net, int batch, const float* x, float* y);

/* grad = d(loss)/d(theta) for a loss whose gradient w.r.t. y = net(x) is dy
 * (all [batch][T][C] FP32); grad: FP32 [param_count]. */
int pitmg_net_backward(pitmg_net* net, int batch, const float* x, const float* dy,
                       float* grad);

/* One Adam step of the master parameters with the given gradient. */
int pitmg_net_adam(pitmg_net* net, const float* grad, float lr);

/* One training step on the samples idx[0..batch) (device int32 indices into
 * X, Y: [count][T][C] FP32 inputs and targets): forward, mean squared error,
 * backward, Adam.  An index outside [0, count) reads as a zero sample.
 * *loss (host, may be NULL) receives the batch loss before the step. */
int pitmg_net_train_step(pitmg_net* net, int batch, const int* idx, int count,
                         const float* X, const float* Y, float lr, double* loss);

/* Training samples from count type-major coarse pairs (r_c, e_c), each of
 * length C T with C = 4p+q: X[i] = node-major r_c / s, Y[i] = e_c / s. */
int pitmg_net_make_samples(pitmg_net* net, int count, int p, int q, const double* r,
                           const double* e, float* X, float* Y);

const char* pitmg_net_last_error(const pitmg_net* net);
void pitmg_net_destroy(pitmg_net* net);

/* Use net for the coarse solve of h when coarse_mode = 1 (NULL detaches).
 * The network's C and T must be 4p+q and the coarsest step count.  The
 * handle borrows the network: keep it alive while attached. */
int pitmg_coarse_net_attach(pitmg_handle* h, pitmg_net* net);

/* Record the (right-hand side, solution) pairs of the next GMRES + SGS
 * coarse solves into r, e ([cap][len_c] FP64 type-major, len_c = (4p+q) T),
 * until cap pairs are held; cap = 0 stops recording.  Buffers are
 * caller-owned and must stay alive while recording. */
int pitmg_coarse_pairs_arm(pitmg_handle* h, double* r, double* e, int cap);
/* Pairs recorded since the last arm. */
int pitmg_coarse_pairs_count(const pitmg_handle* h);

/* ------------------------------------------------------------------------
 * Burgers' equation by Powell's dogleg (Sec. 6: the nonlinear solver whose
 * Gauss-Newton steps are minimum-norm augmented solves, Sec. 3; Sec. 6.2 and
 * Table 6: viscosity continuation down to the inviscid equation).
 *
 * Unknowns x = [u_1..u_n | z~_1..z~_n] on the device, FP64, 2 nx n values:
 * the states at steps 1..n and the scaled controls z~ = gamma z.  The state
 * equation is backward Euler on n steps of dt = T/n, upwind differences on
 * nx interior nodes of [0, 1] (h = 1/(nx+1), zero Dirichlet values) with
 * the convective term in flux form:
 *     F_k = (u_k - u_{k-1})/dt - nu (u_{i+1} - 2u_i + u_{i-1})/h^2
 *           + (u_i^2 - u_{i-1}^2)/(2h) - z~_k/gamma,   u_0 = w0.
 * B = dF gives the unlifted augmented system of Fig. 2 (N_k tridiagonal,
 * V = -I/dt, Z~ = -I/gamma, both diagonal), which the library solves with
 * its lifted cycle (options.unlifted is forced to 1).
 * ------------------------------------------------------------------------ */
typedef struct {
  int nx;                      /* interior nodes: p = q = nx                   */
  int n;                       /* time steps of the finest grid                */
  int n_levels;                /* multigrid levels (n % coarsen^(n_levels-1) = 0) */
  double T;                    /* final time                                   */
  double gamma;                /* control scaling: x holds z~ = gamma z        */
  const double* w0;            /* host, nx values: the state at t = 0          */
} pitmg_burgers;

typedef struct {
  double ftol;                 /* stop when |F(x)| <= ftol |F(x_start)|, per
                                  viscosity (default 1e-8)                     */
  double lin_tol;              /* FGMRES relative tolerance of the Gauss-Newton
                                  solves (default 1e-6, the value of Sec. 6)    */
  int maxit;                   /* dogleg iterations per viscosity (default 50) */
  double eta;                  /* a step is taken when actual / predicted
                                  decrease of |F|^2 exceeds eta (default 1e-4) */
} pitmg_dogleg_params;

typedef struct {
  int iters;                   /* dogleg iterations (trial steps)              */
  int accepted;                /* steps taken                                  */
  int converged;               /* 1 if |F| met ftol                            */
  int solves;                  /* Gauss-Newton augmented solves                */
  int fgmres_iters;            /* their FGMRES steps, summed                   */
  int coarse_calls;            /* coarse-grid solves in them                   */
  int coarse_its;              /* their SGS-preconditioned GMRES steps         */
  double fnorm0, fnorm;        /* |F| at the start and at the end              */
  double ms;                   /* wall time for this viscosity, ms             */
} pitmg_dogleg_stats;

void pitmg_default_dogleg_params(pitmg_dogleg_params* dp);
/* F(x) into F (device, nx n values) for viscosity nu >= 0.  x as above.
 * Synchronises the stream.  PITMG_ERR_INVALID for bad sizes or NULLs. */
int pitmg_burgers_residual(const pitmg_burgers* bp, double nu, const double* x, double* F,
                           void* stream);
/* Dogleg solves of F(x) = 0 for the viscosities nus[0..n_nu) in order, each
 * from the previous solution (x: device, in the starting point, out the
 * last solution).  One dogleg iteration at x: the Gauss-Newton step s_N is
 * the (u, z~) part of the unlifted solve A (s, y) = (0, -F) (FGMRES to
 * lin_tol); g = B^T F; the Cauchy step -tau g, tau = |g|^2/|Bg|^2; the step
 * s_N if |s_N| <= delta, the boundary point along -g if the Cauchy step
 * leaves the radius, else the point of radius delta on the segment between
 * them; rho = (|F(x)|^2 - |F(x+s)|^2)/(|F|^2 - |F + B s|^2); the step is
 * taken when rho > eta; delta becomes |s|/4 when rho < 1/4 and doubles when
 * rho > 3/4 at the boundary; delta starts at |s_N| of the first iteration
 * of each viscosity.  opt: the augmented solver's options (NULL:
 * defaults; unlifted is forced to 1).  st: n_nu entries.  Returns PITMG_OK,
 * PITMG_NOT_CONVERGED when a viscosity ran out of iterations (x is the last
 * iterate), or an error (pitmg_burgers_last_error gives the message). */
int pitmg_burgers_dogleg(const pitmg_burgers* bp, const pitmg_options* opt, const double* nus,
                         int n_nu, double* x, const pitmg_dogleg_params* dp,
                         pitmg_dogleg_stats* st, void* stream);
const char* pitmg_burgers_last_error(void);

/* Bytes of device memory held by the handle. */
long long pitmg_device_bytes(const pitmg_handle* h);

/* Level `level` (0 = finest) of a set-up handle: *n its step count, *flags
 * a bit set: PITMG_LEVEL_FP32 when its sweeps run in FP32, and
 * PITMG_LEVEL_DIAG_VZ when V and Z~ are shared by every step and diagonal
 * (theta = 1 with an identity mass matrix and distributed control, Sec. 6),
 * so the sweeps and products use their diagonals alone, and
 * PITMG_LEVEL_GIN when the level also keeps W_k = G_k^{-1} N_k for its
 * one-step sweeps (FP64, p = q in {64, 128}, diagonal V and Z~).  Either
 * pointer may be NULL.  Returns PITMG_ERR_INVALID for a NULL handle or a
 * level out of range. */
#define PITMG_LEVEL_FP32 1
#define PITMG_LEVEL_DIAG_VZ 2
#define PITMG_LEVEL_GIN 4
int pitmg_level_info(const pitmg_handle* h, int level, int* n, int* flags);

const char* pitmg_status_string(int code);
const char* pitmg_last_error(const pitmg_handle* h);
void pitmg_destroy(pitmg_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* PITMG_H */
