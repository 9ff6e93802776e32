/*
 * richards.h -- C-ABI of the MI355X (gfx950) solver for the 3-D Richards
 * equation, following Bertaccini, D'Ambra, Durastante and Filippone,
 * "Why diffusion-based preconditioning of Richards equation works: spectral
 * analysis and computational experiments at very large scale" (arXiv
 * 2112.05051).
 *
 * What is computed (paper references are sections and labelled equations):
 *   - backward Euler in time on a cell-centred 7-point finite-difference grid
 *     (Section 2.1, eq. (dynamic_of_the_problem));
 *   - each time step solved by a modified inexact Newton method with an
 *     Armijo-Goldstein line search and the Jacobian re-use rules of
 *     eq. (jacobian_update_condition) (Section 3);
 *   - every Newton correction J d = -Phi solved by restarted GMRES, right
 *     preconditioned (eq. (precsystem)) with an aggregation AMG V-cycle
 *     (Section 5.2) built on the diffusion-only operator (end of Section 4).
 *
 * Conventions
 *   - Grid: nx*ny*nz unknowns, index c = i + nx*(j + ny*k), x fastest, k
 *     upward (z is elevation).  Faces are ordered -x,+x,-y,+y,-z,+z.
 *   - Every array argument named *_dev is DEVICE memory (hipMalloc'd, e.g. a
 *     torch tensor's data pointer) holding `double` values in that order,
 *     owned by the caller, only accessed during the call.  Arguments named
 *     *_host are host memory owned by the caller.
 *   - A handle is bound to the HIP stream given at creation; every kernel of
 *     a call is launched on it.  Calls return after their work is complete
 *     unless stated otherwise.  Distinct handles share no state.
 *   - Every function returns a rich_status; RICH_OK = 0, errors < 0,
 *     warnings > 0.  On an error inside rich_step the state stays at the last
 *     accepted time level.
 */
#ifndef RICHARDS_H
#define RICHARDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int rich_status;
#define RICH_OK 0
#define RICH_EINVAL (-1)          /* bad size, spacing, dt, parameter or pointer */
#define RICH_ENOMEM (-2)          /* device allocation failed */
#define RICH_EBUDGET (-3)         /* request does not fit the memory budget */
#define RICH_NONFINITE (-4)       /* NaN/Inf in an input or an iterate */
#define RICH_LINSOLVE_FAIL (-5)   /* GMRES failed with a fresh J and d is no descent direction */
#define RICH_LINESEARCH_FAIL (-6) /* line search failed with a fresh J */
#define RICH_MAXITER (-7)         /* Newton iteration limit reached */
#define RICH_NOT_SPD (-9)         /* coarsest matrix not positive definite */
#define RICH_EHIP (-10)           /* HIP runtime error */
#define RICH_ESTATE (-11)         /* call not valid in the handle's current state */
#define RICH_STEP_TOO_SMALL 2     /* warning: Newton stalled with a fresh J; state kept */

/* interface means of K (Section 2.1; harmonic: named in the abstract).  The
 * integral mean averages K_s k_r(psi) over the heads between the two cells
 * (K_s: the two cells' arithmetic mean) with a 16-point Gauss-Legendre rule. */
#define RICH_MEAN_ARITH 0
#define RICH_MEAN_UPSTREAM 1
#define RICH_MEAN_HARMONIC 2
#define RICH_MEAN_GEOMETRIC 3
#define RICH_MEAN_INTEGRAL 4
/* boundary face types */
#define RICH_BC_NOFLUX 0
#define RICH_BC_DIRICHLET 1
/* arithmetic of the AMG V-cycle (the Newton/GMRES outer loop is always FP64) */
#define RICH_PREC_FP64 0
#define RICH_PREC_MIXED 1

/* The problem statement of Sections 2 and 2.1. */
typedef struct rich_problem {
    int nx, ny, nz;      /* unknowns per axis (>= 1) */
    double hx, hy, hz;   /* grid spacing [cm] (> 0) */
    /* eq. (s(p)): theta = alpha (theta_s - theta_r) / (alpha + |p|^beta) + theta_r
       eq. (K(p)): K = K_s A / (A + |p|^gamma); p >= 0 is saturated */
    double alpha, beta, theta_s, theta_r, A, gamma;
    int mean;            /* RICH_MEAN_* on every face, or on the x and y faces when mean_vertical >= 0 */
    int bc_type[6];      /* RICH_BC_* per face -x,+x,-y,+y,-z,+z */
    double bc_value[6];  /* Dirichlet head [cm] per face */
    double dt;           /* time step [s] (> 0) */
    /* optional Dirichlet patch (Section 6's 3-D test: zero head on a square of the top face):
       boundary nodes of face patch_face (-1: none; the face must be Dirichlet) whose two
       tangential coordinates lie in [patch_lo, patch_hi] (cm; node (i,j) of a face sits at
       ((i+1) h, (j+1) h) along the face's axes in x, y, z order) take patch_value instead of
       bc_value[patch_face] */
    int patch_face;
    double patch_lo[2], patch_hi[2];
    double patch_value;
    int mean_vertical;   /* RICH_MEAN_* on the z faces (Section 2.1: one mean for the horizontal and
                            another for the vertical direction); -1 = the same as mean */
} rich_problem_t;

/* Solver controls (Sections 3 and 6). */
typedef struct rich_solver_opts {
    double fnormtol;     /* Newton stops at ||Phi||_inf <= fnormtol */
    double scsteptol;    /* minimum relative step (eps^(2/3) in the paper) */
    int max_newton;      /* Newton iteration limit per time step */
    int msbset;          /* rebuild J after this many Newton iterations (10) */
    double ls_alpha;     /* Armijo constant (1e-4) */
    double mxnewtstep;   /* maximum ||d||_2; <= 0 -> 1000 max(||p_init||_2, 1) */
    int gmres_restart;   /* m of GMRES(m), 1..64 */
    double eta;          /* GMRES stops at ||J d + Phi||_2 <= eta ||Phi||_2 */
    int gmres_maxit;     /* GMRES iteration limit per Newton correction */
    int amg_max_levels;  /* <= 16 */
    int64_t amg_coarse_size;  /* stop coarsening at <= this many rows (also stops when a level
                                 would keep more than half of the rows and the current level
                                 is at most coarse_dense_max) */
    int amg_sweeps;      /* pairwise matching sweeps per level (3 -> aggregates <= 8) */
    int64_t coarse_dense_max; /* coarsest solved directly when n <= this (<= 8192) */
    int coarse_l1_sweeps;     /* otherwise this many l1-Jacobi sweeps */
    int precision;       /* RICH_PREC_* */
    double gmres_reorth; /* second Gram-Schmidt pass when ||w_after|| < gmres_reorth ||w_before||
                            (0 = never, 0.7071 = always-safe DGKS rule) */
    int aux_dflux;       /* 1: the auxiliary matrix's diagonal also takes the flux-derivative
                            terms -(p_n-p_c)/h^2 dK^AV/dp_c of the diffusion Jacobian (off-diagonal
                            ones dropped: M stays symmetric); 0: frozen conductivity only */
    int amg_refresh;     /* on every rebuild after the first: 0 = refresh the fine level and its
                            smoother only (coarse matrices frozen, Section 6); 1 = also recompute
                            every coarse matrix from the new fine one, aggregates kept */
    int amg_smoothed;    /* number of levels, from the finest, whose prolongator is smoothed
                            (Section 5.2), 0..16: P = (I - omega D^{-1} A) P_t with D = diag(A),
                            omega = 4 / (3 max_i sum_j |a_ij| / a_ii), and coarse matrix P^T A P;
                            the other levels keep the piecewise-constant P_t.  Smoothing costs
                            set-up work and denser coarse levels and saves GMRES iterations */
    int tile_kz;         /* planes per thread block in the tiled fine-level smoother kernels
                            (0 = automatic; a tuning knob, results do not depend on it) */
    int smoother;        /* fine-level smoother of a multi-level hierarchy: RICH_SMOOTH_L1
                            (l1-Jacobi, the default) or RICH_SMOOTH_MCGS (multicolour
                            Gauss-Seidel, colour (i+j+k) mod 2, diagonal m_cc: one backward
                            sweep from zero before and one forward sweep after the coarse
                            correction, the GPU form of the hybrid backward/forward
                            Gauss-Seidel of the paper's experiments, Section 6); coarser
                            levels always take l1-Jacobi */
    int amg_aggregation; /* RICH_AGG_MATCHING (pairwise matching sweeps, the default) or
                            RICH_AGG_VMB: the DSVMB coarsening of Section 5.2, decoupled greedy
                            aggregation (Vanek-Mandel-Brezina) in which every block of amg_block
                            consecutive rows aggregates its own rows and ignores couplings that
                            leave it; j is strongly coupled to i when |a_ij| >= amg_theta
                            sqrt(|a_ii a_jj|); phase 1 roots (rows whose strong neighbours are
                            all free) take their strong neighbourhood, phase 2 attaches each
                            remaining row to its strongest phase-1 neighbour's aggregate,
                            phase 3 groups what is left.  Combine with amg_smoothed for the
                            smoothed prolongator. */
    double amg_theta;    /* strength threshold of RICH_AGG_VMB, 0..1 (0: every coupling is strong;
                            larger values stall the coarsening where the storage term theta'/dt
                            dominates the diagonal) */
    int64_t amg_block;   /* rows per decoupled block of RICH_AGG_VMB, >= 1 (4096) */
    int gmres_block;     /* Arnoldi vectors generated per Gram-Schmidt round of GMRES, 1..10 (10).
                            1: one vector per round (classical Gram-Schmidt, the second pass
                            governed by gmres_reorth).  s >= 2: s-step GMRES (Section 6's
                            right-preconditioned GMRES(m), the same Krylov space and minimal
                            residual): s vectors of the shifted (Newton) power basis
                            q_{t+1} = (J M^{-1} - sigma_t I) q_t are generated, then
                            orthogonalised against the basis and each other in one
                            block round (dots and Gram matrix in one pass, a Cholesky factor
                            of the Gram matrix's Pythagorean complement, one update pass), so
                            the basis is read twice per s vectors instead of twice per vector.
                            From the first vector whose Cholesky pivot keeps less than
                            gmres_reorth of its norm, a round is finished vector by vector
                            with two classical passes, and the following rounds are capped at
                            the vectors before it (at least one; every 8 whole rounds in a row
                            raise the cap by one, up to s).  The Hessenberg matrix follows from the
                            basis change;
                            convergence is tested after every column (the iteration count is
                            that of one-vector rounds), the next round's size is cut to the
                            steps the residual's decay predicts. */
    double gmres_shift;  /* centre c of the s-step basis shifts (0.65) */
    double gmres_shift_span; /* half-width w >= 0 of the shift interval (0.55): sigma_0..sigma_{s-1}
                            are the Leja points of [c - w, c + w] in Leja order (the end of
                            larger modulus first, each next one maximising the product of its
                            distances to the earlier ones on a 4097-point grid); w = 0: every
                            sigma_t = c.  Spread over the spectrum of J M^{-1} (near (0, 1.3])
                            the shifts keep the basis of long rounds well conditioned. */
} rich_solver_opts_t;
#define RICH_SMOOTH_L1 0
#define RICH_SMOOTH_MCGS 1
#define RICH_AGG_MATCHING 0
#define RICH_AGG_VMB 1

/* Per-time-step counters, timings and traffic.  The phases are those the
 * paper's experiments time (Section 6): residual evaluations (Feval), the
 * Jacobian with the auxiliary matrix (assembled together in one pass over
 * the grid), the update of the preconditioner from a new auxiliary matrix
 * (Aux: smoother data and coarse matrices), the full AMG set-up (Setup),
 * the linear solves (LinSol) and everything else (Overhead: line-search
 * vector updates, norms, host decisions).  Times are host wall seconds;
 * bytes are the algorithmic HBM bytes of the kernels each phase launched
 * (the data the operations must move, re-reads excluded) of the kernels of
 * Feval, Jacobian, LinSol and Overhead; set-up and Aux work (sorting,
 * matching, sparse products) is timed but not counted in bytes. */
typedef struct rich_step_stats {
    int status;
    int newton_its, jac_builds, gmres_its, ls_backtracks, amg_setups, linsolve_fails, levels;
    int gmres_rounds;     /* s-step block rounds (gmres_block >= 2) */
    int gmres_redone;     /* of which finished vector by vector from the first vector whose
                             Cholesky pivot kept less than gmres_reorth of its norm */
    double fnorm_inf;     /* ||Phi||_inf at the accepted state */
    double mass_residual; /* dt * sum_c Phi_c at the accepted state */
    double min_lambda;    /* smallest accepted line-search step */
    double opc;           /* operator complexity sum nnz(A_l) / nnz(A_0) */
    double t_feval, t_jac, t_aux, t_setup, t_linsol, t_overhead, t_total;
    double bytes_feval, bytes_jac, bytes_linsol, bytes_overhead;
} rich_step_stats_t;

/* Record of one attempt of the Newton controller (Section 3): the rebuild
 * test of eq. (jacobian_update_condition), the GMRES solve and the line
 * search at one iterate.  An attempt that ends with a retry request (stale
 * J) is followed by another at the same iterate. */
#define RICH_TRACE_TRIALS 48
#define RICH_EV_ACCEPT 0        /* step accepted */
#define RICH_EV_ACCEPT_SHORT 1  /* accepted, shorter than scsteptol, stale J: rebuild next */
#define RICH_EV_RETRY_GMRES 2   /* GMRES failed with a stale J */
#define RICH_EV_RETRY_SLOPE 3   /* d is no descent direction, stale J */
#define RICH_EV_RETRY_LS 4      /* line search failed, stale J */
#define RICH_EV_FAIL_SLOPE 5    /* d is no descent direction, fresh J (RICH_LINSOLVE_FAIL) */
#define RICH_EV_FAIL_LS 6       /* line search failed, fresh J (RICH_LINESEARCH_FAIL) */
#define RICH_EV_STALL 7         /* shorter than scsteptol with a fresh J (RICH_STEP_TOO_SMALL) */
#define RICH_EV_FAIL_OTHER 8    /* set-up error or non-finite residual */
#define RICH_RB_NOJ 1           /* rebuild reasons (bits): no J yet */
#define RICH_RB_MSBSET 2        /* msbset iterations since the last rebuild */
#define RICH_RB_BIGSTEP 4       /* the previous step had ||lam d||_inf > 1.5 */
#define RICH_RB_RETRY 8         /* the previous attempt asked for a retry */
typedef struct rich_newton_event {
    int step;         /* time step, counted from 0 since the handle was created */
    int newton_it;    /* accepted Newton iterations of this step before the attempt */
    int since_build;  /* iterations since the last rebuild, before the rebuild test */
    int reason;       /* RICH_RB_* bits that held (0: J re-used) */
    int gmres_its, gmres_conv, truncated, outcome;
    int ntrial;       /* line-search trials u + lam d in order, the full step first */
    int nback;        /* of which backtracking trials (the rest lengthen a full step) */
    double f0;        /* 0.5 ||Phi(u)||_2^2 at the attempt's iterate */
    double slope;     /* Phi(u)^T J d */
    double dnorm2, dnorminf;  /* of the (possibly truncated) correction d */
    double rel_d;     /* max_i |d_i| / max(|u_i|, 1) */
    double mxstep;    /* maximum step length */
    double lam, f_acc;        /* accepted step and 0.5 ||Phi||^2 there (0 if none) */
    double step_inf, step_rel, fnorm_inf;  /* ||lam d||_inf, relative length, ||Phi||_inf after */
    double trial_lam[RICH_TRACE_TRIALS], trial_f[RICH_TRACE_TRIALS];  /* f = 0.5 ||Phi||^2 */
} rich_newton_event_t;

typedef struct rich_ctx *rich_handle_t;

/* ---------------------------------------------------------------- core -- */

/* Device bytes a handle for (prob, opts) will hold, before the AMG
 * hierarchy (whose size depends on the matrix) -- plus an upper bound for
 * the hierarchy assuming operator complexity <= 3. */
rich_status rich_query_bytes(const rich_problem_t *prob, const rich_solver_opts_t *opts,
                             size_t *bytes);

/* Create a handle.  Ks_dev: N saturated conductivities [cm/s] (> 0), copied.
 * hip_stream: a hipStream_t (NULL = default stream).  The state is
 * undefined until rich_set_state. */
rich_status rich_create(const rich_problem_t *prob, const rich_solver_opts_t *opts,
                        const double *Ks_dev, void *hip_stream, rich_handle_t *out);
rich_status rich_destroy(rich_handle_t h);

/* Copy the head field p (N values) in / out of the handle. */
rich_status rich_set_state(rich_handle_t h, const double *p_dev);
rich_status rich_get_state(rich_handle_t h, double *p_dev);

/* Advance nsteps backward-Euler steps.  stats_host: nsteps entries or NULL.
 * Returns the first error (< 0; the state is then the last good level and
 * no further step is taken), else the largest warning (> 0) any step gave,
 * else RICH_OK. */
rich_status rich_step(rich_handle_t h, int nsteps, rich_step_stats_t *stats_host);

/* Record every attempt of the Newton controller in the following rich_step
 * calls into events_host (host memory, `capacity` entries, owned by the
 * caller and written during rich_step); NULL stops recording.  Arming resets
 * the count.  rich_trace_count gives the number of attempts since arming,
 * which may exceed the capacity (the excess is not stored). */
rich_status rich_trace_newton(rich_handle_t h, rich_newton_event_t *events_host, int capacity);
rich_status rich_trace_count(rich_handle_t h, int64_t *count_host);

const char *rich_status_string(rich_status s);

/* ------------------------------------------------ inspection / parity -- */

/* theta(p) per cell (eq. (s(p)) with rho*phi = 1). */
rich_status rich_eval_theta(rich_handle_t h, const double *p_dev, double *theta_dev);
/* Phi(p) of eq. (dynamic_of_the_problem) with f = 0 and the given theta at
 * the previous level. */
rich_status rich_eval_residual(rich_handle_t h, const double *p_dev, const double *theta_old_dev,
                               double *F_dev);
/* Assemble J(p) and the auxiliary matrix M(p) into the handle and refresh
 * the fine-level smoother; builds the AMG hierarchy if none exists yet. */
rich_status rich_assemble(rich_handle_t h, const double *p_dev);
/* (Re)build the AMG hierarchy from the current auxiliary matrix. */
rich_status rich_setup_hierarchy(rich_handle_t h);
/* y = J x and y = M x with the assembled matrices (FP64). */
rich_status rich_apply_jacobian(rich_handle_t h, const double *x_dev, double *y_dev);
rich_status rich_apply_aux(rich_handle_t h, const double *x_dev, double *y_dev);
/* x = one V-cycle applied to b, in the handle's precision. */
rich_status rich_apply_prec(rich_handle_t h, const double *b_dev, double *x_dev);
/* Solve J x = b by right-preconditioned GMRES(m) from x = 0.  Returns RICH_OK
 * when ||b - J x||_2 <= eta ||b||_2, RICH_LINSOLVE_FAIL otherwise. */
rich_status rich_gmres(rich_handle_t h, const double *b_dev, double *x_dev, int *its_host,
                       double *relres_host);

/* Hierarchy shape.  Level 0 is the auxiliary matrix. */
rich_status rich_levels(rich_handle_t h, int *nlev_host);
rich_status rich_level_size(rich_handle_t h, int level, int64_t *n_host, int64_t *nnz_host);
#define RICH_WHICH_J 0  /* the Jacobian (level ignored) */
#define RICH_WHICH_A 1  /* the level-l AMG matrix, FP64 (level 0 = auxiliary M) */
#define RICH_WHICH_P 2  /* the prolongator of level l -> l+1 (n_l rows, n_{l+1} columns):
                           the smoothed one, or the piecewise-constant P(i, agg(i)) = 1 */
#define RICH_WHICH_PT 3 /* its transpose, the restriction (n_{l+1} rows, n_l columns) */
/* Copy a matrix to host CSR (columns ascending).  *nnz_inout: capacity in,
 * entries written out; RICH_EINVAL if the capacity is too small. */
rich_status rich_export_csr(rich_handle_t h, int which, int level, int64_t *rowptr_host,
                            int32_t *col_host, double *val_host, int64_t *nnz_inout);
/* Aggregate index (level l -> l+1) of every level-l row, to host. */
rich_status rich_export_aggregates(rich_handle_t h, int level, int32_t *agg_host,
                                   int64_t *n_coarse_host);

/* One pairwise matching sweep on a device CSR matrix (int64 rowptr, int32
 * columns ascending, double values): the matching of Section 5.2 (SMATCH),
 * weights w_ij = 1 - 2 a_ij / (a_ii + a_jj) from the row min(i,j), greedy in
 * the strict order (w desc, i asc, j asc), singletons for unmatched rows,
 * coarse indices in increasing order of the smallest member.  agg_dev: n
 * int32 outputs.  Runs on hip_stream and returns when done. */
rich_status rich_match_sweep(int64_t n, const int64_t *rowptr_dev, const int32_t *col_dev,
                             const double *val_dev, int32_t *agg_dev, int64_t *n_coarse_host,
                             void *hip_stream);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): rich_match_sweep
 * with the same arguments and results, whose device work arrays live in a
 * fixed array of RICH_NOALLOC_SCRATCH_BYTES per GPU (reserved for the life
 * of the process on every GPU the library runs on) and which calls no
 * allocator.  The work arrays need about 32 n + 8 nnz bytes (nnz =
 * rowptr[n]); larger inputs return RICH_EBUDGET before any kernel runs.
 * Every call on one GPU uses that GPU's one array, so calls that overlap on
 * a GPU (other host threads, other streams) race and must be serialised by
 * the caller; each call initialises what it reads before using it.  Runs
 * on hip_stream and returns when done. */
#define RICH_NOALLOC_SCRATCH_BYTES (64u << 20)
rich_status rich_match_sweep_noalloc(int64_t n, const int64_t *rowptr_dev, const int32_t *col_dev,
                                     const double *val_dev, int32_t *agg_dev, int64_t *n_coarse_host,
                                     void *hip_stream);

/* ----------------------------------------------------------- profiling -- */
/* Hot kernels whose launches can be timed with HIP events on the handle's
 * stream while profiling is on.  Each launch also adds its algorithmic HBM
 * bytes (the data the operation must move: coefficients, vectors in and
 * out, index arrays of the AMG levels; neighbour re-reads excluded). */
#define RICH_K_SPMV_J 0       /* y = J z inside GMRES (7 FP64 coefficient arrays) */
#define RICH_K_VC0_PRE 1      /* fine level: pre-smooth from zero + residual */
#define RICH_K_VC0_POST 2     /* fine level: prolongation + post-smooth */
#define RICH_K_VC0_RESTRICT 3 /* fine -> level 1 restriction */
#define RICH_K_VC1_PRE 4      /* level 1 (CSR): pre-smooth + residual */
#define RICH_K_VC1_POST 5     /* level 1 (CSR): prolongation + post-smooth */
#define RICH_K_MULTIDOT 6     /* Gram-Schmidt dot block V^T w (first pass) */
#define RICH_K_UPDATE 7       /* w -= V h with ||w||^2 (first pass) */
#define RICH_K_RESIDUAL 8     /* Phi(p) */
#define RICH_K_BLOCK_DOT 9    /* s-step GMRES: block dots V^T Q and Gram matrix Q^T Q */
#define RICH_K_BLOCK_UPDATE 10 /* s-step GMRES: Q <- (Q - V C) R^{-1} */
#define RICH_K_COUNT 11
/* enable != 0: clear the counters and start timing; 0: stop. */
rich_status rich_profile(rich_handle_t h, int enable);
/* Launch count, summed kernel milliseconds and summed algorithmic bytes of
 * one kernel since profiling was enabled (waits for the stream). */
rich_status rich_profile_read(rich_handle_t h, int kernel, int64_t *launches_host, double *ms_host,
                              double *bytes_host);

/* ------------------------------------------------------------- serving -- */
/* Ensemble serving (an addition to the paper's method): independent
 * simulations, each with its own grid, K_s field, interface mean and step
 * count, submitted at any time.  Requests wait in a FIFO queue and are
 * admitted when one of `max_active` workers is free and their device-memory
 * plan (rich_query_bytes plus K_s/p staging) fits the remaining budget; an
 * admitted simulation stays resident on the GPU for all its steps and runs
 * on its own HIP stream, so concurrent simulations overlap on the device.
 * With fused batching (off by default), the resident simulations inside
 * a GMRES solve post each preconditioned product J M^{-1} v to a batcher
 * shared by the simulations of the same grid size and precision; the
 * batcher's thread issues every product posted so far as one batch on its
 * own stream, then the products posted meanwhile, and so on.  A batch runs
 * as one launch per kernel (fine smoother, restriction, each coarse level's
 * smoother, coarsest product, prolongations, J SpMV) over a work list of
 * (simulation, block range).  Simulations whose hierarchy the batched kernels
 * do not cover (smoothed prolongators, one level, no dense coarsest solve)
 * launch on their own stream.
 * A simulation's result equals that of a lone rich_create/rich_step run
 * (bit for bit: every block runs the lone kernel's code on its data).
 * The server uses the device of the stream given at creation, or the device
 * that is current then. */
typedef struct rich_server *rich_server_t;
#define RICH_REQ_QUEUED 0
#define RICH_REQ_RUNNING 1
#define RICH_REQ_DONE 2
/* hip_stream: NULL, or a hipStream_t whose device the server runs on and after
 * whose work (as queued at each rich_server_submit) that request's first
 * kernel runs; with NULL the server uses the device current at creation and
 * orders nothing.  Each worker launches on a non-blocking stream of its own. */
rich_status rich_server_create(size_t hbm_budget_bytes, int max_active, void *hip_stream, rich_server_t *out);
/* Ks_host, p0_host: N host values each, copied.  RICH_EBUDGET if the request
 * alone exceeds the budget.  *req_id receives the request's id. */
rich_status rich_server_submit(rich_server_t s, const rich_problem_t *prob, const rich_solver_opts_t *opts,
                               const double *Ks_host, const double *p0_host, int nsteps, int64_t *req_id);
/* *state: RICH_REQ_*.  Once done: *result is the simulation's status, p_host
 * (N values) its final state, stats_host / step_ms_host (nsteps entries) the
 * per-step counters and wall milliseconds, times_host (3 values) the
 * admission wait [s], the resident time [s] and the number of steps run.
 * Every output pointer may be NULL. */
rich_status rich_server_poll(rich_server_t s, int64_t req_id, int *state, rich_status *result, double *p_host,
                             rich_step_stats_t *stats_host, double *step_ms_host, double *times_host);
/* Batching mode: RICH_BATCH_OFF (the default: every simulation launches on
 * its own stream, which measures faster on the ensembles tried),
 * RICH_BATCH_FUSED (one launch per kernel over the posted products, one
 * thread block per block of work) or RICH_BATCH_PERSISTENT (the same fused
 * launches as persistent grids: a fixed number of thread blocks, each taking
 * blocks of work from a device-side work counter until none is left; every
 * block leaves once the counter passes the launch's total).  Only before the
 * first submission: RICH_ESTATE afterwards; RICH_EINVAL for another mode. */
#define RICH_BATCH_OFF 0
#define RICH_BATCH_FUSED 1
#define RICH_BATCH_PERSISTENT 2
rich_status rich_server_set_batching(rich_server_t s, int mode);
/* Batched flushes so far and the products they carried (their ratio is the
 * mean number of simulations per fused launch). */
rich_status rich_server_batch_stats(rich_server_t s, int64_t *flushes, int64_t *products);
/* Block until no request is queued or running. */
rich_status rich_server_run_until_idle(rich_server_t s);
/* Let running simulations finish, drop queued ones, release the server. */
rich_status rich_server_destroy(rich_server_t s);

#ifdef __cplusplus
}
#endif
#endif
