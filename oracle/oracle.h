/*
 * Plain FP64 CPU oracle for the backward-Euler / inexact-Newton / AMG-GMRES
 * solve of the 3-D Richards equation (Bertaccini, D'Ambra, Durastante,
 * Filippone, arXiv 2112.05051).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this code; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the HIP path.
 *
 * Every routine is a slow, direct transcription of what the paper's equations
 * (and, where the paper is silent, the documented reading) define: plain
 * loops, no blocking, no fusion.
 *
 * Grid: nx*ny*nz unknowns, x fastest: c = i + nx*(j + ny*k); k grows upward
 * (z is elevation).  Faces are numbered 0..5 = -x,+x,-y,+y,-z,+z.
 */
#ifndef RICHARDS_ORACLE_H
#define RICHARDS_ORACLE_H
#include <stdint.h>

#define ORC_ARITH 0
#define ORC_UPSTREAM 1
#define ORC_HARMONIC 2
#define ORC_GEOMETRIC 3
#define ORC_INTEGRAL 4

#define ORC_NOFLUX 0
#define ORC_DIRICHLET 1

/* status codes */
#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_NONFINITE (-4)
#define ORC_LINSOLVE_FAIL (-5)
#define ORC_LINESEARCH_FAIL (-6)
#define ORC_MAXITER (-7)
#define ORC_STEP_TOO_SMALL 2 /* warning: state kept */
#define ORC_NOT_SPD (-9)

typedef struct {
    int nx, ny, nz;
    double hx, hy, hz;
    double alpha, beta, theta_s, theta_r, A, gamma;
    int mean;
    int bc_type[6];
    double bc_value[6];
    double dt;
    int patch_face;                 /* Dirichlet patch on one face (-1: none) */
    double patch_lo[2], patch_hi[2];
    double patch_value;
    int mean_vertical;              /* mean on z faces (-1: the same as mean) */
} orc_problem;

typedef struct {
    double fnormtol, scsteptol;
    int max_newton, msbset;
    double ls_alpha, mxnewtstep;
    int gmres_restart;
    double eta;
    int gmres_maxit;
    int amg_max_levels;
    int64_t amg_coarse_size;
    int amg_sweeps;
    int64_t coarse_dense_max;
    int coarse_l1_sweeps;
    int amg_refresh; /* 0: later rebuilds refresh the smoother only; 1: also the coarse matrices */
    int aux_dflux;   /* 1: the auxiliary matrix's diagonal also takes the flux-derivative terms */
    int amg_smoothed; /* levels (from the finest) with smoothed prolongators; 0: none */
    int smoother;     /* 0: l1-Jacobi on every level; 1: multicolour Gauss-Seidel on the finest
                         level (backward before, forward after the coarse correction) */
    int amg_aggregation; /* 0: pairwise matching sweeps; 1: decoupled greedy (VMB) aggregation */
    double amg_theta;    /* strength threshold of the greedy aggregation */
    int64_t amg_block;   /* rows per decoupled block of the greedy aggregation */
} orc_opts;

typedef struct {
    int64_t n;
    int64_t *rowptr; /* n+1 */
    int32_t *col;
    double *val;
} orc_csr;

typedef struct {
    int status;
    int newton_its, jac_builds, gmres_its, ls_backtracks, amg_setups;
    int linsolve_fails;
    double fnorm_inf;
    double mass_residual;  /* dt * sum_c Phi_c(p_final) (per unit cell volume) */
    double min_lambda;
} orc_stats;

/* ---- constitutive laws, residual, Jacobian, auxiliary matrix ---- */
void orc_laws(const orc_problem *P, double p, double Ks, double out[4]); /* theta, theta', K, K' */
/* interface mean of a face between heads pc and pn (dir = +1: pn on the higher-index side) */
void orc_face_mean(const orc_problem *P, int axis, int dir, double pc, double Ksc, double pn,
                   double Ksn, double out[3]); /* K_f, dK_f/dp_c, dK_f/dp_n */
void orc_laws_array(const orc_problem *P, int64_t n, const double *p, const double *Ks,
                    double *out /* n x 4 */);
void orc_theta(const orc_problem *P, const double *p, double *theta);
void orc_residual(const orc_problem *P, const double *Ks, const double *p, const double *theta_old,
                  double *F);
int64_t orc_pattern_nnz(const orc_problem *P);
void orc_jacobian(const orc_problem *P, const double *Ks, const double *p, int64_t *rowptr,
                  int32_t *col, double *val);
void orc_auxiliary(const orc_problem *P, const double *Ks, const double *p, int64_t *rowptr,
                   int32_t *col, double *val);
void orc_auxiliary_dflux(const orc_problem *P, const double *Ks, const double *p, int64_t *rowptr,
                         int32_t *col, double *val);
void orc_csr_matvec(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                    const double *x, double *y);

/* ---- aggregation ---- */
int64_t orc_match_sweep(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                        int32_t *agg);
int64_t orc_galerkin_nnz(int64_t n, const int64_t *rowptr, const int32_t *col, const int32_t *agg,
                         int64_t nc);
void orc_galerkin(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                  const int32_t *agg, int64_t nc, int64_t *crow, int32_t *ccol, double *cval);

/* ---- smoothed aggregation: P = (I - omega D^{-1} A) P_t, C = P^T (A P) ---- */
int64_t orc_smoothed_prolongator_nnz(int64_t n, const int64_t *rowptr, const int32_t *col,
                                     const int32_t *agg, int64_t nc);
double orc_smoothed_prolongator(int64_t n, const int64_t *rowptr, const int32_t *col,
                                const double *val, const int32_t *agg, int64_t nc, int64_t *prow,
                                int32_t *pcol, double *pval); /* returns omega */
int64_t orc_rap_nnz(int64_t n, const int64_t *rowptr, const int32_t *col, int64_t nc,
                    const int64_t *prow, const int32_t *pcol);
void orc_rap(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, int64_t nc,
             const int64_t *prow, const int32_t *pcol, const double *pval, int64_t *crow,
             int32_t *ccol, double *cval);

/* ---- decoupled greedy aggregation (Vanek-Mandel-Brezina) ---- */
int64_t orc_vmb_aggregate(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                          double theta, int64_t block, int32_t *agg);

/* ---- multicolour Gauss-Seidel ---- */
int orc_greedy_colors(int64_t n, const int64_t *rowptr, const int32_t *col, int32_t *color);
void orc_mcgs_sweep(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                    const int32_t *color, int ncolor, int dir, const double *b, double *x);

/* ---- AMG hierarchy (opaque) ---- */
typedef struct orc_amg orc_amg;
int orc_amg_build(const orc_opts *O, int64_t n, const int64_t *rowptr, const int32_t *col,
                  const double *val, orc_amg **out);
int orc_amg_update_fine(orc_amg *H, const double *val); /* new fine values, same pattern */
int orc_amg_levels(const orc_amg *H);
void orc_amg_level_info(const orc_amg *H, int l, int64_t *n, int64_t *nnz);
void orc_amg_level_export(const orc_amg *H, int l, int64_t *rowptr, int32_t *col, double *val,
                          int32_t *agg /* nullable; only for l < levels-1 */);
int orc_amg_coarse_is_dense(const orc_amg *H);
int64_t orc_amg_prolongator_nnz(const orc_amg *H, int l); /* 0 unless smoothed and l < levels-1 */
void orc_amg_prolongator_export(const orc_amg *H, int l, int64_t *prow, int32_t *pcol,
                                double *pval);
void orc_amg_apply(const orc_amg *H, const double *b, double *x);
void orc_amg_destroy(orc_amg *H);

/* ---- GMRES (right-preconditioned by the hierarchy, or unpreconditioned if H is NULL) ---- */
int orc_gmres(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
              const orc_amg *H, const double *b, double *x, int restart, double eta, int maxit,
              int *its_out, double *relres_out);

/* ---- time stepping ---- */
typedef struct orc_solver orc_solver;
int orc_solver_create(const orc_problem *P, const orc_opts *O, const double *Ks,
                      orc_solver **out);
int orc_solver_step(orc_solver *S, double *p, orc_stats *st);
void orc_solver_destroy(orc_solver *S);

/* ---- record of the Newton controller (Section 3), one entry per attempt ---- */
/* An attempt is one pass of the rebuild test, the linear solve and the line    */
/* search; an attempt that ends with a retry request is followed by another    */
/* attempt at the same Newton iterate.                                          */
#define ORC_TRACE_TRIALS 48
#define ORC_EV_ACCEPT 0        /* step accepted */
#define ORC_EV_ACCEPT_SHORT 1  /* step accepted, shorter than scsteptol, stale J: rebuild next */
#define ORC_EV_RETRY_GMRES 2   /* GMRES failed with a stale J */
#define ORC_EV_RETRY_SLOPE 3   /* d no descent direction, stale J */
#define ORC_EV_RETRY_LS 4      /* line search failed, stale J */
#define ORC_EV_FAIL_SLOPE 5    /* d no descent direction, fresh J: LINSOLVE_FAIL */
#define ORC_EV_FAIL_LS 6       /* line search failed, fresh J: LINESEARCH_FAIL */
#define ORC_EV_STALL 7         /* step shorter than scsteptol with a fresh J: STEP_TOO_SMALL */
#define ORC_EV_FAIL_OTHER 8    /* set-up error or non-finite residual */
#define ORC_RB_NOJ 1           /* rebuild reasons (bits) */
#define ORC_RB_MSBSET 2
#define ORC_RB_BIGSTEP 4
#define ORC_RB_RETRY 8
typedef struct {
    int step;         /* time step, counted from 0 since the solver was created */
    int newton_it;    /* accepted Newton iterations of this step before the attempt */
    int since_build;  /* iterations since the last rebuild, before the rebuild test */
    int reason;       /* ORC_RB_* bits that held at the rebuild test (0: J re-used) */
    int gmres_its, gmres_conv, truncated, outcome;
    int ntrial;       /* line-search trials u + lam d in order, the full step lam = 1 first */
    int nback;        /* of which backtracking trials (the rest lengthen a full step) */
    double f0;        /* 0.5 ||Phi(u)||_2^2 at the attempt's iterate */
    double slope;     /* Phi(u)^T J d */
    double dnorm2, dnorminf;  /* of the (possibly truncated) correction d */
    double rel_d;     /* max_i |d_i| / max(|u_i|, 1) */
    double mxstep;    /* maximum step length */
    double lam, f_acc;        /* accepted step and 0.5 ||Phi||^2 there (lam 0 if none) */
    double step_inf, step_rel, fnorm_inf;  /* ||lam d||_inf, its relative length, ||Phi||_inf after */
    double trial_lam[ORC_TRACE_TRIALS], trial_f[ORC_TRACE_TRIALS];  /* f = 0.5 ||Phi||^2 */
} orc_newton_event;
/* Record the attempts of the following orc_solver_step calls into buf (cap  */
/* entries; NULL stops recording).  Returns the number recorded since armed,  */
/* which may exceed cap (the excess is dropped).                              */
void orc_solver_trace(orc_solver *S, orc_newton_event *buf, int cap);
int orc_solver_trace_len(const orc_solver *S);
/* The last Newton iterate of the most recent step (its state also when the */
/* step failed and p was left at the previous level).                       */
void orc_solver_iterate(const orc_solver *S, double *u);

#endif
