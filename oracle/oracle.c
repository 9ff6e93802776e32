/*
 * Plain FP64 CPU oracle for the Richards-equation solver of arXiv 2112.05051.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product library, with which
 * it shares no code.  Every function is a direct, unblocked transcription of
 * the definition it cites; where the paper is silent the reading used is
 * stated in the comment.
 *
 * Pinning: the laws, residual, Jacobian and auxiliary matrix are pinned by the
 * paper's printed Jacobian entries, central finite differences, mass balance,
 * the hydrostatic steady state and closed-form spectra (tests/test_oracle_*).
 * Matching is pinned by brute force on tiny graphs, the V-cycle by the
 * recursion of Section 5.2 written as dense matrices, GMRES by finite
 * termination; the smoothed prolongator by the 1-D hat functions; the
 * multicolour Gauss-Seidel sweeps by triangular solves in the colour-sorted
 * ordering; the greedy aggregation by hand-worked 1-D and 2-D cases and its
 * invariants.  The Newton / line-search control flow (orc_solver_step)
 * records every attempt (orc_solver_trace); the tests recompute from that
 * record, independently, the Armijo condition at every accepted step (with
 * f re-evaluated at the returned states), each backtracking step as the
 * minimiser of the quadratic or cubic model (numpy solves and polynomial
 * roots), the beta lengthening, the rebuild schedule of
 * eq. (jacobian_update_condition) and the outcome of every attempt.  The
 * coarsest-level l1 sweeps are pinned by the dense sum of the sweep
 * operators.  Iteration counts are "parity unpinned" against the paper,
 * whose workload differs.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* Loops whose iterations are independent (one cell, row or vector element  */
/* each) may run on several threads in the OpenMP build of this file         */
/* (liboracle_omp.so, used only to time the oracle on all host cores).       */
/* Reductions (dot products, norms) and scatter-adds (restriction, Galerkin  */
/* products) stay serial, so both builds give the same results bit for bit.  */
#ifdef _OPENMP
#define ORC_PARALLEL_FOR _Pragma("omp parallel for schedule(static)")
#else
#define ORC_PARALLEL_FOR
#endif

/* ------------------------------------------------------------------------ */
/* Constitutive laws: Section 2, eq. (s(p)) with rho*phi = 1 so s is the     */
/* volumetric water content theta, eq. (K(p)) with K_s per cell, derivatives  */
/* eq. (derivativeofcoefficients) with sgn(p) = -1 for p < 0.  Saturated      */
/* regime p >= 0 (Section 2): K = K_s, theta = theta_s, both derivatives 0.  */
/* ------------------------------------------------------------------------ */
void orc_laws(const orc_problem *P, double p, double Ks, double out[4])
{
    if (p >= 0.0) {
        out[0] = P->theta_s;
        out[1] = 0.0;
        out[2] = Ks;
        out[3] = 0.0;
        return;
    }
    double a = -p; /* |p| */
    double ab = pow(a, P->beta);
    double ag = pow(a, P->gamma);
    double ds = P->theta_s - P->theta_r;
    double dt_den = P->alpha + ab;
    double dk_den = P->A + ag;
    out[0] = P->alpha * ds / dt_den + P->theta_r;
    out[1] = P->alpha * P->beta * ds * pow(a, P->beta - 1.0) / (dt_den * dt_den);
    out[2] = Ks * P->A / dk_den;
    out[3] = Ks * P->A * P->gamma * pow(a, P->gamma - 1.0) / (dk_den * dk_den);
}

void orc_laws_array(const orc_problem *P, int64_t n, const double *p, const double *Ks,
                    double *out /* n x 4 */)
{
    for (int64_t c = 0; c < n; c++)
        orc_laws(P, p[c], Ks[c], out + 4 * c);
}

void orc_theta(const orc_problem *P, const double *p, double *theta)
{
    int64_t n = (int64_t)P->nx * P->ny * P->nz;
    ORC_PARALLEL_FOR
    for (int64_t c = 0; c < n; c++) {
        double L[4];
        orc_laws(P, p[c], 1.0, L);
        theta[c] = L[0];
    }
}

/* ------------------------------------------------------------------------ */
/* Grid faces.  Face f = 0..5 is -x,+x,-y,+y,-z,+z.  A face either joins two */
/* unknowns (interior), or touches a Dirichlet boundary node whose head is    */
/* the face's value (or the patch value where the optional Dirichlet patch  */
/* covers the node: the square of zero head on the top face of Section 6's  */
/* 3-D test) and whose K_s is the adjacent cell's (the paper treats K_s as a */
/* constant), or is a no-flux face, which carries no flux at all.            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int interior;
    int64_t n;
    double pn, Ksn, h;
    int axis, dir;
} face_t;

static int face_info(const orc_problem *P, int i, int j, int k, int f, const double *p,
                     const double *Ks, face_t *F)
{
    int axis = f / 2, dir = (f & 1) ? 1 : -1;
    int ii = i, jj = j, kk = k;
    if (axis == 0) ii += dir;
    else if (axis == 1) jj += dir;
    else kk += dir;
    F->axis = axis;
    F->dir = dir;
    F->h = axis == 0 ? P->hx : (axis == 1 ? P->hy : P->hz);
    int64_t c = (int64_t)i + (int64_t)P->nx * ((int64_t)j + (int64_t)P->ny * k);
    if (ii >= 0 && ii < P->nx && jj >= 0 && jj < P->ny && kk >= 0 && kk < P->nz) {
        F->interior = 1;
        F->n = (int64_t)ii + (int64_t)P->nx * ((int64_t)jj + (int64_t)P->ny * kk);
        F->pn = p[F->n];
        F->Ksn = Ks[F->n];
        return 1;
    }
    if (P->bc_type[f] == ORC_DIRICHLET) {
        F->interior = 0;
        F->n = -1;
        F->pn = P->bc_value[f];
        if (f == P->patch_face) {
            /* the boundary node's coordinates along the face's two axes */
            double u = axis == 0 ? (j + 1) * P->hy : (i + 1) * P->hx;
            double v = axis == 2 ? (j + 1) * P->hy : (k + 1) * P->hz;
            if (u >= P->patch_lo[0] && u <= P->patch_hi[0] && v >= P->patch_lo[1] && v <= P->patch_hi[1])
                F->pn = P->patch_value;
        }
        F->Ksn = Ks[c];
        return 1;
    }
    return 0;
}

/* Gauss-Legendre rule with ORC_GL nodes on [0, 1]: the nodes are the roots */
/* of the Legendre polynomial P_n found by Newton's method from the usual    */
/* cosine estimates, w_i = 2 / ((1 - x_i^2) P_n'(x_i)^2) (halved for [0,1]). */
#define ORC_GL 16
static double gl_t[ORC_GL], gl_w[ORC_GL];
static int gl_ready = 0;

static void gl_init(void)
{
    if (gl_ready) return;
    const int n = ORC_GL;
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; i++) {
        double x = cos(pi * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        gl_t[i] = 0.5 * (1.0 - x);
        gl_w[i] = 1.0 / ((1.0 - x * x) * dp * dp);
    }
    gl_ready = 1;
}

/* Interface means (Section 2.1): arithmetic; upstream eq. (upstream_mean)  */
/* with L the lower-index side, U = L + e_d and ties (p_U - p_L = 0) taking  */
/* K_U; harmonic 2 K_L K_U / (K_L + K_U) (named in the abstract); geometric  */
/* sqrt(K_L K_U); integral mean: the average of K over the heads between    */
/* p_L and p_U, with K_s the arithmetic mean of the two cells' K_s (and     */
/* K(p_U) when the heads are equal, where the paper's printed "p_U" and the */
/* sign of its 1/(p_L - p_U) are typos), evaluated by the ORC_GL-point Gauss-*/
/* Legendre rule on [p_L, p_U] (no closed form for this K(p)); its          */
/* derivatives are those of the rule.  Returns the mean and its partial     */
/* derivatives w.r.t. the cell's and the neighbour's heads (the upstream    */
/* derivative does not differentiate the switch).  With mean_vertical >= 0 */
/* the z faces take that mean instead (Section 2.1's per-direction option). */
static void face_mean(const orc_problem *P, int axis, int dir, double pc, double Ksc, const double Lc[4],
                      double pn, double Ksn, const double Ln[4], double *Kf, double *dc, double *dn)
{
    int mean = (axis == 2 && P->mean_vertical >= 0) ? P->mean_vertical : P->mean;
    double Kc = Lc[2], dKc = Lc[3], Kn = Ln[2], dKn = Ln[3];
    if (mean == ORC_ARITH) {
        *Kf = 0.5 * (Kc + Kn);
        *dc = 0.5 * dKc;
        *dn = 0.5 * dKn;
    } else if (mean == ORC_HARMONIC) {
        double s = Kc + Kn;
        *Kf = 2.0 * Kc * Kn / s;
        *dc = 2.0 * Kn * Kn * dKc / (s * s);
        *dn = 2.0 * Kc * Kc * dKn / (s * s);
    } else if (mean == ORC_GEOMETRIC) {
        double g = sqrt(Kc * Kn);
        *Kf = g;
        *dc = 0.5 * Kn * dKc / g;
        *dn = 0.5 * Kc * dKn / g;
    } else if (mean == ORC_INTEGRAL) {
        gl_init();
        double pL = dir > 0 ? pc : pn, pU = dir > 0 ? pn : pc;
        double Ks = 0.5 * (dir > 0 ? Ksc + Ksn : Ksn + Ksc);
        double q = 0.0, qL = 0.0, qU = 0.0, L[4];
        for (int t = 0; t < ORC_GL; t++) {
            orc_laws(P, pL + (pU - pL) * gl_t[t], Ks, L);
            q += gl_w[t] * L[2];
            qL += gl_w[t] * (1.0 - gl_t[t]) * L[3];
            qU += gl_w[t] * gl_t[t] * L[3];
        }
        *Kf = q;
        *dc = dir > 0 ? qL : qU;
        *dn = dir > 0 ? qU : qL;
    } else { /* upstream */
        double pU, pL;
        if (dir > 0) { pU = pn; pL = pc; }
        else { pU = pc; pL = pn; }
        int take_U = (pU - pL >= 0.0);
        int take_n = (dir > 0) ? take_U : !take_U;
        if (take_n) { *Kf = Kn; *dc = 0.0; *dn = dKn; }
        else { *Kf = Kc; *dc = dKc; *dn = 0.0; }
    }
}

void orc_face_mean(const orc_problem *P, int axis, int dir, double pc, double Ksc, double pn,
                   double Ksn, double out[3])
{
    double Lc[4], Ln[4];
    orc_laws(P, pc, Ksc, Lc);
    orc_laws(P, pn, Ksn, Ln);
    face_mean(P, axis, dir, pc, Ksc, Lc, pn, Ksn, Ln, &out[0], &out[1], &out[2]);
}

/* ------------------------------------------------------------------------ */
/* Residual, eq. (dynamic_of_the_problem) with f = 0, written per face: the  */
/* diffusive flux -K^AV (p_n - p_c)/h^2 and, on z faces, the gravity part    */
/* s*(-(K_c+K_n)/(2 h_z)) with s = +1 for the face above.  Summed over the   */
/* two z faces of an interior cell this is exactly the paper's centred term  */
/* -(K_{k+1} - K_{k-1})/(2 h_z); at a no-flux face nothing is added.        */
/* ------------------------------------------------------------------------ */
void orc_residual(const orc_problem *P, const double *Ks, const double *p, const double *theta_old,
                  double *F)
{
    gl_init(); /* before any thread evaluates an integral mean */
    ORC_PARALLEL_FOR
    for (int k = 0; k < P->nz; k++)
        for (int j = 0; j < P->ny; j++)
            for (int i = 0; i < P->nx; i++) {
                double Lc[4], Ln[4];
                int64_t c = (int64_t)i + (int64_t)P->nx * ((int64_t)j + (int64_t)P->ny * k);
                orc_laws(P, p[c], Ks[c], Lc);
                double acc = (Lc[0] - theta_old[c]) / P->dt;
                for (int f = 0; f < 6; f++) {
                    face_t fc;
                    if (!face_info(P, i, j, k, f, p, Ks, &fc)) continue;
                    orc_laws(P, fc.pn, fc.Ksn, Ln);
                    double Kf, dc, dn;
                    face_mean(P, fc.axis, fc.dir, p[c], Ks[c], Lc, fc.pn, fc.Ksn, Ln, &Kf, &dc, &dn);
                    acc += -Kf * (fc.pn - p[c]) / (fc.h * fc.h);
                    if (fc.axis == 2) acc += fc.dir * (-(Lc[2] + Ln[2]) / (2.0 * P->hz));
                }
                F[c] = acc;
            }
}

/* Fixed 7-point pattern: the cell and its interior neighbours, columns in  */
/* increasing order (-z, -y, -x, c, +x, +y, +z).                            */
int64_t orc_pattern_nnz(const orc_problem *P)
{
    int64_t nnz = 0;
    for (int k = 0; k < P->nz; k++)
        for (int j = 0; j < P->ny; j++)
            for (int i = 0; i < P->nx; i++)
                nnz += 1 + (i > 0) + (i < P->nx - 1) + (j > 0) + (j < P->ny - 1) + (k > 0) +
                       (k < P->nz - 1);
    return nnz;
}

static const int ORDER_LO[3] = {4, 2, 0}; /* -z, -y, -x */
static const int ORDER_HI[3] = {1, 3, 5}; /* +x, +y, +z */

/* which = 0: Jacobian of the residual; which = 1: auxiliary matrix; which =  */
/* 2: auxiliary matrix whose diagonal also takes the flux-derivative terms   */
/* -(p_n - p_c)/h^2 dK^AV/dp_c of the diffusion operator's Jacobian (the     */
/* off-diagonal ones are left out so the matrix stays symmetric).           */
static void assemble(const orc_problem *P, const double *Ks, const double *p, int which,
                     int64_t *rowptr, int32_t *col, double *val)
{
    /* row c holds the cell and its neighbours inside the grid */
    rowptr[0] = 0;
    for (int k = 0; k < P->nz; k++)
        for (int j = 0; j < P->ny; j++)
            for (int i = 0; i < P->nx; i++) {
                int64_t c = (int64_t)i + (int64_t)P->nx * ((int64_t)j + (int64_t)P->ny * k);
                rowptr[c + 1] = rowptr[c] + 1 + (i > 0) + (i + 1 < P->nx) + (j > 0) + (j + 1 < P->ny) +
                                (k > 0) + (k + 1 < P->nz);
            }
    gl_init(); /* before any thread evaluates an integral mean */
    ORC_PARALLEL_FOR
    for (int k = 0; k < P->nz; k++)
        for (int j = 0; j < P->ny; j++)
            for (int i = 0; i < P->nx; i++) {
                double Lc[4], Ln[4];
                int64_t c = (int64_t)i + (int64_t)P->nx * ((int64_t)j + (int64_t)P->ny * k);
                int64_t e = rowptr[c];
                orc_laws(P, p[c], Ks[c], Lc);
                double diag = Lc[1] / P->dt;
                double off[6];
                int64_t nb[6];
                int has[6] = {0, 0, 0, 0, 0, 0};
                for (int f = 0; f < 6; f++) {
                    face_t fc;
                    if (!face_info(P, i, j, k, f, p, Ks, &fc)) continue;
                    orc_laws(P, fc.pn, fc.Ksn, Ln);
                    double Kf, dc, dn;
                    face_mean(P, fc.axis, fc.dir, p[c], Ks[c], Lc, fc.pn, fc.Ksn, Ln, &Kf, &dc, &dn);
                    double h2 = fc.h * fc.h;
                    double dp = fc.pn - p[c];
                    if (which == 0) {
                        /* d/dp_c and d/dp_n of -Kf*dp/h^2 + [z] s*(-(Kc+Kn)/(2hz)) */
                        diag += Kf / h2 - dp / h2 * dc;
                        if (fc.axis == 2) diag += -fc.dir * Lc[3] / (2.0 * P->hz);
                        if (fc.interior) {
                            double v = -Kf / h2 - dp / h2 * dn;
                            if (fc.axis == 2) v += -fc.dir * Ln[3] / (2.0 * P->hz);
                            off[f] = v;
                            nb[f] = fc.n;
                            has[f] = 1;
                        }
                    } else {
                        /* Section 4 / 5.2: Jacobian of the diffusion-only operator with the
                         * conductivity frozen (q_prec = -K grad p), plus the time term. */
                        diag += Kf / h2;
                        if (which == 2) diag += -dp / h2 * dc;
                        if (fc.interior) {
                            off[f] = -Kf / h2;
                            nb[f] = fc.n;
                            has[f] = 1;
                        }
                    }
                }
                for (int t = 0; t < 3; t++)
                    if (has[ORDER_LO[t]]) {
                        col[e] = (int32_t)nb[ORDER_LO[t]];
                        val[e++] = off[ORDER_LO[t]];
                    }
                col[e] = (int32_t)c;
                val[e++] = diag;
                for (int t = 0; t < 3; t++)
                    if (has[ORDER_HI[t]]) {
                        col[e] = (int32_t)nb[ORDER_HI[t]];
                        val[e++] = off[ORDER_HI[t]];
                    }
            }
}

void orc_jacobian(const orc_problem *P, const double *Ks, const double *p, int64_t *rowptr,
                  int32_t *col, double *val)
{
    assemble(P, Ks, p, 0, rowptr, col, val);
}

void orc_auxiliary(const orc_problem *P, const double *Ks, const double *p, int64_t *rowptr,
                   int32_t *col, double *val)
{
    assemble(P, Ks, p, 1, rowptr, col, val);
}

void orc_auxiliary_dflux(const orc_problem *P, const double *Ks, const double *p, int64_t *rowptr,
                         int32_t *col, double *val)
{
    assemble(P, Ks, p, 2, rowptr, col, val);
}

void orc_csr_matvec(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                    const double *x, double *y)
{
    ORC_PARALLEL_FOR
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) s += val[e] * x[col[e]];
        y[i] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Pairwise matching (Section 5.2, SMATCH: aggregation by maximum-weight     */
/* graph matching; the weight is not printed in the paper).  Reading: edge   */
/* {i,j}, i<j, with a_ij != 0 in row i has weight                            */
/*     w_ij = 1 - 2 a_ij / (a_ii + a_jj)                                      */
/* (the matching weight of D'Ambra-Vassilevski with a constant smooth        */
/* vector).  Edges are taken greedily in the strict order (w desc, i asc,    */
/* j asc); a vertex left unmatched is a singleton.  Coarse indices are given */
/* in increasing order of the smallest member.                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    double w;
    int64_t i, j;
} edge_t;

static int edge_cmp(const void *a, const void *b)
{
    const edge_t *x = (const edge_t *)a, *y = (const edge_t *)b;
    if (x->w > y->w) return -1;
    if (x->w < y->w) return 1;
    if (x->i < y->i) return -1;
    if (x->i > y->i) return 1;
    if (x->j < y->j) return -1;
    if (x->j > y->j) return 1;
    return 0;
}

int64_t orc_match_sweep(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                        int32_t *agg)
{
    double *diag = (double *)calloc((size_t)n, sizeof(double));
    int64_t *mate = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t ne = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
            if (col[e] == i) diag[i] = val[e];
            else if (col[e] > i && val[e] != 0.0) ne++;
        }
    edge_t *E = (edge_t *)malloc((size_t)(ne > 0 ? ne : 1) * sizeof(edge_t));
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
            int64_t j = col[e];
            if (j > i && val[e] != 0.0) {
                double w = 1.0 - (2.0 * val[e]) / (diag[i] + diag[j]);
                if (!isfinite(w)) continue;
                E[m].w = w;
                E[m].i = i;
                E[m].j = j;
                m++;
            }
        }
    qsort(E, (size_t)m, sizeof(edge_t), edge_cmp);
    for (int64_t i = 0; i < n; i++) mate[i] = -1;
    for (int64_t t = 0; t < m; t++)
        if (mate[E[t].i] < 0 && mate[E[t].j] < 0) {
            mate[E[t].i] = E[t].j;
            mate[E[t].j] = E[t].i;
        }
    int64_t nc = 0;
    for (int64_t i = 0; i < n; i++) {
        if (mate[i] < 0 || i < mate[i]) agg[i] = (int32_t)(nc++);
        else agg[i] = agg[mate[i]];
    }
    free(E);
    free(mate);
    free(diag);
    return nc;
}

/* Galerkin product with a piecewise-constant prolongator (Section 5.2,      */
/* M_{l+1} = P^T M_l P):  C_IJ = sum over i in I, j in J of a_ij.  The terms  */
/* are accumulated in a fixed order, fine rows ascending and each row in its */
/* column order, so that the result is reproducible bit for bit.            */
static void members_of(int64_t n, const int32_t *agg, int64_t nc, int64_t **mptr_out,
                       int64_t **mem_out)
{
    int64_t *mptr = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    int64_t *mem = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) mptr[agg[i] + 1]++;
    for (int64_t I = 0; I < nc; I++) mptr[I + 1] += mptr[I];
    int64_t *fill = (int64_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
    for (int64_t I = 0; I < nc; I++) fill[I] = mptr[I];
    for (int64_t i = 0; i < n; i++) mem[fill[agg[i]]++] = i;
    free(fill);
    *mptr_out = mptr;
    *mem_out = mem;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

int64_t orc_galerkin_nnz(int64_t n, const int64_t *rowptr, const int32_t *col, const int32_t *agg,
                         int64_t nc)
{
    int64_t *mptr, *mem;
    members_of(n, agg, nc, &mptr, &mem);
    int64_t *mark = (int64_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
    for (int64_t I = 0; I < nc; I++) mark[I] = -1;
    int64_t nnz = 0;
    for (int64_t I = 0; I < nc; I++)
        for (int64_t t = mptr[I]; t < mptr[I + 1]; t++) {
            int64_t i = mem[t];
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
                int64_t J = agg[col[e]];
                if (mark[J] != I) {
                    mark[J] = I;
                    nnz++;
                }
            }
        }
    free(mark);
    free(mptr);
    free(mem);
    return nnz;
}

void orc_galerkin(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                  const int32_t *agg, int64_t nc, int64_t *crow, int32_t *ccol, double *cval)
{
    int64_t *mptr, *mem;
    members_of(n, agg, nc, &mptr, &mem);
    int64_t *mark = (int64_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
    double *acc = (double *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(double));
    int32_t *list = (int32_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int32_t));
    for (int64_t I = 0; I < nc; I++) mark[I] = -1;
    int64_t e_out = 0;
    crow[0] = 0;
    for (int64_t I = 0; I < nc; I++) {
        int64_t len = 0;
        for (int64_t t = mptr[I]; t < mptr[I + 1]; t++) {
            int64_t i = mem[t];
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
                int32_t J = agg[col[e]];
                if (mark[J] != I) {
                    mark[J] = I;
                    acc[J] = 0.0;
                    list[len++] = J;
                }
                acc[J] += val[e];
            }
        }
        qsort(list, (size_t)len, sizeof(int32_t), cmp_i32);
        for (int64_t t = 0; t < len; t++) {
            ccol[e_out] = list[t];
            cval[e_out++] = acc[list[t]];
        }
        crow[I + 1] = e_out;
    }
    free(list);
    free(acc);
    free(mark);
    free(mptr);
    free(mem);
}

/* ------------------------------------------------------------------------ */
/* Smoothed aggregation (Section 5.2: the paper's two coarsening schemes,    */
/* DSVMB and SMATCH, both smooth the piecewise-constant prolongator of the   */
/* aggregates).  One damped-Jacobi step is applied to the tentative          */
/* prolongator P_t (P_t(i, agg(i)) = 1):                                     */
/*     P = (I - omega D^{-1} A) P_t,   D = diag(A),                          */
/*     omega = 4 / (3 rho),   rho = max_i sum_j |a_ij| / a_ii                */
/* (rho is the Gershgorin bound on the spectral radius of D^{-1} A; the     */
/* paper leaves the smoothing parameters to its cited methods).  Row i of P  */
/* has an entry for every aggregate J that row i of A touches:              */
/*     P_iJ = [agg(i) = J] - w_i t_iJ,   w_i = omega / a_ii,                 */
/*     t_iJ = sum of a_ik over the k of row i with agg(k) = J.               */
/* The coarse matrix is C = P^T (A P) (eq. (Vcycle)'s M_{l+1} = P^T M_l P),  */
/* formed as Q = A P and then C = P^T Q.  Every sum runs in a fixed order:  */
/* t_iJ and Q_iJ over k in row i's column order, C_IJ over i ascending, so   */
/* that the result is reproducible bit for bit.  Patterns are structural:    */
/* an entry whose terms cancel is kept with the value zero.                  */
/* ------------------------------------------------------------------------ */
static int64_t csr_find_diag(const int64_t *rowptr, const int32_t *col, int64_t i)
{
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++)
        if (col[e] == i) return e;
    return -1;
}

int64_t orc_smoothed_prolongator_nnz(int64_t n, const int64_t *rowptr, const int32_t *col,
                                     const int32_t *agg, int64_t nc)
{
    int64_t *mark = (int64_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
    for (int64_t J = 0; J < nc; J++) mark[J] = -1;
    int64_t nnz = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
            int32_t J = agg[col[e]];
            if (mark[J] != i) {
                mark[J] = i;
                nnz++;
            }
        }
    free(mark);
    return nnz;
}

double orc_smoothed_prolongator(int64_t n, const int64_t *rowptr, const int32_t *col,
                                const double *val, const int32_t *agg, int64_t nc, int64_t *prow,
                                int32_t *pcol, double *pval)
{
    double rho = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) s += fabs(val[e]);
        double r = s / val[csr_find_diag(rowptr, col, i)];
        if (r > rho) rho = r;
    }
    double omega = 4.0 / (3.0 * rho);
    int64_t *mark = (int64_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
    double *t = (double *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(double));
    int32_t *list = (int32_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int32_t));
    for (int64_t J = 0; J < nc; J++) mark[J] = -1;
    int64_t o = 0;
    prow[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        double w = omega / val[csr_find_diag(rowptr, col, i)];
        int64_t len = 0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
            int32_t J = agg[col[e]];
            if (mark[J] != i) {
                mark[J] = i;
                t[J] = 0.0;
                list[len++] = J;
            }
            t[J] += val[e];
        }
        qsort(list, (size_t)len, sizeof(int32_t), cmp_i32);
        for (int64_t a = 0; a < len; a++) {
            int32_t J = list[a];
            pcol[o] = J;
            pval[o++] = (J == agg[i] ? 1.0 : 0.0) - w * t[J];
        }
        prow[i + 1] = o;
    }
    free(list);
    free(t);
    free(mark);
    return omega;
}

/* Q = A P (n x nc) in CSR with sorted columns; values when qval != NULL. */
static int64_t spgemm_rows(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                           int64_t nc, const int64_t *prow, const int32_t *pcol, const double *pval,
                           int64_t *qrow, int32_t *qcol, double *qval)
{
    int64_t *mark = (int64_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
    double *acc = (double *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(double));
    int32_t *list = (int32_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int32_t));
    for (int64_t J = 0; J < nc; J++) mark[J] = -1;
    int64_t o = 0;
    if (qrow) qrow[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t len = 0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
            int64_t k = col[e];
            for (int64_t f = prow[k]; f < prow[k + 1]; f++) {
                int32_t J = pcol[f];
                if (mark[J] != i) {
                    mark[J] = i;
                    acc[J] = 0.0;
                    list[len++] = J;
                }
                if (qval) acc[J] += val[e] * pval[f];
            }
        }
        if (qrow) {
            qsort(list, (size_t)len, sizeof(int32_t), cmp_i32);
            for (int64_t a = 0; a < len; a++) {
                qcol[o + a] = list[a];
                if (qval) qval[o + a] = acc[list[a]];
            }
            qrow[i + 1] = o + len;
        }
        o += len;
    }
    free(list);
    free(acc);
    free(mark);
    return o;
}

/* P^T in CSR: row I lists the i with P_iI present, ascending. */
static void transpose_csr(int64_t n, int64_t nc, const int64_t *prow, const int32_t *pcol,
                          const double *pval, int64_t *trow, int64_t *tcol, double *tval)
{
    for (int64_t I = 0; I <= nc; I++) trow[I] = 0;
    for (int64_t f = 0; f < prow[n]; f++) trow[pcol[f] + 1]++;
    for (int64_t I = 0; I < nc; I++) trow[I + 1] += trow[I];
    int64_t *fill = (int64_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
    for (int64_t I = 0; I < nc; I++) fill[I] = trow[I];
    for (int64_t i = 0; i < n; i++)
        for (int64_t f = prow[i]; f < prow[i + 1]; f++) {
            int64_t o = fill[pcol[f]]++;
            tcol[o] = i;
            tval[o] = pval[f];
        }
    free(fill);
}

/* C = P^T Q: C_IJ = sum over i ascending of P_iI Q_iJ. */
static int64_t pt_times_q(int64_t n, int64_t nc, const int64_t *trow, const int64_t *tcol,
                          const double *tval, const int64_t *qrow, const int32_t *qcol,
                          const double *qval, int64_t *crow, int32_t *ccol, double *cval)
{
    int64_t *mark = (int64_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
    double *acc = (double *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(double));
    int32_t *list = (int32_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int32_t));
    for (int64_t J = 0; J < nc; J++) mark[J] = -1;
    int64_t o = 0;
    if (crow) crow[0] = 0;
    for (int64_t I = 0; I < nc; I++) {
        int64_t len = 0;
        for (int64_t t = trow[I]; t < trow[I + 1]; t++) {
            int64_t i = tcol[t];
            for (int64_t f = qrow[i]; f < qrow[i + 1]; f++) {
                int32_t J = qcol[f];
                if (mark[J] != I) {
                    mark[J] = I;
                    acc[J] = 0.0;
                    list[len++] = J;
                }
                if (cval) acc[J] += tval[t] * qval[f];
            }
        }
        if (crow) {
            qsort(list, (size_t)len, sizeof(int32_t), cmp_i32);
            for (int64_t a = 0; a < len; a++) {
                ccol[o + a] = list[a];
                if (cval) cval[o + a] = acc[list[a]];
            }
            crow[I + 1] = o + len;
        }
        o += len;
    }
    free(list);
    free(acc);
    free(mark);
    return o;
}

/* Shared driver of orc_rap_nnz / orc_rap: returns nnz(C); fills C when crow. */
static int64_t rap(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                   int64_t nc, const int64_t *prow, const int32_t *pcol, const double *pval,
                   int64_t *crow, int32_t *ccol, double *cval)
{
    int64_t qnnz = spgemm_rows(n, rowptr, col, NULL, nc, prow, pcol, NULL, NULL, NULL, NULL);
    int64_t *qrow = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t *qcol = (int32_t *)malloc((size_t)(qnnz > 0 ? qnnz : 1) * sizeof(int32_t));
    double *qval = pval ? (double *)malloc((size_t)(qnnz > 0 ? qnnz : 1) * sizeof(double)) : NULL;
    spgemm_rows(n, rowptr, col, val, nc, prow, pcol, pval, qrow, qcol, qval);
    int64_t pnnz = prow[n];
    int64_t *trow = (int64_t *)malloc((size_t)(nc + 1) * sizeof(int64_t));
    int64_t *tcol = (int64_t *)malloc((size_t)(pnnz > 0 ? pnnz : 1) * sizeof(int64_t));
    double *tval = (double *)calloc((size_t)(pnnz > 0 ? pnnz : 1), sizeof(double));
    transpose_csr(n, nc, prow, pcol, pval ? pval : tval, trow, tcol, tval);
    int64_t cnnz = pt_times_q(n, nc, trow, tcol, tval, qrow, qcol, qval, crow, ccol, cval);
    free(tval);
    free(tcol);
    free(trow);
    free(qval);
    free(qcol);
    free(qrow);
    return cnnz;
}

int64_t orc_rap_nnz(int64_t n, const int64_t *rowptr, const int32_t *col, int64_t nc,
                    const int64_t *prow, const int32_t *pcol)
{
    return rap(n, rowptr, col, NULL, nc, prow, pcol, NULL, NULL, NULL, NULL);
}

void orc_rap(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, int64_t nc,
             const int64_t *prow, const int32_t *pcol, const double *pval, int64_t *crow,
             int32_t *ccol, double *cval)
{
    rap(n, rowptr, col, val, nc, prow, pcol, pval, crow, ccol, cval);
}

/* ------------------------------------------------------------------------ */
/* AMG hierarchy (Section 5.2).  The aggregates of level l come from        */
/* `amg_sweeps` pairwise matching sweeps, each sweep matching the Galerkin  */
/* product of the previous one, so aggregates hold at most 2^sweeps         */
/* unknowns (the paper caps SMATCH aggregates at 8, i.e. three sweeps).     */
/* The stored coarse matrix is the Galerkin product of level l with the     */
/* composed aggregates (M_{l+1} = P^T M_l P, piecewise-constant P).         */
/* Coarsening stops when a level has at most amg_coarse_size rows, when     */
/* amg_max_levels levels exist, or when the next level would keep more than  */
/* half of the rows while the current one fits the dense coarsest solver.   */
/* Re-use (Section 6): the aggregates are kept for the whole run; later     */
/* rebuilds refresh the fine matrix and its smoother and, when amg_refresh  */
/* is set (the reading used by default), recompute every coarse           */
/* matrix from the new fine one with the same aggregates.                   */
/* The first amg_smoothed levels (from the finest) take the smoothed       */
/* prolongator of orc_smoothed_prolongator and the coarse matrix P^T A P   */
/* of orc_rap; the aggregates still come from the matching sweeps on       */
/* piecewise-constant products, and a refresh recomputes P (with its       */
/* omega) and P^T A P.                                                      */
/* Smoother: l1-Jacobi, D_ii = sum_j |a_ij| (reading of the paper's "l1-     */
/* Jacobi"); with smoother = 1 the finest level takes one multicolour        */
/* Gauss-Seidel sweep instead (orc_mcgs_sweep: backward before, forward      */
/* after the coarse correction, as the paper's experiments of Section 6 use  */
/* backward/forward Gauss-Seidel), the coarser levels keep l1-Jacobi.        */
/* Coarsest: dense Cholesky when n <= coarse_dense_max, else                 */
/* coarse_l1_sweeps l1-Jacobi sweeps from zero (both keep M^{-1} linear).    */
/* ------------------------------------------------------------------------ */
#define ORC_MAXLEV 32
struct orc_amg {
    int nlev;
    int refresh;
    orc_csr A[ORC_MAXLEV];
    int32_t *agg[ORC_MAXLEV];
    orc_csr P[ORC_MAXLEV]; /* smoothed prolongator of level l (n_l rows), or empty */
    double *l1[ORC_MAXLEV];
    int smoother;   /* 1: multicolour Gauss-Seidel on level 0 */
    int32_t *color; /* level-0 colours (smoother 1) */
    int ncolor;
    int dense;
    double *chol; /* n_c x n_c, row-major lower factor */
    int coarse_sweeps;
};

static void csr_free(orc_csr *A)
{
    free(A->rowptr);
    free(A->col);
    free(A->val);
    A->rowptr = NULL;
    A->col = NULL;
    A->val = NULL;
}

/* ------------------------------------------------------------------------ */
/* Decoupled greedy aggregation: the DSVMB coarsening of Section 5.2 (the    */
/* smoothed aggregation of Vanek, Mandel and Brezina, each process          */
/* aggregating its own rows and ignoring couplings to other processes).     */
/* Reading: the "processes" are consecutive blocks of `block` rows; j is     */
/* strongly coupled to i when |a_ij| >= theta sqrt(a_ii a_jj) (j != i, same  */
/* block).  Within a block, rows in index order:                            */
/*  phase 1: a row whose strong neighbours are all unaggregated (and itself  */
/*           too) starts an aggregate holding it and those neighbours;      */
/*  phase 2: every row still free joins the phase-1 aggregate of its         */
/*           strongest strong neighbour that phase 1 aggregated (ties: the   */
/*           lowest index);                                                 */
/*  phase 3: every row still free starts an aggregate holding it and its    */
/*           strong neighbours that are still free.                         */
/* Aggregates are numbered block by block in order of creation.  Returns    */
/* the number of aggregates.                                                 */
/* ------------------------------------------------------------------------ */
int64_t orc_vmb_aggregate(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                          double theta, int64_t block, int32_t *agg)
{
    double *diag = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    int32_t *p1 = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < n; i++) {
        diag[i] = 0.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++)
            if (col[e] == i) diag[i] = val[e];
        agg[i] = -1;
    }
    int64_t nc = 0;
    for (int64_t b0 = 0; b0 < n; b0 += block) {
        int64_t b1 = b0 + block < n ? b0 + block : n;
#define STRONG(i, e) (col[e] != (i) && col[e] >= b0 && col[e] < b1 && \
                      fabs(val[e]) >= theta * sqrt(fabs(diag[i] * diag[col[e]])))
        for (int64_t i = b0; i < b1; i++) { /* phase 1 */
            int ok = agg[i] < 0;
            for (int64_t e = rowptr[i]; ok && e < rowptr[i + 1]; e++)
                if (STRONG(i, e) && agg[col[e]] >= 0) ok = 0;
            if (!ok) continue;
            agg[i] = (int32_t)nc;
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++)
                if (STRONG(i, e)) agg[col[e]] = (int32_t)nc;
            nc++;
        }
        for (int64_t i = b0; i < b1; i++) p1[i] = agg[i];
        for (int64_t i = b0; i < b1; i++) { /* phase 2 */
            if (agg[i] >= 0) continue;
            double best = -1.0;
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
                if (!STRONG(i, e) || p1[col[e]] < 0) continue;
                double s = fabs(val[e]) / sqrt(fabs(diag[i] * diag[col[e]]));
                if (s > best) {
                    best = s;
                    agg[i] = p1[col[e]];
                }
            }
        }
        for (int64_t i = b0; i < b1; i++) { /* phase 3 */
            if (agg[i] >= 0) continue;
            agg[i] = (int32_t)nc;
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++)
                if (STRONG(i, e) && agg[col[e]] < 0) agg[col[e]] = (int32_t)nc;
            nc++;
        }
#undef STRONG
    }
    free(diag);
    free(p1);
    return nc;
}

/* ------------------------------------------------------------------------ */
/* Multicolour Gauss-Seidel (the GPU form of the paper's hybrid Gauss-Seidel */
/* smoother of Section 5.2 / Section 6).  Colouring: greedy in index order,  */
/* colour(i) = the smallest colour no neighbour j < i has; on the 7-point    */
/* grid graph in x-fastest order this is the red-black parity (i+j+k) mod 2. */
/* A sweep visits the colours in ascending (forward, dir = +1) or descending */
/* (backward, dir = -1) order, rows of one colour in index order or its      */
/* reverse, and sets x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii in place: a  */
/* Gauss-Seidel sweep in the colour-sorted ordering.                          */
/* ------------------------------------------------------------------------ */
int orc_greedy_colors(int64_t n, const int64_t *rowptr, const int32_t *col, int32_t *color)
{
    int ncolor = 0;
    int64_t maxdeg = 1;
    for (int64_t i = 0; i < n; i++)
        if (rowptr[i + 1] - rowptr[i] + 1 > maxdeg) maxdeg = rowptr[i + 1] - rowptr[i] + 1;
    char *used = (char *)calloc((size_t)maxdeg + 1, 1);
    for (int64_t i = 0; i < n; i++) {
        memset(used, 0, (size_t)maxdeg + 1);
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
            int64_t j = col[e];
            if (j < i && color[j] <= maxdeg) used[color[j]] = 1;
        }
        int c = 0;
        while (used[c]) c++;
        color[i] = c;
        if (c + 1 > ncolor) ncolor = c + 1;
    }
    free(used);
    return ncolor;
}

void orc_mcgs_sweep(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                    const int32_t *color, int ncolor, int dir, const double *b, double *x)
{
    for (int k = 0; k < ncolor; k++) {
        int c = dir > 0 ? k : ncolor - 1 - k;
        for (int64_t t = 0; t < n; t++) {
            int64_t i = dir > 0 ? t : n - 1 - t;
            if (color[i] != c) continue;
            double s = b[i], d = 0.0;
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
                if (col[e] == i) d = val[e];
                else s -= val[e] * x[col[e]];
            }
            x[i] = s / d;
        }
    }
}

static void l1_diag(const orc_csr *A, double *d)
{
    for (int64_t i = 0; i < A->n; i++) {
        double s = 0.0;
        for (int64_t e = A->rowptr[i]; e < A->rowptr[i + 1]; e++) s += fabs(A->val[e]);
        d[i] = s;
    }
}

static int dense_cholesky(const orc_csr *A, double **out)
{
    int64_t n = A->n;
    double *L = (double *)calloc((size_t)(n * n > 0 ? n * n : 1), sizeof(double));
    for (int64_t i = 0; i < n; i++)
        for (int64_t e = A->rowptr[i]; e < A->rowptr[i + 1]; e++)
            if (A->col[e] <= i) L[i * n + A->col[e]] = A->val[e];
    for (int64_t j = 0; j < n; j++) {
        double s = L[j * n + j];
        for (int64_t k = 0; k < j; k++) s -= L[j * n + k] * L[j * n + k];
        if (!(s > 0.0)) {
            free(L);
            return ORC_NOT_SPD;
        }
        double d = sqrt(s);
        L[j * n + j] = d;
        for (int64_t i = j + 1; i < n; i++) {
            double t = L[i * n + j];
            for (int64_t k = 0; k < j; k++) t -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = t / d;
        }
    }
    *out = L;
    return ORC_OK;
}

static void csr_copy(const orc_csr *S, orc_csr *D)
{
    D->n = S->n;
    int64_t nnz = S->rowptr[S->n];
    D->rowptr = (int64_t *)malloc((size_t)(S->n + 1) * sizeof(int64_t));
    D->col = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    D->val = (double *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    memcpy(D->rowptr, S->rowptr, (size_t)(S->n + 1) * sizeof(int64_t));
    memcpy(D->col, S->col, (size_t)nnz * sizeof(int32_t));
    memcpy(D->val, S->val, (size_t)nnz * sizeof(double));
}

static void galerkin_alloc(const orc_csr *A, const int32_t *agg, int64_t nc, orc_csr *C)
{
    int64_t nnz = orc_galerkin_nnz(A->n, A->rowptr, A->col, agg, nc);
    C->n = nc;
    C->rowptr = (int64_t *)malloc((size_t)(nc + 1) * sizeof(int64_t));
    C->col = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    C->val = (double *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    orc_galerkin(A->n, A->rowptr, A->col, A->val, agg, nc, C->rowptr, C->col, C->val);
}

int orc_amg_build(const orc_opts *O, int64_t n, const int64_t *rowptr, const int32_t *col,
                  const double *val, orc_amg **out)
{
    orc_amg *H = (orc_amg *)calloc(1, sizeof(orc_amg));
    orc_csr fine = {n, (int64_t *)rowptr, (int32_t *)col, (double *)val};
    csr_copy(&fine, &H->A[0]);
    int l = 0;
    int maxl = O->amg_max_levels < ORC_MAXLEV ? O->amg_max_levels : ORC_MAXLEV;
    while (l + 1 < maxl && H->A[l].n > O->amg_coarse_size) {
        orc_csr cur = H->A[l];
        int own = 0; /* whether cur is a temporary */
        int32_t *comp = (int32_t *)malloc((size_t)(H->A[l].n > 0 ? H->A[l].n : 1) * sizeof(int32_t));
        for (int64_t i = 0; i < H->A[l].n; i++) comp[i] = (int32_t)i;
        if (O->amg_aggregation == 1) {
            const orc_csr *A = &H->A[l];
            int64_t nc = orc_vmb_aggregate(A->n, A->rowptr, A->col, A->val, O->amg_theta, O->amg_block, comp);
            if (nc == A->n) {
                free(comp);
                break;
            }
            cur.n = nc; /* only the size is used below */
            cur.rowptr = NULL;
            cur.col = NULL;
            cur.val = NULL;
            own = 1;
        }
        for (int s = 0; s < O->amg_sweeps && O->amg_aggregation != 1; s++) {
            int32_t *a = (int32_t *)malloc((size_t)(cur.n > 0 ? cur.n : 1) * sizeof(int32_t));
            int64_t nc = orc_match_sweep(cur.n, cur.rowptr, cur.col, cur.val, a);
            if (nc == cur.n) {
                free(a);
                break;
            }
            orc_csr nxt;
            galerkin_alloc(&cur, a, nc, &nxt);
            for (int64_t i = 0; i < H->A[l].n; i++) comp[i] = a[comp[i]];
            free(a);
            if (own) csr_free(&cur);
            cur = nxt;
            own = 1;
        }
        if (!own) {
            free(comp);
            break;
        }
        int64_t ncomp = cur.n;
        csr_free(&cur);
        /* a level that shrinks by less than half is not worth its cost when the
         * current level can already be solved directly: stop here instead */
        if (2 * ncomp > H->A[l].n && H->A[l].n <= O->coarse_dense_max) {
            free(comp);
            break;
        }
        H->agg[l] = comp;
        if (l < O->amg_smoothed) {
            const orc_csr *A = &H->A[l];
            orc_csr *Pl = &H->P[l];
            int64_t pnnz = orc_smoothed_prolongator_nnz(A->n, A->rowptr, A->col, comp, ncomp);
            Pl->n = A->n;
            Pl->rowptr = (int64_t *)malloc((size_t)(A->n + 1) * sizeof(int64_t));
            Pl->col = (int32_t *)malloc((size_t)(pnnz > 0 ? pnnz : 1) * sizeof(int32_t));
            Pl->val = (double *)malloc((size_t)(pnnz > 0 ? pnnz : 1) * sizeof(double));
            orc_smoothed_prolongator(A->n, A->rowptr, A->col, A->val, comp, ncomp, Pl->rowptr, Pl->col,
                                     Pl->val);
            int64_t cnnz = orc_rap_nnz(A->n, A->rowptr, A->col, ncomp, Pl->rowptr, Pl->col);
            orc_csr *C = &H->A[l + 1];
            C->n = ncomp;
            C->rowptr = (int64_t *)malloc((size_t)(ncomp + 1) * sizeof(int64_t));
            C->col = (int32_t *)malloc((size_t)(cnnz > 0 ? cnnz : 1) * sizeof(int32_t));
            C->val = (double *)malloc((size_t)(cnnz > 0 ? cnnz : 1) * sizeof(double));
            orc_rap(A->n, A->rowptr, A->col, A->val, ncomp, Pl->rowptr, Pl->col, Pl->val, C->rowptr,
                    C->col, C->val);
        } else {
            galerkin_alloc(&H->A[l], comp, ncomp, &H->A[l + 1]);
        }
        l++;
    }
    H->nlev = l + 1;
    for (int t = 0; t < H->nlev; t++) {
        H->l1[t] = (double *)malloc((size_t)(H->A[t].n > 0 ? H->A[t].n : 1) * sizeof(double));
        l1_diag(&H->A[t], H->l1[t]);
    }
    H->coarse_sweeps = O->coarse_l1_sweeps;
    H->refresh = O->amg_refresh;
    H->smoother = O->smoother;
    if (H->smoother == 1 && H->nlev > 1) {
        H->color = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
        H->ncolor = orc_greedy_colors(n, H->A[0].rowptr, H->A[0].col, H->color);
    }
    H->dense = H->A[H->nlev - 1].n <= O->coarse_dense_max;
    if (H->dense) {
        int st = dense_cholesky(&H->A[H->nlev - 1], &H->chol);
        if (st != ORC_OK) {
            orc_amg_destroy(H);
            return st;
        }
    }
    *out = H;
    return ORC_OK;
}

int orc_amg_update_fine(orc_amg *H, const double *val)
{
    memcpy(H->A[0].val, val, (size_t)H->A[0].rowptr[H->A[0].n] * sizeof(double));
    l1_diag(&H->A[0], H->l1[0]);
    int last = 0; /* last level whose matrix changed */
    if (H->refresh) {
        for (int l = 0; l + 1 < H->nlev; l++) {
            const orc_csr *A = &H->A[l];
            orc_csr *C = &H->A[l + 1];
            /* same aggregates, so the same patterns: recompute the values */
            if (H->P[l].rowptr) {
                orc_csr *Pl = &H->P[l];
                orc_smoothed_prolongator(A->n, A->rowptr, A->col, A->val, H->agg[l], C->n, Pl->rowptr,
                                         Pl->col, Pl->val);
                orc_rap(A->n, A->rowptr, A->col, A->val, C->n, Pl->rowptr, Pl->col, Pl->val, C->rowptr,
                        C->col, C->val);
            } else {
                orc_galerkin(A->n, A->rowptr, A->col, A->val, H->agg[l], C->n, C->rowptr, C->col,
                             C->val);
            }
            l1_diag(C, H->l1[l + 1]);
        }
        last = H->nlev - 1;
    }
    if (H->dense && last == H->nlev - 1) {
        free(H->chol);
        H->chol = NULL;
        return dense_cholesky(&H->A[H->nlev - 1], &H->chol);
    }
    return ORC_OK;
}

int orc_amg_levels(const orc_amg *H) { return H->nlev; }

void orc_amg_level_info(const orc_amg *H, int l, int64_t *n, int64_t *nnz)
{
    *n = H->A[l].n;
    *nnz = H->A[l].rowptr[H->A[l].n];
}

void orc_amg_level_export(const orc_amg *H, int l, int64_t *rowptr, int32_t *col, double *val,
                          int32_t *agg)
{
    const orc_csr *A = &H->A[l];
    memcpy(rowptr, A->rowptr, (size_t)(A->n + 1) * sizeof(int64_t));
    memcpy(col, A->col, (size_t)A->rowptr[A->n] * sizeof(int32_t));
    memcpy(val, A->val, (size_t)A->rowptr[A->n] * sizeof(double));
    if (agg && l < H->nlev - 1) memcpy(agg, H->agg[l], (size_t)A->n * sizeof(int32_t));
}

int orc_amg_coarse_is_dense(const orc_amg *H) { return H->dense; }

int64_t orc_amg_prolongator_nnz(const orc_amg *H, int l)
{
    if (l >= H->nlev - 1 || !H->P[l].rowptr) return 0;
    return H->P[l].rowptr[H->P[l].n];
}

void orc_amg_prolongator_export(const orc_amg *H, int l, int64_t *prow, int32_t *pcol,
                                double *pval)
{
    const orc_csr *Pl = &H->P[l];
    memcpy(prow, Pl->rowptr, (size_t)(Pl->n + 1) * sizeof(int64_t));
    memcpy(pcol, Pl->col, (size_t)Pl->rowptr[Pl->n] * sizeof(int32_t));
    memcpy(pval, Pl->val, (size_t)Pl->rowptr[Pl->n] * sizeof(double));
}

void orc_amg_destroy(orc_amg *H)
{
    if (!H) return;
    for (int l = 0; l < H->nlev; l++) {
        csr_free(&H->A[l]);
        csr_free(&H->P[l]);
        free(H->agg[l]);
        free(H->l1[l]);
    }
    free(H->chol);
    free(H->color);
    free(H);
}

static void coarse_solve(const orc_amg *H, const double *b, double *x)
{
    const orc_csr *A = &H->A[H->nlev - 1];
    int64_t n = A->n;
    if (H->dense) {
        const double *L = H->chol;
        for (int64_t i = 0; i < n; i++) { /* L y = b */
            double s = b[i];
            for (int64_t k = 0; k < i; k++) s -= L[i * n + k] * x[k];
            x[i] = s / L[i * n + i];
        }
        for (int64_t i = n - 1; i >= 0; i--) { /* L^T x = y */
            double s = x[i];
            for (int64_t k = i + 1; k < n; k++) s -= L[k * n + i] * x[k];
            x[i] = s / L[i * n + i];
        }
        return;
    }
    const double *d = H->l1[H->nlev - 1];
    double *r = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int64_t i = 0; i < n; i++) x[i] = 0.0;
    for (int s = 0; s < H->coarse_sweeps; s++) {
        orc_csr_matvec(n, A->rowptr, A->col, A->val, x, r);
        for (int64_t i = 0; i < n; i++) x[i] += (b[i] - r[i]) / d[i];
    }
    free(r);
}

/* Symmetric V-cycle of Section 5.2 with one l1-Jacobi sweep (one backward / */
/* forward multicolour Gauss-Seidel sweep on level 0 with smoother 1) before  */
/* and after the coarse correction; the pre-sweep starts from x = 0.          */
static void vcycle(const orc_amg *H, int l, const double *b, double *x)
{
    if (l == H->nlev - 1) {
        coarse_solve(H, b, x);
        return;
    }
    const orc_csr *A = &H->A[l];
    int64_t n = A->n, nc = H->A[l + 1].n;
    const double *d = H->l1[l];
    const int32_t *agg = H->agg[l];
    double *r = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *bc = (double *)calloc((size_t)(nc > 0 ? nc : 1), sizeof(double));
    double *xc = (double *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(double));
    const int gs = l == 0 && H->smoother == 1;
    if (gs) { /* backward Gauss-Seidel sweep from x = 0 */
        for (int64_t i = 0; i < n; i++) x[i] = 0.0;
        orc_mcgs_sweep(n, A->rowptr, A->col, A->val, H->color, H->ncolor, -1, b, x);
    } else {
        ORC_PARALLEL_FOR
        for (int64_t i = 0; i < n; i++) x[i] = b[i] / d[i];
    }
    orc_csr_matvec(n, A->rowptr, A->col, A->val, x, r);
    ORC_PARALLEL_FOR
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - r[i];
    if (H->P[l].rowptr) { /* b_c = P^T r, then x += P x_c */
        const orc_csr *Pl = &H->P[l];
        for (int64_t i = 0; i < n; i++)
            for (int64_t f = Pl->rowptr[i]; f < Pl->rowptr[i + 1]; f++) bc[Pl->col[f]] += Pl->val[f] * r[i];
        vcycle(H, l + 1, bc, xc);
        ORC_PARALLEL_FOR
        for (int64_t i = 0; i < n; i++) {
            double t = 0.0;
            for (int64_t f = Pl->rowptr[i]; f < Pl->rowptr[i + 1]; f++) t += Pl->val[f] * xc[Pl->col[f]];
            x[i] += t;
        }
    } else {
        for (int64_t i = 0; i < n; i++) bc[agg[i]] += r[i];
        vcycle(H, l + 1, bc, xc);
        ORC_PARALLEL_FOR
        for (int64_t i = 0; i < n; i++) x[i] += xc[agg[i]];
    }
    if (gs) { /* forward Gauss-Seidel sweep */
        orc_mcgs_sweep(n, A->rowptr, A->col, A->val, H->color, H->ncolor, +1, b, x);
    } else {
        orc_csr_matvec(n, A->rowptr, A->col, A->val, x, r);
        ORC_PARALLEL_FOR
        for (int64_t i = 0; i < n; i++) x[i] += (b[i] - r[i]) / d[i];
    }
    free(r);
    free(bc);
    free(xc);
}

void orc_amg_apply(const orc_amg *H, const double *b, double *x) { vcycle(H, 0, b, x); }

/* ------------------------------------------------------------------------ */
/* Restarted GMRES(m), right preconditioned (eq. (precsystem)): Arnoldi on   */
/* J M^{-1} with modified Gram-Schmidt, Givens rotations for the least-      */
/* squares problem, x += M^{-1} V y at the end of each cycle, and the true   */
/* residual recomputed at every restart.  Stops when ||b - J x||_2 <=        */
/* eta ||b||_2 (Section 6) or after maxit Arnoldi steps.  Returns 1 when     */
/* converged, 0 otherwise.                                                   */
/* ------------------------------------------------------------------------ */
static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

int orc_gmres(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
              const orc_amg *H, const double *b, double *x, int restart, double eta, int maxit,
              int *its_out, double *relres_out)
{
    int m = restart;
    double *V = (double *)malloc((size_t)(m + 1) * (size_t)(n > 0 ? n : 1) * sizeof(double));
    double *Hm = (double *)calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = (double *)calloc((size_t)m, sizeof(double));
    double *sn = (double *)calloc((size_t)m, sizeof(double));
    double *g = (double *)calloc((size_t)m + 1, sizeof(double));
    double *y = (double *)calloc((size_t)m, sizeof(double));
    double *z = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *w = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double bnorm = sqrt(dot(n, b, b));
    int total = 0, conv = 0;
    double relres = 0.0;
    for (int64_t i = 0; i < n; i++) x[i] = 0.0;
    if (bnorm == 0.0) {
        conv = 1;
        goto done;
    }
    for (;;) {
        /* true residual r = b - J x, kept in V_0 */
        orc_csr_matvec(n, rowptr, col, val, x, w);
        ORC_PARALLEL_FOR
        for (int64_t i = 0; i < n; i++) V[i] = b[i] - w[i];
        double beta = sqrt(dot(n, V, V));
        relres = beta / bnorm;
        if (beta <= eta * bnorm) {
            conv = 1;
            break;
        }
        if (total >= maxit) break;
        ORC_PARALLEL_FOR
        for (int64_t i = 0; i < n; i++) V[i] /= beta;
        for (int i = 0; i <= m; i++) g[i] = 0.0;
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m && total < maxit; j++) {
            double *vj = V + (size_t)j * n;
            if (H) orc_amg_apply(H, vj, z);
            else memcpy(z, vj, (size_t)n * sizeof(double));
            orc_csr_matvec(n, rowptr, col, val, z, w);
            for (int i = 0; i <= j; i++) {
                double *vi = V + (size_t)i * n;
                double h = dot(n, w, vi);
                Hm[i * m + j] = h;
                ORC_PARALLEL_FOR
                for (int64_t t = 0; t < n; t++) w[t] -= h * vi[t];
            }
            double hn = sqrt(dot(n, w, w));
            Hm[(j + 1) * m + j] = hn;
            if (hn > 0.0) {
                double *vn = V + (size_t)(j + 1) * n;
                ORC_PARALLEL_FOR
                for (int64_t t = 0; t < n; t++) vn[t] = w[t] / hn;
            }
            for (int i = 0; i < j; i++) {
                double a = Hm[i * m + j], c = Hm[(i + 1) * m + j];
                Hm[i * m + j] = cs[i] * a + sn[i] * c;
                Hm[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            double a = Hm[j * m + j], c = Hm[(j + 1) * m + j];
            double rho = sqrt(a * a + c * c);
            cs[j] = a / rho;
            sn[j] = c / rho;
            Hm[j * m + j] = rho;
            Hm[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            total++;
            k = j + 1;
            if (fabs(g[j + 1]) <= eta * bnorm || hn == 0.0) break;
        }
        for (int i = k - 1; i >= 0; i--) { /* back substitution */
            double s = g[i];
            for (int t = i + 1; t < k; t++) s -= Hm[i * m + t] * y[t];
            y[i] = s / Hm[i * m + i];
        }
        ORC_PARALLEL_FOR
        for (int64_t t = 0; t < n; t++) {
            double s = 0.0; /* the basis combination in ascending i, as a serial loop adds it */
            for (int i = 0; i < k; i++) s += y[i] * V[(size_t)i * n + t];
            w[t] = s;
        }
        if (H) orc_amg_apply(H, w, z);
        else memcpy(z, w, (size_t)n * sizeof(double));
        ORC_PARALLEL_FOR
        for (int64_t t = 0; t < n; t++) x[t] += z[t];
    }
done:
    *its_out = total;
    *relres_out = relres;
    free(V);
    free(Hm);
    free(cs);
    free(sn);
    free(g);
    free(y);
    free(z);
    free(w);
    return conv;
}

/* ------------------------------------------------------------------------ */
/* Backward Euler (Section 2.1) + modified inexact Newton (Section 3).       */
/* ------------------------------------------------------------------------ */
struct orc_solver {
    orc_problem P;
    orc_opts O;
    int64_t N, nnz;
    double *Ks;
    orc_csr J, M;
    orc_amg *H;
    int have_J;
    int since_build;
    double *theta_old, *u, *F, *ut, *Ft, *d, *Jd, *ub, *Fb;
    int nstep;                  /* time steps taken */
    orc_newton_event *trace;    /* armed record of the controller (may be NULL) */
    int trace_cap, trace_len;
};

void orc_solver_trace(orc_solver *S, orc_newton_event *buf, int cap)
{
    S->trace = buf;
    S->trace_cap = buf ? cap : 0;
    S->trace_len = 0;
}

int orc_solver_trace_len(const orc_solver *S) { return S->trace_len; }

void orc_solver_iterate(const orc_solver *S, double *u)
{
    memcpy(u, S->u, (size_t)S->N * sizeof(double));
}

static void trace_push(orc_solver *S, const orc_newton_event *ev)
{
    if (!S->trace) return;
    if (S->trace_len < S->trace_cap) S->trace[S->trace_len] = *ev;
    S->trace_len++;
}

static void trace_trial(orc_newton_event *ev, double lam, double f)
{
    if (ev->ntrial < ORC_TRACE_TRIALS) {
        ev->trial_lam[ev->ntrial] = lam;
        ev->trial_f[ev->ntrial] = f;
    }
    ev->ntrial++;
}

static double norm_inf(int64_t n, const double *v)
{
    double m = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double a = fabs(v[i]);
        if (a > m || a != a) m = a;
    }
    return m;
}

static int all_finite(int64_t n, const double *v)
{
    for (int64_t i = 0; i < n; i++)
        if (!isfinite(v[i])) return 0;
    return 1;
}

int orc_solver_create(const orc_problem *P, const orc_opts *O, const double *Ks, orc_solver **out)
{
    if (P->nx < 1 || P->ny < 1 || P->nz < 1 || !(P->hx > 0) || !(P->hy > 0) || !(P->hz > 0) ||
        !(P->dt > 0) || O->gmres_restart < 1)
        return ORC_EINVAL;
    orc_solver *S = (orc_solver *)calloc(1, sizeof(orc_solver));
    S->P = *P;
    S->O = *O;
    S->N = (int64_t)P->nx * P->ny * P->nz;
    S->nnz = orc_pattern_nnz(P);
    int64_t N = S->N;
    S->Ks = (double *)malloc((size_t)N * sizeof(double));
    memcpy(S->Ks, Ks, (size_t)N * sizeof(double));
    S->J.n = S->M.n = N;
    S->J.rowptr = (int64_t *)malloc((size_t)(N + 1) * sizeof(int64_t));
    S->M.rowptr = (int64_t *)malloc((size_t)(N + 1) * sizeof(int64_t));
    S->J.col = (int32_t *)malloc((size_t)S->nnz * sizeof(int32_t));
    S->M.col = (int32_t *)malloc((size_t)S->nnz * sizeof(int32_t));
    S->J.val = (double *)malloc((size_t)S->nnz * sizeof(double));
    S->M.val = (double *)malloc((size_t)S->nnz * sizeof(double));
    double **vecs[] = {&S->theta_old, &S->u, &S->F, &S->ut, &S->Ft, &S->d, &S->Jd, &S->ub, &S->Fb};
    for (size_t t = 0; t < sizeof(vecs) / sizeof(vecs[0]); t++)
        *vecs[t] = (double *)malloc((size_t)N * sizeof(double));
    *out = S;
    return ORC_OK;
}

void orc_solver_destroy(orc_solver *S)
{
    if (!S) return;
    free(S->Ks);
    csr_free(&S->J);
    csr_free(&S->M);
    orc_amg_destroy(S->H);
    double *vecs[] = {S->theta_old, S->u, S->F, S->ut, S->Ft, S->d, S->Jd, S->ub, S->Fb};
    for (size_t t = 0; t < sizeof(vecs) / sizeof(vecs[0]); t++) free(vecs[t]);
    free(S);
}

/* Rebuild J and the auxiliary matrix at u.  The AMG hierarchy is built on   */
/* the first auxiliary matrix of the run only; later rebuilds refresh the    */
/* fine-level matrix and its smoother (Section 6, re-use strategy).          */
static int rebuild(orc_solver *S, const double *u, orc_stats *st)
{
    orc_jacobian(&S->P, S->Ks, u, S->J.rowptr, S->J.col, S->J.val);
    if (S->O.aux_dflux) orc_auxiliary_dflux(&S->P, S->Ks, u, S->M.rowptr, S->M.col, S->M.val);
    else orc_auxiliary(&S->P, S->Ks, u, S->M.rowptr, S->M.col, S->M.val);
    int rc = ORC_OK;
    if (!S->H) {
        rc = orc_amg_build(&S->O, S->N, S->M.rowptr, S->M.col, S->M.val, &S->H);
        st->amg_setups++;
    } else {
        rc = orc_amg_update_fine(S->H, S->M.val);
    }
    S->have_J = 1;
    S->since_build = 0;
    st->jac_builds++;
    return rc;
}

static double half_sq(int64_t n, const double *v) { return 0.5 * dot(n, v, v); }

/* Relative length of a step: max_i |s_i| / max(|u_i|, 1) (identity scaling). */
static double rel_length(int64_t n, const double *s, double lam, const double *u)
{
    double m = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double a = fabs(u[i]);
        double r = fabs(lam * s[i]) / (a > 1.0 ? a : 1.0);
        if (r > m) m = r;
    }
    return m;
}

/*
 * Line search (Section 3, Armijo-Goldstein): backtracking in the style of
 * Dennis & Schnabel's Algorithm A6.3.1 (a published method).  The alpha
 * condition f(u + lam d) <= f0 + alpha lam slope is enforced with f = 0.5
 * ||Phi||^2 and slope = Phi^T (J d); the first reduction minimises the
 * quadratic model, later ones the cubic model through the last two trials,
 * each clamped to [0.1 lam, 0.5 lam].  The beta condition (beta = 0.9) is
 * checked when the full step satisfies the alpha condition and is shorter
 * than the maximum step: lam is then doubled while the alpha condition still
 * holds, the beta condition fails and the step stays within the maximum.
 * Fails when lam drops below scsteptol / rel_length(d).
 * On success u+lam d is in S->ut and its residual in S->Ft.
 */
static int line_search(orc_solver *S, double slope, double mxstep, int truncated, double *lam_out,
                       int *nback, orc_newton_event *ev)
{
    int64_t N = S->N;
    const double alpha = S->O.ls_alpha, beta = 0.9;
    double f0 = half_sq(N, S->F);
    double rl = rel_length(N, S->d, 1.0, S->u);
    double lam_min = rl > 0.0 ? S->O.scsteptol / rl : 0.0;
    double lam = 1.0, lam_prev = 0.0, f_prev = 0.0;
    int have_model = 0; /* a finite trial has been seen: the next model is cubic */
    *nback = 0;
    ev->rel_d = rl;
    for (;;) {
        for (int64_t i = 0; i < N; i++) S->ut[i] = S->u[i] + lam * S->d[i];
        orc_residual(&S->P, S->Ks, S->ut, S->theta_old, S->Ft);
        double ft = half_sq(N, S->Ft);
        trace_trial(ev, lam, ft);
        if (isfinite(ft) && ft <= f0 + alpha * lam * slope) break;
        if (lam < lam_min) return ORC_LINESEARCH_FAIL;
        double lt;
        if (!isfinite(ft)) {
            lt = 0.1 * lam;
        } else if (!have_model) {
            /* minimiser of the quadratic q with q(0) = f0, q'(0) = slope, q(lam) = ft */
            lt = -slope * lam * lam / (2.0 * (ft - f0 - slope * lam));
        } else {
            /* minimiser of the cubic c with c(0) = f0, c'(0) = slope through the
               last two finite trials (lam_prev, f_prev) and (lam, ft) */
            double t1 = ft - f0 - lam * slope;
            double t2 = f_prev - f0 - lam_prev * slope;
            double a = (t1 / (lam * lam) - t2 / (lam_prev * lam_prev)) / (lam - lam_prev);
            double b = (-lam_prev * t1 / (lam * lam) + lam * t2 / (lam_prev * lam_prev)) /
                       (lam - lam_prev);
            if (a == 0.0) {
                lt = -slope / (2.0 * b);
            } else {
                double disc = b * b - 3.0 * a * slope;
                lt = disc < 0.0 ? 0.5 * lam : (-b + sqrt(disc)) / (3.0 * a);
            }
        }
        if (isfinite(ft)) {
            lam_prev = lam;
            f_prev = ft;
            have_model = 1;
        }
        if (!(lt <= 0.5 * lam)) lt = 0.5 * lam;
        if (!(lt >= 0.1 * lam)) lt = 0.1 * lam;
        lam = lt;
        (*nback)++;
    }
    /* beta condition, full step only, when a longer step is allowed */
    if (lam == 1.0 && !truncated) {
        double dn = sqrt(dot(N, S->d, S->d));
        double ft = half_sq(N, S->Ft);
        int tries = 0;
        while (ft < f0 + beta * lam * slope && 2.0 * lam * dn <= mxstep && tries < 10) {
            double lt = 2.0 * lam;
            for (int64_t i = 0; i < N; i++) S->ub[i] = S->u[i] + lt * S->d[i];
            orc_residual(&S->P, S->Ks, S->ub, S->theta_old, S->Fb);
            double fb = half_sq(N, S->Fb);
            trace_trial(ev, lt, fb);
            if (!(isfinite(fb) && fb <= f0 + alpha * lt * slope)) break;
            lam = lt;
            ft = fb;
            memcpy(S->ut, S->ub, (size_t)N * sizeof(double));
            memcpy(S->Ft, S->Fb, (size_t)N * sizeof(double));
            tries++;
        }
    }
    *lam_out = lam;
    return ORC_OK;
}

/*
 * One backward-Euler step: solve Phi(u) = 0 from u = p^l (reading: the
 * previous level is the initial guess) with the modified inexact Newton
 * method of Section 3.  J and the auxiliary matrix are rebuilt when any of
 * eq. (jacobian_update_condition) holds:
 *   - msbset Newton iterations have passed since the last rebuild (the
 *     counter persists across time steps, which re-use the previous step's
 *     Jacobian: Section 6);
 *   - the previous scaled step ||lam d||_inf exceeded 1.5;
 *   - a retry was requested because, with a stale J, GMRES failed, the line
 *     search failed, or the step became shorter than scsteptol.
 * With a fresh J those events end the step with an error (GMRES failure only
 * if d is not a descent direction); the short step ends it with the warning
 * ORC_STEP_TOO_SMALL (>0) and the state is kept.
 */
int orc_solver_step(orc_solver *S, double *p, orc_stats *st)
{
    int64_t N = S->N;
    memset(st, 0, sizeof(*st));
    st->min_lambda = 1.0;
    int step_index = S->nstep++;
    if (!all_finite(N, p)) return st->status = ORC_NONFINITE;
    orc_theta(&S->P, p, S->theta_old);
    memcpy(S->u, p, (size_t)N * sizeof(double));
    orc_residual(&S->P, S->Ks, S->u, S->theta_old, S->F);
    double fnorm = norm_inf(N, S->F);
    if (!isfinite(fnorm)) return st->status = ORC_NONFINITE;
    double mxstep = S->O.mxnewtstep;
    if (!(mxstep > 0.0)) {
        double un = sqrt(dot(N, S->u, S->u));
        mxstep = 1000.0 * (un > 1.0 ? un : 1.0);
    }
    double prev_step = 0.0;
    int retry = 0, status = ORC_OK;
    orc_newton_event ev;
    while (fnorm > S->O.fnormtol) {
        if (st->newton_its >= S->O.max_newton) {
            status = ORC_MAXITER;
            break;
        }
        memset(&ev, 0, sizeof(ev));
        ev.step = step_index;
        ev.newton_it = st->newton_its;
        ev.since_build = S->since_build;
        ev.mxstep = mxstep;
        ev.f0 = half_sq(N, S->F);
        ev.reason = (!S->have_J ? ORC_RB_NOJ : 0) | (S->have_J && S->since_build >= S->O.msbset ? ORC_RB_MSBSET : 0) |
                    (prev_step > 1.5 ? ORC_RB_BIGSTEP : 0) | (retry ? ORC_RB_RETRY : 0);
        int fresh = 0;
        if (ev.reason) {
            int rc = rebuild(S, S->u, st);
            if (rc != ORC_OK) {
                status = rc;
                ev.outcome = ORC_EV_FAIL_OTHER;
                trace_push(S, &ev);
                break;
            }
            fresh = 1;
            retry = 0;
        }
        for (int64_t i = 0; i < N; i++) S->Ft[i] = -S->F[i];
        int its;
        double relres;
        int conv = orc_gmres(N, S->J.rowptr, S->J.col, S->J.val, S->H, S->Ft, S->d,
                             S->O.gmres_restart, S->O.eta, S->O.gmres_maxit, &its, &relres);
        st->gmres_its += its;
        ev.gmres_its = its;
        ev.gmres_conv = conv;
        if (!conv) {
            st->linsolve_fails++;
            if (!fresh) {
                retry = 1;
                ev.outcome = ORC_EV_RETRY_GMRES;
                trace_push(S, &ev);
                continue;
            }
        }
        int truncated = 0;
        double dn = sqrt(dot(N, S->d, S->d));
        if (dn > mxstep) {
            for (int64_t i = 0; i < N; i++) S->d[i] *= mxstep / dn;
            truncated = 1;
        }
        ev.truncated = truncated;
        ev.dnorm2 = sqrt(dot(N, S->d, S->d));
        ev.dnorminf = norm_inf(N, S->d);
        orc_csr_matvec(N, S->J.rowptr, S->J.col, S->J.val, S->d, S->Jd);
        double slope = dot(N, S->F, S->Jd);
        ev.slope = slope;
        if (!(slope < 0.0)) {
            if (!fresh) {
                retry = 1;
                ev.outcome = ORC_EV_RETRY_SLOPE;
                trace_push(S, &ev);
                continue;
            }
            status = ORC_LINSOLVE_FAIL;
            ev.outcome = ORC_EV_FAIL_SLOPE;
            trace_push(S, &ev);
            break;
        }
        double lam;
        int nb;
        int rc = line_search(S, slope, mxstep, truncated, &lam, &nb, &ev);
        st->ls_backtracks += nb;
        ev.nback = nb;
        if (rc != ORC_OK) {
            if (!fresh) {
                retry = 1;
                ev.outcome = ORC_EV_RETRY_LS;
                trace_push(S, &ev);
                continue;
            }
            status = rc;
            ev.outcome = ORC_EV_FAIL_LS;
            trace_push(S, &ev);
            break;
        }
        if (lam < st->min_lambda) st->min_lambda = lam;
        double step_inf = lam * norm_inf(N, S->d);
        double step_rel = rel_length(N, S->d, lam, S->ut);
        memcpy(S->u, S->ut, (size_t)N * sizeof(double));
        memcpy(S->F, S->Ft, (size_t)N * sizeof(double));
        st->newton_its++;
        S->since_build++;
        fnorm = norm_inf(N, S->F);
        ev.lam = lam;
        ev.f_acc = half_sq(N, S->F);
        ev.step_inf = step_inf;
        ev.step_rel = step_rel;
        ev.fnorm_inf = fnorm;
        ev.outcome = ORC_EV_ACCEPT;
        if (!isfinite(fnorm)) {
            status = ORC_NONFINITE;
            ev.outcome = ORC_EV_FAIL_OTHER;
            trace_push(S, &ev);
            break;
        }
        if (fnorm <= S->O.fnormtol) {
            trace_push(S, &ev);
            break;
        }
        if (step_rel < S->O.scsteptol) {
            if (!fresh) {
                retry = 1;
                ev.outcome = ORC_EV_ACCEPT_SHORT;
            } else {
                status = ORC_STEP_TOO_SMALL;
                ev.outcome = ORC_EV_STALL;
                trace_push(S, &ev);
                break;
            }
        }
        trace_push(S, &ev);
        prev_step = step_inf;
    }
    st->fnorm_inf = fnorm;
    if (status == ORC_OK || status == ORC_STEP_TOO_SMALL) {
        memcpy(p, S->u, (size_t)N * sizeof(double));
        double s = 0.0;
        for (int64_t i = 0; i < N; i++) s += S->F[i];
        st->mass_residual = S->P.dt * s;
    }
    st->status = status;
    return status;
}
