// Fine-grid kernels: constitutive laws, residual Phi, Jacobian / auxiliary
// matrix assembly, 7-point stencil products and the fine-level pieces of the
// AMG V-cycle.  One thread per cell, x-fastest cell order, SoA coefficient
// arrays (every load and store of a wavefront is one contiguous run).
#include <algorithm>

#include "common.hpp"

namespace rich {

namespace {

constexpr int TPB = 256;

inline unsigned nblocks(int64_t n, int tpb = TPB) { return xcd_grid(n, tpb); }

struct Cell {
    int i, j, k;
};

template <class G>
__device__ inline Cell cell_of(const G &P, uint32_t c) {
    uint32_t nxy = (uint32_t)P.nx * (uint32_t)P.ny;
    uint32_t k = c / nxy;
    uint32_t rem = c - k * nxy;
    uint32_t j = rem / (uint32_t)P.nx;
    uint32_t i = rem - j * (uint32_t)P.nx;
    return {(int)i, (int)j, (int)k};
}

// Section 2, eq. (s(p)) and eq. (K(p)) with rho*phi = 1 and K_s per cell;
// derivatives eq. (derivativeofcoefficients) for p < 0.  p >= 0 is the
// saturated regime (K = K_s, theta = theta_s, derivatives 0).
// |p|^beta and |p|^gamma share one log: exp(beta*log|p|), exp(gamma*log|p|).
struct Law {
    double th, dth, K, dK;
};

__device__ inline Law laws(const Phys &P, double p, double Ks) {
    Law L;
    if (p >= 0.0) {
        L.th = P.theta_s;
        L.dth = 0.0;
        L.K = Ks;
        L.dK = 0.0;
        return L;
    }
    double a = -p;
    double la = log(a);
    double ab = exp(P.beta * la);
    double ag = exp(P.gamma * la);
    double ds = P.theta_s - P.theta_r;
    double tden = P.alpha + ab;
    double kden = P.A + ag;
    L.th = P.alpha * ds / tden + P.theta_r;
    L.dth = P.alpha * P.beta * ds * (ab / a) / (tden * tden);
    L.K = Ks * P.A / kden;
    L.dK = Ks * P.A * P.gamma * (ag / a) / (kden * kden);
    return L;
}

// One face of cell c.  kind: 0 = none (no-flux face), 1 = interior neighbour,
// 2 = Dirichlet boundary node (head = face value, or the patch value where the
// optional Dirichlet patch covers the node; K_s = the cell's).
struct Face {
    int kind;
    uint32_t n;
    double pn, Ksn, h;
};

__device__ inline Face face(const Phys &P, const Cell &q, uint32_t c, int f, const double *p,
                            const double *Ks) {
    Face F;
    int axis = f >> 1;
    int dir = (f & 1) ? 1 : -1;
    int ii = q.i + (axis == 0 ? dir : 0);
    int jj = q.j + (axis == 1 ? dir : 0);
    int kk = q.k + (axis == 2 ? dir : 0);
    F.h = axis == 0 ? P.hx : (axis == 1 ? P.hy : P.hz);
    int inside = (axis == 0) ? (ii >= 0 && ii < P.nx) : (axis == 1) ? (jj >= 0 && jj < P.ny) : (kk >= 0 && kk < P.nz);
    if (inside) {
        uint32_t stride = axis == 0 ? 1u : (axis == 1 ? (uint32_t)P.nx : (uint32_t)P.nx * (uint32_t)P.ny);
        F.n = dir > 0 ? c + stride : c - stride;
        F.kind = 1;
        F.pn = p[F.n];
        F.Ksn = Ks[F.n];
    } else if (P.bc_type[f] == RICH_BC_DIRICHLET) {
        F.kind = 2;
        F.n = c;
        F.pn = P.bc_value[f];
        if (f == P.patch_face) {
            // the boundary node's coordinates along the face's two axes
            double u = axis == 0 ? (q.j + 1) * P.hy : (q.i + 1) * P.hx;
            double v = axis == 2 ? (q.j + 1) * P.hy : (q.k + 1) * P.hz;
            if (u >= P.patch_lo[0] && u <= P.patch_hi[0] && v >= P.patch_lo[1] && v <= P.patch_hi[1])
                F.pn = P.patch_value;
        }
        F.Ksn = Ks[c];
    } else {
        F.kind = 0;
        F.n = c;
        F.pn = 0.0;
        F.Ksn = 0.0;
    }
    return F;
}

// Interface mean of K and its partial derivatives (Section 2.1).  dir > 0:
// the neighbour is the higher-index side U.  Upstream takes K_U when
// p_U - p_L >= 0, else K_L; harmonic 2 K_L K_U / (K_L + K_U); geometric
// sqrt(K_L K_U); integral: the average of K_s k_r over the heads between p_L
// and p_U (K_s the mean of the two sides), by the Gauss-Legendre rule held in
// Phys, always evaluated from the L side so both cells of a face agree bitwise.
// With mean_vertical >= 0 the z faces take that mean (one mean for the
// horizontal and another for the vertical direction).
// INTEG = false leaves the integral mean out (for kernels launched only when
// no face takes it: its quadrature loop costs registers in every caller).
template <bool INTEG = true>
__device__ inline void mean_of(const Phys &P, int axis, int dir, double pc, const Law &Lc, double Ksc, double pn,
                               const Law &Ln, double Ksn, double &Kf, double &dc, double &dn) {
    int mean = (axis == 2 && P.mean_vertical >= 0) ? P.mean_vertical : P.mean;
    if (mean == RICH_MEAN_ARITH) {
        Kf = 0.5 * (Lc.K + Ln.K);
        dc = 0.5 * Lc.dK;
        dn = 0.5 * Ln.dK;
    } else if (mean == RICH_MEAN_HARMONIC) {
        double s = Lc.K + Ln.K;
        Kf = 2.0 * Lc.K * Ln.K / s;
        dc = 2.0 * Ln.K * Ln.K * Lc.dK / (s * s);
        dn = 2.0 * Lc.K * Lc.K * Ln.dK / (s * s);
    } else if (mean == RICH_MEAN_GEOMETRIC) {
        double g = sqrt(Lc.K * Ln.K);
        Kf = g;
        dc = 0.5 * Ln.K * Lc.dK / g;
        dn = 0.5 * Lc.K * Ln.dK / g;
    } else if (INTEG && mean == RICH_MEAN_INTEGRAL) {
        double pL = dir > 0 ? pc : pn, pU = dir > 0 ? pn : pc;
        double Ks = 0.5 * (dir > 0 ? Ksc + Ksn : Ksn + Ksc);
        double q = 0.0, qL = 0.0, qU = 0.0;
        for (int t = 0; t < RICH_GL; t++) {
            Law L = laws(P, pL + (pU - pL) * P.gl_t[t], Ks);
            q += P.gl_w[t] * L.K;
            qL += P.gl_w[t] * (1.0 - P.gl_t[t]) * L.dK;
            qU += P.gl_w[t] * P.gl_t[t] * L.dK;
        }
        Kf = q;
        dc = dir > 0 ? qL : qU;
        dn = dir > 0 ? qU : qL;
    } else {
        bool take_n = dir > 0 ? (pn - pc >= 0.0) : !(pc - pn >= 0.0);
        if (take_n) {
            Kf = Ln.K;
            dc = 0.0;
            dn = Ln.dK;
        } else {
            Kf = Lc.K;
            dc = Lc.dK;
            dn = 0.0;
        }
    }
}

__global__ void k_theta(Phys P, uint32_t n, const double *__restrict__ p, double *__restrict__ th) {
    uint32_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= n) return;
    th[c] = laws(P, p[c], 1.0).th;
}

// eq. (dynamic_of_the_problem), f = 0: time term plus, per face, the
// diffusive flux -K^AV (p_n - p_c)/h^2 and on z faces the gravity part
// +-(K_c + K_n)/(2 h_z) (the paper's centred -(K_{k+1} - K_{k-1})/(2 h_z)
// written face by face; a no-flux face contributes nothing).
__global__ void k_residual(Phys P, uint32_t n, const double *__restrict__ Ks, const double *__restrict__ p,
                           const double *__restrict__ th_old, double *__restrict__ F) {
    uint32_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= n) return;
    Cell q = cell_of(P, c);
    double pc = p[c];
    Law Lc = laws(P, pc, Ks[c]);
    double acc = (Lc.th - th_old[c]) / P.dt;
#pragma unroll
    for (int f = 0; f < 6; f++) {
        Face fc = face(P, q, c, f, p, Ks);
        if (fc.kind == 0) continue;
        Law Ln = laws(P, fc.pn, fc.Ksn);
        double Kf, dc, dn;
        int dir = (f & 1) ? 1 : -1;
        mean_of(P, f >> 1, dir, pc, Lc, Ks[c], fc.pn, Ln, fc.Ksn, Kf, dc, dn);
        acc += -Kf * (fc.pn - pc) / (fc.h * fc.h);
        if ((f >> 1) == 2) acc += dir * (-(Lc.K + Ln.K) / (2.0 * P.hz));
    }
    F[c] = acc;
}

// Jacobian rows (analytic derivatives of the residual above) and the
// auxiliary matrix of Section 4's closing construction: the Jacobian of the
// diffusion-only flux q = -K grad p with the conductivity frozen, plus the
// time term; with dflux its diagonal also takes the flux-derivative terms
// -(p_n - p_c)/h^2 dK^AV/dp_c (off-diagonal ones dropped, M stays
// symmetric).  Also the l1 row sums of M (diag + sum |off|) as inverses.
__global__ void k_assemble(Phys P, uint32_t n, const double *__restrict__ Ks, const double *__restrict__ p,
                           double *__restrict__ J7, double *__restrict__ M4, float *__restrict__ M4f,
                           double *__restrict__ invd, float *__restrict__ invdf, int dflux) {
    uint32_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= n) return;
    Cell q = cell_of(P, c);
    double pc = p[c];
    Law Lc = laws(P, pc, Ks[c]);
    double jd = Lc.dth / P.dt;
    double md = Lc.dth / P.dt;
    double joff[6] = {0, 0, 0, 0, 0, 0};
    double moff[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int f = 0; f < 6; f++) {
        Face fc = face(P, q, c, f, p, Ks);
        if (fc.kind == 0) continue;
        Law Ln = laws(P, fc.pn, fc.Ksn);
        double Kf, dc, dn;
        int dir = (f & 1) ? 1 : -1;
        mean_of(P, f >> 1, dir, pc, Lc, Ks[c], fc.pn, Ln, fc.Ksn, Kf, dc, dn);
        double h2 = fc.h * fc.h;
        double dp = fc.pn - pc;
        bool zf = (f >> 1) == 2;
        jd += Kf / h2 - dp / h2 * dc;
        if (zf) jd += -dir * Lc.dK / (2.0 * P.hz);
        md += Kf / h2;
        if (dflux) md += -dp / h2 * dc;
        if (fc.kind == 1) {
            double v = -Kf / h2 - dp / h2 * dn;
            if (zf) v += -dir * Ln.dK / (2.0 * P.hz);
            joff[f] = v;
            moff[f] = -Kf / h2;
        }
    }
    J7[(size_t)J_D * n + c] = jd;
    J7[(size_t)J_XM * n + c] = joff[0];
    J7[(size_t)J_XP * n + c] = joff[1];
    J7[(size_t)J_YM * n + c] = joff[2];
    J7[(size_t)J_YP * n + c] = joff[3];
    J7[(size_t)J_ZM * n + c] = joff[4];
    J7[(size_t)J_ZP * n + c] = joff[5];
    M4[(size_t)M_D * n + c] = md;
    M4[(size_t)M_XP * n + c] = moff[1];
    M4[(size_t)M_YP * n + c] = moff[3];
    M4[(size_t)M_ZP * n + c] = moff[5];
    double l1 = md;
#pragma unroll
    for (int f = 0; f < 6; f++) l1 += fabs(moff[f]);
    if (M4f) {
        M4f[(size_t)M_D * n + c] = f32_sat(md);
        M4f[(size_t)M_XP * n + c] = f32_sat(moff[1]);
        M4f[(size_t)M_YP * n + c] = f32_sat(moff[3]);
        M4f[(size_t)M_ZP * n + c] = f32_sat(moff[5]);
    }
    if (invd) invd[c] = 1.0 / l1;
    if (invdf) invdf[c] = f32_sat(1.0 / l1);
}

// ------------------------------------ plane-tiled residual and assembly
// A block owns an FT_X x FT_Y tile of (x, y) columns and a run of z planes.
// For each plane it stages the tile and a one-cell ring around it in LDS
// (heads, K_s and the laws of every cell, each evaluated once; the tile's own
// cells carry their laws over from the plane below, where they were the upper
// neighbours), then computes every face between two cells of the domain once
// (its interface mean and, for the Jacobian, the mean's derivatives) and
// hands it to both cells: the face's term enters the lower-index cell's row
// as it is and the upper cell's with the roles swapped.  Faces on the domain
// boundary are taken per cell as in the one-thread-per-cell kernels.  Each
// cell adds its faces in the order -x, +x, -y, +y, -z, +z.
constexpr int FT_X = 32, FT_Y = 8, FT_TPB = FT_X * FT_Y;
constexpr int FT_RX = FT_X + 2, FT_RY = FT_Y + 2, FT_RING = FT_RX * FT_RY;
constexpr int FT_NRING = FT_RING - FT_TPB;  // ring positions staged per plane (84)
constexpr int FT_NFX = (FT_X + 1) * FT_Y, FT_NFY = FT_X * (FT_Y + 1);

// a face's interface mean and its derivatives w.r.t. the lower and upper heads
struct FaceMean {
    double Kf, dL, dU;
};

// The tile's ring positions, in LDS order of a (FT_RY x FT_RX) array: the
// rows above and below the tile, then the left and right columns.
__device__ inline int ring_pos(int t) {
    if (t < FT_RX) return t;                                  // row 0
    if (t < 2 * FT_RX) return (FT_RY - 1) * FT_RX + (t - FT_RX);  // last row
    t -= 2 * FT_RX;                                           // 0 .. 2 FT_Y - 1
    int r = 1 + t / 2;
    return r * FT_RX + ((t & 1) ? FT_RX - 1 : 0);
}

template <bool JAC, bool INTEG>
__global__ void __launch_bounds__(FT_TPB) k_faces_tiled(Phys P, int kz, const double *__restrict__ Ks,
                                                        const double *__restrict__ p,
                                                        const double *__restrict__ th_old, double *__restrict__ F,
                                                        double *__restrict__ J7, double *__restrict__ M4,
                                                        float *__restrict__ M4f, double *__restrict__ invd,
                                                        float *__restrict__ invdf, int dflux) {
    __shared__ double sp[FT_RING], sks[FT_RING], sK[FT_RING], sdK[JAC ? FT_RING : 1];
    __shared__ double fx[JAC ? 3 : 1][FT_NFX], fy[JAC ? 3 : 1][FT_NFY];
    const int tx = threadIdx.x % FT_X, ty = threadIdx.x / FT_X;
    const int i0 = blockIdx.x * FT_X, j0 = blockIdx.y * FT_Y;
    const int k0 = blockIdx.z * kz, k1 = min(k0 + kz, P.nz);
    const int i = i0 + tx, j = j0 + ty;
    const bool own = i < P.nx && j < P.ny;
    const uint32_t nxy = (uint32_t)P.nx * (uint32_t)P.ny, n = nxy * (uint32_t)P.nz;
    const int me = (ty + 1) * FT_RX + (tx + 1);
    const double hx2 = P.hx * P.hx, hy2 = P.hy * P.hy, hz2 = P.hz * P.hz;
    // the own column: current plane (c), the one above (u) and the face below
    double pc = 0.0, ksc = 0.0, pu = 0.0, ksu = 0.0;
    Law Lc{}, Lu{};
    // residual: diffusive flux and gravity term of the face below / above, as they
    // enter the lower cell's row (the upper cell takes their negatives)
    double q_dn = 0.0, g_dn = 0.0, q_up = 0.0, g_up = 0.0;
    FaceMean m_dn{}, m_up{};                // Jacobian: means of those faces
    double pd = 0.0, dKd = 0.0;             // Jacobian: head and K' of the cell below
    const uint32_t col = own ? (uint32_t)i + (uint32_t)P.nx * (uint32_t)j : 0u;
    if (own) {
        const uint32_t c = col + nxy * (uint32_t)k0;
        pc = p[c];
        ksc = Ks[c];
        Lc = laws(P, pc, ksc);
        if (k0 > 0) {
            const uint32_t cd = c - nxy;
            pd = p[cd];
            const double ksd = Ks[cd];
            const Law Ld = laws(P, pd, ksd);
            double Kf, dL, dU;
            mean_of<INTEG>(P, 2, 1, pd, Ld, ksd, pc, Lc, ksc, Kf, dL, dU);
            q_dn = -Kf * (pc - pd) / hz2;
            g_dn = -(Ld.K + Lc.K) / (2.0 * P.hz);
            m_dn = {Kf, dL, dU};
            dKd = Ld.dK;
        }
    }
    for (int k = k0; k < k1; k++) {
        // stage plane k: the own cells from registers, the ring from memory
        if (own) {
            sp[me] = pc;
            sks[me] = ksc;
            sK[me] = Lc.K;
            if constexpr (JAC) sdK[me] = Lc.dK;
        }
        if (threadIdx.x < FT_NRING) {
            const int pos = ring_pos(threadIdx.x);
            const int gi = i0 - 1 + pos % FT_RX, gj = j0 - 1 + pos / FT_RX;
            if (gi >= 0 && gi < P.nx && gj >= 0 && gj < P.ny) {
                const uint32_t cc = (uint32_t)gi + (uint32_t)P.nx * ((uint32_t)gj + (uint32_t)P.ny * (uint32_t)k);
                const double pr = p[cc], kr = Ks[cc];
                const Law L = laws(P, pr, kr);
                sp[pos] = pr;
                sks[pos] = kr;
                sK[pos] = L.K;
                if constexpr (JAC) sdK[pos] = L.dK;
            }
        }
        // the own column's cell above and the face between
        const bool up = own && k + 1 < P.nz;
        if (up) {
            const uint32_t cu = col + nxy * (uint32_t)(k + 1);
            pu = p[cu];
            ksu = Ks[cu];
            Lu = laws(P, pu, ksu);
            double Kf, dL, dU;
            mean_of<INTEG>(P, 2, 1, pc, Lc, ksc, pu, Lu, ksu, Kf, dL, dU);
            q_up = -Kf * (pu - pc) / hz2;
            g_up = -(Lc.K + Lu.K) / (2.0 * P.hz);
            m_up = {Kf, dL, dU};
        }
        __syncthreads();
        // x faces: face f joins tile columns f - 1 (lower) and f of row r
        for (int t = threadIdx.x; t < FT_NFX; t += FT_TPB) {
            const int f = t % (FT_X + 1), r = t / (FT_X + 1);
            const int iL = i0 + f - 1, jj = j0 + r;
            if (iL >= 0 && iL + 1 < P.nx && jj < P.ny) {
                const int a = (r + 1) * FT_RX + f, b = a + 1;
                Law La{0.0, 0.0, sK[a], JAC ? sdK[a] : 0.0}, Lb{0.0, 0.0, sK[b], JAC ? sdK[b] : 0.0};
                double Kf, dL, dU;
                mean_of<INTEG>(P, 0, 1, sp[a], La, sks[a], sp[b], Lb, sks[b], Kf, dL, dU);
                if constexpr (JAC) {
                    fx[0][t] = Kf;
                    fx[1][t] = dL;
                    fx[2][t] = dU;
                } else {
                    fx[0][t] = -Kf * (sp[b] - sp[a]) / hx2;
                }
            }
        }
        // y faces: face g joins tile rows g - 1 (lower) and g of column c
        for (int t = threadIdx.x; t < FT_NFY; t += FT_TPB) {
            const int c = t % FT_X, g = t / FT_X;
            const int jL = j0 + g - 1, ii = i0 + c;
            if (jL >= 0 && jL + 1 < P.ny && ii < P.nx) {
                const int a = g * FT_RX + c + 1, b = a + FT_RX;
                Law La{0.0, 0.0, sK[a], JAC ? sdK[a] : 0.0}, Lb{0.0, 0.0, sK[b], JAC ? sdK[b] : 0.0};
                double Kf, dL, dU;
                mean_of<INTEG>(P, 1, 1, sp[a], La, sks[a], sp[b], Lb, sks[b], Kf, dL, dU);
                if constexpr (JAC) {
                    fy[0][t] = Kf;
                    fy[1][t] = dL;
                    fy[2][t] = dU;
                } else {
                    fy[0][t] = -Kf * (sp[b] - sp[a]) / hy2;
                }
            }
        }
        __syncthreads();
        if (own) {
            const uint32_t c = col + nxy * (uint32_t)k;
            const Cell q{i, j, k};
            // the face of direction f: interior (shared, from LDS or the column
            // registers) unless it lies on the domain boundary
            const int fxm = ty * (FT_X + 1) + tx, fym = ty * FT_X + tx;
            // whether face f has a neighbour in the domain, and that neighbour's LDS slot (x, y faces)
            auto inside = [&](int f) {
                return f == 0 ? i > 0 : f == 1 ? i + 1 < P.nx : f == 2 ? j > 0 : f == 3 ? j + 1 < P.ny
                     : f == 4 ? k > 0 : k + 1 < P.nz;
            };
            auto slot = [&](int f) { return f == 0 ? me - 1 : f == 1 ? me + 1 : f == 2 ? me - FT_RX : me + FT_RX; };
            if constexpr (!JAC) {
                double acc = (Lc.th - th_old[c]) / P.dt;
#pragma unroll
                for (int f = 0; f < 6; f++) {
                    if (inside(f)) {
                        // the cell is the lower one on its + faces
                        const double v = f == 0 ? fx[0][fxm] : f == 1 ? fx[0][fxm + 1] : f == 2 ? fy[0][fym]
                                       : f == 3 ? fy[0][fym + FT_X] : f == 4 ? q_dn : q_up;
                        acc += (f & 1) ? v : -v;
                        if (f == 4) acc += -g_dn;
                        if (f == 5) acc += g_up;
                        continue;
                    }
                    Face fc = face(P, q, c, f, p, Ks);
                    if (fc.kind == 0) continue;
                    Law Ln = laws(P, fc.pn, fc.Ksn);
                    double Kf, dcc, dnn;
                    int dir = (f & 1) ? 1 : -1;
                    mean_of<INTEG>(P, f >> 1, dir, pc, Lc, ksc, fc.pn, Ln, fc.Ksn, Kf, dcc, dnn);
                    acc += -Kf * (fc.pn - pc) / (fc.h * fc.h);
                    if ((f >> 1) == 2) acc += dir * (-(Lc.K + Ln.K) / (2.0 * P.hz));
                }
                F[c] = acc;
            } else {
                double jd = Lc.dth / P.dt, md = Lc.dth / P.dt;
                double joff[6] = {0, 0, 0, 0, 0, 0}, moff[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
                for (int f = 0; f < 6; f++) {
                    const int axis = f >> 1, dir = (f & 1) ? 1 : -1;
                    double Kf, dcc, dnn, pn, dKn, h2;
                    bool interior;
                    if (inside(f)) {
                        interior = true;
                        FaceMean m;
                        if (f < 2) {
                            const int t = fxm + f;
                            m = {fx[0][t], fx[1][t], fx[2][t]};
                        } else if (f < 4) {
                            const int t = fym + (f - 2) * FT_X;
                            m = {fy[0][t], fy[1][t], fy[2][t]};
                        } else {
                            m = f == 4 ? m_dn : m_up;
                        }
                        Kf = m.Kf;
                        // the cell is the lower one on its + faces
                        dcc = dir > 0 ? m.dL : m.dU;
                        dnn = dir > 0 ? m.dU : m.dL;
                        if (f < 4) {
                            pn = sp[slot(f)];
                            dKn = sdK[slot(f)];
                        } else {
                            pn = f == 4 ? pd : pu;
                            dKn = f == 4 ? dKd : Lu.dK;
                        }
                        h2 = axis == 0 ? hx2 : axis == 1 ? hy2 : hz2;
                    } else {
                        Face fc = face(P, q, c, f, p, Ks);
                        if (fc.kind == 0) continue;
                        interior = false;
                        Law Ln = laws(P, fc.pn, fc.Ksn);
                        mean_of<INTEG>(P, axis, dir, pc, Lc, ksc, fc.pn, Ln, fc.Ksn, Kf, dcc, dnn);
                        pn = fc.pn;
                        dKn = Ln.dK;
                        h2 = fc.h * fc.h;
                    }
                    const double dp = pn - pc;
                    const bool zf = axis == 2;
                    jd += Kf / h2 - dp / h2 * dcc;
                    if (zf) jd += -dir * Lc.dK / (2.0 * P.hz);
                    md += Kf / h2;
                    if (dflux) md += -dp / h2 * dcc;
                    if (interior) {
                        double v = -Kf / h2 - dp / h2 * dnn;
                        if (zf) v += -dir * dKn / (2.0 * P.hz);
                        joff[f] = v;
                        moff[f] = -Kf / h2;
                    }
                }
                J7[(size_t)J_D * n + c] = jd;
                J7[(size_t)J_XM * n + c] = joff[0];
                J7[(size_t)J_XP * n + c] = joff[1];
                J7[(size_t)J_YM * n + c] = joff[2];
                J7[(size_t)J_YP * n + c] = joff[3];
                J7[(size_t)J_ZM * n + c] = joff[4];
                J7[(size_t)J_ZP * n + c] = joff[5];
                M4[(size_t)M_D * n + c] = md;
                M4[(size_t)M_XP * n + c] = moff[1];
                M4[(size_t)M_YP * n + c] = moff[3];
                M4[(size_t)M_ZP * n + c] = moff[5];
                double l1 = md;
#pragma unroll
                for (int f = 0; f < 6; f++) l1 += fabs(moff[f]);
                if (M4f) {
                    M4f[(size_t)M_D * n + c] = f32_sat(md);
                    M4f[(size_t)M_XP * n + c] = f32_sat(moff[1]);
                    M4f[(size_t)M_YP * n + c] = f32_sat(moff[3]);
                    M4f[(size_t)M_ZP * n + c] = f32_sat(moff[5]);
                }
                if (invd) invd[c] = 1.0 / l1;
                if (invdf) invdf[c] = f32_sat(1.0 / l1);
            }
        }
        // carry the column up one plane
        if (up) {
            if constexpr (JAC) {
                pd = pc;
                dKd = Lc.dK;
                m_dn = m_up;
            } else {
                q_dn = q_up;
                g_dn = g_up;
            }
            pc = pu;
            ksc = ksu;
            Lc = Lu;
        }
        __syncthreads();  // the staged plane and faces are overwritten next
    }
}

// y = J x, J in the 7-array stencil form; x may be FP32 (mixed path).  With
// a shift vector (sb non-null) y = J x - sig (sbs[0] sb): the shifted power
// basis of the s-step GMRES, the subtraction after the stencil sum.
template <class TX, class G>
__device__ __forceinline__ void spmv_J_at(const G &P, uint32_t n, const double *__restrict__ J7,
                                          const TX *__restrict__ x, double *__restrict__ y, uint32_t c,
                                          const double *__restrict__ sb = nullptr,
                                          const double *__restrict__ sbs = nullptr, double sig = 0.0) {
    if (c >= n) return;
    Cell q = cell_of(P, c);
    uint32_t nx = P.nx, nxy = (uint32_t)P.nx * (uint32_t)P.ny;
    // J is streamed (non-temporal): its 7 arrays are far larger than the caches
#define JL(t) __builtin_nontemporal_load(J7 + (size_t)(t) * n + c)
    // An absent neighbour's index is clamped to the cell itself, so every load
    // is in bounds and all of them are issued before the first product (a
    // load inside each boundary test would wait for its value before the next
    // one is sent).  The sum keeps the order diag, -x, +x, -y, +y, -z, +z.
    const uint32_t cxm = q.i > 0 ? c - 1 : c, cxp = q.i < P.nx - 1 ? c + 1 : c;
    const uint32_t cym = q.j > 0 ? c - nx : c, cyp = q.j < P.ny - 1 ? c + nx : c;
    const uint32_t czm = q.k > 0 ? c - nxy : c, czp = q.k < P.nz - 1 ? c + nxy : c;
    const double a0 = JL(J_D), a1 = JL(J_XM), a2 = JL(J_XP), a3 = JL(J_YM), a4 = JL(J_YP), a5 = JL(J_ZM),
                 a6 = JL(J_ZP);
#undef JL
    const double x0 = (double)x[c], x1 = (double)x[cxm], x2 = (double)x[cxp], x3 = (double)x[cym],
                 x4 = (double)x[cyp], x5 = (double)x[czm], x6 = (double)x[czp];
    double s = a0 * x0;
    if (q.i > 0) s += a1 * x1;
    if (q.i < P.nx - 1) s += a2 * x2;
    if (q.j > 0) s += a3 * x3;
    if (q.j < P.ny - 1) s += a4 * x4;
    if (q.k > 0) s += a5 * x5;
    if (q.k < P.nz - 1) s += a6 * x6;
    // the shift input is not read again before it leaves the caches: streamed;
    // y is stored streaming too (the Gram-Schmidt dots that read it next run
    // faster than with y left in the caches)
    if (sb) s -= sig * (sbs[0] * __builtin_nontemporal_load(sb + c));
    __builtin_nontemporal_store(s, y + c);
}

template <class TX>
__global__ void k_spmv_J(Phys P, uint32_t n, const double *__restrict__ J7, const TX *__restrict__ x,
                         double *__restrict__ y, const double *__restrict__ sb, const double *__restrict__ sbs,
                         double sig) {
    spmv_J_at(P, n, J7, x, y, blockIdx.x * blockDim.x + threadIdx.x, sb, sbs, sig);
}

// Symmetric stencil M: sum_j m_cj * v_j with the -d couplings read at the lower neighbour.
template <class T, class G, class F>
__device__ inline T mstencil(const G &P, const Cell &q, uint32_t c, uint32_t n, const T *__restrict__ M4, F v) {
    uint32_t nx = P.nx, nxy = (uint32_t)P.nx * (uint32_t)P.ny;
    // absent neighbours clamped to the cell itself: every load is in bounds and
    // all are issued before the first product, as in the J product above
    const uint32_t cxm = q.i > 0 ? c - 1 : c, cxp = q.i < P.nx - 1 ? c + 1 : c;
    const uint32_t cym = q.j > 0 ? c - nx : c, cyp = q.j < P.ny - 1 ? c + nx : c;
    const uint32_t czm = q.k > 0 ? c - nxy : c, czp = q.k < P.nz - 1 ? c + nxy : c;
    const T m0 = M4[(size_t)M_D * n + c], m1 = M4[(size_t)M_XP * n + cxm], m2 = M4[(size_t)M_XP * n + c],
            m3 = M4[(size_t)M_YP * n + cym], m4 = M4[(size_t)M_YP * n + c], m5 = M4[(size_t)M_ZP * n + czm],
            m6 = M4[(size_t)M_ZP * n + c];
    const T v0 = v(c), v1 = v(cxm), v2 = v(cxp), v3 = v(cym), v4 = v(cyp), v5 = v(czm), v6 = v(czp);
    T s = m0 * v0;
    if (q.i > 0) s += m1 * v1;
    if (q.i < P.nx - 1) s += m2 * v2;
    if (q.j > 0) s += m3 * v3;
    if (q.j < P.ny - 1) s += m4 * v4;
    if (q.k > 0) s += m5 * v5;
    if (q.k < P.nz - 1) s += m6 * v6;
    return s;
}

__global__ void k_spmv_M(Phys P, uint32_t n, const double *__restrict__ M4, const double *__restrict__ x,
                         double *__restrict__ y) {
    uint32_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= n) return;
    Cell q = cell_of(P, c);
    y[c] = mstencil<double>(P, q, c, n, M4, [&](uint32_t t) { return x[t]; });
}

// V-cycle, fine level, pre-smoothing from x = 0 and residual in one pass:
// x0 = D^{-1} b (never stored), r = b - M x0.
template <class TB, class T, class G>
__device__ __forceinline__ void st_pre_at(const G &P, uint32_t n, const T *__restrict__ M4,
                                          const T *__restrict__ invd, const TB *__restrict__ b,
                                          const double *__restrict__ bsp, T *__restrict__ r, uint32_t c) {
    if (c >= n) return;
    const TB bs = (TB)bsp[0];
    Cell q = cell_of(P, c);
    T s = mstencil<T>(P, q, c, n, M4, [&](uint32_t t) { return (T)(b[t] * bs) * invd[t]; });
    r[c] = (T)(b[c] * bs) - s;
}

template <class TB, class T>
__global__ void k_st_pre(Phys P, uint32_t n, const T *__restrict__ M4, const T *__restrict__ invd,
                         const TB *__restrict__ b, const double *__restrict__ bsp, T *__restrict__ r) {
    st_pre_at(P, n, M4, invd, b, bsp, r, xcd_block() * blockDim.x + threadIdx.x);
}

// V-cycle, fine level, prolongation: xt = D^{-1} b + P xc (the pre-smoothed
// iterate plus the coarse correction), one streaming pass.
template <class TB, class T>
__device__ __forceinline__ void st_prolong_at(uint32_t n, const T *__restrict__ invd, const TB *__restrict__ b,
                                              const double *__restrict__ bsp, const T *__restrict__ xc,
                                              const int32_t *__restrict__ agg, T *__restrict__ xt, uint32_t c) {
    if (c >= n) return;
    xt[c] = (T)(b[c] * (TB)bsp[0]) * invd[c] + xc[agg[c]];
}

template <class TB, class T>
__global__ void k_st_prolong(uint32_t n, const T *__restrict__ invd, const TB *__restrict__ b,
                             const double *__restrict__ bsp, const T *__restrict__ xc, const int32_t *__restrict__ agg,
                             T *__restrict__ xt) {
    st_prolong_at(n, invd, b, bsp, xc, agg, xt, xcd_block() * blockDim.x + threadIdx.x);
}

// V-cycle, fine level, post-smoothing: x = xt + D^{-1}(b - M xt).
template <class TB, class T, class G>
__device__ __forceinline__ void st_post_at(const G &P, uint32_t n, const T *__restrict__ M4,
                                           const T *__restrict__ invd, const TB *__restrict__ b,
                                           const double *__restrict__ bsp, const T *__restrict__ xt,
                                           T *__restrict__ x, uint32_t c) {
    if (c >= n) return;
    Cell q = cell_of(P, c);
    T s = mstencil<T>(P, q, c, n, M4, [&](uint32_t t) { return xt[t]; });
    x[c] = xt[c] + invd[c] * ((T)(b[c] * (TB)bsp[0]) - s);
}

template <class TB, class T>
__global__ void k_st_post(Phys P, uint32_t n, const T *__restrict__ M4, const T *__restrict__ invd,
                          const TB *__restrict__ b, const double *__restrict__ bsp, const T *__restrict__ xt,
                          T *__restrict__ x) {
    st_post_at(P, n, M4, invd, b, bsp, xt, x, xcd_block() * blockDim.x + threadIdx.x);
}

// 2.5-D versions of the fine-level V-cycle stencils.  A block of 64 x 8
// threads owns a 64 x 8 column tile and walks a chunk of kz planes upward:
// the stencil input u of the planes below and above stays in registers, the
// current plane (with a one-cell halo) and its +x / +y couplings (with the
// lower neighbours' ones) go through LDS, so every cell's data is loaded from
// memory once (halos aside).  Loads run ahead of the arithmetic: while plane
// k is computed, the coefficients and halo inputs of plane k+1 and the
// column inputs of plane k+2 are already in flight; LDS is double-buffered
// by plane parity, so one barrier per plane suffices.  The sums keep the
// order of mstencil (diag, -x, +x, -y, +y, -z, +z).
//   ST25_PRE  : u = D^{-1} bs b (pre-smoothing from zero),  out = bs b - M u
//   ST25_POST : u = D^{-1} bs b + P xc (piecewise-constant prolongation
//               fused),                                     out = u + D^{-1}(bs b - M u)
//   ST25_XT   : u = xt (a stored prolongated iterate),      out as ST25_POST
#ifndef ST25_TY
#define ST25_TY 8
#endif
constexpr int T25X = 64, T25Y = ST25_TY;
#ifndef ST25_MIN_BLOCKS
#define ST25_MIN_BLOCKS 2048
#endif
enum { ST25_PRE = 0, ST25_POST = 1, ST25_XT = 2 };

// The inputs of u at one cell as loaded (u is formed when it is used).
template <class T, class TB>
struct St25In {
    TB b = 0;  // b as loaded: scaled and rounded where it is used
    T d = 0, x = 0;  // D^{-1}, xc[agg] or xt
};

// L: the tile (virtual block) this block computes.
template <class TB, class T, int MODE, class G>
__device__ __forceinline__ void st25_body(const G &P, const T *__restrict__ M4, const T *__restrict__ invd,
                                          const TB *__restrict__ b, const double *__restrict__ bsp,
                                          const T *__restrict__ xc, const int32_t *__restrict__ agg,
                                          T *__restrict__ out, int kz, unsigned L) {
    constexpr bool POST = MODE != ST25_PRE;
    __shared__ T us[2][T25Y + 2][T25X + 2];
    __shared__ T xps[2][T25Y][T25X + 1];
    __shared__ T yps[2][T25Y + 1][T25X];
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const uint32_t n = (uint32_t)nx * (uint32_t)ny * (uint32_t)nz;
    const uint32_t nxy = (uint32_t)nx * (uint32_t)ny;
    // XCD-aware tile order: the blocks one XCD runs are consecutive tiles
    // (x fastest), so the halos a tile shares with its neighbours are mostly
    // fetched once into that XCD's L2.
    const unsigned ntx = (unsigned)(nx + T25X - 1) / T25X, nty = (unsigned)(ny + T25Y - 1) / T25Y;
    if (L >= ntx * nty * (unsigned)((nz + kz - 1) / kz)) return;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int i = (int)(L % ntx) * T25X + tx, j = (int)((L / ntx) % nty) * T25Y + ty;
    const int k0 = (int)(L / (ntx * nty)) * kz, k1 = min(k0 + kz, nz);
    const bool inside = i < nx && j < ny;
    const TB bs = (TB)bsp[0];
    // which halo cell this thread also loads (at most one in x and one in y)
    const bool hxl = tx == 0 && i > 0 && j < ny, hxr = tx == T25X - 1 && i + 1 < nx && j < ny;
    const bool hyl = ty == 0 && j > 0 && i < nx, hyr = ty == T25Y - 1 && j + 1 < ny && i < nx;
    const int hxo = hxl ? -1 : 1;
    const int hyo = hyl ? -nx : nx;
    const bool hx = hxl || hxr, hy = hyl || hyr;

    // a prefetched b is only scaled when it is used: converting it at once
    // would wait for its load, and with it for every load issued before it
    auto bval = [&](const St25In<T, TB> &r) -> T { return (T)(r.b * bs); };
    auto load_in = [&](uint32_t c) {
        St25In<T, TB> r;
        if (MODE != ST25_XT) r.b = b[c];
        if (MODE != ST25_XT) r.d = invd[c];
        if (MODE == ST25_POST) r.x = xc[agg[c]];
        if (MODE == ST25_XT) r.x = xc[c];
        return r;
    };
    auto u_of = [&](const St25In<T, TB> &r) -> T {
        if (MODE == ST25_XT) return r.x;
        T u = bval(r) * r.d;
        if (MODE == ST25_POST) u += r.x;
        return u;
    };
    auto b_of = [&](uint32_t c) -> T { return (T)(b[c] * bs); };

    // plane state: coefficients of plane k (own, and the lower-neighbour
    // halo couplings), halo inputs of plane k, column inputs of k, k+1, k+2
    T m_d = 0, m_xp = 0, m_yp = 0, m_zp = 0, h_xp = 0, h_yp = 0;
    St25In<T, TB> c0, c1, c2, hxin, hyin;
    T u_prev = 0, zp_prev = 0;
    uint32_t c = (uint32_t)i + (uint32_t)nx * ((uint32_t)j + (uint32_t)ny * (uint32_t)k0);
    auto load_plane = [&](uint32_t cc, T &md, T &mxp, T &myp, T &mzp, T &hxp, T &hyp, St25In<T, TB> &hxi,
                          St25In<T, TB> &hyi) {
        if (inside) {
            // a cell's own coefficients are read once: streamed past the caches
            // (the halo couplings below are shared with the neighbouring tiles)
            md = __builtin_nontemporal_load(M4 + (size_t)M_D * n + cc);
            mxp = __builtin_nontemporal_load(M4 + (size_t)M_XP * n + cc);
            myp = __builtin_nontemporal_load(M4 + (size_t)M_YP * n + cc);
            mzp = __builtin_nontemporal_load(M4 + (size_t)M_ZP * n + cc);
        }
        if (hx) {
            hxi = load_in(cc + hxo);
            if (hxl) hxp = M4[(size_t)M_XP * n + cc - 1];
        }
        if (hy) {
            hyi = load_in(cc + hyo);
            if (hyl) hyp = M4[(size_t)M_YP * n + cc - nx];
        }
    };
    if (inside) {
        c0 = load_in(c);
        if (k0 + 1 < nz) c1 = load_in(c + nxy);
        if (k0 > 0) {
            u_prev = u_of(load_in(c - nxy));
            zp_prev = M4[(size_t)M_ZP * n + c - nxy];
        }
    }
    load_plane(c, m_d, m_xp, m_yp, m_zp, h_xp, h_yp, hxin, hyin);
    for (int k = k0; k < k1; k++, c += nxy) {
        const int q = (k - k0) & 1;
        // loads for the next iteration
        T n_d = 0, n_xp = 0, n_yp = 0, n_zp = 0, nh_xp = 0, nh_yp = 0;
        St25In<T, TB> nhx, nhy;
        if (k + 1 < k1) load_plane(c + nxy, n_d, n_xp, n_yp, n_zp, nh_xp, nh_yp, nhx, nhy);
        if (inside && k + 2 < nz && k + 1 < k1) c2 = load_in(c + 2 * nxy);
        // this plane through LDS
        const T u_cur = u_of(c0);
        const T u_nxt = (inside && k + 1 < nz) ? u_of(c1) : (T)0;
        us[q][ty + 1][tx + 1] = inside ? u_cur : (T)0;
        xps[q][ty][tx + 1] = m_xp;
        yps[q][ty + 1][tx] = m_yp;
        if (tx == 0) {
            us[q][ty + 1][0] = hxl ? u_of(hxin) : (T)0;
            xps[q][ty][0] = h_xp;
        }
        if (tx == T25X - 1) us[q][ty + 1][T25X + 1] = hxr ? u_of(hxin) : (T)0;
        if (ty == 0) {
            us[q][0][tx + 1] = hyl ? u_of(hyin) : (T)0;
            yps[q][0][tx] = h_yp;
        }
        if (ty == T25Y - 1) us[q][T25Y + 1][tx + 1] = hyr ? u_of(hyin) : (T)0;
        __syncthreads();
        if (inside) {
            T s = m_d * u_cur;
            if (i > 0) s += xps[q][ty][tx] * us[q][ty + 1][tx];
            if (i < nx - 1) s += xps[q][ty][tx + 1] * us[q][ty + 1][tx + 2];
            if (j > 0) s += yps[q][ty][tx] * us[q][ty][tx + 1];
            if (j < ny - 1) s += yps[q][ty + 1][tx] * us[q][ty + 2][tx + 1];
            if (k > 0) s += zp_prev * u_prev;
            if (k < nz - 1) s += m_zp * u_nxt;
            const T bc = MODE == ST25_XT ? b_of(c) : bval(c0);
            const T dc = MODE == ST25_XT ? invd[c] : c0.d;
            out[c] = POST ? u_cur + dc * (bc - s) : bc - s;
        }
        // rotate (the other LDS buffer is written next: no second barrier)
        u_prev = u_cur;
        zp_prev = m_zp;
        c0 = c1;
        c1 = c2;
        m_d = n_d;
        m_xp = n_xp;
        m_yp = n_yp;
        m_zp = n_zp;
        h_xp = nh_xp;
        h_yp = nh_yp;
        hxin = nhx;
        hyin = nhy;
    }
}

template <class TB, class T, int MODE>
__global__ void __launch_bounds__(T25X * T25Y) k_st25(Phys P, const T *__restrict__ M4, const T *__restrict__ invd,
                                                     const TB *__restrict__ b, const double *__restrict__ bsp,
                                                     const T *__restrict__ xc, const int32_t *__restrict__ agg,
                                                     T *__restrict__ out, int kz) {
    st25_body<TB, T, MODE>(P, M4, invd, b, bsp, xc, agg, out, kz, xcd_block());
}

// Batched forms: one launch over the fine levels of several simulations.
template <class TB, class T>
struct StArgs {
    Grid3 g;
    uint32_t n;
    int kz;
    const T *M4, *invd;
    const TB *b;
    const double *bs;
    const T *xc;
    const int32_t *agg;
    T *xt, *out;
};

template <class TB, class T, int MODE>
__global__ void __launch_bounds__(T25X * T25Y) k_st25_batch(Batch<StArgs<TB, T>> B) {
    for_each_block(B, xcd_block(), [&](unsigned L) {
        const int e = batch_entry(B, L);
        const StArgs<TB, T> &a = B.a[e];
        st25_body<TB, T, MODE>(a.g, a.M4, a.invd, a.b, a.bs, a.xc, a.agg, a.out, a.kz, L - B.begin[e]);
    });
}

// MODE 0: pre-smoothing + residual, 1: prolongation into xt, 2: post-smoothing from xt
template <class TB, class T, int MODE>
__global__ void k_st1_batch(Batch<StArgs<TB, T>> B) {
    for_each_block(B, xcd_block(), [&](unsigned L) {
        const int e = batch_entry(B, L);
        const StArgs<TB, T> &a = B.a[e];
        const uint32_t c = (L - B.begin[e]) * blockDim.x + threadIdx.x;
        if (MODE == 0) st_pre_at(a.g, a.n, a.M4, a.invd, a.b, a.bs, a.out, c);
        if (MODE == 1) st_prolong_at(a.n, a.invd, a.b, a.bs, a.xc, a.agg, a.xt, c);
        if (MODE == 2) st_post_at(a.g, a.n, a.M4, a.invd, a.b, a.bs, a.xt, a.out, c);
    });
}

template <class TX>
struct SpmvArgs {
    Grid3 g;
    uint32_t n;
    const double *J7;
    const TX *x;
    double *y;
    const double *sb, *sbs;  // optional shift: y = J x - sig (sbs[0] sb)
    double sig;
};

template <class TX>
__global__ void k_spmv_J_batch(Batch<SpmvArgs<TX>> B) {
    for_each_block(B, xcd_block(), [&](unsigned L) {
        const int e = batch_entry(B, L);
        const SpmvArgs<TX> &a = B.a[e];
        spmv_J_at(a.g, a.n, a.J7, a.x, a.y, (L - B.begin[e]) * blockDim.x + threadIdx.x, a.sb, a.sbs, a.sig);
    });
}

// The 64-wide tile needs rows of at least about that length to keep its lanes busy.
inline bool use25(const Phys &P) { return P.nx >= 48 && P.ny >= T25Y && P.nz >= 4; }
// Planes per block: the fewest chunks of at most 16 planes that give at least
// ST25_MIN_BLOCKS blocks, with the planes spread evenly over the chunks (a
// short last chunk leaves its blocks' share of the sweep idle).
inline int kz25(const Phys &P) {
    if (P.tile_kz > 0) return P.tile_kz < P.nz ? P.tile_kz : P.nz;
    int64_t tiles = (int64_t)((P.nx + T25X - 1) / T25X) * ((P.ny + T25Y - 1) / T25Y);
    int64_t chunks = std::max<int64_t>((ST25_MIN_BLOCKS + tiles - 1) / tiles, (P.nz + 15) / 16);
    chunks = std::min<int64_t>(chunks, P.nz);
    return (int)((P.nz + chunks - 1) / chunks);
}
inline int64_t tiles25(const Phys &P, int kz) {
    return (int64_t)((P.nx + T25X - 1) / T25X) * ((P.ny + T25Y - 1) / T25Y) * ((P.nz + kz - 1) / kz);
}
inline unsigned grid25(const Phys &P, int kz) { return xcd_grid(tiles25(P, kz), 1); }

// Multicolour Gauss-Seidel on the fine level (the GPU form of the hybrid
// backward/forward Gauss-Seidel smoother of the paper's experiments, Section
// 6): colour (i + j + k) mod 2, so cells of one colour couple only to cells of
// the other; x_c = (b_c - sum_n m_cn x_n) / m_cc, the terms subtracted in
// ascending column order (-z, -y, -x, +x, +y, +z).
template <class T, class G, class F>
__device__ inline T gs_row(const G &P, const Cell &q, uint32_t c, uint32_t n, const T *__restrict__ M4, T bc, F v) {
    uint32_t nx = P.nx, nxy = (uint32_t)P.nx * (uint32_t)P.ny;
    T s = bc;
    if (q.k > 0) s -= M4[(size_t)M_ZP * n + c - nxy] * v(c - nxy);
    if (q.j > 0) s -= M4[(size_t)M_YP * n + c - nx] * v(c - nx);
    if (q.i > 0) s -= M4[(size_t)M_XP * n + c - 1] * v(c - 1);
    if (q.i < P.nx - 1) s -= M4[(size_t)M_XP * n + c] * v(c + 1);
    if (q.j < P.ny - 1) s -= M4[(size_t)M_YP * n + c] * v(c + nx);
    if (q.k < P.nz - 1) s -= M4[(size_t)M_ZP * n + c] * v(c + nxy);
    return s / M4[(size_t)M_D * n + c];
}

// Pre-smoothing, one backward sweep from x = 0: colour 1 takes b / m_cc, then
// colour 0 takes its row with those values (formed on the fly): one pass.
template <class TB, class T>
__global__ void k_gs_pre(Phys P, uint32_t n, const T *__restrict__ M4, const TB *__restrict__ b,
                         const double *__restrict__ bsp, T *__restrict__ x0) {
    uint32_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const TB bs = (TB)bsp[0];
    Cell q = cell_of(P, c);
    const T bc = (T)(b[c] * bs);
    if ((q.i + q.j + q.k) & 1) {
        x0[c] = bc / M4[(size_t)M_D * n + c];
        return;
    }
    x0[c] = gs_row<T>(P, q, c, n, M4, bc, [&](uint32_t t) { return (T)(b[t] * bs) / M4[(size_t)M_D * n + t]; });
}

// r = bs b - M x
template <class TB, class T>
__global__ void k_gs_res(Phys P, uint32_t n, const T *__restrict__ M4, const TB *__restrict__ b,
                         const double *__restrict__ bsp, const T *__restrict__ x, T *__restrict__ r) {
    uint32_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= n) return;
    Cell q = cell_of(P, c);
    T s = mstencil<T>(P, q, c, n, M4, [&](uint32_t t) { return x[t]; });
    r[c] = (T)(b[c] * (TB)bsp[0]) - s;
}

// xt = x0 + P xc (piecewise-constant prolongation)
template <class T>
__global__ void k_gs_prolong(uint32_t n, const T *__restrict__ x0, const T *__restrict__ xc,
                             const int32_t *__restrict__ agg, T *__restrict__ xt) {
    uint32_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= n) return;
    xt[c] = x0[c] + xc[agg[c]];
}

// One colour of a sweep: cells of `color` take their row on x_in; the other
// cells copy x_in when x_out is another vector (in place they keep theirs:
// a cell of `color` reads only cells of the other colour, so it is race free).
template <class TB, class T>
__global__ void k_gs_color(Phys P, uint32_t n, const T *__restrict__ M4, const TB *__restrict__ b,
                           const double *__restrict__ bsp, int color, const T *x_in, T *x_out) {
    uint32_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= n) return;
    Cell q = cell_of(P, c);
    if (((q.i + q.j + q.k) & 1) != color) {
        if (x_out != x_in) x_out[c] = x_in[c];
        return;
    }
    const T bc = (T)(b[c] * (TB)bsp[0]);
    x_out[c] = gs_row<T>(P, q, c, n, M4, bc, [&](uint32_t t) { return x_in[t]; });
}

// Plain l1-Jacobi sweep x_out = x_in + D^{-1}(b - M x_in) (used when the
// fine level is also the coarsest and too large for a direct solve).
template <class TB, class T>
__global__ void k_st_sweep(Phys P, uint32_t n, const T *__restrict__ M4, const T *__restrict__ invd,
                           const TB *__restrict__ b, const T *__restrict__ xin, T *__restrict__ xout, int zero) {
    uint32_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= n) return;
    if (zero) {
        xout[c] = (T)b[c] * invd[c];
        return;
    }
    Cell q = cell_of(P, c);
    T s = mstencil<T>(P, q, c, n, M4, [&](uint32_t t) { return xin[t]; });
    xout[c] = xin[c] + invd[c] * ((T)b[c] - s);
}

__global__ void k_stencil_rowcounts(Phys P, uint32_t n, int64_t *__restrict__ cnt) {
    uint32_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= n) return;
    Cell q = cell_of(P, c);
    cnt[c] = 1 + (q.i > 0) + (q.i < P.nx - 1) + (q.j > 0) + (q.j < P.ny - 1) + (q.k > 0) + (q.k < P.nz - 1);
}

// Stencil -> CSR with ascending columns (-z,-y,-x,c,+x,+y,+z).
__global__ void k_M_to_csr(Phys P, uint32_t n, const double *__restrict__ M4, const int64_t *__restrict__ rowptr,
                           int32_t *__restrict__ col, double *__restrict__ val) {
    uint32_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= n) return;
    Cell q = cell_of(P, c);
    uint32_t nx = P.nx, nxy = (uint32_t)P.nx * (uint32_t)P.ny;
    int64_t e = rowptr[c];
    if (q.k > 0) { col[e] = c - nxy; val[e++] = M4[(size_t)M_ZP * n + c - nxy]; }
    if (q.j > 0) { col[e] = c - nx; val[e++] = M4[(size_t)M_YP * n + c - nx]; }
    if (q.i > 0) { col[e] = c - 1; val[e++] = M4[(size_t)M_XP * n + c - 1]; }
    col[e] = c; val[e++] = M4[(size_t)M_D * n + c];
    if (q.i < P.nx - 1) { col[e] = c + 1; val[e++] = M4[(size_t)M_XP * n + c]; }
    if (q.j < P.ny - 1) { col[e] = c + nx; val[e++] = M4[(size_t)M_YP * n + c]; }
    if (q.k < P.nz - 1) { col[e] = c + nxy; val[e++] = M4[(size_t)M_ZP * n + c]; }
}

__global__ void k_J_to_csr(Phys P, uint32_t n, const double *__restrict__ J7, const int64_t *__restrict__ rowptr,
                           int32_t *__restrict__ col, double *__restrict__ val) {
    uint32_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= n) return;
    Cell q = cell_of(P, c);
    uint32_t nx = P.nx, nxy = (uint32_t)P.nx * (uint32_t)P.ny;
    int64_t e = rowptr[c];
    if (q.k > 0) { col[e] = c - nxy; val[e++] = J7[(size_t)J_ZM * n + c]; }
    if (q.j > 0) { col[e] = c - nx; val[e++] = J7[(size_t)J_YM * n + c]; }
    if (q.i > 0) { col[e] = c - 1; val[e++] = J7[(size_t)J_XM * n + c]; }
    col[e] = c; val[e++] = J7[(size_t)J_D * n + c];
    if (q.i < P.nx - 1) { col[e] = c + 1; val[e++] = J7[(size_t)J_XP * n + c]; }
    if (q.j < P.ny - 1) { col[e] = c + nx; val[e++] = J7[(size_t)J_YP * n + c]; }
    if (q.k < P.nz - 1) { col[e] = c + nxy; val[e++] = J7[(size_t)J_ZP * n + c]; }
}

}  // namespace

static inline uint32_t ncells(const Phys &P) { return (uint32_t)((int64_t)P.nx * P.ny * P.nz); }

rich_status launch_theta(const Phys &P, const double *p, double *theta, hipStream_t s) {
    uint32_t n = ncells(P);
    k_theta<<<nblocks(n), TPB, 0, s>>>(P, n, p, theta);
    LAUNCH_CHECK();
    return RICH_OK;
}

// Grid of the plane-tiled kernels: FT_X x FT_Y columns per block and enough
// planes per block that the launch has about 2048 blocks; false when the
// (x, y) tiling does not fit the launch limits (the one-thread-per-cell
// kernels take those grids).
static bool has_integral(const Phys &P) {
    return P.mean == RICH_MEAN_INTEGRAL || P.mean_vertical == RICH_MEAN_INTEGRAL;
}

static bool faces_grid(const Phys &P, dim3 *g, int *kz) {
    const int64_t tx = (P.nx + FT_X - 1) / FT_X, ty = (P.ny + FT_Y - 1) / FT_Y;
    if (tx > 0x7fffffff || ty > 65535) return false;
    const int64_t want = std::max<int64_t>(1, 2048 / std::max<int64_t>(1, tx * ty));
    int64_t z = (P.nz + want - 1) / want;
    z = std::min<int64_t>(std::max<int64_t>(z, 1), 64);
    const int64_t tz = (P.nz + z - 1) / z;
    if (tz > 65535) return false;
    *g = dim3((unsigned)tx, (unsigned)ty, (unsigned)tz);
    *kz = (int)z;
    return true;
}

rich_status launch_residual(const Phys &P, const double *Ks, const double *p, const double *theta_old,
                            double *F, hipStream_t s) {
    uint32_t n = ncells(P);
    dim3 g;
    int kz;
    if (faces_grid(P, &g, &kz)) {
        if (has_integral(P))
            k_faces_tiled<false, true><<<g, FT_TPB, 0, s>>>(P, kz, Ks, p, theta_old, F, nullptr, nullptr, nullptr,
                                                            nullptr, nullptr, 0);
        else
            k_faces_tiled<false, false><<<g, FT_TPB, 0, s>>>(P, kz, Ks, p, theta_old, F, nullptr, nullptr, nullptr,
                                                             nullptr, nullptr, 0);
    } else
        k_residual<<<nblocks(n), TPB, 0, s>>>(P, n, Ks, p, theta_old, F);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status launch_assemble(const Phys &P, const double *Ks, const double *p, double *J7, double *M4,
                            float *M4f, double *invd, float *invdf, int dflux, hipStream_t s) {
    uint32_t n = ncells(P);
    dim3 g;
    int kz;
    if (faces_grid(P, &g, &kz)) {
        if (has_integral(P))
            k_faces_tiled<true, true><<<g, FT_TPB, 0, s>>>(P, kz, Ks, p, nullptr, nullptr, J7, M4, M4f, invd, invdf,
                                                           dflux);
        else
            k_faces_tiled<true, false><<<g, FT_TPB, 0, s>>>(P, kz, Ks, p, nullptr, nullptr, J7, M4, M4f, invd,
                                                            invdf, dflux);
    } else
        k_assemble<<<nblocks(n), TPB, 0, s>>>(P, n, Ks, p, J7, M4, M4f, invd, invdf, dflux);
    LAUNCH_CHECK();
    return RICH_OK;
}

template <class TX>
rich_status launch_spmv_J(const Phys &P, const double *J7, const TX *x, double *y, hipStream_t s, const double *sb,
                          const double *sbs, double sig) {
    uint32_t n = ncells(P);
    k_spmv_J<TX><<<(n + TPB - 1) / TPB, TPB, 0, s>>>(P, n, J7, x, y, sb, sbs, sig);
    LAUNCH_CHECK();
    return RICH_OK;
}
template rich_status launch_spmv_J<double>(const Phys &, const double *, const double *, double *, hipStream_t,
                                           const double *, const double *, double);
template rich_status launch_spmv_J<float>(const Phys &, const double *, const float *, double *, hipStream_t,
                                          const double *, const double *, double);

rich_status launch_spmv_M(const Phys &P, const double *M4, const double *x, double *y, hipStream_t s) {
    uint32_t n = ncells(P);
    k_spmv_M<<<nblocks(n), TPB, 0, s>>>(P, n, M4, x, y);
    LAUNCH_CHECK();
    return RICH_OK;
}

template <class TB, class T>
rich_status launch_st_pre(const Phys &P, const T *M4, const T *invd, const TB *b, const double *bs, T *r,
                          hipStream_t s) {
    uint32_t n = ncells(P);
    if (use25(P)) {
        int kz = kz25(P);
        k_st25<TB, T, ST25_PRE><<<grid25(P, kz), dim3(T25X, T25Y), 0, s>>>(P, M4, invd, b, bs, nullptr, nullptr, r, kz);
    } else {
        k_st_pre<TB, T><<<nblocks(n), TPB, 0, s>>>(P, n, M4, invd, b, bs, r);
    }
    LAUNCH_CHECK();
    return RICH_OK;
}

template <class TB, class T>
rich_status launch_st_post(const Phys &P, const T *M4, const T *invd, const TB *b, const double *bs, const T *xc,
                           const int32_t *agg, T *x, T *xt, hipStream_t s) {
    uint32_t n = ncells(P);
    if (use25(P)) {
        int kz = kz25(P);
        k_st25<TB, T, ST25_POST><<<grid25(P, kz), dim3(T25X, T25Y), 0, s>>>(P, M4, invd, b, bs, xc, agg, x, kz);
    } else {
        k_st_prolong<TB, T><<<nblocks(n), TPB, 0, s>>>(n, invd, b, bs, xc, agg, xt);
        LAUNCH_CHECK();
        k_st_post<TB, T><<<nblocks(n), TPB, 0, s>>>(P, n, M4, invd, b, bs, xt, x);
    }
    LAUNCH_CHECK();
    return RICH_OK;
}

template <class TB, class T>
rich_status launch_st_post_from(const Phys &P, const T *M4, const T *invd, const TB *b, const double *bs,
                                const T *xt, T *x, hipStream_t s) {
    uint32_t n = ncells(P);
    if (use25(P)) {
        int kz = kz25(P);
        k_st25<TB, T, ST25_XT><<<grid25(P, kz), dim3(T25X, T25Y), 0, s>>>(P, M4, invd, b, bs, xt, nullptr, x, kz);
    } else {
        k_st_post<TB, T><<<nblocks(n), TPB, 0, s>>>(P, n, M4, invd, b, bs, xt, x);
    }
    LAUNCH_CHECK();
    return RICH_OK;
}

template <class TB, class T>
rich_status launch_st_sweeps(const Phys &P, const T *M4, const T *invd, const TB *b, T *x, T *tmp,
                             int sweeps, hipStream_t s) {
    uint32_t n = ncells(P);
    // x <- D^{-1} b is the first sweep from zero; then ping-pong x <-> tmp.
    T *cur = (sweeps % 2 == 1) ? x : tmp;
    k_st_sweep<TB, T><<<nblocks(n), TPB, 0, s>>>(P, n, M4, invd, b, nullptr, cur, 1);
    LAUNCH_CHECK();
    for (int t = 1; t < sweeps; t++) {
        T *nxt = (cur == x) ? tmp : x;
        k_st_sweep<TB, T><<<nblocks(n), TPB, 0, s>>>(P, n, M4, invd, b, cur, nxt, 0);
        LAUNCH_CHECK();
        cur = nxt;
    }
    return RICH_OK;
}

template <class TB, class T>
rich_status launch_gs_pre(const Phys &P, const T *M4, const TB *b, const double *bs, T *x0, T *r, hipStream_t s) {
    uint32_t n = ncells(P);
    k_gs_pre<TB, T><<<nblocks(n), TPB, 0, s>>>(P, n, M4, b, bs, x0);
    LAUNCH_CHECK();
    k_gs_res<TB, T><<<nblocks(n), TPB, 0, s>>>(P, n, M4, b, bs, x0, r);
    LAUNCH_CHECK();
    return RICH_OK;
}

template <class TB, class T>
rich_status launch_gs_post(const Phys &P, const T *M4, const TB *b, const double *bs, const T *x0, const T *xc,
                           const int32_t *agg, T *xt, T *x, hipStream_t s) {
    uint32_t n = ncells(P);
    if (agg) {
        k_gs_prolong<T><<<nblocks(n), TPB, 0, s>>>(n, x0, xc, agg, xt);
        LAUNCH_CHECK();
    }
    // forward sweep: colour 0 in place, then colour 1 into x
    k_gs_color<TB, T><<<nblocks(n), TPB, 0, s>>>(P, n, M4, b, bs, 0, xt, xt);
    LAUNCH_CHECK();
    k_gs_color<TB, T><<<nblocks(n), TPB, 0, s>>>(P, n, M4, b, bs, 1, xt, x);
    LAUNCH_CHECK();
    return RICH_OK;
}

template <class TB, class T>
static StArgs<TB, T> st_args(const FineItem<TB, T> &it, int kz) {
    const Phys &P = *it.P;
    StArgs<TB, T> a;
    a.g = Grid3{P.nx, P.ny, P.nz};
    a.n = ncells(P);
    a.kz = kz;
    a.M4 = it.M4;
    a.invd = it.invd;
    a.b = it.b;
    a.bs = it.bs;
    a.xc = it.xc;
    a.agg = it.agg;
    a.xt = it.xt;
    a.out = it.out;
    return a;
}

// Split the items into those on the tiled kernel and those on the plain one.
template <class TB, class T>
static void st_split(const std::vector<FineItem<TB, T>> &v, std::vector<StArgs<TB, T>> &a25,
                     std::vector<unsigned> &b25, std::vector<StArgs<TB, T>> &a1, std::vector<unsigned> &b1) {
    for (const auto &it : v) {
        const Phys &P = *it.P;
        if (use25(P)) {
            int kz = kz25(P);
            a25.push_back(st_args(it, kz));
            b25.push_back((unsigned)tiles25(P, kz));
        } else {
            a1.push_back(st_args(it, 0));
            b1.push_back((ncells(P) + TPB - 1) / TPB);
        }
    }
}

template <class TB, class T>
rich_status launch_st_pre_batch(const std::vector<FineItem<TB, T>> &v, hipStream_t s, WorkQueue *q) {
    std::vector<StArgs<TB, T>> a25, a1;
    std::vector<unsigned> b25, b1;
    st_split(v, a25, b25, a1, b1);
    using B = Batch<StArgs<TB, T>>;
    RICH_TRY(launch_batches(a25, b25, [&](const B &bt, unsigned g) {
        k_st25_batch<TB, T, ST25_PRE><<<g, dim3(T25X, T25Y), 0, s>>>(bt);
    }, q));
    return launch_batches(a1, b1, [&](const B &bt, unsigned g) { k_st1_batch<TB, T, 0><<<g, TPB, 0, s>>>(bt); }, q);
}

template <class TB, class T>
rich_status launch_st_post_batch(const std::vector<FineItem<TB, T>> &v, hipStream_t s, WorkQueue *q) {
    std::vector<StArgs<TB, T>> a25, a1;
    std::vector<unsigned> b25, b1;
    st_split(v, a25, b25, a1, b1);
    using B = Batch<StArgs<TB, T>>;
    RICH_TRY(launch_batches(a25, b25, [&](const B &bt, unsigned g) {
        k_st25_batch<TB, T, ST25_POST><<<g, dim3(T25X, T25Y), 0, s>>>(bt);
    }, q));
    RICH_TRY(launch_batches(a1, b1, [&](const B &bt, unsigned g) { k_st1_batch<TB, T, 1><<<g, TPB, 0, s>>>(bt); },
                            q));
    return launch_batches(a1, b1, [&](const B &bt, unsigned g) { k_st1_batch<TB, T, 2><<<g, TPB, 0, s>>>(bt); }, q);
}

template <class TX>
rich_status launch_spmv_J_batch(const std::vector<SpmvItem<TX>> &v, hipStream_t s, WorkQueue *q) {
    std::vector<SpmvArgs<TX>> a;
    std::vector<unsigned> nb;
    for (const auto &it : v) {
        const Phys &P = *it.P;
        a.push_back(SpmvArgs<TX>{Grid3{P.nx, P.ny, P.nz}, ncells(P), it.J7, it.x, it.y, it.sb, it.sbs, it.sig});
        nb.push_back((ncells(P) + TPB - 1) / TPB);
    }
    return launch_batches(a, nb, [&](const Batch<SpmvArgs<TX>> &bt, unsigned g) {
        k_spmv_J_batch<TX><<<g, TPB, 0, s>>>(bt);
    }, q);
}
template rich_status launch_spmv_J_batch<double>(const std::vector<SpmvItem<double>> &, hipStream_t, WorkQueue *);
template rich_status launch_spmv_J_batch<float>(const std::vector<SpmvItem<float>> &, hipStream_t, WorkQueue *);

#define INST_ST(TB, T)                                                                                    \
    template rich_status launch_st_pre<TB, T>(const Phys &, const T *, const T *, const TB *, const double *, T *, \
                                              hipStream_t);                                                     \
    template rich_status launch_st_post<TB, T>(const Phys &, const T *, const T *, const TB *, const double *,   \
                                               const T *, const int32_t *, T *, T *, hipStream_t);              \
    template rich_status launch_st_post_from<TB, T>(const Phys &, const T *, const T *, const TB *,              \
                                                    const double *, const T *, T *, hipStream_t);               \
    template rich_status launch_st_sweeps<TB, T>(const Phys &, const T *, const T *, const TB *, T *, T *, int, \
                                                 hipStream_t);                                                  \
    template rich_status launch_st_pre_batch<TB, T>(const std::vector<FineItem<TB, T>> &, hipStream_t,          \
                                                    WorkQueue *);                                               \
    template rich_status launch_gs_pre<TB, T>(const Phys &, const T *, const TB *, const double *, T *, T *,      \
                                              hipStream_t);                                                    \
    template rich_status launch_gs_post<TB, T>(const Phys &, const T *, const TB *, const double *, const T *,   \
                                               const T *, const int32_t *, T *, T *, hipStream_t);             \
    template rich_status launch_st_post_batch<TB, T>(const std::vector<FineItem<TB, T>> &, hipStream_t, WorkQueue *);
INST_ST(double, double)
INST_ST(double, float)
INST_ST(float, float)

rich_status launch_stencil_rowcounts(const Phys &P, int64_t *cnt, hipStream_t s) {
    uint32_t n = ncells(P);
    k_stencil_rowcounts<<<nblocks(n), TPB, 0, s>>>(P, n, cnt);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status launch_stencil_to_csr(const Phys &P, const double *M4, const int64_t *rowptr, int32_t *col,
                                  double *val, hipStream_t s) {
    uint32_t n = ncells(P);
    k_M_to_csr<<<nblocks(n), TPB, 0, s>>>(P, n, M4, rowptr, col, val);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status launch_J_to_csr(const Phys &P, const double *J7, const int64_t *rowptr, int32_t *col,
                            double *val, hipStream_t s) {
    uint32_t n = ncells(P);
    k_J_to_csr<<<nblocks(n), TPB, 0, s>>>(P, n, J7, rowptr, col, val);
    LAUNCH_CHECK();
    return RICH_OK;
}

}  // namespace rich
