// Internal declarations shared by the HIP translation units of librichards.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/richards.h"

struct rich_batcher;

namespace rich {

void set_error(const char *what, const char *file, int line, hipError_t e);
const char *last_error();

#define HIP_TRY(...)                                                    \
    do {                                                                \
        hipError_t e_ = (__VA_ARGS__);                                  \
        if (e_ != hipSuccess) {                                         \
            ::rich::set_error(#__VA_ARGS__, __FILE__, __LINE__, e_);    \
            return RICH_EHIP;                                           \
        }                                                               \
    } while (0)

#define RICH_TRY(...)                   \
    do {                                \
        rich_status s_ = (__VA_ARGS__); \
        if (s_ != RICH_OK) return s_;   \
    } while (0)

#define LAUNCH_CHECK() HIP_TRY(hipGetLastError())

// FP64 -> FP32 for the single-precision copies of the preconditioner: values
// beyond FP32's range saturate at +-FLT_MAX instead of becoming infinite (a
// Newton iterate far outside the physical range makes the auxiliary matrix's
// entries tiny and its inverse diagonal huge); NaN stays NaN.
__device__ inline float f32_sat(double x) {
    constexpr double m = 3.4028234663852886e38;
    return (float)(x > m ? m : (x < -m ? -m : x));
}
template <class TB, class TA>
__device__ inline TB convert(TA x) { return (TB)x; }
template <>
__device__ inline float convert<float, double>(double x) { return f32_sat(x); }

// XCD-aware block order.  Workgroups are dealt round-robin over the 8 XCDs
// (each with its own L2); this maps them so that XCD x processes one
// contiguous range of logical blocks, keeping the +-nx and +-nx*ny stencil
// neighbours of a row in the same L2.  The grid must be a multiple of 8.
constexpr unsigned NXCD = 8;
__device__ inline unsigned xcd_block() {
    unsigned q = gridDim.x / NXCD;
    return (blockIdx.x % NXCD) * q + blockIdx.x / NXCD;
}
inline unsigned xcd_grid(int64_t n, int tpb) {
    int64_t b = (n + tpb - 1) / tpb;
    return (unsigned)((b + NXCD - 1) / NXCD * NXCD);
}

// ------------------------------------------------------- batched launches
// One launch covers the same kernel for several resident simulations: entry
// e owns the virtual blocks [begin[e], begin[e+1]) (in XCD-aware order) and
// has its own arguments; each block runs exactly the code of the lone
// launch on its entry's data, so results do not depend on the batch.
constexpr int RICH_BATCH_MAX = 8;
struct Grid3 {
    int nx, ny, nz;
};
template <class A>
struct Batch {
    int n = 0;
    unsigned begin[RICH_BATCH_MAX + 1] = {};
    A a[RICH_BATCH_MAX];
    // persistent launches: a fixed grid whose blocks take virtual blocks from
    // the device counter *ctr (values from `base` on belong to this launch)
    unsigned long long *ctr = nullptr;
    unsigned long long base = 0;
};
template <class A>
__device__ inline int batch_entry(const Batch<A> &B, unsigned L) {
    int e = 0;
    for (int t = 1; t < B.n; t++) e += L >= B.begin[t] ? 1 : 0;
    return e;
}
// The virtual blocks a thread block of a batched launch runs: its own one
// (XCD-aware order), or, in a persistent launch, one after another from the
// launch's work counter until the counter passes the batch's total.  Every
// block's last fetch finds the total passed and leaves, so each block of the
// grid fetches exactly once more than the virtual blocks it ran: the counter
// advances by total + grid per launch, which the host adds to the next
// launch's base.  f must be block-uniform in its barriers (it is the body of
// the lone launch, whose early returns depend on the virtual block only).
template <class A, class F>
__device__ __forceinline__ void for_each_block(const Batch<A> &B, unsigned first, F &&f) {
    const unsigned total = B.begin[B.n];
    if (!B.ctr) {
        if (first < total) f(first);
        return;
    }
    __shared__ unsigned s_next;
    const bool lead = threadIdx.x == 0 && threadIdx.y == 0;
    for (;;) {
        __syncthreads();  // the previous virtual block is done with LDS and s_next
        if (lead) s_next = (unsigned)(atomicAdd(B.ctr, 1ull) - B.base);
        __syncthreads();
        const unsigned L = s_next;
        if (L >= total) return;
        f(L);
    }
}
// A work counter of persistent batched launches on one stream, with the
// host's account of the values already consumed.
struct WorkQueue {
    unsigned long long *ctr = nullptr;  // device, zero at creation
    unsigned long long next = 0;        // first value of the next launch
    unsigned grid = 1024;               // thread blocks of a persistent launch
};
// Host side: group items into batches of at most RICH_BATCH_MAX and call
// launch(batch, grid) for each (grid = total blocks rounded up to the XCDs,
// or, with a work queue, a persistent grid of at most q->grid blocks).
template <class A, class F>
rich_status launch_batches(const std::vector<A> &items, const std::vector<unsigned> &blocks, F launch,
                           WorkQueue *q = nullptr) {
    for (size_t i0 = 0; i0 < items.size(); i0 += RICH_BATCH_MAX) {
        Batch<A> B;
        size_t i1 = items.size() < i0 + RICH_BATCH_MAX ? items.size() : i0 + RICH_BATCH_MAX;
        B.n = (int)(i1 - i0);
        unsigned tot = 0;
        for (size_t i = i0; i < i1; i++) {
            B.begin[i - i0] = tot;
            B.a[i - i0] = items[i];
            tot += blocks[i];
        }
        B.begin[B.n] = tot;
        if (tot == 0) continue;
        unsigned grid = (tot + NXCD - 1) / NXCD * NXCD;
        if (q) {
            grid = tot < q->grid ? tot : q->grid;
            B.ctr = q->ctr;
            B.base = q->next;
            q->next += (unsigned long long)tot + grid;
        }
        launch(B, grid);
        LAUNCH_CHECK();
    }
    return RICH_OK;
}

// Problem parameters passed by value to the stencil kernels.
constexpr int RICH_GL = 16;
struct Phys {
    int nx, ny, nz;
    double hx, hy, hz;
    double alpha, beta, theta_s, theta_r, A, gamma;
    int mean, mean_vertical;  // mean_vertical: mean of the z faces (-1: mean)
    int bc_type[6];
    double bc_value[6];
    double dt;
    int patch_face;  // Dirichlet patch on one face (-1: none)
    double patch_lo[2], patch_hi[2], patch_value;
    int tile_kz;  // planes per block of the tiled fine-level smoother (0: automatic)
    double gl_t[RICH_GL], gl_w[RICH_GL];  // Gauss-Legendre rule on [0, 1] of the integral mean
};

// Device buffer owned by a context (raw hipMalloc, freed in the context's destructor).
struct DevAlloc {
    std::vector<void *> ptrs;
    size_t bytes = 0;
    template <class T>
    rich_status get(T **out, size_t count) {
        void *p = nullptr;
        size_t b = count * sizeof(T);
        if (b == 0) b = 16;
        if (hipMalloc(&p, b) != hipSuccess) {
            (void)hipGetLastError();
            return RICH_ENOMEM;
        }
        ptrs.push_back(p);
        bytes += b;
        *out = static_cast<T *>(p);
        return RICH_OK;
    }
    void release(void *p) {
        for (auto &q : ptrs)
            if (q == p) {
                (void)hipFree(q);
                q = nullptr;
            }
    }
    ~DevAlloc() {
        for (void *p : ptrs)
            if (p) (void)hipFree(p);
    }
};

// ---------------------------------------------------------------- fine level
// Jacobian: 7 FP64 coefficient arrays of N, slot t*N + c, t = diag,-x,+x,-y,+y,-z,+z.
// Auxiliary M: 4 arrays, t = diag, +x, +y, +z (symmetric; the -d coupling of
// cell c is the +d coupling stored at its lower neighbour).
enum { J_D = 0, J_XM, J_XP, J_YM, J_YP, J_ZM, J_ZP };
enum { M_D = 0, M_XP, M_YP, M_ZP };

rich_status launch_theta(const Phys &P, const double *p, double *theta, hipStream_t s);
rich_status launch_residual(const Phys &P, const double *Ks, const double *p, const double *theta_old,
                            double *F, hipStream_t s);
// Assemble J (7N) and M (4N, FP64) plus M's FP32 copy (may be null) and the
// l1 inverse diagonal of M in FP64 and FP32 (either may be null).
rich_status launch_assemble(const Phys &P, const double *Ks, const double *p, double *J7, double *M4,
                            float *M4f, double *invd, float *invdf, int dflux, hipStream_t s);
template <class TX>
rich_status launch_spmv_J(const Phys &P, const double *J7, const TX *x, double *y, hipStream_t s,
                          const double *sb = nullptr, const double *sbs = nullptr, double sig = 0.0);
rich_status launch_spmv_M(const Phys &P, const double *M4, const double *x, double *y, hipStream_t s);
rich_status launch_stencil_to_csr(const Phys &P, const double *M4, const int64_t *rowptr,
                                  int32_t *col, double *val, hipStream_t s);
rich_status launch_J_to_csr(const Phys &P, const double *J7, const int64_t *rowptr, int32_t *col,
                            double *val, hipStream_t s);
rich_status launch_stencil_rowcounts(const Phys &P, int64_t *rowptr_plus1, hipStream_t s);

// fine-level V-cycle pieces (TB: type of the right-hand side, T: arithmetic)
// the right-hand side is bs[0] * b (bs: a device scalar)
template <class TB, class T>
rich_status launch_st_pre(const Phys &P, const T *M4, const T *invd, const TB *b, const double *bs, T *r,
                          hipStream_t s);
// xt (scratch, N) receives the prolongated iterate before post-smoothing
template <class TB, class T>
rich_status launch_st_post(const Phys &P, const T *M4, const T *invd, const TB *b, const double *bs, const T *xc,
                           const int32_t *agg, T *x, T *xt, hipStream_t s);
// Multicolour Gauss-Seidel fine level: x0 = one backward sweep from zero on
// M x = bs b, r = bs b - M x0; post: xt = x0 + P xc (when agg is set; else xt
// already holds the prolongated iterate), one forward sweep from xt into x
// (xt is overwritten).
template <class TB, class T>
rich_status launch_gs_pre(const Phys &P, const T *M4, const TB *b, const double *bs, T *x0, T *r, hipStream_t s);
template <class TB, class T>
rich_status launch_gs_post(const Phys &P, const T *M4, const TB *b, const double *bs, const T *x0, const T *xc,
                           const int32_t *agg, T *xt, T *x, hipStream_t s);

// One simulation's part of a batched fine-level V-cycle step (same meaning as
// the arguments of launch_st_pre / launch_st_post; xt: N scratch).
template <class TB, class T>
struct FineItem {
    const Phys *P;
    const T *M4, *invd;
    const TB *b;
    const double *bs;
    const T *xc;
    const int32_t *agg;
    T *xt;
    T *out;
};
template <class TB, class T>
rich_status launch_st_pre_batch(const std::vector<FineItem<TB, T>> &items, hipStream_t s, WorkQueue *q = nullptr);
template <class TB, class T>
rich_status launch_st_post_batch(const std::vector<FineItem<TB, T>> &items, hipStream_t s, WorkQueue *q = nullptr);
template <class TX>
struct SpmvItem {
    const Phys *P;
    const double *J7;
    const TX *x;
    double *y;
    const double *sb = nullptr, *sbs = nullptr;  // optional shift: y = J x - sig (sbs[0] sb)
    double sig = 0.0;
};
template <class TX>
rich_status launch_spmv_J_batch(const std::vector<SpmvItem<TX>> &items, hipStream_t s, WorkQueue *q = nullptr);
template <class TB, class T>
rich_status launch_st_sweeps(const Phys &P, const T *M4, const T *invd, const TB *b, T *x, T *tmp,
                             int sweeps, hipStream_t s);

// ------------------------------------------------------------ vector kernels
constexpr int RED_BLOCKS = 1024;   // fixed block count of every reduction (deterministic order)
constexpr int RED_THREADS = 256;
constexpr int GMRES_BLOCK_MAX = 10; // largest round of the s-step GMRES
constexpr int BLK_BUF = 1024;       // doubles per s-step result or coefficient buffer (>= 65 * 10 + 100)

// Basis vectors are stored unnormalised: the true V_i is vs[i] * stored V_i.
// out[i] = V_i . w (i < k), out[k] = w . w; reduced in fixed order.
rich_status launch_multidot(const double *V, int64_t ldv, int k, const double *vs, const double *w, int64_t n,
                            double *partial, double *out, hipStream_t s);
// w -= sum_i h_i V_i (i < k, h and vs on device); out[0] = ||w||^2 (after update)
rich_status launch_update_norm(const double *V, int64_t ldv, int k, const double *h, const double *vs, double *w,
                               int64_t n, double *partial, double *out, hipStream_t s);
// Block Gram-Schmidt of the s-step GMRES (S <= 6 raw block vectors Q_k at
// stride ldv, nv <= 66 basis vectors with device scales vs).
// launch_block_dot: out[i*S + k] = (vs_i V_i) . Q_k (i < nv, k < S), then the
// upper triangle of Q^T Q by rows (S(S+1)/2 values); partial needs
// RED_BLOCKS * block_partial_size(nv, S) doubles.  Deterministic.
rich_status launch_block_dot(const double *V, int64_t ldv, int nv, const double *vs, const double *Q, int S,
                             int64_t n, double *partial, double *out, hipStream_t s);
int block_partial_size(int nv, int S);
// Q_t <- sum_{k<=t} (Q_k - sum_i C_ik vs_i V_i) Rinv_kt in place; cf (device):
// C row-major (nv x S), then Rinv row-major (S x S, upper triangular).
rich_status launch_block_update(const double *V, int64_t ldv, int nv, const double *vs, const double *cf, double *Q,
                                int S, int64_t n, hipStream_t s);
// vs[0] = 1 / sqrt(ww[0]) on the device
rich_status launch_set_scale(double *vs, const double *ww, hipStream_t s);
// out[0] = x.y (deterministic)
rich_status launch_dot(const double *x, const double *y, int64_t n, double *partial, double *out,
                       hipStream_t s);
// out[0] = max |x_i| (NaN propagates), out[1] = sum x_i, out[2] = x.x
rich_status launch_norms(const double *x, int64_t n, double *partial, double *out, hipStream_t s);
// out[0] = max_i |a*d_i| / max(|u_i|, 1)
rich_status launch_rel_length(const double *d, const double *u, int64_t n, double *partial,
                              double *out, hipStream_t s);
rich_status launch_scale(double *x, double a, int64_t n, hipStream_t s);
rich_status launch_scale_dev(double *x, const double *inv_of, int64_t n, hipStream_t s);
// y = a*x + b*y
rich_status launch_axpby(double a, const double *x, double b, double *y, int64_t n, hipStream_t s);
// z = x + a*y
rich_status launch_xpay_to(const double *x, double a, const double *y, double *z, int64_t n,
                           hipStream_t s);
template <class TX>
rich_status launch_add_to(double *y, const TX *x, int64_t n, hipStream_t s);
// y = sum_i c_i V_i, c and vs on device (k entries)
rich_status launch_lincomb(const double *V, int64_t ldv, int k, const double *c, const double *vs, double *y,
                           int64_t n, hipStream_t s);
// y = b - y
rich_status launch_b_minus(const double *b, double *y, int64_t n, hipStream_t s);
// y = sp[0] * x (sp a device scalar)
rich_status launch_scale_copy(const double *x, const double *sp, double *y, int64_t n, hipStream_t s);
rich_status launch_negate_to(const double *x, double *y, int64_t n, hipStream_t s);
template <class TA, class TB>
rich_status launch_cast(const TA *a, TB *b, int64_t n, hipStream_t s);
rich_status launch_fill_i32(int32_t *x, int32_t v, int64_t n, hipStream_t s);
rich_status launch_fill_u64(unsigned long long *x, unsigned long long v, int64_t n, hipStream_t s);
rich_status launch_fill_f64(double *x, double v, int64_t n, hipStream_t s);

// exclusive scan of int64 counts in place: out[0] = 0, out[i] = sum_{k<i} in[k];
// out has n+1 entries; tmp needs scan_tmp_size(n) int64 entries.
int64_t scan_tmp_size(int64_t n);
rich_status scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp,
                               hipStream_t s);

// ---------------------------------------------------------------------- AMG
struct Level {
    int64_t n = 0, nnz = 0;
    int64_t *rowptr = nullptr;  // CSR (levels >= 1 only)
    int32_t *col = nullptr;
    double *val = nullptr;
    float *valf = nullptr;
    double *invd = nullptr;     // 1 / sum_j |a_ij|
    float *invdf = nullptr;
    int32_t *agg = nullptr;     // to level+1 (n)
    int64_t *mptr = nullptr;    // members of each coarse row (n_{l+1} + 1)
    int32_t *mem = nullptr;     // (n)
    // V-cycle work vectors, in the cycle's precision
    void *b = nullptr, *x = nullptr, *r = nullptr;
    // smoothed aggregation (to level+1): prolongator P (n rows), its transpose
    // PT (n_{l+1} rows), Q = A P (kept for the numeric refreshes) and the bits
    // of rho = max_i sum_j |a_ij| / a_ii; prow == nullptr for piecewise-constant P
    int64_t pnnz = 0, qnnz = 0;
    int64_t *prow = nullptr, *trow = nullptr, *qrow = nullptr;
    int32_t *pcol = nullptr, *tcol = nullptr, *qcol = nullptr;
    double *pval = nullptr, *tval = nullptr, *qval = nullptr;
    float *pvalf = nullptr, *tvalf = nullptr;
    unsigned long long *rho = nullptr;
    // row blocks of the CSR-stream kernels (levels >= 1): block b holds the
    // rows whose first entry lies in [b STREAM_CHUNK, (b+1) STREAM_CHUNK)
    int64_t nrb = 0;
    int64_t *rb = nullptr;  // nrb + 1 (first row, its first entry) pairs; nullptr: rows too long, plain CSR kernels
    int sg = 1;             // lanes per row in the kernels' reduction phase
};
constexpr int STREAM_CHUNK = 1536, STREAM_MAXROW = 512;

struct Hierarchy {
    int nlev = 0;
    Level L[16];
    bool dense = false;          // coarsest solved by dense inverse
    double *cinv = nullptr;      // n_c x n_c inverse (row-major), FP64
    float *cinvf = nullptr;
    double *cws = nullptr;       // workspace of the inverse (kept: refreshes must not allocate)
    int64_t nnz_total = 0;
    DevAlloc mem;
};

// one matching sweep on a device CSR (setup-time); returns n_coarse
rich_status match_sweep(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                        int32_t *agg, int64_t *nc_out, hipStream_t s);
// The device work arrays of one matching sweep of n rows and nnz entries,
// carved in this order from one buffer of match_ws_bytes(n, nnz) bytes
// (each array 256-byte aligned).
struct MatchWs {
    double *diag = nullptr, *wts = nullptr;
    int32_t *mate = nullptr, *cand = nullptr;
    int64_t *flag = nullptr, *id = nullptr, *stmp = nullptr;
    int32_t *still = nullptr;
};
size_t match_ws_bytes(int64_t n, int64_t nnz);
MatchWs match_ws_carve(void *base, int64_t n, int64_t nnz);
// the sweep on given work arrays; h_still: host int the round loop reads
// the device's "still free" flag into (pinned or pageable)
rich_status match_sweep_ws(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                           int32_t *agg, int64_t *nc_out, const MatchWs &w, int *h_still, hipStream_t s);
// C = P^T A P for piecewise-constant P given by agg (canonical summation order)
struct CsrDev {
    int64_t n = 0, nnz = 0;
    int64_t *rowptr = nullptr;
    int32_t *col = nullptr;
    double *val = nullptr;
};
rich_status galerkin(const CsrDev &A, const int32_t *agg, int64_t nc, CsrDev *C, DevAlloc &mem,
                     hipStream_t s);
// pattern of P^T A P given the members of every coarse row; values by galerkin_numeric
rich_status galerkin_symbolic(const CsrDev &A, const int32_t *agg, int64_t nc, const int64_t *mptr,
                              const int32_t *mem, CsrDev *C, DevAlloc &mem_out, hipStream_t s);
rich_status galerkin_numeric(const CsrDev &A, const int32_t *agg, const int64_t *mptr, const int32_t *mem,
                             const CsrDev &C, hipStream_t s);
// Fused serving launches (solver.hip): a batcher gathers the preconditioned
// products of the GMRES solves of the simulations attached to it and its
// thread issues them as batched launches on its own stream (on the device
// current at creation).
// persistent: its batched launches run as persistent grids on a work queue
rich_batcher *batcher_create(bool persistent);
void batcher_destroy(rich_batcher *B);
rich_status batcher_attach(rich_handle_t h, rich_batcher *B);
void batcher_stats(rich_batcher *B, int64_t *flushes, int64_t *items);

rich_status members(const int32_t *agg, int64_t n, int64_t nc, int64_t *mptr, int32_t *mem,
                    hipStream_t s);
rich_status csr_invd(const CsrDev &A, double *invd, float *invdf, hipStream_t s);
// dense row-major inverse of an SPD CSR matrix (blocked Gauss-Jordan; RICH_NOT_SPD on a
// non-positive pivot); ws holds dense_inverse_ws(n) doubles
int64_t dense_inverse_ws(int64_t n);
rich_status dense_inverse(const CsrDev &A, double *D, double *ws, hipStream_t s);
rich_status compose_agg(int32_t *comp, const int32_t *a, int64_t n, hipStream_t s);
// Decoupled greedy aggregation of A over blocks of `block` rows (strength
// threshold theta); agg (n) receives aggregate ids, *nc their number.
rich_status vmb_aggregate(const CsrDev &A, double theta, int64_t block, int32_t *agg, int64_t *nc, hipStream_t s);

// r = b - A x0 (x0 = D^{-1} b, the pre-smoothed iterate from zero, stored by the restriction)
template <class TB, class T>
rich_status launch_csr_pre(const Level &Lv, const T *val, const T *x0, const TB *b, T *r, hipStream_t s);
// Batched coarse-level V-cycle steps over several simulations (levels with
// CSR-stream row blocks and a piecewise-constant prolongator only).
// CsrItem: pre: out = r = b - A x0;  post: out = x = post-smooth(x0 + P xc)
// (the level's r buffer holds x0 + P xc).
template <class T>
struct CsrItem {
    const Level *Lv;
    const T *val, *invd, *b, *x0, *xc;
    T *out;
};
template <class T>
struct RestrictItem {
    const Level *Lv;  // the finer level (its members lists)
    const T *r;
    T *bc;
    int64_t nc;
    const T *invdc;
    T *x0c;
};
template <class T>
struct GemvItem {
    const T *Ainv, *b;
    T *x;
    int64_t n;
};
template <class T>
rich_status launch_csr_pre_batch(const std::vector<CsrItem<T>> &items, hipStream_t s, WorkQueue *q = nullptr);
template <class T>
rich_status launch_csr_post_batch(const std::vector<CsrItem<T>> &items, hipStream_t s, WorkQueue *q = nullptr);
template <class T>
rich_status launch_restrict_batch(const std::vector<RestrictItem<T>> &items, hipStream_t s, WorkQueue *q = nullptr);
template <class T>
rich_status launch_dense_gemv_batch(const std::vector<GemvItem<T>> &items, hipStream_t s, WorkQueue *q = nullptr);
// x = post-smooth(x0 + P xc); the level's r buffer holds the prolongated iterate
template <class TB, class T>
rich_status launch_csr_post(const Level &Lv, const T *val, const T *invd, const TB *b, const T *x0,
                            const T *xc, T *x, hipStream_t s);
// bc = P^T r, and x0c = invdc * bc when x0c is set
template <class T>
rich_status launch_restrict(const Level &Lv, const T *r, T *bc, int64_t nc, const T *invdc, T *x0c,
                            hipStream_t s);
template <class TB, class T>
rich_status launch_dense_gemv(const T *Ainv, const TB *b, T *x, int64_t n, hipStream_t s);
template <class TB, class T>
rich_status launch_csr_sweeps(const Level &Lv, const T *val, const T *invd, const TB *b, T *x, T *tmp,
                              int sweeps, hipStream_t s);
rich_status launch_csr_spmv(const CsrDev &A, const double *x, double *y, hipStream_t s);

// Row blocks of a CSR level for the CSR-stream V-cycle kernels (left unset
// when a row is longer than STREAM_MAXROW).
rich_status stream_blocks(Level &Lv, DevAlloc &mem, hipStream_t s);

// Smoothed aggregation.  Patterns of P, PT, Q = A P and C = P^T Q for the
// aggregates agg (members mptr/mem) of the fine level A; the arrays go to mem_out.
rich_status sa_symbolic(const CsrDev &A, const int32_t *agg, int64_t nc, const int64_t *mptr,
                        const int32_t *mem, Level &Lf, CsrDev *C, bool mixed, DevAlloc &mem_out,
                        hipStream_t s);
// Values of P, PT, Q and C (and the FP32 copies of P and PT when mixed), in
// the oracle's summation order.
rich_status sa_numeric(const CsrDev &A, const int32_t *agg, Level &Lf, const CsrDev &C, bool mixed,
                       hipStream_t s);
// bc = P^T r (and x0c = invdc * bc when x0c is set)
template <class T>
rich_status launch_sa_restrict(const Level &Lv, const T *r, T *bc, int64_t nc, const T *invdc, T *x0c,
                               hipStream_t s);
// xt = x0 + P xc, x0 given or D^{-1} (bs b) (bs: device scalar, or nullptr for 1)
template <class TB, class T>
rich_status launch_sa_prolong(const Level &Lv, const T *invd, const TB *b, const double *bs, const T *x0,
                              const T *xc, T *xt, hipStream_t s);
// fine level, post-smoothing from a stored prolongated iterate xt
template <class TB, class T>
rich_status launch_st_post_from(const Phys &P, const T *M4, const T *invd, const TB *b, const double *bs,
                                const T *xt, T *x, hipStream_t s);

template <int G, class T>
__device__ inline T group_sum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_down(v, o, G);
    return v;
}

}  // namespace rich
