// Host control of the solver and the C-ABI entry points: the backward-Euler
// time loop, the modified inexact Newton method with line search (Section
// 3), restarted right-preconditioned GMRES (eq. (precsystem)), the AMG
// V-cycle driver and hierarchy set-up (Section 5.2).  Every vector operation
// runs on the GPU; the host only reads back the few scalars each decision
// needs.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>

#include "common.hpp"
#include "krylov_host.hpp"

namespace rich {

static thread_local char g_err[512] = "";

void set_error(const char *what, const char *file, int line, hipError_t e) {
    snprintf(g_err, sizeof(g_err), "%s failed at %s:%d: %s", what, file, line, hipGetErrorString(e));
}
const char *last_error() { return g_err; }

static double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace rich

using namespace rich;

struct rich_ctx {
    Phys P;
    rich_solver_opts_t O;
    int64_t N = 0;
    hipStream_t s = nullptr;
    bool mixed = false;
    DevAlloc mem;
    // fields
    double *Ks = nullptr, *p = nullptr, *theta_old = nullptr;
    double *u = nullptr, *F = nullptr, *ut = nullptr, *Ft = nullptr, *d = nullptr, *Jd = nullptr;
    double *ub = nullptr, *Fb = nullptr, *rhs = nullptr, *work = nullptr;
    // fine matrices
    double *J7 = nullptr, *M4 = nullptr, *invd0 = nullptr;
    float *M4f = nullptr, *invd0f = nullptr;
    // GMRES
    int m = 0;
    int64_t ldv = 0;           // basis stride: N rounded up to 64 (aligned vectors)
    double *V = nullptr;       // (m+1) x ldv
    void *z = nullptr;         // N, V-cycle output (FP32 or FP64)
    void *ztmp = nullptr;      // N, sweep scratch for a one-level hierarchy
    double *partial = nullptr; // RED_BLOCKS * (m + 2)
    double *dres = nullptr;    // device scalars (m + 8)
    double *dres2 = nullptr;
    double *hres = nullptr;    // pinned host mirror (2 * (m + 8))
    double *vs = nullptr;      // device scale of every stored basis vector (m + 1)
    double *one = nullptr;     // device constant 1.0
    double *hbuf = nullptr;    // device Arnoldi results, one row of (m + 4) per iteration
    double *hall = nullptr;    // pinned host mirror of hbuf
    double *dblk = nullptr;    // s-step rounds: block dots [0, BLK_BUF), coefficients [BLK_BUF, 2 BLK_BUF)
    double shifts[GMRES_BLOCK_MAX] = {};  // s-step basis shifts sigma_t, in the order they are used
    int scap = 1;                          // s-step round size cap (gmres_block at first)
    int sgood = 0;                         // rounds taken whole since the cap last changed
    double *hblk = nullptr;    // pinned host mirror of dblk
    double *bsc = nullptr;     // N: scaled right-hand side for a one-level hierarchy
    std::vector<hipEvent_t> iter_ev;  // one per Arnoldi iteration
    // fused serving launches: the batcher this simulation posts its
    // preconditioned products to (null: launched on its own stream)
    rich_batcher *batcher = nullptr;
    hipEvent_t bev = nullptr;          // inputs of the posted product are ready
    bool in_batch = false;             // inside a GMRES solve that posts to the batcher
    // AMG
    Hierarchy *H = nullptr;
    bool have_J = false;
    int since_build = 0;
    // stats of the step in progress, and the phase whose bytes kernels add to
    rich_step_stats_t *cur = nullptr;
    double *phase_bytes = nullptr;
    // record of the Newton controller (rich_trace_newton)
    int nstep = 0;
    rich_newton_event_t *trace = nullptr;
    int trace_cap = 0;
    int64_t trace_len = 0;
    // optional per-kernel event timing
    struct KProf {
        int64_t launches = 0;
        double bytes = 0.0, ms = 0.0;
        std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    };
    bool profiling = false;
    KProf prof[RICH_K_COUNT];
    std::vector<hipEvent_t> event_pool;
    ~rich_ctx() {
        delete H;
        if (hres) (void)hipHostFree(hres);
        if (hall) (void)hipHostFree(hall);
        if (hblk) (void)hipHostFree(hblk);
        for (auto e : iter_ev) (void)hipEventDestroy(e);
        if (bev) (void)hipEventDestroy(bev);
        for (auto &k : prof)
            for (auto &e : k.pending) {
                (void)hipEventDestroy(e.first);
                (void)hipEventDestroy(e.second);
            }
        for (auto e : event_pool) (void)hipEventDestroy(e);
    }
};

namespace {

rich_status sync(rich_ctx *h) {
    HIP_TRY(hipStreamSynchronize(h->s));
    return RICH_OK;
}

// read n device doubles into the pinned mirror
rich_status readback(rich_ctx *h, const double *dev, int n, double *out) {
    HIP_TRY(hipMemcpyAsync(h->hres, dev, n * sizeof(double), hipMemcpyDeviceToHost, h->s));
    HIP_TRY(hipStreamSynchronize(h->s));
    memcpy(out, h->hres, n * sizeof(double));
    return RICH_OK;
}

// ||x||_inf, sum x, ||x||_2^2
rich_status norms(rich_ctx *h, const double *x, double out[3]) {
    RICH_TRY(launch_norms(x, h->N, h->partial, h->dres, h->s));
    return readback(h, h->dres, 3, out);
}

rich_status dotp(rich_ctx *h, const double *x, const double *y, double *out) {
    RICH_TRY(launch_dot(x, y, h->N, h->partial, h->dres, h->s));
    return readback(h, h->dres, 1, out);
}

// ---------------------------------------------------------- profiling
// Collect the elapsed time of every pending (start, stop) event pair.
rich_status prof_harvest(rich_ctx *h) {
    HIP_TRY(hipStreamSynchronize(h->s));
    for (auto &k : h->prof) {
        for (auto &e : k.pending) {
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, e.first, e.second));
            k.ms += ms;
            h->event_pool.push_back(e.first);
            h->event_pool.push_back(e.second);
        }
        k.pending.clear();
    }
    return RICH_OK;
}

rich_status prof_event(rich_ctx *h, hipEvent_t *e) {
    if (!h->event_pool.empty()) {
        *e = h->event_pool.back();
        h->event_pool.pop_back();
        return RICH_OK;
    }
    HIP_TRY(hipEventCreate(e));
    return RICH_OK;
}

// Add a launch's algorithmic bytes to the phase in progress.
inline void charge(rich_ctx *h, double bytes) {
    if (h->phase_bytes) *h->phase_bytes += bytes;
}

// Launch through `f`, bracketed by events when profiling is on.
template <class F>
rich_status timed(rich_ctx *h, int id, double bytes, F &&f) {
    charge(h, bytes);
    if (!h->profiling || id >= RICH_K_COUNT) return f();
    hipEvent_t a, b;
    RICH_TRY(prof_event(h, &a));
    RICH_TRY(prof_event(h, &b));
    HIP_TRY(hipEventRecord(a, h->s));
    rich_status st = f();
    HIP_TRY(hipEventRecord(b, h->s));
    auto &k = h->prof[id];
    k.pending.push_back({a, b});
    k.launches++;
    k.bytes += bytes;
    if (k.pending.size() >= 2048) RICH_TRY(prof_harvest(h));
    return st;
}

// ------------------------------------------------------------- hierarchy
rich_status build_hierarchy(rich_ctx *h) {
    delete h->H;
    h->H = new Hierarchy();
    Hierarchy &H = *h->H;
    hipStream_t s = h->s;
    const Phys &P = h->P;
    int64_t N = h->N;
    DevAlloc tmp;
    // level-0 CSR of M, kept for the numeric refreshes of the coarse matrices
    CsrDev A0;
    A0.n = N;
    int64_t *cnt, *stmp;
    RICH_TRY(tmp.get(&cnt, N));
    RICH_TRY(tmp.get(&stmp, scan_tmp_size(N)));
    RICH_TRY(H.mem.get(&A0.rowptr, N + 1));
    RICH_TRY(launch_stencil_rowcounts(P, cnt, s));
    RICH_TRY(scan_exclusive_i64(cnt, A0.rowptr, N, stmp, s));
    HIP_TRY(hipMemcpyAsync(&A0.nnz, A0.rowptr + N, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RICH_TRY(sync(h));
    RICH_TRY(H.mem.get(&A0.col, A0.nnz));
    RICH_TRY(H.mem.get(&A0.val, A0.nnz));
    RICH_TRY(launch_stencil_to_csr(P, h->M4, A0.rowptr, A0.col, A0.val, s));
    H.L[0].rowptr = A0.rowptr;
    H.L[0].col = A0.col;
    H.L[0].val = A0.val;

    H.L[0].n = N;
    H.L[0].nnz = A0.nnz;
    H.nnz_total = A0.nnz;
    CsrDev levA = A0;
    int l = 0;
    int maxl = h->O.amg_max_levels < 16 ? h->O.amg_max_levels : 16;
    while (l + 1 < maxl && levA.n > h->O.amg_coarse_size) {
        CsrDev cur = levA;
        bool own = false;
        DevAlloc *cur_mem = nullptr;
        int32_t *comp;
        RICH_TRY(H.mem.get(&comp, levA.n));
        RICH_TRY(compose_agg(comp, nullptr, levA.n, s));
        int64_t nc_vmb = levA.n;
        if (h->O.amg_aggregation == RICH_AGG_VMB) {
            RICH_TRY(vmb_aggregate(levA, h->O.amg_theta, h->O.amg_block, comp, &nc_vmb, s));
            own = nc_vmb < levA.n;
        }
        for (int sw = 0; sw < h->O.amg_sweeps && h->O.amg_aggregation == RICH_AGG_MATCHING; sw++) {
            DevAlloc *am = new DevAlloc();
            int32_t *a;
            rich_status st = am->get(&a, cur.n);
            int64_t nc = 0;
            if (st == RICH_OK) st = match_sweep(cur.n, cur.rowptr, cur.col, cur.val, a, &nc, s);
            if (st != RICH_OK) {
                delete am;
                delete cur_mem;
                return st;
            }
            if (nc == cur.n) {
                delete am;
                break;
            }
            DevAlloc *nm = new DevAlloc();
            CsrDev nxt;
            st = galerkin(cur, a, nc, &nxt, *nm, s);
            if (st == RICH_OK) st = compose_agg(comp, a, levA.n, s);
            if (st == RICH_OK) st = sync(h);
            delete am;
            if (st != RICH_OK) {
                delete nm;
                delete cur_mem;
                return st;
            }
            delete cur_mem;  // previous intermediate
            cur_mem = nm;
            cur = nxt;
            own = true;
        }
        if (!own) {
            H.mem.release(comp);
            break;
        }
        int64_t nc = h->O.amg_aggregation == RICH_AGG_VMB ? nc_vmb : cur.n;
        delete cur_mem;  // the pairwise products served the matching only
        // a level that keeps more than half of the rows is not worth its cost
        // once the current level fits the dense coarsest solver: stop here
        if (2 * nc > levA.n && levA.n <= h->O.coarse_dense_max) {
            H.mem.release(comp);
            break;
        }
        Level &Lf = H.L[l];
        Lf.agg = comp;
        RICH_TRY(H.mem.get(&Lf.mptr, nc + 1));
        RICH_TRY(H.mem.get(&Lf.mem, levA.n));
        RICH_TRY(members(comp, levA.n, nc, Lf.mptr, Lf.mem, s));
        // the coarse matrix: Galerkin product with the composed aggregates,
        // through the piecewise-constant or the smoothed prolongator
        CsrDev C;
        if (l < h->O.amg_smoothed) {
            RICH_TRY(sa_symbolic(levA, comp, nc, Lf.mptr, Lf.mem, Lf, &C, h->mixed, H.mem, s));
            RICH_TRY(sa_numeric(levA, comp, Lf, C, h->mixed, s));
        } else {
            RICH_TRY(galerkin_symbolic(levA, comp, nc, Lf.mptr, Lf.mem, &C, H.mem, s));
            RICH_TRY(galerkin_numeric(levA, comp, Lf.mptr, Lf.mem, C, s));
        }
        RICH_TRY(sync(h));
        Level &Lc = H.L[l + 1];
        Lc.n = C.n;
        Lc.nnz = C.nnz;
        Lc.rowptr = C.rowptr;
        Lc.col = C.col;
        Lc.val = C.val;
        H.nnz_total += C.nnz;
        levA.n = Lc.n;
        levA.nnz = Lc.nnz;
        levA.rowptr = Lc.rowptr;
        levA.col = Lc.col;
        levA.val = Lc.val;
        l++;
    }
    H.nlev = l + 1;
    // smoother data, FP32 copies, work vectors
    size_t esz = h->mixed ? sizeof(float) : sizeof(double);
    for (int t = 0; t < H.nlev; t++) {
        Level &Lv = H.L[t];
        if (t > 0) {
            CsrDev A{Lv.n, Lv.nnz, Lv.rowptr, Lv.col, Lv.val};
            RICH_TRY(H.mem.get(&Lv.invd, Lv.n));
            if (h->mixed) {
                RICH_TRY(H.mem.get(&Lv.invdf, Lv.n));
                RICH_TRY(H.mem.get(&Lv.valf, Lv.nnz));
                RICH_TRY(launch_cast(Lv.val, Lv.valf, Lv.nnz, s));
            }
            RICH_TRY(csr_invd(A, Lv.invd, Lv.invdf, s));
            // levels smoothed inside the cycle get their CSR-stream row blocks
            if (t < H.nlev - 1) RICH_TRY(stream_blocks(Lv, H.mem, s));
        }
        char *b, *x, *r;
        RICH_TRY(H.mem.get(&b, Lv.n * esz));
        RICH_TRY(H.mem.get(&x, Lv.n * esz));
        RICH_TRY(H.mem.get(&r, Lv.n * esz));
        Lv.b = b;
        Lv.x = x;
        Lv.r = r;
    }
    // coarsest solver
    Level &Lc = H.L[H.nlev - 1];
    H.dense = Lc.n <= h->O.coarse_dense_max;
    if (H.dense) {
        RICH_TRY(H.mem.get(&H.cinv, Lc.n * Lc.n));
        RICH_TRY(H.mem.get(&H.cws, dense_inverse_ws(Lc.n)));
        CsrDev A{Lc.n, Lc.nnz, Lc.rowptr, Lc.col, Lc.val};
        RICH_TRY(dense_inverse(A, H.cinv, H.cws, s));
        if (h->mixed) {
            RICH_TRY(H.mem.get(&H.cinvf, Lc.n * Lc.n));
            RICH_TRY(launch_cast(H.cinv, H.cinvf, Lc.n * Lc.n, s));
        }
    }
    RICH_TRY(sync(h));
    return RICH_OK;
}

// After a rebuild of M: the fine level's smoother data come with the
// assembly; with amg_refresh every coarse matrix is recomputed from the new
// fine matrix through the fixed aggregates (values only; the patterns do not
// change), then its smoother data and the coarsest inverse.  Without it
// (the paper's re-use) only a one-level hierarchy needs its inverse redone.
rich_status refresh_hierarchy(rich_ctx *h) {
    Hierarchy &H = *h->H;
    hipStream_t s = h->s;
    bool all = h->O.amg_refresh != 0;
    if (!all && H.nlev > 1) return RICH_OK;
    RICH_TRY(launch_stencil_to_csr(h->P, h->M4, H.L[0].rowptr, H.L[0].col, H.L[0].val, s));
    if (all) {
        for (int l = 0; l + 1 < H.nlev; l++) {
            Level &Lf = H.L[l], &Lc = H.L[l + 1];
            CsrDev A{Lf.n, Lf.nnz, Lf.rowptr, Lf.col, Lf.val};
            CsrDev C{Lc.n, Lc.nnz, Lc.rowptr, Lc.col, Lc.val};
            if (Lf.prow) RICH_TRY(sa_numeric(A, Lf.agg, Lf, C, h->mixed, s));
            else RICH_TRY(galerkin_numeric(A, Lf.agg, Lf.mptr, Lf.mem, C, s));
            RICH_TRY(csr_invd(C, Lc.invd, Lc.invdf, s));
            if (h->mixed) RICH_TRY(launch_cast(Lc.val, Lc.valf, Lc.nnz, s));
        }
    }
    if (H.dense) {
        Level &Lc = H.L[H.nlev - 1];
        CsrDev A{Lc.n, Lc.nnz, Lc.rowptr, Lc.col, Lc.val};
        RICH_TRY(dense_inverse(A, H.cinv, H.cws, s));
        if (h->mixed) RICH_TRY(launch_cast(H.cinv, H.cinvf, Lc.n * Lc.n, s));
    }
    return sync(h);
}

// ---------------------------------------------------------------- V-cycle
template <class T>
const T *lvval(const Level &L);
template <>
const double *lvval<double>(const Level &L) { return L.val; }
template <>
const float *lvval<float>(const Level &L) { return L.valf; }
template <class T>
const T *lvinvd(const Level &L);
template <>
const double *lvinvd<double>(const Level &L) { return L.invd; }
template <>
const float *lvinvd<float>(const Level &L) { return L.invdf; }

// z = V-cycle(b): one l1-Jacobi sweep before and after each coarse
// correction, the pre-sweep from zero (Section 5.2, symmetric V-cycle).
// The right-hand side is bs[0] * b (bs a device scalar: the basis vectors are
// stored unnormalised).
template <class T>
rich_status vcycle(rich_ctx *h, const double *b, const double *bs, T *z) {
    Hierarchy &H = *h->H;
    hipStream_t s = h->s;
    const T *M4 = h->mixed ? (const T *)(const void *)h->M4f : (const T *)(const void *)h->M4;
    const T *invd0 = h->mixed ? (const T *)(const void *)h->invd0f : (const T *)(const void *)h->invd0;
    const T *cinv = h->mixed ? (const T *)(const void *)H.cinvf : (const T *)(const void *)H.cinv;
    if (H.nlev == 1) {
        const double n = (double)h->N, t = sizeof(T);
        RICH_TRY(launch_scale_copy(b, bs, h->bsc, h->N, s));
        charge(h, 16 * n);
        if (H.dense) {
            charge(h, n * n * t + 8 * n + t * n);
            return launch_dense_gemv<double, T>(cinv, h->bsc, z, h->N, s);
        }
        charge(h, h->O.coarse_l1_sweeps * n * (5 * t + 16));
        return launch_st_sweeps<double, T>(h->P, M4, invd0, h->bsc, z, (T *)h->ztmp, h->O.coarse_l1_sweeps, s);
    }
    const double t = sizeof(T), n0 = (double)h->N, n1 = (double)H.L[1].n;
    const bool gs = h->O.smoother == RICH_SMOOTH_MCGS;
    // down
    RICH_TRY(timed(h, RICH_K_VC0_PRE, gs ? n0 * (16 + 12 * t) : n0 * (8 + 6 * t), [&] {
        if (gs) return launch_gs_pre<double, T>(h->P, M4, b, bs, (T *)H.L[0].x, (T *)H.L[0].r, s);
        return launch_st_pre<double, T>(h->P, M4, invd0, b, bs, (T *)H.L[0].r, s);
    }));
    const Level &L0 = H.L[0];
    // (+ the coarse pre-smoothed iterate and the inverse diagonal it needs, below the coarsest level)
    double rbytes = (L0.prow ? (double)L0.pnnz * (4 + 2 * t) + n1 * (8 + t) : n0 * (t + 4) + n1 * (8 + t)) +
                    (H.nlev > 2 ? 2 * t * n1 : 0.0);
    // each restriction also stores the next level's pre-smoothed iterate
    // x0 = D^{-1} b in its x buffer, except for the coarsest level
    auto x0_of = [&](int l) { return l < H.nlev - 1 ? (T *)H.L[l].x : nullptr; };
    RICH_TRY(timed(h, RICH_K_VC0_RESTRICT, rbytes, [&] {
        return launch_restrict<T>(H.L[0], (const T *)H.L[0].r, (T *)H.L[1].b, H.L[1].n, lvinvd<T>(H.L[1]), x0_of(1),
                                  s);
    }));
    for (int l = 1; l < H.nlev - 1; l++) {
        Level &Lv = H.L[l];
        double bytes = (double)Lv.nnz * (4 + t) + (double)Lv.n * (8 + 3 * t);
        RICH_TRY(timed(h, l == 1 ? RICH_K_VC1_PRE : RICH_K_COUNT, bytes, [&] {
            return launch_csr_pre<T, T>(Lv, lvval<T>(Lv), (const T *)Lv.x, (const T *)Lv.b, (T *)Lv.r, s);
        }));
        charge(h, (double)Lv.n * (t + 4) + (double)H.L[l + 1].n * (8 + t + (l + 1 < H.nlev - 1 ? 2 * t : 0)));
        RICH_TRY(launch_restrict<T>(Lv, (const T *)Lv.r, (T *)H.L[l + 1].b, H.L[l + 1].n, lvinvd<T>(H.L[l + 1]),
                                    x0_of(l + 1), s));
    }
    // coarsest
    Level &Lc = H.L[H.nlev - 1];
    if (H.dense) {
        charge(h, (double)Lc.n * Lc.n * t + 2.0 * Lc.n * t);
        RICH_TRY(launch_dense_gemv<T, T>(cinv, (const T *)Lc.b, (T *)Lc.x, Lc.n, s));
    } else {
        charge(h, h->O.coarse_l1_sweeps * ((double)Lc.nnz * (4 + t) + (double)Lc.n * (8 + 4 * t)));
        RICH_TRY(launch_csr_sweeps<T, T>(Lc, lvval<T>(Lc), lvinvd<T>(Lc), (const T *)Lc.b, (T *)Lc.x, (T *)Lc.r,
                                         h->O.coarse_l1_sweeps, s));
    }
    // up
    for (int l = H.nlev - 2; l >= 1; l--) {
        Level &Lv = H.L[l];
        double bytes = (double)Lv.nnz * (4 + t) + (double)Lv.n * (12 + 7 * t) + (double)H.L[l + 1].n * t;
        RICH_TRY(timed(h, l == 1 ? RICH_K_VC1_POST : RICH_K_COUNT, bytes, [&] {
            return launch_csr_post<T, T>(Lv, lvval<T>(Lv), lvinvd<T>(Lv), (const T *)Lv.b, (const T *)Lv.x,
                                         (const T *)H.L[l + 1].x, (T *)Lv.x, s);
        }));
    }
    if (gs) {
        // x0 + P xc into the level's r buffer, then the forward Gauss-Seidel sweep
        return timed(h, RICH_K_VC0_POST, n0 * (20 + 12 * t) + n1 * t, [&] {
            T *xt = (T *)H.L[0].r;
            const T *x0 = (const T *)H.L[0].x, *xc = (const T *)H.L[1].x;
            if (L0.prow) RICH_TRY(launch_sa_prolong<double, T>(L0, invd0, b, bs, x0, xc, xt, s));
            return launch_gs_post<double, T>(h->P, M4, b, bs, x0, xc, L0.prow ? nullptr : L0.agg, xt, z, s);
        });
    }
    if (L0.prow) {
        // smoothed prolongation into the level's r buffer, then post-smoothing
        double pbytes = n0 * (12 + 6 * t) + n1 * t + (double)L0.pnnz * (4 + t) + n0 * (8 + 2 * t);
        return timed(h, RICH_K_VC0_POST, pbytes, [&] {
            T *xt = (T *)H.L[0].r;
            RICH_TRY(launch_sa_prolong<double, T>(L0, invd0, b, bs, nullptr, (const T *)H.L[1].x, xt, s));
            return launch_st_post_from<double, T>(h->P, M4, invd0, b, bs, xt, z, s);
        });
    }
    return timed(h, RICH_K_VC0_POST, n0 * (12 + 6 * t) + n1 * t, [&] {
        return launch_st_post<double, T>(h->P, M4, invd0, b, bs, (const T *)H.L[1].x, H.L[0].agg, z, (T *)H.L[0].r,
                                         s);
    });
}

rich_status apply_prec(rich_ctx *h, const double *b, const double *bs) {
    if (h->mixed) return vcycle<float>(h, b, bs, (float *)h->z);
    return vcycle<double>(h, b, bs, (double *)h->z);
}

// y = J z, or y = J z - sig (sbs[0] sb) with a shift vector
rich_status spmv_J_z(rich_ctx *h, double *y, const double *sb = nullptr, const double *sbs = nullptr,
                     double sig = 0.0) {
    if (sig == 0.0) sb = nullptr;
    double bytes = (double)h->N * (56 + 8 + (h->mixed ? 4 : 8) + (sb ? 8 : 0));
    return timed(h, RICH_K_SPMV_J, bytes, [&] {
        if (h->mixed) return launch_spmv_J<float>(h->P, h->J7, (const float *)h->z, y, h->s, sb, sbs, sig);
        return launch_spmv_J<double>(h->P, h->J7, (const double *)h->z, y, h->s, sb, sbs, sig);
    });
}

// ------------------------------------------------- fused serving launches
// Resident simulations of a server post each preconditioned product
// w = J M^{-1} (bs b) (or M^{-1} b alone, w null) of their GMRES solves to a
// shared batcher.  The batcher's own thread issues the posted products as one
// batch on the batcher's stream once every attached simulation that is inside
// a GMRES solve has posted, or once the oldest post has waited BATCH_WINDOW_S
// (a simulation busy elsewhere holds no one up for longer), then gathers the
// next batch.  A batch is one launch per kernel and V-cycle level: the fine
// smoother, restriction, coarse smoothers, coarsest product, prolongations and
// the J SpMV each cover every simulation in it.  Each simulation's stream
// waits for its inputs before and for the batch after.  Every block runs the
// code of the lone launch on its own simulation's data, so a simulation's
// results are the same alone and in a batch.  An error while issuing a batch
// is returned to every product posted from then on.
constexpr double BATCH_WINDOW_S = 100e-6;

struct BatchReq {
    rich_ctx *h;
    const double *b, *bs;
    double *w;
    double sig;  // w = J M^{-1} (bs b) - sig (bs b)
    uint64_t ticket;
};

}  // namespace

struct rich_batcher {
    std::mutex mu;
    std::condition_variable cv;     // posts, and finished issues
    hipStream_t s = nullptr;
    hipEvent_t done = nullptr;      // recorded after each batch
    std::thread thread;             // issues the batches
    bool stop = false;
    int in_solve = 0;               // attached simulations inside a GMRES solve
    std::chrono::steady_clock::time_point first;  // time of the oldest pending post
    std::vector<BatchReq> pend;     // posted products
    uint64_t posted = 0;            // tickets handed out
    uint64_t issued = 0;            // products with ticket < issued are issued
    rich_status last = RICH_OK;     // first error of an issue, sticky
    int64_t flushes = 0, items = 0;
    bool persistent = false;        // launches as persistent grids taking work from `queue`
    WorkQueue queue;                // device work counter of those launches (on stream s)
};

namespace {

template <class T>
const T *m4_of(const rich_ctx *h) {
    return h->mixed ? (const T *)(const void *)h->M4f : (const T *)(const void *)h->M4;
}
template <class T>
const T *invd0_of(const rich_ctx *h) {
    return h->mixed ? (const T *)(const void *)h->invd0f : (const T *)(const void *)h->invd0;
}

// A simulation can join a batch when its V-cycle has the shape the batched
// kernels cover: a piecewise-constant hierarchy of two or more levels with a
// dense coarsest solve and CSR-stream row blocks on every smoothed coarse level.
bool batchable(const rich_ctx *h) {
    const Hierarchy *H = h->H;
    if (!H || H->nlev < 2 || !H->dense || h->O.smoother != RICH_SMOOTH_L1) return false;
    for (int l = 0; l < H->nlev - 1; l++) {
        if (H->L[l].prow) return false;
        if (l >= 1 && !H->L[l].rb) return false;
    }
    return true;
}

template <class T>
rich_status apply_batch(const std::vector<BatchReq> &rq, hipStream_t s, WorkQueue *q) {
    if (rq.empty()) return RICH_OK;
    auto x0_of = [](const Hierarchy &H, int l) { return l < H.nlev - 1 ? (T *)H.L[l].x : nullptr; };
    int maxlev = 0;
    for (const auto &q : rq) maxlev = std::max(maxlev, q.h->H->nlev);
    std::vector<FineItem<double, T>> f;
    std::vector<RestrictItem<T>> ri;
    std::vector<CsrItem<T>> ci;
    std::vector<GemvItem<T>> gi;
    // down: fine pre-smoothing + residual, restriction
    for (const auto &q : rq) {
        Hierarchy &H = *q.h->H;
        f.push_back({&q.h->P, m4_of<T>(q.h), invd0_of<T>(q.h), q.b, q.bs, nullptr, nullptr, nullptr, (T *)H.L[0].r});
        ri.push_back({&H.L[0], (const T *)H.L[0].r, (T *)H.L[1].b, H.L[1].n, lvinvd<T>(H.L[1]), x0_of(H, 1)});
    }
    RICH_TRY(launch_st_pre_batch<double, T>(f, s, q));
    RICH_TRY(launch_restrict_batch<T>(ri, s, q));
    for (int l = 1; l < maxlev - 1; l++) {
        ci.clear();
        ri.clear();
        for (const auto &q : rq) {
            Hierarchy &H = *q.h->H;
            if (l >= H.nlev - 1) continue;
            Level &Lv = H.L[l];
            ci.push_back({&Lv, lvval<T>(Lv), nullptr, (const T *)Lv.b, (const T *)Lv.x, nullptr, (T *)Lv.r});
            ri.push_back({&Lv, (const T *)Lv.r, (T *)H.L[l + 1].b, H.L[l + 1].n, lvinvd<T>(H.L[l + 1]),
                          x0_of(H, l + 1)});
        }
        RICH_TRY(launch_csr_pre_batch<T>(ci, s, q));
        RICH_TRY(launch_restrict_batch<T>(ri, s, q));
    }
    // coarsest
    for (const auto &q : rq) {
        Hierarchy &H = *q.h->H;
        Level &Lc = H.L[H.nlev - 1];
        const T *cinv = q.h->mixed ? (const T *)(const void *)H.cinvf : (const T *)(const void *)H.cinv;
        gi.push_back({cinv, (const T *)Lc.b, (T *)Lc.x, Lc.n});
    }
    RICH_TRY(launch_dense_gemv_batch<T>(gi, s, q));
    // up: prolongation + post-smoothing
    for (int l = maxlev - 2; l >= 1; l--) {
        ci.clear();
        for (const auto &q : rq) {
            Hierarchy &H = *q.h->H;
            if (l >= H.nlev - 1) continue;
            Level &Lv = H.L[l];
            ci.push_back({&Lv, lvval<T>(Lv), lvinvd<T>(Lv), (const T *)Lv.b, (const T *)Lv.x,
                          (const T *)H.L[l + 1].x, (T *)Lv.x});
        }
        RICH_TRY(launch_csr_post_batch<T>(ci, s, q));
    }
    f.clear();
    std::vector<SpmvItem<T>> sp;
    for (const auto &q : rq) {
        Hierarchy &H = *q.h->H;
        f.push_back({&q.h->P, m4_of<T>(q.h), invd0_of<T>(q.h), q.b, q.bs, (const T *)H.L[1].x, H.L[0].agg,
                     (T *)H.L[0].r, (T *)q.h->z});
        if (q.w) {
            SpmvItem<T> it{&q.h->P, q.h->J7, (const T *)q.h->z, q.w};
            if (q.sig != 0.0) {
                it.sb = q.b;
                it.sbs = q.bs;
                it.sig = q.sig;
            }
            sp.push_back(it);
        }
    }
    RICH_TRY(launch_st_post_batch<double, T>(f, s, q));
    return launch_spmv_J_batch<T>(sp, s, q);
}

// Issue one batch on the batcher's stream (batcher thread, lock not held).
rich_status issue_batch(rich_batcher *B, const std::vector<BatchReq> &rq) {
    std::vector<BatchReq> mixed, fp64;
    for (const auto &q : rq) {
        HIP_TRY(hipStreamWaitEvent(B->s, q.h->bev, 0));
        (q.h->mixed ? mixed : fp64).push_back(q);
    }
    WorkQueue *q = B->persistent ? &B->queue : nullptr;
    RICH_TRY(apply_batch<float>(mixed, B->s, q));
    RICH_TRY(apply_batch<double>(fp64, B->s, q));
    HIP_TRY(hipEventRecord(B->done, B->s));
    for (const auto &q : rq) HIP_TRY(hipStreamWaitEvent(q.h->s, B->done, 0));
    return RICH_OK;
}

void batcher_main(rich_batcher *B, int device) {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(B->mu);
    for (;;) {
        B->cv.wait(lk, [&] { return B->stop || !B->pend.empty(); });
        if (B->pend.empty()) return;  // stopping, nothing left
        const auto deadline = B->first + std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                                              std::chrono::duration<double>(BATCH_WINDOW_S));
        B->cv.wait_until(lk, deadline, [&] { return B->stop || (int)B->pend.size() >= B->in_solve; });
        std::vector<BatchReq> rq;
        rq.swap(B->pend);
        lk.unlock();
        rich_status st = issue_batch(B, rq);
        lk.lock();
        if (st != RICH_OK && B->last == RICH_OK) B->last = st;
        B->issued = rq.back().ticket + 1;
        B->flushes++;
        B->items += (int64_t)rq.size();
        B->cv.notify_all();
    }
}

// w = J M^{-1} (bs b) - sig (bs b) (w null: z = M^{-1} (bs b) only), through
// the batcher when the simulation is in a batched solve, else on its own
// stream.
rich_status prec_product(rich_ctx *h, const double *b, const double *bs, double *w, double sig = 0.0) {
    if (!h->in_batch) {
        RICH_TRY(apply_prec(h, b, bs));
        return w ? spmv_J_z(h, w, b, bs, sig) : RICH_OK;
    }
    rich_batcher *B = h->batcher;
    HIP_TRY(hipEventRecord(h->bev, h->s));
    std::unique_lock<std::mutex> lk(B->mu);
    const uint64_t t = B->posted++;
    if (B->pend.empty()) B->first = std::chrono::steady_clock::now();
    B->pend.push_back({h, b, bs, w, sig, t});
    B->cv.notify_all();
    B->cv.wait(lk, [&] { return B->issued > t; });
    return B->last;
}

// Membership of a GMRES solve in the batch (RAII).
struct BatchScope {
    rich_ctx *h;
    explicit BatchScope(rich_ctx *hh) : h(hh) {
        if (!h->batcher || !batchable(h)) return;
        std::lock_guard<std::mutex> lk(h->batcher->mu);
        h->batcher->in_solve++;
        h->in_batch = true;
    }
    ~BatchScope() {
        if (!h->in_batch) return;
        rich_batcher *B = h->batcher;
        std::lock_guard<std::mutex> lk(B->mu);
        h->in_batch = false;
        B->in_solve--;
        B->cv.notify_all();  // the pending batch may be complete now
    }
};

rich_status add_z(rich_ctx *h, double *x) {
    if (h->mixed) return launch_add_to<float>(x, (const float *)h->z, h->N, h->s);
    return launch_add_to<double>(x, (const double *)h->z, h->N, h->s);
}

// ------------------------------------------------------------------ GMRES
// Right-preconditioned restarted GMRES(m) on J M^{-1}: classical Gram-Schmidt
// (one fused dot block and one fused update per iteration; a second pass
// when the norm drops below gmres_reorth of its value), Givens rotations on
// the host, x += M^{-1} V y at the end of each cycle, true residual at every
// restart.  Stops at ||b - J x||_2 <= eta ||b||_2 or after maxit Arnoldi steps.
// Basis vectors are stored unnormalised with their scale on the device, so an
// Arnoldi step needs no host value: the host enqueues iteration j+1 before it
// reads iteration j's Hessenberg column, and only a (rare) second
// Gram-Schmidt pass makes it wait and redo the speculative step.
constexpr double GMRES_SPEC_MARGIN = 4.0;
constexpr int64_t GMRES_SPEC_MIN_ROWS = (int64_t)1 << 21;

rich_status gmres_classic(rich_ctx *h, const double *b, double *x, int *its_out, double *relres_out,
                          bool *conv_out) {
    int64_t N = h->N, ld = h->ldv;
    int m = h->m;
    const int W = m + 4;
    hipStream_t s = h->s;
    double eta = h->O.eta;
    std::vector<double> Hm((m + 1) * m), cs(m), sn(m), g(m + 1), y(m), hv(m + 8);
    double nb[3];
    RICH_TRY(norms(h, b, nb));
    double bnorm = std::sqrt(nb[2]);
    RICH_TRY(launch_fill_f64(x, 0.0, N, s));
    charge(h, 16.0 * N);
    int total = 0;
    bool conv = false;
    double relres = 0.0;
    if (bnorm == 0.0) {
        *its_out = 0;
        *relres_out = 0.0;
        *conv_out = true;
        return RICH_OK;
    }
    if (!std::isfinite(bnorm)) return RICH_NONFINITE;
    BatchScope batch_scope(h);
    auto enqueue = [&](int j) -> rich_status {
        double *vj = h->V + (size_t)j * ld;
        double *w = h->V + (size_t)(j + 1) * ld;
        double *hb = h->hbuf + (size_t)j * W;
        RICH_TRY(prec_product(h, vj, h->vs + j, w));
        RICH_TRY(timed(h, RICH_K_MULTIDOT, (double)N * 8 * (j + 2),
                       [&] { return launch_multidot(h->V, ld, j + 1, h->vs, w, N, h->partial, hb, s); }));
        RICH_TRY(timed(h, RICH_K_UPDATE, (double)N * 8 * (j + 3), [&] {
            return launch_update_norm(h->V, ld, j + 1, hb, h->vs, w, N, h->partial, hb + j + 2, s);
        }));
        RICH_TRY(launch_set_scale(h->vs + j + 1, hb + j + 2, s));
        HIP_TRY(hipMemcpyAsync(h->hall + (size_t)j * W, hb, (j + 3) * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(h->iter_ev[j], s));
        return RICH_OK;
    };
    bool first = true;
    for (;;) {
        // true residual into V_0 (stored unnormalised, scale 1/beta on the device)
        if (first) {
            HIP_TRY(hipMemcpyAsync(h->V, b, N * sizeof(double), hipMemcpyDeviceToDevice, s));
            charge(h, 16.0 * N);
        } else {
            RICH_TRY(launch_spmv_J<double>(h->P, h->J7, x, h->V, s));
            RICH_TRY(launch_b_minus(b, h->V, N, s));
            charge(h, 72.0 * N + 24.0 * N);
        }
        charge(h, 8.0 * N);  // norms of V_0
        first = false;
        double rn[3];
        RICH_TRY(norms(h, h->V, rn));
        double beta = std::sqrt(rn[2]);
        if (!std::isfinite(beta)) return RICH_NONFINITE;
        relres = beta / bnorm;
        if (beta <= eta * bnorm) {
            conv = true;
            break;
        }
        if (total >= h->O.gmres_maxit) break;
        RICH_TRY(launch_set_scale(h->vs, h->dres + 2, s));  // dres[2] = ||V_0||^2 from norms()
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0, queued = -1;
        for (int j = 0; j < m && total < h->O.gmres_maxit; j++) {
            if (queued < j) {
                RICH_TRY(enqueue(j));
                queued = j;
            }
            // Step j + 1 is queued before step j is read back (it needs nothing
            // from the host), unless, on a grid large enough that an iteration
            // costs far more than a host round trip, the residual estimate
            // extrapolated with the last reduction factor says step j is about
            // to meet the tolerance: a speculative step past convergence is a
            // whole wasted iteration, a missed one only a round trip.
            bool speculate = true;
            if (N >= GMRES_SPEC_MIN_ROWS && j >= 1 && g[j - 1] != 0.0) {
                const double pred = std::fabs(g[j]) * (std::fabs(g[j]) / std::fabs(g[j - 1]));
                speculate = pred > GMRES_SPEC_MARGIN * eta * bnorm;
            }
            if (speculate && j + 1 < m && total + 1 < h->O.gmres_maxit && queued < j + 1) {
                RICH_TRY(enqueue(j + 1));
                queued = j + 1;
            }
            HIP_TRY(hipEventSynchronize(h->iter_ev[j]));
            const double *hr = h->hall + (size_t)j * W;
            for (int i = 0; i <= j; i++) hv[i] = hr[i];
            double ww0 = hr[j + 1], ww1 = hr[j + 2];
            if (std::sqrt(ww1) < h->O.gmres_reorth * std::sqrt(ww0)) {
                // second Gram-Schmidt pass on V_{j+1}; the speculative step j+1 used
                // the once-orthogonalised vector and is redone
                double *w = h->V + (size_t)(j + 1) * ld;
                RICH_TRY(sync(h));
                RICH_TRY(launch_multidot(h->V, ld, j + 1, h->vs, w, N, h->partial, h->dres, s));
                RICH_TRY(launch_update_norm(h->V, ld, j + 1, h->dres, h->vs, w, N, h->partial, h->dres2, s));
                RICH_TRY(launch_set_scale(h->vs + j + 1, h->dres2, s));
                HIP_TRY(hipMemcpyAsync(h->hres, h->dres, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
                HIP_TRY(hipMemcpyAsync(h->hres + (m + 8), h->dres2, sizeof(double), hipMemcpyDeviceToHost, s));
                RICH_TRY(sync(h));
                for (int i = 0; i <= j; i++) hv[i] += h->hres[i];
                ww1 = h->hres[m + 8];
                queued = j;
            }
            double hn = std::sqrt(ww1);
            if (!std::isfinite(hn)) return RICH_NONFINITE;
            for (int i = 0; i <= j; i++) Hm[i * m + j] = hv[i];
            Hm[(j + 1) * m + j] = hn;
            for (int i = 0; i < j; i++) {
                double a = Hm[i * m + j], c = Hm[(i + 1) * m + j];
                Hm[i * m + j] = cs[i] * a + sn[i] * c;
                Hm[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            double a = Hm[j * m + j], c = Hm[(j + 1) * m + j];
            double rho = std::sqrt(a * a + c * c);
            cs[j] = a / rho;
            sn[j] = c / rho;
            Hm[j * m + j] = rho;
            Hm[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            total++;
            k = j + 1;
            if (std::fabs(g[j + 1]) <= eta * bnorm || hn == 0.0) break;
        }
        for (int i = k - 1; i >= 0; i--) {
            double sum = g[i];
            for (int t = i + 1; t < k; t++) sum -= Hm[i * m + t] * y[t];
            y[i] = sum / Hm[i * m + i];
        }
        memcpy(h->hres, y.data(), k * sizeof(double));
        HIP_TRY(hipMemcpyAsync(h->dres, h->hres, k * sizeof(double), hipMemcpyHostToDevice, s));
        RICH_TRY(launch_lincomb(h->V, ld, k, h->dres, h->vs, h->work, N, s));
        RICH_TRY(prec_product(h, h->work, h->one, nullptr));
        RICH_TRY(add_z(h, x));
        charge(h, 8.0 * (k + 1) * N + (16.0 + (h->mixed ? 4 : 8)) * N);
        RICH_TRY(sync(h));  // hres is reused before the next read
    }
    *its_out = total;
    *relres_out = relres;
    *conv_out = conv;
    return RICH_OK;
}

// ------------------------------------------------------------ s-step GMRES
// The same restarted right-preconditioned GMRES(m) with the Arnoldi vectors
// generated s at a time (gmres_block = s >= 2).  A round starting at basis
// vector v_j0 applies the preconditioned operator s times to the shifted
// (Newton) power basis q_0 = v_j0, q_{t+1} = (J M^{-1} - sigma_t I) q_t (the
// shift term fused into the J product), then orthogonalises q_1..q_s against
// v_0..v_j0 and each other in one block round: one pass gives C = V^T Q and
// the Gram matrix G = Q^T Q, the host factors the Pythagorean complement
// G - C^T C = R^T R (Cholesky), and one pass writes (Q - V C) R^{-1}, the
// next s orthonormal basis vectors.  The vectors before the first whose
// pivot keeps less than gmres_reorth of its norm (or is not positive) are
// taken from the block round; that one and the rest are orthogonalised
// vector by vector with two classical passes.  The Hessenberg columns j0..j0+s-1 follow from the coordinates of
// the q_t in the new basis: with S the coordinates of q_0..q_s and H_prev
// the earlier columns, J M^{-1} [v_j0..v_{j0+s-1}] =
// (S_{:,1..s} + S_{:,0..s-1} diag(sigma) - H_prev S_{0..j0-1, 0..s-1}) Sb^{-1},
// Sb the (upper triangular) rows j0..j0+s-1 of S's first s columns.  The
// residual estimate is tested after every column, as one vector at a time
// would, and the next round is cut to the steps the estimate's decay over
// the last round predicts.  The shifts, Leja points of an interval over
// the spectrum of J M^{-1}, keep the basis of long rounds well conditioned.
// A round finished vector by vector from its (a+1)-th vector caps the next
// rounds at max(a, 1) vectors; every SCAP_GROW rounds in a row taken whole
// raise the cap by one, up to s (the cap is kept from call to call).
constexpr int SCAP_GROW = 8;
rich_status gmres_sstep(rich_ctx *h, const double *b, double *x, int *its_out, double *relres_out,
                        bool *conv_out) {
    const int64_t N = h->N, ld = h->ldv;
    const int m = h->m, S = h->O.gmres_block;
    const double *sig = h->shifts, eta = h->O.eta, reorth = h->O.gmres_reorth;
    hipStream_t s = h->s;
    // Hr: the cycle's Hessenberg matrix as computed; Hm: its rotated copy
    std::vector<double> Hr((size_t)(m + 1) * m), Hm((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    double nb[3];
    RICH_TRY(norms(h, b, nb));
    const double bnorm = std::sqrt(nb[2]);
    RICH_TRY(launch_fill_f64(x, 0.0, N, s));
    charge(h, 16.0 * N);
    int total = 0;
    bool conv = false;
    double relres = 0.0;
    if (bnorm == 0.0) {
        *its_out = 0;
        *relres_out = 0.0;
        *conv_out = true;
        return RICH_OK;
    }
    if (!std::isfinite(bnorm)) return RICH_NONFINITE;
    BatchScope batch_scope(h);
    double *dout = h->dblk, *dcf = h->dblk + BLK_BUF;
    double *hout = h->hblk, *hcf = h->hblk + BLK_BUF;
    bool first = true;
    for (;;) {
        // true residual into V_0 (stored unnormalised, scale 1/beta on the device)
        if (first) {
            HIP_TRY(hipMemcpyAsync(h->V, b, N * sizeof(double), hipMemcpyDeviceToDevice, s));
            charge(h, 16.0 * N);
        } else {
            RICH_TRY(launch_spmv_J<double>(h->P, h->J7, x, h->V, s));
            RICH_TRY(launch_b_minus(b, h->V, N, s));
            charge(h, 72.0 * N + 24.0 * N);
        }
        charge(h, 8.0 * N);  // norms of V_0
        first = false;
        double rn[3];
        RICH_TRY(norms(h, h->V, rn));
        const double beta = std::sqrt(rn[2]);
        if (!std::isfinite(beta)) return RICH_NONFINITE;
        relres = beta / bnorm;
        if (beta <= eta * bnorm) {
            conv = true;
            break;
        }
        if (total >= h->O.gmres_maxit) break;
        RICH_TRY(launch_set_scale(h->vs, h->dres + 2, s));  // dres[2] = ||V_0||^2 from norms()
        std::fill(g.begin(), g.end(), 0.0);
        std::fill(Hr.begin(), Hr.end(), 0.0);
        g[0] = beta;
        int j0 = 0, k = 0, ss_next = S;
        bool stop = false;
        // Hessenberg column j (in Hr) into the rotated factor and the residual estimate
        auto add_column = [&](int j) {
            const double hn = Hr[(size_t)(j + 1) * m + j];
            for (int i = 0; i <= j + 1; i++) Hm[(size_t)i * m + j] = Hr[(size_t)i * m + j];
            for (int i = 0; i < j; i++) {
                double a = Hm[(size_t)i * m + j], cc = Hm[(size_t)(i + 1) * m + j];
                Hm[(size_t)i * m + j] = cs[i] * a + sn[i] * cc;
                Hm[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * cc;
            }
            double a = Hm[(size_t)j * m + j], cc = Hm[(size_t)(j + 1) * m + j];
            double rho = std::sqrt(a * a + cc * cc);
            cs[j] = a / rho;
            sn[j] = cc / rho;
            Hm[(size_t)j * m + j] = rho;
            Hm[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            total++;
            k = j + 1;
            if (std::fabs(g[j + 1]) <= eta * bnorm || hn == 0.0 || total >= h->O.gmres_maxit) stop = true;
        };
        // one classical Arnoldi step per column (normalised inputs, second
        // pass on cancellation): the round's power basis overflowed
        auto classical_round = [&](int ss) -> rich_status {
            for (int c = 0; c < ss && !stop; c++) {
                const int j = j0 + c;
                double *w = h->V + (size_t)(j + 1) * ld;
                RICH_TRY(prec_product(h, h->V + (size_t)j * ld, h->vs + j, w));
                std::vector<double> hv(j + 1, 0.0);
                double ww0 = 0.0, ww = 0.0;
                for (int pass = 0; pass < 2; pass++) {
                    RICH_TRY(timed(h, pass ? RICH_K_COUNT : RICH_K_MULTIDOT, 8.0 * N * (j + 2), [&] {
                        return launch_multidot(h->V, ld, j + 1, h->vs, w, N, h->partial, h->dres, s);
                    }));
                    RICH_TRY(timed(h, pass ? RICH_K_COUNT : RICH_K_UPDATE, 8.0 * N * (j + 3), [&] {
                        return launch_update_norm(h->V, ld, j + 1, h->dres, h->vs, w, N, h->partial, h->dres2, s);
                    }));
                    HIP_TRY(hipMemcpyAsync(h->hres, h->dres, (j + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
                    HIP_TRY(hipMemcpyAsync(h->hres + (m + 8), h->dres2, sizeof(double), hipMemcpyDeviceToHost, s));
                    RICH_TRY(sync(h));
                    for (int i = 0; i <= j; i++) hv[i] += h->hres[i];
                    if (pass == 0) ww0 = h->hres[j + 1];
                    ww = h->hres[m + 8];
                    if (!(std::sqrt(ww) < h->O.gmres_reorth * std::sqrt(ww0))) break;
                }
                RICH_TRY(launch_set_scale(h->vs + j + 1, h->dres2, s));
                const double hn = std::sqrt(ww);
                if (!std::isfinite(hn)) return RICH_NONFINITE;
                for (int i = 0; i <= j; i++) Hr[(size_t)i * m + j] = hv[i];
                Hr[(size_t)(j + 1) * m + j] = hn;
                add_column(j);
            }
            return RICH_OK;
        };
        while (!stop && j0 < m && total < h->O.gmres_maxit) {
            int ss = std::min(std::min(std::min(ss_next, h->scap), m - j0), h->O.gmres_maxit - total);
            const int nv = j0 + 1;
            double *Q = h->V + (size_t)nv * ld;
            const double g_start = std::fabs(g[j0]);
            // the power basis: raw vectors (scale 1) in slots nv .. nv+ss-1
            RICH_TRY(launch_fill_f64(h->vs + nv, 1.0, ss, s));
            for (int t = 0; t < ss; t++)
                RICH_TRY(prec_product(h, h->V + (size_t)(j0 + t) * ld, h->vs + j0 + t,
                                      h->V + (size_t)(j0 + t + 1) * ld, sig[t]));
            const int nout = block_partial_size(nv, ss);
            RICH_TRY(timed(h, RICH_K_BLOCK_DOT, 8.0 * N * (nv + ss), [&] {
                return launch_block_dot(h->V, ld, nv, h->vs, Q, ss, N, h->partial, dout, s);
            }));
            HIP_TRY(hipMemcpyAsync(hout, dout, nout * sizeof(double), hipMemcpyDeviceToHost, s));
            RICH_TRY(sync(h));
            bool finite = true;
            for (int t = 0; t < nout; t++) finite = finite && std::isfinite(hout[t]);
            if (!finite) {
                RICH_TRY(classical_round(ss));
                j0 += ss;
                ss_next = S;
                continue;
            }
            // coordinates of q_1..q_ss in v_0..v_{j0+ss}: C (nv x ss), R (ss x ss, upper),
            // row stride sw (ss may shrink below)
            const int sw = ss;
            std::vector<double> C((size_t)nv * sw), R((size_t)sw * sw, 0.0), Gm((size_t)sw * sw);
            for (int t = 0; t < nv * ss; t++) C[t] = hout[t];
            for (int a = 0, t = nv * ss; a < ss; a++)
                for (int c = a; c < ss; c++, t++) Gm[a * ss + c] = Gm[c * ss + a] = hout[t];
            // Cholesky factor of the complement, pivot by pivot: vectors 0..nok-1
            // keep more than gmres_reorth of their norm
            int nok = ss;
            bool overflow = false;
            for (int a = 0; a < ss && nok == ss; a++) {
                for (int c = a; c < ss; c++) {
                    double pac = Gm[a * ss + c];
                    for (int i = 0; i < nv; i++) pac -= C[i * ss + a] * C[i * ss + c];
                    for (int r = 0; r < a; r++) pac -= R[r * ss + a] * R[r * ss + c];
                    if (c == a) {
                        if (!(pac > 0.0) || !(pac > reorth * reorth * Gm[a * ss + a])) {
                            nok = a;
                            break;
                        }
                        R[a * ss + a] = std::sqrt(pac);
                    } else {
                        R[a * ss + c] = pac / R[a * ss + a];
                    }
                }
            }
            if (h->cur) {
                h->cur->gmres_rounds++;
                if (nok < ss) h->cur->gmres_redone++;
            }
            if (nok < ss) {
                h->scap = std::max(nok, 1);
                h->sgood = 0;
            } else if (++h->sgood >= SCAP_GROW && h->scap < S) {
                h->scap++;
                h->sgood = 0;
            }
            if (nok > 0) {
                // the leading nok vectors in one block update; coefficients: C's
                // first nok columns, then the inverse of R's leading block
                for (int i = 0; i < nv; i++)
                    for (int t = 0; t < nok; t++) hcf[i * nok + t] = C[i * ss + t];
                double *ri = hcf + nv * nok;
                for (int t = 0; t < nok * nok; t++) ri[t] = 0.0;
                for (int c = 0; c < nok; c++) {
                    ri[c * nok + c] = 1.0 / R[c * ss + c];
                    for (int a = c - 1; a >= 0; a--) {
                        double acc = 0.0;
                        for (int r = a + 1; r <= c; r++) acc += R[a * ss + r] * ri[r * nok + c];
                        ri[a * nok + c] = -acc / R[a * ss + a];
                    }
                }
                HIP_TRY(hipMemcpyAsync(dcf, hcf, (nv * nok + nok * nok) * sizeof(double), hipMemcpyHostToDevice, s));
                RICH_TRY(timed(h, RICH_K_BLOCK_UPDATE, 8.0 * N * (nv + 2 * nok), [&] {
                    return launch_block_update(h->V, ld, nv, h->vs, dcf, Q, nok, N, s);
                }));
            }
            if (nok < ss) {
                // the rest vector by vector: two classical passes against
                // everything before it (the block's new vectors included)
                for (int t = nok; t < ss; t++) {
                    for (int i = 0; i < nv; i++) C[i * sw + t] = 0.0;
                    for (int r = 0; r < ss; r++) R[r * sw + t] = 0.0;
                }
                for (int t = nok; t < ss; t++) {
                    const int slot = nv + t;
                    double *w = h->V + (size_t)slot * ld;
                    double ww = 0.0;
                    for (int pass = 0; pass < 2; pass++) {
                        RICH_TRY(timed(h, RICH_K_COUNT, 8.0 * N * (slot + 1), [&] {
                            return launch_multidot(h->V, ld, slot, h->vs, w, N, h->partial, h->dres, s);
                        }));
                        RICH_TRY(timed(h, RICH_K_COUNT, 8.0 * N * (slot + 2), [&] {
                            return launch_update_norm(h->V, ld, slot, h->dres, h->vs, w, N, h->partial, h->dres2, s);
                        }));
                        HIP_TRY(hipMemcpyAsync(h->hres, h->dres, slot * sizeof(double), hipMemcpyDeviceToHost, s));
                        HIP_TRY(hipMemcpyAsync(h->hres + (m + 8), h->dres2, sizeof(double), hipMemcpyDeviceToHost, s));
                        RICH_TRY(sync(h));
                        for (int i = 0; i < nv; i++) C[i * sw + t] += h->hres[i];
                        for (int r = 0; r < t; r++) R[r * sw + t] += h->hres[nv + r];
                        ww = h->hres[m + 8];
                    }
                    RICH_TRY(launch_set_scale(h->vs + slot, h->dres2, s));
                    R[t * sw + t] = std::sqrt(ww);
                    if (!std::isfinite(R[t * sw + t])) {
                        overflow = true;
                        break;
                    }
                    if (!(ww > 0.0)) {  // q_{t+1} lies in the space spanned so far: the cycle ends here
                        ss = t + 1;
                        break;
                    }
                }
            }
            if (overflow) {
                RICH_TRY(classical_round(ss));
                j0 += ss;
                ss_next = S;
                continue;
            }
            // Hessenberg columns j0 .. j0+ss-1 from the coordinates
            const int K = nv + ss, W1 = ss + 1;
            std::vector<double> Sh((size_t)K * W1, 0.0), X((size_t)K * ss);
            Sh[(size_t)j0 * W1] = 1.0;
            for (int t = 0; t < ss; t++) {
                for (int i = 0; i < nv; i++) Sh[(size_t)i * W1 + t + 1] = C[i * sw + t];
                for (int r = 0; r <= t; r++) Sh[(size_t)(nv + r) * W1 + t + 1] = R[r * sw + t];
            }
            for (int r = 0; r < K; r++)
                for (int c = 0; c < ss; c++) {
                    double v = Sh[(size_t)r * W1 + c + 1] + sig[c] * Sh[(size_t)r * W1 + c];
                    for (int q = (r > 0 ? r - 1 : 0); q < j0; q++) v -= Hr[(size_t)r * m + q] * Sh[(size_t)q * W1 + c];
                    X[(size_t)r * ss + c] = v;
                }
            // X <- X Sb^{-1}, Sb[a][c] = Sh[j0 + a][c] (upper triangular)
            for (int c = 0; c < ss; c++) {
                const double d = Sh[(size_t)(j0 + c) * W1 + c];
                for (int r = 0; r < K; r++) {
                    double v = X[(size_t)r * ss + c];
                    for (int a = 0; a < c; a++) v -= X[(size_t)r * ss + a] * Sh[(size_t)(j0 + a) * W1 + c];
                    X[(size_t)r * ss + c] = v / d;
                }
            }
            bool xfinite = true;
            for (int t = 0; t < K * ss; t++) xfinite = xfinite && std::isfinite(X[t]);
            if (!xfinite) {
                RICH_TRY(classical_round(ss));
                j0 += ss;
                ss_next = S;
                continue;
            }
            for (int c = 0; c < ss && !stop; c++) {
                const int j = j0 + c;
                for (int r = 0; r <= j + 1; r++) Hr[(size_t)r * m + j] = X[(size_t)r * ss + c];
                add_column(j);
            }
            j0 += ss;
            // the next round: as many vectors as the decay of the residual
            // estimate over this round predicts are still needed (at most s)
            ss_next = S;
            const double g_end = std::fabs(g[j0]);
            if (!stop && g_end > 0.0 && g_end < g_start) {
                const double need = std::log(eta * bnorm / g_end) / (std::log(g_end / g_start) / ss);
                if (need < S) ss_next = std::max(1, (int)std::ceil(need));
            }
        }
        for (int i = k - 1; i >= 0; i--) {
            double sum = g[i];
            for (int t = i + 1; t < k; t++) sum -= Hm[(size_t)i * m + t] * y[t];
            y[i] = sum / Hm[(size_t)i * m + i];
        }
        memcpy(h->hres, y.data(), k * sizeof(double));
        HIP_TRY(hipMemcpyAsync(h->dres, h->hres, k * sizeof(double), hipMemcpyHostToDevice, s));
        RICH_TRY(launch_lincomb(h->V, ld, k, h->dres, h->vs, h->work, N, s));
        RICH_TRY(prec_product(h, h->work, h->one, nullptr));
        RICH_TRY(add_z(h, x));
        charge(h, 8.0 * (k + 1) * N + (16.0 + (h->mixed ? 4 : 8)) * N);
        RICH_TRY(sync(h));  // hres is reused before the next read
    }
    *its_out = total;
    *relres_out = relres;
    *conv_out = conv;
    return RICH_OK;
}

rich_status gmres(rich_ctx *h, const double *b, double *x, int *its_out, double *relres_out, bool *conv_out) {
    if (h->O.gmres_block >= 2) return gmres_sstep(h, b, x, its_out, relres_out, conv_out);
    return gmres_classic(h, b, x, its_out, relres_out, conv_out);
}

// ----------------------------------------------------------------- Newton
// Host seconds since t0, added to one phase timer of the step in progress.
struct PhaseClock {
    rich_ctx *h;
    double *timer, *bytes_sink, *saved_sink, t0;
    PhaseClock(rich_ctx *hh, double *t, double *b) : h(hh), timer(t), bytes_sink(b), saved_sink(hh->phase_bytes) {
        t0 = now_s();
        if (h->cur) h->phase_bytes = b;
    }
    ~PhaseClock() { h->phase_bytes = saved_sink; }
    rich_status stop() {
        if (!h->cur) return RICH_OK;
        RICH_TRY(sync(h));
        *timer += now_s() - t0;
        return RICH_OK;
    }
};

rich_status feval(rich_ctx *h, const double *u, double *F) {
    rich_step_stats_t *st = h->cur;
    PhaseClock clk(h, st ? &st->t_feval : nullptr, st ? &st->bytes_feval : nullptr);
    RICH_TRY(timed(h, RICH_K_RESIDUAL, (double)h->N * 32,
                   [&] { return launch_residual(h->P, h->Ks, u, h->theta_old, F, h->s); }));
    return clk.stop();
}

// J and M at u in one pass over the grid; then the preconditioner: the full
// AMG set-up the first time, else its numeric update from the new M.
rich_status rebuild(rich_ctx *h, const double *u) {
    rich_step_stats_t *st = h->cur;
    {
        PhaseClock clk(h, st ? &st->t_jac : nullptr, st ? &st->bytes_jac : nullptr);
        charge(h, (double)h->N * (16 + 56 + 32 + 8 + (h->mixed ? 20 : 0)));
        RICH_TRY(launch_assemble(h->P, h->Ks, u, h->J7, h->M4, h->mixed ? h->M4f : nullptr, h->invd0,
                                 h->mixed ? h->invd0f : nullptr, h->O.aux_dflux, h->s));
        RICH_TRY(sync(h));
        RICH_TRY(clk.stop());
    }
    if (st) st->jac_builds++;
    if (!h->H) {
        PhaseClock clk(h, st ? &st->t_setup : nullptr, nullptr);
        RICH_TRY(build_hierarchy(h));
        RICH_TRY(clk.stop());
        if (st) st->amg_setups++;
    } else {
        PhaseClock clk(h, st ? &st->t_aux : nullptr, nullptr);
        RICH_TRY(refresh_hierarchy(h));
        RICH_TRY(clk.stop());
    }
    h->have_J = true;
    h->since_build = 0;
    return RICH_OK;
}

// f = 0.5 ||F||^2 and ||F||_inf
rich_status fnorms(rich_ctx *h, const double *F, double *f_half, double *finf) {
    double n3[3];
    charge(h, 8.0 * h->N);
    RICH_TRY(norms(h, F, n3));
    *f_half = 0.5 * n3[2];
    *finf = n3[0];
    return RICH_OK;
}

void record_trial(rich_newton_event_t *ev, double lam, double f) {
    if (ev->ntrial < RICH_TRACE_TRIALS) {
        ev->trial_lam[ev->ntrial] = lam;
        ev->trial_f[ev->ntrial] = f;
    }
    ev->ntrial++;
}

// Next trial step of the backtracking line search after the trial
// (lam, f(u + lam d)) failed the Armijo condition: Dennis & Schnabel's
// Algorithm A6.3.1, a published method.  The model of f along d takes
// f(0) = f0 and f'(0) = slope; the first reduction minimises the parabola
// through the trial, later ones the cubic through the last two finite trials.
// A non-finite trial gives no model and cuts the step to a tenth.  The result
// is kept in [0.1 lam, 0.5 lam].
struct Backtrack {
    double f0, slope;
    bool have = false;     // a finite trial is on record: cubic model next
    double lp = 0.0, fp = 0.0;

    double next(double lam, double ft) {
        double lt;
        if (!std::isfinite(ft)) {
            lt = 0.1 * lam;
        } else {
            const double r = ft - f0 - slope * lam;  // what the linear model misses at lam
            if (!have) {
                lt = -slope * lam * lam / (2.0 * r);
            } else {
                // c(x) = f0 + slope x + b x^2 + a x^3 through (lp, fp) and (lam, ft)
                const double rp = fp - f0 - slope * lp;
                const double l2 = lam * lam, p2 = lp * lp;
                const double det = l2 * p2 * (lp - lam);
                const double b = (r * p2 * lp - rp * l2 * lam) / det;
                const double a = (rp * l2 - r * p2) / det;
                if (a == 0.0) {
                    lt = -slope / (2.0 * b);
                } else {
                    const double disc = b * b - 3.0 * a * slope;
                    if (disc < 0.0) lt = 0.5 * lam;
                    else if (b >= 0.0) lt = -slope / (b + std::sqrt(disc));  // the root c' = 0, no cancellation
                    else lt = (std::sqrt(disc) - b) / (3.0 * a);
                }
            }
            have = true;
            lp = lam;
            fp = ft;
        }
        if (!(lt <= 0.5 * lam)) lt = 0.5 * lam;  // also catches NaN
        if (!(lt >= 0.1 * lam)) lt = 0.1 * lam;
        return lt;
    }
};

// Line search of Section 3 (Armijo-Goldstein) along d from u.  Trials are
// taken until f(u + lam d) <= f0 + alpha lam slope; below the smallest step
// scsteptol / max_i(|d_i| / max(|u_i|, 1)) it gives up.  A full step that
// was not truncated and beats the beta = 0.9 bound of the linear model is
// doubled while the doubled step keeps the Armijo condition and stays within
// the maximum step (at most ten times).  On success ut/Ft hold the point.
rich_status line_search(rich_ctx *h, double f0, double slope, double mxstep, bool truncated, double dnorm,
                        rich_newton_event_t *ev, double *lam_out) {
    const int64_t N = h->N;
    const double alpha = h->O.ls_alpha, beta = 0.9;
    charge(h, 16.0 * N);
    RICH_TRY(launch_rel_length(h->d, h->u, N, h->partial, h->dres, h->s));
    RICH_TRY(readback(h, h->dres, 1, &ev->rel_d));
    const double lam_min = ev->rel_d > 0.0 ? h->O.scsteptol / ev->rel_d : 0.0;
    auto armijo = [&](double lam, double f) { return std::isfinite(f) && f <= f0 + alpha * lam * slope; };
    auto trial = [&](double lam, double *x, double *Fx, double *f) -> rich_status {
        charge(h, 24.0 * N);
        RICH_TRY(launch_xpay_to(h->u, lam, h->d, x, N, h->s));
        RICH_TRY(feval(h, x, Fx));
        double finf;
        RICH_TRY(fnorms(h, Fx, f, &finf));
        record_trial(ev, lam, *f);
        return RICH_OK;
    };
    Backtrack model{f0, slope};
    double lam = 1.0, ft;
    for (;;) {
        RICH_TRY(trial(lam, h->ut, h->Ft, &ft));
        if (armijo(lam, ft)) break;
        if (lam < lam_min) return RICH_LINESEARCH_FAIL;
        lam = model.next(lam, ft);
        ev->nback++;
    }
    if (lam == 1.0 && !truncated) {
        for (int k = 0; k < 10 && ft < f0 + beta * lam * slope && 2.0 * lam * dnorm <= mxstep; k++) {
            double fb;
            RICH_TRY(trial(2.0 * lam, h->ub, h->Fb, &fb));
            if (!armijo(2.0 * lam, fb)) break;
            lam *= 2.0;
            ft = fb;
            std::swap(h->ut, h->ub);
            std::swap(h->Ft, h->Fb);
        }
    }
    *lam_out = lam;
    return RICH_OK;
}

struct CurGuard {
    rich_ctx *h;
    ~CurGuard() {
        h->cur = nullptr;
        h->phase_bytes = nullptr;
    }
};

void push_event(rich_ctx *h, const rich_newton_event_t &ev) {
    if (!h->trace) return;
    if (h->trace_len < h->trace_cap) h->trace[h->trace_len] = ev;
    h->trace_len++;
}

// One backward-Euler step (Section 2.1) by the modified inexact Newton
// method of Section 3, from the previous level.  Each attempt first applies
// the rebuild test of eq. (jacobian_update_condition): J (with M and the
// preconditioner) is rebuilt when none exists yet, after msbset iterations
// since the last rebuild (the count carries over from step to step: J is
// re-used across steps, Section 6), after a step with ||lam d||_inf > 1.5,
// or when the previous attempt asked for a retry.  A stale J that lets
// GMRES fail, gives no descent direction or makes the line search fail is
// rebuilt and the attempt repeated; with a fresh J these end the step.  A
// step shorter than scsteptol asks for a rebuild (stale J) or ends the step
// with the warning RICH_STEP_TOO_SMALL (fresh J, state kept).
rich_status newton_step(rich_ctx *h, rich_step_stats_t *st) {
    const int64_t N = h->N;
    hipStream_t s = h->s;
    memset(st, 0, sizeof(*st));
    st->min_lambda = 1.0;
    h->cur = st;
    h->phase_bytes = &st->bytes_overhead;
    CurGuard guard{h};
    const int step_index = h->nstep++;
    const double t_start = now_s();
    double pn[3];
    RICH_TRY(norms(h, h->p, pn));
    if (!std::isfinite(pn[0])) return st->status = RICH_NONFINITE;
    RICH_TRY(launch_theta(h->P, h->p, h->theta_old, s));
    HIP_TRY(hipMemcpyAsync(h->u, h->p, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    charge(h, 8.0 * N + 16.0 * N + 16.0 * N);
    RICH_TRY(feval(h, h->u, h->F));
    double f0, fnorm;
    RICH_TRY(fnorms(h, h->F, &f0, &fnorm));
    if (!std::isfinite(fnorm)) return st->status = RICH_NONFINITE;
    double mxstep = h->O.mxnewtstep;
    if (!(mxstep > 0.0)) mxstep = 1000.0 * std::max(std::sqrt(pn[2]), 1.0);

    double prev_step = 0.0;  // ||lam d||_inf of the last accepted step of this time step
    bool retry = false;
    rich_status status = RICH_OK;
    rich_newton_event_t ev;
    // ends the attempt: record it and, for a retry, ask for a rebuild
    auto finish = [&](int outcome) {
        ev.outcome = outcome;
        push_event(h, ev);
        retry = outcome == RICH_EV_RETRY_GMRES || outcome == RICH_EV_RETRY_SLOPE || outcome == RICH_EV_RETRY_LS ||
                outcome == RICH_EV_ACCEPT_SHORT;
    };
    while (fnorm > h->O.fnormtol) {
        if (st->newton_its >= h->O.max_newton) {
            status = RICH_MAXITER;
            break;
        }
        memset(&ev, 0, sizeof(ev));
        ev.step = step_index;
        ev.newton_it = st->newton_its;
        ev.since_build = h->since_build;
        ev.mxstep = mxstep;
        ev.f0 = f0;
        if (!h->have_J) ev.reason |= RICH_RB_NOJ;
        else if (h->since_build >= h->O.msbset) ev.reason |= RICH_RB_MSBSET;
        if (prev_step > 1.5) ev.reason |= RICH_RB_BIGSTEP;
        if (retry) ev.reason |= RICH_RB_RETRY;
        const bool fresh = ev.reason != 0;
        if (fresh) {
            rich_status rc = rebuild(h, h->u);
            if (rc != RICH_OK) {
                status = rc;
                finish(RICH_EV_FAIL_OTHER);
                break;
            }
        }
        retry = false;
        // linear solve J d = -F
        int its;
        double relres;
        bool conv;
        {
            PhaseClock clk(h, &st->t_linsol, &st->bytes_linsol);
            charge(h, 16.0 * N);
            RICH_TRY(launch_negate_to(h->F, h->rhs, N, s));
            RICH_TRY(gmres(h, h->rhs, h->d, &its, &relres, &conv));
            RICH_TRY(clk.stop());
        }
        st->gmres_its += its;
        ev.gmres_its = its;
        ev.gmres_conv = conv;
        if (!conv) {
            st->linsolve_fails++;
            if (!fresh) {
                finish(RICH_EV_RETRY_GMRES);
                continue;
            }
        }
        // step limit, slope of f along d
        double dn3[3];
        charge(h, 8.0 * N);
        RICH_TRY(norms(h, h->d, dn3));
        double dn = std::sqrt(dn3[2]);
        if (dn > mxstep) {
            charge(h, 16.0 * N + 8.0 * N);
            RICH_TRY(launch_scale(h->d, mxstep / dn, N, s));
            RICH_TRY(norms(h, h->d, dn3));
            dn = std::sqrt(dn3[2]);
            ev.truncated = 1;
        }
        ev.dnorm2 = dn;
        ev.dnorminf = dn3[0];
        charge(h, 72.0 * N + 16.0 * N);
        RICH_TRY(launch_spmv_J<double>(h->P, h->J7, h->d, h->Jd, s));
        RICH_TRY(dotp(h, h->F, h->Jd, &ev.slope));
        if (!(ev.slope < 0.0)) {
            if (!fresh) {
                finish(RICH_EV_RETRY_SLOPE);
                continue;
            }
            status = RICH_LINSOLVE_FAIL;
            finish(RICH_EV_FAIL_SLOPE);
            break;
        }
        double lam;
        rich_status rc = line_search(h, f0, ev.slope, mxstep, ev.truncated != 0, dn, &ev, &lam);
        st->ls_backtracks += ev.nback;
        if (rc == RICH_LINESEARCH_FAIL) {
            if (!fresh) {
                finish(RICH_EV_RETRY_LS);
                continue;
            }
            status = rc;
            finish(RICH_EV_FAIL_LS);
            break;
        }
        RICH_TRY(rc);
        // accept u + lam d
        st->min_lambda = std::min(st->min_lambda, lam);
        ev.lam = lam;
        ev.step_inf = lam * ev.dnorminf;
        charge(h, 16.0 * N);
        RICH_TRY(launch_rel_length(h->d, h->ut, N, h->partial, h->dres, s));
        RICH_TRY(readback(h, h->dres, 1, &ev.step_rel));
        ev.step_rel *= lam;
        std::swap(h->u, h->ut);
        std::swap(h->F, h->Ft);
        st->newton_its++;
        h->since_build++;
        RICH_TRY(fnorms(h, h->F, &f0, &fnorm));
        ev.f_acc = f0;
        ev.fnorm_inf = fnorm;
        if (!std::isfinite(fnorm)) {
            status = RICH_NONFINITE;
            finish(RICH_EV_FAIL_OTHER);
            break;
        }
        if (fnorm <= h->O.fnormtol) {
            finish(RICH_EV_ACCEPT);
            break;
        }
        if (ev.step_rel < h->O.scsteptol) {
            if (fresh) {
                status = RICH_STEP_TOO_SMALL;
                finish(RICH_EV_STALL);
                break;
            }
            finish(RICH_EV_ACCEPT_SHORT);
        } else {
            finish(RICH_EV_ACCEPT);
        }
        prev_step = ev.step_inf;
    }
    st->fnorm_inf = fnorm;
    if (status == RICH_OK || status == RICH_STEP_TOO_SMALL) {
        HIP_TRY(hipMemcpyAsync(h->p, h->u, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        double fn[3];
        charge(h, 16.0 * N + 8.0 * N);
        RICH_TRY(norms(h, h->F, fn));
        st->mass_residual = h->P.dt * fn[1];
    }
    if (h->H) {
        st->levels = h->H->nlev;
        st->opc = (double)h->H->nnz_total / (double)h->H->L[0].nnz;
    }
    RICH_TRY(sync(h));
    st->t_total = now_s() - t_start;
    st->t_overhead = st->t_total - (st->t_feval + st->t_jac + st->t_aux + st->t_setup + st->t_linsol);
    st->status = status;
    return status;
}

rich_status validate(const rich_problem_t *P, const rich_solver_opts_t *O) {
    if (!P || !O) return RICH_EINVAL;
    if (P->nx < 1 || P->ny < 1 || P->nz < 1) return RICH_EINVAL;
    int64_t n = (int64_t)P->nx * P->ny * P->nz;
    if (n >= (int64_t)1 << 31) return RICH_EINVAL;
    if (!(P->hx > 0) || !(P->hy > 0) || !(P->hz > 0) || !(P->dt > 0)) return RICH_EINVAL;
    if (P->mean < 0 || P->mean > 4) return RICH_EINVAL;
    if (P->mean_vertical < -1 || P->mean_vertical > 4) return RICH_EINVAL;
    if (P->patch_face < -1 || P->patch_face > 5) return RICH_EINVAL;
    if (P->patch_face >= 0 && (P->bc_type[P->patch_face] != RICH_BC_DIRICHLET || !std::isfinite(P->patch_value)))
        return RICH_EINVAL;
    for (int f = 0; f < 6; f++)
        if (P->bc_type[f] != RICH_BC_NOFLUX && P->bc_type[f] != RICH_BC_DIRICHLET) return RICH_EINVAL;
    if (!(P->alpha > 0) || !(P->A > 0) || !(P->beta > 1) || !(P->gamma > 1)) return RICH_EINVAL;
    if (O->gmres_restart < 1 || O->gmres_restart > 64 || O->gmres_maxit < 1) return RICH_EINVAL;
    if (O->amg_max_levels < 1 || O->amg_sweeps < 1 || O->amg_sweeps > 6) return RICH_EINVAL;
    if (O->coarse_dense_max < 0 || O->coarse_dense_max > 8192 || O->coarse_l1_sweeps < 1) return RICH_EINVAL;
    if (O->precision != RICH_PREC_FP64 && O->precision != RICH_PREC_MIXED) return RICH_EINVAL;
    if (O->amg_refresh != 0 && O->amg_refresh != 1) return RICH_EINVAL;
    if (O->aux_dflux != 0 && O->aux_dflux != 1) return RICH_EINVAL;
    if (O->amg_smoothed < 0 || O->amg_smoothed > 16) return RICH_EINVAL;
    if (O->tile_kz < 0 || O->tile_kz > 4096) return RICH_EINVAL;
    if (O->smoother != RICH_SMOOTH_L1 && O->smoother != RICH_SMOOTH_MCGS) return RICH_EINVAL;
    if (O->amg_aggregation != RICH_AGG_MATCHING && O->amg_aggregation != RICH_AGG_VMB) return RICH_EINVAL;
    if (O->amg_aggregation == RICH_AGG_VMB && (!(O->amg_theta >= 0.0 && O->amg_theta <= 1.0) || O->amg_block < 1))
        return RICH_EINVAL;
    if (!(O->gmres_reorth >= 0.0 && O->gmres_reorth < 1.0)) return RICH_EINVAL;
    if (O->gmres_block < 1 || O->gmres_block > GMRES_BLOCK_MAX || !std::isfinite(O->gmres_shift) ||
        !(O->gmres_shift_span >= 0.0) || !std::isfinite(O->gmres_shift_span))
        return RICH_EINVAL;
    if (!(O->eta > 0) || !(O->fnormtol > 0) || O->max_newton < 1 || O->msbset < 1) return RICH_EINVAL;
    return RICH_OK;
}

// Gauss-Legendre nodes and weights on [0, 1]: roots of the Legendre
// polynomial P_n by Newton's method (three-term recurrence, cosine starting
// values), weights 2 / ((1 - x^2) P_n'(x)^2), both mapped from [-1, 1].
void gauss_legendre01(double *t, double *w, int n) {
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; i++) {
        double x = std::cos(pi * (i + 0.75) / (n + 0.5)), d = 1.0;
        for (int it = 0; it < 100; it++) {
            double a = 1.0, b = x;
            for (int k = 2; k <= n; k++) {
                double c = ((2.0 * k - 1.0) * x * b - (k - 1.0) * a) / k;
                a = b;
                b = c;
            }
            d = n * (x * b - a) / (x * x - 1.0);
            double step = b / d;
            x -= step;
            if (std::fabs(step) < 1e-16) break;
        }
        t[i] = 0.5 * (1.0 - x);
        w[i] = 1.0 / ((1.0 - x * x) * d * d);
    }
}

Phys to_phys(const rich_problem_t *P) {
    Phys q;
    q.nx = P->nx;
    q.ny = P->ny;
    q.nz = P->nz;
    q.hx = P->hx;
    q.hy = P->hy;
    q.hz = P->hz;
    q.alpha = P->alpha;
    q.beta = P->beta;
    q.theta_s = P->theta_s;
    q.theta_r = P->theta_r;
    q.A = P->A;
    q.gamma = P->gamma;
    q.mean = P->mean;
    q.mean_vertical = P->mean_vertical;
    for (int f = 0; f < 6; f++) {
        q.bc_type[f] = P->bc_type[f];
        q.bc_value[f] = P->bc_value[f];
    }
    q.dt = P->dt;
    q.patch_face = P->patch_face;
    for (int t = 0; t < 2; t++) {
        q.patch_lo[t] = P->patch_lo[t];
        q.patch_hi[t] = P->patch_hi[t];
    }
    q.patch_value = P->patch_value;
    q.tile_kz = 0;
    gauss_legendre01(q.gl_t, q.gl_w, RICH_GL);
    return q;
}

}  // namespace

// ============================================================== C-ABI ====
extern "C" {

const char *rich_status_string(rich_status s) {
    switch (s) {
    case RICH_OK: return "ok";
    case RICH_EINVAL: return "invalid argument";
    case RICH_ENOMEM: return "device allocation failed";
    case RICH_EBUDGET: return "memory budget exceeded";
    case RICH_NONFINITE: return "non-finite value";
    case RICH_LINSOLVE_FAIL: return "linear solver failed with a fresh Jacobian";
    case RICH_LINESEARCH_FAIL: return "line search failed with a fresh Jacobian";
    case RICH_MAXITER: return "Newton iteration limit reached";
    case RICH_NOT_SPD: return "coarsest matrix not positive definite";
    case RICH_EHIP: return rich::last_error()[0] ? rich::last_error() : "HIP runtime error";
    case RICH_ESTATE: return "call not valid in the current state";
    case RICH_STEP_TOO_SMALL: return "Newton step below scsteptol with a fresh Jacobian";
    default: return "unknown status";
    }
}

rich_status rich_query_bytes(const rich_problem_t *prob, const rich_solver_opts_t *opts, size_t *bytes) {
    RICH_TRY(validate(prob, opts));
    if (!bytes) return RICH_EINVAL;
    size_t N = (size_t)prob->nx * prob->ny * prob->nz;
    size_t m = opts->gmres_restart;
    bool mixed = opts->precision == RICH_PREC_MIXED;
    size_t b = 0;
    b += N * 8 * 15;                    // fields and Newton work vectors
    b += N * 8 * 7 + N * 8 * 5;         // J, M, l1 diagonal
    if (mixed) b += N * 4 * 5;          // FP32 copies
    b += (m + 1) * N * 8;               // Krylov basis
    b += N * 8 * 2;                     // preconditioner output and scratch
    size_t esz = mixed ? 4 : 8;
    // hierarchy bound: operator complexity <= 3, 12-byte CSR entries plus value copies
    size_t nnz0 = 7 * N;
    b += 2 * nnz0 * (12 + esz) + N * (8 + esz + 3 * esz + 8) * 2;
    if (opts->amg_smoothed) {
        // level 0 dominates: P and PT (~4.2 entries per fine row), Q = A P
        // (~12 per row), coarse levels about twice as dense, and the scratch
        // of the symbolic products during set-up
        b += 2 * (5 * N) * (12 + 8 + esz);
        b += 14 * N * 12;
        b += nnz0 * (12 + esz);
        b += 200 * N;
    }
    size_t nc = (size_t)(opts->coarse_dense_max);
    b += nc * nc * (8 + esz);
    *bytes = b;
    return RICH_OK;
}

rich_status rich_create(const rich_problem_t *prob, const rich_solver_opts_t *opts, const double *Ks_dev,
                        void *hip_stream, rich_handle_t *out) {
    RICH_TRY(validate(prob, opts));
    if (!Ks_dev || !out) return RICH_EINVAL;
    rich_ctx *h = new rich_ctx();
    h->P = to_phys(prob);
    h->P.tile_kz = opts->tile_kz;
    h->O = *opts;
    h->N = (int64_t)prob->nx * prob->ny * prob->nz;
    h->s = (hipStream_t)hip_stream;
    h->mixed = opts->precision == RICH_PREC_MIXED;
    h->m = opts->gmres_restart;
    leja_points(opts->gmres_shift - opts->gmres_shift_span, opts->gmres_shift + opts->gmres_shift_span,
                GMRES_BLOCK_MAX, h->shifts);
    h->scap = opts->gmres_block;
    int64_t N = h->N;
    rich_status st = RICH_OK;
    auto G = [&](auto **p, size_t n) {
        if (st == RICH_OK) st = h->mem.get(p, n);
    };
    G(&h->Ks, N);
    G(&h->p, N);
    G(&h->theta_old, N);
    G(&h->u, N);
    G(&h->F, N);
    G(&h->ut, N);
    G(&h->Ft, N);
    G(&h->d, N);
    G(&h->Jd, N);
    G(&h->ub, N);
    G(&h->Fb, N);
    G(&h->rhs, N);
    G(&h->work, N);
    G(&h->J7, 7 * N);
    G(&h->M4, 4 * N);
    G(&h->invd0, N);
    if (h->mixed) {
        G(&h->M4f, 4 * N);
        G(&h->invd0f, N);
    }
    h->ldv = (N + 63) / 64 * 64;
    G(&h->V, (size_t)(h->m + 1) * h->ldv);
    char *z = nullptr, *zt = nullptr;
    G(&z, N * 8);
    G(&zt, N * 8);
    h->z = z;
    h->ztmp = zt;
    G(&h->partial, (size_t)RED_BLOCKS * std::max(3 * (h->m + 2), block_partial_size(h->m + 1, GMRES_BLOCK_MAX)));
    G(&h->dblk, 2 * BLK_BUF);
    G(&h->dres, h->m + 8);
    G(&h->dres2, 8);
    G(&h->vs, h->m + 2);
    G(&h->one, 1);
    G(&h->hbuf, (size_t)(h->m + 1) * (h->m + 4));
    G(&h->bsc, N);
    if (st == RICH_OK && hipHostMalloc((void **)&h->hres, 2 * (h->m + 8) * sizeof(double)) != hipSuccess)
        st = RICH_ENOMEM;
    if (st == RICH_OK &&
        hipHostMalloc((void **)&h->hall, (size_t)(h->m + 1) * (h->m + 4) * sizeof(double)) != hipSuccess)
        st = RICH_ENOMEM;
    if (st == RICH_OK && hipHostMalloc((void **)&h->hblk, 2 * BLK_BUF * sizeof(double)) != hipSuccess)
        st = RICH_ENOMEM;
    for (int j = 0; st == RICH_OK && j <= h->m; j++) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) st = RICH_EHIP;
        else h->iter_ev.push_back(e);
    }
    if (st == RICH_OK) st = launch_fill_f64(h->one, 1.0, 1, h->s);
    if (st == RICH_OK) st = launch_fill_f64(h->vs, 1.0, h->m + 2, h->s);
    if (st == RICH_OK && hipMemcpyAsync(h->Ks, Ks_dev, N * sizeof(double), hipMemcpyDeviceToDevice, h->s) != hipSuccess)
        st = RICH_EHIP;
    if (st == RICH_OK) st = launch_fill_f64(h->p, 0.0, N, h->s);
    if (st == RICH_OK && hipStreamSynchronize(h->s) != hipSuccess) st = RICH_EHIP;
    if (st != RICH_OK) {
        delete h;
        return st;
    }
    *out = h;
    return RICH_OK;
}

rich_status rich_destroy(rich_handle_t h) {
    if (!h) return RICH_EINVAL;
    (void)hipStreamSynchronize(h->s);
    delete h;
    return RICH_OK;
}

rich_status rich_set_state(rich_handle_t h, const double *p_dev) {
    if (!h || !p_dev) return RICH_EINVAL;
    HIP_TRY(hipMemcpyAsync(h->p, p_dev, h->N * sizeof(double), hipMemcpyDeviceToDevice, h->s));
    return sync(h);
}

rich_status rich_get_state(rich_handle_t h, double *p_dev) {
    if (!h || !p_dev) return RICH_EINVAL;
    HIP_TRY(hipMemcpyAsync(p_dev, h->p, h->N * sizeof(double), hipMemcpyDeviceToDevice, h->s));
    return sync(h);
}

rich_status rich_step(rich_handle_t h, int nsteps, rich_step_stats_t *stats_host) {
    if (!h || nsteps < 0) return RICH_EINVAL;
    rich_status warn = RICH_OK;
    for (int t = 0; t < nsteps; t++) {
        rich_step_stats_t st;
        rich_status rc = newton_step(h, &st);
        if (rc < 0 && st.status >= 0) st.status = rc;  // an error raised below the controller
        if (stats_host) stats_host[t] = st;
        if (rc < 0) return rc;
        warn = std::max(warn, rc);
    }
    return warn;
}

rich_status rich_trace_newton(rich_handle_t h, rich_newton_event_t *events_host, int capacity) {
    if (!h || (events_host && capacity < 0)) return RICH_EINVAL;
    h->trace = events_host;
    h->trace_cap = events_host ? capacity : 0;
    h->trace_len = 0;
    return RICH_OK;
}

rich_status rich_trace_count(rich_handle_t h, int64_t *count_host) {
    if (!h || !count_host) return RICH_EINVAL;
    *count_host = h->trace_len;
    return RICH_OK;
}

rich_status rich_eval_theta(rich_handle_t h, const double *p_dev, double *theta_dev) {
    if (!h || !p_dev || !theta_dev) return RICH_EINVAL;
    RICH_TRY(launch_theta(h->P, p_dev, theta_dev, h->s));
    return sync(h);
}

rich_status rich_eval_residual(rich_handle_t h, const double *p_dev, const double *theta_old_dev, double *F_dev) {
    if (!h || !p_dev || !theta_old_dev || !F_dev) return RICH_EINVAL;
    RICH_TRY(launch_residual(h->P, h->Ks, p_dev, theta_old_dev, F_dev, h->s));
    return sync(h);
}

rich_status rich_assemble(rich_handle_t h, const double *p_dev) {
    if (!h || !p_dev) return RICH_EINVAL;
    return rebuild(h, p_dev);
}

rich_status rich_setup_hierarchy(rich_handle_t h) {
    if (!h) return RICH_EINVAL;
    if (!h->have_J) return RICH_ESTATE;
    return build_hierarchy(h);
}

rich_status rich_apply_jacobian(rich_handle_t h, const double *x_dev, double *y_dev) {
    if (!h || !x_dev || !y_dev) return RICH_EINVAL;
    if (!h->have_J) return RICH_ESTATE;
    RICH_TRY(launch_spmv_J<double>(h->P, h->J7, x_dev, y_dev, h->s));
    return sync(h);
}

rich_status rich_apply_aux(rich_handle_t h, const double *x_dev, double *y_dev) {
    if (!h || !x_dev || !y_dev) return RICH_EINVAL;
    if (!h->have_J) return RICH_ESTATE;
    RICH_TRY(launch_spmv_M(h->P, h->M4, x_dev, y_dev, h->s));
    return sync(h);
}

rich_status rich_apply_prec(rich_handle_t h, const double *b_dev, double *x_dev) {
    if (!h || !b_dev || !x_dev) return RICH_EINVAL;
    if (!h->H) return RICH_ESTATE;
    RICH_TRY(apply_prec(h, b_dev, h->one));
    if (h->mixed) RICH_TRY(launch_cast<float, double>((const float *)h->z, x_dev, h->N, h->s));
    else HIP_TRY(hipMemcpyAsync(x_dev, h->z, h->N * sizeof(double), hipMemcpyDeviceToDevice, h->s));
    return sync(h);
}

rich_status rich_gmres(rich_handle_t h, const double *b_dev, double *x_dev, int *its_host, double *relres_host) {
    if (!h || !b_dev || !x_dev) return RICH_EINVAL;
    if (!h->H) return RICH_ESTATE;
    int its;
    double rr;
    bool conv;
    RICH_TRY(gmres(h, b_dev, x_dev, &its, &rr, &conv));
    if (its_host) *its_host = its;
    if (relres_host) *relres_host = rr;
    RICH_TRY(sync(h));
    return conv ? RICH_OK : RICH_LINSOLVE_FAIL;
}

rich_status rich_levels(rich_handle_t h, int *nlev_host) {
    if (!h || !nlev_host) return RICH_EINVAL;
    *nlev_host = h->H ? h->H->nlev : 0;
    return RICH_OK;
}

rich_status rich_level_size(rich_handle_t h, int level, int64_t *n_host, int64_t *nnz_host) {
    if (!h || !h->H || level < 0 || level >= h->H->nlev) return RICH_EINVAL;
    if (n_host) *n_host = h->H->L[level].n;
    if (nnz_host) *nnz_host = h->H->L[level].nnz;
    return RICH_OK;
}

rich_status rich_export_csr(rich_handle_t h, int which, int level, int64_t *rowptr_host, int32_t *col_host,
                            double *val_host, int64_t *nnz_inout) {
    if (!h || !rowptr_host || !col_host || !val_host || !nnz_inout) return RICH_EINVAL;
    if (!h->have_J) return RICH_ESTATE;
    int64_t N = h->N;
    if (which == RICH_WHICH_J || (which == RICH_WHICH_A && level == 0)) {
        DevAlloc tmp;
        int64_t *cnt, *stmp, *rp;
        int32_t *col;
        double *val;
        RICH_TRY(tmp.get(&cnt, N));
        RICH_TRY(tmp.get(&stmp, scan_tmp_size(N)));
        RICH_TRY(tmp.get(&rp, N + 1));
        RICH_TRY(launch_stencil_rowcounts(h->P, cnt, h->s));
        RICH_TRY(scan_exclusive_i64(cnt, rp, N, stmp, h->s));
        int64_t nnz;
        HIP_TRY(hipMemcpyAsync(&nnz, rp + N, sizeof(int64_t), hipMemcpyDeviceToHost, h->s));
        RICH_TRY(sync(h));
        if (*nnz_inout < nnz) {
            *nnz_inout = nnz;
            return RICH_EINVAL;
        }
        RICH_TRY(tmp.get(&col, nnz));
        RICH_TRY(tmp.get(&val, nnz));
        if (which == RICH_WHICH_J) RICH_TRY(launch_J_to_csr(h->P, h->J7, rp, col, val, h->s));
        else RICH_TRY(launch_stencil_to_csr(h->P, h->M4, rp, col, val, h->s));
        HIP_TRY(hipMemcpyAsync(rowptr_host, rp, (N + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, h->s));
        HIP_TRY(hipMemcpyAsync(col_host, col, nnz * sizeof(int32_t), hipMemcpyDeviceToHost, h->s));
        HIP_TRY(hipMemcpyAsync(val_host, val, nnz * sizeof(double), hipMemcpyDeviceToHost, h->s));
        RICH_TRY(sync(h));
        *nnz_inout = nnz;
        return RICH_OK;
    }
    if (which == RICH_WHICH_P || which == RICH_WHICH_PT) {
        if (!h->H || level < 0 || level >= h->H->nlev - 1) return RICH_EINVAL;
        const Level &Lp = h->H->L[level];
        const int64_t nc = h->H->L[level + 1].n;
        const bool tr = which == RICH_WHICH_PT;
        const int64_t nnz = Lp.prow ? Lp.pnnz : Lp.n, nrows = tr ? nc : Lp.n;
        if (*nnz_inout < nnz) {
            *nnz_inout = nnz;
            return RICH_EINVAL;
        }
        if (Lp.prow) {  // smoothed: P and its transpose are stored
            HIP_TRY(hipMemcpyAsync(rowptr_host, tr ? Lp.trow : Lp.prow, (nrows + 1) * sizeof(int64_t),
                                   hipMemcpyDeviceToHost, h->s));
            HIP_TRY(hipMemcpyAsync(col_host, tr ? Lp.tcol : Lp.pcol, nnz * sizeof(int32_t), hipMemcpyDeviceToHost,
                                   h->s));
            HIP_TRY(hipMemcpyAsync(val_host, tr ? Lp.tval : Lp.pval, nnz * sizeof(double), hipMemcpyDeviceToHost,
                                   h->s));
            RICH_TRY(sync(h));
            // columns ascending within each row, as for every exported matrix
            std::vector<std::pair<int32_t, double>> row;
            for (int64_t r = 0; r < nrows; r++) {
                row.clear();
                for (int64_t e = rowptr_host[r]; e < rowptr_host[r + 1]; e++) row.push_back({col_host[e], val_host[e]});
                std::sort(row.begin(), row.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
                for (int64_t e = rowptr_host[r], k = 0; e < rowptr_host[r + 1]; e++, k++) {
                    col_host[e] = row[k].first;
                    val_host[e] = row[k].second;
                }
            }
        } else {  // piecewise constant: P(i, agg(i)) = 1, built from the aggregate map
            std::vector<int32_t> agg(Lp.n);
            HIP_TRY(hipMemcpyAsync(agg.data(), Lp.agg, Lp.n * sizeof(int32_t), hipMemcpyDeviceToHost, h->s));
            RICH_TRY(sync(h));
            if (!tr) {
                for (int64_t i = 0; i <= Lp.n; i++) rowptr_host[i] = i;
                for (int64_t i = 0; i < Lp.n; i++) col_host[i] = agg[i];
            } else {
                std::fill(rowptr_host, rowptr_host + nc + 1, 0);
                for (int64_t i = 0; i < Lp.n; i++) rowptr_host[agg[i] + 1]++;
                for (int64_t c = 0; c < nc; c++) rowptr_host[c + 1] += rowptr_host[c];
                std::vector<int64_t> pos(rowptr_host, rowptr_host + nc);
                for (int64_t i = 0; i < Lp.n; i++) col_host[pos[agg[i]]++] = (int32_t)i;  // members ascending
            }
            std::fill(val_host, val_host + nnz, 1.0);
        }
        *nnz_inout = nnz;
        return RICH_OK;
    }
    if (which != RICH_WHICH_A || !h->H || level < 0 || level >= h->H->nlev) return RICH_EINVAL;
    const Level &Lv = h->H->L[level];
    if (*nnz_inout < Lv.nnz) {
        *nnz_inout = Lv.nnz;
        return RICH_EINVAL;
    }
    HIP_TRY(hipMemcpyAsync(rowptr_host, Lv.rowptr, (Lv.n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, h->s));
    HIP_TRY(hipMemcpyAsync(col_host, Lv.col, Lv.nnz * sizeof(int32_t), hipMemcpyDeviceToHost, h->s));
    HIP_TRY(hipMemcpyAsync(val_host, Lv.val, Lv.nnz * sizeof(double), hipMemcpyDeviceToHost, h->s));
    RICH_TRY(sync(h));
    *nnz_inout = Lv.nnz;
    return RICH_OK;
}

rich_status rich_export_aggregates(rich_handle_t h, int level, int32_t *agg_host, int64_t *n_coarse_host) {
    if (!h || !h->H || !agg_host || level < 0 || level >= h->H->nlev - 1) return RICH_EINVAL;
    const Level &Lv = h->H->L[level];
    HIP_TRY(hipMemcpyAsync(agg_host, Lv.agg, Lv.n * sizeof(int32_t), hipMemcpyDeviceToHost, h->s));
    RICH_TRY(sync(h));
    if (n_coarse_host) *n_coarse_host = h->H->L[level + 1].n;
    return RICH_OK;
}

rich_status rich_profile(rich_handle_t h, int enable) {
    if (!h) return RICH_EINVAL;
    RICH_TRY(prof_harvest(h));
    if (enable) {
        for (auto &k : h->prof) {
            k.launches = 0;
            k.bytes = 0.0;
            k.ms = 0.0;
        }
    }
    h->profiling = enable != 0;
    return RICH_OK;
}

rich_status rich_profile_read(rich_handle_t h, int kernel, int64_t *launches_host, double *ms_host,
                              double *bytes_host) {
    if (!h || kernel < 0 || kernel >= RICH_K_COUNT) return RICH_EINVAL;
    RICH_TRY(prof_harvest(h));
    const auto &k = h->prof[kernel];
    if (launches_host) *launches_host = k.launches;
    if (ms_host) *ms_host = k.ms;
    if (bytes_host) *bytes_host = k.bytes;
    return RICH_OK;
}

rich_status rich_match_sweep(int64_t n, const int64_t *rowptr_dev, const int32_t *col_dev, const double *val_dev,
                             int32_t *agg_dev, int64_t *n_coarse_host, void *hip_stream) {
    if (n < 0 || n >= ((int64_t)1 << 31) || !rowptr_dev || !col_dev || !val_dev || !agg_dev || !n_coarse_host)
        return RICH_EINVAL;
    return match_sweep(n, rowptr_dev, col_dev, val_dev, agg_dev, n_coarse_host, (hipStream_t)hip_stream);
}

}  // extern "C"

// ------------------------------------------------- batcher (server side)
namespace rich {

rich_batcher *batcher_create(bool persistent) {
    rich_batcher *B = new rich_batcher();
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess || hipStreamCreateWithFlags(&B->s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&B->done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        batcher_destroy(B);
        return nullptr;
    }
    if (persistent) {
        // the work counter starts at zero (a fill kernel, not a memset) and is
        // only ever advanced by the launches on B->s
        if (hipMalloc((void **)&B->queue.ctr, sizeof(unsigned long long)) != hipSuccess ||
            launch_fill_u64(B->queue.ctr, 0ull, 1, B->s) != RICH_OK || hipStreamSynchronize(B->s) != hipSuccess) {
            (void)hipGetLastError();
            batcher_destroy(B);
            return nullptr;
        }
        B->persistent = true;
    }
    B->thread = std::thread(batcher_main, B, device);
    return B;
}

// Every attached simulation has finished before the batcher is destroyed.
void batcher_destroy(rich_batcher *B) {
    if (!B) return;
    if (B->thread.joinable()) {
        {
            std::lock_guard<std::mutex> lk(B->mu);
            B->stop = true;
        }
        B->cv.notify_all();
        B->thread.join();
    }
    if (B->s) {
        (void)hipStreamSynchronize(B->s);
        (void)hipStreamDestroy(B->s);
    }
    if (B->done) (void)hipEventDestroy(B->done);
    if (B->queue.ctr) (void)hipFree(B->queue.ctr);
    delete B;
}

rich_status batcher_attach(rich_handle_t h, rich_batcher *B) {
    if (!h) return RICH_EINVAL;
    if (B && !h->bev) HIP_TRY(hipEventCreateWithFlags(&h->bev, hipEventDisableTiming));
    h->batcher = B;
    return RICH_OK;
}

void batcher_stats(rich_batcher *B, int64_t *flushes, int64_t *items) {
    std::lock_guard<std::mutex> lk(B->mu);
    if (flushes) *flushes = B->flushes;
    if (items) *items = B->items;
}

}  // namespace rich
