// Aggregation AMG (Section 5.2): parallel pairwise matching, piecewise-
// constant Galerkin products, l1 smoother data, the CSR pieces of the
// V-cycle and the dense coarsest-level solve.
#include "common.hpp"

#include <algorithm>
#include <cstring>

namespace rich {

namespace {

constexpr int TPB = 256;

inline unsigned nblocks(int64_t n, int tpb = TPB) { return (unsigned)((n + tpb - 1) / tpb); }

// --------------------------------------------------------------- matching
// Edge {i,j} (i != j) carries the value a_{lo,hi} of row lo = min(i,j) and
// weight w = 1 - 2 a_{lo,hi} / (a_lolo + a_hihi); edges with a zero value or
// a non-finite weight do not exist.  The strict order is (w desc, lo asc,
// hi asc).  A vertex matches its best free neighbour when that neighbour's
// best free neighbour is the vertex itself (locally dominant edge): repeated
// until no free vertex has a free neighbour, this gives exactly the greedy
// matching that scans all edges in the strict order.

__device__ inline double find_entry(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                    const double *__restrict__ val, int64_t row, int32_t c, bool *found) {
    int64_t lo = rowptr[row], hi = rowptr[row + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) >> 1;
        int32_t cm = col[mid];
        if (cm == c) {
            *found = true;
            return val[mid];
        }
        if (cm < c) lo = mid + 1;
        else hi = mid - 1;
    }
    *found = false;
    return 0.0;
}

__global__ void k_diag(int64_t n, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                       const double *__restrict__ val, double *__restrict__ diag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = 0.0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++)
        if (col[e] == i) d = val[e];
    diag[i] = d;
}

// The edge weights of a sweep, once: w[e] = 1 - 2 a_lo,hi / (d_lo + d_hi) for
// the entry e = (i, j), the coupling a read in the lower-numbered row; NaN
// where the entry can never be a candidate (the diagonal, a coupling missing
// from the lower row, a zero coupling).  k_candidates skips every entry
// whose weight is not finite.
__global__ void k_match_weights(int64_t n, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                const double *__restrict__ val, const double *__restrict__ diag,
                                double *__restrict__ w) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
        int32_t j = col[e];
        double we = __builtin_nan("");
        if (j != i) {
            int64_t lo = j < i ? j : i, hi = j < i ? i : j;
            bool found = true;
            double a = lo == i ? val[e] : find_entry(rowptr, col, val, lo, (int32_t)hi, &found);
            if (found && a != 0.0) we = 1.0 - (2.0 * a) / (diag[lo] + diag[hi]);
        }
        w[e] = we;
    }
}

// One matching round: every free row proposes its free neighbour of largest
// weight (ties to the smaller (lo, hi) pair); -1 when there is none.
__global__ void k_candidates(int64_t n, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                             const double *__restrict__ w, const int32_t *__restrict__ mate,
                             int32_t *__restrict__ cand) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (mate[i] != -1) {
        cand[i] = -1;
        return;
    }
    int32_t best = -1;
    double bw = 0.0;
    int64_t blo = 0, bhi = 0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
        int32_t j = col[e];
        if (j == i || mate[j] != -1) continue;
        double we = w[e];
        if (!isfinite(we)) continue;
        int64_t lo = j < i ? j : i, hi = j < i ? i : j;
        bool better = best < 0 || we > bw || (we == bw && (lo < blo || (lo == blo && hi < bhi)));
        if (better) {
            best = j;
            bw = we;
            blo = lo;
            bhi = hi;
        }
    }
    cand[i] = best;
}

__global__ void k_commit(int64_t n, const int32_t *__restrict__ cand, int32_t *__restrict__ mate,
                         int *__restrict__ still_free) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (mate[i] != -1) return;
    int32_t c = cand[i];
    if (c < 0) {
        mate[i] = -2;  // no free neighbour left: a singleton for good
    } else if (cand[c] == (int32_t)i) {
        mate[i] = c;
    } else {
        *still_free = 1;
    }
}

__global__ void k_leaders(int64_t n, const int32_t *__restrict__ mate, int64_t *__restrict__ flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t m = mate[i];
    flag[i] = (m < 0 || i < m) ? 1 : 0;
}

__global__ void k_number(int64_t n, const int32_t *__restrict__ mate, const int64_t *__restrict__ id,
                         int32_t *__restrict__ agg) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t m = mate[i];
    agg[i] = (int32_t)((m < 0 || i < m) ? id[i] : id[m]);
}

// ------------------------------------- decoupled greedy (VMB) aggregation
// DSVMB coarsening (Section 5.2): each block of `block` consecutive rows (a
// "process") aggregates its own rows, ignoring couplings that leave the block,
// so the blocks are independent: one thread per block runs the three greedy
// phases over its rows in index order.  j is strongly coupled to i when
// |a_ij| >= theta sqrt(|a_ii a_jj|).  Phase 1: a free row whose strong
// neighbours are all free starts an aggregate with them; phase 2: a free row
// joins the phase-1 aggregate of its strongest strong neighbour aggregated in
// phase 1 (first in column order on ties); phase 3: a free row starts an
// aggregate with its free strong neighbours.  Ids are block-local here and
// offset by the aggregates of the earlier blocks afterwards.
__global__ void k_row_diag(int64_t n, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                           const double *__restrict__ val, double *__restrict__ diag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = 0.0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++)
        if (col[e] == i) d = val[e];
    diag[i] = d;
}

__global__ void k_vmb_block(int64_t n, int64_t block, int64_t nblk, const int64_t *__restrict__ rowptr,
                            const int32_t *__restrict__ col, const double *__restrict__ val,
                            const double *__restrict__ diag, double theta, int32_t *__restrict__ agg,
                            int32_t *__restrict__ p1, int64_t *__restrict__ count) {
#pragma clang fp contract(off)
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblk) return;
    const int64_t b0 = b * block, b1 = b0 + block < n ? b0 + block : n;
    auto strong = [&](int64_t i, int64_t e) {
        int64_t j = col[e];
        return j != i && j >= b0 && j < b1 && fabs(val[e]) >= theta * sqrt(fabs(diag[i] * diag[j]));
    };
    int32_t nc = 0;
    for (int64_t i = b0; i < b1; i++) agg[i] = -1;
    for (int64_t i = b0; i < b1; i++) {  // phase 1
        bool ok = agg[i] < 0;
        for (int64_t e = rowptr[i]; ok && e < rowptr[i + 1]; e++)
            if (strong(i, e) && agg[col[e]] >= 0) ok = false;
        if (!ok) continue;
        agg[i] = nc;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++)
            if (strong(i, e)) agg[col[e]] = nc;
        nc++;
    }
    for (int64_t i = b0; i < b1; i++) p1[i] = agg[i];
    for (int64_t i = b0; i < b1; i++) {  // phase 2
        if (agg[i] >= 0) continue;
        double best = -1.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
            if (!strong(i, e) || p1[col[e]] < 0) continue;
            double sv = fabs(val[e]) / sqrt(fabs(diag[i] * diag[col[e]]));
            if (sv > best) {
                best = sv;
                agg[i] = p1[col[e]];
            }
        }
    }
    for (int64_t i = b0; i < b1; i++) {  // phase 3
        if (agg[i] >= 0) continue;
        agg[i] = nc;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++)
            if (strong(i, e) && agg[col[e]] < 0) agg[col[e]] = nc;
        nc++;
    }
    count[b] = nc;
}

__global__ void k_vmb_offset(int64_t n, int64_t block, const int64_t *__restrict__ off, int32_t *__restrict__ agg) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    agg[i] += (int32_t)off[i / block];
}

// ---------------------------------------------------------------- Galerkin
__global__ void k_count_members(int64_t n, const int32_t *__restrict__ agg, int64_t *__restrict__ cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    atomicAdd((unsigned long long *)&cnt[agg[i]], 1ull);
}

__global__ void k_place_members(int64_t n, const int32_t *__restrict__ agg, const int64_t *__restrict__ mptr,
                                unsigned int *__restrict__ cursor, int32_t *__restrict__ mem) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t I = agg[i];
    unsigned int pos = atomicAdd(&cursor[I], 1u);
    mem[mptr[I] + pos] = (int32_t)i;
}

// Members were placed in arbitrary order; sort each (small) list ascending.
__global__ void k_sort_members(int64_t nc, const int64_t *__restrict__ mptr, int32_t *__restrict__ mem) {
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    int64_t a = mptr[I], b = mptr[I + 1];
    for (int64_t t = a + 1; t < b; t++) {
        int32_t v = mem[t];
        int64_t u = t - 1;
        while (u >= a && mem[u] > v) {
            mem[u + 1] = mem[u];
            u--;
        }
        mem[u + 1] = v;
    }
}

// Symbolic product: the coarse columns J = agg[j] reached from the member
// rows of coarse row I, sorted and unique.  Each coarse row owns a scratch
// segment as long as the sum of its members' row lengths (an upper bound).
__global__ void k_seg_len(int64_t nc, const int64_t *__restrict__ mptr, const int32_t *__restrict__ mem,
                          const int64_t *__restrict__ rowptr, int64_t *__restrict__ seg) {
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    int64_t s = 0;
    for (int64_t t = mptr[I]; t < mptr[I + 1]; t++) s += rowptr[mem[t] + 1] - rowptr[mem[t]];
    seg[I] = s;
}

__global__ void k_sym_collect(int64_t nc, const int64_t *__restrict__ mptr, const int32_t *__restrict__ mem,
                              const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                              const int32_t *__restrict__ agg, const int64_t *__restrict__ segptr,
                              int32_t *__restrict__ scratch, int64_t *__restrict__ cnt) {
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    int32_t *buf = scratch + segptr[I];
    int64_t len = 0;
    for (int64_t t = mptr[I]; t < mptr[I + 1]; t++) {
        int32_t i = mem[t];
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
            // insert agg[col] into the sorted unique prefix buf[0..len)
            int32_t J = agg[col[e]];
            int64_t u = len;
            while (u > 0 && buf[u - 1] > J) u--;
            if (u > 0 && buf[u - 1] == J) continue;
            for (int64_t v = len; v > u; v--) buf[v] = buf[v - 1];
            buf[u] = J;
            len++;
        }
    }
    cnt[I] = len;
}

__global__ void k_sym_write(int64_t nc, const int64_t *__restrict__ segptr, const int32_t *__restrict__ scratch,
                            const int64_t *__restrict__ crow, int32_t *__restrict__ ccol) {
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    const int32_t *buf = scratch + segptr[I];
    int64_t o = crow[I], n = crow[I + 1] - o;
    for (int64_t a = 0; a < n; a++) ccol[o + a] = buf[a];
}

// Numeric product on a fixed pattern: members ascending, each fine row in
// column order, every term added to its coarse entry in that order (the
// oracle's order), starting from zero.  One thread per coarse row; rows of up
// to GAL_REG entries accumulate in LDS (column-major over the block's 64
// threads, so dynamic indexing never spills to scratch memory), longer rows
// directly in the output.
constexpr int GAL_REG = 32;
__global__ void __launch_bounds__(64) k_gal_numeric(int64_t nc, const int64_t *__restrict__ mptr,
                                                    const int32_t *__restrict__ mem, const int64_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ col, const double *__restrict__ val,
                                                    const int32_t *__restrict__ agg, const int64_t *__restrict__ crow,
                                                    const int32_t *__restrict__ ccol, double *__restrict__ cval) {
    __shared__ double acc_s[GAL_REG * 64];
    __shared__ int32_t cj_s[GAL_REG * 64];
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    const int t = threadIdx.x;
    int64_t a = crow[I], b = crow[I + 1];
    int len = (int)(b - a);
    if (len <= GAL_REG) {
        for (int e = 0; e < len; e++) {
            cj_s[e * 64 + t] = ccol[a + e];
            acc_s[e * 64 + t] = 0.0;
        }
        for (int64_t q = mptr[I]; q < mptr[I + 1]; q++) {
            int32_t i = mem[q];
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
                int32_t J = agg[col[e]];
                int lo = 0, hi = len - 1;
                while (lo < hi) {
                    int mid = (lo + hi) >> 1;
                    if (cj_s[mid * 64 + t] < J) lo = mid + 1;
                    else hi = mid;
                }
                acc_s[lo * 64 + t] += val[e];
            }
        }
        for (int e = 0; e < len; e++) cval[a + e] = acc_s[e * 64 + t];
        return;
    }
    for (int64_t e = a; e < b; e++) cval[e] = 0.0;
    for (int64_t q = mptr[I]; q < mptr[I + 1]; q++) {
        int32_t i = mem[q];
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
            int32_t J = agg[col[e]];
            int64_t lo = a, hi = b - 1;
            while (lo < hi) {
                int64_t mid = (lo + hi) >> 1;
                if (ccol[mid] < J) lo = mid + 1;
                else hi = mid;
            }
            cval[lo] += val[e];
        }
    }
}

__global__ void k_csr_invd(int64_t n, const int64_t *__restrict__ rowptr, const double *__restrict__ val,
                           double *__restrict__ invd, float *__restrict__ invdf) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) s += fabs(val[e]);
    if (invd) invd[i] = 1.0 / s;
    if (invdf) invdf[i] = f32_sat(1.0 / s);
}

__global__ void k_compose(int64_t n, int32_t *__restrict__ comp, const int32_t *__restrict__ a) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) comp[i] = a[comp[i]];
}

__global__ void k_iota(int64_t n, int32_t *__restrict__ x) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = (int32_t)i;
}

// ----------------------------------------------------- V-cycle, CSR levels
// Rows are processed by groups of G lanes (4 or 8, by the level's mean row
// length) that stride over the row's entries; the group sum is formed with
// shuffles in a fixed lane order.

// pre-smoothing from zero and residual: x0 = D^{-1} b (stored by the
// restriction that produced b), r = b - A x0
template <int G, class TB, class T>
__global__ void k_csr_pre(int64_t n, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                          const T *__restrict__ val, const T *__restrict__ x0, const TB *__restrict__ b,
                          T *__restrict__ r) {
    int64_t row = ((int64_t)xcd_block() * blockDim.x + threadIdx.x) / G;
    int lane = threadIdx.x % G;
    if (row >= n) return;
    T s = 0;
    for (int64_t e = rowptr[row] + lane; e < rowptr[row + 1]; e += G) s += val[e] * x0[col[e]];
    s = group_sum<G>(s);
    if (lane == 0) r[row] = (T)b[row] - s;
}

// prolongation: xt = x0 + P xc
template <class T>
__device__ __forceinline__ void csr_prolong_at(int64_t n, const T *__restrict__ x0, const T *__restrict__ xc,
                                               const int32_t *__restrict__ agg, T *__restrict__ xt, int64_t row) {
    if (row >= n) return;
    xt[row] = x0[row] + xc[agg[row]];
}

template <class T>
__global__ void k_csr_prolong(int64_t n, const T *__restrict__ x0, const T *__restrict__ xc,
                              const int32_t *__restrict__ agg, T *__restrict__ xt) {
    csr_prolong_at(n, x0, xc, agg, xt, (int64_t)xcd_block() * blockDim.x + threadIdx.x);
}

// post-smoothing: x = xt + D^{-1}(b - A xt)
template <int G, class TB, class T>
__global__ void k_csr_post(int64_t n, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                           const T *__restrict__ val, const T *__restrict__ invd, const TB *__restrict__ b,
                           const T *__restrict__ xt, T *__restrict__ x) {
    int64_t row = ((int64_t)xcd_block() * blockDim.x + threadIdx.x) / G;
    int lane = threadIdx.x % G;
    if (row >= n) return;
    T s = 0;
    for (int64_t e = rowptr[row] + lane; e < rowptr[row + 1]; e += G) s += val[e] * xt[col[e]];
    s = group_sum<G>(s);
    if (lane == 0) x[row] = xt[row] + invd[row] * ((T)b[row] - s);
}

template <int G, class TB, class T>
__global__ void k_csr_sweep(int64_t n, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                            const T *__restrict__ val, const T *__restrict__ invd, const TB *__restrict__ b,
                            const T *__restrict__ xin, T *__restrict__ xout, int zero) {
    int64_t row = ((int64_t)xcd_block() * blockDim.x + threadIdx.x) / G;
    int lane = threadIdx.x % G;
    if (row >= n) return;
    if (zero) {
        if (lane == 0) xout[row] = (T)b[row] * invd[row];
        return;
    }
    T s = 0;
    for (int64_t e = rowptr[row] + lane; e < rowptr[row + 1]; e += G) s += val[e] * xin[col[e]];
    s = group_sum<G>(s);
    if (lane == 0) xout[row] = xin[row] + invd[row] * ((T)b[row] - s);
}

// ------------------------------------------------ CSR-stream levels
// A block takes a run of whole rows holding at most STREAM_CHUNK +
// STREAM_MAXROW - 1 entries: its threads first form the products of all the
// run's entries in entry order (coalesced loads, neighbouring gathers) into
// LDS, then one thread per row adds its row's products in order.
constexpr int STREAM_LDS = STREAM_CHUNK + STREAM_MAXROW;
// PRE: v = x0, out = b - A x0;  POST: v = xt, out = xt + D^{-1}(b - A xt).
// G lanes add up a row.
template <int G, class TB, class T, bool POST>
__device__ __forceinline__ void csr_stream_body(const int64_t *__restrict__ rb, const int64_t *__restrict__ rowptr,
                                                const int32_t *__restrict__ col, const T *__restrict__ val,
                                                const T *__restrict__ invd, const TB *__restrict__ b,
                                                const T *__restrict__ v, T *__restrict__ out, int64_t blk) {
    constexpr int PER = STREAM_LDS / 256;  // entries per thread in the product phase
    __shared__ T prod[STREAM_LDS];
    // the block's first and end rows and their first entries, read together,
    // so that the entry loads below need not wait for the row pointers
    int64_t r0 = rb[2 * blk], r1 = rb[2 * blk + 2];
    if (r0 >= r1) return;
    int64_t e0 = rb[2 * blk + 1], e1 = rb[2 * blk + 3];
    // the reduction phase's first row pointers are loaded ahead of the products
    const int lane = threadIdx.x % G;
    int64_t row0 = r0 + threadIdx.x / G;
    int64_t ra = row0 < r1 ? rowptr[row0] : 0, rbe = row0 < r1 ? rowptr[row0 + 1] : 0;
    // the row's b, D^{-1} and v of the final update, loaded with its row
    // pointers so that the write after the group sum does not wait for them
    T pb = 0, pd = 0, pv = 0;
    auto row_in = [&](int64_t row) {
        if (row < r1) {
            pb = (T)b[row];
            if (POST) {
                pd = invd[row];
                pv = v[row];
            }
        }
    };
    row_in(row0);
    // every load of the product phase is issued before the first use
    int32_t cj[PER];
    T vv[PER];
#pragma unroll
    for (int q = 0; q < PER; q++) {
        int64_t e = e0 + threadIdx.x + 256 * q;
        // the matrix entries are read once per sweep: streamed past the caches
        cj[q] = e < e1 ? __builtin_nontemporal_load(col + e) : 0;
        vv[q] = e < e1 ? __builtin_nontemporal_load(val + e) : (T)0;
    }
    T xs[PER];
#pragma unroll
    for (int q = 0; q < PER; q++) xs[q] = v[cj[q]];
#pragma unroll
    for (int q = 0; q < PER; q++) {
        int64_t e = e0 + threadIdx.x + 256 * q;
        if (e < e1) prod[e - e0] = vv[q] * xs[q];
    }
    __syncthreads();
    // every lane of a group runs the same number of row iterations (shuffles)
    for (int64_t rbase = r0; rbase < r1; rbase += blockDim.x / G) {
        int64_t row = rbase + threadIdx.x / G;
        if (rbase != r0) {
            ra = row < r1 ? rowptr[row] : 0;
            rbe = row < r1 ? rowptr[row + 1] : 0;
            row_in(row);
        }
        T s = 0;
        if (row < r1)
            for (int64_t e = ra + lane; e < rbe; e += G) s += prod[e - e0];
        s = group_sum<G>(s);
        if (lane == 0 && row < r1) {
            if (POST) out[row] = pv + pd * (pb - s);
            else out[row] = pb - s;
        }
    }
}

template <int G, class TB, class T, bool POST>
__global__ void __launch_bounds__(256) k_csr_stream(const int64_t *__restrict__ rb, const int64_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ col, const T *__restrict__ val,
                                                    const T *__restrict__ invd, const TB *__restrict__ b,
                                                    const T *__restrict__ v, T *__restrict__ out) {
    csr_stream_body<G, TB, T, POST>(rb, rowptr, col, val, invd, b, v, out, xcd_block());
}

// rb[2b] = first row whose first entry is at or past b * STREAM_CHUNK and
// rb[2b + 1] = that row's first entry; the blocks past the last chunk (grid
// padding) are empty
__global__ void k_stream_rb(int64_t n, int64_t nrb, int64_t ngrid, const int64_t *__restrict__ rowptr,
                            int64_t *__restrict__ rb) {
    int64_t blk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (blk > ngrid) return;
    int64_t lo = n;
    if (blk < nrb) {
        int64_t target = blk * (int64_t)STREAM_CHUNK, hi = n;
        lo = 0;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (rowptr[mid] < target) lo = mid + 1;
            else hi = mid;
        }
    }
    rb[2 * blk] = lo;
    rb[2 * blk + 1] = rowptr[lo];
}

__global__ void k_max_rowlen(int64_t n, const int64_t *__restrict__ rowptr, int *__restrict__ too_long) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && rowptr[i + 1] - rowptr[i] > STREAM_MAXROW) too_long[0] = 1;
}

// bc[I] = sum over the members of I (ascending) of r
// (and x0c[I] = D_c^{-1} bc[I], the coarse pre-smoothed iterate, when x0c is set)
// A block of RESTRICT_TPB threads takes RESTRICT_TPB consecutive coarse rows:
// their member lists are one contiguous stretch of mem, which the block reads
// with coalesced loads, gathering the r values into LDS in member order; each
// thread then adds its row's values in that order (the same sums as a thread
// walking its list alone).  A stretch longer than the LDS falls back to the
// per-thread walk.
constexpr int RESTRICT_TPB = 256, RESTRICT_LDS = 2048;
template <class T>
__device__ __forceinline__ void restrict_block(int64_t nc, const int64_t *__restrict__ mptr,
                                               const int32_t *__restrict__ mem, const T *__restrict__ r,
                                               T *__restrict__ bc, const T *__restrict__ invdc,
                                               T *__restrict__ x0c, int64_t blk) {
    __shared__ T rv[RESTRICT_LDS];
    const int64_t I0 = blk * RESTRICT_TPB;
    if (I0 >= nc) return;
    const int64_t I1 = I0 + RESTRICT_TPB < nc ? I0 + RESTRICT_TPB : nc;
    const int64_t I = I0 + threadIdx.x;
    const int64_t t0 = mptr[I0], t1 = mptr[I1];
    const bool staged = t1 - t0 <= RESTRICT_LDS;
    // the thread's own row bounds are loaded before the staging, which issues
    // all its member-index loads, then all its gathers (a gather waiting for
    // its index one at a time would serialise eight round trips to memory);
    // a slot past the stretch reads member t0 and is not stored
    const int64_t a = I < nc ? mptr[I] : 0, e = I < nc ? mptr[I + 1] : 0;
    if (staged && t1 > t0) {
        constexpr int PER = RESTRICT_LDS / RESTRICT_TPB;
        int32_t m[PER];
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int64_t t = t0 + threadIdx.x + (int64_t)q * RESTRICT_TPB;
            // the member lists are read once per cycle: streamed past the caches
            m[q] = __builtin_nontemporal_load(mem + (t < t1 ? t : t0));
        }
        T x[PER];
#pragma unroll
        for (int q = 0; q < PER; q++) x[q] = r[m[q]];
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int64_t t = t0 + threadIdx.x + (int64_t)q * RESTRICT_TPB;
            if (t < t1) rv[t - t0] = x[q];
        }
        __syncthreads();
    }
    if (I >= nc) return;
    T s = 0;
    if (staged)
        for (int64_t t = a; t < e; t++) s += rv[t - t0];
    else
        for (int64_t t = a; t < e; t++) s += r[mem[t]];
    bc[I] = s;
    if (x0c) x0c[I] = s * invdc[I];
}

template <class T>
__global__ void __launch_bounds__(RESTRICT_TPB) k_restrict(int64_t nc, const int64_t *__restrict__ mptr,
                                                           const int32_t *__restrict__ mem, const T *__restrict__ r,
                                                           T *__restrict__ bc, const T *__restrict__ invdc,
                                                           T *__restrict__ x0c) {
    restrict_block(nc, mptr, mem, r, bc, invdc, x0c, xcd_block());
}

// x = Ainv b, one wavefront per row (row-major Ainv)
template <class TB, class T>
__device__ __forceinline__ void dense_gemv_at(const T *__restrict__ Ainv, const TB *__restrict__ b,
                                              T *__restrict__ x, int64_t n, int64_t blk) {
    int64_t row = (blk * blockDim.x + threadIdx.x) / 64;
    int lane = threadIdx.x % 64;
    if (row >= n) return;
    // four independent partial sums per lane keep four row segments in flight
    const T *__restrict__ a = Ainv + row * n;
    T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    int64_t j = lane;
    for (; j + 192 < n; j += 256) {
        s0 += a[j] * (T)b[j];
        s1 += a[j + 64] * (T)b[j + 64];
        s2 += a[j + 128] * (T)b[j + 128];
        s3 += a[j + 192] * (T)b[j + 192];
    }
    for (; j < n; j += 64) s0 += a[j] * (T)b[j];
    T s = (s0 + s1) + (s2 + s3);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (lane == 0) x[row] = s;
}

template <class TB, class T>
__global__ void k_dense_gemv(const T *__restrict__ Ainv, const TB *__restrict__ b, T *__restrict__ x, int64_t n) {
    dense_gemv_at(Ainv, b, x, n, blockIdx.x);
}

// ---------------------------------------- batched coarse-level launches
// The coarse-level V-cycle kernels over several simulations at once (same
// per-block code as the lone launches above).
template <class T>
struct CoarseArgs {
    int64_t n;
    const int64_t *rb, *rowptr;
    const int32_t *col;
    const T *val, *invd, *b, *v;
    T *out;
    const int32_t *agg;  // prolongation / restriction maps
    const int64_t *mptr;
    const int32_t *mem;
    T *x0c;
};

// MODE 0: restriction (b = r, out = bc, invd = invdc), 1: prolongation
// xt = x0 + P xc (b = x0, v = xc, out = xt), 2: dense coarsest product
// (val = Ainv, b = bc, out = x)
template <class T, int MODE>
__global__ void k_coarse_batch(Batch<CoarseArgs<T>> B) {
    for_each_block(B, MODE == 2 ? blockIdx.x : xcd_block(), [&](unsigned L) {
        const int e = batch_entry(B, L);
        const CoarseArgs<T> &a = B.a[e];
        const int64_t blk = (int64_t)(L - B.begin[e]);
        if (MODE == 0) restrict_block(a.n, a.mptr, a.mem, a.b, a.out, a.invd, a.x0c, blk);
        if (MODE == 1) csr_prolong_at(a.n, a.b, a.v, a.agg, a.out, blk * blockDim.x + threadIdx.x);
        if (MODE == 2) dense_gemv_at(a.val, a.b, a.out, a.n, blk);
    });
}

template <int G, class T, bool POST>
__global__ void __launch_bounds__(256) k_csr_stream_batch(Batch<CoarseArgs<T>> B) {
    for_each_block(B, xcd_block(), [&](unsigned L) {
        const int e = batch_entry(B, L);
        const CoarseArgs<T> &a = B.a[e];
        csr_stream_body<G, T, T, POST>(a.rb, a.rowptr, a.col, a.val, a.invd, a.b, a.v, a.out, L - B.begin[e]);
    });
}

__global__ void k_csr_spmv(int64_t n, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                           const double *__restrict__ val, const double *__restrict__ x, double *__restrict__ y) {
    int64_t row = ((int64_t)xcd_block() * blockDim.x + threadIdx.x) / 8;
    int lane = threadIdx.x % 8;
    if (row >= n) return;
    double s = 0;
    for (int64_t e = rowptr[row] + lane; e < rowptr[row + 1]; e += 8) s += val[e] * x[col[e]];
    s = group_sum<8>(s);
    if (lane == 0) y[row] = s;
}

// ----------------------------------------------- dense coarsest inverse
__global__ void k_csr_to_dense(int64_t n, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                               const double *__restrict__ val, double *__restrict__ D) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) D[i * n + col[e]] = val[e];
}

// Blocked Gauss-Jordan inversion of an SPD matrix (no pivoting: every
// leading block of an SPD matrix and every Schur complement stay SPD).  For
// the pivot block K = [k0, k0+b):  P = D_KK,  R_K: = P^{-1} D_K: (with P^{-1}
// itself in the K columns),  S_:K = D_:K (old), then
//   D_ij <- R_{i-k0, j}                                  for i in K,
//   D_ij <- [j not in K] D_ij - sum_t S_it R_tj          otherwise.
constexpr int GJB = 64;  // pivot block

// P^{-1} by scalar Gauss-Jordan in LDS (one workgroup, b <= 64).  The block
// is padded to 64 x 64 with the identity (its inverse is then diag(P^{-1}, I)),
// each of the 1024 threads owns four fixed entries, and the block is
// double-buffered so that one barrier per pivot suffices.
__global__ void __launch_bounds__(1024) k_bgj_pivot(const double *__restrict__ D, int64_t n, int64_t k0, int b,
                                                    double *__restrict__ Pinv, int *__restrict__ bad) {
    __shared__ double A[2][GJB][GJB + 1];
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        int t = tid + 1024 * q, i = t >> 6, j = t & 63;
        A[0][i][j] = (i < b && j < b) ? D[(k0 + i) * n + k0 + j] : (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    int cur = 0;
    for (int k = 0; k < b; k++, cur ^= 1) {
        double p = A[cur][k][k];
        if (!(p > 0.0)) {
            if (tid == 0) *bad = 1;
            p = 1.0;  // keep going; the caller reports the failure
        }
        const double ip = 1.0 / p;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            int t = tid + 1024 * q, i = t >> 6, j = t & 63;
            double v;
            if (i == k) v = (j == k) ? ip : A[cur][k][j] * ip;
            else if (j == k) v = -A[cur][i][k] * ip;
            else v = A[cur][i][j] - A[cur][i][k] * ip * A[cur][k][j];
            A[cur ^ 1][i][j] = v;
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
        int t = tid + 1024 * q, i = t >> 6, j = t & 63;
        if (i < b && j < b) Pinv[i * GJB + j] = A[cur][i][j];
    }
}

// R (b x n): one thread per entry, blockIdx.y = row r of the pivot block.
__global__ void k_bgj_panel_R(const double *__restrict__ D, int64_t n, int64_t k0, int b,
                              const double *__restrict__ Pinv, double *__restrict__ R) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int r = blockIdx.y;
    if (j >= n || r >= b) return;
    double v;
    if (j >= k0 && j < k0 + b) {
        v = Pinv[r * GJB + (j - k0)];
    } else {
        v = 0.0;
        for (int t = 0; t < b; t++) v += Pinv[r * GJB + t] * D[(k0 + t) * n + j];
    }
    R[(int64_t)r * n + j] = v;
}

// S (n x GJB): the old column block, one thread per entry.
__global__ void k_bgj_panel_S(const double *__restrict__ D, int64_t n, int64_t k0, int b, double *__restrict__ S) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * GJB) return;
    int64_t j = t / GJB;
    int c = (int)(t - j * GJB);
    if (c < b) S[t] = D[j * n + k0 + c];
}

// Rank-b update on 64x64 tiles with FP64 matrix cores: the four wavefronts of
// a block each own 16 rows of the tile and accumulate four 16x16 blocks with
// v_mfma_f64_16x16x4f64 over the (zero-padded) 64-long inner dimension.
// Operand layout of that instruction: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; result register v of lane l is D[l/16 + 4v][l%16].
typedef double rich_d4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_bgj_update(double *__restrict__ D, int64_t n, int64_t k0, int b,
                                                     const double *__restrict__ R, const double *__restrict__ S) {
    __shared__ double Ss[GJB][GJB + 1];  // [row in tile][t]
    __shared__ double Rs[GJB][GJB + 1];  // [t][col in tile]
    int64_t i0 = (int64_t)blockIdx.y * GJB, j0 = (int64_t)blockIdx.x * GJB;
    for (int t = threadIdx.x; t < GJB * GJB; t += blockDim.x) {
        int r = t / GJB, c = t - r * GJB;
        int64_t gi = i0 + r, gj = j0 + c;
        Ss[r][c] = (gi < n && c < b) ? S[gi * GJB + c] : 0.0;
        Rs[r][c] = (r < b && gj < n) ? R[(int64_t)r * n + gj] : 0.0;
    }
    __syncthreads();
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    const int li = l % 16, lk = l / 16;
    rich_d4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; c++) acc[c] = (rich_d4){0.0, 0.0, 0.0, 0.0};
    for (int t = 0; t < GJB; t += 4) {
        double a = Ss[16 * w + li][t + lk];
#pragma unroll
        for (int c = 0; c < 4; c++) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Rs[t + lk][16 * c + li], acc[c], 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < 4; c++) {
        int64_t gj = j0 + 16 * c + li;
        if (gj >= n) continue;
        bool colK = gj >= k0 && gj < k0 + b;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            int64_t gi = i0 + 16 * w + lk + 4 * v;
            if (gi >= n) continue;
            bool rowK = gi >= k0 && gi < k0 + b;
            double out;
            if (rowK) out = R[(gi - k0) * n + gj];
            else out = (colK ? 0.0 : D[gi * n + gj]) - acc[c][v];
            D[gi * n + gj] = out;
        }
    }
}

}  // namespace

// ------------------------------------------------------------------ host
namespace {
size_t ws_round(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

size_t match_ws_bytes(int64_t n, int64_t nnz) {
    const size_t un = (size_t)(n > 0 ? n : 1);
    return ws_round(un * 8) + ws_round((size_t)(nnz > 0 ? nnz : 1) * 8) + 2 * ws_round(un * 4) +
           ws_round(un * 8) + ws_round((un + 1) * 8) + ws_round((size_t)scan_tmp_size(n) * 8) + ws_round(4);
}

MatchWs match_ws_carve(void *base, int64_t n, int64_t nnz) {
    const size_t un = (size_t)(n > 0 ? n : 1);
    char *p = static_cast<char *>(base);
    MatchWs w;
    auto take = [&](size_t b) {
        char *q = p;
        p += ws_round(b);
        return q;
    };
    w.diag = (double *)take(un * 8);
    w.wts = (double *)take((size_t)(nnz > 0 ? nnz : 1) * 8);
    w.mate = (int32_t *)take(un * 4);
    w.cand = (int32_t *)take(un * 4);
    w.flag = (int64_t *)take(un * 8);
    w.id = (int64_t *)take((un + 1) * 8);
    w.stmp = (int64_t *)take((size_t)scan_tmp_size(n) * 8);
    w.still = (int32_t *)take(4);
    return w;
}

rich_status match_sweep_ws(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, int32_t *agg,
                           int64_t *nc_out, const MatchWs &w, int *h_still, hipStream_t s) {
    if (n == 0) {
        *nc_out = 0;
        return RICH_OK;
    }
    k_diag<<<nblocks(n), TPB, 0, s>>>(n, rowptr, col, val, w.diag);
    LAUNCH_CHECK();
    // the weights do not change between rounds: computed once
    k_match_weights<<<nblocks(n), TPB, 0, s>>>(n, rowptr, col, val, w.diag, w.wts);
    LAUNCH_CHECK();
    RICH_TRY(launch_fill_i32(w.mate, -1, n, s));
    for (int64_t round = 0;; round++) {
        RICH_TRY(launch_fill_i32(w.still, 0, 1, s));
        // a few rounds per host check; extra rounds after completion are no-ops
        for (int t = 0; t < 4; t++) {
            k_candidates<<<nblocks(n), TPB, 0, s>>>(n, rowptr, col, w.wts, w.mate, w.cand);
            k_commit<<<nblocks(n), TPB, 0, s>>>(n, w.cand, w.mate, w.still);
        }
        LAUNCH_CHECK();
        HIP_TRY(hipMemcpyAsync(h_still, w.still, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (!*h_still) break;
        if (round > 4 * n + 16) return RICH_EHIP;  // every round matches or retires at least one vertex
    }
    k_leaders<<<nblocks(n), TPB, 0, s>>>(n, w.mate, w.flag);
    LAUNCH_CHECK();
    RICH_TRY(scan_exclusive_i64(w.flag, w.id, n, w.stmp, s));
    k_number<<<nblocks(n), TPB, 0, s>>>(n, w.mate, w.id, agg);
    LAUNCH_CHECK();
    int64_t nc = 0;
    HIP_TRY(hipMemcpyAsync(&nc, w.id + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *nc_out = nc;
    return RICH_OK;
}

rich_status match_sweep(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, int32_t *agg,
                        int64_t *nc_out, hipStream_t s) {
    if (n == 0) {
        *nc_out = 0;
        return RICH_OK;
    }
    int64_t nnz = 0;
    HIP_TRY(hipMemcpyAsync(&nnz, rowptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    DevAlloc tmp;
    char *base;
    RICH_TRY(tmp.get(&base, match_ws_bytes(n, nnz)));
    int *h_still = nullptr;
    HIP_TRY(hipHostMalloc((void **)&h_still, sizeof(int)));
    rich_status st = match_sweep_ws(n, rowptr, col, val, agg, nc_out, match_ws_carve(base, n, nnz), h_still, s);
    (void)hipHostFree(h_still);
    return st;
}

rich_status vmb_aggregate(const CsrDev &A, double theta, int64_t block, int32_t *agg, int64_t *nc_out,
                          hipStream_t s) {
    *nc_out = 0;
    if (A.n == 0) return RICH_OK;
    const int64_t nblk = (A.n + block - 1) / block;
    DevAlloc tmp;
    double *diag;
    int32_t *p1;
    int64_t *cnt, *off, *stmp;
    RICH_TRY(tmp.get(&diag, A.n));
    RICH_TRY(tmp.get(&p1, A.n));
    RICH_TRY(tmp.get(&cnt, nblk + 1));
    RICH_TRY(tmp.get(&off, nblk + 1));
    RICH_TRY(tmp.get(&stmp, scan_tmp_size(nblk + 1)));
    k_row_diag<<<nblocks(A.n), TPB, 0, s>>>(A.n, A.rowptr, A.col, A.val, diag);
    LAUNCH_CHECK();
    HIP_TRY(hipMemsetAsync(cnt, 0, (nblk + 1) * sizeof(int64_t), s));
    k_vmb_block<<<(unsigned)((nblk + 63) / 64), 64, 0, s>>>(A.n, block, nblk, A.rowptr, A.col, A.val, diag, theta,
                                                             agg, p1, cnt);
    LAUNCH_CHECK();
    RICH_TRY(scan_exclusive_i64(cnt, off, nblk + 1, stmp, s));  // off[nblk] = total
    k_vmb_offset<<<nblocks(A.n), TPB, 0, s>>>(A.n, block, off, agg);
    LAUNCH_CHECK();
    HIP_TRY(hipMemcpyAsync(nc_out, off + nblk, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));  // tmp is freed on return
    return RICH_OK;
}

rich_status members(const int32_t *agg, int64_t n, int64_t nc, int64_t *mptr, int32_t *mem, hipStream_t s) {
    DevAlloc tmp;
    int64_t *cnt, *stmp;
    unsigned int *cursor;
    RICH_TRY(tmp.get(&cnt, nc));
    RICH_TRY(tmp.get(&cursor, nc));
    RICH_TRY(tmp.get(&stmp, scan_tmp_size(nc)));
    HIP_TRY(hipMemsetAsync(cnt, 0, nc * sizeof(int64_t), s));
    HIP_TRY(hipMemsetAsync(cursor, 0, nc * sizeof(unsigned int), s));
    if (n > 0) {
        k_count_members<<<nblocks(n), TPB, 0, s>>>(n, agg, cnt);
        LAUNCH_CHECK();
    }
    RICH_TRY(scan_exclusive_i64(cnt, mptr, nc, stmp, s));
    if (n > 0) {
        k_place_members<<<nblocks(n), TPB, 0, s>>>(n, agg, mptr, cursor, mem);
        LAUNCH_CHECK();
    }
    if (nc > 0) {
        k_sort_members<<<nblocks(nc), TPB, 0, s>>>(nc, mptr, mem);
        LAUNCH_CHECK();
    }
    HIP_TRY(hipStreamSynchronize(s));  // tmp is freed on return
    return RICH_OK;
}

rich_status galerkin_symbolic(const CsrDev &A, const int32_t *agg, int64_t nc, const int64_t *mptr,
                              const int32_t *mem, CsrDev *C, DevAlloc &mem_out, hipStream_t s) {
    DevAlloc tmp;
    int64_t *seg, *segptr, *cnt, *stmp;
    int32_t *scratch;
    RICH_TRY(tmp.get(&seg, nc));
    RICH_TRY(tmp.get(&segptr, nc + 1));
    RICH_TRY(tmp.get(&cnt, nc));
    RICH_TRY(tmp.get(&stmp, scan_tmp_size(nc)));
    RICH_TRY(tmp.get(&scratch, A.nnz));
    C->n = nc;
    RICH_TRY(mem_out.get(&C->rowptr, nc + 1));
    if (nc > 0) {
        k_seg_len<<<nblocks(nc), TPB, 0, s>>>(nc, mptr, mem, A.rowptr, seg);
        LAUNCH_CHECK();
    }
    RICH_TRY(scan_exclusive_i64(seg, segptr, nc, stmp, s));
    if (nc > 0) {
        k_sym_collect<<<nblocks(nc, 64), 64, 0, s>>>(nc, mptr, mem, A.rowptr, A.col, agg, segptr, scratch, cnt);
        LAUNCH_CHECK();
    }
    RICH_TRY(scan_exclusive_i64(cnt, C->rowptr, nc, stmp, s));
    int64_t nnz = 0;
    HIP_TRY(hipMemcpyAsync(&nnz, C->rowptr + nc, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    C->nnz = nnz;
    RICH_TRY(mem_out.get(&C->col, nnz));
    RICH_TRY(mem_out.get(&C->val, nnz));
    if (nc > 0) {
        k_sym_write<<<nblocks(nc), TPB, 0, s>>>(nc, segptr, scratch, C->rowptr, C->col);
        LAUNCH_CHECK();
    }
    HIP_TRY(hipStreamSynchronize(s));  // tmp is freed on return
    return RICH_OK;
}

rich_status galerkin_numeric(const CsrDev &A, const int32_t *agg, const int64_t *mptr, const int32_t *mem,
                             const CsrDev &C, hipStream_t s) {
    if (C.n == 0) return RICH_OK;
    k_gal_numeric<<<nblocks(C.n, 64), 64, 0, s>>>(C.n, mptr, mem, A.rowptr, A.col, A.val, agg, C.rowptr, C.col,
                                                  C.val);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status galerkin(const CsrDev &A, const int32_t *agg, int64_t nc, CsrDev *C, DevAlloc &mem_out,
                     hipStream_t s) {
    DevAlloc tmp;
    int64_t *mptr;
    int32_t *mem;
    RICH_TRY(tmp.get(&mptr, nc + 1));
    RICH_TRY(tmp.get(&mem, A.n));
    RICH_TRY(members(agg, A.n, nc, mptr, mem, s));
    RICH_TRY(galerkin_symbolic(A, agg, nc, mptr, mem, C, mem_out, s));
    RICH_TRY(galerkin_numeric(A, agg, mptr, mem, *C, s));
    HIP_TRY(hipStreamSynchronize(s));
    return RICH_OK;
}

rich_status stream_blocks(Level &Lv, DevAlloc &mem, hipStream_t s) {
    if (Lv.n == 0) return RICH_OK;
    DevAlloc tmp;
    int *flag;
    RICH_TRY(tmp.get(&flag, 1));
    HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), s));
    k_max_rowlen<<<nblocks(Lv.n), TPB, 0, s>>>(Lv.n, Lv.rowptr, flag);
    LAUNCH_CHECK();
    int too_long = 0;
    HIP_TRY(hipMemcpyAsync(&too_long, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (too_long) return RICH_OK;
    int64_t nrb = (Lv.nnz + STREAM_CHUNK - 1) / STREAM_CHUNK;
    // lanes per row in the reduction phase, by the mean row length
    int64_t mean = Lv.nnz / Lv.n;
    Lv.sg = mean < 8 ? 1 : mean < 16 ? 2 : mean < 32 ? 4 : 8;
    // the launch grid is rounded up to a multiple of the XCD count: pad with empty blocks
    int64_t ngrid = xcd_grid(nrb, 1);
    RICH_TRY(mem.get(&Lv.rb, 2 * (ngrid + 1)));
    k_stream_rb<<<nblocks(ngrid + 1), TPB, 0, s>>>(Lv.n, nrb, ngrid, Lv.rowptr, Lv.rb);
    LAUNCH_CHECK();
    Lv.nrb = ngrid;
    HIP_TRY(hipStreamSynchronize(s));  // tmp is freed on return
    return RICH_OK;
}

rich_status csr_invd(const CsrDev &A, double *invd, float *invdf, hipStream_t s) {
    if (A.n == 0) return RICH_OK;
    k_csr_invd<<<nblocks(A.n), TPB, 0, s>>>(A.n, A.rowptr, A.val, invd, invdf);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status compose_agg(int32_t *comp, const int32_t *a, int64_t n, hipStream_t s) {
    if (n == 0) return RICH_OK;
    if (a == nullptr) {
        k_iota<<<nblocks(n), TPB, 0, s>>>(n, comp);
    } else {
        k_compose<<<nblocks(n), TPB, 0, s>>>(n, comp, a);
    }
    LAUNCH_CHECK();
    return RICH_OK;
}

// Inverse of an SPD CSR matrix into a dense row-major n x n buffer, using
// the workspace of dense_inverse_ws (no allocation: it runs on every refresh).
int64_t dense_inverse_ws(int64_t n) { return (int64_t)GJB * GJB + 2 * (int64_t)GJB * n + 1; }

rich_status dense_inverse(const CsrDev &A, double *D, double *ws, hipStream_t s) {
    int64_t n = A.n;
    if (n == 0) return RICH_OK;
    double *Pinv = ws, *R = ws + GJB * GJB, *S = R + (int64_t)GJB * n;
    int *bad = reinterpret_cast<int *>(S + (int64_t)GJB * n);
    HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int), s));
    HIP_TRY(hipMemsetAsync(D, 0, (size_t)n * n * sizeof(double), s));
    k_csr_to_dense<<<nblocks(n), TPB, 0, s>>>(n, A.rowptr, A.col, A.val, D);
    LAUNCH_CHECK();
    unsigned tiles = (unsigned)((n + GJB - 1) / GJB);
    for (int64_t k0 = 0; k0 < n; k0 += GJB) {
        int b = (int)std::min<int64_t>(GJB, n - k0);
        k_bgj_pivot<<<1, 1024, 0, s>>>(D, n, k0, b, Pinv, bad);
        k_bgj_panel_R<<<dim3(nblocks(n), b), TPB, 0, s>>>(D, n, k0, b, Pinv, R);
        k_bgj_panel_S<<<nblocks(n * GJB), TPB, 0, s>>>(D, n, k0, b, S);
        k_bgj_update<<<dim3(tiles, tiles), 256, 0, s>>>(D, n, k0, b, R, S);
    }
    LAUNCH_CHECK();
    int hb = 0;
    HIP_TRY(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return hb ? RICH_NOT_SPD : RICH_OK;
}

// lanes per row: 4 for short rows, 8 otherwise
static inline bool short_rows(const Level &Lv) { return Lv.nnz < 16 * Lv.n; }

template <class TB, class T, bool POST>
void launch_stream(const Level &Lv, const T *val, const T *invd, const TB *b, const T *v, T *out, hipStream_t s) {
    unsigned g = (unsigned)Lv.nrb;
    switch (Lv.sg) {
    case 1: k_csr_stream<1, TB, T, POST><<<g, 256, 0, s>>>(Lv.rb, Lv.rowptr, Lv.col, val, invd, b, v, out); break;
    case 2: k_csr_stream<2, TB, T, POST><<<g, 256, 0, s>>>(Lv.rb, Lv.rowptr, Lv.col, val, invd, b, v, out); break;
    case 4: k_csr_stream<4, TB, T, POST><<<g, 256, 0, s>>>(Lv.rb, Lv.rowptr, Lv.col, val, invd, b, v, out); break;
    default: k_csr_stream<8, TB, T, POST><<<g, 256, 0, s>>>(Lv.rb, Lv.rowptr, Lv.col, val, invd, b, v, out); break;
    }
}

template <class TB, class T>
rich_status launch_csr_pre(const Level &Lv, const T *val, const T *x0, const TB *b, T *r, hipStream_t s) {
    if (Lv.n == 0) return RICH_OK;
    if (Lv.rb) {
        launch_stream<TB, T, false>(Lv, val, nullptr, b, x0, r, s);
        LAUNCH_CHECK();
        return RICH_OK;
    }
    if (short_rows(Lv))
        k_csr_pre<4, TB, T><<<xcd_grid(Lv.n * 4, TPB), TPB, 0, s>>>(Lv.n, Lv.rowptr, Lv.col, val, x0, b, r);
    else
        k_csr_pre<8, TB, T><<<xcd_grid(Lv.n * 8, TPB), TPB, 0, s>>>(Lv.n, Lv.rowptr, Lv.col, val, x0, b, r);
    LAUNCH_CHECK();
    return RICH_OK;
}

template <class TB, class T>
rich_status launch_csr_post(const Level &Lv, const T *val, const T *invd, const TB *b, const T *x0, const T *xc,
                            T *x, hipStream_t s) {
    if (Lv.n == 0) return RICH_OK;
    T *xt = (T *)Lv.r;  // the residual of this level is dead by now
    if (Lv.prow) {
        RICH_TRY(launch_sa_prolong<TB, T>(Lv, invd, b, nullptr, x0, xc, xt, s));
    } else {
        k_csr_prolong<T><<<xcd_grid(Lv.n, TPB), TPB, 0, s>>>(Lv.n, x0, xc, Lv.agg, xt);
        LAUNCH_CHECK();
    }
    if (Lv.rb)
        launch_stream<TB, T, true>(Lv, val, invd, b, xt, x, s);
    else if (short_rows(Lv))
        k_csr_post<4, TB, T><<<xcd_grid(Lv.n * 4, TPB), TPB, 0, s>>>(Lv.n, Lv.rowptr, Lv.col, val, invd, b, xt, x);
    else
        k_csr_post<8, TB, T><<<xcd_grid(Lv.n * 8, TPB), TPB, 0, s>>>(Lv.n, Lv.rowptr, Lv.col, val, invd, b, xt, x);
    LAUNCH_CHECK();
    return RICH_OK;
}

template <class T>
rich_status launch_restrict(const Level &Lv, const T *r, T *bc, int64_t nc, const T *invdc, T *x0c, hipStream_t s) {
    if (nc == 0) return RICH_OK;
    if (Lv.prow) return launch_sa_restrict<T>(Lv, r, bc, nc, invdc, x0c, s);
    k_restrict<T><<<xcd_grid(nc, RESTRICT_TPB), RESTRICT_TPB, 0, s>>>(nc, Lv.mptr, Lv.mem, r, bc, invdc, x0c);
    LAUNCH_CHECK();
    return RICH_OK;
}

template <class TB, class T>
rich_status launch_dense_gemv(const T *Ainv, const TB *b, T *x, int64_t n, hipStream_t s) {
    if (n == 0) return RICH_OK;
    k_dense_gemv<TB, T><<<nblocks(n * 64), TPB, 0, s>>>(Ainv, b, x, n);
    LAUNCH_CHECK();
    return RICH_OK;
}

template <class TB, class T>
rich_status launch_csr_sweeps(const Level &Lv, const T *val, const T *invd, const TB *b, T *x, T *tmp, int sweeps,
                              hipStream_t s) {
    if (Lv.n == 0) return RICH_OK;
    T *cur = (sweeps % 2 == 1) ? x : tmp;
    unsigned g = xcd_grid(Lv.n * 8, TPB);
    k_csr_sweep<8, TB, T><<<g, TPB, 0, s>>>(Lv.n, Lv.rowptr, Lv.col, val, invd, b, nullptr, cur, 1);
    LAUNCH_CHECK();
    for (int t = 1; t < sweeps; t++) {
        T *nxt = (cur == x) ? tmp : x;
        k_csr_sweep<8, TB, T><<<g, TPB, 0, s>>>(Lv.n, Lv.rowptr, Lv.col, val, invd, b, cur, nxt, 0);
        LAUNCH_CHECK();
        cur = nxt;
    }
    return RICH_OK;
}

rich_status launch_csr_spmv(const CsrDev &A, const double *x, double *y, hipStream_t s) {
    if (A.n == 0) return RICH_OK;
    k_csr_spmv<<<xcd_grid(A.n * 8, TPB), TPB, 0, s>>>(A.n, A.rowptr, A.col, A.val, x, y);
    LAUNCH_CHECK();
    return RICH_OK;
}

// ---------------------------------------- batched coarse-level launchers
template <class T>
static CoarseArgs<T> coarse_args() {
    CoarseArgs<T> a;
    memset(&a, 0, sizeof(a));
    return a;
}

template <class T, bool POST>
static rich_status stream_batch(const std::vector<CsrItem<T>> &v, hipStream_t s, WorkQueue *q) {
    for (int G : {1, 2, 4, 8}) {
        std::vector<CoarseArgs<T>> a;
        std::vector<unsigned> nb;
        for (const auto &it : v) {
            const Level &Lv = *it.Lv;
            int g = Lv.sg == 1 || Lv.sg == 2 || Lv.sg == 4 ? Lv.sg : 8;
            if (g != G || Lv.n == 0) continue;
            CoarseArgs<T> c = coarse_args<T>();
            c.n = Lv.n;
            c.rb = Lv.rb;
            c.rowptr = Lv.rowptr;
            c.col = Lv.col;
            c.val = it.val;
            c.invd = it.invd;
            c.b = it.b;
            c.v = POST ? (const T *)Lv.r : it.x0;
            c.out = it.out;
            a.push_back(c);
            nb.push_back((unsigned)Lv.nrb);
        }
        using B = Batch<CoarseArgs<T>>;
        switch (G) {
        case 1: RICH_TRY(launch_batches(a, nb, [&](const B &bt, unsigned g) { k_csr_stream_batch<1, T, POST><<<g, 256, 0, s>>>(bt); }, q)); break;
        case 2: RICH_TRY(launch_batches(a, nb, [&](const B &bt, unsigned g) { k_csr_stream_batch<2, T, POST><<<g, 256, 0, s>>>(bt); }, q)); break;
        case 4: RICH_TRY(launch_batches(a, nb, [&](const B &bt, unsigned g) { k_csr_stream_batch<4, T, POST><<<g, 256, 0, s>>>(bt); }, q)); break;
        default: RICH_TRY(launch_batches(a, nb, [&](const B &bt, unsigned g) { k_csr_stream_batch<8, T, POST><<<g, 256, 0, s>>>(bt); }, q)); break;
        }
    }
    return RICH_OK;
}

template <class T>
rich_status launch_csr_pre_batch(const std::vector<CsrItem<T>> &v, hipStream_t s, WorkQueue *q) {
    return stream_batch<T, false>(v, s, q);
}

template <class T>
rich_status launch_csr_post_batch(const std::vector<CsrItem<T>> &v, hipStream_t s, WorkQueue *q) {
    // xt = x0 + P xc into each level's r buffer, then post-smoothing from xt
    std::vector<CoarseArgs<T>> a;
    std::vector<unsigned> nb;
    for (const auto &it : v) {
        const Level &Lv = *it.Lv;
        CoarseArgs<T> c = coarse_args<T>();
        c.n = Lv.n;
        c.b = it.x0;
        c.v = it.xc;
        c.agg = Lv.agg;
        c.out = (T *)Lv.r;
        a.push_back(c);
        nb.push_back((unsigned)((Lv.n + TPB - 1) / TPB));
    }
    RICH_TRY(launch_batches(a, nb, [&](const Batch<CoarseArgs<T>> &bt, unsigned g) {
        k_coarse_batch<T, 1><<<g, TPB, 0, s>>>(bt);
    }, q));
    return stream_batch<T, true>(v, s, q);
}

template <class T>
rich_status launch_restrict_batch(const std::vector<RestrictItem<T>> &v, hipStream_t s, WorkQueue *q) {
    std::vector<CoarseArgs<T>> a;
    std::vector<unsigned> nb;
    for (const auto &it : v) {
        CoarseArgs<T> c = coarse_args<T>();
        c.n = it.nc;
        c.mptr = it.Lv->mptr;
        c.mem = it.Lv->mem;
        c.b = it.r;
        c.out = it.bc;
        c.invd = it.invdc;
        c.x0c = it.x0c;
        a.push_back(c);
        nb.push_back((unsigned)((it.nc + TPB - 1) / TPB));
    }
    return launch_batches(a, nb, [&](const Batch<CoarseArgs<T>> &bt, unsigned g) {
        k_coarse_batch<T, 0><<<g, TPB, 0, s>>>(bt);
    }, q);
}

template <class T>
rich_status launch_dense_gemv_batch(const std::vector<GemvItem<T>> &v, hipStream_t s, WorkQueue *q) {
    std::vector<CoarseArgs<T>> a;
    std::vector<unsigned> nb;
    for (const auto &it : v) {
        CoarseArgs<T> c = coarse_args<T>();
        c.n = it.n;
        c.val = it.Ainv;
        c.b = it.b;
        c.out = it.x;
        a.push_back(c);
        nb.push_back((unsigned)((it.n * 64 + TPB - 1) / TPB));
    }
    return launch_batches(a, nb, [&](const Batch<CoarseArgs<T>> &bt, unsigned g) {
        k_coarse_batch<T, 2><<<g, TPB, 0, s>>>(bt);
    }, q);
}

#define INST_BATCH(T)                                                                              \
    template rich_status launch_csr_pre_batch<T>(const std::vector<CsrItem<T>> &, hipStream_t, WorkQueue *);      \
    template rich_status launch_csr_post_batch<T>(const std::vector<CsrItem<T>> &, hipStream_t, WorkQueue *);     \
    template rich_status launch_restrict_batch<T>(const std::vector<RestrictItem<T>> &, hipStream_t, WorkQueue *); \
    template rich_status launch_dense_gemv_batch<T>(const std::vector<GemvItem<T>> &, hipStream_t, WorkQueue *);
INST_BATCH(double)
INST_BATCH(float)

#define INST_CSR(TB, T)                                                                                         \
    template rich_status launch_csr_pre<TB, T>(const Level &, const T *, const T *, const TB *, T *, hipStream_t); \
    template rich_status launch_csr_post<TB, T>(const Level &, const T *, const T *, const TB *, const T *,        \
                                                const T *, T *, hipStream_t);                                     \
    template rich_status launch_dense_gemv<TB, T>(const T *, const TB *, T *, int64_t, hipStream_t);               \
    template rich_status launch_csr_sweeps<TB, T>(const Level &, const T *, const T *, const TB *, T *, T *, int,  \
                                                  hipStream_t);
INST_CSR(double, double)
INST_CSR(double, float)
INST_CSR(float, float)
template rich_status launch_restrict<double>(const Level &, const double *, double *, int64_t, const double *,
                                             double *, hipStream_t);
template rich_status launch_restrict<float>(const Level &, const float *, float *, int64_t, const float *, float *,
                                            hipStream_t);

}  // namespace rich
