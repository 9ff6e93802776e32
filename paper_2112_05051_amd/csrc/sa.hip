// Smoothed aggregation (Section 5.2: both coarsening schemes of the paper,
// DSVMB and SMATCH, smooth the piecewise-constant prolongator P_t of the
// aggregates).  One damped-Jacobi step is applied to P_t:
//     P = (I - omega D^{-1} A) P_t,  D = diag(A),
//     omega = 4 / (3 rho),  rho = max_i sum_j |a_ij| / a_ii,
// so that P_iJ = [agg(i) = J] - (omega / a_ii) t_iJ with t_iJ the sum of the
// a_ik of row i whose column k lies in aggregate J.  The coarse matrix is
// C = P^T (A P), formed as Q = A P and C = PT Q with PT the transpose of P.
//
// Every value is computed in a fixed order (t_iJ and Q_iJ over row i's
// entries in column order, C_IJ over the rows i of PT row I ascending),
// products are rounded before they are added (no contraction), and the max
// defining rho is exact in any order, so the coarse matrices are reproducible
// bit for bit; the matching of the next level depends on their exact values.
//
// Patterns are structural and built once per hierarchy (the aggregates and
// the fine pattern do not change on a refresh): row r of a product collects
// the sorted distinct candidates of its input rows in a scratch segment of
// its own, sized by the number of candidates.
#include "common.hpp"

namespace rich {

namespace {

constexpr int TPB = 256;
inline unsigned nblocks(int64_t n, int tpb = TPB) { return (unsigned)((n + tpb - 1) / tpb); }

// first position in col[a, b) holding J (J is known to be present)
__device__ inline int64_t find_col(const int32_t *__restrict__ col, int64_t a, int64_t b, int32_t J) {
    int64_t lo = a, hi = b - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (col[mid] < J) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Candidates of output row r: for t in [xptr[r], xptr[r+1]) with k = xidx[t],
// either k itself (yptr == nullptr) or every ycol[f], f in [yptr[k], yptr[k+1]);
// each candidate is mapped through agg when agg != nullptr.
__global__ void k_union_seglen(int64_t nr, const int64_t *__restrict__ xptr, const int32_t *__restrict__ xidx,
                               const int64_t *__restrict__ yptr, int64_t *__restrict__ seg) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    if (!yptr) {
        seg[r] = xptr[r + 1] - xptr[r];
        return;
    }
    int64_t s = 0;
    for (int64_t t = xptr[r]; t < xptr[r + 1]; t++) s += yptr[xidx[t] + 1] - yptr[xidx[t]];
    seg[r] = s;
}

__global__ void k_union_collect(int64_t nr, const int64_t *__restrict__ xptr, const int32_t *__restrict__ xidx,
                                const int64_t *__restrict__ yptr, const int32_t *__restrict__ ycol,
                                const int32_t *__restrict__ agg, const int64_t *__restrict__ segptr,
                                int32_t *__restrict__ scratch, int64_t *__restrict__ cnt) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    int32_t *buf = scratch + segptr[r];
    int64_t len = 0;
    auto insert = [&](int32_t J) {
        int64_t u = len;
        while (u > 0 && buf[u - 1] > J) u--;
        if (u > 0 && buf[u - 1] == J) return;
        for (int64_t v = len; v > u; v--) buf[v] = buf[v - 1];
        buf[u] = J;
        len++;
    };
    for (int64_t t = xptr[r]; t < xptr[r + 1]; t++) {
        int32_t k = xidx[t];
        if (!yptr) {
            insert(agg ? agg[k] : k);
            continue;
        }
        for (int64_t f = yptr[k]; f < yptr[k + 1]; f++) insert(agg ? agg[ycol[f]] : ycol[f]);
    }
    cnt[r] = len;
}

__global__ void k_union_write(int64_t nr, const int64_t *__restrict__ segptr, const int32_t *__restrict__ scratch,
                              const int64_t *__restrict__ orow, int32_t *__restrict__ ocol) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    const int32_t *buf = scratch + segptr[r];
    int64_t o = orow[r], n = orow[r + 1] - o;
    for (int64_t a = 0; a < n; a++) ocol[o + a] = buf[a];
}

// rho: row ratios sum_j |a_ij| / a_ii (column order), block maximum, then one
// atomic maximum per block on the bit pattern (positive doubles order as
// their bits; the result does not depend on the order).
__global__ void __launch_bounds__(256) k_sa_rho(int64_t n, const int64_t *__restrict__ rowptr,
                                                const int32_t *__restrict__ col, const double *__restrict__ val,
                                                unsigned long long *__restrict__ rho_bits) {
    __shared__ unsigned long long red[256];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long m = 0;
    if (i < n) {
        double s = 0.0, d = 0.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
            s += fabs(val[e]);
            if (col[e] == i) d = val[e];
        }
        m = (unsigned long long)__double_as_longlong(s / d);
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o && red[threadIdx.x + o] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(rho_bits, red[0]);
}

__global__ void k_zero_u64(unsigned long long *x) {
    if (threadIdx.x == 0 && blockIdx.x == 0) x[0] = 0ull;
}

// P_iJ = [agg(i) = J] - (omega / a_ii) t_iJ
__global__ void k_sa_pnum(int64_t n, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                          const double *__restrict__ val, const int32_t *__restrict__ agg,
                          const unsigned long long *__restrict__ rho_bits, const int64_t *__restrict__ prow,
                          const int32_t *__restrict__ pcol, double *__restrict__ pval) {
#pragma clang fp contract(off)
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double rho = __longlong_as_double((long long)rho_bits[0]);
    double omega = 4.0 / (3.0 * rho);
    int64_t p0 = prow[i], p1 = prow[i + 1];
    double d = 0.0;
    for (int64_t f = p0; f < p1; f++) pval[f] = 0.0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
        if (col[e] == i) d = val[e];
        int64_t f = find_col(pcol, p0, p1, agg[col[e]]);
        pval[f] = pval[f] + val[e];
    }
    double w = omega / d;
    int32_t own = agg[i];
    for (int64_t f = p0; f < p1; f++) {
        double q = w * pval[f];
        pval[f] = (pcol[f] == own ? 1.0 : 0.0) - q;
    }
}

// PT values: PT_Ii = P_iI
__global__ void k_sa_tval(int64_t nc, const int64_t *__restrict__ trow, const int32_t *__restrict__ tcol,
                          const int64_t *__restrict__ prow, const int32_t *__restrict__ pcol,
                          const double *__restrict__ pval, double *__restrict__ tval) {
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    for (int64_t t = trow[I]; t < trow[I + 1]; t++) {
        int32_t i = tcol[t];
        tval[t] = pval[find_col(pcol, prow[i], prow[i + 1], (int32_t)I)];
    }
}

// Q_iJ = sum over row i of A (column order) of a_ik P_kJ.  One thread per
// row; rows of up to SA_REG entries accumulate in LDS (column-major over the
// block's 64 threads, so the dynamic indexing never spills to scratch
// memory), longer ones in the output.
constexpr int SA_REG = 32;
__global__ void __launch_bounds__(64) k_sa_qnum(int64_t n, const int64_t *__restrict__ rowptr,
                                                const int32_t *__restrict__ col, const double *__restrict__ val,
                                                const int64_t *__restrict__ prow, const int32_t *__restrict__ pcol,
                                                const double *__restrict__ pval, const int64_t *__restrict__ qrow,
                                                const int32_t *__restrict__ qcol, double *__restrict__ qval) {
#pragma clang fp contract(off)
    __shared__ double acc_s[SA_REG * 64];
    __shared__ int32_t cj_s[SA_REG * 64];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = threadIdx.x;
    int64_t q0 = qrow[i], q1 = qrow[i + 1];
    int len = (int)(q1 - q0);
    if (len <= SA_REG) {
        for (int e = 0; e < len; e++) {
            cj_s[e * 64 + t] = qcol[q0 + e];
            acc_s[e * 64 + t] = 0.0;
        }
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
            int32_t k = col[e];
            double a = val[e];
            for (int64_t f = prow[k]; f < prow[k + 1]; f++) {
                int32_t J = pcol[f];
                int lo = 0, hi = len - 1;
                while (lo < hi) {
                    int mid = (lo + hi) >> 1;
                    if (cj_s[mid * 64 + t] < J) lo = mid + 1;
                    else hi = mid;
                }
                double prod = a * pval[f];
                acc_s[lo * 64 + t] = acc_s[lo * 64 + t] + prod;
            }
        }
        for (int e = 0; e < len; e++) qval[q0 + e] = acc_s[e * 64 + t];
        return;
    }
    for (int64_t f = q0; f < q1; f++) qval[f] = 0.0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
        int32_t k = col[e];
        double a = val[e];
        for (int64_t f = prow[k]; f < prow[k + 1]; f++) {
            int64_t o = find_col(qcol, q0, q1, pcol[f]);
            double prod = a * pval[f];
            qval[o] = qval[o] + prod;
        }
    }
}

// C_IJ = sum over the rows i of PT row I (ascending) of PT_Ii Q_iJ, with LDS
// accumulators as in k_sa_qnum.
constexpr int SA_CREG = 64;
__global__ void __launch_bounds__(64) k_sa_cnum(int64_t nc, const int64_t *__restrict__ trow,
                                                const int32_t *__restrict__ tcol, const double *__restrict__ tval,
                                                const int64_t *__restrict__ qrow, const int32_t *__restrict__ qcol,
                                                const double *__restrict__ qval, const int64_t *__restrict__ crow,
                                                const int32_t *__restrict__ ccol, double *__restrict__ cval) {
#pragma clang fp contract(off)
    __shared__ double acc_s[SA_CREG * 64];
    __shared__ int32_t cj_s[SA_CREG * 64];
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    const int t = threadIdx.x;
    int64_t c0 = crow[I], c1 = crow[I + 1];
    int len = (int)(c1 - c0);
    if (len <= SA_CREG) {
        for (int e = 0; e < len; e++) {
            cj_s[e * 64 + t] = ccol[c0 + e];
            acc_s[e * 64 + t] = 0.0;
        }
        for (int64_t q = trow[I]; q < trow[I + 1]; q++) {
            int32_t i = tcol[q];
            double p = tval[q];
            for (int64_t f = qrow[i]; f < qrow[i + 1]; f++) {
                int32_t J = qcol[f];
                int lo = 0, hi = len - 1;
                while (lo < hi) {
                    int mid = (lo + hi) >> 1;
                    if (cj_s[mid * 64 + t] < J) lo = mid + 1;
                    else hi = mid;
                }
                double prod = p * qval[f];
                acc_s[lo * 64 + t] = acc_s[lo * 64 + t] + prod;
            }
        }
        for (int e = 0; e < len; e++) cval[c0 + e] = acc_s[e * 64 + t];
        return;
    }
    for (int64_t f = c0; f < c1; f++) cval[f] = 0.0;
    for (int64_t q = trow[I]; q < trow[I + 1]; q++) {
        int32_t i = tcol[q];
        double p = tval[q];
        for (int64_t f = qrow[i]; f < qrow[i + 1]; f++) {
            int64_t o = find_col(ccol, c0, c1, qcol[f]);
            double prod = p * qval[f];
            cval[o] = cval[o] + prod;
        }
    }
}

// V-cycle: bc = P^T r (and x0c = D_c^{-1} bc when x0c is set), G lanes per coarse row
template <int G, class T>
__global__ void k_sa_restrict(int64_t nc, const int64_t *__restrict__ trow, const int32_t *__restrict__ tcol,
                              const T *__restrict__ tval, const T *__restrict__ r, T *__restrict__ bc,
                              const T *__restrict__ invdc, T *__restrict__ x0c) {
    int64_t I = ((int64_t)xcd_block() * blockDim.x + threadIdx.x) / G;
    int lane = threadIdx.x % G;
    if (I >= nc) return;
    T s = 0;
    for (int64_t t = trow[I] + lane; t < trow[I + 1]; t += G) s += tval[t] * r[tcol[t]];
    s = group_sum<G>(s);
    if (lane == 0) {
        bc[I] = s;
        if (x0c) x0c[I] = s * invdc[I];
    }
}

// V-cycle: xt = x0 + P xc with x0 given or D^{-1} (bs b), G lanes per fine row
template <int G, class TB, class T>
__global__ void k_sa_prolong(int64_t n, const int64_t *__restrict__ prow, const int32_t *__restrict__ pcol,
                             const T *__restrict__ pval, const T *__restrict__ invd, const TB *__restrict__ b,
                             const double *__restrict__ bsp, const T *__restrict__ x0, const T *__restrict__ xc,
                             T *__restrict__ xt) {
    int64_t i = ((int64_t)xcd_block() * blockDim.x + threadIdx.x) / G;
    int lane = threadIdx.x % G;
    if (i >= n) return;
    T s = 0;
    for (int64_t f = prow[i] + lane; f < prow[i + 1]; f += G) s += pval[f] * xc[pcol[f]];
    s = group_sum<G>(s);
    if (lane == 0) {
        if (x0) {
            xt[i] = x0[i] + s;
        } else {
            T bi = bsp ? (T)(b[i] * (TB)bsp[0]) : (T)b[i];
            xt[i] = bi * invd[i] + s;
        }
    }
}

// Sorted-union pattern of nr output rows (see k_union_collect) into out.
rich_status union_pattern(int64_t nr, const int64_t *xptr, const int32_t *xidx, const int64_t *yptr,
                          const int32_t *ycol, const int32_t *agg, int64_t **orow, int32_t **ocol, int64_t *onnz,
                          DevAlloc &mem_out, hipStream_t s) {
    DevAlloc tmp;
    int64_t *seg, *segptr, *cnt, *stmp;
    RICH_TRY(tmp.get(&seg, nr));
    RICH_TRY(tmp.get(&segptr, nr + 1));
    RICH_TRY(tmp.get(&cnt, nr));
    RICH_TRY(tmp.get(&stmp, scan_tmp_size(nr)));
    RICH_TRY(mem_out.get(orow, nr + 1));
    if (nr > 0) {
        k_union_seglen<<<nblocks(nr), TPB, 0, s>>>(nr, xptr, xidx, yptr, seg);
        LAUNCH_CHECK();
    }
    RICH_TRY(scan_exclusive_i64(seg, segptr, nr, stmp, s));
    int64_t total = 0;
    HIP_TRY(hipMemcpyAsync(&total, segptr + nr, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int32_t *scratch;
    RICH_TRY(tmp.get(&scratch, total));
    if (nr > 0) {
        k_union_collect<<<nblocks(nr, 64), 64, 0, s>>>(nr, xptr, xidx, yptr, ycol, agg, segptr, scratch, cnt);
        LAUNCH_CHECK();
    }
    RICH_TRY(scan_exclusive_i64(cnt, *orow, nr, stmp, s));
    HIP_TRY(hipMemcpyAsync(onnz, *orow + nr, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    RICH_TRY(mem_out.get(ocol, *onnz));
    if (nr > 0) {
        k_union_write<<<nblocks(nr), TPB, 0, s>>>(nr, segptr, scratch, *orow, *ocol);
        LAUNCH_CHECK();
    }
    HIP_TRY(hipStreamSynchronize(s));  // tmp is freed on return
    return RICH_OK;
}

}  // namespace

rich_status sa_symbolic(const CsrDev &A, const int32_t *agg, int64_t nc, const int64_t *mptr, const int32_t *mem,
                        Level &Lf, CsrDev *C, bool mixed, DevAlloc &mem_out, hipStream_t s) {
    int64_t n = A.n;
    // P: row i holds the aggregates its row of A touches
    RICH_TRY(union_pattern(n, A.rowptr, A.col, nullptr, nullptr, agg, &Lf.prow, &Lf.pcol, &Lf.pnnz, mem_out, s));
    // PT: row I holds the rows that touch I, i.e. (A being structurally
    // symmetric) the neighbours of the members of I
    int64_t tnnz = 0;
    RICH_TRY(union_pattern(nc, mptr, mem, A.rowptr, A.col, nullptr, &Lf.trow, &Lf.tcol, &tnnz, mem_out, s));
    if (tnnz != Lf.pnnz) return RICH_EINVAL;  // A not structurally symmetric
    // Q = A P and C = PT Q
    RICH_TRY(union_pattern(n, A.rowptr, A.col, Lf.prow, Lf.pcol, nullptr, &Lf.qrow, &Lf.qcol, &Lf.qnnz, mem_out, s));
    C->n = nc;
    RICH_TRY(union_pattern(nc, Lf.trow, Lf.tcol, Lf.qrow, Lf.qcol, nullptr, &C->rowptr, &C->col, &C->nnz, mem_out, s));
    RICH_TRY(mem_out.get(&C->val, C->nnz));
    RICH_TRY(mem_out.get(&Lf.pval, Lf.pnnz));
    RICH_TRY(mem_out.get(&Lf.tval, Lf.pnnz));
    RICH_TRY(mem_out.get(&Lf.qval, Lf.qnnz));
    RICH_TRY(mem_out.get(&Lf.rho, 1));
    if (mixed) {
        RICH_TRY(mem_out.get(&Lf.pvalf, Lf.pnnz));
        RICH_TRY(mem_out.get(&Lf.tvalf, Lf.pnnz));
    }
    return RICH_OK;
}

rich_status sa_numeric(const CsrDev &A, const int32_t *agg, Level &Lf, const CsrDev &C, bool mixed, hipStream_t s) {
    int64_t n = A.n, nc = C.n;
    if (n == 0) return RICH_OK;
    k_zero_u64<<<1, 64, 0, s>>>(Lf.rho);
    k_sa_rho<<<nblocks(n, 256), 256, 0, s>>>(n, A.rowptr, A.col, A.val, Lf.rho);
    k_sa_pnum<<<nblocks(n), TPB, 0, s>>>(n, A.rowptr, A.col, A.val, agg, Lf.rho, Lf.prow, Lf.pcol, Lf.pval);
    LAUNCH_CHECK();
    if (nc > 0) {
        k_sa_tval<<<nblocks(nc), TPB, 0, s>>>(nc, Lf.trow, Lf.tcol, Lf.prow, Lf.pcol, Lf.pval, Lf.tval);
        LAUNCH_CHECK();
    }
    k_sa_qnum<<<nblocks(n, 64), 64, 0, s>>>(n, A.rowptr, A.col, A.val, Lf.prow, Lf.pcol, Lf.pval, Lf.qrow, Lf.qcol,
                                            Lf.qval);
    LAUNCH_CHECK();
    if (nc > 0) {
        k_sa_cnum<<<nblocks(nc, 64), 64, 0, s>>>(nc, Lf.trow, Lf.tcol, Lf.tval, Lf.qrow, Lf.qcol, Lf.qval, C.rowptr,
                                                 C.col, C.val);
        LAUNCH_CHECK();
    }
    if (mixed) {
        RICH_TRY(launch_cast(Lf.pval, Lf.pvalf, Lf.pnnz, s));
        RICH_TRY(launch_cast(Lf.tval, Lf.tvalf, Lf.pnnz, s));
    }
    return RICH_OK;
}

template <class T>
const T *sa_tv(const Level &L);
template <>
const double *sa_tv<double>(const Level &L) { return L.tval; }
template <>
const float *sa_tv<float>(const Level &L) { return L.tvalf; }
template <class T>
const T *sa_pv(const Level &L);
template <>
const double *sa_pv<double>(const Level &L) { return L.pval; }
template <>
const float *sa_pv<float>(const Level &L) { return L.pvalf; }

template <class T>
rich_status launch_sa_restrict(const Level &Lv, const T *r, T *bc, int64_t nc, const T *invdc, T *x0c,
                               hipStream_t s) {
    if (nc == 0) return RICH_OK;
    if (Lv.pnnz < 16 * nc)
        k_sa_restrict<8, T><<<xcd_grid(nc * 8, TPB), TPB, 0, s>>>(nc, Lv.trow, Lv.tcol, sa_tv<T>(Lv), r, bc, invdc,
                                                                    x0c);
    else
        k_sa_restrict<16, T><<<xcd_grid(nc * 16, TPB), TPB, 0, s>>>(nc, Lv.trow, Lv.tcol, sa_tv<T>(Lv), r, bc,
                                                                      invdc, x0c);
    LAUNCH_CHECK();
    return RICH_OK;
}

template <class TB, class T>
rich_status launch_sa_prolong(const Level &Lv, const T *invd, const TB *b, const double *bs, const T *x0,
                              const T *xc, T *xt, hipStream_t s) {
    if (Lv.n == 0) return RICH_OK;
    k_sa_prolong<4, TB, T><<<xcd_grid(Lv.n * 4, TPB), TPB, 0, s>>>(Lv.n, Lv.prow, Lv.pcol, sa_pv<T>(Lv), invd, b,
                                                                     bs, x0, xc, xt);
    LAUNCH_CHECK();
    return RICH_OK;
}

template rich_status launch_sa_restrict<double>(const Level &, const double *, double *, int64_t, const double *,
                                                double *, hipStream_t);
template rich_status launch_sa_restrict<float>(const Level &, const float *, float *, int64_t, const float *, float *,
                                               hipStream_t);
template rich_status launch_sa_prolong<double, double>(const Level &, const double *, const double *, const double *,
                                                       const double *, const double *, double *, hipStream_t);
template rich_status launch_sa_prolong<double, float>(const Level &, const float *, const double *, const double *,
                                                      const float *, const float *, float *, hipStream_t);
template rich_status launch_sa_prolong<float, float>(const Level &, const float *, const float *, const double *,
                                                     const float *, const float *, float *, hipStream_t);

}  // namespace rich
