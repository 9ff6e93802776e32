// Vector kernels for the Krylov and Newton loops: deterministic reductions
// (fixed grid, per-block partials, then one fixed-order pass), the fused
// classical Gram-Schmidt dot block and update, axpy-type updates, casts and
// an exclusive scan for the setup phase.
#include "common.hpp"

namespace rich {

namespace {

constexpr int TPB = 256;
constexpr int WAVE = 64;
constexpr int KMAX = 66;  // GMRES restart (<= 64) + 2

inline unsigned nblocks(int64_t n, int tpb = TPB) { return (unsigned)((n + tpb - 1) / tpb); }

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_down(v, o, WAVE);
    return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        double u = __shfl_down(v, o, WAVE);
        v = (u > v || u != u) ? u : v;
    }
    return v;
}

// Block sum of one value per thread, result valid in thread 0.
__device__ inline double block_sum(double v, double *sh) {
    v = wave_sum(v);
    int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int t = 0; t < (int)(blockDim.x / WAVE); t++) r += sh[t];
    return r;
}

__device__ inline double block_max(double v, double *sh) {
    v = wave_max(v);
    int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int t = 0; t < (int)(blockDim.x / WAVE); t++) r = (sh[t] > r || sh[t] != sh[t]) ? sh[t] : r;
    return r;
}

// Dot products of w with V_0..V_{K-1} and w.w, partial per block.  K is a
// compile-time constant so every load of a row pair is issued before its
// use; rows are taken in pairs with 16-byte loads (the basis stride ldv is a
// multiple of 2 and the vectors are 16-byte aligned).  The odd last row of
// an odd n is added by the first thread of block 0.
// Register budget of the basis kernels on large vectors.  Their launch
// (RED_BLOCKS blocks of RED_THREADS) holds 4 waves per SIMD, yet scheduled for
// the default occupancy the compiler loads one or two basis vectors at a time,
// each product waiting for its own load.  Allowing 256 VGPRs (two waves per
// SIMD) lets it issue the loads of all K vectors of a row pair up front.  On
// short vectors the kernels are latency-bound and the second round of blocks
// that two waves per SIMD imply costs more than it saves: there the default
// schedule (the _small kernels) runs.  Both compute the same sums.
#define RED_WPE_ATTR __attribute__((amdgpu_waves_per_eu(2, 2)))
constexpr int64_t RED_WIDE_MIN = int64_t(1) << 21;
template <int K>
__device__ __forceinline__ void multidot_body(const double *__restrict__ V, int64_t ldv, const double *__restrict__ w,
                                              int64_t n, double *__restrict__ partial) {
    __shared__ double sh[RED_THREADS / WAVE];
    double acc[K + 1];
#pragma unroll
    for (int i = 0; i <= K; i++) acc[i] = 0.0;
    const int64_t n2 = n >> 1;
    const double2 *__restrict__ w2 = reinterpret_cast<const double2 *>(w);
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n2; c += (int64_t)gridDim.x * blockDim.x) {
        double2 wc = w2[c];
        double2 v[K];
        // the basis is streamed (non-temporal): it is far larger than the caches
        typedef double d2v __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int i = 0; i < K; i++) {
            d2v t = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(V + (size_t)i * ldv) + c);
            v[i] = make_double2(t.x, t.y);
        }
#pragma unroll
        for (int i = 0; i < K; i++) acc[i] += v[i].x * wc.x + v[i].y * wc.y;
        acc[K] += wc.x * wc.x + wc.y * wc.y;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        double wc = w[n - 1];
#pragma unroll
        for (int i = 0; i < K; i++) acc[i] += V[(size_t)i * ldv + n - 1] * wc;
        acc[K] += wc * wc;
    }
#pragma unroll
    for (int i = 0; i <= K; i++) {
        double r = block_sum(acc[i], sh);
        if (threadIdx.x == 0) partial[(size_t)blockIdx.x * (K + 1) + i] = r;
    }
}

template <int K>
__global__ void __launch_bounds__(RED_THREADS) RED_WPE_ATTR k_multidot(const double *__restrict__ V, int64_t ldv,
                                                                     const double *__restrict__ w, int64_t n,
                                                                     double *__restrict__ partial) {
    multidot_body<K>(V, ldv, w, n, partial);
}

template <int K>
__global__ void __launch_bounds__(RED_THREADS) k_multidot_small(const double *__restrict__ V, int64_t ldv,
                                                                const double *__restrict__ w, int64_t n,
                                                                double *__restrict__ partial) {
    multidot_body<K>(V, ldv, w, n, partial);
}

// out[i] = sum_b partial[b*(m) + i], b ascending (one block per output),
// times scale[i] for i < nscale (basis vectors stored with a scale factor).
__global__ void k_reduce_partials(const double *__restrict__ partial, int m, int nb, double *__restrict__ out,
                                  const double *__restrict__ scale = nullptr, int nscale = 0) {
    __shared__ double sh[RED_THREADS / WAVE];
    int i = blockIdx.x;
    double a = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) a += partial[(size_t)b * m + i];
    double r = block_sum(a, sh);
    if (threadIdx.x == 0) out[i] = (i < nscale) ? r * scale[i] : r;
}

// vs[0] = 1/sqrt(ww[0]) (0 for a zero vector): the scale of a new basis vector.
__global__ void k_set_scale(double *__restrict__ vs, const double *__restrict__ ww) {
    if (threadIdx.x == 0 && blockIdx.x == 0) vs[0] = ww[0] > 0.0 ? 1.0 / sqrt(ww[0]) : 0.0;
}

__global__ void k_reduce_max(const double *__restrict__ partial, int m, int nb, double *__restrict__ out) {
    __shared__ double sh[RED_THREADS / WAVE];
    double a = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        double v = partial[(size_t)b * m];
        a = (v > a || v != v) ? v : a;
    }
    double r = block_max(a, sh);
    if (threadIdx.x == 0) out[0] = r;
}

// w -= sum_i h_i (vs_i V_i) and the partial sums of ||w||^2, K compile-time, row pairs.
template <int K>
__device__ __forceinline__ void update_norm_body(const double *__restrict__ V, int64_t ldv,
                                                 const double *__restrict__ h, const double *__restrict__ vs,
                                                 double *__restrict__ w, int64_t n, double *__restrict__ partial) {
    __shared__ double sh[RED_THREADS / WAVE];
    double hr[K];
#pragma unroll
    for (int i = 0; i < K; i++) hr[i] = h[i] * vs[i];
    double acc = 0.0;
    const int64_t n2 = n >> 1;
    // the basis is streamed past the caches; w, the next basis vector, is
    // kept cacheable (the V-cycle reads it next)
    typedef double d2v __attribute__((ext_vector_type(2)));
    d2v *__restrict__ w2 = reinterpret_cast<d2v *>(w);
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n2; c += (int64_t)gridDim.x * blockDim.x) {
        d2v wc = w2[c];
        d2v v[K];
#pragma unroll
        for (int i = 0; i < K; i++) v[i] = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(V + (size_t)i * ldv) + c);
#pragma unroll
        for (int i = 0; i < K; i++) {
            wc.x -= hr[i] * v[i].x;
            wc.y -= hr[i] * v[i].y;
        }
        w2[c] = wc;  // the next basis vector: read again at once by the V-cycle
        acc += wc.x * wc.x + wc.y * wc.y;
    }

    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        double wc = w[n - 1];
#pragma unroll
        for (int i = 0; i < K; i++) wc -= hr[i] * V[(size_t)i * ldv + n - 1];
        w[n - 1] = wc;
        acc += wc * wc;
    }
    double r = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

template <int K>
__global__ void __launch_bounds__(RED_THREADS) RED_WPE_ATTR k_update_norm(const double *__restrict__ V, int64_t ldv,
                                                                        const double *__restrict__ h,
                                                                        const double *__restrict__ vs,
                                                                        double *__restrict__ w, int64_t n,
                                                                        double *__restrict__ partial) {
    update_norm_body<K>(V, ldv, h, vs, w, n, partial);
}

template <int K>
__global__ void __launch_bounds__(RED_THREADS) k_update_norm_small(const double *__restrict__ V, int64_t ldv,
                                                                   const double *__restrict__ h,
                                                                   const double *__restrict__ vs,
                                                                   double *__restrict__ w, int64_t n,
                                                                   double *__restrict__ partial) {
    update_norm_body<K>(V, ldv, h, vs, w, n, partial);
}

// ---- block Gram-Schmidt of the s-step GMRES ----
// Partial sums of C = V^T Q, the dots of the S raw block vectors Q_0..Q_{S-1}
// with nv basis vectors (stored unnormalised: their scales are applied in the
// reduction), and of the Gram matrix Q^T Q.  The four waves of a block walk
// the same row pairs: wave g takes basis vectors [g GV, min(nv, (g+1) GV)),
// the last wave also the Gram matrix, so the Q values of a row pair are
// fetched from memory once and read by the other waves from the caches; the
// basis is streamed past the caches.  Per block: C row-major (i S + k), then
// (when gram) the upper triangle of the Gram matrix by rows.
template <int S, int GV>
__device__ __forceinline__ void block_dot_body(const double *__restrict__ V, int64_t ldv, int nv, bool gram,
                                               const double *__restrict__ Q, int64_t n,
                                               double *__restrict__ partial, int mout) {
    constexpr int NG = S * (S + 1) / 2;
    typedef double d2v __attribute__((ext_vector_type(2)));
    const int lane = threadIdx.x % WAVE, g = threadIdx.x / WAVE;
    const int i0 = g * GV;
    const int ng = nv - i0 < GV ? (nv - i0 > 0 ? nv - i0 : 0) : GV;  // uniform in the wave
    const bool dog = gram && g == RED_THREADS / WAVE - 1;
    double acc[GV][S], gm[NG];
#pragma unroll
    for (int i = 0; i < GV; i++)
#pragma unroll
        for (int k = 0; k < S; k++) acc[i][k] = 0.0;
#pragma unroll
    for (int t = 0; t < NG; t++) gm[t] = 0.0;
    const int64_t n2 = n >> 1;
    for (int64_t c = (int64_t)blockIdx.x * WAVE + lane; c < n2; c += (int64_t)gridDim.x * WAVE) {
        d2v q[S], v[GV];
#pragma unroll
        for (int k = 0; k < S; k++) q[k] = reinterpret_cast<const d2v *>(Q + (size_t)k * ldv)[c];
#pragma unroll
        for (int i = 0; i < GV; i++)
            if (i < ng) v[i] = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(V + (size_t)(i0 + i) * ldv) + c);
#pragma unroll
        for (int i = 0; i < GV; i++)
            if (i < ng)
#pragma unroll
                for (int k = 0; k < S; k++) acc[i][k] += v[i].x * q[k].x + v[i].y * q[k].y;
        if (dog) {
            int t = 0;
#pragma unroll
            for (int k = 0; k < S; k++)
#pragma unroll
                for (int l = k; l < S; l++, t++) gm[t] += q[k].x * q[l].x + q[k].y * q[l].y;
        }
    }
    if ((n & 1) && blockIdx.x == 0 && lane == 0) {
        double q[S];
#pragma unroll
        for (int k = 0; k < S; k++) q[k] = Q[(size_t)k * ldv + n - 1];
#pragma unroll
        for (int i = 0; i < GV; i++)
            if (i < ng) {
                const double vi = V[(size_t)(i0 + i) * ldv + n - 1];
#pragma unroll
                for (int k = 0; k < S; k++) acc[i][k] += vi * q[k];
            }
        if (dog) {
            int t = 0;
#pragma unroll
            for (int k = 0; k < S; k++)
#pragma unroll
                for (int l = k; l < S; l++, t++) gm[t] += q[k] * q[l];
        }
    }
    double *out = partial + (size_t)blockIdx.x * mout;
#pragma unroll
    for (int i = 0; i < GV; i++)
        if (i < ng)
#pragma unroll
            for (int k = 0; k < S; k++) {
                const double r = wave_sum(acc[i][k]);
                if (lane == 0) out[(i0 + i) * S + k] = r;
            }
    if (dog)
#pragma unroll
        for (int t = 0; t < NG; t++) {
            const double r = wave_sum(gm[t]);
            if (lane == 0) out[nv * S + t] = r;
        }
}

template <int S, int GV>
__global__ void __launch_bounds__(RED_THREADS) RED_WPE_ATTR k_block_dot(const double *__restrict__ V, int64_t ldv,
                                                                      int nv, bool gram,
                                                                      const double *__restrict__ Q, int64_t n,
                                                                      double *__restrict__ partial, int mout) {
    block_dot_body<S, GV>(V, ldv, nv, gram, Q, n, partial, mout);
}

template <int S, int GV>
__global__ void __launch_bounds__(RED_THREADS) k_block_dot_small(const double *__restrict__ V, int64_t ldv, int nv,
                                                                 bool gram, const double *__restrict__ Q, int64_t n,
                                                                 double *__restrict__ partial, int mout) {
    block_dot_body<S, GV>(V, ldv, nv, gram, Q, n, partial, mout);
}

// The same sums for rounds of 7..10 vectors, with the Gram matrix spread
// over the four waves (entry t by wave t mod 4) so that the accumulators of
// GV <= 6 basis vectors stay within the register budget.  Same output layout.
// The wave index is a template argument: each wave's Gram entries are fixed at
// compile time and their accumulators stay in registers.  The round's vectors
// are read from HBM once per block (each wave loads every fourth one into
// LDS) instead of once per wave.
typedef double d2v_t __attribute__((ext_vector_type(2)));
template <int S, int GV, int G>
__device__ __forceinline__ void block_dot_wave_wide(const double *__restrict__ V, int64_t ldv, int nv, bool gram,
                                                    const double *__restrict__ Q, int64_t n,
                                                    double *__restrict__ partial, int mout,
                                                    d2v_t (*__restrict__ qs)[S][WAVE]) {
    constexpr int NG = S * (S + 1) / 2;
    constexpr int NW = RED_THREADS / WAVE;
    constexpr int NGW = (NG - G + NW - 1) / NW;  // Gram entries of this wave: t = G, G + NW, ...
    typedef d2v_t d2v;
    const int lane = threadIdx.x % WAVE;
    constexpr int i0 = G * GV;
    const int ng = nv - i0 < GV ? (nv - i0 > 0 ? nv - i0 : 0) : GV;
    double acc[GV][S], gm[NGW > 0 ? NGW : 1];
#pragma unroll
    for (int i = 0; i < GV; i++)
#pragma unroll
        for (int k = 0; k < S; k++) acc[i][k] = 0.0;
#pragma unroll
    for (int u = 0; u < NGW; u++) gm[u] = 0.0;
    const int64_t n2 = n >> 1;
    // block-uniform trip count (the barrier below); lanes past the end add zeros
    int buf = 0;
    for (int64_t base = (int64_t)blockIdx.x * WAVE; base < n2; base += (int64_t)gridDim.x * WAVE) {
        const int64_t c = base + lane;
        const bool act = c < n2;
        const d2v zero = {0.0, 0.0};
        d2v q[S], v[GV];
        // this wave's share of the round's vectors (k = G, G + NW, ...) into LDS
#pragma unroll
        for (int k = G; k < S; k += NW) qs[buf][k][lane] = act ? reinterpret_cast<const d2v *>(Q + (size_t)k * ldv)[c] : zero;
#pragma unroll
        for (int i = 0; i < GV; i++)
            if (i < ng)
                v[i] = act ? __builtin_nontemporal_load(reinterpret_cast<const d2v *>(V + (size_t)(i0 + i) * ldv) + c)
                           : zero;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < S; k++) q[k] = qs[buf][k][lane];
        buf ^= 1;  // the other buffer is next written after the next barrier
#pragma unroll
        for (int i = 0; i < GV; i++)
            if (i < ng)
#pragma unroll
                for (int k = 0; k < S; k++) acc[i][k] += v[i].x * q[k].x + v[i].y * q[k].y;
        if (gram) {
#pragma unroll
            for (int k = 0; k < S; k++)
#pragma unroll
                for (int l = k; l < S; l++) {
                    const int t = k * S - k * (k - 1) / 2 + (l - k);  // row-major upper triangle
                    if (t % NW == G) gm[t / NW] += q[k].x * q[l].x + q[k].y * q[l].y;
                }
        }
    }
    if ((n & 1) && blockIdx.x == 0 && lane == 0) {
        double q[S];
#pragma unroll
        for (int k = 0; k < S; k++) q[k] = Q[(size_t)k * ldv + n - 1];
#pragma unroll
        for (int i = 0; i < GV; i++)
            if (i < ng) {
                const double vi = V[(size_t)(i0 + i) * ldv + n - 1];
#pragma unroll
                for (int k = 0; k < S; k++) acc[i][k] += vi * q[k];
            }
        if (gram) {
#pragma unroll
            for (int k = 0; k < S; k++)
#pragma unroll
                for (int l = k; l < S; l++) {
                    const int t = k * S - k * (k - 1) / 2 + (l - k);
                    if (t % NW == G) gm[t / NW] += q[k] * q[l];
                }
        }
    }
    double *out = partial + (size_t)blockIdx.x * mout;
#pragma unroll
    for (int i = 0; i < GV; i++)
        if (i < ng)
#pragma unroll
            for (int k = 0; k < S; k++) {
                const double r = wave_sum(acc[i][k]);
                if (lane == 0) out[(i0 + i) * S + k] = r;
            }
    if (gram) {
#pragma unroll
        for (int u = 0; u < NGW; u++) {
            const double r = wave_sum(gm[u]);
            if (lane == 0) out[nv * S + G + u * NW] = r;
        }
    }
}

template <int S, int GV>
__device__ __forceinline__ void block_dot_body_wide(const double *__restrict__ V, int64_t ldv, int nv, bool gram,
                                                    const double *__restrict__ Q, int64_t n,
                                                    double *__restrict__ partial, int mout) {
    static_assert(RED_THREADS / WAVE == 4, "four waves per block");
    __shared__ d2v_t qs[2][S][WAVE];  // the round's vectors at the block's rows, double-buffered
    switch (threadIdx.x / WAVE) {
    case 0: block_dot_wave_wide<S, GV, 0>(V, ldv, nv, gram, Q, n, partial, mout, qs); break;
    case 1: block_dot_wave_wide<S, GV, 1>(V, ldv, nv, gram, Q, n, partial, mout, qs); break;
    case 2: block_dot_wave_wide<S, GV, 2>(V, ldv, nv, gram, Q, n, partial, mout, qs); break;
    default: block_dot_wave_wide<S, GV, 3>(V, ldv, nv, gram, Q, n, partial, mout, qs); break;
    }
}

// Launches with at most this many basis vectors per wave take the copy
// compiled for the default occupancy also on long vectors: their few
// accumulators leave room for four waves per SIMD, whose loads in flight
// pay more than the hoisted loads of the two-wave schedule (256^3, rounds of
// up to 10: 621 -> 556 us per round's dots).
#ifndef WIDE_DOT_DEFAULT_OCC_GV
#define WIDE_DOT_DEFAULT_OCC_GV 2
#endif
template <int S, int GV>
__global__ void __launch_bounds__(RED_THREADS) RED_WPE_ATTR k_block_dot_wide(const double *__restrict__ V,
                                                                           int64_t ldv, int nv, bool gram,
                                                                           const double *__restrict__ Q, int64_t n,
                                                                           double *__restrict__ partial, int mout) {
    block_dot_body_wide<S, GV>(V, ldv, nv, gram, Q, n, partial, mout);
}

template <int S, int GV>
__global__ void __launch_bounds__(RED_THREADS) k_block_dot_wide_small(const double *__restrict__ V, int64_t ldv,
                                                                      int nv, bool gram,
                                                                      const double *__restrict__ Q, int64_t n,
                                                                      double *__restrict__ partial, int mout) {
    block_dot_body_wide<S, GV>(V, ldv, nv, gram, Q, n, partial, mout);
}

// out_c[j] = vs[j / S] * sum_b partial[b*m + j] for j < nvs (the C entries),
// out_g[j - nvs] = sum_b partial[b*m + j] after (the Gram matrix); b ascending.
__global__ void k_reduce_block(const double *__restrict__ partial, int m, int nb, int S, int nvs,
                               const double *__restrict__ vs, double *__restrict__ out_c,
                               double *__restrict__ out_g) {
    __shared__ double sh[RED_THREADS / WAVE];
    const int j = blockIdx.x;
    double a = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) a += partial[(size_t)b * m + j];
    const double r = block_sum(a, sh);
    if (threadIdx.x == 0) {
        if (j < nvs)
            out_c[j] = r * vs[j / S];
        else
            out_g[j - nvs] = r;
    }
}

// The block vectors orthonormalised in place:
//   Q_t <- sum_{k <= t} (Q_k - sum_i C_ik (vs_i V_i)) Rinv_kt,  t < S,
// cf: C row-major (nv x S), then Rinv row-major (S x S, upper triangular).
// The coefficients (with the basis scales folded in) sit in LDS; the basis
// is streamed past the caches, the new vectors are stored cacheable (the
// last one is the next preconditioner input, the others are read by the
// next block's dots).
constexpr int BLK_VCHUNK = 32;  // basis vectors per dot launch (4 waves x 8)
template <int S>
__device__ __forceinline__ void block_update_body(const double *__restrict__ V, int64_t ldv, int nv,
                                                  const double *__restrict__ vs, const double *__restrict__ cf,
                                                  double *__restrict__ Q, int64_t n) {
    __shared__ double cs[(KMAX + GMRES_BLOCK_MAX) * GMRES_BLOCK_MAX];
    for (int t = threadIdx.x; t < nv * S; t += blockDim.x) cs[t] = cf[t] * vs[t / S];
    for (int t = threadIdx.x; t < S * S; t += blockDim.x) cs[nv * S + t] = cf[nv * S + t];
    __syncthreads();
    const double *__restrict__ ri = cs + nv * S;
    typedef double d2v __attribute__((ext_vector_type(2)));
    const int64_t n2 = n >> 1;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n2; c += (int64_t)gridDim.x * blockDim.x) {
        d2v q[S];
#pragma unroll
        for (int k = 0; k < S; k++) q[k] = reinterpret_cast<const d2v *>(Q + (size_t)k * ldv)[c];
        // CH basis values in flight at a time (fewer for wide rounds: their
        // coefficients of a chunk are held in registers too)
        constexpr int CH = S <= 6 ? 8 : 4;
        int i = 0;
        for (; i + CH <= nv; i += CH) {
            d2v v[CH];
#pragma unroll
            for (int u = 0; u < CH; u++)
                v[u] = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(V + (size_t)(i + u) * ldv) + c);
#pragma unroll
            for (int u = 0; u < CH; u++)
#pragma unroll
                for (int k = 0; k < S; k++) {
                    const double a = cs[(i + u) * S + k];
                    q[k].x -= a * v[u].x;
                    q[k].y -= a * v[u].y;
                }
        }
        for (; i < nv; i++) {
            const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(V + (size_t)i * ldv) + c);
#pragma unroll
            for (int k = 0; k < S; k++) {
                const double a = cs[i * S + k];
                q[k].x -= a * v.x;
                q[k].y -= a * v.y;
            }
        }
        // times Rinv, in place from the last column down (column t uses k <= t)
#pragma unroll
        for (int t = S - 1; t >= 0; t--) {
            d2v o = q[0] * ri[t];
#pragma unroll
            for (int k = 1; k <= t; k++) {
                o.x += q[k].x * ri[k * S + t];
                o.y += q[k].y * ri[k * S + t];
            }
            q[t] = o;
        }
#pragma unroll
        for (int k = 0; k < S; k++) reinterpret_cast<d2v *>(Q + (size_t)k * ldv)[c] = q[k];
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        double q[S];
#pragma unroll
        for (int k = 0; k < S; k++) q[k] = Q[(size_t)k * ldv + n - 1];
        for (int i = 0; i < nv; i++) {
            const double v = V[(size_t)i * ldv + n - 1];
#pragma unroll
            for (int k = 0; k < S; k++) q[k] -= cs[i * S + k] * v;
        }
#pragma unroll
        for (int t = S - 1; t >= 0; t--) {
            double o = q[0] * ri[t];
#pragma unroll
            for (int k = 1; k <= t; k++) o += q[k] * ri[k * S + t];
            q[t] = o;
        }
#pragma unroll
        for (int k = 0; k < S; k++) Q[(size_t)k * ldv + n - 1] = q[k];
    }
}

template <int S>
__global__ void __launch_bounds__(RED_THREADS) RED_WPE_ATTR k_block_update(const double *__restrict__ V, int64_t ldv,
                                                                         int nv, const double *__restrict__ vs,
                                                                         const double *__restrict__ cf,
                                                                         double *__restrict__ Q, int64_t n) {
    block_update_body<S>(V, ldv, nv, vs, cf, Q, n);
}

template <int S>
__global__ void __launch_bounds__(RED_THREADS) k_block_update_small(const double *__restrict__ V, int64_t ldv,
                                                                    int nv, const double *__restrict__ vs,
                                                                    const double *__restrict__ cf,
                                                                    double *__restrict__ Q, int64_t n) {
    block_update_body<S>(V, ldv, nv, vs, cf, Q, n);
}

__global__ void k_dot(const double *__restrict__ x, const double *__restrict__ y, int64_t n,
                      double *__restrict__ partial) {
    __shared__ double sh[RED_THREADS / WAVE];
    double acc = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        acc += x[c] * y[c];
    double r = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// partial[b*3 + 0] = max |x|, +1 = sum x, +2 = sum x^2
__global__ void k_norms(const double *__restrict__ x, int64_t n, double *__restrict__ partial) {
    __shared__ double sh[RED_THREADS / WAVE];
    double mx = 0.0, s = 0.0, s2 = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        double v = x[c];
        double a = fabs(v);
        mx = (a > mx || a != a) ? a : mx;
        s += v;
        s2 += v * v;
    }
    double r0 = block_max(mx, sh);
    double r1 = block_sum(s, sh);
    double r2 = block_sum(s2, sh);
    if (threadIdx.x == 0) {
        partial[(size_t)blockIdx.x * 3 + 0] = r0;
        partial[(size_t)blockIdx.x * 3 + 1] = r1;
        partial[(size_t)blockIdx.x * 3 + 2] = r2;
    }
}

__global__ void k_rel_length(const double *__restrict__ d, const double *__restrict__ u, int64_t n,
                             double *__restrict__ partial) {
    __shared__ double sh[RED_THREADS / WAVE];
    double mx = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        double a = fabs(u[c]);
        double r = fabs(d[c]) / (a > 1.0 ? a : 1.0);
        mx = (r > mx || r != r) ? r : mx;
    }
    double r0 = block_max(mx, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r0;
}

__global__ void k_scale(double *__restrict__ x, double a, int64_t n) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) x[c] *= a;
}

__global__ void k_scale_dev(double *__restrict__ x, const double *__restrict__ s, int64_t n) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) x[c] /= s[0];
}

__global__ void k_axpby(double a, const double *__restrict__ x, double b, double *__restrict__ y, int64_t n) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) y[c] = a * x[c] + b * y[c];
}

__global__ void k_xpay_to(const double *__restrict__ x, double a, const double *__restrict__ y,
                          double *__restrict__ z, int64_t n) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) z[c] = x[c] + a * y[c];
}

template <class TX>
__global__ void k_add_to(double *__restrict__ y, const TX *__restrict__ x, int64_t n) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) y[c] += (double)x[c];
}

__global__ void k_lincomb(const double *__restrict__ V, int64_t ldv, int k, const double *__restrict__ cf,
                          const double *__restrict__ vs, double *__restrict__ y, int64_t n) {
    __shared__ double cs[KMAX];
    for (int i = threadIdx.x; i < k; i += blockDim.x) cs[i] = cf[i] * vs[i];
    __syncthreads();
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    // eight basis values are loaded before their products (the sum keeps the
    // order i = 0, 1, ...); the basis is streamed past the caches
    double s = 0.0;
    int i = 0;
    for (; i + 8 <= k; i += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) v[u] = __builtin_nontemporal_load(V + (size_t)(i + u) * ldv + c);
#pragma unroll
        for (int u = 0; u < 8; u++) s += cs[i + u] * v[u];
    }
    for (; i < k; i++) s += cs[i] * __builtin_nontemporal_load(V + (size_t)i * ldv + c);
    y[c] = s;
}

__global__ void k_scale_copy(const double *__restrict__ x, const double *__restrict__ sp, double *__restrict__ y,
                             int64_t n) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) y[c] = x[c] * sp[0];
}

__global__ void k_b_minus(const double *__restrict__ b, double *__restrict__ y, int64_t n) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) y[c] = b[c] - y[c];
}

__global__ void k_negate_to(const double *__restrict__ x, double *__restrict__ y, int64_t n) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) y[c] = -x[c];
}

template <class TA, class TB>
__global__ void k_cast(const TA *__restrict__ a, TB *__restrict__ b, int64_t n) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) b[c] = convert<TB>(a[c]);
}

__global__ void k_fill_i32(int32_t *x, int32_t v, int64_t n) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) x[c] = v;
}

__global__ void k_fill_u64(unsigned long long *x, unsigned long long v, int64_t n) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) x[c] = v;
}

__global__ void k_fill_f64(double *x, double v, int64_t n) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) x[c] = v;
}

// ---- exclusive scan (3 phases: block sums, scan of block sums, add) ----
constexpr int SCAN_TPB = 256;
constexpr int SCAN_PER_THREAD = 8;
constexpr int SCAN_CHUNK = SCAN_TPB * SCAN_PER_THREAD;

__device__ inline int64_t block_scan_excl(int64_t v, int64_t *sh, int64_t *total) {
    // Hillis-Steele in LDS (SCAN_TPB entries)
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < SCAN_TPB; o <<= 1) {
        int64_t t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t incl = sh[threadIdx.x];
    *total = sh[SCAN_TPB - 1];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_blocksums(const int64_t *__restrict__ in, int64_t n, int64_t *__restrict__ bsum) {
    __shared__ int64_t sh[SCAN_TPB];
    int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    int64_t s = 0;
    for (int t = 0; t < SCAN_PER_THREAD; t++)
        if (base + t < n) s += in[base + t];
    int64_t tot;
    (void)block_scan_excl(s, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void k_scan_top(int64_t *__restrict__ bsum, int64_t nb) {
    // single block: exclusive scan of nb block sums, in place
    __shared__ int64_t sh[SCAN_TPB];
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += SCAN_TPB) {
        int64_t i = base + threadIdx.x;
        int64_t v = i < nb ? bsum[i] : 0;
        int64_t tot;
        int64_t ex = block_scan_excl(v, sh, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
}

__global__ void k_scan_final(const int64_t *__restrict__ in, int64_t n, const int64_t *__restrict__ boff,
                             int64_t *__restrict__ out) {
    __shared__ int64_t sh[SCAN_TPB];
    int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    int64_t vals[SCAN_PER_THREAD];
    int64_t s = 0;
    for (int t = 0; t < SCAN_PER_THREAD; t++) {
        vals[t] = (base + t < n) ? in[base + t] : 0;
        s += vals[t];
    }
    int64_t tot;
    int64_t ex = block_scan_excl(s, sh, &tot);
    int64_t run = boff[blockIdx.x] + ex;
    for (int t = 0; t < SCAN_PER_THREAD; t++) {
        if (base + t < n) out[base + t] = run;
        run += vals[t];
    }
    if (base + SCAN_PER_THREAD >= n && base < n) out[n] = run;  // the thread holding the last element
}

}  // namespace

#define RICH_CASES_1_64(X)                                                                                    \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) \
    X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32) X(33) X(34) X(35) X(36)   \
    X(37) X(38) X(39) X(40) X(41) X(42) X(43) X(44) X(45) X(46) X(47) X(48) X(49) X(50) X(51) X(52) X(53)   \
    X(54) X(55) X(56) X(57) X(58) X(59) X(60) X(61) X(62) X(63) X(64)

rich_status launch_multidot(const double *V, int64_t ldv, int k, const double *vs, const double *w, int64_t n,
                            double *partial, double *out, hipStream_t s) {
    if (k < 1 || k > 64 || (ldv & 1)) return RICH_EINVAL;
    switch (k) {
#define X(K)                                                                         \
    case K:                                                                          \
        if (n >= RED_WIDE_MIN)                                                       \
            k_multidot<K><<<RED_BLOCKS, RED_THREADS, 0, s>>>(V, ldv, w, n, partial); \
        else                                                                         \
            k_multidot_small<K><<<RED_BLOCKS, RED_THREADS, 0, s>>>(V, ldv, w, n, partial); \
        break;
        RICH_CASES_1_64(X)
#undef X
    }
    LAUNCH_CHECK();
    k_reduce_partials<<<k + 1, RED_THREADS, 0, s>>>(partial, k + 1, RED_BLOCKS, out, vs, k);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status launch_update_norm(const double *V, int64_t ldv, int k, const double *h, const double *vs, double *w,
                               int64_t n, double *partial, double *out, hipStream_t s) {
    if (k < 1 || k > 64 || (ldv & 1)) return RICH_EINVAL;
    switch (k) {
#define X(K)                                                                            \
    case K:                                                                             \
        if (n >= RED_WIDE_MIN)                                                          \
            k_update_norm<K><<<RED_BLOCKS, RED_THREADS, 0, s>>>(V, ldv, h, vs, w, n, partial); \
        else                                                                            \
            k_update_norm_small<K><<<RED_BLOCKS, RED_THREADS, 0, s>>>(V, ldv, h, vs, w, n, partial); \
        break;
        RICH_CASES_1_64(X)
#undef X
    }
    LAUNCH_CHECK();
    k_reduce_partials<<<1, RED_THREADS, 0, s>>>(partial, 1, RED_BLOCKS, out);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status launch_block_dot(const double *V, int64_t ldv, int nv, const double *vs, const double *Q, int S,
                             int64_t n, double *partial, double *out, hipStream_t s) {
    if (nv < 1 || nv > KMAX || S < 1 || S > GMRES_BLOCK_MAX || (ldv & 1)) return RICH_EINVAL;
    const bool wide = n >= RED_WIDE_MIN;
    // basis vectors per launch: 4 waves x 8, x 6 for rounds of 7..10
    const int chunk = S <= 6 ? BLK_VCHUNK : 24;
    double *pc = partial;
    for (int i0 = 0; i0 < nv; i0 += chunk) {
        const int nc = nv - i0 < chunk ? nv - i0 : chunk;
        const bool gram = i0 == 0;
        const int gv = (nc + 3) / 4;
        const int mout = nc * S + (gram ? S * (S + 1) / 2 : 0);
        const double *Vc = V + (size_t)i0 * ldv;
        switch (S * 16 + gv) {
#define XG(SS, G)                                                                                         \
    case SS * 16 + G:                                                                                     \
        if (wide)                                                                                         \
            k_block_dot<SS, G><<<RED_BLOCKS, RED_THREADS, 0, s>>>(Vc, ldv, nc, gram, Q, n, pc, mout);       \
        else                                                                                              \
            k_block_dot_small<SS, G><<<RED_BLOCKS, RED_THREADS, 0, s>>>(Vc, ldv, nc, gram, Q, n, pc, mout); \
        break;
#define XS(SS) XG(SS, 1) XG(SS, 2) XG(SS, 3) XG(SS, 4) XG(SS, 5) XG(SS, 6) XG(SS, 7) XG(SS, 8)
            XS(1) XS(2) XS(3) XS(4) XS(5) XS(6)
#undef XS
#undef XG
#define XG(SS, G)                                                                                              \
    case SS * 16 + G:                                                                                          \
        if (wide && G > WIDE_DOT_DEFAULT_OCC_GV)                                                               \
            k_block_dot_wide<SS, G><<<RED_BLOCKS, RED_THREADS, 0, s>>>(Vc, ldv, nc, gram, Q, n, pc, mout);       \
        else                                                                                                   \
            k_block_dot_wide_small<SS, G><<<RED_BLOCKS, RED_THREADS, 0, s>>>(Vc, ldv, nc, gram, Q, n, pc, mout); \
        break;
#define XS(SS) XG(SS, 1) XG(SS, 2) XG(SS, 3) XG(SS, 4) XG(SS, 5) XG(SS, 6)
            XS(7) XS(8) XS(9) XS(10)
#undef XS
#undef XG
        default: return RICH_EINVAL;
        }
        LAUNCH_CHECK();
        k_reduce_block<<<mout, RED_THREADS, 0, s>>>(pc, mout, RED_BLOCKS, S, nc * S, vs + i0, out + (size_t)i0 * S,
                                                    out + (size_t)nv * S);
        LAUNCH_CHECK();
        pc += (size_t)RED_BLOCKS * mout;
    }
    return RICH_OK;
}

rich_status launch_block_update(const double *V, int64_t ldv, int nv, const double *vs, const double *cf, double *Q,
                                int S, int64_t n, hipStream_t s) {
    if (nv < 1 || nv > KMAX || S < 1 || S > GMRES_BLOCK_MAX || (ldv & 1)) return RICH_EINVAL;
    const bool wide = n >= RED_WIDE_MIN;
    switch (S) {
#define X(SS)                                                                                             \
    case SS:                                                                                              \
        if (wide)                                                                                         \
            k_block_update<SS><<<RED_BLOCKS, RED_THREADS, 0, s>>>(V, ldv, nv, vs, cf, Q, n);              \
        else                                                                                              \
            k_block_update_small<SS><<<RED_BLOCKS, RED_THREADS, 0, s>>>(V, ldv, nv, vs, cf, Q, n);        \
        break;
        X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10)
#undef X
    default: return RICH_EINVAL;
    }
    LAUNCH_CHECK();
    return RICH_OK;
}

int block_partial_size(int nv, int S) { return nv * S + S * (S + 1) / 2; }

rich_status launch_dot(const double *x, const double *y, int64_t n, double *partial, double *out, hipStream_t s) {
    k_dot<<<RED_BLOCKS, RED_THREADS, 0, s>>>(x, y, n, partial);
    LAUNCH_CHECK();
    k_reduce_partials<<<1, RED_THREADS, 0, s>>>(partial, 1, RED_BLOCKS, out);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status launch_norms(const double *x, int64_t n, double *partial, double *out, hipStream_t s) {
    k_norms<<<RED_BLOCKS, RED_THREADS, 0, s>>>(x, n, partial);
    LAUNCH_CHECK();
    k_reduce_max<<<1, RED_THREADS, 0, s>>>(partial, 3, RED_BLOCKS, out);
    LAUNCH_CHECK();
    k_reduce_partials<<<2, RED_THREADS, 0, s>>>(partial + 1, 3, RED_BLOCKS, out + 1);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status launch_rel_length(const double *d, const double *u, int64_t n, double *partial, double *out,
                              hipStream_t s) {
    k_rel_length<<<RED_BLOCKS, RED_THREADS, 0, s>>>(d, u, n, partial);
    LAUNCH_CHECK();
    k_reduce_max<<<1, RED_THREADS, 0, s>>>(partial, 1, RED_BLOCKS, out);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status launch_scale(double *x, double a, int64_t n, hipStream_t s) {
    k_scale<<<nblocks(n), TPB, 0, s>>>(x, a, n);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status launch_scale_dev(double *x, const double *inv_of, int64_t n, hipStream_t s) {
    k_scale_dev<<<nblocks(n), TPB, 0, s>>>(x, inv_of, n);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status launch_axpby(double a, const double *x, double b, double *y, int64_t n, hipStream_t s) {
    k_axpby<<<nblocks(n), TPB, 0, s>>>(a, x, b, y, n);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status launch_xpay_to(const double *x, double a, const double *y, double *z, int64_t n, hipStream_t s) {
    k_xpay_to<<<nblocks(n), TPB, 0, s>>>(x, a, y, z, n);
    LAUNCH_CHECK();
    return RICH_OK;
}

template <class TX>
rich_status launch_add_to(double *y, const TX *x, int64_t n, hipStream_t s) {
    k_add_to<TX><<<nblocks(n), TPB, 0, s>>>(y, x, n);
    LAUNCH_CHECK();
    return RICH_OK;
}
template rich_status launch_add_to<double>(double *, const double *, int64_t, hipStream_t);
template rich_status launch_add_to<float>(double *, const float *, int64_t, hipStream_t);

rich_status launch_lincomb(const double *V, int64_t ldv, int k, const double *c, const double *vs, double *y,
                           int64_t n, hipStream_t s) {
    k_lincomb<<<nblocks(n), TPB, 0, s>>>(V, ldv, k, c, vs, y, n);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status launch_scale_copy(const double *x, const double *sp, double *y, int64_t n, hipStream_t s) {
    k_scale_copy<<<nblocks(n), TPB, 0, s>>>(x, sp, y, n);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status launch_b_minus(const double *b, double *y, int64_t n, hipStream_t s) {
    k_b_minus<<<nblocks(n), TPB, 0, s>>>(b, y, n);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status launch_negate_to(const double *x, double *y, int64_t n, hipStream_t s) {
    k_negate_to<<<nblocks(n), TPB, 0, s>>>(x, y, n);
    LAUNCH_CHECK();
    return RICH_OK;
}

template <class TA, class TB>
rich_status launch_cast(const TA *a, TB *b, int64_t n, hipStream_t s) {
    k_cast<TA, TB><<<nblocks(n), TPB, 0, s>>>(a, b, n);
    LAUNCH_CHECK();
    return RICH_OK;
}
template rich_status launch_cast<double, float>(const double *, float *, int64_t, hipStream_t);
template rich_status launch_cast<float, double>(const float *, double *, int64_t, hipStream_t);
template rich_status launch_cast<double, double>(const double *, double *, int64_t, hipStream_t);
template rich_status launch_cast<float, float>(const float *, float *, int64_t, hipStream_t);

rich_status launch_fill_i32(int32_t *x, int32_t v, int64_t n, hipStream_t s) {
    if (n == 0) return RICH_OK;
    k_fill_i32<<<nblocks(n), TPB, 0, s>>>(x, v, n);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status launch_fill_u64(unsigned long long *x, unsigned long long v, int64_t n, hipStream_t s) {
    if (n == 0) return RICH_OK;
    k_fill_u64<<<nblocks(n), TPB, 0, s>>>(x, v, n);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status launch_fill_f64(double *x, double v, int64_t n, hipStream_t s) {
    if (n == 0) return RICH_OK;
    k_fill_f64<<<nblocks(n), TPB, 0, s>>>(x, v, n);
    LAUNCH_CHECK();
    return RICH_OK;
}

rich_status launch_set_scale(double *vs, const double *ww, hipStream_t s) {
    k_set_scale<<<1, 64, 0, s>>>(vs, ww);
    LAUNCH_CHECK();
    return RICH_OK;
}

int64_t scan_tmp_size(int64_t n) { return (n + SCAN_CHUNK - 1) / SCAN_CHUNK + 1; }

rich_status scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s) {
    if (n == 0) {
        HIP_TRY(hipMemsetAsync(out, 0, sizeof(int64_t), s));
        return RICH_OK;
    }
    int64_t nb = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    k_scan_blocksums<<<(unsigned)nb, SCAN_TPB, 0, s>>>(in, n, tmp);
    LAUNCH_CHECK();
    k_scan_top<<<1, SCAN_TPB, 0, s>>>(tmp, nb);
    LAUNCH_CHECK();
    k_scan_final<<<(unsigned)nb, SCAN_TPB, 0, s>>>(in, n, tmp, out);
    LAUNCH_CHECK();
    return RICH_OK;
}

}  // namespace rich
