// so_fallback.h -- full-size path for the pairs whose occupied-block
// elimination met a zero pivot or too much growth (so_form.h).  Rare and
// simple: recompute B = X C' X^T for the pair, then for every node the
// Pfaffian of A = s_k B + c_k J (m x m, J materialised) by Householder
// tridiagonalisation with the matrix in LDS, lane = row.  No shortcut, so
// it is exact to rounding whatever B_OO is.  The grid is fixed; blocks stride
// over the queue, whose length is read on the device.
#pragma once
#include "so_common.h"

// Row i of the complex walker matrix X from Xall (A order): Re X_O[i] and
// Im X_O[i] for i < eta, X_U[i - eta] (real) otherwise.
__device__ __forceinline__ double2 fb_xrow(const double *Xw, int i, int col, int eta, int T) {
    if (i < eta) return c_make(Xw[ao_index(i, col, T)], Xw[ao_index(eta + i, col, T)]);
    return c_make(Xw[ao_index(eta + i, col, T)], 0.0);
}

// Pfaffian of the m x m complex skew matrix in LDS (row stride lda; the
// upper and lower triangles both present) by Householder tridiagonalisation,
// lane q = row; destroys the matrix.  ubuf, ybuf: m complex of LDS scratch.
// Returns the same value in every lane.  Starts and ends with a barrier.
__device__ __forceinline__ double2 hh_pf_lds(double2 *A, int lda, int m, double2 *ubuf, double2 *ybuf, int q) {
    __syncthreads();
    double2 pf = c_make(1, 0);
    for (int k = 0; k < m; k += 2) {
        const double2 x = (q > k && q < m) ? A[q * lda + k] : c_make(0, 0);
        const double nx2 = grp_sum<64>(c_abs2(x));
        const double2 xf = grp_bcast<64>(x, k + 1);
        const double nx = sqrt(nx2);
        const double ax = sqrt(c_abs2(xf));
        const double2 phs = ax > 0.0 ? c_scale(xf, 1.0 / ax) : c_make(1, 0);
        const double2 alpha = c_scale(phs, -nx);
        pf = c_mul(pf, alpha);
        if (k + 2 >= m) break;
        const double beta = nx > 0.0 ? 1.0 / (nx2 + nx * ax) : 0.0;
        const double2 u = (q == k + 1) ? c_sub(xf, alpha) : x;
        if (q >= k + 1 && q < m) ubuf[q] = c_conj(u);
        __syncthreads();
        double2 y = c_make(0, 0);
        if (q >= k + 2 && q < m)
            for (int j = k + 1; j < m; ++j) y = c_fma(A[q * lda + j], ubuf[j], y);
        y = c_scale(y, beta);
        if (q >= k + 2 && q < m) ybuf[q] = y;
        __syncthreads();
        if (q >= k + 2 && q < m)
            for (int j = k + 2; j < m; ++j)
                A[q * lda + j] = c_fma(u, ybuf[j], c_fma(c_neg(y), c_conj(ubuf[j]), A[q * lda + j]));
        __syncthreads();
    }
    __syncthreads();
    return pf;
}

// grid FB_GRID, 64 threads; Bscratch holds FB_GRID matrices of m x m.
__global__ __launch_bounds__(64) void k_fallback(int n, int eta, const double *__restrict__ Xa,
                                                 const double *__restrict__ Ca, NodeTab tab,
                                                 const uint32_t *__restrict__ fb_count,
                                                 const int64_t *__restrict__ fb_list, int64_t fb_cap, int64_t S_total,
                                                 double2 *__restrict__ Bscratch, double2 *__restrict__ pairs) {
    __shared__ double2 A[SO_MMAX * (SO_MMAX + 1)];
    __shared__ double2 trow[2 * SO_NMAX];
    __shared__ double2 ubuf[SO_MMAX];
    __shared__ double2 ybuf[SO_MMAX];
    const int q = threadIdx.x;
    const int d = 2 * n, m = 2 * n - eta, ne = n - eta, LDA = m + 1;
    const int T = so_tiles(n), DP = 16 * T;
    const int64_t cnt = min((int64_t)(*fb_count), fb_cap);
    double2 *Bg = Bscratch + (size_t)blockIdx.x * m * m;
    for (int64_t e = blockIdx.x; e < cnt; e += gridDim.x) {
        const int64_t gs = fb_list[e];
        const int64_t w = gs / S_total, s = gs - w * S_total;
        const double *Xw = Xa + (size_t)w * DP * DP;
        const double *C = Ca + (size_t)s * DP * DP;
        for (int i = 0; i < m; ++i) {
            __syncthreads();
            if (q < d) {
                double2 acc = c_make(0, 0);
                for (int mu = 0; mu < d; ++mu)
                    acc = c_fma(fb_xrow(Xw, i, mu, eta, T), c_make(C[ao_index(mu, q, T)], 0.0), acc);
                trow[q] = acc;
            }
            __syncthreads();
            if (q < m) {
                double2 acc = c_make(0, 0);
                for (int nu = 0; nu < d; ++nu) acc = c_fma(trow[nu], fb_xrow(Xw, q, nu, eta, T), acc);
                Bg[i * m + q] = acc;
            }
        }
        __syncthreads();
        double2 o = c_make(0, 0);
        for (int node = 0; node < tab.K; ++node) {
            const double2 sk = tab.s[node], ck = tab.c[node];
            __syncthreads();
            if (q < m)
                for (int j = 0; j < m; ++j) {
                    // exact antisymmetry: the lower triangle is the negated upper one
                    double2 v = (j > q) ? Bg[q * m + j] : ((j < q) ? c_neg(Bg[j * m + q]) : c_make(0, 0));
                    v = c_mul(v, sk);
                    if (q >= eta && j >= eta) {
                        const int t = q - eta;
                        if (j - eta == 2 * ne - 1 - t) v = c_add(v, c_scale(ck, t < ne ? 1.0 : -1.0));
                    }
                    A[q * LDA + j] = v;
                }
            __syncthreads();
            const double2 pf = hh_pf_lds(A, LDA, m, ubuf, ybuf, q);
            o = c_fma(tab.wf[node], pf, o);
        }
        if (q == 0) pairs[w * S_total + s] = o;
    }
}
