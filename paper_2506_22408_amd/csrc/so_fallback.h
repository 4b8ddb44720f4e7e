// so_fallback.h -- full-size path for the pairs whose elimination met a zero
// pivot or too much growth (so_pair.h, so_form.h).  Rare on Haar shadows;
// on signed-permutation shadows with single-mode walkers (the first steps of
// a run on the paper's ensemble) most pairs land here, so the operands are
// staged in LDS once per pair.  For every node e_j of the reduced table it
// takes the Pfaffian of B + e_j J (m x m, J materialised) by Householder
// tridiagonalisation with the matrix in LDS, lane = row, and the pair value
// o = sum_j v_j Pf(B + e_j J).  Q(c) = Pf(B + c J) has degree ne = n - eta in
// c, so its values at the ne + 1 nodes of the table determine the estimator
// exactly; no block of B has to be invertible, so the value is exact to
// rounding whatever B_KK is.
//
// Work: first the queue of flagged pairs; then, only if the queue overflowed,
// a scan of the pair array for the pairs marked SO_PAIR_MARK (so_common.h).
// Every flagged pair therefore reaches this path.  The grid is fixed; blocks
// stride over the queue, whose length is read on the device, and over the
// pair array.
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
// Returns the same value in every lane.  Starts and ends with a barrier.  With
// act = false the wave neither reads nor writes and only keeps the barriers
// (the second wave of a two-wave workgroup); its return value is then
// meaningless.
__device__ __forceinline__ double2 hh_pf_lds(double2 *A, int lda, int m, double2 *ubuf, double2 *ybuf, int q,
                                             bool act = true) {
    __syncthreads();
    double2 pf = c_make(1, 0);
    for (int k = 0; k < m; k += 2) {
        const double2 x = (act && q > k && q < m) ? A[q * lda + k] : c_make(0, 0);
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
        if (act && q >= k + 1 && q < m) ubuf[q] = c_conj(u);
        __syncthreads();
        double2 y = c_make(0, 0);
        if (act && q >= k + 2 && q < m)
            for (int j = k + 1; j < m; ++j) y = c_fma(A[q * lda + j], ubuf[j], y);
        y = c_scale(y, beta);
        if (act && q >= k + 2 && q < m) ybuf[q] = y;
        __syncthreads();
        if (act && q >= k + 2 && q < m)
            for (int j = k + 2; j < m; ++j)
                A[q * lda + j] = c_fma(u, ybuf[j], c_fma(c_neg(y), c_conj(ubuf[j]), A[q * lda + j]));
        __syncthreads();
    }
    __syncthreads();
    return pf;
}

// Two Pfaffians at once for m <= 32, one per 32-lane half of the wave: half
// h = l / 32 works on A + h hA with its vectors at u + h hv, y + h hv (lane
// q = l % 32 = row); otherwise as hh_pf_lds.  Every lane of a half returns
// its half's value.  Starts and ends with a barrier.
__device__ __forceinline__ double2 hh_pf_lds2(double2 *A0, int lda, int m, double2 *u0, double2 *y0, int hA, int hv,
                                              int l) {
    const int h = l >> 5, q = l & 31;
    double2 *A = A0 + h * hA;
    double2 *ubuf = u0 + h * hv;
    double2 *ybuf = y0 + h * hv;
    __syncthreads();
    double2 pf = c_make(1, 0);
    for (int k = 0; k < m; k += 2) {
        const double2 x = (q > k && q < m) ? A[q * lda + k] : c_make(0, 0);
        const double nx2 = grp_sum<32>(c_abs2(x));
        const double2 xf = grp_bcast<32>(x, k + 1);
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

// Dynamic LDS of k_fallback (bytes), m = 2n - eta, d = 2n: the staged
// operands C' (d x d) and Xall (d x (d + 1), rows padded to an odd stride),
// which the node matrices overlay once B is built (two of m x (m + 1)
// complex for m <= 32, when the two halves of the wave take a node each,
// else one); then B (m x m complex), kept across the nodes; then the
// Householder vectors (2m complex per node matrix), the first d of which
// also serve as the formation's row buffer.
__host__ __device__ inline int fb_node_mats(int n, int eta) { return 2 * n - eta <= 32 ? 2 : 1; }
__host__ __device__ inline size_t fb_stage_bytes(int n, int eta) {
    const size_t m = (size_t)(2 * n - eta), d = (size_t)(2 * n);
    size_t stage = (d * d + d * (d + 1)) * sizeof(double);
    const size_t a = (size_t)fb_node_mats(n, eta) * m * (m + 1) * sizeof(double2);
    if (a > stage) stage = a;
    return (stage + 15) & ~(size_t)15;
}
__host__ __device__ inline size_t fb_lds_bytes(int n, int eta) {
    const size_t m = (size_t)(2 * n - eta);
    return fb_stage_bytes(n, eta) + (m * m + 2 * m * fb_node_mats(n, eta)) * sizeof(double2);
}

// o_ws of walker w and shadow s on the full-size path (one wave); lds is the
// block's dynamic LDS (fb_lds_bytes).  Every lane returns the value.
__device__ __forceinline__ double2 fb_pair(int n, int eta, const double *__restrict__ Xa,
                                           const double *__restrict__ Ca, const RedTab &tab, int Ke, int64_t w,
                                           int64_t s, char *lds, int q) {
    const int d = 2 * n, m = 2 * n - eta, ne = n - eta, LDA = m + 1, LX = d + 1;
    const int T = so_tiles(n), DP = 16 * T;
    const double *Xw = Xa + (size_t)w * DP * DP;
    const double *C = Ca + (size_t)s * DP * DP;
    double *Cs = reinterpret_cast<double *>(lds);
    double *Xr = Cs + d * d;
    double2 *A = reinterpret_cast<double2 *>(lds);
    double2 *Bl = reinterpret_cast<double2 *>(lds + fb_stage_bytes(n, eta));
    double2 *ubuf = Bl + m * m;
    double2 *ybuf = ubuf + m;
    double2 *trow = ubuf;   // d <= 2m complex
    __syncthreads();        // the previous pair's reads are done
    // both operands in storage order (coalesced), to row-major LDS
    for (int f = q; f < DP * DP; f += 64) {
        int row, col;
        ao_rowcol(f, T, row, col);
        if (row < d && col < d) {
            Cs[row * d + col] = C[f];
            Xr[row * LX + col] = Xw[f];
        }
    }
    __syncthreads();
    // X[i] = Xall[i] + i Xall[eta + i] for an occupied row, Xall[eta + i] (real) otherwise
    auto xel = [&](int i, int mu) -> double2 {
        return i < eta ? c_make(Xr[i * LX + mu], Xr[(eta + i) * LX + mu]) : c_make(Xr[(eta + i) * LX + mu], 0.0);
    };
    // B = X C' X^T, one row per step: trow = X[i] C', then B[i][q] = trow . X[q]
    for (int i = 0; i < m; ++i) {
        double2 acc = c_make(0, 0);
        if (q < d)
            for (int mu = 0; mu < d; ++mu) acc = c_fma(xel(i, mu), c_make(Cs[mu * d + q], 0.0), acc);
        __syncthreads();   // the previous row's reads of trow are done
        if (q < d) trow[q] = acc;
        __syncthreads();
        if (q < m) {
            double2 b = c_make(0, 0);
            for (int nu = 0; nu < d; ++nu) b = c_fma(trow[nu], xel(q, nu), b);
            Bl[i * m + q] = b;
        }
    }
    __syncthreads();
    double2 o = c_make(0, 0);
    if (fb_node_mats(n, eta) == 2) {
        // two nodes per pass, one per 32-lane half
        const int h = q >> 5, qq = q & 31, hA = m * LDA;
        for (int node = 0; node < Ke; node += 2) {
            const int jn = node + h;
            const bool live = jn < Ke;
            const double2 ck = tab.e[live ? jn : node];
            double2 *Ah = A + h * hA;
            __syncthreads();
            if (qq < m)
                for (int j = 0; j < m; ++j) {
                    double2 v = (j > qq) ? Bl[qq * m + j] : ((j < qq) ? c_neg(Bl[j * m + qq]) : c_make(0, 0));
                    if (qq >= eta && j >= eta) {
                        const int t = qq - eta;
                        if (j - eta == 2 * ne - 1 - t) v = c_add(v, c_scale(ck, t < ne ? 1.0 : -1.0));
                    }
                    Ah[qq * LDA + j] = v;
                }
            const double2 pf = hh_pf_lds2(A, LDA, m, ubuf, ubuf + m, hA, 2 * m, q);
            if (live) o = c_fma(tab.v[jn], pf, o);
        }
        // each half holds its nodes' share: the total in every lane
        return c_make(o.x + __shfl_xor(o.x, 32, 64), o.y + __shfl_xor(o.y, 32, 64));
    }
    for (int node = 0; node < Ke; ++node) {
        const double2 ck = tab.e[node];
        __syncthreads();
        if (q < m)
            for (int j = 0; j < m; ++j) {
                // exact antisymmetry: the lower triangle is the negated upper one
                double2 v = (j > q) ? Bl[q * m + j] : ((j < q) ? c_neg(Bl[j * m + q]) : c_make(0, 0));
                if (q >= eta && j >= eta) {
                    const int t = q - eta;
                    if (j - eta == 2 * ne - 1 - t) v = c_add(v, c_scale(ck, t < ne ? 1.0 : -1.0));
                }
                A[q * LDA + j] = v;
            }
        __syncthreads();
        const double2 pf = hh_pf_lds(A, LDA, m, ubuf, ybuf, q);
        o = c_fma(tab.v[node], pf, o);
    }
    return o;
}

// any grid, 64 threads, fb_lds_bytes(n, eta) of dynamic LDS.  pairs is
// [W][S_total]; Ke = ne + 1 nodes of the reduced table.
__global__ __launch_bounds__(64) void k_fallback(int n, int eta, const double *__restrict__ Xa,
                                                 const double *__restrict__ Ca, RedTab tab, int Ke,
                                                 const so_u64 *__restrict__ fb_count,
                                                 const int64_t *__restrict__ fb_list, int64_t fb_cap, int64_t W,
                                                 int64_t S_total, double2 *__restrict__ pairs) {
    extern __shared__ __align__(16) char fb_lds[];
    const int q = threadIdx.x;
    const int64_t queued = (int64_t)(*fb_count);
    const int64_t cnt = min(queued, fb_cap);
    for (int64_t e = blockIdx.x; e < cnt; e += gridDim.x) {
        const int64_t gs = fb_list[e];
        const int64_t w = gs / S_total, s = gs - w * S_total;
        const double2 o = fb_pair(n, eta, Xa, Ca, tab, Ke, w, s, fb_lds, q);
        if (q == 0) pairs[gs] = o;
    }
    if (queued <= fb_cap) return;
    // the queue overflowed: the pairs it could not hold carry the mark.  Each
    // block scans its own 64-pair chunks; a found pair is written only by the
    // block that found it, and no queued pair is ever marked.
    const int64_t total = W * S_total;
    for (int64_t base = (int64_t)blockIdx.x * 64; base < total; base += (int64_t)gridDim.x * 64) {
        const int64_t e = base + q;
        const bool mk = e < total && so_is_pair_mark(pairs[e]);
        unsigned long long mask = __ballot(mk);
        while (mask) {
            const int b = __ffsll(mask) - 1;
            mask &= mask - 1;
            const int64_t gs = base + b;
            const int64_t w = gs / S_total, s = gs - w * S_total;
            const double2 o = fb_pair(n, eta, Xa, Ca, tab, Ke, w, s, fb_lds, q);
            if (q == 0) pairs[gs] = o;
        }
    }
}
