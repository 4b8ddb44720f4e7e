// so_energy.h -- local energy from the shadows (section "Force bias and local
// energy": eqs. local_energy, ham_cholesky_decom, energy_tb_diff,
// Pfaffian_der, Pfaffian_2nd_der).
//
// H = sum_pq t_pq a_p^dag a_q + 1/2 sum_g Lhat_g^2, Lhat_g = sum_pq L^g_pq
// a_p^dag a_q with real symmetric L^g.  A one-body operator moves the walker
// to e^{lambda Lhat}|phi>, which acts on the Majorana rows of X as
// X -> X e^{lambda K}, [Lhat, gamma_rho] = sum_sigma K[rho][sigma] gamma_sigma;
// for a real symmetric L, K = L (x) sigma_y (2 x 2 blocks, sigma_y =
// [[0,-i],[i,0]]), so K^T = -K.  Per node (A = c J + s B, Pf, A^{-1}), with
//   Yt = X^T A^{-1} X,  Z = C' Yt,  W = C' Yt C' = Z C'   (d x d),
// the derivatives of eq. Pfaffian_2nd_der become
//   tr(A^{-1} A'_g)        = 2 s tr(Z K_g),
//   sum_g tr(A^{-1} A''_g) = s tr(Yt M),   M = sum_g (K_g^2 C' + 2 K_g C' K_g^T + C' K_g^T K_g^T),
//   sum_g tr(A^{-1} A'_g A^{-1} A'_g) = s^2 [2 sum_g tr(Z K_g Z K_g) - 2 sum_g tr(Yt K_g W K_g)],
// and with V_pqrs = sum_g L^g_pq L^g_rs
//   sum_g tr(P K_g R K_g) = sum_pqrs V_pqrs tr(P^(sp) sigma_y R^(qr) sigma_y)
// over the 2 x 2 blocks P^(sp), R^(qr): an n^4 contraction per node instead
// of n_gamma products of d x d matrices.  M depends on the shadow only:
//   M = (K2 (x) I) C' + C' (K2 (x) I) - 2 sum_qr V_pqrs sigma_y C'^(qr) sigma_y  (block (p, s)),
// K2 = sum_g L^g L^g.  The node's energy is
//   E = s tr(Z K_t) + 1/4 [s tr(Yt M) - sum_g tr(A^{-1}A'_g A^{-1}A'_g) + 1/2 sum_g tr(A^{-1}A'_g)^2],
// K_t the Majorana matrix of t, and the pair's numerator e = sum_k w_k Pf_k E_k
// beside o = sum_k w_k Pf_k.  The node matrices must be invertible, so the
// nodes avoid z = -1, a root of every pair's Pfaffian when n - eta is odd;
// the host places n - eta + 1 of them a third of a step off the roots of unity.
#pragma once
#include "so_common.h"

#define SO_EN_NMAX 24
#define SO_EN_THREADS 256

struct EnTab {
    double2 s[SO_KMAX];   // node matrices c J + s B
    double2 c[SO_KMAX];
    double2 w[SO_KMAX];   // weights (interpolation, channel, prefactor, row-order sign)
    int K;
};

// Vt[(s n + p) n^2 + q n + r] = V_pqrs = sum_g L[p n + q][g] L[r n + s][g]
__global__ __launch_bounds__(256) void k_energy_v(int n, int ng, const double *__restrict__ L,
                                                  double *__restrict__ Vt) {
    const int n2 = n * n;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n2 * n2) return;
    const int sp = e / n2, qr = e - sp * n2;
    const int s = sp / n, p = sp - s * n, q = qr / n, r = qr - q * n;
    const double *a = L + (size_t)(p * n + q) * ng;
    const double *b = L + (size_t)(r * n + s) * ng;
    double acc = 0.0;
    for (int g = 0; g < ng; ++g) acc = fma(a[g], b[g], acc);
    Vt[e] = acc;
}

// K2 = sum_g L^g L^g (n x n) and Kt, the Majorana matrix of t (d x d):
//   Kt[2r][2q] = Kt[2r+1][2q+1] = (t_qr - t_rq)/2,
//   Kt[2r][2q+1] = -i (t_rq + t_qr)/2,  Kt[2r+1][2q] = i (t_rq + t_qr)/2.
// One block.
__global__ __launch_bounds__(256) void k_energy_small(int n, int ng, const double *__restrict__ L,
                                                      const double2 *__restrict__ t, double *__restrict__ K2,
                                                      double2 *__restrict__ Kt) {
    const int d = 2 * n;
    for (int e = threadIdx.x; e < n * n; e += 256) {
        const int p = e / n, s = e - p * n;
        double acc = 0.0;
        for (int q = 0; q < n; ++q)
            for (int g = 0; g < ng; ++g) acc = fma(L[(size_t)(p * n + q) * ng + g], L[(size_t)(q * n + s) * ng + g], acc);
        K2[e] = acc;
    }
    for (int e = threadIdx.x; e < d * d; e += 256) {
        const int mu = e / d, nu = e - mu * d;
        const int r = mu >> 1, a = mu & 1, q = nu >> 1, b = nu & 1;
        const double2 tqr = t[q * n + r], trq = t[r * n + q];
        double2 v;
        if (a == b) v = c_scale(c_sub(tqr, trq), 0.5);
        else {
            const double2 h = c_scale(c_add(trq, tqr), 0.5);          // (t_rq + t_qr)/2
            v = a == 0 ? c_make(h.y, -h.x) : c_make(-h.y, h.x);       // -i h or i h
        }
        Kt[e] = v;
    }
}

// Per shadow: M = (K2 (x) I) C' + C' (K2 (x) I) - 2 sum_qr V_pqrs sigma_y C'^(qr) sigma_y,
// with sigma_y c sigma_y = [[c11, -c10], [-c01, c00]] for a real 2 x 2 block c.
// Ms [S][d][d] row-major.  One block per shadow; C' read from its A-order copy.
template <int T>
__global__ __launch_bounds__(256) void k_energy_shadow(int n, const double *__restrict__ Ca,
                                                       const double *__restrict__ Vt, const double *__restrict__ K2,
                                                       double *__restrict__ Ms, double *__restrict__ Cr) {
    constexpr int DP = 16 * T;
    __shared__ double C[DP * DP];
    const int d = 2 * n, n2 = n * n;
    const int64_t s0 = blockIdx.x;
    const double *Cg = Ca + s0 * DP * DP;
    for (int e = threadIdx.x; e < d * d; e += 256) {
        const int mu = e / d, nu = e - mu * d;
        const double c = Cg[ao_index(mu, nu, T)];
        C[mu * DP + nu] = c;
        Cr[s0 * d * d + e] = c;
    }
    __syncthreads();
    double *out = Ms + s0 * d * d;
    for (int e = threadIdx.x; e < d * d; e += 256) {
        const int mu = e / d, nu = e - mu * d;
        const int p = mu >> 1, a = mu & 1, s = nu >> 1, b = nu & 1;
        double acc = 0.0;
        for (int q = 0; q < n; ++q) {
            acc = fma(K2[p * n + q], C[(2 * q + a) * DP + nu], acc);
            acc = fma(C[mu * DP + 2 * q + b], K2[q * n + s], acc);
        }
        const double sg = ((a + b) & 1) ? -1.0 : 1.0;
        double v3 = 0.0;
        const double *vrow = Vt + (size_t)(s * n + p) * n2;
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r) v3 = fma(vrow[q * n + r], C[(2 * q + 1 - a) * DP + 2 * r + 1 - b], v3);
        out[e] = acc - 2.0 * sg * v3;
    }
}

__device__ __forceinline__ double en_wsum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Row-major complex copy of the walker matrix X (m x d) from Xall in A order.
template <int T>
__global__ __launch_bounds__(256) void k_energy_walker(int n, int eta, const double *__restrict__ Xa,
                                                       double2 *__restrict__ Xr) {
    constexpr int DP = 16 * T;
    const int d = 2 * n, m = 2 * n - eta;
    const int64_t w0 = blockIdx.x;
    const double *Xg = Xa + w0 * DP * DP;
    for (int e = threadIdx.x; e < m * d; e += 256) {
        const int i = e / d, mu = e - i * d;
        Xr[w0 * m * d + e] = i < eta ? c_make(Xg[ao_index(i, mu, T)], Xg[ao_index(eta + i, mu, T)])
                                     : c_make(Xg[ao_index(eta + i, mu, T)], 0.0);
    }
}

// block-wide sum of two complex values (all threads get the result): a
// fixed-order reduction within each wave, then the four wave sums in order
__device__ __forceinline__ void en_sum2(double2 &a, double2 &b, double2 *red) {
    const int t = threadIdx.x, wv = t >> 6;
    const double ar = en_wsum(a.x), ai = en_wsum(a.y), br = en_wsum(b.x), bi = en_wsum(b.y);
    if ((t & 63) == 0) {
        red[wv] = c_make(ar, ai);
        red[4 + wv] = c_make(br, bi);
    }
    __syncthreads();
    a = c_add(c_add(red[0], red[1]), c_add(red[2], red[3]));
    b = c_add(c_add(red[4], red[5]), c_add(red[6], red[7]));
    __syncthreads();
}

// index and value of the largest |x|^2 among the first 64 threads (a pivot
// search has at most m - 1 <= 47 candidates; ties: smallest index),
// broadcast to the block through one barrier.
__device__ __forceinline__ int en_argmax(double v, int idx, double *rv, int *ri, double &best) {
    const int t = threadIdx.x;
    if (t < 64) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(v, o);
            const int oi = __shfl_xor(idx, o);
            if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
        }
        if (t == 0) { rv[0] = v; ri[0] = idx; }
    }
    __syncthreads();
    best = rv[0];
    return ri[0];
}

// LDS of k_energy_pair, in complex entries: B [m][m], A [max(m^2, 2 n^2)]
// (the node matrix and its inverse, then zeta^T, row stride n + 1), YZ [d][d]
// (A^{-1} X, then Z), Yt [d][d].  X and C' are read through the caches from
// row-major copies.  At n = 16, eta = 8 this is 52 KB: three blocks per CU;
// at most 141 KB (n = 24, eta = 2): one block.
__host__ __device__ inline size_t energy_lds_bytes(int n, int eta) {
    const size_t d = 2 * n, m = 2 * n - eta, n2 = (size_t)n * n;
    const size_t asz = m * m > 2 * n2 ? m * m : 2 * n2;
    return 16 * (m * m + asz + 2 * d * d);
}

// One block of 256 threads per (walker, shadow) pair; grid (S, W).
//   Xa, Ca      walker matrices and shadow covariances in A order (so_prep.h)
//   Ms          per-shadow M (d x d), Vt the n^4 table, Kt (d x d)
//   opair/epair [W][S] complex out: o_ws and the numerator e_ws
// Matrices are row-major with their own row length (d or m).  Up to 16 modes
// three blocks share a CU (168 VGPRs, some spills).  Beyond, the node matrices
// mostly leave LDS for one or two blocks (115 KB at n = 24, eta = 12), and the
// register budget of two blocks avoids the spills (1.26x at that shape).
template <int T>
__global__ __launch_bounds__(SO_EN_THREADS, T == 3 ? 2 : 3) void k_energy_pair(int n_in, int eta_in, const double2 *__restrict__ Xr,
                                                               const double *__restrict__ Cr,
                                                               const double *__restrict__ Ms,
                                                               const double *__restrict__ Vt,
                                                               const double2 *__restrict__ Kt, EnTab tab, int64_t S,
                                                               double2 *__restrict__ opair,
                                                               double2 *__restrict__ epair,
                                                               int32_t *__restrict__ wst) {
    constexpr int DM = 16 * T;                      // bound on d and m
    constexpr int NE = DM * DM / SO_EN_THREADS;     // bound on elements per thread
    extern __shared__ double2 esm[];
    __shared__ double2 red[8];
    __shared__ double rv[1];
    __shared__ int ri[1];
    __shared__ int piv[DM];
    const int t = threadIdx.x;
    const int n = n_in, eta = eta_in;
    const int d = 2 * n, m = 2 * n - eta, ne = n - eta, n2 = n * n;
    const int asz = m * m > 2 * n2 ? m * m : 2 * n2;
    double2 *Bm = esm;                // m x m
    double2 *A = Bm + m * m;          // m x m; later zeta^T (n (n + 1))
    double2 *YZ = A + asz;            // d x d
    double2 *Yt = YZ + d * d;         // d x d
    const int64_t s0 = blockIdx.x, w0 = blockIdx.y;
    const double2 *X = Xr + w0 * m * d;    // m x d, row-major (global, cached)
    const double *C = Cr + s0 * d * d;     // d x d, row-major (global, cached)
    const double *Mg = Ms + s0 * d * d;
    // B = X (C' X^T): YZ[j][mu] = sum_nu C'[mu][nu] X[j][nu], B[i][j] = sum_mu X[i][mu] YZ[j][mu]
    for (int e = t; e < m * d; e += SO_EN_THREADS) {
        const int j = e / d, mu = e - j * d;
        double2 acc = c_make(0.0, 0.0);
        for (int nu = 0; nu < d; ++nu) acc = c_add(acc, c_scale(X[j * d + nu], C[mu * d + nu]));
        YZ[e] = acc;
    }
    __syncthreads();
    for (int e = t; e < m * m; e += SO_EN_THREADS) {
        const int i = e / m, j = e - i * m;
        double2 acc = c_make(0.0, 0.0);
        for (int mu = 0; mu < d; ++mu) acc = c_fma(X[i * d + mu], YZ[j * d + mu], acc);
        Bm[e] = acc;
    }
    __syncthreads();
    double2 osum = c_make(0.0, 0.0), esum = c_make(0.0, 0.0);
    bool singular = false;
    for (int k = 0; k < tab.K; ++k) {
        // the sizes, the LDS layout and the thread index again, through opaque
        // moves: what derives from them is recomputed per node (scalar unit,
        // one vector add) instead of being hoisted out of the node loop and
        // kept live, and spilled, through every stage of it
        int n = n_in, eta = eta_in;
        asm volatile("" : "+s"(n), "+s"(eta));
        int t = threadIdx.x;
        asm volatile("" : "+v"(t));
        const int d = 2 * n, m = 2 * n - eta, ne = n - eta, n2 = n * n;
        const int asz = m * m > 2 * n2 ? m * m : 2 * n2;
        double2 *Bm = esm;
        double2 *A = Bm + m * m;
        double2 *YZ = A + asz;
        double2 *Yt = YZ + d * d;
        // zeta^T with the odd row stride n + 1 (in complex entries): the
        // contraction reads it at a few rows q per wave, which a stride of n
        // would put on the same LDS banks
        const int ZS = n + 1;
        double2 *zetaT = A;
        const double2 *X = Xr + w0 * m * d;
        const double *C = Cr + s0 * d * d;
        const double *Mg = Ms + s0 * d * d;
        auto build_a = [&](double2 sk, double2 ck) {
            for (int e = t; e < m * m; e += SO_EN_THREADS) {
                const int i = e / m, j = e - i * m;
                double2 v = c_mul(sk, Bm[e]);
                if (i >= eta && j >= eta) {
                    const int u = i - eta, v2 = j - eta;
                    if (u < ne && v2 == 2 * ne - 1 - u) v = c_add(v, ck);
                    else if (u >= ne && v2 == 2 * ne - 1 - u) v = c_sub(v, ck);
                }
                A[e] = v;
            }
            __syncthreads();
        };
        const double2 sk = tab.s[k], ck = tab.c[k], wk = tab.w[k];
        // ---- Pf(A) and YZ = A^{-1} X by one pairwise (Parlett-Reid) elimination
        // with partial pivoting that carries X as right-hand sides (A destroyed).
        // Step k eliminates the 2 x 2 pivot [[0, a], [-a, 0]] (a = A[k][k+1]):
        //   A_ij += (A[k+1][i] A[k][j] - A[k][i] A[k+1][j]) / a,   i, j >= k+2,
        //   X_i  += (A[k+1][i] X_k  - A[k][i] X_{k+1}) / a,        i >= k+2,
        // and Pf(A) is the signed product of the pivots.  Rows k, k+1 keep their
        // values as pivot rows, which the back substitution then uses. ----
        build_a(sk, ck);
        for (int e = t; e < m * d; e += SO_EN_THREADS) YZ[e] = X[e];
        __syncthreads();
        double2 pf = c_make(1.0, 0.0);
        bool sing = false;
        for (int kk = 0; kk < m - 1; kk += 2) {
            const int j = kk + 1 + t;
            double best;
            const int p = en_argmax(j < m ? c_abs2(A[kk * m + j]) : -1.0, j < m ? j : m, rv, ri, best);
            if (best == 0.0) { pf = c_make(0.0, 0.0); sing = true; break; }
            if (t == 0) piv[kk] = p;
            if (p != kk + 1) {
                for (int c = t; c < m; c += SO_EN_THREADS) {
                    const double2 x = A[(kk + 1) * m + c];
                    A[(kk + 1) * m + c] = A[p * m + c];
                    A[p * m + c] = x;
                }
                for (int c = t; c < d; c += SO_EN_THREADS) {
                    const double2 x = YZ[(kk + 1) * d + c];
                    YZ[(kk + 1) * d + c] = YZ[p * d + c];
                    YZ[p * d + c] = x;
                }
                __syncthreads();
                for (int r = t; r < m; r += SO_EN_THREADS) {
                    const double2 x = A[r * m + kk + 1];
                    A[r * m + kk + 1] = A[r * m + p];
                    A[r * m + p] = x;
                }
                __syncthreads();
                pf = c_neg(pf);
            }
            const double2 a = A[kk * m + kk + 1];
            pf = c_mul(pf, a);
            const double2 ia = c_inv(a);
            const int rem = m - kk - 2;
            for (int e = t; e < rem * rem; e += SO_EN_THREADS) {
                const int i = kk + 2 + e / rem, jj = kk + 2 + e % rem;
                const double2 num = c_sub(c_mul(A[(kk + 1) * m + i], A[kk * m + jj]),
                                          c_mul(A[kk * m + i], A[(kk + 1) * m + jj]));
                A[i * m + jj] = c_fma(num, ia, A[i * m + jj]);
            }
            for (int e = t; e < rem * d; e += SO_EN_THREADS) {
                const int i = kk + 2 + e / d, mu = e % d;
                const double2 num = c_sub(c_mul(A[(kk + 1) * m + i], YZ[kk * d + mu]),
                                          c_mul(A[kk * m + i], YZ[(kk + 1) * d + mu]));
                YZ[i * d + mu] = c_fma(num, ia, YZ[i * d + mu]);
            }
            __syncthreads();
        }
        osum = c_fma(wk, pf, osum);
        if (sing) {
            singular = true;
            continue;
        }
        // back substitution, last pivot pair first: with r = X~ - sum_{j >= k+2} A[.][j] Y_j
        // over rows k, k+1, the 2 x 2 pivot gives Y_k = -r_{k+1} / a, Y_{k+1} = r_k / a
        for (int kk = m - 2; kk >= 0; kk -= 2) {
            const double2 ia = c_inv(A[kk * m + kk + 1]);
            for (int mu = t; mu < d; mu += SO_EN_THREADS) {
                double2 r0 = YZ[kk * d + mu], r1 = YZ[(kk + 1) * d + mu];
                for (int jj = kk + 2; jj < m; ++jj) {
                    const double2 yj = YZ[jj * d + mu];
                    r0 = c_sub(r0, c_mul(A[kk * m + jj], yj));
                    r1 = c_sub(r1, c_mul(A[(kk + 1) * m + jj], yj));
                }
                YZ[kk * d + mu] = c_neg(c_mul(r1, ia));
                YZ[(kk + 1) * d + mu] = c_mul(r0, ia);
            }
            __syncthreads();
        }
        // undo the symmetric interchanges on the solution, last first
        for (int kk = m - 2; kk >= 0; kk -= 2) {
            const int p = piv[kk];
            if (p != kk + 1) {
                for (int mu = t; mu < d; mu += SO_EN_THREADS) {
                    const double2 x = YZ[(kk + 1) * d + mu];
                    YZ[(kk + 1) * d + mu] = YZ[p * d + mu];
                    YZ[p * d + mu] = x;
                }
                __syncthreads();
            }
        }
        // ---- Yt = X^T YZ, then YZ = Z = C' Yt (a compile-time bound on the
        // elements per thread, so that one thread's accumulations interleave) ----
        {
            double2 acc[NE];
#pragma unroll
            for (int u = 0; u < NE; ++u) acc[u] = c_make(0.0, 0.0);
            for (int i = 0; i < m; ++i)
#pragma unroll
                for (int u = 0; u < NE; ++u) {
                    const int e = t + u * SO_EN_THREADS, a = e / d, b = e - a * d;
                    if (e < d * d) acc[u] = c_fma(X[i * d + a], YZ[i * d + b], acc[u]);
                }
#pragma unroll
            for (int u = 0; u < NE; ++u)
                if (t + u * SO_EN_THREADS < d * d) Yt[t + u * SO_EN_THREADS] = acc[u];
        }
        __syncthreads();
        {
            double2 acc[NE];
#pragma unroll
            for (int u = 0; u < NE; ++u) acc[u] = c_make(0.0, 0.0);
            for (int c = 0; c < d; ++c)
#pragma unroll
                for (int u = 0; u < NE; ++u) {
                    const int e = t + u * SO_EN_THREADS, a = e / d, b = e - a * d;
                    if (e < d * d) acc[u] = c_add(acc[u], c_scale(Yt[c * d + b], C[a * d + c]));
                }
#pragma unroll
            for (int u = 0; u < NE; ++u)
                if (t + u * SO_EN_THREADS < d * d) YZ[t + u * SO_EN_THREADS] = acc[u];
        }
        __syncthreads();
        double2 *Z = YZ;
        // zeta_pq = tr(Z^(qp) sigma_y) = i (Z[2q][2p+1] - Z[2q+1][2p]), and its transpose
        for (int e = t; e < n2; e += SO_EN_THREADS) {
            const int p = e / n, q = e - p * n;
            const double2 df = c_sub(Z[(2 * q) * d + 2 * p + 1], Z[(2 * q + 1) * d + 2 * p]);
            const double2 z = c_make(-df.y, df.x);
            zetaT[q * ZS + p] = z;
        }
        __syncthreads();
        // one-body s tr(Z Kt) and s tr(Yt M)
        double2 one = c_make(0.0, 0.0), bs = c_make(0.0, 0.0);
        for (int e = t; e < d * d; e += SO_EN_THREADS) {
            const int a = e / d, b = e - a * d;
            one = c_fma(Z[e], Kt[b * d + a], one);
            bs = c_add(bs, c_scale(Yt[e], Mg[b * d + a]));
        }
        en_sum2(one, bs, red);
        // c1 = sum V_pqrs tr(Z^(sp) sy Z^(qr) sy), c2 = sum V_pqrs tr(Yt^(sp) sy W^(qr) sy),
        // asq = sum V_pqrs zeta_pq zeta_rs (= sum_g (tr(Z K_g))^2, tr(Z K_g) = sum_pq L^g_pq zeta_pq);
        // tr(P sy R sy) = P00 R11 - P01 R01 - P10 R10 + P11 R00 for 2 x 2 blocks
        double2 c1 = c_make(0.0, 0.0), c2 = c_make(0.0, 0.0), asq = c_make(0.0, 0.0);
        // c1 = sum_sp V tr(Z^(sp) sy Z^(qr) sy) is linear in Z^(sp): with
        // a_ab = sum_sp V_pqrs Z^(sp)_ab,  c1 = sum_qr z11 a00 - z01 a01 - z10 a10 + z00 a11;
        // likewise c2 from b_ab = sum_sp V_pqrs Yt^(sp)_ab and the W^(qr) blocks, and
        // asq = sum_qr sum_s zeta_rs sum_p V_pqrs zeta_pq.  The first half of the
        // threads accumulates a (and asq), the second half b, each thread for the
        // two columns (q, r) = c0 + t' and c0 + t' + half of each chunk of 256
        // columns c0: one LDS read of a 2 x 2 block then feeds both columns.
        for (int c0 = 0; c0 < n2; c0 += SO_EN_THREADS) {
            constexpr int half = SO_EN_THREADS / 2;
            const bool bset = t >= half;
            const int ca = c0 + (bset ? t - half : t), cb = ca + half;
            const bool hb = cb < n2;
            auto contract = [&](auto with_as) {
                constexpr bool AS = decltype(with_as)::value;
                const int qa = ca / n, ra = ca - qa * n;
                const int qb = hb ? cb / n : qa, rb = hb ? cb - qb * n : ra;
                const double *va = Vt + ca, *vb = Vt + (hb ? cb : ca);
                const double2 *src = AS ? Z : Yt;
                double2 x00 = c_make(0.0, 0.0), x01 = x00, x10 = x00, x11 = x00;
                double2 y00 = x00, y01 = x00, y10 = x00, y11 = x00;
                double2 asa = x00, asb = x00;
                for (int s = 0; s < n; ++s) {
                    const double2 *row = src + (2 * s) * d;
                    const size_t so = (size_t)(s * n) * n2;
                    double2 pa = c_make(0.0, 0.0), pb = pa;
                    auto term = [&](int p, double v, double w) {
                        const double2 *blk = row + 2 * p;
                        const double2 e00 = blk[0], e01 = blk[1], e10 = blk[d], e11 = blk[d + 1];
                        x00 = c_add(x00, c_scale(e00, v));
                        x01 = c_add(x01, c_scale(e01, v));
                        x10 = c_add(x10, c_scale(e10, v));
                        x11 = c_add(x11, c_scale(e11, v));
                        y00 = c_add(y00, c_scale(e00, w));
                        y01 = c_add(y01, c_scale(e01, w));
                        y10 = c_add(y10, c_scale(e10, w));
                        y11 = c_add(y11, c_scale(e11, w));
                        if constexpr (AS) {
                            pa = c_add(pa, c_scale(zetaT[qa * ZS + p], v));
                            pb = c_add(pb, c_scale(zetaT[qb * ZS + p], w));
                        }
                    };
                    int p = 0;
                    for (; p + 4 <= n; p += 4) {
                        double v[4], w[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            v[u] = va[so + (size_t)(p + u) * n2];
                            w[u] = vb[so + (size_t)(p + u) * n2];
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) term(p + u, v[u], w[u]);
                    }
                    for (; p < n; ++p) term(p, va[so + (size_t)p * n2], vb[so + (size_t)p * n2]);
                    if constexpr (AS) {
                        asq = c_fma(pa, zetaT[s * ZS + ra], asq);
                        if (hb) asq = c_fma(pb, zetaT[s * ZS + rb], asq);
                    }
                }
                // combine with the column's own block: Z^(qr) for c1, W^(qr) = (Z C')^(qr) for c2
                auto fin = [&](int q, int r, double2 f00, double2 f01, double2 f10, double2 f11) {
                    double2 g00, g01, g10, g11;
                    if constexpr (AS) {
                        g00 = Z[(2 * q) * d + 2 * r];
                        g01 = Z[(2 * q) * d + 2 * r + 1];
                        g10 = Z[(2 * q + 1) * d + 2 * r];
                        g11 = Z[(2 * q + 1) * d + 2 * r + 1];
                    } else {
                        g00 = c_make(0.0, 0.0), g01 = g00, g10 = g00, g11 = g00;
                        for (int c = 0; c < d; ++c) {
                            const double k0 = C[c * d + 2 * r], k1 = C[c * d + 2 * r + 1];
                            const double2 za = Z[(2 * q) * d + c], zb = Z[(2 * q + 1) * d + c];
                            g00 = c_add(g00, c_scale(za, k0));
                            g01 = c_add(g01, c_scale(za, k1));
                            g10 = c_add(g10, c_scale(zb, k0));
                            g11 = c_add(g11, c_scale(zb, k1));
                        }
                    }
                    double2 v = c_mul(g11, f00);
                    v = c_sub(v, c_mul(g01, f01));
                    v = c_sub(v, c_mul(g10, f10));
                    return c_fma(g00, f11, v);
                };
                double2 acc = fin(qa, ra, x00, x01, x10, x11);
                if (hb) acc = c_add(acc, fin(qb, rb, y00, y01, y10, y11));
                if constexpr (AS) c1 = c_add(c1, acc);
                else c2 = c_add(c2, acc);
            };
            if (ca < n2) {
                if (bset) contract(std::integral_constant<bool, false>{});
                else contract(std::integral_constant<bool, true>{});
            }
        }
        en_sum2(c1, c2, red);
        double2 dummy = c_make(0.0, 0.0);
        en_sum2(asq, dummy, red);
        const double2 s2 = c_mul(sk, sk);
        const double2 csum = c_scale(c_mul(s2, c_sub(c1, c2)), 2.0);
        const double2 asum = c_scale(c_mul(s2, asq), 4.0);
        // E = s tr(Z Kt) + 1/4 [s tr(Yt M) - csum + asum / 2]
        double2 E = c_mul(sk, one);
        E = c_add(E, c_scale(c_add(c_sub(c_mul(sk, bs), csum), c_scale(asum, 0.5)), 0.25));
        esum = c_fma(c_mul(wk, pf), E, esum);
        __syncthreads();   // zeta lives in A, which the next node rebuilds
    }
    if (t == 0) {
        const int64_t ix = w0 * S + s0;
        opair[ix] = osum;
        epair[ix] = esum;
        if (singular && wst) atomicOr(wst + w0, SO_WSTAT_SINGULAR);
    }
}

// Per walker, in a fixed order: S_w = (1/S) sum_s o_ws, N_w = (1/S) sum_s e_ws,
// E_w = N_w / S_w; NaN for a walker flagged rank-deficient, as in the overlap
// path, and N_w, E_w NaN for a walker with a singular node matrix.  The pair
// terms were evaluated at the walker's orthonormal factor Qf (Phi = Qf R,
// k_walker_prep); the state, and with it <Psi_T|phi> and <Psi_T|H|phi>, is
// linear in det R, so S_w and N_w are multiplied by det R = exp(logdet[w])
// while E_w comes from the unscaled sums and stays finite where S_w and N_w
// leave the double range.  With scale_pairs the caller's single-shadow terms
// are multiplied by det R as well.  One block of 256 threads per walker.
__global__ __launch_bounds__(256) void k_energy_reduce(int64_t S, double2 *__restrict__ opair,
                                                       double2 *__restrict__ epair, double2 *__restrict__ overlap,
                                                       double2 *__restrict__ numer, double2 *__restrict__ energy,
                                                       int32_t *__restrict__ wst, const double2 *__restrict__ logdet,
                                                       int scale_pairs) {
    __shared__ double2 red[8];
    const int t = threadIdx.x;
    const int64_t w = blockIdx.x;
    const double mg = exp(logdet[w].x);
    const double2 dr = c_make(mg * cos(logdet[w].y), mg * sin(logdet[w].y));
    double2 so = c_make(0.0, 0.0), se = c_make(0.0, 0.0);
    for (int64_t s = t; s < S; s += 256) {
        const double2 o = opair[w * S + s], e = epair[w * S + s];
        so = c_add(so, o);
        se = c_add(se, e);
        if (scale_pairs) {
            opair[w * S + s] = c_mul(o, dr);
            epair[w * S + s] = c_mul(e, dr);
        }
    }
    en_sum2(so, se, red);
    if (t == 0) {
        const double inv = 1.0 / (double)S;
        so = c_scale(so, inv);
        se = c_scale(se, inv);
        if (wst && (wst[w] & SO_WSTAT_RANK)) so = se = c_make(NAN, NAN);
        bool fin = isfinite(so.x) && isfinite(so.y) && isfinite(se.x) && isfinite(se.y);
        // a singular node matrix leaves its energy term undefined: no number
        const bool sing = wst && (wst[w] & SO_WSTAT_SINGULAR);
        if (sing) se = c_make(NAN, NAN);
        const double2 el = c_mul(se, c_inv(so));
        so = c_mul(so, dr);
        se = c_mul(se, dr);
        fin = fin && isfinite(so.x) && isfinite(so.y) && (sing || (isfinite(se.x) && isfinite(se.y)));
        if (wst && !fin) wst[w] |= SO_WSTAT_NONFINITE;
        if (overlap) overlap[w] = so;
        if (numer) numer[w] = se;
        if (energy) energy[w] = el;
    }
}
