// so_rdm.h -- one-particle reduced density matrix from the shadows
// (Supp. "Reduced Density Matrices").
//
// For a product of two Majoranas the shadow estimator is
// C(2n,2)/C(n,1) pf(i C'_s|_{mu nu}) = (2n - 1) i C'_s[mu][nu], so the whole
// Majorana two-point matrix is M = (2n - 1)/S sum_s C'_s with
//   sum_s C'_s = X - X^T,   X = sum_{s, j} beta_{s,j} q_{s,2j} q_{s,2j+1}^T,
// q_{s,r} the rows of Q_s and beta_{s,j} = (-1)^{b_{s,j}} (C_b Q is a signed
// swap of row pairs).  X is one dense contraction over K = n S row pairs; it
// runs on v_mfma_f64_16x16x4f64 with the rows read straight from Q (each
// element of Q is read once), a partial X per block, then a fixed-order sum.
// The fermionic elements follow from gamma_{2j-1} = a_j + a_j^dag,
// gamma_{2j} = -i (a_j - a_j^dag) (eqs. majorana_op, 1rdm_off_diagonal,
// 1rdm_diagonal), 0-based: mode p <-> Majoranas 2p, 2p+1 and, with
// <gamma_mu gamma_nu> = i M[mu][nu] (mu != nu),
//   <a_p^dag a_q> = 1/4 (<g_2p g_2q> + i <g_2p g_2q+1> - i <g_2p+1 g_2q> + <g_2p+1 g_2q+1>)
//   <a_p^dag a_p> = 1/2 (1 + i <g_2p g_2p+1>).
#pragma once
#include "so_common.h"

// grid: blocks of 4 waves; block b takes shadows [b spb, (b+1) spb), its
// wave w the sub-range [w sw, (w+1) sw) of it (sw = ceil(spb / 4)); the four
// partial X are added in LDS in wave order and the block writes its X
// (DP x DP, row-major) to part[b].  Lane l, k-step: row pair k = 4 step +
// l/16 of the wave's range (pair k = (shadow k / n, j = k % n)), tile I of
// A holds beta q_{2j}[16 I + l%16] and tile J of B holds q_{2j+1}[16 J + l%16].
template <int T>
__global__ __launch_bounds__(256) void k_rdm_partial(int n, const double *__restrict__ Q,
                                                     const uint64_t *__restrict__ bits, int64_t S, int64_t spb,
                                                     double *__restrict__ part) {
    constexpr int DP = 16 * T;
    __shared__ double Xl[DP * DP];
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, c = l & 15, g = l >> 4;
    const int d = 2 * n;
    const int64_t sw = (spb + 3) / 4;
    const int64_t b0 = (int64_t)blockIdx.x * spb, b1 = min(S, b0 + spb);
    const int64_t s0 = min(b1, b0 + wv * sw), s1 = min(b1, s0 + sw);
    so_d4 X[T][T];
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = 0; J < T; ++J) X[I][J] = so_d4{0.0, 0.0, 0.0, 0.0};
    if (s0 < s1) {
        const int64_t kend = (s1 - s0) * n;   // row pairs of the range
        // this lane's row pair: shadow s, pair j (k = g, g + 4, ...); the
        // operands of the next step are loaded before this step's products
        int64_t s = s0;
        int j = g;
        while (j >= n) { j -= n; ++s; }
        double a[T], b[T];
        auto load = [&](int64_t kk) {
            const bool live = kk < kend;
            const int64_t sl = live ? s : s0;
            const int jl = live ? j : 0;
            const double *q0 = Q + (size_t)sl * d * d + (size_t)(2 * jl) * d;
            const double beta = ((bits[sl] >> jl) & 1u) ? -1.0 : 1.0;
#pragma unroll
            for (int I = 0; I < T; ++I) {
                const int col = 16 * I + c;
                a[I] = (live && col < d) ? beta * q0[col] : 0.0;
                b[I] = (live && col < d) ? q0[d + col] : 0.0;
            }
            j += 4;
            while (j >= n) { j -= n; ++s; }
        };
        load(g);
        for (int64_t k = g; k - g < kend; k += 4) {
            double ac[T], bc[T];
#pragma unroll
            for (int I = 0; I < T; ++I) {
                ac[I] = a[I];
                bc[I] = b[I];
            }
            if (k - g + 4 < kend) load(k + 4);
#pragma unroll
            for (int I = 0; I < T; ++I)
#pragma unroll
                for (int J = 0; J < T; ++J) X[I][J] = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[I], bc[J], X[I][J], 0, 0, 0);
        }
    }
    // register r of tile (I, J) holds X[16 I + 4 r + l/16][16 J + l%16];
    // the waves add their X into Xl one after the other (fixed order)
    for (int v = 0; v < 4; ++v) {
        if (wv == v) {
#pragma unroll
            for (int I = 0; I < T; ++I)
#pragma unroll
                for (int J = 0; J < T; ++J)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int e = (16 * I + 4 * r + g) * DP + 16 * J + c;
                        Xl[e] = (v == 0) ? X[I][J][r] : Xl[e] + X[I][J][r];
                    }
        }
        __syncthreads();
    }
    double *out = part + (size_t)blockIdx.x * DP * DP;
    for (int e = threadIdx.x; e < DP * DP; e += 256) out[e] = Xl[e];
}

// Xsum[e] = sum over the nw block partials, deterministic: block b takes
// entries [64 b, 64 b + 64); thread (group h, entry i) sums the partials
// h, h + 16, ... in order, then the 16 group sums are added in group order.
__global__ __launch_bounds__(1024) void k_rdm_sum(int dp2, int nw, const double *__restrict__ part,
                                                  double *__restrict__ Xsum) {
    __shared__ double gs[16][64];
    const int i = threadIdx.x & 63, h = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + i;
    double acc = 0.0;
    if (e < dp2)
        for (int w = h; w < nw; w += 16) acc += part[(size_t)w * dp2 + e];
    gs[h][i] = acc;
    __syncthreads();
    if (h == 0 && e < dp2) {
        double t = 0.0;
        for (int q = 0; q < 16; ++q) t += gs[q][i];
        Xsum[e] = t;
    }
}

// M = (2n-1)/S (X - X^T) (zero diagonal) into majorana[d][d] (if given) and
// the n x n matrix <a_p^dag a_q> (times 2 for the trial state) into rdm.
// One block of 256 threads.
__global__ __launch_bounds__(256) void k_rdm_out(int n, int DP, const double *__restrict__ Xsum, double scale,
                                                 double trial, double *__restrict__ majorana,
                                                 double2 *__restrict__ rdm) {
    const int d = 2 * n;
    auto Mv = [&](int mu, int nu) -> double {
        return mu == nu ? 0.0 : scale * (Xsum[mu * DP + nu] - Xsum[nu * DP + mu]);
    };
    if (majorana)
        for (int e = threadIdx.x; e < d * d; e += 256) majorana[e] = Mv(e / d, e % d);
    for (int e = threadIdx.x; e < n * n; e += 256) {
        const int p = e / n, q = e % n;
        double2 v;
        if (p == q) {
            // 1/2 (1 + i <g_2p g_2p+1>) with <g g> = i M
            v = c_make(0.5 * (1.0 - Mv(2 * p, 2 * p + 1)), 0.0);
        } else {
            // 1/4 (i M_{2p,2q} - M_{2p,2q+1} + M_{2p+1,2q} + i M_{2p+1,2q+1})
            v = c_make(0.25 * (-Mv(2 * p, 2 * q + 1) + Mv(2 * p + 1, 2 * q)),
                       0.25 * (Mv(2 * p, 2 * q) + Mv(2 * p + 1, 2 * q + 1)));
        }
        rdm[e] = c_scale(v, trial);
    }
}
