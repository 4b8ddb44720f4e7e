// so_nodes.h -- node Pfaffians Pf(S + e_j J) of the Schur complement
// S (M2 x M2, M2 = 2(n - eta)) at the ne + 1 nodes e_j of the node table, and the
// weighted node sum per pair (so_common.h, node table).
//
// In the compact order every row of S belongs to an empty orbital and J
// pairs row t with row M2-1-t: J[t][M2-1-t] = +1, J[M2-1-t][t] = -1 (t < M2/2).
//
// Pfaffian by Householder tridiagonalisation (the unitary alternative to
// Parlett-Reid among Wimmer's Pfaffian algorithms): at even step k the
// column x = A[k+1:, k] is mapped to alpha e_1 by H = I - beta u u^H on the
// indices k+1..M2-1; H A H^T = H A conj(H) keeps A skew, multiplies Pf by
// det H = -1 and leaves A[k][k+1] = -alpha, so Pf gains the factor alpha.
// The trailing block is updated by the skew rank-2 form
//   A <- A + beta (u y^T - y u^T),  y = A conj(u),
// and the Pfaffian continues on the indices k+2..M2-1.  There is no pivot
// search and no row exchange: the data flow is static, so every broadcast
// source is a compile-time lane and every register index a constant (each
// step is its own template instance).  J is never stored: the registers hold
// S and the J terms are added to x and y explicitly.
//
// Mappings (one node matrix per 16-lane DPP row, 4 per wave):
//   M2 <= 16: lane q owns row q (pf1_step);
//   M2 <= 32: lane q < M2/2 owns rows q and M2-1-q (pf2_step), so a lane
//             holds a J pair and the rows retired from the top are spread;
//   larger M2: one node per wave, lane = row, broadcasts through LDS.
#pragma once
#include "so_common.h"

// ---- M2 <= 16, lane q owns row q ------------------------------------------------
struct Nd1Ctx {
    int q;
    bool act;
    double2 ck;
};

template <int M2>
__device__ __forceinline__ double2 partner_val(double2 v, int q) {
    if constexpr (M2 == 16) return mirror16c(v);          // lane 15 - q
    else if constexpr (M2 == 8) return mirror8c(v);       // lane 7 - q
    else return grp_bcast<16>(v, (M2 - 1 - q) & 15);
}

// HJ = false: the matrix is the registers alone (no c J term; ck unused)
template <int M2, int K, bool HJ = true>
__device__ __forceinline__ void pf1_step(const Nd1Ctx &cx, double2 (&R)[M2], double2 &pf) {
    const int q = cx.q;
    // x_i = A[i][K] for rows i > K; J[i][K] != 0 only for i = M2-1-K, which is
    // still active iff K < M2/2, and then J[i][K] = -1
    double2 x = c_sel(cx.act && q > K, R[K], c_make(0, 0));
    if constexpr (HJ && K < M2 / 2) x = c_sel(cx.act && q == M2 - 1 - K, c_sub(x, cx.ck), x);
    const double nx2 = sum16(c_abs2(x));
    const double2 xf = bc16c<K + 1>(x);
    const double nx = sqrt(nx2);
    const double ax = sqrt(c_abs2(xf));
    const double iax = 1.0 / (ax > 0.0 ? ax : 1.0);
    const double2 phs = c_make(ax > 0.0 ? xf.x * iax : 1.0, ax > 0.0 ? xf.y * iax : 0.0);
    const double2 alpha = c_scale(phs, -nx);
    pf = c_mul(pf, alpha);
    if constexpr (K + 2 < M2) {
        const double beta = (nx > 0.0 ? 1.0 : 0.0) / (nx > 0.0 ? nx2 + nx * ax : 1.0);
        const double2 u = c_sel(q == K + 1, c_sub(xf, alpha), x);
        const double2 v = c_conj(u);
        // y_i = sum_{j>K} A_ij conj(u_j)
        double2 y = c_make(0, 0);
        {
            double d2 = nx, d1 = nx;
            [&]<int... I>(std::integer_sequence<int, I...>) {
                (([&] {
                     constexpr int j = K + 1 + I;
                     y = c_fma(R[j], bc16cd<j>(v, d2), y);
                     d2 = d1;
                     d1 = y.x;
                 }()), ...);
            }(std::make_integer_sequence<int, M2 - K - 1>{});
        }
        if constexpr (HJ) {   // J[q][M2-1-q] conj(u_{M2-1-q}), with J[q][.] = +1 for q < M2/2, -1 otherwise
            const double2 vp = partner_val<M2>(v, q);
            const int p = M2 - 1 - q;
            const double2 t = c_fma(c_scale(cx.ck, q < M2 / 2 ? 1.0 : -1.0), vp, y);
            y = c_sel(cx.act && p > K, t, y);
        }
        y = c_scale(y, beta);
        const double2 ny = c_neg(y);
        // A_ij += u_i y_j - y_i u_j for j >= K+2
        {
            double d2 = ny.x, d1 = ny.y;
            [&]<int... I>(std::integer_sequence<int, I...>) {
                (([&] {
                     constexpr int j = K + 2 + I;
                     const double2 yb = bc16cd<j>(y, d2);
                     const double2 ub = bc16cd<j>(u, d2);
                     R[j] = c_fma(u, yb, c_fma(ny, ub, R[j]));
                     d2 = d1;
                     d1 = R[j].x;
                 }()), ...);
            }(std::make_integer_sequence<int, M2 - K - 2>{});
        }
        pf1_step<M2, K + 2, HJ>(cx, R, pf);
    }
}

// ---- M2 <= 32, lane q < M2/2 owns rows q and M2-1-q ---------------------------------
struct Nd2Ctx {
    int q;
    bool act;
    double2 ck;
};

template <int M, int J>
__device__ __forceinline__ double2 row_val(double2 v0, double2 v1) {
    if constexpr (J < M / 2) return bc16c<J>(v0);
    else return bc16c<M - 1 - J>(v1);
}
template <int M, int J>
__device__ __forceinline__ double2 row_val_dep(double2 v0, double2 v1, double dep) {
    if constexpr (J < M / 2) return bc16cd<J>(v0, dep);
    else return bc16cd<M - 1 - J>(v1, dep);
}

template <int M, int K>
__device__ __forceinline__ void pf2_step(const Nd2Ctx &cx, double2 (&R0)[M], double2 (&R1)[M], double2 &pf) {
    constexpr int L = M / 2;
    const int q = cx.q;
    const int rb = M - 1 - q;
    // x_i = A[i][K] for the owned rows i > K.  J[q][M-1-q] would lie in column
    // K only for q = M-1-K < K, a retired row, so only the slot-1 row meets J.
    double2 x0 = c_sel(cx.act && q > K, R0[K], c_make(0, 0));
    double2 x1 = c_sel(cx.act && rb > K, R1[K], c_make(0, 0));
    x1 = c_sel(cx.act && q == K, c_sub(x1, cx.ck), x1);      // J[M-1-q][q] = -1
    const double nx2 = sum16(c_abs2(x0) + c_abs2(x1));
    const double2 xf = row_val<M, K + 1>(x0, x1);
    const double nx = sqrt(nx2);
    const double ax = sqrt(c_abs2(xf));
    const double iax = 1.0 / (ax > 0.0 ? ax : 1.0);
    const double2 phs = c_make(ax > 0.0 ? xf.x * iax : 1.0, ax > 0.0 ? xf.y * iax : 0.0);
    const double2 alpha = c_scale(phs, -nx);
    pf = c_mul(pf, alpha);
    if constexpr (K + 2 < M) {
        const double beta = (nx > 0.0 ? 1.0 : 0.0) / (nx > 0.0 ? nx2 + nx * ax : 1.0);
        const double2 piv = c_sub(xf, alpha);
        double2 u0 = x0, u1 = x1;
        if constexpr (K + 1 < L) u0 = c_sel(q == K + 1, piv, x0);
        else u1 = c_sel(q == M - 2 - K, piv, x1);
        const double2 v0 = c_conj(u0), v1 = c_conj(u1);
        double2 y0 = c_make(0, 0), y1 = c_make(0, 0);
        {
            double d2 = nx, d1 = nx;
            [&]<int... I>(std::integer_sequence<int, I...>) {
                (([&] {
                     constexpr int j = K + 1 + I;
                     const double2 ub = row_val_dep<M, j>(v0, v1, d2);
                     y0 = c_fma(R0[j], ub, y0);
                     y1 = c_fma(R1[j], ub, y1);
                     d2 = d1;
                     d1 = y0.x;
                 }()), ...);
            }(std::make_integer_sequence<int, M - K - 1>{});
        }
        {   // J terms couple the lane's own two rows
            const double2 t0 = c_fma(cx.ck, v1, y0);
            const double2 t1 = c_sub(y1, c_mul(cx.ck, v0));
            y0 = c_sel(cx.act && rb > K, t0, y0);
            y1 = c_sel(cx.act && q > K, t1, y1);
        }
        y0 = c_scale(y0, beta);
        y1 = c_scale(y1, beta);
        const double2 ny0 = c_neg(y0), ny1 = c_neg(y1);
        {
            double d2 = ny0.x, d1 = ny1.x;
            [&]<int... I>(std::integer_sequence<int, I...>) {
                (([&] {
                     constexpr int j = K + 2 + I;
                     const double2 yb = row_val_dep<M, j>(y0, y1, d2);
                     const double2 ub = row_val_dep<M, j>(u0, u1, d2);
                     R0[j] = c_fma(u0, yb, c_fma(ny0, ub, R0[j]));
                     R1[j] = c_fma(u1, yb, c_fma(ny1, ub, R1[j]));
                     d2 = d1;
                     d1 = R0[j].x;
                 }()), ...);
            }(std::make_integer_sequence<int, M - K - 2>{});
        }
        pf2_step<M, K + 2>(cx, R0, R1, pf);
    }
}

// ---- the node kernel ---------------------------------------------------------
// One wave handles PPB = 4 consecutive pairs of a chunk: their 4 K (pair,
// node) items run K rounds on the 4 lane groups; the node values go to LDS
// and each pair's sum is taken in node order (deterministic), then scaled by
// the pair's pfo.  RPL = rows per lane (1 or 2).
template <int M2, int RPL>
__global__ __launch_bounds__(64) void k_nodes(const double2 *__restrict__ Sbuf, const double2 *__restrict__ Pbuf,
                                              NodeTab tab, int64_t npairs, int64_t S_total, int64_t s0, int Sc,
                                              double2 *__restrict__ pairs) {
    constexpr int PPB = 4;
    __shared__ double2 vals[PPB * SO_KMAX];
    const int lane = threadIdx.x;
    const int g = lane >> 4, q = lane & 15;
    const int64_t P0 = (int64_t)blockIdx.x * PPB;
    const int K = tab.Ke;
    for (int r = 0; r < K; ++r) {
        const int item = r * PPB + g;
        const int pl = item / K, node = item - pl * K;
        const int64_t pair = (P0 + pl < npairs) ? P0 + pl : P0;
        double2 pf = c_make(1, 0);
        if constexpr (M2 > 0 && RPL == 1) {
            Nd1Ctx cx;
            cx.q = q;
            cx.act = q < M2;
            cx.ck = tab.e[node];
            const double2 *row = Sbuf + pair * (M2 * M2) + (cx.act ? q : 0) * M2;
            double2 R[M2];
#pragma unroll
            for (int j = 0; j < M2; ++j) R[j] = row[j];
            pf1_step<M2, 0>(cx, R, pf);
        } else if constexpr (M2 > 0) {
            Nd2Ctx cx;
            cx.q = q;
            cx.act = q < M2 / 2;
            cx.ck = tab.e[node];
            const double2 *row0 = Sbuf + pair * (M2 * M2) + (cx.act ? q : 0) * M2;
            const double2 *row1 = Sbuf + pair * (M2 * M2) + (cx.act ? M2 - 1 - q : 0) * M2;
            double2 R0[M2], R1[M2];
#pragma unroll
            for (int j = 0; j < M2; ++j) {
                R0[j] = row0[j];
                R1[j] = row1[j];
            }
            pf2_step<M2, 0>(cx, R0, R1, pf);
        }
        if (q == 0) vals[item] = c_mul(pf, tab.v[node]);
    }
    __syncthreads();
    if (lane < PPB) {
        const int64_t pair = P0 + lane;
        if (pair < npairs) {
            double2 acc = c_make(0, 0);
            for (int node = 0; node < K; ++node) acc = c_add(acc, vals[lane * K + node]);
            const double2 pb = Pbuf[pair];
            const int64_t w = pair / Sc, sl = pair - w * Sc;
            pairs[w * S_total + s0 + sl] = so_is_pair_mark(pb) ? pb : c_mul(acc, pb);
        }
    }
}

// ---- 32 < M2 <= SO_MMAX: one node per wave, lane = row, LDS broadcasts --------------------
__global__ __launch_bounds__(64) void k_nodes_wide(int M2, const double2 *__restrict__ Sbuf,
                                                   const double2 *__restrict__ Pbuf, NodeTab tab, int64_t npairs,
                                                   int64_t S_total, int64_t s0, int Sc,
                                                   double2 *__restrict__ pairs) {
    __shared__ double2 A[SO_MMAX * (SO_MMAX + 1)];
    __shared__ double2 ubuf[SO_MMAX];
    __shared__ double2 ybuf[SO_MMAX];
    const int q = threadIdx.x;
    const int64_t pair = blockIdx.x;
    const double2 *Sg = Sbuf + pair * (int64_t)M2 * M2;
    const int LDA = SO_MMAX + 1;
    double2 acc = c_make(0, 0);
    for (int node = 0; node < tab.Ke; ++node) {
        const double2 ck = tab.e[node];
        __syncthreads();
        if (q < M2)
            for (int j = 0; j < M2; ++j) {
                double2 v = Sg[q * M2 + j];
                if (j == M2 - 1 - q) v = c_add(v, c_scale(ck, q < M2 / 2 ? 1.0 : -1.0));
                A[q * LDA + j] = v;
            }
        __syncthreads();
        double2 pf = c_make(1, 0);
        for (int k = 0; k < M2; k += 2) {
            const double2 x = (q > k && q < M2) ? A[q * LDA + k] : c_make(0, 0);
            const double nx2 = grp_sum<64>(c_abs2(x));
            const double2 xf = grp_bcast<64>(x, k + 1);
            const double nx = sqrt(nx2);
            const double ax = sqrt(c_abs2(xf));
            const double2 phs = ax > 0.0 ? c_scale(xf, 1.0 / ax) : c_make(1, 0);
            const double2 alpha = c_scale(phs, -nx);
            pf = c_mul(pf, alpha);
            if (k + 2 >= M2) break;
            const double beta = nx > 0.0 ? 1.0 / (nx2 + nx * ax) : 0.0;
            const double2 u = (q == k + 1) ? c_sub(xf, alpha) : x;
            if (q >= k + 1 && q < M2) ubuf[q] = c_conj(u);
            __syncthreads();
            double2 y = c_make(0, 0);
            if (q >= k + 2 && q < M2)
                for (int j = k + 1; j < M2; ++j) y = c_fma(A[q * LDA + j], ubuf[j], y);
            y = c_scale(y, beta);
            if (q >= k + 2 && q < M2) ybuf[q] = y;
            __syncthreads();
            if (q >= k + 2 && q < M2)
                for (int j = k + 2; j < M2; ++j)
                    A[q * LDA + j] = c_fma(u, ybuf[j], c_fma(c_neg(y), c_conj(ubuf[j]), A[q * LDA + j]));
            __syncthreads();
        }
        acc = c_fma(tab.v[node], pf, acc);
    }
    if (q == 0) {
        const double2 pb = Pbuf[pair];
        const int64_t w = pair / Sc, sl = pair - w * Sc;
        pairs[w * S_total + s0 + sl] = so_is_pair_mark(pb) ? pb : c_mul(acc, pb);
    }
}
