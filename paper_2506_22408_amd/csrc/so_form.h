// so_form.h -- pair formation and the node-independent part of the node
// Pfaffians.
//
// For a pair (w, s) the node matrices are A_k = s_k B + c_k J with
// B = X C' X^T (eq. b_mat) and J the selected vacuum covariance (eq. a_mat),
// which vanishes on the occupied rows and columns.  Eliminating the occupied
// indices first by pairwise (Parlett-Reid) steps therefore never touches J:
//   Pf(s B + c J) = s^{eta/2} Pf(B_OO) Pf(s S + c J),
//   S = B_UU - B_UO B_OO^{-1} B_OU,
// so S (2ne x 2ne, ne = n - eta) and pfo = Pf(B_OO) are computed once per
// pair and every node works on the smaller matrix s S + c J.  Pivoting is
// confined to the occupied block; when it meets a zero pivot or S grows
// beyond SO_SCHUR_GROWTH x max|B| the pair is queued for the full-size path
// (so_fallback.h), which uses no elimination shortcut.
#pragma once
#include "so_common.h"

#define FORM_RB 8                 // rows of T = X C' held at a time
#define SO_SCHUR_GROWTH 1.0e3

__device__ __forceinline__ double block_max256(double v, double *red) {
    v = fmax(v, __shfl_xor(v, 32, 64));
    v = fmax(v, __shfl_xor(v, 16, 64));
    v = fmax(v, __shfl_xor(v, 8, 64));
    v = fmax(v, __shfl_xor(v, 4, 64));
    v = fmax(v, __shfl_xor(v, 2, 64));
    v = fmax(v, __shfl_xor(v, 1, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    return r;
}

// grid (W, ceil(Sc / spb)), 256 threads.  Dynamic LDS: X (m x 2n), T block
// (FORM_RB x 2n), B (m x (m+1)) as complex, then C' (2n x 2n) as real when
// cs_lds (else C' is read from global memory).
__global__ __launch_bounds__(256) void k_form_schur(int n, int eta, const double2 *__restrict__ X,
                                                    const double *__restrict__ Cp, int64_t S_total, int64_t s0,
                                                    int Sc, int spb, int cs_lds, double2 *__restrict__ Sbuf,
                                                    double2 *__restrict__ Pbuf, uint32_t *__restrict__ fb_count,
                                                    int64_t *__restrict__ fb_list, int64_t fb_cap,
                                                    int32_t *__restrict__ wstat) {
    extern __shared__ double2 lds2[];
    __shared__ double red[4];
    __shared__ int s_piv;
    __shared__ double s_pmax;
    const int d = 2 * n, m = 2 * n - eta, M2 = m - eta, LDB = m + 1;
    double2 *Xs = lds2;
    double2 *Ts = Xs + m * d;
    double2 *Bs = Ts + FORM_RB * d;
    double *Cs = reinterpret_cast<double *>(Bs + m * LDB);
    const int tid = threadIdx.x;
    const int w = blockIdx.x;
    const double2 *Xg = X + (size_t)w * m * d;
    for (int e = tid; e < m * d; e += 256) Xs[e] = Xg[e];
    const int sl0 = blockIdx.y * spb;
    const int sl1 = min(Sc, sl0 + spb);
    for (int sl = sl0; sl < sl1; ++sl) {
        const double *Cg = Cp + (size_t)(s0 + sl) * d * d;
        __syncthreads();
        if (cs_lds)
            for (int e = tid; e < d * d; e += 256) Cs[e] = Cg[e];
        const double *Csrc = cs_lds ? Cs : Cg;
        double lmax = 0.0;
        // B = X C' X^T, upper triangle computed, lower written as its negation
        for (int i0 = 0; i0 < m; i0 += FORM_RB) {
            const int rb = min(FORM_RB, m - i0);
            __syncthreads();
            for (int e = tid; e < rb * d; e += 256) {
                const int i = i0 + e / d, nu = e % d;
                double ar = 0.0, ai = 0.0;
                for (int mu = 0; mu < d; ++mu) {
                    const double2 xv = Xs[i * d + mu];
                    const double c = Csrc[mu * d + nu];
                    ar = fma(xv.x, c, ar);
                    ai = fma(xv.y, c, ai);
                }
                Ts[e] = c_make(ar, ai);
            }
            __syncthreads();
            for (int e = tid; e < rb * m; e += 256) {
                const int i = i0 + e / m, j = e % m;
                if (j < i) continue;
                double2 acc = c_make(0, 0);
                if (j > i)
                    for (int nu = 0; nu < d; ++nu) acc = c_fma(Ts[(i - i0) * d + nu], Xs[j * d + nu], acc);
                Bs[i * LDB + j] = acc;
                Bs[j * LDB + i] = c_neg(acc);
                lmax = fmax(lmax, c_abs2(acc));
            }
        }
        const double maxB2 = block_max256(lmax, red);   // also orders the B writes
        // eliminate the occupied indices 0..eta-1 pairwise
        double2 pfo = c_make(1, 0);
        bool zero = false;
        for (int k = 0; k < eta; k += 2) {
            if (tid < 64) {
                const int p = k + 1 + tid;
                double v = (p < eta) ? c_abs2(Bs[k * LDB + p]) : -1.0;
                int pi = p;
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
                    const double ov = __shfl_xor(v, off, 64);
                    const int op = __shfl_xor(pi, off, 64);
                    if (ov > v || (ov == v && op < pi)) { v = ov; pi = op; }
                }
                if (tid == 0) { s_piv = pi; s_pmax = v; }
            }
            __syncthreads();
            const int p = s_piv;
            if (!(s_pmax > 0.0)) { zero = true; break; }
            if (p != k + 1) {
                for (int j = tid; j < m; j += 256) {
                    const double2 t = Bs[(k + 1) * LDB + j];
                    Bs[(k + 1) * LDB + j] = Bs[p * LDB + j];
                    Bs[p * LDB + j] = t;
                }
                __syncthreads();
                for (int i = tid; i < m; i += 256) {
                    const double2 t = Bs[i * LDB + k + 1];
                    Bs[i * LDB + k + 1] = Bs[i * LDB + p];
                    Bs[i * LDB + p] = t;
                }
                __syncthreads();
                pfo = c_neg(pfo);
            }
            const double2 a = Bs[k * LDB + k + 1];
            pfo = c_mul(pfo, a);
            const double2 ia = c_inv(a);
            const int rem = m - k - 2;
            // A_ij -= (A_{i,k+1} A_{k,j} - A_{i,k} A_{k+1,j}) / a on the trailing block
            for (int e = tid; e < rem * rem; e += 256) {
                const int i = k + 2 + e / rem, j = k + 2 + e % rem;
                const double2 t = c_sub(c_mul(Bs[i * LDB + k + 1], Bs[k * LDB + j]),
                                        c_mul(Bs[i * LDB + k], Bs[(k + 1) * LDB + j]));
                Bs[i * LDB + j] = c_sub(Bs[i * LDB + j], c_mul(t, ia));
            }
            __syncthreads();
        }
        const int64_t pair = (int64_t)w * Sc + sl;
        double smax = 0.0;
        double2 *Sg = Sbuf + pair * (int64_t)M2 * M2;
        for (int e = tid; e < M2 * M2; e += 256) {
            const double2 v = Bs[(eta + e / M2) * LDB + eta + e % M2];
            Sg[e] = v;
            smax = fmax(smax, c_abs2(v));
        }
        const double maxS2 = block_max256(smax, red);
        const bool flag = zero || !(maxS2 <= SO_SCHUR_GROWTH * SO_SCHUR_GROWTH * maxB2);
        if (tid == 0) {
            Pbuf[pair] = pfo;
            if (flag) {
                const uint32_t idx = atomicAdd(fb_count, 1u);
                if ((int64_t)idx < fb_cap) fb_list[idx] = (int64_t)w * S_total + s0 + sl;
                else atomicOr(&wstat[w], SO_WSTAT_FALLBACK_LOST);
            }
        }
    }
}
