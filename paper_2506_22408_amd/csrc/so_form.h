// so_form.h -- pair formation on the matrix cores and the node-independent
// part of the node Pfaffians.
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
//
// Formation.  The empty rows of X are real, so with the real d x d matrix
// Xall = [Re X_O; Im X_O; X_U] (so_prep.h) the pair needs two real products,
//   U = C' Xall^T,   P = Xall U = Xall C' Xall^T,
// on v_mfma_f64_16x16x4f64, or on v_mfma_f32_16x16x4f32 with single-precision
// operands and accumulation in the mixed-precision mode (so_common.h for the
// operand orders).  The accumulator of U's tile (I, J), register r, is
// exactly the B operand of P at k-step 4 I + r, so U never leaves the
// registers.  P is antisymmetric;
// only its tiles I <= J are formed.  Then, with i, j < eta and t, u < 2ne,
//   B_OO[i][j] = P[i][j] - P[eta+i][eta+j] + i (P[i][eta+j] + P[eta+i][j])
//   B_OU[i][t] = P[i][2eta+t] + i P[eta+i][2eta+t]
//   B_UU[t][u] = P[2eta+t][2eta+u].
//
// Elimination.  Only the eta occupied rows R = [B_OO | B_OU] are kept (in
// LDS); by antisymmetry every entry the pairwise step needs below them is a
// negated entry of R.  Step k (pivot pair k, k+1, a = R[k][k+1]) adds
//   (R[k+1][i] R[k][j] - R[k][i] R[k+1][j]) / a
// to every trailing entry (i, j), which for i, j empty is a rank-2 update of
// S, accumulated in registers starting from B_UU.
#pragma once
#include "so_common.h"

#define SO_SCHUR_GROWTH 1.0e3

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// LDS (dynamic): P as DP x (DP + 1) doubles, then R as eta x m complex.
__host__ __device__ inline size_t form_lds_bytes_t(int T, int eta, int m) {
    const int DP = 16 * T;
    const size_t pb = ((size_t)DP * (DP + 1) * sizeof(double) + 15) & ~(size_t)15;
    return pb + (size_t)eta * m * sizeof(double2);
}

// grid (W, ceil(Sc / spw)), one wave per block: walker blockIdx.x, shadows
// s0 + [blockIdx.y spw, ...) of the chunk.  NS >= ceil((2ne)^2 / 64) entries
// of S per lane: lane l holds S[e / M2][e % M2], e = l + 64 q.
template <int T, int NS, bool MIX>
__global__ __launch_bounds__(64) void k_form_mfma(int n, int eta, const void *__restrict__ Xa,
                                                  const void *__restrict__ Ca, int64_t S_total, int64_t s0,
                                                  int Sc, int spw, double2 *__restrict__ Sbuf,
                                                  double2 *__restrict__ Pbuf, so_u64 *__restrict__ fb_count,
                                                  int64_t *__restrict__ fb_list, int64_t fb_cap,
                                                  int32_t *__restrict__ wstat) {
    constexpr int KK = 4 * T, DP = 16 * T, LDP = DP + 1;
    // operands in FP64 (MIX = false) or single precision (MIX = true)
    using Op = typename std::conditional<MIX, float, double>::type;
    using Vec = typename std::conditional<MIX, float4, double2>::type;
    using Acc = typename std::conditional<MIX, so_f4, so_d4>::type;
    constexpr int MATV = DP * DP * (int)sizeof(Op) / (int)sizeof(Vec);   // vectors per stored matrix
    extern __shared__ double lds[];
    double *Pl = lds;
    double2 *Rl = reinterpret_cast<double2 *>(reinterpret_cast<char *>(lds) +
                                              ((DP * LDP * sizeof(double) + 15) & ~(size_t)15));
    const int l = threadIdx.x;
    const int w = blockIdx.x;
    const int m = 2 * n - eta, ne = n - eta, M2 = 2 * ne;

    Op xa[T][KK];
    load_ops<T>(static_cast<const Vec *>(Xa) + (size_t)w * MATV, xa, l);
    // P[a][b] for any a, b < DP from the stored tiles I <= J
    auto Pget = [&](int a, int b) -> double {
        return ((a >> 4) <= (b >> 4)) ? Pl[a * LDP + b] : -Pl[b * LDP + a];
    };

    const int sl0 = blockIdx.y * spw;
    const int sl1 = min(Sc, sl0 + spw);
    for (int sl = sl0; sl < sl1; ++sl) {
        Op ca[T][KK];
        load_ops<T>(static_cast<const Vec *>(Ca) + (size_t)(s0 + sl) * MATV, ca, l);
        Acc P[T][T], U[T][T];
        form_p<T>(xa, ca, P, U);

        __syncthreads();   // the previous pair's reads of Pl and Rl are done
#pragma unroll
        for (int I = 0; I < T; ++I)
#pragma unroll
            for (int J = I; J < T; ++J)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    Pl[p_row(P[I][J], I, r, l) * LDP + 16 * J + (l & 15)] = (double)P[I][J][r];
        __syncthreads();

        // R = [B_OO | B_OU] and S = B_UU
        double bmax = 0.0;
        for (int e = l; e < eta * m; e += 64) {
            const int i = e / m, j = e - i * m;
            double2 v;
            if (j < eta) {
                v.x = Pget(i, j) - Pget(eta + i, eta + j);
                v.y = Pget(i, eta + j) + Pget(eta + i, j);
            } else {
                const int c = eta + j;   // 2 eta + (j - eta)
                v.x = Pget(i, c);
                v.y = Pget(eta + i, c);
            }
            Rl[e] = v;
            bmax = fmax(bmax, c_abs2(v));
        }
        double2 Sv[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int e = l + 64 * q;
            Sv[q] = c_make(0.0, 0.0);
            if (e < M2 * M2) {
                const int i = e / M2, j = e - i * M2;
                Sv[q].x = Pget(2 * eta + i, 2 * eta + j);
                bmax = fmax(bmax, Sv[q].x * Sv[q].x);
            }
        }
        bmax = wave_max(bmax);
        __syncthreads();

        // eliminate the occupied indices pairwise
        double2 pfo = c_make(1.0, 0.0);
        bool zero = false;
        for (int k = 0; k < eta; k += 2) {
            const int pc = k + 1 + l;
            double pv = (pc < eta) ? c_abs2(Rl[k * m + pc]) : -1.0;
            int pi = pc;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double ov = __shfl_xor(pv, off, 64);
                const int op = __shfl_xor(pi, off, 64);
                if (ov > pv || (ov == pv && op < pi)) { pv = ov; pi = op; }
            }
            if (!(pv > 0.0)) { zero = true; break; }
            const int p = pi;
            if (p != k + 1) {
                if (l < m) {
                    const double2 t0 = Rl[(k + 1) * m + l], t1 = Rl[p * m + l];
                    Rl[(k + 1) * m + l] = t1;
                    Rl[p * m + l] = t0;
                }
                __syncthreads();
                if (l < eta) {
                    const double2 t0 = Rl[l * m + k + 1], t1 = Rl[l * m + p];
                    Rl[l * m + k + 1] = t1;
                    Rl[l * m + p] = t0;
                }
                __syncthreads();
                pfo = c_neg(pfo);
            }
            const double2 a = Rl[k * m + k + 1];
            pfo = c_mul(pfo, a);
            const double2 ia = c_inv(a);
            const double2 *r0 = Rl + k * m + eta;         // R[k][eta + .]
            const double2 *r1 = Rl + (k + 1) * m + eta;   // R[k+1][eta + .]
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const int e = l + 64 * q;
                if (e < M2 * M2) {
                    const int i = e / M2, j = e - i * M2;
                    const double2 t = c_sub(c_mul(r1[i], r0[j]), c_mul(r0[i], r1[j]));
                    Sv[q] = c_fma(t, ia, Sv[q]);
                }
            }
            const int j = k + 2 + l;
            if (k + 2 < eta && j < m) {
                const double2 rkj = Rl[k * m + j], rk1j = Rl[(k + 1) * m + j];
                for (int i = k + 2; i < eta; ++i) {
                    const double2 t = c_sub(c_mul(Rl[(k + 1) * m + i], rkj), c_mul(Rl[k * m + i], rk1j));
                    Rl[i * m + j] = c_fma(t, ia, Rl[i * m + j]);
                }
            }
            __syncthreads();
        }

        const int64_t pair = (int64_t)w * Sc + sl;
        double smax = 0.0;
        double2 *Sg = Sbuf + pair * (int64_t)M2 * M2;
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int e = l + 64 * q;
            if (e < M2 * M2) {
                Sg[e] = Sv[q];
                smax = fmax(smax, c_abs2(Sv[q]));
            }
        }
        smax = wave_max(smax);
        const bool flag = zero || !(smax <= SO_SCHUR_GROWTH * SO_SCHUR_GROWTH * bmax);
        if (l == 0) {
            double2 pv = pfo;
            if (flag) {
                // queued for the full-size path, or marked for its scan when the queue is full
                const so_u64 idx = atomicAdd(fb_count, 1ull);
                if ((int64_t)idx < fb_cap) fb_list[idx] = (int64_t)w * S_total + s0 + sl;
                else pv = so_pair_mark();
            }
            Pbuf[pair] = pv;
        }
    }
}
