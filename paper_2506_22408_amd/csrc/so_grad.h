// so_grad.h -- first derivative of the overlap with respect to the walker
// ("Force bias and local energy": d Pf(A) = Pf(A)/2 Tr(A^{-1} dA)).
//
// Per pair, o = sum_j v_j Q(e_j) with Q(c) = Pf(B + c J) (node table,
// so_common.h), so
//   d o = 1/2 Tr(Abar dB) = Tr(Abar dX C' X^T),  Abar = sum_j v_j Q(e_j) (B + e_j J)^{-1}.
// Q(c) (B + c J)^{-1} is a polynomial of degree <= ne in c as well (its
// entries are Pfaffians of minors), so the same ne + 1 points are exact.
// With K = O u U1, L = U2 and the pencil of so_pair.h, the block inverse of
// B + c J gives, for Y(c) = B_KK^{-1} (B_KL + c J_KL) = Y0 + c Y1 and
// N(c) = M(c)^{-1}:
//   (B + cJ)^{-1} = [[B_KK^{-1} + Y N Y^T, -Y N], [-N Y^T, N]],
// hence, with A_p = sum_j v_j Pf(M_j) e_j^p N_j (p = 0, 1, 2) and pfk = Pf(B_KK),
//   Abar_LL = pfk A_0,
//   Abar_KL = -pfk Z,        Z  = Y0 A_0 + Y1 A_1,
//   Abar_LK =  pfk Z^T,
//   Abar_KK = o B_KK^{-1} + pfk (Z Y0^T + Z' Y1^T),   Z' = Y0 A_1 + Y1 A_2.
// Y0, Y1 and B_KK^{-1} come from the pivoted elimination of K and a back
// substitution; N_j and Pf(M_j) from Gauss-Jordan passes over [M_j | I] (Pf as
// the root of det M_j = Pf(M_j)^2 that the pivots give, pf_sign_row).  Each node's
// Pf(M_j) weights both its N_j and its share of o, so the large parts of
// o B_KK^{-1} and Y N Y^T cancel node by node when B_KK is ill conditioned
// (interpolating Pf(M) N from ne - 1 other nodes, a polynomial of degree
// ne - 2, saves a node pass but loses that pairing: measured up to 1e-10
// relative error in Abar where the per-node sums stay near 1e-13).
// A pair whose elimination is flagged (so_pair.h) takes the full-size route:
// Pf and inverse of every B + e_j J.
//
// The pair then contributes F = C' X^T Abar (2n x m) to its walker's sum; the
// per-walker gather (k_grad_walker) turns sum_s F into d(sum_s o)/d Phi
// through X's dependence on Phi: the occupied rows are linear in Phi, the
// empty ones depend on it through G^{-1}, G = [Phi | Phi_perp] (the general
// walker matrix, which is holomorphic in Phi and equals X at the point).
#pragma once
#include "so_common.h"
#include "so_fallback.h"
#include "so_pair.h"

// shapes of the derivative path: n <= 16 (two MFMA tiles), m = n + ne <= 24
#define SO_GRAD_NMAX 16
#define SO_GRAD_MMAX 24

// ---- Gauss-Jordan with partial pivoting on the first nr columns of the
// nr x nc system G (row-major, LDS), one column per lane (nc <= 64), nr <=
// NRM.  Leaves [I | G^{-1} rhs].  Returns false on an exactly zero pivot
// column (the rest of the elimination is then skipped).  The pivot key is the
// high word of |G[r][k]|^2 with its low 6 bits replaced by 63 - lane (the high
// word of a non-negative double orders like the value).  The row loop of the
// update is unrolled to NRM so that a step's LDS accesses are issued
// together.  The barriers do not depend on the data: every step executes the
// same three.  With act = false the wave neither reads nor writes G and
// returns true (the second wave of a two-wave workgroup calls it that way to
// keep the barriers: its pivot search would race with the active wave's row
// swap, which no barrier separates from it).
template <int NRM>
__device__ __forceinline__ bool gj_wave(double2 *G, int nr, int nc, int l, bool act = true) {
    bool ok = true;
    for (int k = 0; k < nr; ++k) {
        int p = k;
        if (act && ok) {
            const int r = k + l;
            unsigned key = 0u;
            if (r < nr) {
                const unsigned hw = (unsigned)(__double_as_longlong(c_abs2(G[r * nc + k])) >> 32);
                key = (hw & ~63u) | (unsigned)(63 - l);
            }
            const unsigned kmax = wave_max_u32(key);
            if (kmax < 64u) ok = false;
            else p = k + (63 - (int)(kmax & 63u));
        }
        const bool work = act && ok && l < nc;
        if (work && p != k) {
            const double2 t0 = G[k * nc + l], t1 = G[p * nc + l];
            G[k * nc + l] = t1;
            G[p * nc + l] = t0;
        }
        __syncthreads();
        const double2 ip = work ? c_inv_nr(G[k * nc + k]) : c_make(0.0, 0.0);
        __syncthreads();
        if (work) G[k * nc + l] = c_mul(G[k * nc + l], ip);
        __syncthreads();
        if (work) {
            const double2 gk = G[k * nc + l];
#pragma unroll
            for (int rr = 0; rr < NRM; ++rr) {
                if (rr < nr && rr != k) {
                    const double2 f = G[rr * nc + k];
                    G[rr * nc + l] = c_fma(c_neg(f), gk, G[rr * nc + l]);
                }
            }
        }
        __syncthreads();
    }
    return ok;
}

// Inverse of one node matrix M(c) = M0 + c M1 + c^2 M2 (NE x NE skew, NE <= 8,
// upper triangles at Mup, Mup + NT, Mup + 2 NT) by Gauss-Jordan with partial
// pivoting on one 16-lane row, entirely in registers: lane c < NE holds
// column c of M(c) and lane NE + y column y of the identity; the steps use DPP
// broadcasts inside the row.  On return lane NE + y holds column y of
// M(c)^{-1} in col[0..NE).  The pivot is the largest |M[r][k]|, the first one
// on ties; a zero pivot column sets sing.  det receives det M(c), the signed
// product of the pivots, and the upper triangle of M(c) is left at Mf
// (row-major, NE x NE) for pf_sign_row.
template <int NE>
__device__ __forceinline__ void gj_node_row(const double2 *Mup, double2 cj, int c, bool &sing, double2 (&col)[NE],
                                            double2 &det, double2 *Mf) {
    constexpr int NT = NE * (NE - 1) / 2;
    const double2 cj2 = c_mul(cj, cj);
#pragma unroll
    for (int r = 0; r < NE; ++r) {
        double2 v = c_make(0.0, 0.0);
        if (c < NE) {
            if (r != c) {
                const int a = r < c ? r : c, b = r < c ? c : r;
                const int ei = a * (2 * NE - 1 - a) / 2 + (b - a - 1);
                v = c_fma(cj2, Mup[2 * NT + ei], c_fma(cj, Mup[NT + ei], Mup[ei]));
                if (r > c) v = c_neg(v);
            }
        } else if (c - NE == r) {
            v = c_make(1.0, 0.0);
        }
        col[r] = v;
        if (c < NE && r < c) Mf[r * NE + c] = v;
    }
    bool zero = false;
    det = c_make(1.0, 0.0);
    [&]<int... K>(std::integer_sequence<int, K...>) {
        (([&] {
             constexpr int k = K;
             double best = -1.0;
             int bi = k;
#pragma unroll
             for (int r = k; r < NE; ++r) {
                 const double a = c_abs2(col[r]);
                 if (a > best) { best = a; bi = r; }
             }
             const double bk = bc16<k>(best);
             const int p = __builtin_amdgcn_mov_dpp(bi, 0x150 + k, 0xf, 0xf, false);
             zero = zero || !(bk > 0.0);
#pragma unroll
             for (int r = k + 1; r < NE; ++r)
                 if (r == p) {
                     const double2 tmp = col[k];
                     col[k] = col[r];
                     col[r] = tmp;
                 }
             const double2 piv = bc16c<k>(col[k]);
             det = c_mul(p != k ? c_neg(det) : det, piv);
             col[k] = c_mul(col[k], c_inv_nr(bk > 0.0 ? piv : c_make(1.0, 0.0)));
#pragma unroll
             for (int r = 0; r < NE; ++r)
                 if (r != k) {
                     const double2 f = bc16c<k>(col[r]);
                     col[r] = c_fma(c_neg(f), col[k], col[r]);
                 }
         }()), ...);
    }(std::make_integer_sequence<int, NE>{});
    if (zero) sing = true;
}

// Pfaffian of the skew matrix on the index set MASK (bits of 0..5), from its
// upper entries u[a][b] (a < b), by expansion along the first index: the
// compile-time recursion unrolls into the (k-1)!! products of k indices
// directly (15 for six).
template <unsigned MASK>
__device__ __forceinline__ double2 pf_expand(const double2 (&u)[6][6]) {
    if constexpr (MASK == 0u) {
        return c_make(1.0, 0.0);
    } else {
        constexpr int a = __builtin_ctz(MASK);
        constexpr unsigned rest = MASK & (MASK - 1u);
        double2 acc = c_make(0.0, 0.0);
        [&]<int... B>(std::integer_sequence<int, B...>) {
            ([&] {
                if constexpr ((rest >> B) & 1u) {
                    constexpr unsigned sub = rest & ~(1u << B);
                    constexpr bool neg = __builtin_popcount(rest & ((1u << B) - 1u)) & 1;
                    double2 term;
                    if constexpr (sub == 0u) term = u[a][B];
                    else term = c_mul(u[a][B], pf_expand<sub>(u));
                    acc = neg ? c_sub(acc, term) : c_add(acc, term);
                }
            }(), ...);
        }(std::make_integer_sequence<int, 6>{});
        return acc;
    }
}

// principal square root, sqrt((|z| + |Re z|) / 2) first so that neither part
// cancels
__device__ __forceinline__ double2 c_sqrt(double2 z) {
    const double r = hypot(z.x, z.y);
    if (r == 0.0) return c_make(0.0, 0.0);
    const double t = sqrt(0.5 * (r + fabs(z.x)));
    const double u = z.y / (2.0 * t);
    return z.x >= 0.0 ? c_make(t, u) : c_make(fabs(u), copysign(t, z.y));
}

// Pf(M) of one node matrix from det M = Pf(M)^2 (the pivots of gj_node_row,
// the same elimination as the node's inverse): of the two roots, the one
// nearer the expansion of Pf along row 0, sum_y (-1)^(y+1) M[0][y]
// Pf(M without 0, y), whose lanes q < NE - 1 each expand one minor of the
// upper triangle at Mf (left there by this wave; a wave's LDS instructions
// execute in order, and the clobber keeps the compiler from moving the reads
// above the writes).  The expansion only chooses the sign: where it cancels
// it may be inaccurate, but it would take an error larger than |Pf(M)| to
// choose the wrong root.  Returns Pf(M) in every lane of the row.
template <int NE>
__device__ __forceinline__ double2 pf_sign_row(const double2 *Mf, int q, double2 det) {
    constexpr int K = NE - 2;
    asm volatile("" ::: "memory");
    double2 a = c_make(0.0, 0.0);
    if (q < NE - 1) {
        const int y = q + 1;
        double2 u[6][6];
        int rr[K > 0 ? K : 1];
#pragma unroll
        for (int i = 0; i < K; ++i) rr[i] = i + 1 + (i + 1 >= y ? 1 : 0);
#pragma unroll
        for (int i = 0; i < K; ++i)
#pragma unroll
            for (int j = i + 1; j < K; ++j) u[i][j] = Mf[rr[i] * NE + rr[j]];
        a = c_mul(Mf[y], pf_expand<(1u << K) - 1u>(u));
        if (!(y & 1)) a = c_neg(a);
    }
    a = c_make(sum16(a.x), sum16(a.y));
    const double2 s = c_sqrt(det);
    return c_abs2(c_sub(s, a)) <= c_abs2(c_add(s, a)) ? s : c_neg(s);
}

// ---- formation shared by the two waves: wave J forms column tile J, U[., J]
// = C' Xall^T[., J] and then P[I][J] = Xall[I] U[., J] for I <= J, and stores
// its tiles (both triangles of P).  With one tile (T = 1) wave 1 only keeps
// the barriers.  Starts and ends with a barrier, as pair_formation does.
template <int T, int J>
__device__ __forceinline__ void form_column(const double2 *__restrict__ Xv, const double2 *__restrict__ Cv,
                                            double *Pl, int l, int ld) {
    constexpr int KK = 4 * T;
    double xa[T][KK], ca[T][KK];
    load_ops<T>(Xv, xa, l);
    load_ops<T>(Cv, ca, l);
    so_d4 U[T], P[J + 1];
#pragma unroll
    for (int I = 0; I < T; ++I) U[I] = so_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < KK; ++kk)
#pragma unroll
        for (int I = 0; I < T; ++I) U[I] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[I][kk], xa[J][kk], U[I], 0, 0, 0);
#pragma unroll
    for (int I = 0; I <= J; ++I) P[I] = so_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < KK; ++kk)
#pragma unroll
        for (int I = 0; I <= J; ++I)
            P[I] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[I][kk], U[kk >> 2][kk & 3], P[I], 0, 0, 0);
    __syncthreads();   // region RP is free
#pragma unroll
    for (int I = 0; I <= J; ++I)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int a = 16 * I + 4 * r + (l >> 4), bcol = 16 * J + (l & 15);
            Pl[a * ld + bcol] = P[I][r];
            if (J > I) Pl[bcol * ld + a] = -P[I][r];
        }
}
template <int T>
__device__ __forceinline__ void formation_two_waves(const double2 *__restrict__ Xv, const double2 *__restrict__ Cv,
                                                    double *Pl, int l, int ld, int wv) {
    static_assert(T <= 2, "two waves, one column tile each");
    if (wv == 0)
        form_column<T, 0>(Xv, Cv, Pl, l, ld);
    else if constexpr (T == 2)
        form_column<T, 1>(Xv, Cv, Pl, l, ld);
    else
        __syncthreads();
    const int z = ld - 1;   // the zero row and column (16 T)
    if (wv == 0)
        for (int c = l; c <= z; c += 64) {
            Pl[z * ld + c] = 0.0;
            Pl[c * ld + z] = 0.0;
        }
    __syncthreads();
}

// LDS regions of k_grad_pair (bytes), in order RP, RB, RR, RG, RS.
//   RP: P, then the trailing block (the pencil's source), then the node
//       inverses N_j, then Abar;
//   RB: B, then the back substitution's solution rows (n x (n + 2NE + 1));
//   RR: the rows K of Z, then A_0, A_1, A_2 and Z, Z';
//   RG: the node passes' scratch (M_j, one per 16-lane row), then
//       [Y0 | Y1 | B_KK^{-1}] (n x (n + 2NE + 1));
//   RS: M0, M1, M2, Pf(M(e_j)), the pivots of B_KK, the pivot permutation and
//       cross-wave scratch.
// The full-size route's [B + cJ | I] (m x 2m) and its Householder vectors span
// RR and RG.
struct GradLds {
    size_t rp, rb, rr, rg, rs, total;
};
__host__ __device__ inline GradLds grad_lds(int T, int n, int NE) {
    const int DP = 16 * T, LDP = DP + 1, m = n + NE;
    GradLds g;
    auto al = [](size_t v) { return (v + 15) & ~(size_t)15; };
    g.rp = al((size_t)LDP * LDP * sizeof(double));
    const size_t wrows = (size_t)n * (n + 2 * NE + 1);   // solution rows (padded stride)
    g.rb = al(((size_t)m * m > wrows ? (size_t)m * m : wrows) * sizeof(double2));
    if (al((size_t)m * m * sizeof(double2)) > g.rp) g.rp = al((size_t)m * m * sizeof(double2));
    if (al((size_t)NE * (2 * NE - 1) * sizeof(double2)) > g.rp) g.rp = al((size_t)NE * (2 * NE - 1) * sizeof(double2));
    // the node inverses are written while the first wave fills RB: RP holds them all
    if (al((size_t)(NE + 1) * NE * NE * sizeof(double2)) > g.rp) g.rp = al((size_t)(NE + 1) * NE * NE * sizeof(double2));
    size_t rr = (size_t)n * (n + 2 * NE);
    if ((size_t)3 * NE * NE + 2 * n * NE > rr) rr = (size_t)3 * NE * NE + 2 * n * NE;
    g.rr = al(rr * sizeof(double2));
    size_t rg = (size_t)n * (n + 2 * NE + 1);
    const size_t full = ((size_t)2 * m * m + 2 * m) * sizeof(double2);
    if (full > g.rr + rg * sizeof(double2)) rg = (full - g.rr + sizeof(double2) - 1) / sizeof(double2);
    // the node passes' scratch: one NE x NE matrix per 16-lane row of the two waves
    if ((size_t)8 * NE * NE > rg) rg = (size_t)8 * NE * NE;
    g.rg = al(rg * sizeof(double2));
    // M0, M1, M2, Pf(M(e_j)), the pivots, the permutation (n ints) and 4 doubles of scratch
    g.rs = al((size_t)(3 * (NE * (NE - 1) / 2) + (NE + 1) + SO_GRAD_NMAX / 2) * sizeof(double2) +
              SO_GRAD_NMAX * sizeof(int) + 4 * sizeof(double));
    g.total = g.rp + g.rb + g.rr + g.rg + g.rs;
    return g;
}

// grid (W, Gy), two waves (128 threads) per block working on one pair at a
// time: walker blockIdx.x, shadows [blockIdx.y spw, ...).  Writes its partial
// sums of F (2n x m, row-major) and of o to Fpart[(w Gy + gy) 2nm ...] and
// Opart[w Gy + gy].  Both waves execute every barrier; steps that one wave
// does alone contain none.
template <int T, int NE>
__global__ __launch_bounds__(128, 2) void k_grad_pair(int n_in, int eta_in, const double2 *__restrict__ Xa,
                                                      const double2 *__restrict__ Ca, int64_t S_total, int spw,
                                                      RedTab tab, double2 *__restrict__ Fpart,
                                                      double2 *__restrict__ Opart, int32_t *__restrict__ wstat) {
    constexpr int NTH = 128;
    constexpr int DP = 16 * T, LDP = DP + 1, MAT2 = DP * DP / 2;
    constexpr int KE = NE + 1;
    constexpr int NT = NE * (NE - 1) / 2;
    constexpr int NT2 = NE * (2 * NE - 1);
    constexpr int NTQ = (NT2 + NTH - 1) / NTH;
    constexpr int KK = 4 * T;
    constexpr int TM = (8 * T + NE + 15) / 16;              // 16-row tiles of F^T (m = n + NE <= 8T + NE)
    // GW, SWP: row strides of RG and of the solution rows, odd in complex
    // entries so that a column read by consecutive rows spreads over the banks
    const int n = n_in, eta = eta_in;
    const int m = n + NE, d = 2 * n;
    const int t0 = threadIdx.x, wv = t0 >> 6, w = blockIdx.x;
    // trailing entries (a < b) of the 2NE x 2NE block handled by this thread
    int ta[NTQ], tb[NTQ];
#pragma unroll
    for (int q = 0; q < NTQ; ++q) {
        int e = t0 + NTH * q, a = 0;
        if (e >= NT2) e = 0;
        while (e >= 2 * NE - 1 - a) { e -= 2 * NE - 1 - a; ++a; }
        ta[q] = a;
        tb[q] = a + 1 + e;
    }
    const double2 *Xw = Xa + (size_t)w * MAT2;
    // F^T = sum over the range of Abar''^T (Xall C'^T), real and imaginary
    // parts, in the matrix-core accumulators: wave wv holds the column tile
    // J = wv (tile (I, J), register r, lane l: F^T[16 I + 4 r + l/16][16 J + l%16])
    so_d4 FT[2][TM];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int I = 0; I < TM; ++I) FT[p][I] = so_d4{0.0, 0.0, 0.0, 0.0};
    double2 oacc = c_make(0.0, 0.0);
    int32_t wflags = 0;

    const int64_t s0 = (int64_t)blockIdx.y * spw;
    const int64_t s1 = min(S_total, s0 + spw);
    for (int64_t s = s0; s < s1; ++s) {
        // n and eta through an opaque move as well: the uniform values derived
        // from them (LDS offsets, row strides) are recomputed per pair on the
        // scalar unit instead of being hoisted out of the shadow loop, where
        // they would exceed the scalar registers and be kept in vector-register
        // lanes (a vector instruction per reload)
        int n = n_in, eta = eta_in;
        asm volatile("" : "+s"(n), "+s"(eta));
        const int m = n + NE, d = 2 * n, WR = n + 2 * NE, GW = n + 2 * NE + 1, SWP = n + 2 * NE + 1;
        extern __shared__ double lds[];
        const GradLds L = grad_lds(T, n, NE);
        char *base = reinterpret_cast<char *>(lds);
        double *RP = reinterpret_cast<double *>(base);
        double2 *RA = reinterpret_cast<double2 *>(base);   // over P once B is built
        double2 *NJ = RA;                                  // node inverses, before Abar
        double2 *RB = reinterpret_cast<double2 *>(base + L.rp);
        double2 *RR = reinterpret_cast<double2 *>(base + L.rp + L.rb);
        double2 *RG = reinterpret_cast<double2 *>(base + L.rp + L.rb + L.rr);
        double2 *RS = reinterpret_cast<double2 *>(base + L.rp + L.rb + L.rr + L.rg);
        double2 *Mup = RS;                       // M0, M1, M2 upper triangles
        double2 *pfm = RS + 3 * NT;              // Pf(M(e_j))
        double2 *piv = pfm + KE;                 // the pivots a of B_KK's 2 x 2 blocks
        int *pis = reinterpret_cast<int *>(piv + SO_GRAD_NMAX / 2);
        double *xred = reinterpret_cast<double *>(pis + SO_GRAD_NMAX);
        double2 *Ahat = RR;                      // A_0, A_1, A_2 (NE x NE each)
        double2 *Zr = RR + 3 * NE * NE;          // Z, Z' (n x NE each)
        double2 *ubuf = RR + 2 * m * m;          // Householder vectors of the full-size route
        double2 *ybuf = ubuf + m;
        auto rre = [&](int i) -> int { return i < eta ? i : eta + i; };
        auto rim = [&](int i) -> int { return i < eta ? eta + i : DP; };
        // J of the stored order: +1 at (eta+t, eta+2ne-1-t), -1 at the transpose
        auto Jel = [&](int i, int j) -> double {
            if (i < eta || j < eta) return 0.0;
            const int u = i - eta, v = j - eta;
            return (u + v == 2 * NE - 1) ? (u < NE ? 1.0 : -1.0) : 0.0;
        };
        // block-wide maximum of a value that each wave has reduced
        auto block_max = [&](double v) -> double {
            if ((t0 & 63) == 0) xred[wv] = v;
            __syncthreads();
            const double r = fmax(xred[0], xred[1]);
            __syncthreads();
            return r;
        };
        // the thread index through an opaque move: indices derived from it are
        // recomputed per pair instead of being hoisted out of the shadow loop,
        // where they would stay live (and spill) through every stage
        int t = t0;
        asm volatile("" : "+v"(t));
        const int l = t & 63;
        const double2 *Cs = Ca + (size_t)s * MAT2;
        // P = Xall C' Xall^T, each wave forming one column tile
        formation_two_waves<T>(Xw, Cs, RP, l, LDP, wv);

        // ---------------- B (m x m), then R = rows K of Z
        double bmax = 0.0;
        for (int e = t; e < m * m; e += NTH) {
            const int i = e / m, j = e - i * m;
            const int ir = rre(i) * LDP, ii = rim(i) * LDP, jr = rre(j), ji = rim(j);
            const double2 v = c_make(RP[ir + jr] - RP[ii + ji], RP[ir + ji] + RP[ii + jr]);
            RB[e] = v;
            bmax = fmax(bmax, c_abs2(v));
        }
        bmax = block_max(wave_max(bmax));   // its barriers also publish B
        const double rbmax = rcp_nr(fmax(bmax, 1e-300));
        for (int e = t; e < n * WR; e += NTH) {
            const int i = e / WR, j = e - i * WR;
            RR[e] = (j < m) ? RB[i * m + j] : c_make(Jel(i, n + (j - m)), 0.0);
        }
        double2 tv[NTQ];
#pragma unroll
        for (int q = 0; q < NTQ; ++q) {
            tv[q] = c_make(0.0, 0.0);
            if (t + NTH * q < NT2 && tb[q] < NE) tv[q] = RB[(n + ta[q]) * m + n + tb[q]];
        }
        __syncthreads();

        // ---------------- elimination of K, pencil, node Pfaffians
        double2 pfk;
        int perm = l;
        const bool flag = elim_bordered<NE, NTQ, NTH>(n, WR, RR, ta, tb, tv, bmax, rbmax, t, pfk, &perm, xred);
        double2 o = c_make(0.0, 0.0);
        if (!flag) {
            // ---------------- the pencil M0, M1, M2 from the trailing block, staged
            // through RP (P is no longer needed)
            double2 *TT = reinterpret_cast<double2 *>(RP);
#pragma unroll
            for (int q = 0; q < NTQ; ++q)
                if (t + NTH * q < NT2) TT[t + NTH * q] = tv[q];
            __syncthreads();
            auto tix = [&](int a, int bb) -> int { return a * (2 * NE - 1) - a * (a - 1) / 2 + (bb - a - 1); };
            for (int e = t; e < NT; e += NTH) {
                int x = 0, r = e;
                while (r >= NE - 1 - x) { r -= NE - 1 - x; ++x; }
                const int y = x + 1 + r;
                Mup[e] = TT[tix(x, y)];
                Mup[NT + e] = c_sub(TT[tix(x, NE + y)], TT[tix(y, NE + x)]);
                Mup[2 * NT + e] = TT[tix(NE + x, NE + y)];
            }
            __syncthreads();
            // ---------------- two things at once, with no barrier in either:
            // wave 0 solves for Y0, Y1 and B_KK^{-1} (back substitution with the
            // pivot rows) and then takes the estimator nodes from 8 on; wave 1 takes
            // Pf(M_j) and N_j = M_j^{-1} of nodes 0..7, four per pass (one per
            // 16-lane row).  The nodes do not depend on the solve.
            const int g4 = (t >> 4) & 3, q16 = t & 15;
            bool sing = false;
            auto node_pass = [&](int j) {
                const double2 cj = tab.e[j < KE ? j : KE - 1];
                double2 col[NE], det;
                bool sg = false;
                double2 *Mf = RG + (wv * 4 + g4) * NE * NE;   // this row's scratch: RG is free until the scatter
                gj_node_row<NE>(Mup, cj, q16, sg, col, det, Mf);
                if (j < KE) {
                    sing = sing || sg;
                    if (q16 >= NE && q16 < 2 * NE) {
                        const int y = q16 - NE;
#pragma unroll
                        for (int x = 0; x < NE; ++x) NJ[(j * NE + x) * NE + y] = col[x];
                    }
                }
                const double2 pf = pf_sign_row<NE>(Mf, q16, det);   // after the inverse is stored
                if (q16 == 0 && j < KE) pfm[j] = pf;
            };
            // U [Y' | W] = [R_LE | I] in the pivoted order (U = the rows of R, block
            // upper triangular with pivots [[0, a], [-a, 0]]); then, with pi the
            // permutation, Y[pi(i)] = Y'[i] and B_KK^{-1}[pi(i)][pi(j)] = (-W D W^T)[i][j]
            // (P B_KK P^T = L D L^T = -U^T D^{-1} U).  Lane c < 2NE + n of wave 0
            // holds column c of the right-hand side; the solution goes to RB (free:
            // the full-size route is ruled out) and then, reordered, to RG.
            constexpr int NRM = 8 * T;
            const int SW = 2 * NE + n;
            if (wv == 0) {
                double2 rhs[NRM];
#pragma unroll
                for (int i = 0; i < NRM; ++i) {
                    rhs[i] = c_make(0.0, 0.0);
                    if (i < n && l < SW)
                        rhs[i] = l < 2 * NE ? RR[i * WR + n + l] : c_make(i == l - 2 * NE ? 1.0 : 0.0, 0.0);
                }
#pragma unroll
                for (int bb = 0; bb < NRM / 2; ++bb) {
                    const int k = NRM - 2 - 2 * bb;
                    if (k < n) {
                        const double2 a = RR[k * WR + k + 1];
                        if (l == 0) piv[k / 2] = a;
                        const double2 ia = c_inv_nr(a);
                        const double2 yk1 = c_mul(rhs[k], ia), yk = c_neg(c_mul(rhs[k + 1], ia));
                        rhs[k] = yk;
                        rhs[k + 1] = yk1;
#pragma unroll
                        for (int i = 0; i < k; ++i)
                            rhs[i] = c_fma(c_neg(RR[i * WR + k]), yk, c_fma(c_neg(RR[i * WR + k + 1]), yk1, rhs[i]));
                    }
                }
                if (l < n) pis[l] = perm;
#pragma unroll
                for (int i = 0; i < NRM; ++i)
                    if (i < n && l < SW) RB[i * SWP + l] = rhs[i];
                for (int j0 = 8; j0 < KE; j0 += 4) node_pass(j0 + g4);
            } else {
                for (int j0 = 0; j0 < (KE < 8 ? KE : 8); j0 += 4) node_pass(j0 + g4);
            }
            if (sing) wflags |= SO_WSTAT_SINGULAR;
            __syncthreads();
            for (int e = t; e < n * 2 * NE; e += NTH) {
                const int i = e / (2 * NE), c = e - i * (2 * NE);
                RG[pis[i] * GW + c] = RB[i * SWP + c];
            }
            for (int e = t; e < n * n; e += NTH) {
                const int i = e / n, j = e - i * n;
                const double2 *wi = RB + i * SWP + 2 * NE, *wj = RB + j * SWP + 2 * NE;
                double2 acc = c_make(0.0, 0.0);
                for (int k = 0; k < n; k += 2)
                    acc = c_fma(piv[k / 2], c_sub(c_mul(wi[k], wj[k + 1]), c_mul(wi[k + 1], wj[k])), acc);
                RG[pis[i] * GW + 2 * NE + pis[j]] = c_neg(acc);
            }
            for (int j = 0; j < KE; ++j) o = c_fma(tab.v[j], pfm[j], o);
            o = c_mul(o, pfk);
            // ---------------- A_p = sum_j v_j Pf(M_j) e_j^p N_j (p = 0, 1, 2), in the
            // same phase (the node results were complete at the last barrier)
            for (int e = t; e < 3 * NE * NE; e += NTH) {
                const int pw = e / (NE * NE), xy = e - pw * NE * NE;
                double2 acc = c_make(0.0, 0.0);
                for (int j = 0; j < KE; ++j) {
                    double2 cf = c_mul(tab.v[j], pfm[j]);
                    if (pw >= 1) cf = c_mul(cf, tab.e[j]);
                    if (pw == 2) cf = c_mul(cf, tab.e[j]);
                    acc = c_fma(cf, NJ[j * NE * NE + xy], acc);
                }
                Ahat[e] = acc;
            }
            __syncthreads();
            // ---------------- Z, Z' (n x NE)
            // Y0 = RG[:, 0:NE], Y1 = RG[:, NE:2NE], B_KK^{-1} = RG[:, 2NE:2NE+n]
            for (int e = t; e < n * NE; e += NTH) {
                const int i = e / NE, x = e - i * NE;
                double2 z = c_make(0, 0), zp = c_make(0, 0);
                for (int y = 0; y < NE; ++y) {
                    const double2 y0 = RG[i * GW + y], y1 = RG[i * GW + NE + y];
                    z = c_fma(y0, Ahat[y * NE + x], c_fma(y1, Ahat[NE * NE + y * NE + x], z));
                    zp = c_fma(y0, Ahat[NE * NE + y * NE + x], c_fma(y1, Ahat[2 * NE * NE + y * NE + x], zp));
                }
                Zr[e] = z;
                Zr[n * NE + e] = zp;
            }
            __syncthreads();
            // ---------------- Abar (m x m) into RA
            for (int e = t; e < m * m; e += NTH) {
                const int i = e / m, j = e - i * m;
                double2 v;
                if (i < n && j < n) {
                    double2 acc = c_make(0, 0);
                    for (int x = 0; x < NE; ++x)
                        acc = c_fma(Zr[i * NE + x], RG[j * GW + x],
                                    c_fma(Zr[n * NE + i * NE + x], RG[j * GW + NE + x], acc));
                    v = c_fma(o, RG[i * GW + 2 * NE + j], c_mul(pfk, acc));
                } else if (i < n) {
                    v = c_neg(c_mul(pfk, Zr[i * NE + (j - n)]));
                } else if (j < n) {
                    v = c_mul(pfk, Zr[j * NE + (i - n)]);
                } else {
                    v = c_mul(pfk, Ahat[(i - n) * NE + (j - n)]);
                }
                RA[e] = v;
            }
            __syncthreads();
        } else {
            // ---------------- full-size route: Pf and inverse of every B + e_j J;
            // wave 0 reduces, wave 1 takes the same decisions and barriers
            o = c_make(0.0, 0.0);
            for (int e = t; e < m * m; e += NTH) RA[e] = c_make(0.0, 0.0);
            double2 *Aug = RR;   // m x 2m over RR and RG
            const int AW = 2 * m;
            for (int j = 0; j < KE; ++j) {
                const double2 cj = tab.e[j];
                __syncthreads();
                for (int e = t; e < m * m; e += NTH) {
                    const int i = e / m, c = e - i * m;
                    Aug[i * AW + c] = c_add(RB[e], c_scale(cj, Jel(i, c)));
                }
                const double2 qw = hh_pf_lds(Aug, AW, m, ubuf, ybuf, l, wv == 0);
                if (t == 0) { xred[0] = qw.x; xred[1] = qw.y; }
                __syncthreads();
                const double2 qj = c_make(xred[0], xred[1]);
                for (int e = t; e < m * AW; e += NTH) {
                    const int i = e / AW, c = e - i * AW;
                    Aug[e] = (c < m) ? c_add(RB[i * m + c], c_scale(cj, Jel(i, c)))
                                     : c_make((c - m == i) ? 1.0 : 0.0, 0.0);
                }
                __syncthreads();
                const bool gok = gj_wave<8 * T + NE>(Aug, m, AW, l, wv == 0);
                if (!gok) wflags |= SO_WSTAT_SINGULAR;   // wave 0 only (wave 1 gets true)
                const double2 f = c_mul(tab.v[j], qj);
                o = c_fma(tab.v[j], qj, o);
                for (int e = t; e < m * m; e += NTH) {
                    const int i = e / m, c = e - i * m;
                    RA[e] = c_fma(f, Aug[i * AW + m + c], RA[e]);
                }
            }
            __syncthreads();
        }
        oacc = c_add(oacc, o);

        // ---------------- F += (C' X^T) Abar = U Abar'' with U = C' Xall^T (d x DP)
        // and Abar'' (DP x m) the rows of Abar placed on the rows of Xall:
        // Abar''[rre(i)] = Abar[i], Abar''[rim(i)] = i Abar[i].  On the matrix
        // cores as F^T += Abar''^T U^T: U^T = Xall C'^T from the operands, its
        // tile (I, J) register r being the B operand at k-step 4 I + r.  Wave wv
        // takes the column tile J = wv.
#pragma unroll
        for (int J = 0; J < T; ++J) {
            if (J != wv) continue;   // wave J takes column tile J (a compile-time index)
            // operands: all of Xall, and tile J of C' only
            double xa[T][KK], cj[KK];
            load_ops<T>(Xw, xa, l);
#pragma unroll
            for (int h = 0; h < 2 * T; ++h) {
                const double2 v = Cs[(J * 2 * T + h) * 64 + l];
                cj[2 * h] = v.x;
                cj[2 * h + 1] = v.y;
            }
            so_d4 Ut[T];
#pragma unroll
            for (int I = 0; I < T; ++I) Ut[I] = so_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < KK; ++kk)
#pragma unroll
                for (int I = 0; I < T; ++I)
                    Ut[I] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[I][kk], cj[kk], Ut[I], 0, 0, 0);
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                // A operand: Abar''[k][c], k = 4 kk + l/16 a row of Xall, c = 16 I + l%16
                const int k = 4 * kk + (l >> 4);
                const int i = k < eta ? k : k - eta;
                const bool imag = k >= eta && k < 2 * eta;
#pragma unroll
                for (int I = 0; I < TM; ++I) {
                    const int c = 16 * I + (l & 15);
                    double2 a = c_make(0.0, 0.0);
                    if (k < d && c < m) a = RA[i * m + c];
                    if (imag) a = c_make(-a.y, a.x);
                    FT[0][I] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, Ut[kk >> 2][kk & 3], FT[0][I], 0, 0, 0);
                    FT[1][I] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, Ut[kk >> 2][kk & 3], FT[1][I], 0, 0, 0);
                }
            }
        }
        __syncthreads();   // Abar reads done before the next formation
    }
    const int64_t part = (int64_t)w * gridDim.y + blockIdx.y;
    const int l = t0 & 63;
    if (wv < T) {
        const int J = wv;
#pragma unroll
        for (int I = 0; I < TM; ++I)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = 16 * I + 4 * r + (l >> 4), mu = 16 * J + (l & 15);
                if (c < m && mu < d) Fpart[part * (int64_t)(d * m) + mu * m + c] = c_make(FT[0][I][r], FT[1][I][r]);
            }
    }
    if (t0 == 0) Opart[part] = oacc;
    if (l == 0 && wflags) atomicOr(&wstat[w], wflags);
}

// One workgroup of 64 per walker: F = sum over the walker's partials (fixed
// order), o = sum_s o_ws, then the gather
//   d o / d Phi_pj = (F[2p][j] - i F[2p+1][j]) / sqrt2
//                  - sum_t conj(g_t[p]) sum_q Phi+_jq h_t[q],
//   h_t[q] = (F[2q][r0] + i F[2q+1][r0] - i F[2q][r1] + F[2q+1][r1]) / 2,
// with r0 = eta + t, r1 = eta + 2ne - 1 - t the stored rows of empty orbital t,
// g_t its complement vector ((G^{-1})_{eta+t, p} = conj(g_t[p])) and
// Phi+ = (Phi^H Phi)^{-1} Phi^H the first eta rows of G^{-1}.  Then
// D = (d sum_s o / d Phi) / sum_s o, G = D Phi^T, S_w = sum_s o / S.
// With rf and logdet, phi is the orthonormal factor Qf of the walker
// Phi = Qf R (k_walker_prep) and the pairs were evaluated at Qf.  The
// overlap is multilinear in the orbitals, S(Psi A) = det A S(Psi) for every
// invertible eta x eta A, so S(Phi) = det R S(Qf), D(Phi) = D(Qf) R^{-T} and
// G(Phi) = G(Qf): the outputs reach every walker norm that a double can hold
// without a node Pfaffian leaving the double range.
__global__ __launch_bounds__(64) void k_grad_walker(int n, int eta, const double2 *__restrict__ phi,
                                                    const double *__restrict__ Xa, const double2 *__restrict__ Fpart,
                                                    const double2 *__restrict__ Opart, int Gy, int64_t S_total,
                                                    double2 *__restrict__ overlap, double2 *__restrict__ dlog,
                                                    double2 *__restrict__ green, int32_t *__restrict__ wstat, int logout,
                                                    const double2 *__restrict__ rf, const double2 *__restrict__ logdet) {
    __shared__ double2 Fs[2 * SO_GRAD_NMAX * SO_GRAD_MMAX];
    __shared__ double2 Ph[SO_GRAD_NMAX * SO_GRAD_NMAX];        // Phi (n x eta)
    __shared__ double2 Gm[SO_GRAD_NMAX * 2 * SO_GRAD_NMAX];    // [Phi^H Phi | I] (eta x 2 eta)
    __shared__ double2 Pp[SO_GRAD_NMAX * SO_GRAD_NMAX];        // Phi+ (eta x n)
    __shared__ double2 Hh[SO_GRAD_NMAX * SO_GRAD_NMAX];        // h_t[q] (ne x n)
    __shared__ double2 Vv[SO_GRAD_NMAX * SO_GRAD_NMAX];        // V[j][t] (eta x ne)
    __shared__ double2 Dd[SO_GRAD_NMAX * SO_GRAD_NMAX];        // D (n x eta)
    const int l = threadIdx.x, w = blockIdx.x;
    const int ne = n - eta, m = 2 * n - eta, d = 2 * n, T = so_tiles(n), DP = 16 * T;
    const int dm = d * m;
    for (int e = l; e < dm; e += 64) {
        double2 acc = c_make(0, 0);
        for (int g = 0; g < Gy; ++g) acc = c_add(acc, Fpart[((int64_t)w * Gy + g) * dm + e]);
        Fs[e] = acc;
    }
    double2 osum = c_make(0, 0);
    for (int g = 0; g < Gy; ++g) osum = c_add(osum, Opart[(int64_t)w * Gy + g]);
    const double2 *pw = phi + (size_t)w * n * eta;
    for (int e = l; e < n * eta; e += 64) Ph[e] = pw[e];
    __syncthreads();
    // [Phi^H Phi | I] -> [I | (Phi^H Phi)^{-1}]
    const int gw = 2 * eta;
    for (int e = l; e < eta * gw; e += 64) {
        const int a = e / gw, c = e - a * gw;
        double2 v = c_make(0, 0);
        if (c < eta)
            for (int p = 0; p < n; ++p) v = c_fma(c_conj(Ph[p * eta + a]), Ph[p * eta + c], v);
        else
            v = c_make((c - eta == a) ? 1.0 : 0.0, 0.0);
        Gm[e] = v;
    }
    __syncthreads();
    const bool ok = gj_wave<SO_GRAD_NMAX>(Gm, eta, gw, l);
    for (int e = l; e < eta * n; e += 64) {
        const int j = e / n, q = e - j * n;
        double2 v = c_make(0, 0);
        for (int a = 0; a < eta; ++a) v = c_fma(Gm[j * gw + eta + a], c_conj(Ph[q * eta + a]), v);
        Pp[e] = v;
    }
    for (int e = l; e < ne * n; e += 64) {
        const int t = e / n, q = e - t * n;
        const int r0 = eta + t, r1 = eta + 2 * ne - 1 - t;
        const double2 a = Fs[(2 * q) * m + r0], b = Fs[(2 * q + 1) * m + r0];
        const double2 c = Fs[(2 * q) * m + r1], dd = Fs[(2 * q + 1) * m + r1];
        // (a + i b - i c + dd) / 2
        Hh[e] = c_scale(c_make(a.x - b.y + c.y + dd.x, a.y + b.x - c.x + dd.y), 0.5);
    }
    __syncthreads();
    for (int e = l; e < eta * ne; e += 64) {
        const int j = e / ne, t = e - j * ne;
        double2 v = c_make(0, 0);
        for (int q = 0; q < n; ++q) v = c_fma(Pp[j * n + q], Hh[t * n + q], v);
        Vv[e] = v;
    }
    __syncthreads();
    const double *Xw = Xa + (size_t)w * DP * DP;
    const double rs2 = 0.70710678118654752440;
    const bool zero = (osum.x == 0.0 && osum.y == 0.0);
    // a rank-deficient walker (flagged by k_walker_prep) has no derivative: NaN
    const bool rank = (wstat[w] & SO_WSTAT_RANK) != 0;
    const double2 rinv = zero ? c_make(0, 0) : c_inv(osum);
    for (int e = l; e < n * eta; e += 64) {
        const int p = e / eta, j = e - p * eta;
        const double2 f0 = Fs[(2 * p) * m + j], f1 = Fs[(2 * p + 1) * m + j];
        double2 gv = c_scale(c_make(f0.x + f1.y, f0.y - f1.x), rs2);   // (f0 - i f1) / sqrt2
        for (int t = 0; t < ne; ++t) {
            const double2 gt = c_make(Xw[ao_index(2 * eta + t, 2 * p, T)], Xw[ao_index(2 * eta + t, 2 * p + 1, T)]);
            gv = c_sub(gv, c_mul(c_conj(gt), Vv[j * ne + t]));
        }
        const double2 dv = (zero || rank) ? c_make(NAN, NAN) : c_mul(gv, rinv);
        Dd[e] = dv;
        if (!rf) dlog[(size_t)w * n * eta + e] = dv;
    }
    __syncthreads();
    if (green)
        for (int e = l; e < n * n; e += 64) {
            const int p = e / n, q = e - p * n;
            double2 v = c_make(0, 0);
            for (int j = 0; j < eta; ++j) v = c_fma(Dd[p * eta + j], Ph[q * eta + j], v);
            green[(size_t)w * n * n + e] = v;
        }
    // with rf: phi holds the orthonormal factor Qf of the caller's walker
    // Phi = Qf R.  G = D Phi^T does not change (the state is the same up to
    // scale), and D(Phi) = D(Qf) R^{-T}: row p of D solves D[p] R^T = D(Qf)[p]
    if (rf) {
        __syncthreads();
        if (l < n) {
            const double2 *Rw = rf + (size_t)w * eta * eta;
            double2 *Dr = Dd + l * eta;
            for (int j = eta - 1; j >= 0; --j) {
                double2 v = Dr[j];
                for (int i = j + 1; i < eta; ++i) v = c_sub(v, c_mul(Dr[i], Rw[j * eta + i]));
                Dr[j] = c_mul(v, c_inv(Rw[j * eta + j]));
                dlog[(size_t)w * n * eta + l * eta + j] = Dr[j];
            }
        }
    }
    if (l == 0) {
        int32_t st = wstat[w];
        double2 r = c_scale(osum, 1.0 / (double)S_total);
        if (st & SO_WSTAT_RANK) r = c_make(NAN, NAN);
        if (zero) st |= SO_WSTAT_ZERO;
        if (!ok) st |= SO_WSTAT_RANK;
        if (!isfinite(r.x) || !isfinite(r.y)) st |= SO_WSTAT_NONFINITE;
        if (logout) {
            r = c_log(r);
            if (logdet) r = c_make(r.x + logdet[w].x, remainder(r.y + logdet[w].y, 2.0 * M_PI));
        } else if (logdet) {
            const double mg = exp(logdet[w].x);
            r = c_mul(c_make(mg * cos(logdet[w].y), mg * sin(logdet[w].y)), r);
            if (!isfinite(r.x) || !isfinite(r.y)) st |= SO_WSTAT_NONFINITE;
        }
        overlap[w] = r;
        wstat[w] = st;
    }
}
