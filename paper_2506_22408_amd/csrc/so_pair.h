// so_pair.h -- the fused pair kernel: formation on the matrix cores, one
// elimination per pair that leaves a small quadratic pencil, and the node
// Pfaffians of that pencil, one (pair, node) per lane.
//
// Index sets in the stored row order (so_prep.h): O = occupied (eta), U1 =
// the first ne empty rows, U2 = the last ne (ne = n - eta).  J pairs U1 row t
// with U2 row ne - 1 - t and vanishes on K x K, K = O u U1.  With E the U1 x U2
// block of J and L = U2, the Schur complement of B_KK in B + c J is
//   M(c) = B_LL - (B_LK + c J_LK) B_KK^{-1} (B_KL + c J_KL) = M0 + c M1 + c^2 M2,
// so Pf(B + c J) = Pf(B_KK) Pf(M(c)) with M0, M1, M2 skew ne x ne.  The three
// come from one elimination of K in the bordered skew matrix
//   Z = [[B_KK, B_KL, J_KL], [B_LK, B_LL, 0], [J_LK, 0, 0]]:
// its trailing block T = [[T_LL, T_LE], [T_EL, T_EE]] gives M0 = T_LL,
// M1 = T_LE + T_EL = T_LE - T_LE^T, M2 = T_EE.
//
// Elimination: pairwise (Parlett-Reid) steps over K with partial pivoting over
// all remaining indices of K (J vanishes on K x K, so any order is valid and
// B_KK can be well conditioned even where B_OO is not); only the rows of K are
// stored (R, in LDS), entries below them follow by antisymmetry, and the
// trailing T is accumulated in registers from the pivot rows, as in so_form.h.
// Pivoting bounds the multipliers of the K columns only, so the pivot rows'
// entries in the L and E columns are watched as well: a zero pivot, or those
// entries or T beyond SO_SCHUR_GROWTH x max(max|B|, 1), queues the pair for
// the full-size path (so_fallback.h).
//
// Nodes: Q(c) = Pf(B + c J) is evaluated at the ne + 1 nodes e_j (roots of
// unity turned by a third of a step, node table in shadowov.hip) and
// weighted by v_j (node table, so_common.h).  Each lane forms M(e_j) for its
// (pair, node) and reduces it by Householder tridiagonalisation entirely in
// registers (static indices), so a wave runs NB = 64 / (ne + 1) pairs'
// nodes at once.  Above ne = 8 a lane cannot hold a whole node matrix; there
// each 16-lane row takes one (pair, node), lane q holding row q (so_nodes.h,
// pf1_step), four per pass over the batch's NB (ne + 1) items.
#pragma once
#include "so_common.h"
#include "so_form.h"
#include "so_nodes.h"

#ifndef SO_ROW_NODE_BATCH
#define SO_ROW_NODE_BATCH 1
#endif

// ---- per-lane Householder Pfaffian of an N x N complex skew matrix -----------
// A[i][j] for i < j holds the matrix (the rest is implied).  At even step k the
// column c_i = A[i][k] = -A[k][i] (i > k) is mapped to alpha e_{k+1}, alpha =
// -phase(c_{k+1}) |c|; Pf gains alpha and the trailing block k+2.. gets
// A += beta (u y^T - y u^T), y = A conj(u), beta = 1 / (|c|^2 + |c| |c_{k+1}|).
// pf_lane_from<N, K0> runs the steps K0, K0 + 2, ... on A[K0.., K0..].
struct HhStep {
    double2 alpha;
    double beta;
};
__device__ __forceinline__ HhStep hh_setup(double nx2, double2 x0) {
    const double nx = sqrt(nx2);
    const double ax = sqrt(c_abs2(x0));
    const double rax = 1.0 / (ax > 0.0 ? ax : 1.0);
    const double2 phs = ax > 0.0 ? c_scale(x0, rax) : c_make(1.0, 0.0);
    HhStep h;
    h.alpha = c_scale(phs, -nx);
    const double den = nx2 + nx * ax;
    h.beta = den > 0.0 ? 1.0 / den : 0.0;
    return h;
}

template <int N, int K0>
__device__ __forceinline__ double2 pf_lane_from(double2 (&A)[N][N]) {
    double2 pf = c_make(1.0, 0.0);
#pragma unroll
    for (int k = K0; k < N; k += 2) {
        double nx2 = 0.0;
#pragma unroll
        for (int i = k + 1; i < N; ++i) nx2 += c_abs2(A[k][i]);
        const double2 x0 = c_neg(A[k][k + 1]);
        const HhStep h = hh_setup(nx2, x0);
        pf = c_mul(pf, h.alpha);
        if (k + 2 < N) {
            double2 u[N];
            u[k + 1] = c_sub(x0, h.alpha);
#pragma unroll
            for (int i = k + 2; i < N; ++i) u[i] = c_neg(A[k][i]);
            double2 y[N];
#pragma unroll
            for (int q = k + 2; q < N; ++q) {
                double2 acc = c_make(0.0, 0.0);
#pragma unroll
                for (int j = k + 1; j < N; ++j) {
                    if (j == q) continue;
                    const double2 aqj = (q < j) ? A[q][j] : c_neg(A[j][q]);
                    acc = c_fma(aqj, c_conj(u[j]), acc);
                }
                y[q] = c_scale(acc, h.beta);
            }
#pragma unroll
            for (int q = k + 2; q < N; ++q)
#pragma unroll
                for (int j = q + 1; j < N; ++j) A[q][j] = c_fma(u[q], y[j], c_fma(c_neg(y[q]), u[j], A[q][j]));
        }
    }
    return pf;
}

// ---- formation: P = Xall C'_s Xall^T into LDS -------------------------------
// Pl is ld x ld doubles, row-major, for ld - 1 >= d = 2n (the rows and columns
// of P beyond d are zero, since Xall is zero-padded, and are not stored); both
// triangles of P are written and row and column ld - 1 are zeroed (an empty
// orbital's missing imaginary part points there).  Ends with a barrier.
//
// MIX = false: FP64 operands (double2 pairs in A order) on
// v_mfma_f64_16x16x4f64.  MIX = true: single-precision operands (float4
// quads, C' rows in the order sig16) on v_mfma_f32_16x16x4f32 with
// single-precision accumulation; P is widened to FP64 when it is stored and
// everything after the formation runs in FP64.  FULL: ld = 16 T + 1 (2n =
// DP), so every tile entry is stored without a bounds test.
// Stores the upper P tiles (both triangles of P) at stride ld, zeroes row and
// column ld - 1; starts and ends with a barrier.
template <int T, bool FULL, typename Acc>
__device__ __forceinline__ void pair_store(const Acc (&P)[T][T], double *Pl, int l, int ld) {
    __syncthreads();   // region A is free
    const int z = ld - 1;   // the zero row and column
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = I; J < T; ++J)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int a = p_row(P[I][J], I, r, l), bcol = 16 * J + (l & 15);
                const double v = (double)P[I][J][r];
                if (FULL || (a < z && bcol < z)) {
                    Pl[a * ld + bcol] = v;
                    if (J > I) Pl[bcol * ld + a] = -v;   // P is antisymmetric
                }
            }
    // row and column z are zero (R overlays them, so they are rewritten per pair)
    for (int c = l; c <= z; c += 64) {
        Pl[z * ld + c] = 0.0;
        Pl[c * ld + z] = 0.0;
    }
    __syncthreads();
}

template <int T, bool MIX, bool FULL = false>
__device__ __forceinline__ void pair_formation(const void *__restrict__ Xv, const void *__restrict__ Cv,
                                               double *Pl, int l, int ld) {
    constexpr int KK = 4 * T;
    using Op = typename std::conditional<MIX, float, double>::type;
    using Vec = typename std::conditional<MIX, float4, double2>::type;
    using Acc = typename std::conditional<MIX, so_f4, so_d4>::type;
    // operands: the walker's Xall (re-read from L2 per pair: keeping it live
    // through the elimination and node stages costs occupancy) and C'_s
    Op xa[T][KK], ca[T][KK];
    load_ops<T>(static_cast<const Vec *>(Xv), xa, l);
    load_ops<T>(static_cast<const Vec *>(Cv), ca, l);
    Acc P[T][T], U[T][T];
    form_p<T>(xa, ca, P, U);
    pair_store<T, FULL>(P, Pl, l, ld);
}

// ---- formation for a signed-permutation shadow (FP64) ----------------------------
// There C' = Q^T C_b Q is a signed matching: row mu has its one entry s_mu =
// +-1 at column pi(mu).  match_s[mu] = pi(mu) | 0x100 if s_mu = -1, 0x200 for
// the zero padding rows mu >= 2n, negative if the row is not of that form.
// U = C' Xall^T is then the signed gather U[mu][j] = s_mu Xall[j][pi(mu)],
// written straight into the register layout the MFMA product would give
// (register r of lane l of tile (I, J): U[16 I + 4 r + l/16][16 J + l%16]);
// P = Xall U on the matrix cores as in form_p.  A row that is not a signed
// matching makes P NaN, so the pair value and the walker's status report it.
template <int T>
__device__ __forceinline__ void pair_formation_perm(const void *__restrict__ Xv, const int32_t *__restrict__ match_s,
                                                    double *Pl, int l, int ld) {
    constexpr int KK = 4 * T;
    const double *Xd = static_cast<const double *>(Xv);
    double xa[T][KK];
    load_ops<T>(static_cast<const double2 *>(Xv), xa, l);
    so_d4 U[T][T], P[T][T];
    bool bad = false;
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int mm = match_s[16 * I + 4 * r + (l >> 4)];
            bad = bad || mm < 0;
            const int c = mm & 0xff;
            const double sg = (mm & 0x200) ? 0.0 : ((mm & 0x100) ? -1.0 : 1.0);
#pragma unroll
            for (int J = 0; J < T; ++J) U[I][J][r] = sg * Xd[ao_index(16 * J + (l & 15), mm < 0 ? 0 : c, T)];
        }
    if (bad) {
#pragma unroll
        for (int I = 0; I < T; ++I)
#pragma unroll
            for (int J = 0; J < T; ++J) U[I][J] = so_d4{__builtin_nan(""), __builtin_nan(""), __builtin_nan(""),
                                                        __builtin_nan("")};
    }
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = 0; J < T; ++J) P[I][J] = so_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < KK; ++kk)
#pragma unroll
        for (int I = 0; I < T; ++I)
#pragma unroll
            for (int J = I; J < T; ++J)
                P[I][J] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[I][kk], U[kk >> 2][J][kk & 3], P[I][J], 0, 0, 0);
    pair_store<T, true>(P, Pl, l, ld);
}

// ---- pairwise elimination of K in the bordered rows ---------------------------
// Rl: the rows K of Z (n x WR complex, LDS); tv: this thread's trailing entries
// (ta < tb) of the 2NE x 2NE block, updated in place; rbmax = 1 / max|B|^2.
// Returns true when the pair needs the full-size path (zero pivot or growth);
// pfk = Pf(B_KK).  The rows of R are left as they were when each served as a
// pivot row, with the K columns in the final pivoted order: rows k, k+1 of
// pair k/2 are then rows k, k+1 of U in P B_KK P^T = L D L^T, U = D L^T (D:
// the 2 x 2 pivots [[0, a], [-a, 0]]).  With a non-null perm, lane i < n of
// every wave gets perm = the original index of pivoted position i.
// NTH threads (one or two waves) share the work; t = threadIdx.x.  Every wave
// takes the pivot decisions itself from the same data, so they agree and the
// barriers stay uniform; with two waves the final growth maximum is combined
// through xred (two doubles of LDS).
template <int NE, int NTQ, int NTH = 64>
__device__ __forceinline__ bool elim_bordered(int n, int WR, double2 *Rl, const int (&ta)[NTQ], const int (&tb)[NTQ],
                                              double2 (&tv)[NTQ], double bmax, double rbmax, int t, double2 &pfk,
                                              int *perm = nullptr, double *xred = nullptr) {
    static_assert(NTH == 64 || NTH == 128, "one or two waves");
    constexpr int NT2 = NE * (2 * NE - 1);
    const int l = t & 63;
    pfk = c_make(1.0, 0.0);
    int pi = l;
    bool zero = false;
    for (int k = 0; k < n; k += 2) {
        // partner: the largest |R[k][p]|, p in (k, n), smallest p on near-ties.
        // The key is |R[k][p]|^2 / max|B|^2 in single precision with its 6 low
        // bits replaced by 63 - lane; non-negative floats order as unsigned
        // integers, so one maximum gives both; non-candidates hold 0.
        const int pc = k + 1 + l;
        unsigned key = 0u;
        if (pc < n) {
            const float f = (float)(c_abs2(Rl[k * WR + pc]) * rbmax);
            key = (__float_as_uint(f) & ~63u) | (unsigned)(63 - l);
        }
        const unsigned kmax = wave_max_u32(key);
        // below 64: every candidate is zero relative to max|B| (or underflows
        // single precision there); otherwise the low bits name a candidate
        // lane (a NaN candidate included), so p < n
        if (kmax < 64u) { zero = true; break; }
        const int p = k + 1 + (63 - (int)(kmax & 63u));
        if (p != k + 1) {
            if (t < WR) {
                const double2 t0 = Rl[(k + 1) * WR + t], t1 = Rl[p * WR + t];
                Rl[(k + 1) * WR + t] = t1;
                Rl[p * WR + t] = t0;
            }
            __syncthreads();
            if (t < n) {
                const double2 t0 = Rl[t * WR + k + 1], t1 = Rl[t * WR + p];
                Rl[t * WR + k + 1] = t1;
                Rl[t * WR + p] = t0;
            }
            __syncthreads();
            pfk = c_neg(pfk);
            if (perm) pi = __shfl(pi, l == k + 1 ? p : (l == p ? k + 1 : l), 64);
        }
        const double2 a = Rl[k * WR + k + 1];
        pfk = c_mul(pfk, a);
        const double2 ia = c_inv_nr(a);
        const double2 *r0 = Rl + k * WR;
        const double2 *r1 = Rl + (k + 1) * WR;
#pragma unroll
        for (int q = 0; q < NTQ; ++q) {
            if (t + NTH * q < NT2) {
                const int ca_ = n + ta[q], cb_ = n + tb[q];
                const double2 tt = c_sub(c_mul(r1[ca_], r0[cb_]), c_mul(r0[ca_], r1[cb_]));
                tv[q] = c_fma(tt, ia, tv[q]);
            }
        }
        // rows i in [k+2, n), columns j in [k+2, WR); groups of 32 threads take
        // alternate rows: R[i][j] += R[k+1][i] tau_j - R[k][i] sigma_j with the
        // scaled pivot rows tau = R[k] / a, sigma = R[k+1] / a
        const int h = t >> 5;
        for (int j = k + 2 + (t & 31); j < WR; j += 32) {
            const double2 tau = c_mul(r0[j], ia), nsig = c_neg(c_mul(r1[j], ia));
            for (int i = k + 2 + h; i < n; i += NTH / 32) {
                double2 *rij = Rl + i * WR + j;
                *rij = c_fma(r1[i], tau, c_fma(r0[i], nsig, *rij));
            }
        }
        __syncthreads();
    }
    // growth of the unpivoted columns: at the end every row of R is the pivot
    // row it was when it was used, so its L and E entries are all there is to watch
    double gmax = 0.0;
    for (int e = t; e < n * 2 * NE; e += NTH) {
        const int i = e / (2 * NE), c = e - i * (2 * NE);
        gmax = fmax(gmax, c_abs2(Rl[i * WR + n + c]));
    }
    double tmax = 0.0;
#pragma unroll
    for (int q = 0; q < NTQ; ++q) tmax = fmax(tmax, c_abs2(tv[q]));
    tmax = wave_max(fmax(tmax, gmax));
    if constexpr (NTH == 128) {
        if (l == 0) xred[t >> 6] = tmax;
        __syncthreads();
        tmax = fmax(xred[0], xred[1]);
        __syncthreads();
    }
    const bool flag = zero || !(tmax <= SO_SCHUR_GROWTH * SO_SCHUR_GROWTH * fmax(bmax, 1.0));
    if (perm) *perm = pi;
    return flag;
}

// Pf(M(c)) of the pencil M(c) = M0 + c M1 + c^2 M2 (ne x ne, ne <= 16, even)
// whose upper triangles are stored row by row at slot, slot + NT, slot + 2 NT
// (NT = NE (NE - 1) / 2), on one 16-lane row: lane q = l % 16 builds row q of
// M(c) and the row reduces it (pf1_step without a J term).  Every lane of the
// row returns the Pfaffian.
template <int NE>
__device__ __forceinline__ double2 pencil_pf_row(const double2 *slot, double2 c, int q) {
    constexpr int NT = NE * (NE - 1) / 2;
    const double2 c2 = c_mul(c, c);
    Nd1Ctx cx;
    cx.q = q;
    cx.act = q < NE;
    cx.ck = c_make(0.0, 0.0);
    double2 R[NE];
#pragma unroll
    for (int y = 0; y < NE; ++y) {
        // entry (q, y) from the upper triangles: (x, z) = (min, max)
        const int x = q < y ? q : y, z = q < y ? y : q;
        const int e = x * (2 * NE - x - 1) / 2 + (z - x - 1);
        R[y] = c_make(0.0, 0.0);
        if (cx.act && q != y) {
            const double2 v = c_fma(c2, slot[2 * NT + e], c_fma(c, slot[NT + e], slot[e]));
            R[y] = q < y ? v : c_neg(v);
        }
    }
    double2 pf = c_make(1.0, 0.0);
    pf1_step<NE, 0, false>(cx, R, pf);
    return pf;
}

// Pairs whose node Pfaffians run together.  Up to ne = 8 a lane takes one
// (pair, node), so 64 / (ne + 1) pairs fill the wave; above, a 16-lane row
// takes one (pair, node) and a pass takes four whatever the batch, so a
// single pair per batch still keeps most rows busy and saves the LDS of the
// other slots: at n = 24 (three tiles, ne = 12) 7 waves per CU fit instead
// of 5, which measured 1.19x faster than a batch of 4 (1.24x at n = 20).
__host__ __device__ constexpr int pair_node_batch(int ne) { return ne <= 8 ? 64 / (ne + 1) : SO_ROW_NODE_BATCH; }

// LDS per wave: region A = max(P ((2n+1) x (2n+1) f64), R (n x (n + 2 NE) c128),
// T (NE (2NE - 1) c128), node values), then the batch: NB slots of
// 3 NE (NE-1)/2 + 1 complex (M0, M1, M2 upper triangles, Pf(B_KK)).
__host__ __device__ inline size_t pair_lds_bytes(int T, int n, int NE) {
    (void)T;
    const int NB = pair_node_batch(NE);
    size_t a = (size_t)(2 * n + 1) * (2 * n + 1) * sizeof(double);
    const size_t r = (size_t)n * (n + 2 * NE) * sizeof(double2);
    const size_t t = (size_t)NE * (2 * NE - 1) * sizeof(double2);
    const size_t v = (size_t)64 * sizeof(double2);
    if (r > a) a = r;
    if (t > a) a = t;
    if (v > a) a = v;
    a = (a + 15) & ~(size_t)15;
    return a + (size_t)NB * (3 * (NE * (NE - 1) / 2) + 1) * sizeof(double2);
}

// One walker w over the shadows [sb0, sb1): formation, elimination, node
// Pfaffians and the pair values pairs[w S_total + s].  One wave; the LDS
// layout is pair_lds_bytes(T, n, NE).  Xa and Ca hold the walker and shadow
// matrices in FP64 (MIX = false) or single precision (MIX = true), DP x DP
// elements each, in the formation's operand order.  FULL: n = 8 T, so P's
// row stride is the compile-time 16 T + 1 and its stores need no bounds
// test (measured 1.6% of k_pair at n = 16 and 3.5% at n = 24).  OPAQUE_LANE:
// see below.  PERM: every shadow is a signed permutation, match holds the
// signed matchings of the C'_s (DP entries per shadow, pair_formation_perm).
template <int T, int NE, bool MIX, bool FULL, bool OPAQUE_LANE, bool PERM = false>
__device__ __forceinline__ void pair_range(int n, int eta, const void *__restrict__ Xa,
                                           const void *__restrict__ Ca, int64_t S_total, const RedTab &tab,
                                           double2 *__restrict__ pairs, so_u64 *__restrict__ fb_count,
                                           int64_t *__restrict__ fb_list, int64_t fb_cap,
                                           int32_t *__restrict__ wstat, int w, int64_t sb0, int64_t sb1,
                                           const int32_t *__restrict__ match = nullptr) {
    static_assert(!PERM || (FULL && !MIX), "the signed-permutation formation is FP64, n = 8T");
    constexpr int DP = 16 * T;
    constexpr size_t MATB = (size_t)DP * DP * (MIX ? sizeof(float) : sizeof(double));   // bytes per matrix
    constexpr int KE = NE + 1;
    constexpr int NB = pair_node_batch(NE);
    constexpr int NT = NE * (NE - 1) / 2;         // upper entries of one NE x NE matrix
    constexpr int NT2 = NE * (2 * NE - 1);        // upper entries of the 2NE x 2NE trailing block
    constexpr int NTQ = (NT2 + 63) / 64;          // trailing entries per lane
    constexpr int SLOT = 3 * NT + 1;
    extern __shared__ double lds[];
    double *Pl = lds;
    double2 *Rl = reinterpret_cast<double2 *>(lds);
    double2 *Tl = reinterpret_cast<double2 *>(lds);
    double2 *Vl = reinterpret_cast<double2 *>(lds);
    // P is (2n + 1) x (2n + 1); row and column 2n are zero
    const int LDP = FULL ? DP + 1 : 2 * n + 1;
    size_t abytes = (size_t)LDP * LDP * sizeof(double);
    {
        const size_t r = (size_t)n * (n + 2 * NE) * sizeof(double2);
        const size_t t = (size_t)NT2 * sizeof(double2);
        if (r > abytes) abytes = r;
        if (t > abytes) abytes = t;
        if (64 * sizeof(double2) > abytes) abytes = 64 * sizeof(double2);
        abytes = (abytes + 15) & ~(size_t)15;
    }
    double2 *Bt = reinterpret_cast<double2 *>(reinterpret_cast<char *>(lds) + abytes);   // batch slots

    // in the batch kernel, the lane index through an opaque move: nothing
    // derived from it can be hoisted out of the loop over work items (where
    // it would stay live beside the other kernel classes' state); the plain
    // kernel keeps the hoisting (measured 1% faster at n = 16)
    int l = threadIdx.x;
    if constexpr (OPAQUE_LANE) asm volatile("" : "+v"(l));
    const int WR = n + 2 * NE;              // columns of R: K (n), L (NE), E (NE)

    // this lane's trailing entries (a < b) of the 2NE x 2NE block
    int ta[NTQ], tb[NTQ];
#pragma unroll
    for (int q = 0; q < NTQ; ++q) {
        int e = l + 64 * q, a = 0;
        if (e >= NT2) e = 0;
        while (e >= 2 * NE - 1 - a) { e -= 2 * NE - 1 - a; ++a; }
        ta[q] = a;
        tb[q] = a + 1 + e;
    }

    const char *Xw = static_cast<const char *>(Xa) + (size_t)w * MATB;
    auto Pget = [&](int a, int b) -> double { return Pl[a * LDP + b]; };
    // Xall rows of the real and imaginary parts of stored row i; an empty
    // orbital's row is real, and its imaginary part points at the zero row 2n
    auto rre = [&](int i) -> int { return i < eta ? i : eta + i; };
    auto rim = [&](int i) -> int { return i < eta ? eta + i : LDP - 1; };
    auto Bget = [&](int i, int j) -> double2 {
        const int ir = rre(i) * LDP, ii = rim(i) * LDP, jr = rre(j), ji = rim(j);
        return c_make(Pl[ir + jr] - Pl[ii + ji], Pl[ir + ji] + Pl[ii + jr]);
    };

    for (int64_t bs = sb0; bs < sb1; bs += NB) {
        const int nb = (int)min((int64_t)NB, sb1 - bs);
        for (int b = 0; b < nb; ++b) {
            const int64_t s = bs + b;
            // ---------------- formation: P = Xall C' Xall^T
            if constexpr (PERM)
                pair_formation_perm<T>(Xw, match + s * DP, Pl, l, LDP);
            else
                pair_formation<T, MIX, FULL>(Xw, static_cast<const char *>(Ca) + (size_t)s * MATB, Pl, l, LDP);

            // ---------------- R = rows K of Z, trailing T = [[B_LL, 0], [0, 0]]
            constexpr int RPL = (8 * T * (8 * T + NE) + 63) / 64;   // B entries of R per lane (n <= 8 T)
            // the lane index through an opaque move: the entry indices and LDS
            // addresses below are then computed here, not hoisted out of the
            // shadow loop where they would stay live through the other stages
            int lr = l;
            asm volatile("" : "+v"(lr));
            const int WB = n + NE;                    // B columns of R: K and L
            const float rWB = 1.0f / (float)WB;
            double2 rv[RPL];
            double bmax = 0.0;
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                const int e = lr + 64 * q;
                rv[q] = c_make(0.0, 0.0);
                if (e < n * WB) {
                    // e / WB through a float reciprocal: e < 2^10, so the
                    // quotient's fractional part stays clear of the rounding
                    const int i = (int)(((float)e + 0.5f) * rWB), j = e - i * WB;
                    rv[q] = Bget(i, j);               // K and L columns are stored indices
                    bmax = fmax(bmax, c_abs2(rv[q]));
                }
                // finish this entry before the next one's loads (register pressure)
                asm volatile("" : "+v"(rv[q].x), "+v"(rv[q].y) : : "memory");
            }
            double2 tv[NTQ];
#pragma unroll
            for (int q = 0; q < NTQ; ++q) {
                tv[q] = c_make(0.0, 0.0);
                if (l + 64 * q < NT2 && tb[q] < NE) {
                    tv[q].x = Pget(2 * eta + NE + ta[q], 2 * eta + NE + tb[q]);
                    bmax = fmax(bmax, tv[q].x * tv[q].x);
                }
            }
            bmax = wave_max(bmax);
            const double rbmax = rcp_nr(fmax(bmax, 1e-300));
            __syncthreads();   // P reads done
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                const int e = lr + 64 * q;
                if (e < n * WB) {
                    const int i = (int)(((float)e + 0.5f) * rWB), j = e - i * WB;
                    Rl[i * WR + j] = rv[q];
                }
            }
            // E columns: J's U1 x U2 block, J[eta + t][eta + 2ne - 1 - t] = +1
            for (int e = lr; e < n * NE; e += 64) {
                const int i = e / NE, v = e - i * NE;
                Rl[i * WR + n + NE + v] = c_make((i >= eta && i - eta == NE - 1 - v) ? 1.0 : 0.0, 0.0);
            }
            __syncthreads();

            // ---------------- pairwise elimination of K
            double2 pfk;
            const bool flag = elim_bordered<NE, NTQ>(n, WR, Rl, ta, tb, tv, bmax, rbmax, l, pfk);
            bool queued = true;   // (lane 0) a flagged pair found room in the queue
            if (l == 0 && flag) {
                const so_u64 idx = atomicAdd(fb_count, 1ull);
                if ((int64_t)idx < fb_cap) fb_list[idx] = (int64_t)w * S_total + s;
                else queued = false;
            }
            // ---------------- M0, M1, M2 (upper triangles) and Pf(B_KK) into the batch slot
            __syncthreads();   // R reads done
#pragma unroll
            for (int q = 0; q < NTQ; ++q)
                if (l + 64 * q < NT2) Tl[l + 64 * q] = flag ? c_make(0.0, 0.0) : tv[q];
            __syncthreads();
            double2 *slot = Bt + b * SLOT;
            // upper-triangle index of (a, b), a < b < 2NE
            auto tix = [&](int a, int bb) -> int { return a * (2 * NE - 1) - a * (a - 1) / 2 + (bb - a - 1); };
            for (int e = l; e < NT; e += 64) {
                int x = 0, r = e;
                while (r >= NE - 1 - x) { r -= NE - 1 - x; ++x; }
                const int y = x + 1 + r;
                slot[e] = Tl[tix(x, y)];                                              // M0
                slot[NT + e] = c_sub(Tl[tix(x, NE + y)], Tl[tix(y, NE + x)]);         // M1
                slot[2 * NT + e] = Tl[tix(NE + x, NE + y)];                           // M2
            }
            // a flagged pair's value comes from the full-size path: zero here,
            // or the mark when the queue had no room (the full-size kernel scans for it)
            if (l == 0) slot[3 * NT] = flag ? (queued ? c_make(0.0, 0.0) : so_pair_mark()) : pfk;
        }
        // ---------------- node Pfaffians of the batch
        __syncthreads();
        int ln = l;
        asm volatile("" : "+v"(ln));   // as above: no hoisting out of the loops
        if constexpr (NE > 8) {
            // one (pair, node) per 16-lane row, lane q < NE owning row q of
            // M(e_j); four items per pass (pf1_step without a J term)
            const int g = ln >> 4, q = ln & 15;
            for (int it0 = 0; it0 < NB * KE; it0 += 4) {
                const int item = it0 + g;
                const int pb = item / KE, nj = item - pb * KE;
                const double2 pf = pencil_pf_row<NE>(Bt + (pb < nb ? pb : 0) * SLOT, tab.e[nj], q);
                if (q == 0 && pb < nb) Vl[item] = c_mul(pf, tab.v[nj]);
            }
            __syncthreads();
            if (l < nb) {
                double2 acc = c_make(0.0, 0.0);
                for (int j = 0; j < KE; ++j) acc = c_add(acc, Vl[l * KE + j]);
                const double2 pk = Bt[l * SLOT + 3 * NT];
                pairs[(int64_t)w * S_total + bs + l] = so_is_pair_mark(pk) ? pk : c_mul(acc, pk);
            }
            continue;
        }
        const int pb = ln / KE, nj = ln - pb * KE;
        double2 val = c_make(0.0, 0.0);
        if (pb < nb) {
            const double2 *slot = Bt + pb * SLOT;
            const double2 cj = tab.e[nj];
            const double2 cj2 = c_mul(cj, cj);
            // M(c) = M0 + c M1 + c^2 M2, upper triangle, row by row
            double2 A[NE][NE];
            int e = 0;
#pragma unroll
            for (int x = 0; x < NE - 1; ++x) {
#pragma unroll
                for (int y = x + 1; y < NE; ++y) {
                    A[x][y] = c_fma(cj2, slot[2 * NT + e], c_fma(cj, slot[NT + e], slot[e]));
                    ++e;
                }
                // finish each row before the next row's loads are issued, so the
                // three operands per entry are not all held at once
#pragma unroll
                for (int y = x + 1; y < NE; ++y) asm volatile("" : "+v"(A[x][y].x), "+v"(A[x][y].y));
                asm volatile("" ::: "memory");
            }
            val = c_mul(pf_lane_from<NE, 0>(A), tab.v[nj]);
        }
        Vl[l] = val;
        __syncthreads();
        if (l < nb) {
            double2 acc = c_make(0.0, 0.0);
            for (int j = 0; j < KE; ++j) acc = c_add(acc, Vl[l * KE + j]);
            const double2 pk = Bt[l * SLOT + 3 * NT];
            pairs[(int64_t)w * S_total + bs + l] = so_is_pair_mark(pk) ? pk : c_mul(acc, pk);
        }
    }
}

// Register levels of the kernel classes (T, NE, formation precision), from
// the VGPRs each class's kernel needs in the compiler's resource report:
// level 0 fits 168 (three waves per SIMD), level 1 fits 256 without spills
// when alone (two waves per SIMD), level 2 is the rest.  The kernels of level
// 0 are built for three waves per SIMD; the batch kernel of level L holds
// the classes of level <= L.
__host__ __device__ constexpr int pair_class_level(int T, int NE, bool mix) {
    if (T == 1) return NE <= 6 ? 0 : 1;
    if (T == 2) {
        if (NE <= 6) return 0;
        if (NE == 10) return mix ? 0 : 1;
        return 1;
    }
    // T == 3: the FP64 classes other than ne = 10 are kept out of level 1,
    // whose batch kernel then holds the uneven reaction-path set without more
    // spills
    if (mix) return NE <= 4 ? 0 : 1;
    return NE == 10 ? 1 : 2;
}

// grid (W, ceil(S_total / spw)) from shadow group sy0, one wave per block;
// spw is a multiple of pair_node_batch(NE).  Three waves per SIMD for the
// classes of level 0, two otherwise (the three-tile instances would take
// more than 256 registers).
template <int T, int NE, bool MIX, bool FULL, bool PERM = false>
__global__ __launch_bounds__(64, pair_class_level(T, NE, MIX) == 0 ? 3 : 2) void k_pair(int n, int eta, const void *__restrict__ Xa,
                                             const void *__restrict__ Ca, int64_t S_total, int64_t sy0, int spw,
                                             RedTab tab, double2 *__restrict__ pairs,
                                             so_u64 *__restrict__ fb_count, int64_t *__restrict__ fb_list,
                                             int64_t fb_cap, int32_t *__restrict__ wstat,
                                             const int32_t *__restrict__ match) {
    const int64_t sb0 = (sy0 + blockIdx.y) * (int64_t)spw;
    const int64_t sb1 = min(S_total, sb0 + spw);
    pair_range<T, NE, MIX, FULL, false, PERM>(n, eta, Xa, Ca, S_total, tab, pairs, fb_count, fb_list, fb_cap, wstat,
                                              (int)blockIdx.x, sb0, sb1, match);
}
