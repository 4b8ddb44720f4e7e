// shadowov.hip -- MI355X (gfx950) kernels and C ABI for the matchgate-shadow
// overlap estimator of QC-AFQMC (Zhao et al., arXiv:2506.22408).
//
// Per walker x shadow pair the estimator forms the Majorana-basis matrix
// B = X C' X^T (eq. b_mat, with X the selected rows of W M_phi and
// C' = Q^T C_b Q), evaluates Pf(A(z)) with A(z) = C_0^(s) + z B (eq. a_mat)
// at K interpolation nodes, and combines the node values with weights that
// carry the interpolation, the inverse-channel factors C(2N,2x)/C(N,x) and
// the prefactor of o_p (section "Classical shadows and the evaluation of
// overlaps").  The shadow average S_w closes the path.
//
// Kernels (one HIP stream, no host round trip inside a call):
//   k_walker_prep   X_w (m x 2n) from Phi_w; Householder completion of col(Phi)
//   k_shadow_prep   C'_s = Q_s^T C_b Q_s
//   k_form          B_ws = X_w C'_s X_w^T for a chunk of shadows  (FP64)
//   k_pfaff<M,...>  sum_k w_k Pf(A(z_k)) per pair; one node matrix per lane
//                   group, rows in registers, Householder tridiagonalisation
//   k_reduce        S_w = (1/S) sum_s o_ws in a fixed order (deterministic)
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <utility>

#include "shadowov.h"

// --------------------------------------------------------------------------
// small complex helpers on double2 (x = re, y = im)
// --------------------------------------------------------------------------
__device__ __forceinline__ double2 c_make(double r, double i) { double2 v; v.x = r; v.y = i; return v; }
__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return c_make(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return c_make(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_scale(double2 a, double s) { return c_make(a.x * s, a.y * s); }
__device__ __forceinline__ double2 c_conj(double2 a) { return c_make(a.x, -a.y); }
__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
    return c_make(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// c + a * b
__device__ __forceinline__ double2 c_fma(double2 a, double2 b, double2 c) {
    return c_make(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ double c_abs2(double2 a) { return fma(a.x, a.x, a.y * a.y); }

template <int W>
__device__ __forceinline__ double grp_sum(double v) {
#pragma unroll
    for (int off = W / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, W);
    return v;
}
template <int W>
__device__ __forceinline__ double2 grp_bcast(double2 v, int src) {
    return c_make(__shfl(v.x, src, W), __shfl(v.y, src, W));
}

// Node table passed by value: K <= SO_KMAX.
#define SO_KMAX 49
struct NodeTab {
    double2 s[SO_KMAX];   // factor applied to B in the node matrix
    double2 c[SO_KMAX];   // factor applied to the selected vacuum covariance J
    double2 w[SO_KMAX];   // node weight (with any rescaling folded in)
    int K;
    int unit_b;           // 1: every s_k == 1 (rows start as B itself)
};

// --------------------------------------------------------------------------
// k_walker_prep: X_w from Phi_w (Supp. "Matrix Definitions", W and M_phi).
// Occupied orbital j (row j):  X[j,2p] = Phi_pj/sqrt2, X[j,2p+1] = -i Phi_pj/sqrt2.
// Empty orbital J = eta+u with an orthonormal basis vector g of col(Phi)^perp
// (from a Householder QR of Phi): selected rows r0 = eta+2u, r0+1:
//   X[r0,2p] = Re g_p, X[r0,2p+1] = Im g_p, X[r0+1,2p] = -Im g_p, X[r0+1,2p+1] = Re g_p.
// The rows are written in the physical order described before k_pfaff.
// One 64-lane workgroup per walker, lane = orbital row p (n <= 32).
// --------------------------------------------------------------------------
#define SO_NMAX 32
#define SO_NMAX_SUPPORTED 24   // formation LDS budget (X, C', T block) below 64 KB
__global__ __launch_bounds__(64) void k_walker_prep(int n, int eta, const double2 *__restrict__ phi,
                                                    double2 *__restrict__ X, int32_t *__restrict__ wstat) {
    __shared__ double2 R[SO_NMAX][SO_NMAX];
    __shared__ double2 V[SO_NMAX][SO_NMAX];
    __shared__ double betas[SO_NMAX];
    const int w = blockIdx.x;
    const int p = threadIdx.x;
    const int m = 2 * n - eta;
    const int d = 2 * n;
    const double2 *ph = phi + (size_t)w * n * eta;
    double2 *Xw = X + (size_t)w * m * d;
    double fro = 0.0;
    int finite = 1;
    if (p < n)
        for (int j = 0; j < eta; ++j) {
            double2 v = ph[p * eta + j];
            R[p][j] = v;
            fro += c_abs2(v);
            if (!isfinite(v.x) || !isfinite(v.y)) finite = 0;
        }
    fro = grp_sum<64>(fro);
    finite = __all(finite);
    const double fnorm = sqrt(fro);
    int rank_ok = 1;
    __syncthreads();
    for (int j = 0; j < eta; ++j) {
        double2 x = (p < n && p >= j) ? R[p][j] : c_make(0, 0);
        double nx2 = grp_sum<64>(c_abs2(x));
        double nx = sqrt(nx2);
        if (!(nx > 1e-13 * fnorm)) rank_ok = 0;
        double2 x0 = R[j][j];
        double ax = sqrt(c_abs2(x0));
        double2 phs = ax > 0 ? c_scale(x0, 1.0 / ax) : c_make(1, 0);
        double2 v = x;
        if (p == j) v = c_add(v, c_scale(phs, nx));
        double beta = (nx > 0) ? 1.0 / (nx2 + nx * ax) : 0.0;   // 2 / (v^H v)
        if (p < n) V[p][j] = v;
        if (p == 0) betas[j] = beta;
        __syncthreads();
        for (int c = j; c < eta; ++c) {
            double2 r = (p < n) ? R[p][c] : c_make(0, 0);
            double2 t = c_mul(c_conj(v), r);
            double sr = grp_sum<64>(t.x), si = grp_sum<64>(t.y);
            double2 s = c_scale(c_make(sr, si), beta);
            __syncthreads();
            if (p < n && p >= j) R[p][c] = c_sub(r, c_mul(s, v));
            __syncthreads();
        }
    }
    const double rs2 = 0.70710678118654752440;
    const int ne = n - eta;
    // occupied rows (physical rows ne .. ne+eta-1)
    if (p < n)
        for (int j = 0; j < eta; ++j) {
            double2 v = ph[p * eta + j];
            Xw[(size_t)(ne + j) * d + 2 * p] = c_scale(v, rs2);
            Xw[(size_t)(ne + j) * d + 2 * p + 1] = c_make(v.y * rs2, -v.x * rs2);
        }
    // empty rows: g = H_0 ... H_{eta-1} e_{eta+u}
    for (int u = 0; u < n - eta; ++u) {
        double2 g = c_make(p == eta + u ? 1.0 : 0.0, 0.0);
        for (int j = eta - 1; j >= 0; --j) {
            double2 vj = (p < n) ? V[p][j] : c_make(0, 0);
            double2 t = c_mul(c_conj(vj), g);
            double sr = grp_sum<64>(t.x), si = grp_sum<64>(t.y);
            double2 s = c_scale(c_make(sr, si), betas[j]);
            if (p < n) g = c_sub(g, c_mul(s, vj));
        }
        if (p < n) {   // physical rows u and m-1-u
            const int r0 = u, r1 = m - 1 - u;
            Xw[(size_t)r0 * d + 2 * p] = c_make(g.x, 0.0);
            Xw[(size_t)r0 * d + 2 * p + 1] = c_make(g.y, 0.0);
            Xw[(size_t)r1 * d + 2 * p] = c_make(-g.y, 0.0);
            Xw[(size_t)r1 * d + 2 * p + 1] = c_make(g.x, 0.0);
        }
    }
    if (p == 0 && wstat) wstat[w] = (rank_ok ? 0 : SO_WSTAT_RANK) | (finite ? 0 : SO_WSTAT_NONFINITE);
}

// --------------------------------------------------------------------------
// k_shadow_prep: C'_s = Q^T C_b Q (eq. b_mat; Supp. covariance matrix),
// C'_{mu nu} = sum_j beta_j (Q_{2j,mu} Q_{2j+1,nu} - Q_{2j+1,mu} Q_{2j,nu}).
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_shadow_prep(int n, const double *__restrict__ Q,
                                                     const uint64_t *__restrict__ bits, double *__restrict__ Cp) {
    extern __shared__ double Qs[];
    const int d = 2 * n;
    const int s = blockIdx.x;
    const double *Qg = Q + (size_t)s * d * d;
    for (int e = threadIdx.x; e < d * d; e += blockDim.x) Qs[e] = Qg[e];
    __syncthreads();
    const uint64_t b = bits[s];
    double *Cg = Cp + (size_t)s * d * d;
    for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
        const int mu = e / d, nu = e % d;
        double acc = 0.0;
        for (int j = 0; j < n; ++j) {
            const double beta = ((b >> j) & 1u) ? -1.0 : 1.0;
            acc = fma(beta, Qs[(2 * j) * d + mu] * Qs[(2 * j + 1) * d + nu] - Qs[(2 * j + 1) * d + mu] * Qs[(2 * j) * d + nu], acc);
        }
        Cg[e] = acc;
    }
}

// --------------------------------------------------------------------------
// k_form: B_ws = X_w C'_s X_w^T (eq. b_mat), m x m complex antisymmetric,
// written full (the lower triangle as the negated upper one) for the shadows
// of one chunk.  grid (W, ceil(Sc / spb)); dynamic LDS: X (m x 2n c128),
// C' (2n x 2n f64) and a block of FORM_RB rows of T = X C' (c128).
// --------------------------------------------------------------------------
#define FORM_RB 8
__global__ __launch_bounds__(256) void k_form(int n, int m, const double2 *__restrict__ X,
                                              const double *__restrict__ Cp, int64_t s0, int Sc, int spb,
                                              double2 *__restrict__ B) {
    extern __shared__ double2 lds2[];
    const int d = 2 * n;
    double2 *Xs = lds2;
    double2 *Ts = Xs + m * d;
    double *Cs = reinterpret_cast<double *>(Ts + FORM_RB * d);
    const int w = blockIdx.x;
    const double2 *Xg = X + (size_t)w * m * d;
    for (int e = threadIdx.x; e < m * d; e += blockDim.x) Xs[e] = Xg[e];
    const int sl0 = blockIdx.y * spb;
    const int sl1 = min(Sc, sl0 + spb);
    for (int sl = sl0; sl < sl1; ++sl) {
        const double *Cg = Cp + (size_t)(s0 + sl) * d * d;
        __syncthreads();
        for (int e = threadIdx.x; e < d * d; e += blockDim.x) Cs[e] = Cg[e];
        double2 *Bg = B + ((size_t)w * Sc + sl) * m * m;
        for (int i0 = 0; i0 < m; i0 += FORM_RB) {
            const int rb = min(FORM_RB, m - i0);
            __syncthreads();
            for (int e = threadIdx.x; e < rb * d; e += blockDim.x) {
                const int i = i0 + e / d, nu = e % d;
                double ar = 0.0, ai = 0.0;
                for (int mu = 0; mu < d; ++mu) {
                    const double2 xv = Xs[i * d + mu];
                    const double c = Cs[mu * d + nu];
                    ar = fma(xv.x, c, ar);
                    ai = fma(xv.y, c, ai);
                }
                Ts[e] = c_make(ar, ai);
            }
            __syncthreads();
            for (int e = threadIdx.x; e < rb * m; e += blockDim.x) {
                const int i = i0 + e / m, j = e % m;
                if (j < i) continue;
                double2 acc = c_make(0, 0);
                if (j > i)
                    for (int nu = 0; nu < d; ++nu) acc = c_fma(Ts[(i - i0) * d + nu], Xs[j * d + nu], acc);
                Bg[(size_t)i * m + j] = acc;
                Bg[(size_t)j * m + i] = c_make(-acc.x, -acc.y);
            }
        }
    }
}

// --------------------------------------------------------------------------
// Row order of X, B and the node matrices ("physical order").  The selected
// indices of the paper (occupied orbitals first, then the two Majoranas of
// each empty orbital) are stored permuted: with ne = n - eta empty orbitals,
// the pair of empty orbital t sits at rows (t, M-1-t) and the occupied
// orbitals fill rows ne .. ne+eta-1.  The selected vacuum covariance J then
// has J[t][M-1-t] = +1, J[M-1-t][t] = -1 (t < ne) and nothing else.  The
// Pfaffian of the permuted matrix differs by det(P) = +-1, folded into the
// node weights on the host.
// --------------------------------------------------------------------------

// DPP helpers within 16-lane rows
template <int CTRL>
__device__ __forceinline__ double dpp_f64_32(double v) {
    const long long b = __double_as_longlong(v);
    int lo = (int)b, hi = (int)(b >> 32);
    lo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
// broadcast lane SRC of each 16-lane row (row_newbcast, a 64-bit DPP move)
template <int SRC>
__device__ __forceinline__ double bc16(double v) {
    long long b = __double_as_longlong(v);
    b = __builtin_amdgcn_update_dpp(b, b, 0x150 + SRC, 0xf, 0xf, false);
    return __longlong_as_double(b);
}
template <int SRC>
__device__ __forceinline__ double2 bc16c(double2 v) { return c_make(bc16<SRC>(v.x), bc16<SRC>(v.y)); }
// same broadcast, with the (unused) old operand tied to `dep` so that it is
// neither merged with an earlier broadcast of the same value nor hoisted
// above the computation of `dep`
template <int SRC>
__device__ __forceinline__ double bc16d(double v, double dep) {
    asm("" : "+v"(v) : "v"(dep));   // v now depends on dep (no instruction emitted)
    return bc16<SRC>(v);
}
template <int SRC>
__device__ __forceinline__ double2 bc16cd(double2 v, double dep) { return c_make(bc16d<SRC>(v.x, dep), bc16d<SRC>(v.y, dep)); }
// sum over the 16 lanes of a row (rotations, every lane gets the total)
__device__ __forceinline__ double sum16(double v) {
    v += dpp_f64_32<0x128>(v);   // row_ror:8
    v += dpp_f64_32<0x124>(v);   // row_ror:4
    v += dpp_f64_32<0x122>(v);   // row_ror:2
    v += dpp_f64_32<0x121>(v);   // row_ror:1
    return v;
}

// --------------------------------------------------------------------------
// k_pfaff: per pair o = sum_k w_k Pf(s_k B + c_k J) (J = C_0^(s) in physical
// order, see above).
//
// Pfaffian by Householder tridiagonalisation (the unitary alternative to
// Parlett-Reid in Wimmer's Pfaffian algorithms): at even step k the column
// x = A[k+1:, k] is mapped to alpha e_1 by H = I - beta u u^H acting on
// indices k+1..m-1; H A H^T = H A conj(H) keeps A skew, multiplies Pf by
// det H = -1 and leaves A[k][k+1] = -alpha, so Pf gains the factor alpha.
// The trailing block is updated by the skew rank-2 form
//   A <- A + beta (u y^T - y u^T),  y = A conj(u)
// and the Pfaffian continues on indices k+2..m-1.  No pivot search and no
// row/column exchange: the data flow is static, so every broadcast source is
// a compile-time lane.
//
// Mapping: one node matrix per 16-lane DPP row (4 per wave); lane q < M/2
// owns rows q and M-1-q in registers (rows retire from the top, so both ends
// are paired to keep lanes busy).  Row j is owned by lane j (slot 0) for
// j < M/2 and by lane M-1-j (slot 1) otherwise; its values reach the other
// lanes by row_newbcast.  J is not stored: the registers hold s_k B and the
// J terms (which couple a lane's own two rows) are added explicitly.  Every
// elimination step is its own template instance, so register indices are
// constants.
// --------------------------------------------------------------------------
template <int M>
struct PfCtx {
    int q, ne;
    bool act;
    double2 ck;
};

template <int M, int J>
__device__ __forceinline__ double2 row_val(double2 v0, double2 v1) {
    // value held for row J by its owner lane, broadcast to the whole row
    if constexpr (J < M / 2) return bc16c<J>(v0);
    else return bc16c<M - 1 - J>(v1);
}

template <int M, int J>
__device__ __forceinline__ double2 row_val_dep(double2 v0, double2 v1, double dep) {
    if constexpr (J < M / 2) return bc16cd<J>(v0, dep);
    else return bc16cd<M - 1 - J>(v1, dep);
}

template <int M, int K>
__device__ __forceinline__ void pf_step(const PfCtx<M> &cx, double2 (&R0)[M], double2 (&R1)[M], double2 &pf) {
    constexpr int L = M / 2;
    const int q = cx.q;
    const int rb = M - 1 - q;
    const bool jq = cx.act && q < cx.ne;   // this lane's rows are a J pair
    // x_i = A[i][K] for the owned rows i > K; all conditionals are selects
    // (no divergent branches, which would make the allocator spill rows)
    const bool a0 = cx.act && q > K, a1 = cx.act && rb > K;
    double2 x0 = c_make(a0 ? R0[K].x : 0.0, a0 ? R0[K].y : 0.0);
    double2 x1 = c_make(a1 ? R1[K].x : 0.0, a1 ? R1[K].y : 0.0);
    // J[q][M-1-q] = +1 would lie in column K only for q = M-1-K < K, a row
    // already retired, so only the slot-1 row can meet J in column K.
    {
        const bool h = jq && q == K;      // J[M-1-q][q] = -1
        x1 = c_make(h ? x1.x - cx.ck.x : x1.x, h ? x1.y - cx.ck.y : x1.y);
    }
    const double nx2 = sum16(c_abs2(x0) + c_abs2(x1));
    const double2 xf = row_val<M, K + 1>(x0, x1);
    const double nx = sqrt(nx2);
    const double ax = sqrt(c_abs2(xf));
    // divisions are unconditional (a select on the operand, not a branch)
    const double iax = 1.0 / (ax > 0.0 ? ax : 1.0);
    const double2 phs = c_make(ax > 0.0 ? xf.x * iax : 1.0, ax > 0.0 ? xf.y * iax : 0.0);
    const double2 alpha = c_scale(phs, -nx);
    pf = c_mul(pf, alpha);
    if constexpr (K + 2 < M) {
        const double den = nx2 + nx * ax;
        const double beta = (nx > 0.0 ? 1.0 : 0.0) / (nx > 0.0 ? den : 1.0);
        const double2 piv = c_sub(xf, alpha);
        double2 u0 = x0, u1 = x1;
        if constexpr (K + 1 < L) {
            const bool h = (q == K + 1);
            u0 = c_make(h ? piv.x : x0.x, h ? piv.y : x0.y);
        } else {
            const bool h = (q == M - 2 - K);
            u1 = c_make(h ? piv.x : x1.x, h ? piv.y : x1.y);
        }
        const double2 v0 = c_conj(u0), v1 = c_conj(u1);
        // y_i = sum_{j>K} A_ij conj(u_j) for the owned rows (J: own partner row).
        // Each broadcast carries a dependence on the partial sum of two
        // columns earlier, which bounds how far the scheduler can hoist it.
        double2 y0 = c_make(0, 0), y1 = c_make(0, 0);
        {
            double d2 = nx, d1 = nx;
            [&]<int... I>(std::integer_sequence<int, I...>) {
                (([&] {
                     constexpr int jj = K + 1 + I;
                     const double2 ub = row_val_dep<M, jj>(v0, v1, d2);
                     y0 = c_fma(R0[jj], ub, y0);
                     y1 = c_fma(R1[jj], ub, y1);
                     d2 = d1;
                     d1 = y0.x;
                 }()), ...);
            }(std::make_integer_sequence<int, M - K - 1>{});
        }
        {   // J terms: J[q][M-1-q] conj(u_{M-1-q}) and J[M-1-q][q] conj(u_q)
            const bool h0 = jq && rb > K, h1 = jq && q > K;
            const double2 t0 = c_fma(cx.ck, v1, y0);
            const double2 t1 = c_sub(y1, c_mul(cx.ck, v0));
            y0 = c_make(h0 ? t0.x : y0.x, h0 ? t0.y : y0.y);
            y1 = c_make(h1 ? t1.x : y1.x, h1 ? t1.y : y1.y);
        }
        y0 = c_scale(y0, beta);
        y1 = c_scale(y1, beta);
        const double2 ny0 = c_make(-y0.x, -y0.y), ny1 = c_make(-y1.x, -y1.y);
        // A_ij += u_i y_j - y_i u_j on the trailing block j >= K+2, with the
        // same two-column dependence on the broadcasts
        {
            double d2 = ny0.x, d1 = ny1.x;
            [&]<int... I>(std::integer_sequence<int, I...>) {
                (([&] {
                     constexpr int jj = K + 2 + I;
                     const double2 yb = row_val_dep<M, jj>(y0, y1, d2);
                     const double2 ub = row_val_dep<M, jj>(u0, u1, d2);
                     R0[jj] = c_fma(u0, yb, c_fma(ny0, ub, R0[jj]));
                     R1[jj] = c_fma(u1, yb, c_fma(ny1, ub, R1[jj]));
                     d2 = d1;
                     d1 = R0[jj].x;
                 }()), ...);
            }(std::make_integer_sequence<int, M - K - 2>{});
        }
        pf_step<M, K + 2>(cx, R0, R1, pf);
    }
}

template <int M>
__global__ __launch_bounds__(64) void k_pfaff(const double2 *__restrict__ B, int ne, NodeTab tab,
                                              int64_t S, int64_t s0, int Sc, double2 *__restrict__ pairs) {
    constexpr int L = M / 2;
    constexpr int LD = M + 1;   // padded LDS row stride (bank spread)
    static_assert(M % 2 == 0 && L <= 16, "k_pfaff covers m <= 32");
    __shared__ double2 Bs[M * LD];

    const int lane = threadIdx.x;
    const int64_t pair = blockIdx.x;
    const int64_t w = pair / Sc, sl = pair % Sc;

    const double2 *Bp = B + pair * (int64_t)(M * M);
    for (int e = lane; e < M * M; e += 64) Bs[(e / M) * LD + (e % M)] = Bp[e];
    __syncthreads();

    PfCtx<M> cx;
    const int g = lane >> 4;
    cx.q = lane & 15;
    cx.act = cx.q < L;
    cx.ne = ne;
    const int ra = cx.act ? cx.q : 0, rb = cx.act ? (M - 1 - cx.q) : 0;

    double2 acc = c_make(0, 0);
    const int K = tab.K;
    const int rounds = (K + 3) / 4;
    for (int rd = 0; rd < rounds; ++rd) {
        const int kn = rd * 4 + g;
        const bool valid = kn < K;
        const int kk = valid ? kn : 0;
        const double2 sk = tab.s[kk];
        cx.ck = tab.c[kk];
        double2 R0[M], R1[M];
        if (tab.unit_b) {
#pragma unroll
            for (int j = 0; j < M; ++j) { R0[j] = Bs[ra * LD + j]; R1[j] = Bs[rb * LD + j]; }
        } else {
#pragma unroll
            for (int j = 0; j < M; ++j) { R0[j] = c_mul(Bs[ra * LD + j], sk); R1[j] = c_mul(Bs[rb * LD + j], sk); }
        }
        double2 pf = c_make(1, 0);
        pf_step<M, 0>(cx, R0, R1, pf);
        if (valid) acc = c_fma(tab.w[kk], pf, acc);
    }
    // fixed-order sum over the four node groups
    double2 tot = c_make(0, 0);
#pragma unroll
    for (int gg = 0; gg < 4; ++gg) tot = c_add(tot, grp_bcast<64>(acc, gg * 16));
    if (lane == 0) pairs[w * S + s0 + sl] = tot;
}

// --------------------------------------------------------------------------
// k_pfaff_wide: same estimate for 32 < m <= 64, one node matrix per wave,
// lane q < m owns row q; broadcasts go through LDS.  Used for n >= 18 with
// few electrons and for the n = 24 workload.
// --------------------------------------------------------------------------
template <int M, int K>
__device__ __forceinline__ void pfw_step(double2 (&R)[M], double2 *ubuf, double2 *ybuf, int q, int ne,
                                         double2 ck, double2 &pf) {
    const bool act = q < M;
    // J partner of row q and the sign of J[q][partner]
    const int pq = (q < ne) ? (M - 1 - q) : ((q >= M - ne && q < M) ? (M - 1 - q) : -1);
    const double sg = (q < ne) ? 1.0 : -1.0;
    double2 x = c_make(0, 0);
    if (act && q > K) {
        x = R[K];
        if (pq == K) x = c_add(x, c_scale(ck, sg));
    }
    const double nx2 = grp_sum<64>(c_abs2(x));
    const double2 xf = grp_bcast<64>(x, K + 1);
    const double nx = sqrt(nx2);
    const double ax = sqrt(c_abs2(xf));
    const double2 phs = ax > 0.0 ? c_scale(xf, 1.0 / ax) : c_make(1, 0);
    const double2 alpha = c_scale(phs, -nx);
    pf = c_mul(pf, alpha);
    if constexpr (K + 2 < M) {
        const double beta = nx > 0.0 ? 1.0 / (nx2 + nx * ax) : 0.0;
        double2 u = x;
        if (q == K + 1) u = c_sub(xf, alpha);
        if (act && q >= K + 1) ubuf[q] = c_conj(u);
        __syncthreads();
        double2 y = c_make(0, 0);
#pragma unroll
        for (int j = K + 1; j < M; ++j) y = c_fma(R[j], ubuf[j], y);
        if (pq > K) y = c_fma(c_scale(ck, sg), ubuf[pq], y);
        y = c_scale(y, beta);
        if (act && q >= K + 2) ybuf[q] = y;
        __syncthreads();
        const double2 ny = c_make(-y.x, -y.y);
#pragma unroll
        for (int j = K + 2; j < M; ++j) R[j] = c_fma(u, ybuf[j], c_fma(ny, c_conj(ubuf[j]), R[j]));
        __syncthreads();
        pfw_step<M, K + 2>(R, ubuf, ybuf, q, ne, ck, pf);
    }
}

template <int M>
__global__ __launch_bounds__(64) void k_pfaff_wide(const double2 *__restrict__ B, int ne, NodeTab tab,
                                                   int64_t S, int64_t s0, int Sc, double2 *__restrict__ pairs) {
    static_assert(M <= 64 && M % 2 == 0, "k_pfaff_wide covers m <= 64");
    __shared__ double2 ubuf[M];
    __shared__ double2 ybuf[M];
    const int q = threadIdx.x;
    const int64_t pair = blockIdx.x;
    const int64_t w = pair / Sc, sl = pair % Sc;
    const double2 *Bp = B + pair * (int64_t)(M * M);
    const int r = q < M ? q : 0;
    double2 acc = c_make(0, 0);
    for (int kn = 0; kn < tab.K; ++kn) {
        const double2 sk = tab.s[kn];
        double2 R[M];
#pragma unroll
        for (int j = 0; j < M; ++j) R[j] = tab.unit_b ? Bp[r * M + j] : c_mul(Bp[r * M + j], sk);
        double2 pf = c_make(1, 0);
        pfw_step<M, 0>(R, ubuf, ybuf, q, ne, tab.c[kn], pf);
        acc = c_fma(tab.w[kn], pf, acc);
    }
    if (q == 0) pairs[w * S + s0 + sl] = acc;
}

// --------------------------------------------------------------------------
// k_reduce: S_w = (1/S) sum_s o_ws, fixed order: lane l sums s = l, l+64, ...
// then a fixed butterfly.  Sets SO_WSTAT_NONFINITE.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_reduce(const double2 *__restrict__ pairs, int64_t S,
                                               double2 *__restrict__ out, int32_t *__restrict__ wstat) {
    const int w = blockIdx.x;
    const int lane = threadIdx.x;
    const double2 *pw = pairs + (size_t)w * S;
    double ar = 0.0, ai = 0.0;
    for (int64_t s = lane; s < S; s += 64) {
        double2 v = pw[s];
        ar += v.x;
        ai += v.y;
    }
    ar = grp_sum<64>(ar);
    ai = grp_sum<64>(ai);
    if (lane == 0) {
        const double inv = 1.0 / (double)S;
        double2 r = c_make(ar * inv, ai * inv);
        int32_t st = wstat ? wstat[w] : 0;
        if (st & SO_WSTAT_RANK) r = c_make(NAN, NAN);
        if (!isfinite(r.x) || !isfinite(r.y)) st |= SO_WSTAT_NONFINITE;
        out[w] = r;
        if (wstat) wstat[w] = st;
    }
}

// ==========================================================================
// host side
// ==========================================================================
namespace {

// ---- double-double arithmetic for the Chebyshev weights (ill-conditioned
// Vandermonde solve); see Dekker / Knuth error-free transformations.
struct dd { double hi, lo; };
inline dd dd_two_sum(double a, double b) {
    double s = a + b, bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
inline dd dd_add(dd a, dd b) {
    dd s = dd_two_sum(a.hi, b.hi);
    double lo = s.lo + a.lo + b.lo;
    return dd_two_sum(s.hi, lo);
}
inline dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
inline dd dd_mul(dd a, dd b) {
    double p = a.hi * b.hi;
    double e = std::fma(a.hi, b.hi, -p);
    e += a.hi * b.lo + a.lo * b.hi;
    return dd_two_sum(p, e);
}
inline dd dd_div(dd a, dd b) {
    double q1 = a.hi / b.hi;
    dd r = dd_add(a, dd_neg(dd_mul({q1, 0.0}, b)));
    double q2 = r.hi / b.hi;
    r = dd_add(r, dd_neg(dd_mul({q2, 0.0}, b)));
    double q3 = r.hi / b.hi;
    dd q = dd_two_sum(q1, q2);
    return dd_add(q, {q3, 0.0});
}
inline dd dd_from(double a) { return {a, 0.0}; }

struct cld { long double re, im; };

int mvalue(int n, int eta) { return 2 * n - eta; }

// compiled Pfaffian sizes
bool m_supported(int m) { return m >= 2 && m <= 48 && (m % 2 == 0); }

bool params_ok(const so_params *p, int *K_out) {
    if (!p) return false;
    if (p->n < 2 || p->n > SO_NMAX_SUPPORTED) return false;
    if (p->eta < 2 || p->eta > p->n || (p->eta & 1)) return false;
    if (p->nodes != SO_NODES_UNIT && p->nodes != SO_NODES_CHEBYSHEV) return false;
    if (p->precision != SO_PREC_FP64 && p->precision != SO_PREC_MIXED) return false;
    if (p->flags & ~SO_FLAG_PAPER_NORM) return false;
    const int ell = p->n - p->eta / 2;
    const int K = p->n_nodes ? p->n_nodes : p->n + 1;
    if (K < ell + 1 || K > SO_KMAX) return false;
    if (K_out) *K_out = K;
    return true;
}

// Node weights: Pf(A(z)) = sum_{x=0}^{l} c_x z^x with l = n - eta/2, and
// o = pref sum_x mu_x c_x with mu_x = C(2n,2x)/C(n,x) and
// pref = 2 i^{eta/2} / 2^{n - eta/2} (estimator o_p, times 2 unless
// SO_FLAG_PAPER_NORM).  Interpolation at the nodes gives o = sum_k w_k p_k,
// w = pref V^{-T} mu, V_{kx} = z_k^x.
void compute_weights(const so_params *p, int K, double2 *z, double2 *w) {
    const int n = p->n, eta = p->eta, ell = n - eta / 2;
    long double mu[SO_KMAX];
    for (int x = 0; x < K; ++x) {
        if (x > ell) { mu[x] = 0.0L; continue; }
        // C(2n,2x) and C(n,x) as exact integers (n <= 32: C(64,32) < 2^64)
        unsigned long long a = 1, b = 1;
        for (int t = 1; t <= 2 * x; ++t) a = a * (unsigned long long)(2 * n - 2 * x + t) / t;
        for (int t = 1; t <= x; ++t) b = b * (unsigned long long)(n - x + t) / t;
        mu[x] = (long double)a / (long double)b;
    }
    // pref = 2 i^{eta/2} 2^{-(n-eta/2)}
    const long double mag = ldexpl((p->flags & SO_FLAG_PAPER_NORM) ? 1.0L : 2.0L, -(n - eta / 2));
    cld pref;
    switch ((eta / 2) % 4) {
        case 0: pref = {mag, 0.0L}; break;
        case 1: pref = {0.0L, mag}; break;
        case 2: pref = {-mag, 0.0L}; break;
        default: pref = {0.0L, -mag}; break;
    }
    if (p->nodes == SO_NODES_UNIT) {
        const long double two_pi = 6.283185307179586476925286766559005768L;
        for (int k = 0; k < K; ++k) {
            long double sr = 0.0L, si = 0.0L;
            for (int x = 0; x <= ell && x < K; ++x) {
                const long double th = -two_pi * (long double)((long long)k * x % K) / K;
                sr += mu[x] * cosl(th);
                si += mu[x] * sinl(th);
            }
            sr /= K;
            si /= K;
            w[k].x = (double)(pref.re * sr - pref.im * si);
            w[k].y = (double)(pref.re * si + pref.im * sr);
            const long double tk = two_pi * (long double)k / K;
            z[k].x = (double)cosl(tk);
            z[k].y = (double)sinl(tk);
        }
    } else {
        const long double pi = 3.141592653589793238462643383279502884L;
        double zr[SO_KMAX];
        for (int k = 0; k < K; ++k) {
            zr[k] = (double)cosl((2.0L * k + 1.0L) * pi / (2.0L * K));
            z[k].x = zr[k];
            z[k].y = 0.0;
        }
        // solve V^T v = mu in double-double (V^T_{xk} = z_k^x), partial pivoting
        static dd A[SO_KMAX][SO_KMAX + 1];
        for (int x = 0; x < K; ++x) {
            for (int k = 0; k < K; ++k) {
                dd zz = dd_from(1.0);
                for (int e = 0; e < x; ++e) zz = dd_mul(zz, dd_from(zr[k]));
                A[x][k] = zz;
            }
            long double mx = mu[x];
            double h = (double)mx;
            A[x][K] = {h, (double)(mx - (long double)h)};
        }
        for (int c = 0; c < K; ++c) {
            int pr = c;
            for (int r = c + 1; r < K; ++r)
                if (std::fabs(A[r][c].hi) > std::fabs(A[pr][c].hi)) pr = r;
            if (pr != c)
                for (int j = 0; j <= K; ++j) { dd t = A[c][j]; A[c][j] = A[pr][j]; A[pr][j] = t; }
            for (int r = c + 1; r < K; ++r) {
                dd f = dd_div(A[r][c], A[c][c]);
                for (int j = c; j <= K; ++j) A[r][j] = dd_add(A[r][j], dd_neg(dd_mul(f, A[c][j])));
            }
        }
        dd sol[SO_KMAX];
        for (int r = K - 1; r >= 0; --r) {
            dd s = A[r][K];
            for (int j = r + 1; j < K; ++j) s = dd_add(s, dd_neg(dd_mul(A[r][j], sol[j])));
            sol[r] = dd_div(s, A[r][r]);
        }
        for (int k = 0; k < K; ++k) {
            const long double v = (long double)sol[k].hi + (long double)sol[k].lo;
            w[k].x = (double)(pref.re * v);
            w[k].y = (double)(pref.im * v);
        }
    }
}

// Node table for the kernels.  Unit-circle nodes use the rescaled matrix
// B + conj(z) J = A(z)/z (|z| = 1), Pf(A(z)) = z^{m/2} Pf(B + conj(z) J), so
// the register rows start as B itself; Chebyshev nodes use z B + J.
void build_nodetab(const so_params *p, int K, NodeTab *t) {
    double2 z[SO_KMAX], w[SO_KMAX];
    compute_weights(p, K, z, w);
    const int m = mvalue(p->n, p->eta);
    // sign of the selected-index permutation into physical order (det P)
    const int ne = p->n - p->eta;
    int perm[96];
    for (int i = 0; i < p->eta; ++i) perm[i] = ne + i;
    for (int u = 0; u < ne; ++u) { perm[p->eta + 2 * u] = u; perm[p->eta + 2 * u + 1] = m - 1 - u; }
    int inv = 0;
    for (int i = 0; i < m; ++i)
        for (int j = i + 1; j < m; ++j) inv += perm[i] > perm[j];
    const double psign = (inv & 1) ? -1.0 : 1.0;
    for (int k = 0; k < K; ++k) { w[k].x *= psign; w[k].y *= psign; }
    std::memset(t, 0, sizeof(*t));
    t->K = K;
    t->unit_b = (p->nodes == SO_NODES_UNIT) ? 1 : 0;
    for (int k = 0; k < K; ++k) {
        if (p->nodes == SO_NODES_UNIT) {
            const long double two_pi = 6.283185307179586476925286766559005768L;
            const long double th = two_pi * (long double)((long long)k * (m / 2) % K) / K;   // z^{m/2}
            const double cr = (double)cosl(th), ci = (double)sinl(th);
            t->s[k].x = 1.0; t->s[k].y = 0.0;
            t->c[k].x = z[k].x; t->c[k].y = -z[k].y;
            t->w[k].x = w[k].x * cr - w[k].y * ci;
            t->w[k].y = w[k].x * ci + w[k].y * cr;
        } else {
            t->s[k] = z[k];
            t->c[k].x = 1.0; t->c[k].y = 0.0;
            t->w[k] = w[k];
        }
    }
}

struct Layout {
    size_t off_X, off_C, off_B, off_pairs, off_stat, total;
    int Sc;
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

constexpr size_t kBChunkBytes = (size_t)512 << 20;   // budget for one chunk of B matrices

Layout make_layout(int n, int eta, int64_t W, int64_t S, bool need_pairs) {
    Layout L{};
    const int m = mvalue(n, eta), d = 2 * n;
    const size_t per_shadow = (size_t)W * m * m * sizeof(double2);
    int64_t Sc = (int64_t)(kBChunkBytes / (per_shadow ? per_shadow : 1));
    if (Sc < 1) Sc = 1;
    if (Sc > S) Sc = S;
    L.Sc = (int)Sc;
    size_t o = 0;
    L.off_X = o; o = align_up(o + (size_t)W * m * d * sizeof(double2));
    L.off_C = o; o = align_up(o + (size_t)S * d * d * sizeof(double));
    L.off_B = o; o = align_up(o + (size_t)W * Sc * m * m * sizeof(double2));
    L.off_pairs = o; o = align_up(o + (need_pairs ? (size_t)W * S * sizeof(double2) : 0));
    L.off_stat = o; o = align_up(o + (size_t)W * sizeof(int32_t));
    L.total = o;
    return L;
}

template <int M>
hipError_t launch_pfaff_m(const double2 *B, int ne, const NodeTab &tab, int64_t S, int64_t s0, int Sc,
                          int64_t npairs, double2 *pairs, hipStream_t st) {
    dim3 grid((unsigned)npairs);
    if constexpr (M <= 32) {
        hipLaunchKernelGGL((k_pfaff<M>), grid, dim3(64), 0, st, B, ne, tab, S, s0, Sc, pairs);
    } else {
        hipLaunchKernelGGL((k_pfaff_wide<M>), grid, dim3(64), 0, st, B, ne, tab, S, s0, Sc, pairs);
    }
    return hipGetLastError();
}

hipError_t launch_pfaff(int m, const double2 *B, int ne, const NodeTab &tab, int64_t S, int64_t s0, int Sc,
                        int64_t npairs, double2 *pairs, hipStream_t st) {
    switch (m) {
#define SO_CASE(MM) case MM: return launch_pfaff_m<MM>(B, ne, tab, S, s0, Sc, npairs, pairs, st);
        SO_CASE(2) SO_CASE(4) SO_CASE(6) SO_CASE(8) SO_CASE(10) SO_CASE(12) SO_CASE(14) SO_CASE(16)
        SO_CASE(18) SO_CASE(20) SO_CASE(22) SO_CASE(24) SO_CASE(26) SO_CASE(28) SO_CASE(30) SO_CASE(32)
        SO_CASE(34) SO_CASE(36) SO_CASE(38) SO_CASE(40) SO_CASE(42) SO_CASE(44) SO_CASE(46) SO_CASE(48)
#undef SO_CASE
        default: return hipErrorInvalidValue;
    }
}

// ---- optional per-kernel timing (benchmarks): HIP events around launches
enum { PROF_PFAFF = 0, PROF_FORM = 1, PROF_NKIND = 2 };
struct ProfRec { hipEvent_t a, b; int kind; int64_t units; };
struct ProfState {
    bool on = false;
    ProfRec *recs = nullptr;
    size_t n = 0, cap = 0;
};
ProfState g_prof;

hipError_t prof_begin(hipStream_t st, hipEvent_t *a) {
    if (!g_prof.on) return hipSuccess;
    hipError_t e = hipEventCreate(a);
    if (e == hipSuccess) e = hipEventRecord(*a, st);
    return e;
}
hipError_t prof_end(hipStream_t st, hipEvent_t a, int kind, int64_t units) {
    if (!g_prof.on) return hipSuccess;
    hipEvent_t b;
    hipError_t e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e != hipSuccess) return e;
    if (g_prof.n == g_prof.cap) {
        size_t nc = g_prof.cap ? 2 * g_prof.cap : 1024;
        ProfRec *nr = static_cast<ProfRec *>(realloc(g_prof.recs, nc * sizeof(ProfRec)));
        if (!nr) return hipErrorOutOfMemory;
        g_prof.recs = nr;
        g_prof.cap = nc;
    }
    g_prof.recs[g_prof.n++] = ProfRec{a, b, kind, units};
    return hipSuccess;
}

}  // namespace

// ==========================================================================
// C ABI
// ==========================================================================
extern "C" {

int so_max_n(void) { return SO_NMAX_SUPPORTED; }

int so_supported(int n, int eta) {
    if (n < 2 || n > SO_NMAX_SUPPORTED || eta < 2 || eta > n || (eta & 1)) return 0;
    return m_supported(mvalue(n, eta)) ? 1 : 0;
}

so_status so_workspace_size(const so_params *p, int64_t n_walkers, int64_t n_shadows, int with_grad,
                            size_t *bytes) {
    int K;
    if (!bytes || !params_ok(p, &K) || n_walkers < 1 || n_shadows < 1) return SO_ERR_ARG;
    if (!so_supported(p->n, p->eta)) return SO_ERR_UNSUPPORTED;
    (void)with_grad;
    Layout L = make_layout(p->n, p->eta, n_walkers, n_shadows, true);
    *bytes = L.total;
    return SO_OK;
}

so_status so_node_weights(const so_params *p, so_c64 *nodes, so_c64 *weights, int *n_nodes) {
    int K;
    if (!params_ok(p, &K) || !nodes || !weights) return SO_ERR_ARG;
    double2 z[SO_KMAX], w[SO_KMAX];
    compute_weights(p, K, z, w);
    for (int k = 0; k < K; ++k) {
        nodes[k].re = z[k].x; nodes[k].im = z[k].y;
        weights[k].re = w[k].x; weights[k].im = w[k].y;
    }
    if (n_nodes) *n_nodes = K;
    return SO_OK;
}

so_status shadow_overlap(const so_params *p, const so_c64 *phi, int64_t n_walkers, const double *Q,
                         const uint64_t *bits, int64_t n_shadows, so_c64 *overlap, so_c64 *pair_out,
                         int32_t *status, void *workspace, size_t workspace_bytes, void *stream) {
    int K;
    if (!params_ok(p, &K) || !phi || !Q || !bits || !overlap || n_walkers < 1 || n_shadows < 1)
        return SO_ERR_ARG;
    if (!so_supported(p->n, p->eta)) return SO_ERR_UNSUPPORTED;
    if (p->precision != SO_PREC_FP64) return SO_ERR_UNSUPPORTED;
    if (n_walkers > (int64_t)INT32_MAX || n_shadows > (int64_t)INT32_MAX) return SO_ERR_ARG;
    const int n = p->n, eta = p->eta, m = mvalue(n, eta), d = 2 * n;
    Layout L = make_layout(n, eta, n_walkers, n_shadows, true);
    if (!workspace || workspace_bytes < L.total) return SO_ERR_WORKSPACE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(workspace);
    double2 *X = reinterpret_cast<double2 *>(ws + L.off_X);
    double *Cp = reinterpret_cast<double *>(ws + L.off_C);
    double2 *Bb = reinterpret_cast<double2 *>(ws + L.off_B);
    double2 *pairs = pair_out ? reinterpret_cast<double2 *>(pair_out) : reinterpret_cast<double2 *>(ws + L.off_pairs);
    int32_t *wst = status ? status : reinterpret_cast<int32_t *>(ws + L.off_stat);
    NodeTab tab;
    build_nodetab(p, K, &tab);
    const int64_t W = n_walkers, S = n_shadows;

    hipLaunchKernelGGL(k_walker_prep, dim3((unsigned)W), dim3(64), 0, st, n, eta,
                       reinterpret_cast<const double2 *>(phi), X, wst);
    if (hipGetLastError() != hipSuccess) return SO_ERR_HIP;
    hipLaunchKernelGGL(k_shadow_prep, dim3((unsigned)S), dim3(256), (size_t)d * d * sizeof(double), st, n, Q,
                       bits, Cp);
    if (hipGetLastError() != hipSuccess) return SO_ERR_HIP;
    const int spb = 8;
    const size_t form_lds = (size_t)(m + FORM_RB) * d * sizeof(double2) + (size_t)d * d * sizeof(double);
    for (int64_t s0 = 0; s0 < S; s0 += L.Sc) {
        const int Sc = (int)((S - s0) < L.Sc ? (S - s0) : L.Sc);
        dim3 fgrid((unsigned)W, (unsigned)((Sc + spb - 1) / spb));
        hipEvent_t ea = nullptr, eb = nullptr;
        if (prof_begin(st, &ea) != hipSuccess) return SO_ERR_HIP;
        hipLaunchKernelGGL(k_form, fgrid, dim3(256), form_lds, st, n, m, X, Cp, s0, Sc, spb, Bb);
        if (hipGetLastError() != hipSuccess) return SO_ERR_HIP;
        if (prof_end(st, ea, PROF_FORM, W * Sc) != hipSuccess) return SO_ERR_HIP;
        if (prof_begin(st, &eb) != hipSuccess) return SO_ERR_HIP;
        if (launch_pfaff(m, Bb, n - eta, tab, S, s0, Sc, W * Sc, pairs, st) != hipSuccess) return SO_ERR_HIP;
        if (prof_end(st, eb, PROF_PFAFF, W * Sc) != hipSuccess) return SO_ERR_HIP;
    }
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)W), dim3(64), 0, st, pairs, S,
                       reinterpret_cast<double2 *>(overlap), wst);
    if (hipGetLastError() != hipSuccess) return SO_ERR_HIP;
    return SO_OK;
}

so_status shadow_overlap_grad(const so_params *p, const so_c64 *phi, int64_t n_walkers, const double *Q,
                              const uint64_t *bits, int64_t n_shadows, so_c64 *overlap, so_c64 *dlog,
                              so_c64 *green, int32_t *status, void *workspace, size_t workspace_bytes,
                              void *stream) {
    (void)p; (void)phi; (void)n_walkers; (void)Q; (void)bits; (void)n_shadows; (void)overlap;
    (void)dlog; (void)green; (void)status; (void)workspace; (void)workspace_bytes; (void)stream;
    return SO_ERR_UNSUPPORTED;
}

so_status so_profile_enable(int on) {
    g_prof.on = on != 0;
    return SO_OK;
}

so_status so_profile_read(int kind, double *ms, int64_t *launches, int64_t *units) {
    if (kind < 0 || kind >= PROF_NKIND || !ms || !launches || !units) return SO_ERR_ARG;
    double tot = 0.0;
    int64_t cnt = 0, un = 0;
    size_t keep = 0;
    for (size_t i = 0; i < g_prof.n; ++i) {
        ProfRec &r = g_prof.recs[i];
        if (r.kind != kind) { g_prof.recs[keep++] = r; continue; }
        float t = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
            return SO_ERR_HIP;
        tot += t;
        ++cnt;
        un += r.units;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof.n = keep;
    *ms = tot;
    *launches = cnt;
    *units = un;
    return SO_OK;
}

const char *so_status_string(int s) {
    switch (s) {
        case SO_OK: return "ok";
        case SO_ERR_ARG: return "invalid argument";
        case SO_ERR_UNSUPPORTED: return "unsupported (n, eta) or mode";
        case SO_ERR_HIP: return "HIP launch failed";
        case SO_ERR_WORKSPACE: return "workspace missing or too small";
        default: return "unknown status";
    }
}

}  // extern "C"
