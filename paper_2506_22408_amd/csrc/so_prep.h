// so_prep.h -- per-walker and per-shadow preparation kernels.
//
// Row order of X, B and the node matrices.  The paper's selected index set
// (first Majorana of each occupied orbital, both Majoranas of each empty
// orbital) is stored as [occupied (eta rows), empty (2 ne rows)] with
// ne = n - eta; the two rows of empty orbital t sit at eta + t and
// eta + 2ne - 1 - t.  The selected vacuum covariance J is then zero on the
// occupied rows and J[eta+t][eta+2ne-1-t] = +1, J[eta+2ne-1-t][eta+t] = -1.
// The Pfaffian in this order differs from the paper's order by the sign of
// the permutation, folded into the node weights on the host.
#pragma once
#include "so_common.h"

// --------------------------------------------------------------------------
// k_walker_prep: the walker matrix X_w (Supp. "Matrix Definitions": the
// selected rows of W M_phi, with the walker's orbital rotation
// G = [Phi | Phi_perp]), stored as the real d x d matrix (d = 2n)
//   Xall = [Re X_O ; Im X_O ; X_U]
// in MFMA A order (so_common.h).  X_O (eta x d, complex) holds the occupied
// rows and X_U (2ne x d) the empty rows, which are real.  Occupied orbital j:
//   X_O[j,2p] = Phi_pj/sqrt2, X_O[j,2p+1] = -i Phi_pj/sqrt2.
// Empty orbital t with an orthonormal basis vector g of col(Phi)^perp (from a
// Householder QR of Phi): X_U row t = (Re g_p, Im g_p)_p and X_U row 2ne-1-t =
// (-Im g_p, Re g_p)_p.  Row i of B is X_O row i (i < eta) or X_U row i - eta.
// One 64-lane workgroup per walker, lane = orbital row p (n <= 32).  Block 0
// also clears the fallback-queue counter of this call.
//
// With logdet (the overlap path): the occupied rows are taken from the
// orthonormal factor instead, Phi = Qf R (the same Householder QR), and
// logdet[w] = log det R = sum_j log|R_jj| + i sum_j arg R_jj.  The estimator
// is multilinear in the walker's orbitals, o(Phi) = det R o(Qf), so the
// kernels evaluate o(Qf), whose node Pfaffians are bounded for every walker
// norm, and k_reduce applies det R (in log form when the log output is asked
// for).  Without logdet (derivative and energy paths, which differentiate
// through Phi) X_O comes from Phi itself.  With qf and rf (the derivative
// path) the factors Qf (n x eta) and R (eta x eta) are written out as well:
// the derivative is then taken at Qf and carried back to Phi
// (k_grad_walker).
// --------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_walker_prep(int n, int eta, const double2 *__restrict__ phi,
                                                    double *__restrict__ Xa, int32_t *__restrict__ wstat,
                                                    so_u64 *__restrict__ fb_count,
                                                    double2 *__restrict__ logdet = nullptr,
                                                    double2 *__restrict__ qf = nullptr,
                                                    double2 *__restrict__ rf = nullptr) {
    __shared__ double2 R[SO_NMAX][SO_NMAX];
    __shared__ double2 V[SO_NMAX][SO_NMAX];
    __shared__ double betas[SO_NMAX];
    const int w = blockIdx.x;
    const int p = threadIdx.x;
    if (w == 0 && p == 0 && fb_count) *fb_count = 0ull;
    const int d = 2 * n;
    const int ne = n - eta;
    const int T = so_tiles(n), DP = 16 * T;
    const double2 *ph = phi + (size_t)w * n * eta;
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
    double lmag = 0.0, larg = 0.0;   // log det R (lane-uniform)
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
        // H x = -phs nx e_j: R_jj = -phs nx
        lmag += log(nx);
        larg += atan2(-phs.y, -phs.x);
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
    // with rf: R (eta x eta, upper triangular, row-major) before R's rows are reused
    if (rf && p < eta)
        for (int c = 0; c < eta; ++c) rf[((size_t)w * eta + p) * eta + c] = c >= p ? R[p][c] : c_make(0, 0);
    __syncthreads();
    // g_t = H_0 ... H_{eta-1} e_{eta+t}, kept in R[t][.] (R is no longer
    // needed); with logdet also the orthonormal factor's columns
    // q_j = H_0 ... H_{eta-1} e_j, kept in R[ne + j][.]
    const int ncols = logdet ? ne + eta : ne;
    for (int t = 0; t < ncols; ++t) {
        const int e = t < ne ? eta + t : t - ne;
        double2 g = c_make(p == e ? 1.0 : 0.0, 0.0);
        for (int j = eta - 1; j >= 0; --j) {
            double2 vj = (p < n) ? V[p][j] : c_make(0, 0);
            double2 tt = c_mul(c_conj(vj), g);
            double sr = grp_sum<64>(tt.x), si = grp_sum<64>(tt.y);
            double2 s = c_scale(c_make(sr, si), betas[j]);
            if (p < n) g = c_sub(g, c_mul(s, vj));
        }
        if (p < n) R[t][p] = g;
    }
    __syncthreads();
    const double rs2 = 0.70710678118654752440;
    double *Xw = Xa + (size_t)w * DP * DP;
    for (int f = p; f < DP * DP; f += 64) {
        int row, col;
        ao_rowcol(f, T, row, col);
        double val = 0.0;
        if (row < d && col < d) {
            const int q = col >> 1, odd = col & 1;
            if (row < 2 * eta) {
                const int j = row < eta ? row : row - eta;
                const double2 v = logdet ? R[ne + j][q] : ph[q * eta + j];
                if (row < eta) val = odd ? v.y * rs2 : v.x * rs2;    // Re X_O
                else val = odd ? -v.x * rs2 : v.y * rs2;            // Im X_O
            } else {
                const int u = row - 2 * eta;
                if (u < ne) {
                    const double2 g = R[u][q];
                    val = odd ? g.y : g.x;
                } else {
                    const double2 g = R[2 * ne - 1 - u][q];
                    val = odd ? g.x : -g.y;
                }
            }
        }
        Xw[f] = val;
    }
    if (p == 0 && wstat) wstat[w] = (rank_ok ? 0 : SO_WSTAT_RANK) | (finite ? 0 : SO_WSTAT_NONFINITE);
    if (p == 0 && logdet) logdet[w] = c_make(lmag, remainder(larg, 2.0 * M_PI));
    // with qf: the orthonormal factor (n x eta, row-major like Phi)
    if (qf && logdet && p < n)
        for (int j = 0; j < eta; ++j) qf[((size_t)w * n + p) * eta + j] = R[ne + j][p];
}

// --------------------------------------------------------------------------
// k_shadow_prep: C'_s = Q^T C_b Q (eq. b_mat; Supp. covariance matrix),
// C'_{mu nu} = sum_j beta_j (Q_{2j,mu} Q_{2j+1,nu} - Q_{2j+1,mu} Q_{2j,nu}),
// written in MFMA A order, zero-padded to DP x DP.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_shadow_prep(int n, const double *__restrict__ Q,
                                                     const uint64_t *__restrict__ bits, double *__restrict__ Ca) {
    extern __shared__ double Qs[];
    const int d = 2 * n;
    const int T = so_tiles(n), DP = 16 * T;
    const int s = blockIdx.x;
    const double *Qg = Q + (size_t)s * d * d;
    for (int e = threadIdx.x; e < d * d; e += blockDim.x) Qs[e] = Qg[e];
    __syncthreads();
    const uint64_t b = bits[s];
    double *Cg = Ca + (size_t)s * DP * DP;
    for (int f = threadIdx.x; f < DP * DP; f += blockDim.x) {
        int mu, nu;
        ao_rowcol(f, T, mu, nu);
        double acc = 0.0;
        if (mu < d && nu < d)
            for (int j = 0; j < n; ++j) {
                const double beta = ((b >> j) & 1u) ? -1.0 : 1.0;
                acc = fma(beta, Qs[(2 * j) * d + mu] * Qs[(2 * j + 1) * d + nu] - Qs[(2 * j + 1) * d + mu] * Qs[(2 * j) * d + nu], acc);
            }
        Cg[f] = acc;
    }
}

// --------------------------------------------------------------------------
// k_to_f32: single-precision copies of the walker matrices (sig = 0) or the
// shadow covariances (sig = 1, rows in the order sig16) for the
// mixed-precision formation, from the FP64 matrices in A order.  count
// matrices of DP x DP; grid (ceil(DP^2 / 256), up to 65535), the y blocks
// striding over the matrices.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_to_f32(int T, int sig, int64_t count, const double *__restrict__ A64,
                                                float *__restrict__ A32) {
    const int DP = 16 * T;
    const int f = blockIdx.x * 256 + threadIdx.x;
    if (f >= DP * DP) return;
    int row, col;
    ao32_rowcol(f, T, row, col);
    if (sig) row = sig16(row);
    const int src = ao_index(row, col, T);
    for (int64_t g = blockIdx.y; g < count; g += gridDim.y) {
        const size_t base = (size_t)g * DP * DP;
        A32[base + f] = (float)A64[base + src];
    }
}

// k_perm_match: for a signed-permutation shadow C'_s = Q^T C_b Q is a signed
// matching (one entry +-1 per row, computed exactly from entries 0 and +-1).
// match[s][mu] = pi(mu) | 0x100 if the entry is -1, for the rows mu < 2n;
// 0x200 for the padding rows mu < DP; -1 for a row that is not one entry +-1
// among zeros.  Grid S, 64 threads.
__global__ __launch_bounds__(64) void k_perm_match(int n, const double *__restrict__ Ca, int32_t *__restrict__ match) {
    const int mu = threadIdx.x, d = 2 * n, T = so_tiles(n), DP = 16 * T;
    if (mu >= DP) return;
    const int64_t s = blockIdx.x;
    int32_t out = 0x200;
    if (mu < d) {
        const double *C = Ca + (size_t)s * DP * DP;
        int cnt = 0, col = 0;
        double v = 0.0;
        for (int c = 0; c < d; ++c) {
            const double x = C[ao_index(mu, c, T)];
            if (x != 0.0) {
                ++cnt;
                col = c;
                v = x;
            }
        }
        out = (cnt == 1 && (v == 1.0 || v == -1.0)) ? (col | (v < 0.0 ? 0x100 : 0)) : -1;
    }
    match[s * DP + mu] = out;
}

