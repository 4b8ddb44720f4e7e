/*
 * shadow_oracle.c -- plain FP64 CPU oracle for the matchgate-shadow overlap
 * estimator of QC-AFQMC (Zhao et al., arXiv:2506.22408).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the HIP library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * Every function follows the paper's statement of the method:
 *   - covariance of a shadow  C' = Q^T C_b Q          (Supp. "Matrix
 *     Definitions", covariance matrix; main text eq. b_mat)
 *   - walker matrix X = selected rows of W M_phi       (Supp. "Matrix
 *     Definitions", W and M_phi; main text eq. b_mat)
 *   - B = X C' X^T and A(z) = C_0^(s) + z B            (eqs. a_mat, b_mat)
 *   - Pf(A(z_k)) at the interpolation nodes            (section "Classical
 *     shadows and the evaluation of overlaps", Pfaffian via Wimmer's
 *     Parlett-Reid elimination)
 *   - o = sum_k w_k Pf(A(z_k)); the node weights w_k carry the polynomial
 *     interpolation and the inverse-channel factors C(2N,2x)/C(N,x) together
 *     with the prefactor i^{eta/2}/2^{N-eta/2} of the estimator o_p; they are
 *     computed by the Python side of the oracle and passed in.
 *   - derivative of the Pfaffian, dPf = Pf/2 Tr(A^{-1} dA)  (eq. Pfaffian_der)
 *
 * Readings where the paper is ambiguous (all documented in the design notes):
 *   W is used where the paper prints W^*, and W^T where it prints W^dagger;
 *   the selected index set s holds the first Majorana of each occupied mode
 *   and both Majoranas of each empty mode, in increasing order; a general
 *   (non-orthonormal) walker is handled with G = [Phi | Phi_perp] and G^{-1}.
 *
 * Layouts: complex numbers are C99 double complex (two doubles, re then im).
 *   phi  [W][n][eta]   row-major (phi[w][p][j] = Phi_{pj})
 *   Q    [S][2n][2n]   row-major real
 *   bits [S]           bit j (0-based) is b_{j+1}
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define OR_OK 0
#define OR_ERR_ARG 1
#define OR_ERR_RANK 2
#define OR_ERR_SINGULAR 3
#define OR_ERR_NOMEM 4

/* ------------------------------------------------------------------------ */
/* Pfaffian of a complex skew-symmetric m x m matrix (row-major), by the
 * Parlett-Reid elimination with partial pivoting that the paper takes from
 * Wimmer.  At each even step k the entry of largest modulus in row k right
 * of the diagonal is moved to position (k, k+1) by a symmetric row/column
 * interchange (which flips the sign), the pivot A[k][k+1] multiplies the
 * result, and the Schur complement of the 2x2 pivot block replaces the
 * trailing matrix:  A_ij <- A_ij - tau_i v_j + v_i tau_j  with
 * tau = A[k][.]/A[k][k+1] and v = A[k+1][.].  A zero pivot row means Pf = 0.
 * Ties pick the smallest index.  The input is not modified.                */
int or_pfaffian(int m, const cplx *A_in, cplx *pf_out)
{
    if (m < 0 || !A_in || !pf_out) return OR_ERR_ARG;
    if (m == 0) { *pf_out = 1.0; return OR_OK; }
    if (m & 1) { *pf_out = 0.0; return OR_OK; }
    cplx *A = (cplx *)malloc(sizeof(cplx) * (size_t)m * (size_t)m);
    cplx *tau = (cplx *)malloc(sizeof(cplx) * (size_t)m);
    cplx *v = (cplx *)malloc(sizeof(cplx) * (size_t)m);
    if (!A || !tau || !v) { free(A); free(tau); free(v); return OR_ERR_NOMEM; }
    memcpy(A, A_in, sizeof(cplx) * (size_t)m * (size_t)m);
    cplx pf = 1.0;
    for (int k = 0; k < m - 1; k += 2) {
        int p = k + 1;
        double best = cabs(A[(size_t)k * m + k + 1]);
        for (int j = k + 2; j < m; ++j) {
            double a = cabs(A[(size_t)k * m + j]);
            if (a > best) { best = a; p = j; }
        }
        if (best == 0.0) { pf = 0.0; break; }
        if (p != k + 1) {
            for (int j = 0; j < m; ++j) {               /* swap rows k+1, p */
                cplx t = A[(size_t)(k + 1) * m + j];
                A[(size_t)(k + 1) * m + j] = A[(size_t)p * m + j];
                A[(size_t)p * m + j] = t;
            }
            for (int i = 0; i < m; ++i) {               /* swap cols k+1, p */
                cplx t = A[(size_t)i * m + k + 1];
                A[(size_t)i * m + k + 1] = A[(size_t)i * m + p];
                A[(size_t)i * m + p] = t;
            }
            pf = -pf;
        }
        cplx a = A[(size_t)k * m + k + 1];
        pf *= a;
        for (int i = k + 2; i < m; ++i) {
            tau[i] = A[(size_t)k * m + i] / a;
            v[i] = A[(size_t)(k + 1) * m + i];
        }
        for (int i = k + 2; i < m; ++i)
            for (int j = k + 2; j < m; ++j)
                A[(size_t)i * m + j] += v[i] * tau[j] - tau[i] * v[j];
    }
    *pf_out = pf;
    free(A); free(tau); free(v);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Covariance of one shadow, C' = Q^T C_b Q, with
 * C_b = (+)_j [[0, (-1)^{b_j}], [-(-1)^{b_j}, 0]]  (Supp. covariance matrix;
 * the product Q_p^T C_b Q_p of eq. b_mat).                                  */
void or_covariance(int n, const double *Q, uint64_t bits, double *Cp)
{
    int d = 2 * n;
    double *Cb = (double *)calloc((size_t)d * d, sizeof(double));
    double *T = (double *)calloc((size_t)d * d, sizeof(double));
    for (int j = 0; j < n; ++j) {
        double beta = ((bits >> j) & 1u) ? -1.0 : 1.0;
        Cb[(size_t)(2 * j) * d + 2 * j + 1] = beta;
        Cb[(size_t)(2 * j + 1) * d + 2 * j] = -beta;
    }
    for (int a = 0; a < d; ++a)                 /* T = C_b Q */
        for (int c = 0; c < d; ++c) {
            double s = 0.0;
            for (int b = 0; b < d; ++b) s += Cb[(size_t)a * d + b] * Q[(size_t)b * d + c];
            T[(size_t)a * d + c] = s;
        }
    for (int a = 0; a < d; ++a)                 /* C' = Q^T T */
        for (int c = 0; c < d; ++c) {
            double s = 0.0;
            for (int b = 0; b < d; ++b) s += Q[(size_t)b * d + a] * T[(size_t)b * d + c];
            Cp[(size_t)a * d + c] = s;
        }
    free(Cb); free(T);
}

/* ------------------------------------------------------------------------ */
/* Orthonormal basis of the orthogonal complement of col(Phi), by Householder
 * QR: Phi = H_0 ... H_{eta-1} [R; 0], complement = H_0 ... H_{eta-1} e_{eta+u}.
 * Returns OR_ERR_RANK if a diagonal entry of R is negligible.               */
int or_complement(int n, int eta, const cplx *phi, cplx *perp)
{
    cplx *R = (cplx *)malloc(sizeof(cplx) * (size_t)n * eta);
    cplx *V = (cplx *)calloc((size_t)n * eta, sizeof(cplx));   /* reflectors */
    double *beta = (double *)calloc((size_t)eta, sizeof(double));
    memcpy(R, phi, sizeof(cplx) * (size_t)n * eta);
    double fro = 0.0;
    for (int i = 0; i < n * eta; ++i) fro += creal(phi[i] * conj(phi[i]));
    fro = sqrt(fro);
    int status = OR_OK;
    for (int j = 0; j < eta; ++j) {
        double nx = 0.0;
        for (int i = j; i < n; ++i) nx += creal(R[(size_t)i * eta + j] * conj(R[(size_t)i * eta + j]));
        nx = sqrt(nx);
        if (!(nx > 1e-13 * fro)) { status = OR_ERR_RANK; break; }
        cplx x0 = R[(size_t)j * eta + j];
        cplx ph = (cabs(x0) > 0.0) ? x0 / cabs(x0) : 1.0;
        /* v = x + ph*|x| e_0 ; H = I - beta v v^H, beta = 2/(v^H v) */
        for (int i = j; i < n; ++i) V[(size_t)i * eta + j] = R[(size_t)i * eta + j];
        V[(size_t)j * eta + j] += ph * nx;
        double vv = 0.0;
        for (int i = j; i < n; ++i) vv += creal(V[(size_t)i * eta + j] * conj(V[(size_t)i * eta + j]));
        beta[j] = 2.0 / vv;
        for (int c = j; c < eta; ++c) {             /* R <- H R */
            cplx s = 0.0;
            for (int i = j; i < n; ++i) s += conj(V[(size_t)i * eta + j]) * R[(size_t)i * eta + c];
            s *= beta[j];
            for (int i = j; i < n; ++i) R[(size_t)i * eta + c] -= s * V[(size_t)i * eta + j];
        }
    }
    if (status == OR_OK) {
        int nc = n - eta;
        for (int u = 0; u < nc; ++u) {
            cplx *col = (cplx *)calloc((size_t)n, sizeof(cplx));
            col[eta + u] = 1.0;
            for (int j = eta - 1; j >= 0; --j) {    /* col <- H_j col */
                cplx s = 0.0;
                for (int i = j; i < n; ++i) s += conj(V[(size_t)i * eta + j]) * col[i];
                s *= beta[j];
                for (int i = j; i < n; ++i) col[i] -= s * V[(size_t)i * eta + j];
            }
            for (int i = 0; i < n; ++i) perp[(size_t)i * nc + u] = col[i];
            free(col);
        }
    }
    free(R); free(V); free(beta);
    return status;
}

/* Plain complex inverse by Gauss-Jordan elimination with partial pivoting. */
static int cinv(int m, const cplx *A_in, cplx *Ainv)
{
    cplx *A = (cplx *)malloc(sizeof(cplx) * (size_t)m * m);
    memcpy(A, A_in, sizeof(cplx) * (size_t)m * m);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) Ainv[(size_t)i * m + j] = (i == j) ? 1.0 : 0.0;
    for (int c = 0; c < m; ++c) {
        int p = c;
        double best = cabs(A[(size_t)c * m + c]);
        for (int r = c + 1; r < m; ++r)
            if (cabs(A[(size_t)r * m + c]) > best) { best = cabs(A[(size_t)r * m + c]); p = r; }
        if (best == 0.0) { free(A); return OR_ERR_SINGULAR; }
        if (p != c)
            for (int j = 0; j < m; ++j) {
                cplx t = A[(size_t)c * m + j]; A[(size_t)c * m + j] = A[(size_t)p * m + j]; A[(size_t)p * m + j] = t;
                t = Ainv[(size_t)c * m + j]; Ainv[(size_t)c * m + j] = Ainv[(size_t)p * m + j]; Ainv[(size_t)p * m + j] = t;
            }
        cplx piv = A[(size_t)c * m + c];
        for (int j = 0; j < m; ++j) { A[(size_t)c * m + j] /= piv; Ainv[(size_t)c * m + j] /= piv; }
        for (int r = 0; r < m; ++r) {
            if (r == c) continue;
            cplx f = A[(size_t)r * m + c];
            if (f == 0.0) continue;
            for (int j = 0; j < m; ++j) {
                A[(size_t)r * m + j] -= f * A[(size_t)c * m + j];
                Ainv[(size_t)r * m + j] -= f * Ainv[(size_t)c * m + j];
            }
        }
    }
    free(A);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Walker matrix X (m x 2n, m = 2n - eta): the selected rows of W M_phi
 * (Supp. "Matrix Definitions"), with G = [Phi | Phi_perp] standing for the
 * orbital rotation (V = G^{-1}) and the 0-based Majorana index 2p for
 * gamma_{2p+1} = a_p + a_p^dag, 2p+1 for gamma_{2p+2} = -i(a_p - a_p^dag).
 * Occupied mode j (row j):        X[j,2p] = G_pj/sqrt2, X[j,2p+1] = -i G_pj/sqrt2
 * Empty mode J = eta+u (rows r0 = eta+2u, r0+1), with g = (G^{-1})_{Jp}:
 *   X[r0,2p]   = (g + G_pJ)/2,      X[r0,2p+1]   = i (g - G_pJ)/2
 *   X[r0+1,2p] = -i (g - G_pJ)/2,   X[r0+1,2p+1] = (g + G_pJ)/2
 * For a unitary G these are the rows of the realified rotation.             */
int or_xmatrix(int n, int eta, const cplx *phi, const cplx *perp, cplx *X, cplx *Ginv_out)
{
    int nc = n - eta, d = 2 * n;
    cplx *G = (cplx *)malloc(sizeof(cplx) * (size_t)n * n);
    cplx *Gi = (cplx *)malloc(sizeof(cplx) * (size_t)n * n);
    for (int p = 0; p < n; ++p) {
        for (int j = 0; j < eta; ++j) G[(size_t)p * n + j] = phi[(size_t)p * eta + j];
        for (int u = 0; u < nc; ++u) G[(size_t)p * n + eta + u] = perp[(size_t)p * nc + u];
    }
    int st = cinv(n, G, Gi);
    if (st != OR_OK) { free(G); free(Gi); return OR_ERR_RANK; }
    const double rs2 = 1.0 / sqrt(2.0);
    for (int j = 0; j < eta; ++j)
        for (int p = 0; p < n; ++p) {
            X[(size_t)j * d + 2 * p] = G[(size_t)p * n + j] * rs2;
            X[(size_t)j * d + 2 * p + 1] = -I * G[(size_t)p * n + j] * rs2;
        }
    for (int u = 0; u < nc; ++u) {
        int J = eta + u, r0 = eta + 2 * u;
        for (int p = 0; p < n; ++p) {
            cplx g = Gi[(size_t)J * n + p], h = G[(size_t)p * n + J];
            X[(size_t)r0 * d + 2 * p] = (g + h) / 2;
            X[(size_t)r0 * d + 2 * p + 1] = I * (g - h) / 2;
            X[(size_t)(r0 + 1) * d + 2 * p] = -I * (g - h) / 2;
            X[(size_t)(r0 + 1) * d + 2 * p + 1] = (g + h) / 2;
        }
    }
    if (Ginv_out) memcpy(Ginv_out, Gi, sizeof(cplx) * (size_t)n * n);
    free(G); free(Gi);
    return OR_OK;
}

/* B = X C' X^T (eq. b_mat with the selection applied). */
static void bmatrix(int m, int d, const cplx *X, const double *Cp, cplx *B)
{
    cplx *T = (cplx *)malloc(sizeof(cplx) * (size_t)m * d);
    for (int i = 0; i < m; ++i)
        for (int nu = 0; nu < d; ++nu) {
            cplx s = 0.0;
            for (int mu = 0; mu < d; ++mu) s += X[(size_t)i * d + mu] * Cp[(size_t)mu * d + nu];
            T[(size_t)i * d + nu] = s;
        }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            cplx s = 0.0;
            for (int nu = 0; nu < d; ++nu) s += T[(size_t)i * d + nu] * X[(size_t)j * d + nu];
            B[(size_t)i * m + j] = s;
        }
    free(T);
}

/* A(z) = C_0^(s) + z B (eq. a_mat): the selected vacuum covariance is zero on
 * the occupied rows/columns and [[0,1],[-1,0]] on each empty-mode pair.      */
static void amatrix(int n, int eta, const cplx *B, cplx z, cplx *A)
{
    int m = 2 * n - eta;
    for (int i = 0; i < m * m; ++i) A[i] = z * B[i];
    for (int u = 0; u < n - eta; ++u) {
        int r0 = eta + 2 * u;
        A[(size_t)r0 * m + r0 + 1] += 1.0;
        A[(size_t)(r0 + 1) * m + r0] -= 1.0;
    }
}

/* One walker x shadow estimate o = sum_k w_k Pf(A(z_k)), for a given
 * complement Phi_perp.  node_out (K values) is optional.                   */
int or_pair_perp(int n, int eta, int K, const cplx *nodes, const cplx *weights,
                 const cplx *phi, const cplx *perp, const double *Q, uint64_t bits,
                 cplx *o_out, cplx *node_out)
{
    int d = 2 * n, m = 2 * n - eta;
    cplx *X = (cplx *)malloc(sizeof(cplx) * (size_t)m * d);
    double *Cp = (double *)malloc(sizeof(double) * (size_t)d * d);
    cplx *B = (cplx *)malloc(sizeof(cplx) * (size_t)m * m);
    cplx *A = (cplx *)malloc(sizeof(cplx) * (size_t)m * m);
    int st = or_xmatrix(n, eta, phi, perp, X, NULL);
    if (st == OR_OK) {
        or_covariance(n, Q, bits, Cp);
        bmatrix(m, d, X, Cp, B);
        cplx o = 0.0;
        for (int k = 0; k < K; ++k) {
            cplx pk;
            amatrix(n, eta, B, nodes[k], A);
            or_pfaffian(m, A, &pk);
            if (node_out) node_out[k] = pk;
            o += weights[k] * pk;
        }
        *o_out = o;
    }
    free(X); free(Cp); free(B); free(A);
    return st;
}

int or_pair(int n, int eta, int K, const cplx *nodes, const cplx *weights,
            const cplx *phi, const double *Q, uint64_t bits, cplx *o_out, cplx *node_out)
{
    cplx *perp = (cplx *)malloc(sizeof(cplx) * (size_t)n * (size_t)(n - eta > 0 ? n - eta : 1));
    int st = or_complement(n, eta, phi, perp);
    if (st == OR_OK) st = or_pair_perp(n, eta, K, nodes, weights, phi, perp, Q, bits, o_out, node_out);
    free(perp);
    return st;
}

/* Estimates for a list of (walker, shadow) pairs, or for all W x S pairs in
 * walker-major order when pw/ps are NULL.  OpenMP over pairs; nthreads <= 0
 * keeps the runtime default.  status[i] gets the per-pair return code.      */
int or_overlap_pairs(int n, int eta, int K, const cplx *nodes, const cplx *weights,
                     const cplx *phi, long W, const double *Q, const uint64_t *bits, long S,
                     const long *pw, const long *ps, long npairs,
                     cplx *out, cplx *node_out, int *status, int nthreads)
{
    if (n < 1 || eta < 1 || eta > n || (eta & 1) || K < 1) return OR_ERR_ARG;
    long total = (pw && ps) ? npairs : W * S;
    int d = 2 * n;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (long i = 0; i < total; ++i) {
        long w = (pw && ps) ? pw[i] : i / S;
        long s = (pw && ps) ? ps[i] : i % S;
        int st = or_pair(n, eta, K, nodes, weights, phi + (size_t)w * n * eta,
                         Q + (size_t)s * d * d, bits[s], &out[i],
                         node_out ? node_out + (size_t)i * K : NULL);
        if (status) status[i] = st;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Holomorphic derivative d o / d Phi (n x eta) of one pair estimate, from the
 * Pfaffian derivative dPf(A) = Pf(A)/2 Tr(A^{-1} dA) (eq. Pfaffian_der) and
 * the chain rule through A_k = C_0^(s) + z_k B, B = X C' X^T and X(Phi)
 * (Phi_perp held fixed, G^{-1} differentiated as -G^{-1} dG G^{-1}).
 * With F = C' X^T Abar, Abar = sum_k w_k Pf(A_k) z_k A_k^{-1}, one has
 * do = sum_{r,mu} dX_{r,mu} F_{mu,r}.  Returns OR_ERR_SINGULAR if some
 * node matrix is singular.                                                  */
int or_pair_grad(int n, int eta, int K, const cplx *nodes, const cplx *weights,
                 const cplx *phi, const double *Q, uint64_t bits,
                 cplx *o_out, cplx *dodphi)
{
    int d = 2 * n, m = 2 * n - eta, nc = n - eta;
    cplx *perp = (cplx *)malloc(sizeof(cplx) * (size_t)n * (size_t)(nc > 0 ? nc : 1));
    cplx *X = (cplx *)malloc(sizeof(cplx) * (size_t)m * d);
    cplx *Gi = (cplx *)malloc(sizeof(cplx) * (size_t)n * n);
    double *Cp = (double *)malloc(sizeof(double) * (size_t)d * d);
    cplx *B = (cplx *)malloc(sizeof(cplx) * (size_t)m * m);
    cplx *A = (cplx *)malloc(sizeof(cplx) * (size_t)m * m);
    cplx *Ai = (cplx *)malloc(sizeof(cplx) * (size_t)m * m);
    cplx *Ab = (cplx *)calloc((size_t)m * m, sizeof(cplx));
    cplx *T = (cplx *)malloc(sizeof(cplx) * (size_t)d * m);
    cplx *F = (cplx *)malloc(sizeof(cplx) * (size_t)d * m);
    int st = or_complement(n, eta, phi, perp);
    if (st == OR_OK) st = or_xmatrix(n, eta, phi, perp, X, Gi);
    if (st == OR_OK) {
        or_covariance(n, Q, bits, Cp);
        bmatrix(m, d, X, Cp, B);
        cplx o = 0.0;
        for (int k = 0; k < K && st == OR_OK; ++k) {
            cplx pk;
            amatrix(n, eta, B, nodes[k], A);
            or_pfaffian(m, A, &pk);
            o += weights[k] * pk;
            if (cinv(m, A, Ai) != OR_OK) { st = OR_ERR_SINGULAR; break; }
            cplx f = weights[k] * pk * nodes[k];
            for (int i = 0; i < m * m; ++i) Ab[i] += f * Ai[i];
        }
        *o_out = o;
    }
    if (st == OR_OK) {
        /* T = X^T Abar (d x m), F = C' T (d x m) */
        for (int mu = 0; mu < d; ++mu)
            for (int r = 0; r < m; ++r) {
                cplx s = 0.0;
                for (int i = 0; i < m; ++i) s += X[(size_t)i * d + mu] * Ab[(size_t)i * m + r];
                T[(size_t)mu * m + r] = s;
            }
        for (int mu = 0; mu < d; ++mu)
            for (int r = 0; r < m; ++r) {
                cplx s = 0.0;
                for (int nu = 0; nu < d; ++nu) s += Cp[(size_t)mu * d + nu] * T[(size_t)nu * m + r];
                F[(size_t)mu * m + r] = s;
            }
        /* pseudo-inverse rows Phi^+_{jq} = (G^{-1})_{jq}, j < eta */
        const double rs2 = 1.0 / sqrt(2.0);
        for (int p = 0; p < n; ++p)
            for (int j = 0; j < eta; ++j) {
                /* occupied row j: dX[j,2p] = 1/sqrt2, dX[j,2p+1] = -i/sqrt2 */
                cplx g = rs2 * (F[(size_t)(2 * p) * m + j] - I * F[(size_t)(2 * p + 1) * m + j]);
                /* empty rows: d(G^{-1})_{Jq} = -(G^{-1})_{Jp} (G^{-1})_{jq} */
                for (int u = 0; u < nc; ++u) {
                    int J = eta + u, r0 = eta + 2 * u;
                    cplx a = Gi[(size_t)J * n + p];
                    cplx h = 0.0;
                    for (int q = 0; q < n; ++q) {
                        cplx dg = -a * Gi[(size_t)j * n + q];
                        /* dX[r0,2q] = dg/2, dX[r0,2q+1] = i dg/2,
                           dX[r0+1,2q] = -i dg/2, dX[r0+1,2q+1] = dg/2 */
                        h += dg * 0.5 * (F[(size_t)(2 * q) * m + r0] + I * F[(size_t)(2 * q + 1) * m + r0]
                                         - I * F[(size_t)(2 * q) * m + r0 + 1] + F[(size_t)(2 * q + 1) * m + r0 + 1]);
                    }
                    g += h;
                }
                dodphi[(size_t)p * eta + j] = g;
            }
    }
    free(perp); free(X); free(Gi); free(Cp); free(B); free(A); free(Ai); free(Ab); free(T); free(F);
    return st;
}

/* Per-walker sums over shadows: osum[w] = sum_s o_ws and
 * gsum[w] = sum_s d o_ws / d Phi_w (n x eta).  OpenMP over walkers.        */
int or_grad_walkers(int n, int eta, int K, const cplx *nodes, const cplx *weights,
                    const cplx *phi, long W, const double *Q, const uint64_t *bits, long S,
                    cplx *osum, cplx *gsum, int *status, int nthreads)
{
    if (n < 1 || eta < 1 || eta > n || (eta & 1) || K < 1) return OR_ERR_ARG;
    int d = 2 * n;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (long w = 0; w < W; ++w) {
        cplx *g = (cplx *)malloc(sizeof(cplx) * (size_t)n * eta);
        cplx os = 0.0;
        for (int i = 0; i < n * eta; ++i) gsum[(size_t)w * n * eta + i] = 0.0;
        int st = OR_OK;
        for (long s = 0; s < S && st == OR_OK; ++s) {
            cplx o;
            st = or_pair_grad(n, eta, K, nodes, weights, phi + (size_t)w * n * eta,
                              Q + (size_t)s * d * d, bits[s], &o, g);
            if (st != OR_OK) break;
            os += o;
            for (int i = 0; i < n * eta; ++i) gsum[(size_t)w * n * eta + i] += g[i];
        }
        osum[w] = os;
        if (status) status[w] = st;
        free(g);
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Local energy ("Force bias and local energy": eqs. local_energy,
 * ham_cholesky_decom, energy_tb_diff, Pfaffian_der, Pfaffian_2nd_der).
 *
 * H = sum_pq t_pq a_p^dag a_q + 1/2 sum_g Lhat_g^2 with
 * Lhat_g = sum_pq L^g_pq a_p^dag a_q (v_0 = the one-body part t and
 * v_g = i Lhat_g in H = v_0 - 1/2 sum_g v_g^2).  A one-body operator Lhat
 * moves the walker to e^{lambda Lhat}|phi>, a determinant whose defining
 * operators are e^{lambda Lhat} b e^{-lambda Lhat}; on the Majorana
 * coefficient rows of X this is X -> X e^{lambda K} with
 * [Lhat, gamma_rho] = sum_sigma K[rho][sigma] gamma_sigma.  From
 * [a_p^dag a_q, a_r^dag] = delta_qr a_p^dag and [a_p^dag a_q, a_r] =
 * -delta_pr a_q, with gamma_2r = a_r + a_r^dag and
 * gamma_2r+1 = -i (a_r - a_r^dag) (0-based):
 *   K[2r][2q]   = (L_qr - L_rq)/2,   K[2r][2q+1]   = -i (L_rq + L_qr)/2,
 *   K[2r+1][2q] = i (L_rq + L_qr)/2, K[2r+1][2q+1] = (L_qr - L_rq)/2.       */
void or_kmatrix(int n, const cplx *L, cplx *Km)
{
    int d = 2 * n;
    for (int i = 0; i < d * d; ++i) Km[i] = 0.0;
    for (int r = 0; r < n; ++r)
        for (int q = 0; q < n; ++q) {
            cplx s = (L[(size_t)q * n + r] - L[(size_t)r * n + q]) / 2;
            cplx t = (L[(size_t)r * n + q] + L[(size_t)q * n + r]) / 2;
            Km[(size_t)(2 * r) * d + 2 * q] = s;
            Km[(size_t)(2 * r) * d + 2 * q + 1] = -I * t;
            Km[(size_t)(2 * r + 1) * d + 2 * q] = I * t;
            Km[(size_t)(2 * r + 1) * d + 2 * q + 1] = s;
        }
}

/* C = A B for complex d x d matrices (B given as complex) */
static void cmul_dd(int d, const cplx *A, const cplx *B, cplx *C)
{
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            cplx s = 0.0;
            for (int k = 0; k < d; ++k) s += A[(size_t)i * d + k] * B[(size_t)k * d + j];
            C[(size_t)i * d + j] = s;
        }
}

/* Bd = X D X^T (m x m) for a complex d x d matrix D */
static void sandwich(int m, int d, const cplx *X, const cplx *D, cplx *Bd)
{
    cplx *T = (cplx *)malloc(sizeof(cplx) * (size_t)m * d);
    for (int i = 0; i < m; ++i)
        for (int nu = 0; nu < d; ++nu) {
            cplx s = 0.0;
            for (int mu = 0; mu < d; ++mu) s += X[(size_t)i * d + mu] * D[(size_t)mu * d + nu];
            T[(size_t)i * d + nu] = s;
        }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            cplx s = 0.0;
            for (int nu = 0; nu < d; ++nu) s += T[(size_t)i * d + nu] * X[(size_t)j * d + nu];
            Bd[(size_t)i * m + j] = s;
        }
    free(T);
}

/* dB/dlambda and d^2B/dlambda^2 at lambda = 0 for B(lambda) =
 * X e^{lambda K} C' e^{lambda K^T} X^T:
 *   B1 = X (K C' + C' K^T) X^T,  B2 = X (K^2 C' + 2 K C' K^T + C' (K^T)^2) X^T. */
static void bderivs(int m, int d, const cplx *X, const double *Cp, const cplx *Km, cplx *B1, cplx *B2)
{
    size_t dd = (size_t)d * d;
    cplx *C = (cplx *)malloc(sizeof(cplx) * dd);
    cplx *Kt = (cplx *)malloc(sizeof(cplx) * dd);
    cplx *KC = (cplx *)malloc(sizeof(cplx) * dd);
    cplx *CKt = (cplx *)malloc(sizeof(cplx) * dd);
    cplx *KKC = (cplx *)malloc(sizeof(cplx) * dd);
    cplx *KCKt = (cplx *)malloc(sizeof(cplx) * dd);
    cplx *CKtKt = (cplx *)malloc(sizeof(cplx) * dd);
    cplx *D = (cplx *)malloc(sizeof(cplx) * dd);
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            C[(size_t)i * d + j] = Cp[(size_t)i * d + j];
            Kt[(size_t)i * d + j] = Km[(size_t)j * d + i];
        }
    cmul_dd(d, Km, C, KC);
    cmul_dd(d, C, Kt, CKt);
    cmul_dd(d, Km, KC, KKC);
    cmul_dd(d, KC, Kt, KCKt);
    cmul_dd(d, CKt, Kt, CKtKt);
    for (size_t i = 0; i < dd; ++i) D[i] = KC[i] + CKt[i];
    sandwich(m, d, X, D, B1);
    for (size_t i = 0; i < dd; ++i) D[i] = KKC[i] + 2.0 * KCKt[i] + CKtKt[i];
    sandwich(m, d, X, D, B2);
    free(C); free(Kt); free(KC); free(CKt); free(KKC); free(KCKt); free(CKtKt); free(D);
}

/* One pair: o = sum_k w_k Pf(A_k) and the numerator
 *   e = sum_k w_k [ dPf_k[t] + 1/2 sum_g d2Pf_k[L_g] ],
 *   dPf  = Pf/2 tr(A^{-1} A'),
 *   d2Pf = Pf/2 { tr(A^{-1} A'') - tr(A^{-1} A' A^{-1} A') + 1/2 tr(A^{-1} A')^2 },
 * A' = z B1, A'' = z B2 (the two lambdas of eq. Pfaffian_2nd_der move the
 * walker along the same operator, so dA/dlambda_1 = dA/dlambda_2 = A' and
 * d^2A/dlambda_1 dlambda_2 = A'').  Kt is the d x d K of t, Kg the ng K's
 * of the L_g.  OR_ERR_SINGULAR if a node matrix is singular.               */
int or_pair_energy(int n, int eta, int K, const cplx *nodes, const cplx *weights,
                   const cplx *phi, const double *Q, uint64_t bits,
                   const cplx *Kt, int ng, const cplx *Kg, cplx *o_out, cplx *e_out)
{
    int d = 2 * n, m = 2 * n - eta, nc = n - eta, nop = ng + 1;
    size_t mm = (size_t)m * m;
    cplx *perp = (cplx *)malloc(sizeof(cplx) * (size_t)n * (size_t)(nc > 0 ? nc : 1));
    cplx *X = (cplx *)malloc(sizeof(cplx) * (size_t)m * d);
    double *Cp = (double *)malloc(sizeof(double) * (size_t)d * d);
    cplx *B = (cplx *)malloc(sizeof(cplx) * mm);
    cplx *B1 = (cplx *)malloc(sizeof(cplx) * mm * nop);
    cplx *B2 = (cplx *)malloc(sizeof(cplx) * mm * nop);
    cplx *A = (cplx *)malloc(sizeof(cplx) * mm);
    cplx *Ai = (cplx *)malloc(sizeof(cplx) * mm);
    cplx *P = (cplx *)malloc(sizeof(cplx) * mm);
    int st = or_complement(n, eta, phi, perp);
    if (st == OR_OK) st = or_xmatrix(n, eta, phi, perp, X, NULL);
    if (st == OR_OK) {
        or_covariance(n, Q, bits, Cp);
        bmatrix(m, d, X, Cp, B);
        for (int op = 0; op < nop; ++op)
            bderivs(m, d, X, Cp, op == 0 ? Kt : Kg + (size_t)(op - 1) * d * d, B1 + op * mm, B2 + op * mm);
        cplx o = 0.0, e = 0.0;
        for (int k = 0; k < K && st == OR_OK; ++k) {
            cplx pk, z = nodes[k];
            amatrix(n, eta, B, z, A);
            or_pfaffian(m, A, &pk);
            o += weights[k] * pk;
            if (cinv(m, A, Ai) != OR_OK) { st = OR_ERR_SINGULAR; break; }
            for (int op = 0; op < nop; ++op) {
                const cplx *b1 = B1 + op * mm, *b2 = B2 + op * mm;
                cplx tr1 = 0.0, tr2 = 0.0, trq = 0.0;
                for (int i = 0; i < m; ++i)
                    for (int j = 0; j < m; ++j) {
                        tr1 += Ai[(size_t)i * m + j] * z * b1[(size_t)j * m + i];
                        tr2 += Ai[(size_t)i * m + j] * z * b2[(size_t)j * m + i];
                    }
                if (op == 0) {
                    e += weights[k] * pk / 2 * tr1;
                    continue;
                }
                for (int i = 0; i < m; ++i)          /* P = A^{-1} A' */
                    for (int j = 0; j < m; ++j) {
                        cplx s = 0.0;
                        for (int l = 0; l < m; ++l) s += Ai[(size_t)i * m + l] * z * b1[(size_t)l * m + j];
                        P[(size_t)i * m + j] = s;
                    }
                for (int i = 0; i < m; ++i)
                    for (int j = 0; j < m; ++j) trq += P[(size_t)i * m + j] * P[(size_t)j * m + i];
                e += 0.5 * weights[k] * pk / 2 * (tr2 - trq + 0.5 * tr1 * tr1);
            }
        }
        *o_out = o;
        *e_out = e;
    }
    free(perp); free(X); free(Cp); free(B); free(B1); free(B2); free(A); free(Ai); free(P);
    return st;
}

/* Pairs (list pw/ps, or all W x S walker-major) of o_ws and e_ws for the
 * Hamiltonian (t [n][n] complex, L [n*n][ng] real with L[p n + q][g] =
 * L^g_pq).  OpenMP over pairs.                                              */
int or_energy_pairs(int n, int eta, int K, const cplx *nodes, const cplx *weights,
                    const cplx *phi, long W, const double *Q, const uint64_t *bits, long S,
                    const long *pw, const long *ps, long npairs,
                    const cplx *t, const double *L, int ng,
                    cplx *o_out, cplx *e_out, int *status, int nthreads)
{
    if (n < 1 || eta < 1 || eta > n || (eta & 1) || K < 1 || ng < 0) return OR_ERR_ARG;
    int d = 2 * n;
    size_t dd = (size_t)d * d;
    cplx *Kt = (cplx *)malloc(sizeof(cplx) * dd);
    cplx *Kg = (cplx *)malloc(sizeof(cplx) * dd * (size_t)(ng > 0 ? ng : 1));
    cplx *Lg = (cplx *)malloc(sizeof(cplx) * (size_t)n * n);
    or_kmatrix(n, t, Kt);
    for (int g = 0; g < ng; ++g) {
        for (int pq = 0; pq < n * n; ++pq) Lg[pq] = L[(size_t)pq * ng + g];
        or_kmatrix(n, Lg, Kg + (size_t)g * dd);
    }
    long total = (pw && ps) ? npairs : W * S;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (long i = 0; i < total; ++i) {
        long w = (pw && ps) ? pw[i] : i / S;
        long s = (pw && ps) ? ps[i] : i % S;
        int st = or_pair_energy(n, eta, K, nodes, weights, phi + (size_t)w * n * eta, Q + (size_t)s * dd,
                                bits[s], Kt, ng, Kg, &o_out[i], &e_out[i]);
        if (status) status[i] = st;
    }
    free(Kt); free(Kg); free(Lg);
    return OR_OK;
}
