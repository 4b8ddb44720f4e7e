// so_vce.h -- virtual correlation energy: full-space walker -> active-space
// walker and prefactor (section "Virtual correlation energy", eq.
// vce_overlap; Supp. "Virtual Correlation Energy Derivation").
//
// Spatial orbitals 0..N_c-1 are the frozen core, N_c..N_c+N_a-1 the active
// space, the rest virtual; the trial state has the core filled in each spin
// and the virtual orbitals empty, so only the core rows C (N_c x N_e) and the
// active rows A (N_a x N_e) of a spin's walker (N_e = N_c + n_spin columns)
// enter.  With a unitary V = [V_c, V'] whose first N_c columns span the row
// space of C (so C V' = 0), det [C; chi^dag A] det V = det(C V_c) det(chi^dag A V'),
// and A V' = Q R gives the spin's active walker Q.  The paper takes V from
// an SVD of C; here the reflections of an LQ factorisation of C serve:
//   C H_1 ... H_Nc = [L, 0],  V = H_1 ... H_Nc,  det V = (-1)^Nc,  det(C V_c) = prod L_kk,
// and A V' = Q R by Householder QR (det R = prod R_kk).  Any such V gives the
// same det(C V_c) det(R) / det(V), which equals the paper's
// det(Sigma_c) det(R) / (det(U_c^dag) det(V)).  Over both spins
//   <Psi_T|phi> = (-1)^(N_c n_alpha) prod_spin [det(L) det(R) / det(V)] <Psi_T,a|phi~_a>,
// the sign being the column order of the paper's block V (V_c^a, V_c^b,
// V_c^a', V_c^b') against spin-by-spin blocks.  phi~_a = diag(Q^a, Q^b) over
// the 2 N_a active modes (alpha orbitals first), alpha electrons first.
#pragma once
#include "so_common.h"

#define SO_VCE_NAMAX 12          // active spatial orbitals: n = 2 N_a <= 24 modes
#define SO_VCE_LDS_MAX 65536     // bytes of LDS one walker's matrices may take

struct VceDims {
    int nb, nc, na, nal, nbe;    // N_B, N_c, N_a, n_alpha, n_beta
};

// LDS layout of k_vce_prep, in complex entries: M [(N_c + N_a) x ld] with
// ld = N_c + max(n_alpha, n_beta), the row reflector u [ld], the column
// reflectors [ns_max][N_a] and the active walker of the spin [N_a][ns_max].
__host__ __device__ inline size_t vce_lds_entries(const VceDims &v) {
    const int nsm = v.nal > v.nbe ? v.nal : v.nbe;
    const int ld = v.nc + nsm;
    return (size_t)(v.nc + v.na) * ld + ld + 2 * (size_t)nsm * v.na;
}

__device__ __forceinline__ double vce_wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// One wave per walker; the two spins one after the other.
//   pha [W][N_B][N_c + n_alpha], phb [W][N_B][N_c + n_beta]  (row-major)
//   act [W][2 N_a][n_alpha + n_beta]                           (out)
//   pref [W]                                                   (out)
// A row or column whose norm is exactly zero (a rank-deficient core or
// projected active block) gives a zero prefactor and the identity reflection,
// so the active walker stays orthonormal and the full overlap is exactly 0;
// a non-finite input propagates to the outputs.
__global__ __launch_bounds__(64) void k_vce_prep(VceDims v, const double2 *__restrict__ pha,
                                                 const double2 *__restrict__ phb, double2 *__restrict__ act,
                                                 double2 *__restrict__ pref) {
    extern __shared__ double2 vsm[];
    __shared__ double qbeta[SO_VCE_NAMAX];
    const int t = threadIdx.x;
    const int64_t w = blockIdx.x;
    const int nsm = v.nal > v.nbe ? v.nal : v.nbe;
    const int ld = v.nc + nsm, rows = v.nc + v.na;
    const int eta = v.nal + v.nbe, n = 2 * v.na;
    double2 *M = vsm;
    double2 *u = M + (size_t)rows * ld;
    double2 *Ur = u + ld;
    double2 *Qm = Ur + (size_t)nsm * v.na;
    double2 ptot = c_make(((v.nc * v.nal) & 1) ? -1.0 : 1.0, 0.0);
    for (int sp = 0; sp < 2; ++sp) {
        const int ns = sp ? v.nbe : v.nal;
        const int ne = v.nc + ns;
        const double2 *src = (sp ? phb : pha) + w * (int64_t)v.nb * ne;
        for (int e = t; e < rows * ne; e += 64) {
            const int r = e / ne, c = e - r * ne;
            M[r * ld + c] = src[(size_t)r * ne + c];
        }
        __syncthreads();
        double2 det = c_make(1.0, 0.0);
        // LQ of the core rows: row k, columns k..ne-1, reflected onto L_kk e_1
        for (int k = 0; k < v.nc; ++k) {
            const int len = ne - k;
            double s = 0.0;
            for (int j = t; j < len; j += 64) s += c_abs2(M[k * ld + k + j]);
            s = vce_wave_sum(s);
            if (s == 0.0) {
                det = c_make(0.0, 0.0);
                continue;
            }
            // y = conj(x) as a column; H y = alpha e_1 with alpha = -e^{i arg y0} |y|,
            // u = y - alpha e_1, H = I - u u^H / (s + |y0| |y|); then x H = conj(alpha) e_1^T
            const double nrm = sqrt(s);
            const double2 y0 = c_conj(M[k * ld + k]);
            const double a0 = sqrt(c_abs2(y0));
            const double2 ph = a0 > 0.0 ? c_scale(y0, 1.0 / a0) : c_make(1.0, 0.0);
            const double2 alpha = c_scale(ph, -nrm);
            const double beta = 1.0 / (s + a0 * nrm);
            for (int j = t; j < len; j += 64) u[j] = j == 0 ? c_sub(y0, alpha) : c_conj(M[k * ld + k + j]);
            __syncthreads();
            for (int r = k + t; r < rows; r += 64) {
                double2 dot = c_make(0.0, 0.0);
                for (int j = 0; j < len; ++j) dot = c_fma(M[r * ld + k + j], u[j], dot);
                dot = c_scale(dot, beta);
                for (int j = 0; j < len; ++j) M[r * ld + k + j] = c_sub(M[r * ld + k + j], c_mul(dot, c_conj(u[j])));
            }
            __syncthreads();
            det = c_neg(c_mul(det, c_conj(alpha)));   // L_kk = conj(alpha); det H = -1 divides
        }
        // QR of A V' (rows N_c.., columns N_c..): column k reflected onto R_kk e_1
        double2 *Ap = M + (size_t)v.nc * ld + v.nc;
        for (int k = 0; k < ns; ++k) {
            const int len = v.na - k;
            double2 *uk = Ur + (size_t)k * v.na;
            double s = 0.0;
            for (int i = t; i < len; i += 64) s += c_abs2(Ap[(k + i) * ld + k]);
            s = vce_wave_sum(s);
            if (s == 0.0) {
                det = c_make(0.0, 0.0);
                if (t == 0) qbeta[k] = 0.0;
                __syncthreads();
                continue;
            }
            const double nrm = sqrt(s);
            const double2 y0 = Ap[k * ld + k];
            const double a0 = sqrt(c_abs2(y0));
            const double2 ph = a0 > 0.0 ? c_scale(y0, 1.0 / a0) : c_make(1.0, 0.0);
            const double2 alpha = c_scale(ph, -nrm);
            const double beta = 1.0 / (s + a0 * nrm);
            for (int i = t; i < len; i += 64) uk[i] = i == 0 ? c_sub(y0, alpha) : Ap[(k + i) * ld + k];
            if (t == 0) qbeta[k] = beta;
            __syncthreads();
            for (int c = k + t; c < ns; c += 64) {
                double2 dot = c_make(0.0, 0.0);
                for (int i = 0; i < len; ++i) dot = c_fma(c_conj(uk[i]), Ap[(k + i) * ld + c], dot);
                dot = c_scale(dot, beta);
                for (int i = 0; i < len; ++i) Ap[(k + i) * ld + c] = c_sub(Ap[(k + i) * ld + c], c_mul(uk[i], dot));
            }
            __syncthreads();
            det = c_mul(det, alpha);                   // R_kk = alpha
        }
        // Q = H'_1 ... H'_ns [I; 0], applied from the last reflection
        for (int e = t; e < v.na * ns; e += 64) {
            const int i = e / ns, c = e - i * ns;
            Qm[e] = c_make(i == c ? 1.0 : 0.0, 0.0);
        }
        __syncthreads();
        for (int k = ns - 1; k >= 0; --k) {
            const int len = v.na - k;
            const double2 *uk = Ur + (size_t)k * v.na;
            const double bk = qbeta[k];
            for (int c = t; c < ns; c += 64) {
                if (bk == 0.0) break;
                double2 dot = c_make(0.0, 0.0);
                for (int i = 0; i < len; ++i) dot = c_fma(c_conj(uk[i]), Qm[(k + i) * ns + c], dot);
                dot = c_scale(dot, bk);
                for (int i = 0; i < len; ++i) Qm[(k + i) * ns + c] = c_sub(Qm[(k + i) * ns + c], c_mul(uk[i], dot));
            }
            __syncthreads();
        }
        // this spin's rows of phi~_a: Q in its column block, zeros elsewhere
        double2 *dst = act + w * (int64_t)n * eta + (size_t)(sp ? v.na : 0) * eta;
        const int c0 = sp ? v.nal : 0;
        for (int e = t; e < v.na * eta; e += 64) {
            const int i = e / eta, c = e - i * eta, cc = c - c0;
            dst[e] = (cc >= 0 && cc < ns) ? Qm[i * ns + cc] : c_make(0.0, 0.0);
        }
        ptot = c_mul(ptot, det);
        __syncthreads();
    }
    if (t == 0) pref[w] = ptot;
}

// overlap[w] *= pref[w]; in log form overlap[w] += log pref[w], the phase
// brought back to (-pi, pi]
__global__ __launch_bounds__(256) void k_vce_scale(int64_t W, const double2 *__restrict__ pref,
                                                   double2 *__restrict__ overlap, int logout) {
    const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (w >= W) return;
    if (!logout) {
        overlap[w] = c_mul(pref[w], overlap[w]);
        return;
    }
    const double two_pi = 6.283185307179586;
    double2 v = c_add(c_log(pref[w]), overlap[w]);
    v.y -= two_pi * rint(v.y / two_pi);
    if (v.y <= -0.5 * two_pi) v.y += two_pi;
    overlap[w] = v;
}
