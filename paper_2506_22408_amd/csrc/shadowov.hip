// shadowov.hip -- MI355X (gfx950) kernels and C ABI for the matchgate-shadow
// overlap estimator of QC-AFQMC (Zhao et al., arXiv:2506.22408).
//
// Per walker x shadow pair the estimator forms the Majorana-basis matrix
// B = X C' X^T (eq. b_mat, X the selected rows of W M_phi, C' = Q^T C_b Q),
// takes Pf(A(z)) with A(z) = C_0^(s) + z B (eq. a_mat) at K interpolation
// nodes and combines the node values with weights that carry the
// interpolation, the inverse-channel factors C(2N,2x)/C(N,x) and the
// prefactor of o_p (section "Classical shadows and the evaluation of
// overlaps"); the shadow average S_w closes the path.
//
// Kernels, all on the caller's stream, per call:
//   k_walker_prep   X_w from Phi_w (so_prep.h)
//   k_shadow_prep   C'_s = Q_s^T C_b Q_s (so_prep.h)
//   when ne = n - eta is even and 2 <= ne <= 12:
//     k_pair        formation, elimination of K = O u U1 down to the pencil
//                   M0 + c M1 + c^2 M2, node Pfaffians, weighted sum (so_pair.h)
//   otherwise, per chunk of shadows:
//     k_form_mfma   B_ws on the matrix cores, then the node-independent
//                   elimination of the occupied indices: S_ws and Pf(B_OO)
//                   (so_form.h)
//     k_nodes       node Pfaffians Pf(s_k S + c_k J), weighted sum (so_nodes.h)
//   (shadow_overlap_batched: one k_pair_batch launch for all fused problems, so_batch.h)
//   k_fallback      full-size path for the rare pairs flagged above (so_fallback.h)
//   k_reduce        S_w = (1/S) sum_s o_ws, fixed order (deterministic)
// and for the derivative (shadow_overlap_grad), after the two prep kernels:
//   k_grad_pair     per (walker, shadow range): Abar per pair and the partial
//                   sums of F = C' X^T Abar and of o (so_grad.h)
//   k_grad_walker   per walker: sums, gather, D_w, G_w, S_w (so_grad.h)
#include "shadowov.h"

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "so_common.h"
#include "so_prep.h"
#include "so_form.h"
#include "so_nodes.h"
#include "so_fallback.h"
#include "so_pair.h"
#include "so_grad.h"
#include "so_force.h"
#include "so_batch.h"
#include "so_rdm.h"
#include "so_vce.h"
#include "so_energy.h"

// --------------------------------------------------------------------------
// k_reduce: S_w = (1/S) sum_s o_ws, fixed order: lane l sums s = l, l+64, ...
// then a fixed butterfly.  Sets SO_WSTAT_NONFINITE; rank-deficient walkers
// get NaN.  With logdet (the pairs are those of the orthonormal factor,
// k_walker_prep) S_w = det R times the mean, or log S_w = log det R + log of
// the mean with the log output; with scale_pairs the pair values are
// rescaled by det R in place (the caller asked for them).
// --------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_reduce(double2 *__restrict__ pairs, int64_t S,
                                               double2 *__restrict__ out, int32_t *__restrict__ wstat,
                                               int logout, const double2 *__restrict__ logdet, int scale_pairs) {
    const int w = blockIdx.x;
    const int lane = threadIdx.x;
    double2 *pw = pairs + (size_t)w * S;
    double2 f = c_make(1.0, 0.0);
    if (logdet) {
        const double2 ld = logdet[w];
        const double mg = exp(ld.x);
        f = c_make(mg * cos(ld.y), mg * sin(ld.y));
        if (wstat[w] & SO_WSTAT_RANK) f = c_make(NAN, NAN);   // no orthonormal factor: NaN pairs too
    }
    double ar = 0.0, ai = 0.0;
    for (int64_t s = lane; s < S; s += 64) {
        const double2 v = pw[s];
        ar += v.x;
        ai += v.y;
        if (scale_pairs) pw[s] = c_mul(f, v);
    }
    ar = grp_sum<64>(ar);
    ai = grp_sum<64>(ai);
    if (lane == 0) {
        const double inv = 1.0 / (double)S;
        double2 r = c_make(ar * inv, ai * inv);
        int32_t st = wstat[w];
        if (st & SO_WSTAT_RANK) r = c_make(NAN, NAN);
        if (!isfinite(r.x) || !isfinite(r.y)) st |= SO_WSTAT_NONFINITE;
        if (logout) {
            if (r.x == 0.0 && r.y == 0.0) st |= SO_WSTAT_ZERO;
            r = c_log(r);
            if (logdet) {
                const double2 ld = logdet[w];
                r = c_make(r.x + ld.x, remainder(r.y + ld.y, 2.0 * M_PI));
            }
        } else if (logdet) {
            r = c_mul(f, r);
            if (!isfinite(r.x) || !isfinite(r.y)) st |= SO_WSTAT_NONFINITE;
        }
        out[w] = r;
        wstat[w] = st;
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

bool params_ok(const so_params *p, int *K_out) {
    if (!p) return false;
    if (p->n < 2 || p->n > SO_NMAX_SUPPORTED) return false;
    if (p->eta < 2 || p->eta > p->n || (p->eta & 1)) return false;
    if (p->nodes != SO_NODES_UNIT && p->nodes != SO_NODES_CHEBYSHEV) return false;
    if (p->precision != SO_PREC_FP64 && p->precision != SO_PREC_MIXED) return false;
    if (p->flags & ~(SO_FLAG_PAPER_NORM | SO_FLAG_LOG_OUTPUT | SO_FLAG_BATCH_BY_LEVEL | SO_FLAG_SIGNED_PERM)) return false;
    const int ell = p->n - p->eta / 2;
    const int K = p->n_nodes ? p->n_nodes : p->n + 1;
    if (K < ell + 1 || K > SO_KMAX) return false;
    if (K_out) *K_out = K;
    return true;
}

// Estimator terms: Pf(A(z)) = sum_{x=0}^{l} c_x z^x with l = n - eta/2, and
// o = pref sum_x mu_x c_x with mu_x = C(2n,2x)/C(n,x) and
// pref = 2 i^{eta/2} / 2^{n - eta/2} (estimator o_p, times 2 unless
// SO_FLAG_PAPER_NORM).  mu_x is filled for x < nmu (zero beyond l).
void estimator_terms(const so_params *p, int nmu, long double *mu, cld *pref) {
    const int n = p->n, eta = p->eta, ell = n - eta / 2;
    for (int x = 0; x < nmu; ++x) {
        if (x > ell) { mu[x] = 0.0L; continue; }
        // C(2n,2x) and C(n,x) as exact integers (n <= 32: C(64,32) < 2^64)
        unsigned long long a = 1, b = 1;
        for (int t = 1; t <= 2 * x; ++t) a = a * (unsigned long long)(2 * n - 2 * x + t) / t;
        for (int t = 1; t <= x; ++t) b = b * (unsigned long long)(n - x + t) / t;
        mu[x] = (long double)a / (long double)b;
    }
    const long double mag = ldexpl((p->flags & SO_FLAG_PAPER_NORM) ? 1.0L : 2.0L, -(n - eta / 2));
    switch ((eta / 2) % 4) {
        case 0: *pref = {mag, 0.0L}; break;
        case 1: *pref = {0.0L, mag}; break;
        case 2: *pref = {-mag, 0.0L}; break;
        default: *pref = {0.0L, -mag}; break;
    }
}

// Node weights: interpolation at the nodes gives o = sum_k w_k p_k,
// w = pref V^{-T} mu, V_{kx} = z_k^x.
void compute_weights(const so_params *p, int K, double2 *z, double2 *w) {
    const int n = p->n, eta = p->eta, ell = n - eta / 2;
    long double mu[SO_KMAX];
    cld pref;
    estimator_terms(p, K, mu, &pref);
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

// Node table.  With Q(c) = Pf(B + c J) = sum_x A_x c^x (degree ne = n - eta;
// B and J in the stored row order of so_prep.h), Pf(J + z B) = z^{m/2} Q(1/z),
// so the coefficient of z^y in Pf(A(z)) is A_{m/2-y} and
// o = pref psign sum_{x=0}^{ne} mu_{m/2-x} A_x whatever the node family.  Q at
// the nodes e_j = exp(2 pi i (j + 1/3)/(ne+1)) (the roots of unity turned by a
// third of a step) gives A_x = (1/(ne+1)) sum_j Q(e_j) e_j^{-x} (for
// 0 <= x, y <= ne, sum_j e_j^{x-y} vanishes unless x = y), hence
// o = sum_j v_j Q(e_j) with v_j = (pref psign/(ne+1)) sum_x mu_{m/2-x} e_j^{-x}.
// The turn keeps the nodes off +-1 and +-i, where Q of a signed-permutation
// shadow has exact roots (modes whose two Majoranas it maps onto one mode),
// so the node matrices the derivative inverts stay regular.  The reduced path takes
// Q(e_j) as Pf(B_KK) Pf(M(e_j)) (so_pair.h) or pfo Pf(S + e_j J) (so_nodes.h),
// the full-size path as Pf(B + e_j J) itself (so_fallback.h).  psign is the
// sign of the permutation from the paper's selected order to the stored one.
// Sign of the permutation from the paper's row order (occupied 0..eta-1,
// then eta+2u, eta+2u+1 for empty u) to the kernels' order (so_prep.h).
double row_order_sign(int n, int eta) {
    const int m = mvalue(n, eta), ne = n - eta;
    int perm[2 * SO_NMAX];
    for (int i = 0; i < eta; ++i) perm[i] = i;
    for (int u = 0; u < ne; ++u) { perm[eta + 2 * u] = eta + u; perm[eta + 2 * u + 1] = eta + 2 * ne - 1 - u; }
    int inv = 0;
    for (int i = 0; i < m; ++i)
        for (int j = i + 1; j < m; ++j) inv += perm[i] > perm[j];
    return (inv & 1) ? -1.0 : 1.0;
}

void build_nodetab(const so_params *p, int K, NodeTab *t) {
    const int n = p->n, eta = p->eta, m = mvalue(n, eta), ne = n - eta;
    const double psign = row_order_sign(n, eta);
    std::memset(t, 0, sizeof(*t));
    t->K = K;
    const long double two_pi = 6.283185307179586476925286766559005768L;
    long double mu[SO_KMAX];
    cld pref;
    estimator_terms(p, SO_KMAX, mu, &pref);
    // c_j = exp(2 pi i (3j + 1) / (3 Ke)): angles in units of 2 pi / (3 Ke), exact mod 3 Ke
    const int Ke = ne + 1, K3 = 3 * Ke;
    t->Ke = Ke;
    for (int j = 0; j < Ke; ++j) {
        long double sr = 0.0L, si = 0.0L;
        for (int x = 0; x <= ne; ++x) {
            const long double th = -two_pi * (long double)((long long)(3 * j + 1) * x % K3) / K3;   // c_j^{-x}
            sr += mu[m / 2 - x] * cosl(th);
            si += mu[m / 2 - x] * sinl(th);
        }
        sr *= psign / (long double)Ke;
        si *= psign / (long double)Ke;
        t->v[j] = make_double2((double)(pref.re * sr - pref.im * si), (double)(pref.re * si + pref.im * sr));
        const long double te = two_pi * (long double)(3 * j + 1) / K3;
        t->e[j] = make_double2((double)cosl(te), (double)sinl(te));
    }
}

constexpr size_t kSChunkBytes = (size_t)512 << 20;   // budget for one chunk of S matrices
constexpr int FB_GRID = 2048;                          // blocks of the fallback kernel
constexpr int kFormShadowsPerWave = 8;                 // shadows per formation wave
constexpr int kPairBatchesPerWave = 2;                 // node batches per fused wave
#ifndef SO_ROW_BATCHES_PER_WAVE
#define SO_ROW_BATCHES_PER_WAVE 8
#endif
constexpr int kRowBatchesPerWave = SO_ROW_BATCHES_PER_WAVE;   // the same for ne > 8 (single-pair batches)
constexpr int64_t kRdmBlocks = 1024;                    // blocks of the density-matrix reduction (1024 measured best of 512, 1024, 2048 at n = 16 and 24)

struct Layout {
    size_t off_X, off_C, off_S, off_P, off_pairs, off_stat, off_fbc, off_fbl, off_F, off_O, off_M, off_LD;
    size_t off_QF, off_RF;     // derivative path: the walkers' QR factors Phi = Qf R
    size_t off_X32, off_C32;   // single-precision formation operands (mixed precision)
    size_t total;
    int Sc;
    int64_t fb_cap;
    int Gy;   // shadow ranges per walker of the derivative kernel
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// the fused pair kernel covers an even ne = n - eta with 2 <= ne <= 12
// (node Pfaffians per lane up to ne = 8, per 16-lane row above)
bool fused_ok(int n, int eta) {
    const int ne = n - eta;
    return ne >= 2 && ne <= 12 && (ne % 2) == 0;
}

// shadow ranges per walker for k_grad_pair: enough waves to fill the chip
int grad_ranges(int64_t W, int64_t S) {
    int64_t gy = (8192 + W - 1) / W;
    if (gy > S) gy = S;
    if (gy < 1) gy = 1;
    return (int)gy;
}

bool grad_ok(int n, int eta) { return fused_ok(n, eta) && n - eta <= 8 && so_tiles(n) <= 2; }

Layout make_layout(int n, int eta, int64_t W, int64_t S, bool with_grad = false, bool mixed = false) {
    Layout L{};
    const int m = mvalue(n, eta), DP = 16 * so_tiles(n), M2 = m - eta;
    const size_t per_shadow = (size_t)W * ((size_t)M2 * M2 + 1) * sizeof(double2);
    int64_t Sc = (int64_t)(kSChunkBytes / per_shadow);
    if (Sc < 1) Sc = 1;
    if (Sc > S) Sc = S;
    if (fused_ok(n, eta)) Sc = 0;   // no Schur-complement chunks
    L.Sc = (int)Sc;
    int64_t cap = W * S / 256;
    if (cap < 4096) cap = 4096;
    if (cap > W * S) cap = W * S;
    L.fb_cap = cap;
    size_t o = 0;
    L.off_X = o; o = align_up(o + (size_t)W * DP * DP * sizeof(double));
    L.off_C = o; o = align_up(o + (size_t)S * DP * DP * sizeof(double));
    L.off_M = o; o = align_up(o + (size_t)S * DP * sizeof(int32_t));   // signed matchings (SO_FLAG_SIGNED_PERM)
    L.off_LD = o; o = align_up(o + (size_t)W * sizeof(double2));          // log det R per walker
    L.off_S = o; o = align_up(o + (size_t)W * Sc * M2 * M2 * sizeof(double2));
    L.off_P = o; o = align_up(o + (size_t)W * Sc * sizeof(double2));
    L.off_pairs = o; o = align_up(o + (size_t)W * S * sizeof(double2));
    L.off_stat = o; o = align_up(o + (size_t)W * sizeof(int32_t));
    L.off_fbc = o; o = align_up(o + sizeof(so_u64));
    L.off_fbl = o; o = align_up(o + (size_t)cap * sizeof(int64_t));
    L.Gy = 0;
    L.off_F = L.off_O = L.off_QF = L.off_RF = o;
    if (with_grad) {
        L.Gy = grad_ranges(W, S);
        L.off_F = o; o = align_up(o + (size_t)W * L.Gy * 2 * n * m * sizeof(double2));
        L.off_O = o; o = align_up(o + (size_t)W * L.Gy * sizeof(double2));
        L.off_QF = o; o = align_up(o + (size_t)W * n * eta * sizeof(double2));
        L.off_RF = o; o = align_up(o + (size_t)W * eta * eta * sizeof(double2));
    }
    L.off_X32 = L.off_C32 = o;
    if (mixed) {
        L.off_X32 = o; o = align_up(o + (size_t)W * DP * DP * sizeof(float));
        L.off_C32 = o; o = align_up(o + (size_t)S * DP * DP * sizeof(float));
    }
    L.total = o;
    return L;
}

// Formation launch: T = ceil(2n/16) tiles, NS = S entries per lane rounded
// up to a power of two.
struct FormArgs {
    int n, eta;
    bool mix;                 // single-precision formation operands
    const void *Xa, *Ca;
    int64_t S_total, s0;
    int Sc, spw;
    double2 *Sb, *Pb;
    so_u64 *fbc;
    int64_t *fbl, fb_cap;
    int32_t *wst;
    int64_t W;
};

template <int T, int NS>
hipError_t launch_form_tn(const FormArgs &a, hipStream_t st) {
    const int m = mvalue(a.n, a.eta);
    const size_t lds = form_lds_bytes_t(T, a.eta, m);
    dim3 grid((unsigned)a.W, (unsigned)((a.Sc + a.spw - 1) / a.spw));
    if (a.mix)
        hipLaunchKernelGGL((k_form_mfma<T, NS, true>), grid, dim3(64), lds, st, a.n, a.eta, a.Xa, a.Ca, a.S_total,
                           a.s0, a.Sc, a.spw, a.Sb, a.Pb, a.fbc, a.fbl, a.fb_cap, a.wst);
    else
        hipLaunchKernelGGL((k_form_mfma<T, NS, false>), grid, dim3(64), lds, st, a.n, a.eta, a.Xa, a.Ca, a.S_total,
                           a.s0, a.Sc, a.spw, a.Sb, a.Pb, a.fbc, a.fbl, a.fb_cap, a.wst);
    return hipGetLastError();
}

template <int T>
hipError_t launch_form_t(const FormArgs &a, int ns, hipStream_t st) {
    if (ns <= 1) return launch_form_tn<T, 1>(a, st);
    if (ns <= 2) return launch_form_tn<T, 2>(a, st);
    if (ns <= 4) return launch_form_tn<T, 4>(a, st);
    if constexpr (T >= 2) {
        if (ns <= 8) return launch_form_tn<T, 8>(a, st);
        if (ns <= 16) return launch_form_tn<T, 16>(a, st);
    }
    if constexpr (T >= 3) {
        if (ns <= 32) return launch_form_tn<T, 32>(a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_form(const FormArgs &a, hipStream_t st) {
    const int M2 = 2 * (a.n - a.eta);
    const int ns = (M2 * M2 + 63) / 64;
    switch (so_tiles(a.n)) {
        case 1: return launch_form_t<1>(a, ns, st);
        case 2: return launch_form_t<2>(a, ns, st);
        case 3: return launch_form_t<3>(a, ns, st);
        default: return hipErrorInvalidValue;
    }
}

// Fused pair kernel: T = ceil(2n/16), NE = ne.  The grid's y extent is
// limited to 65535, so long shadow ranges go in several launches.
template <int T, int NE, bool MIX>
hipError_t launch_pair_tn(int n, int eta, const void *Xa, const void *Ca, int64_t W, int64_t S,
                          const RedTab &rt, double2 *pairs, so_u64 *fbc, int64_t *fbl, int64_t fb_cap,
                          int32_t *wst, const int32_t *match, hipStream_t st) {
    constexpr int NB = pair_node_batch(NE);
    const int spw = NB * (NE > 8 ? kRowBatchesPerWave : kPairBatchesPerWave);
    const size_t lds = pair_lds_bytes(T, n, NE);
    const int64_t ny = (S + spw - 1) / spw;
    for (int64_t y0 = 0; y0 < ny; y0 += 65535) {
        const int64_t gy = (ny - y0) < 65535 ? (ny - y0) : 65535;
        bool done = false;
        if constexpr (!MIX) {
            if (match && n == 8 * T) {   // signed-permutation shadows: gather formation
                hipLaunchKernelGGL((k_pair<T, NE, false, true, true>), dim3((unsigned)W, (unsigned)gy), dim3(64), lds,
                                   st, n, eta, Xa, Ca, S, y0, spw, rt, pairs, fbc, fbl, fb_cap, wst, match);
                done = true;
            }
        }
        if (done) {
        } else if (n == 8 * T) {
            hipLaunchKernelGGL((k_pair<T, NE, MIX, true>), dim3((unsigned)W, (unsigned)gy), dim3(64), lds, st, n, eta,
                               Xa, Ca, S, y0, spw, rt, pairs, fbc, fbl, fb_cap, wst, nullptr);
        } else {
            hipLaunchKernelGGL((k_pair<T, NE, MIX, false>), dim3((unsigned)W, (unsigned)gy), dim3(64), lds, st, n, eta,
                               Xa, Ca, S, y0, spw, rt, pairs, fbc, fbl, fb_cap, wst, nullptr);
        }
        if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    }
    return hipSuccess;
}

template <int T, bool MIX>
hipError_t launch_pair_t(int n, int eta, const void *Xa, const void *Ca, int64_t W, int64_t S,
                         const RedTab &rt, double2 *pairs, so_u64 *fbc, int64_t *fbl, int64_t fb_cap, int32_t *wst,
                         const int32_t *match, hipStream_t st) {
    switch (n - eta) {
        case 2: return launch_pair_tn<T, 2, MIX>(n, eta, Xa, Ca, W, S, rt, pairs, fbc, fbl, fb_cap, wst, match, st);
        case 4: return launch_pair_tn<T, 4, MIX>(n, eta, Xa, Ca, W, S, rt, pairs, fbc, fbl, fb_cap, wst, match, st);
        case 6: return launch_pair_tn<T, 6, MIX>(n, eta, Xa, Ca, W, S, rt, pairs, fbc, fbl, fb_cap, wst, match, st);
        case 8: return launch_pair_tn<T, 8, MIX>(n, eta, Xa, Ca, W, S, rt, pairs, fbc, fbl, fb_cap, wst, match, st);
        default: break;
    }
    if constexpr (T >= 2) {   // ne > 8 needs n > 8
        switch (n - eta) {
            case 10: return launch_pair_tn<T, 10, MIX>(n, eta, Xa, Ca, W, S, rt, pairs, fbc, fbl, fb_cap, wst, match, st);
            case 12: return launch_pair_tn<T, 12, MIX>(n, eta, Xa, Ca, W, S, rt, pairs, fbc, fbl, fb_cap, wst, match, st);
            default: break;
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_pair(int n, int eta, bool mix, const void *Xa, const void *Ca, int64_t W, int64_t S,
                       const NodeTab &tab, double2 *pairs, so_u64 *fbc, int64_t *fbl, int64_t fb_cap, int32_t *wst,
                       const int32_t *match, hipStream_t st) {
    RedTab rt;
    std::memset(&rt, 0, sizeof(rt));
    for (int j = 0; j < tab.Ke; ++j) { rt.e[j] = tab.e[j]; rt.v[j] = tab.v[j]; }
    switch (so_tiles(n) * 2 + (mix ? 1 : 0)) {
        case 2: return launch_pair_t<1, false>(n, eta, Xa, Ca, W, S, rt, pairs, fbc, fbl, fb_cap, wst, match, st);
        case 3: return launch_pair_t<1, true>(n, eta, Xa, Ca, W, S, rt, pairs, fbc, fbl, fb_cap, wst, match, st);
        case 4: return launch_pair_t<2, false>(n, eta, Xa, Ca, W, S, rt, pairs, fbc, fbl, fb_cap, wst, match, st);
        case 5: return launch_pair_t<2, true>(n, eta, Xa, Ca, W, S, rt, pairs, fbc, fbl, fb_cap, wst, match, st);
        case 6: return launch_pair_t<3, false>(n, eta, Xa, Ca, W, S, rt, pairs, fbc, fbl, fb_cap, wst, match, st);
        case 7: return launch_pair_t<3, true>(n, eta, Xa, Ca, W, S, rt, pairs, fbc, fbl, fb_cap, wst, match, st);
        default: return hipErrorInvalidValue;
    }
}

template <int M2>
hipError_t launch_nodes_m(const double2 *Sb, const double2 *Pb, const NodeTab &tab, int64_t npairs,
                          int64_t S, int64_t s0, int Sc, double2 *pairs, hipStream_t st) {
    if constexpr (M2 <= 16) {
        dim3 grid((unsigned)((npairs + 3) / 4));
        hipLaunchKernelGGL((k_nodes<M2, 1>), grid, dim3(64), 0, st, Sb, Pb, tab, npairs, S, s0, Sc, pairs);
    } else if constexpr (M2 <= 32) {
        dim3 grid((unsigned)((npairs + 3) / 4));
        hipLaunchKernelGGL((k_nodes<M2, 2>), grid, dim3(64), 0, st, Sb, Pb, tab, npairs, S, s0, Sc, pairs);
    } else {
        hipLaunchKernelGGL(k_nodes_wide, dim3((unsigned)npairs), dim3(64), 0, st, M2, Sb, Pb, tab, npairs, S, s0,
                           Sc, pairs);
    }
    return hipGetLastError();
}

hipError_t launch_nodes(int M2, const double2 *Sb, const double2 *Pb, const NodeTab &tab, int64_t npairs, int64_t S,
                        int64_t s0, int Sc, double2 *pairs, hipStream_t st) {
    switch (M2) {
#define SO_CASE(MM) case MM: return launch_nodes_m<MM>(Sb, Pb, tab, npairs, S, s0, Sc, pairs, st);
        SO_CASE(0) SO_CASE(2) SO_CASE(4) SO_CASE(6) SO_CASE(8) SO_CASE(10) SO_CASE(12) SO_CASE(14) SO_CASE(16)
        SO_CASE(18) SO_CASE(20) SO_CASE(22) SO_CASE(24) SO_CASE(26) SO_CASE(28) SO_CASE(30) SO_CASE(32)
        SO_CASE(34) SO_CASE(36) SO_CASE(38) SO_CASE(40) SO_CASE(42) SO_CASE(44)
#undef SO_CASE
        default: return hipErrorInvalidValue;
    }
}

// ---- optional per-kernel timing (benchmarks): HIP events around launches
enum { PROF_PFAFF = 0, PROF_FORM = 1, PROF_PAIR = 2, PROF_GRAD = 3, PROF_RDM = 4, PROF_VCE = 5, PROF_ENERGY = 6, PROF_NKIND = 7 };
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

// ---- one problem's plan: validated sizes, workspace pointers, node table
struct ProbPlan {
    int n, eta, m, d, M2, K;
    int64_t W, S;
    Layout L;
    NodeTab tab;
    const double2 *phi;
    const double *Q;
    const uint64_t *bits;
    double2 *overlap, *pairs, *Sb, *Pb;
    const double2 *Xa, *Ca;   // FP64 operands (full-size path; formation unless mixed)
    double *Xw, *Cw;
    bool mix;                 // mixed precision: single-precision formation operands
    bool logout;              // SO_FLAG_LOG_OUTPUT
    int32_t *match;           // signed matchings of the C'_s, or null (SO_FLAG_SIGNED_PERM)
    double2 *logdet;          // log det R per walker (the walkers' orthonormal factors are evaluated)
    bool user_pairs;          // the caller asked for the pair values
    float *X32, *C32;
    const void *Xf, *Cf;      // the formation's operands
    int32_t *wst;
    so_u64 *fbc;
    int64_t *fbl;
};

so_status plan_problem(const so_params *p, const so_c64 *phi, int64_t W, const double *Q, const uint64_t *bits,
                       int64_t S, so_c64 *overlap, so_c64 *pair_out, int32_t *status, char *ws, size_t bytes,
                       ProbPlan *P) {
    int K;
    if (!params_ok(p, &K) || !phi || !Q || !bits || !overlap || W < 1 || S < 1) return SO_ERR_ARG;
    if (!so_supported(p->n, p->eta)) return SO_ERR_UNSUPPORTED;
    if (W > (int64_t)INT32_MAX || S > (int64_t)INT32_MAX) return SO_ERR_ARG;
    P->n = p->n;
    P->eta = p->eta;
    P->m = mvalue(p->n, p->eta);
    P->d = 2 * p->n;
    P->M2 = P->m - p->eta;
    P->K = K;
    P->W = W;
    P->S = S;
    P->mix = p->precision == SO_PREC_MIXED;
    P->logout = (p->flags & SO_FLAG_LOG_OUTPUT) != 0;
    P->L = make_layout(p->n, p->eta, W, S, false, P->mix);
    if (!ws || bytes < P->L.total) return SO_ERR_WORKSPACE;
    build_nodetab(p, K, &P->tab);
    P->phi = reinterpret_cast<const double2 *>(phi);
    P->Q = Q;
    P->bits = bits;
    P->overlap = reinterpret_cast<double2 *>(overlap);
    P->Xw = reinterpret_cast<double *>(ws + P->L.off_X);
    P->Cw = reinterpret_cast<double *>(ws + P->L.off_C);
    P->Xa = reinterpret_cast<const double2 *>(P->Xw);
    P->Ca = reinterpret_cast<const double2 *>(P->Cw);
    P->X32 = reinterpret_cast<float *>(ws + P->L.off_X32);
    P->C32 = reinterpret_cast<float *>(ws + P->L.off_C32);
    P->Xf = P->mix ? static_cast<const void *>(P->X32) : static_cast<const void *>(P->Xa);
    P->Cf = P->mix ? static_cast<const void *>(P->C32) : static_cast<const void *>(P->Ca);
    P->Sb = reinterpret_cast<double2 *>(ws + P->L.off_S);
    P->Pb = reinterpret_cast<double2 *>(ws + P->L.off_P);
    P->pairs = pair_out ? reinterpret_cast<double2 *>(pair_out) : reinterpret_cast<double2 *>(ws + P->L.off_pairs);
    P->user_pairs = pair_out != nullptr;
    P->logdet = reinterpret_cast<double2 *>(ws + P->L.off_LD);
    P->wst = status ? status : reinterpret_cast<int32_t *>(ws + P->L.off_stat);
    P->fbc = reinterpret_cast<so_u64 *>(ws + P->L.off_fbc);
    P->fbl = reinterpret_cast<int64_t *>(ws + P->L.off_fbl);
    // the gather formation: FP64, fused kernel, n = 8T
    const bool perm = (p->flags & SO_FLAG_SIGNED_PERM) && !P->mix && fused_ok(P->n, P->eta) &&
                      P->n == 8 * so_tiles(P->n);
    P->match = perm ? reinterpret_cast<int32_t *>(ws + P->L.off_M) : nullptr;
    return SO_OK;
}

// walker and shadow preparation (X_w, C'_s; clears the fallback queue)
hipError_t enqueue_prep(const ProbPlan &P, hipStream_t st) {
    hipLaunchKernelGGL(k_walker_prep, dim3((unsigned)P.W), dim3(64), 0, st, P.n, P.eta, P.phi, P.Xw, P.wst, P.fbc,
                       P.logdet);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_shadow_prep, dim3((unsigned)P.S), dim3(256), (size_t)P.d * P.d * sizeof(double), st, P.n,
                       P.Q, P.bits, P.Cw);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (P.match) {
        hipLaunchKernelGGL(k_perm_match, dim3((unsigned)P.S), dim3(64), 0, st, P.n, P.Cw, P.match);
        e = hipGetLastError();
    }
    if (e != hipSuccess || !P.mix) return e;
    // single-precision formation operands (the FP64 ones stay for the full-size path)
    const int T = so_tiles(P.n), DP = 16 * T;
    const unsigned bx = (unsigned)((DP * DP + 255) / 256);
    hipLaunchKernelGGL(k_to_f32, dim3(bx, (unsigned)(P.W < 65535 ? P.W : 65535)), dim3(256), 0, st, T, 0, P.W,
                       P.Xw, P.X32);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_to_f32, dim3(bx, (unsigned)(P.S < 65535 ? P.S : 65535)), dim3(256), 0, st, T, 1, P.S,
                       P.Cw, P.C32);
    return hipGetLastError();
}

// the two-kernel path (n - eta odd, 0 or above 8): formation + Schur
// complement per chunk of shadows, then the node Pfaffians of the chunk
hipError_t enqueue_two_kernel(const ProbPlan &P, hipStream_t st) {
    FormArgs fa{P.n, P.eta, P.mix, P.Xf, P.Cf, P.S, 0, 0, kFormShadowsPerWave, P.Sb, P.Pb, P.fbc, P.fbl, P.L.fb_cap,
                P.wst, P.W};
    for (int64_t s0 = 0; s0 < P.S; s0 += P.L.Sc) {
        const int Sc = (int)((P.S - s0) < P.L.Sc ? (P.S - s0) : P.L.Sc);
        fa.s0 = s0;
        fa.Sc = Sc;
        hipEvent_t ea = nullptr, eb = nullptr;
        hipError_t e = prof_begin(st, &ea);
        if (e == hipSuccess) e = launch_form(fa, st);
        if (e == hipSuccess) e = prof_end(st, ea, PROF_FORM, P.W * Sc);
        if (e == hipSuccess) e = prof_begin(st, &eb);
        if (e == hipSuccess) e = launch_nodes(P.M2, P.Sb, P.Pb, P.tab, P.W * Sc, P.S, s0, Sc, P.pairs, st);
        if (e == hipSuccess) e = prof_end(st, eb, PROF_PFAFF, P.W * Sc);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// the full-size path for the flagged pairs, then S_w
hipError_t enqueue_finish(const ProbPlan &P, hipStream_t st) {
    RedTab rt;
    std::memset(&rt, 0, sizeof(rt));
    for (int j = 0; j < P.tab.Ke; ++j) { rt.e[j] = P.tab.e[j]; rt.v[j] = P.tab.v[j]; }
    // the largest shapes (n = 24, small eta) need more than the default 64 KiB
    static const bool fb_attr = [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_fallback),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)fb_lds_bytes(SO_NMAX_SUPPORTED, 0));
        return true;
    }();
    (void)fb_attr;
    hipLaunchKernelGGL(k_fallback, dim3(FB_GRID), dim3(64), fb_lds_bytes(P.n, P.eta), st, P.n, P.eta, P.Xw, P.Cw,
                       rt, P.tab.Ke, P.fbc, P.fbl, P.L.fb_cap, P.W, P.S, P.pairs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)P.W), dim3(64), 0, st, P.pairs, P.S, P.overlap, P.wst,
                       P.logout ? 1 : 0, P.logdet, P.user_pairs ? 1 : 0);
    return hipGetLastError();
}

// ---- batches: one fused launch, XCD-aware LPT order, tuning knobs
constexpr int kBatchMax = 16;
constexpr int kDefaultWavesPerCU = 8;

int device_cus() {
    static int cached = 0;
    if (!cached) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cached = v;
        else
            cached = 256;
    }
    return cached;
}

// node batch of the fused kernel (pairs whose nodes run together)
int node_batch(int ne) { return pair_node_batch(ne); }

int item_shadows(const so_problem &pr, int ne) {
    const int nb = node_batch(ne);
    int spw = pr.shadows_per_item > 0 ? pr.shadows_per_item : nb * kPairBatchesPerWave;
    spw = ((spw + nb - 1) / nb) * nb;
    return spw;
}

// relative cost of one pair (formation + elimination + node Pfaffians)
double pair_cost(int n, int eta) {
    const double ne = n - eta, m = 2.0 * n - eta;
    return 16.0 * n * n * m + 8.0 * n * m * m + 8.0 * (n * n * (n + 2 * ne)) + (ne + 1) * 8.0 * ne * ne * ne;
}

#ifndef SO_BATCH_ROUNDS
#define SO_BATCH_ROUNDS 1
#endif
constexpr int kBatchRounds = SO_BATCH_ROUNDS;   // rounds of the batch queues (1: LPT order)

// device region of one batch launch: the job table and its header
struct BatchRegion {
    BatchJob *jobs;
    BatchHdr *hdr;
};
size_t batch_region_bytes() {
    return align_up((size_t)SO_BATCH_MAXJOBS * sizeof(BatchJob)) + align_up(sizeof(BatchHdr));
}
BatchRegion batch_region(char *base) {
    BatchRegion r;
    r.jobs = reinterpret_cast<BatchJob *>(base);
    r.hdr = reinterpret_cast<BatchHdr *>(base + align_up((size_t)SO_BATCH_MAXJOBS * sizeof(BatchJob)));
    return r;
}

template <int LEVEL>
hipError_t launch_batch_t(bool mix, int64_t grid, size_t lds, const BatchRegion &rg, hipStream_t st) {
    if (mix)
        hipLaunchKernelGGL((k_pair_batch<LEVEL, true>), dim3((unsigned)grid), dim3(64), lds, st, rg.jobs, rg.hdr);
    else
        hipLaunchKernelGGL((k_pair_batch<LEVEL, false>), dim3((unsigned)grid), dim3(64), lds, st, rg.jobs, rg.hdr);
    return hipGetLastError();
}

// One fused launch over the problems ix[0..nj) (one formation
// precision; ix in longest-processing-time order), shadows [0, S_limit) of
// each (S_limit <= 0: all).  The job table and the header are written by
// kernels, so the sequence can be captured into a graph.
hipError_t launch_batch(const ProbPlan *plans, const so_problem *probs, const int *ix, int nj, int64_t S_limit,
                        int waves_per_cu, int rounds, const BatchRegion &rg, hipStream_t st) {
    BatchHdr hdr;
    std::memset(&hdr, 0, sizeof(hdr));
    hdr.njobs = nj;
    int level = 0;
    size_t lds = 0;
    int64_t items = 0, pairs = 0;
    if (rounds < 1) rounds = 1;
    for (int k = 0; k < nj; ++k) {
        const ProbPlan &P = plans[ix[k]];
        BatchJob jb;
        std::memset(&jb, 0, sizeof(jb));
        const int64_t S = (S_limit > 0 && S_limit < P.S) ? S_limit : P.S;
        const int T = so_tiles(P.n), NE = P.n - P.eta;
        jb.Xa = P.Xf;
        jb.Ca = P.Cf;
        jb.pairs = P.pairs;
        jb.fb_count = P.fbc;
        jb.fb_list = P.fbl;
        jb.wstat = P.wst;
        jb.fb_cap = P.L.fb_cap;
        jb.S = P.S;
        jb.n = P.n;
        jb.eta = P.eta;
        jb.W = (int)P.W;
        jb.spw = item_shadows(probs[ix[k]], NE);
        jb.cls = 16 * T + NE + (P.n == 8 * T ? 256 : 0);   // + 256: the n = 8T instance
        const int64_t nY = (S + jb.spw - 1) / jb.spw;
        for (int x = 0; x < SO_BATCH_XCD; ++x) {
            const int64_t Wx = (P.W - x + SO_BATCH_XCD - 1) / SO_BATCH_XCD;
            jb.len[x] = Wx > 0 ? Wx * nY : 0;
            jb.per_round[x] = (jb.len[x] + rounds - 1) / rounds;
            hdr.round_len[x] += jb.per_round[x];
            items += jb.len[x];
        }
        for (int j = 0; j < P.tab.Ke; ++j) { jb.tab.e[j] = P.tab.e[j]; jb.tab.v[j] = P.tab.v[j]; }
        hipLaunchKernelGGL(k_batch_setup, dim3(1), dim3(64), 0, st, jb, rg.jobs + k);
        if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
        const int lv = pair_class_level(T, NE, P.mix);
        if (lv > level) level = lv;
        const size_t b = pair_lds_bytes(T, P.n, NE);
        if (b > lds) lds = b;
        pairs += P.W * S;
    }
    int64_t qmax = 0;
    for (int x = 0; x < SO_BATCH_XCD; ++x) {
        hdr.qlen[x] = (int64_t)rounds * hdr.round_len[x];
        if (hdr.qlen[x] > qmax) qmax = hdr.qlen[x];
    }
    (void)items;
    (void)waves_per_cu;
    const int64_t grid = (int64_t)SO_BATCH_XCD * qmax;
    if (grid < 1 || grid > (int64_t)INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_header, dim3(1), dim3(64), 0, st, hdr, rg.hdr);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    hipEvent_t ea = nullptr;
    hipError_t e = prof_begin(st, &ea);
    if (e != hipSuccess) return e;
    const bool mix = plans[ix[0]].mix;
    switch (level) {
        case 0: e = launch_batch_t<0>(mix, grid, lds, rg, st); break;
        case 1: e = launch_batch_t<1>(mix, grid, lds, rg, st); break;
        default: e = launch_batch_t<2>(mix, grid, lds, rg, st); break;
    }
    if (e == hipSuccess) e = prof_end(st, ea, PROF_PAIR, pairs);
    return e;
}

size_t batch_layout(const so_problem *probs, int n_probs, size_t *offs) {
    size_t o = 0;
    for (int k = 0; k < n_probs; ++k) {
        offs[k] = o;
        o = align_up(o + make_layout(probs[k].params.n, probs[k].params.eta, probs[k].n_walkers,
                                     probs[k].n_shadows, false, probs[k].params.precision == SO_PREC_MIXED)
                             .total);
    }
    offs[n_probs] = o;                                   // two launch regions (FP64, mixed)
    return o + 2 * batch_region_bytes();
}

bool problem_ok(const so_problem &pr) {
    int K;
    return params_ok(&pr.params, &K) && pr.n_walkers >= 1 && pr.n_shadows >= 1 && pr.phi && pr.Q && pr.bits &&
           pr.overlap;
}

// one-particle density matrix: blocks of the partial kernel and their shadows
struct RdmPlan {
    int T, DP;
    int64_t blocks, spb;
    size_t bytes;
};
RdmPlan rdm_plan(int n, int64_t S) {
    RdmPlan r;
    r.T = so_tiles(n);
    r.DP = 16 * r.T;
    r.blocks = S < kRdmBlocks ? S : kRdmBlocks;
    r.spb = (S + r.blocks - 1) / r.blocks;
    r.blocks = (S + r.spb - 1) / r.spb;
    r.bytes = (size_t)(r.blocks + 1) * r.DP * r.DP * sizeof(double);
    return r;
}

// VCE dimensions: core and active blocks inside the basis, at most
// SO_VCE_NAMAX active orbitals, and one walker's matrices within the LDS
// budget of k_vce_prep.
bool vce_dims_ok(const so_vce_dims *d, VceDims *v) {
    if (!d) return false;
    v->nb = d->n_basis; v->nc = d->n_core; v->na = d->n_active; v->nal = d->n_alpha; v->nbe = d->n_beta;
    if (v->nc < 0 || v->na < 1 || v->na > SO_VCE_NAMAX || v->nal < 0 || v->nbe < 0) return false;
    if (v->nal > v->na || v->nbe > v->na || v->nal + v->nbe < 1) return false;
    if (v->nb < v->nc + v->na) return false;
    return vce_lds_entries(*v) * sizeof(double2) <= SO_VCE_LDS_MAX;
}

hipError_t launch_vce_prep(const VceDims &v, const so_c64 *pa, const so_c64 *pb, int64_t W, double2 *act,
                           double2 *pref, hipStream_t st) {
    hipEvent_t ea = nullptr;
    hipError_t e = prof_begin(st, &ea);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_vce_prep, dim3((unsigned)W), dim3(64), vce_lds_entries(v) * sizeof(double2), st, v,
                       reinterpret_cast<const double2 *>(pa), reinterpret_cast<const double2 *>(pb), act, pref);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return prof_end(st, ea, PROF_VCE, W);
}

// Workspace of so_local_energy: walker matrices and shadow covariances in A
// order, the Hamiltonian tables, the per-shadow M, per-pair values, status.
struct EnLayout {
    size_t off_X, off_C, off_V, off_K2, off_Kt, off_M, off_o, off_e, off_stat, off_Xr, off_Cr, off_LD, total;
};
EnLayout energy_layout(int n, int64_t W, int64_t S) {
    const int T = so_tiles(n), DP = 16 * T, d = 2 * n;
    EnLayout L;
    size_t o = 0;
    L.off_X = o; o = align_up(o + (size_t)W * DP * DP * sizeof(double));
    L.off_C = o; o = align_up(o + (size_t)S * DP * DP * sizeof(double));
    L.off_V = o; o = align_up(o + (size_t)n * n * n * n * sizeof(double));
    L.off_K2 = o; o = align_up(o + (size_t)n * n * sizeof(double));
    L.off_Kt = o; o = align_up(o + (size_t)d * d * sizeof(double2));
    L.off_M = o; o = align_up(o + (size_t)S * d * d * sizeof(double));
    L.off_o = o; o = align_up(o + (size_t)W * S * sizeof(double2));
    L.off_e = o; o = align_up(o + (size_t)W * S * sizeof(double2));
    L.off_stat = o; o = align_up(o + (size_t)W * sizeof(int32_t));
    L.off_Xr = o; o = align_up(o + (size_t)W * (2 * n - 2) * d * sizeof(double2));   // m <= 2n - 2
    L.off_Cr = o; o = align_up(o + (size_t)S * d * d * sizeof(double));
    L.off_LD = o; o = align_up(o + (size_t)W * sizeof(double2));   // log det R per walker
    L.total = o;
    return L;
}

// Nodes of the local energy.  Pf(C_0 + z B) = z^{eta/2} R(z) with deg R = n - eta
// (its coefficients vanish below x = eta/2), for the walker and for every
// walker along e^{lambda Lhat}, which keeps eta particles; so K' = n - eta + 1
// nodes determine R, its lambda-derivatives and the estimator.  They sit on
// the unit circle a third of a step off the roots of unity,
// z_k = exp(2 pi i (k + 1/3) / K'), which never meets +-1 or +-i (z = -1 is a
// root of every pair's Pfaffian when n - eta is odd), and
//   w_k = pref psign / K' sum_{x = eta/2}^{ell} mu_x z_k^{-x}.
void energy_nodetab(const so_params *p, EnTab *t) {
    const int n = p->n, eta = p->eta, ell = n - eta / 2, Kp = n - eta + 1;
    long double mu[SO_KMAX];
    cld pref;
    estimator_terms(p, SO_KMAX, mu, &pref);
    const double psign = row_order_sign(n, eta);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    std::memset(t, 0, sizeof(*t));
    t->K = Kp;
    for (int k = 0; k < Kp; ++k) {
        const long double th = two_pi * ((long double)k + 1.0L / 3.0L) / Kp;
        long double sr = 0.0L, si = 0.0L;
        for (int x = eta / 2; x <= ell; ++x) {
            sr += mu[x] * cosl(-x * th);
            si += mu[x] * sinl(-x * th);
        }
        sr /= Kp;
        si /= Kp;
        t->s[k] = make_double2((double)cosl(th), (double)sinl(th));
        t->c[k] = make_double2(1.0, 0.0);
        t->w[k] = make_double2((double)(pref.re * sr - pref.im * si) * psign, (double)(pref.re * si + pref.im * sr) * psign);
    }
}

bool energy_args_ok(const so_params *p, int64_t W, int64_t S, int n_gamma, int *K) {
    if (!params_ok(p, K) || W < 1 || S < 1 || n_gamma < 0) return false;
    if (W > 65535 || S > (int64_t)INT32_MAX) return false;
    return true;
}

size_t vce_extra_bytes(int64_t W, int n, int eta) {
    return align_up((size_t)W * n * eta * sizeof(double2)) + align_up((size_t)W * sizeof(double2));
}

}  // namespace

// ==========================================================================
// Library-owned scratch of shadow_overlap_noalloc: one static device array
// per GPU, held until the process ends.  Host code never uses the array's
// name as an address (on the host it is only a stand-in for the symbol): the
// device address comes from hipGetSymbolAddress, once per device with that
// device current, and is kept per device.
// ==========================================================================
__device__ __align__(256) unsigned char scratch[SO_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// device address of this device's scratch array (set-up on the first call)
hipError_t scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
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
    return (mvalue(n, eta) <= SO_MMAX) ? 1 : 0;
}

so_status so_workspace_size(const so_params *p, int64_t n_walkers, int64_t n_shadows, int with_grad,
                            size_t *bytes) {
    int K;
    if (!bytes || !params_ok(p, &K) || n_walkers < 1 || n_shadows < 1) return SO_ERR_ARG;
    if (!so_supported(p->n, p->eta)) return SO_ERR_UNSUPPORTED;
    *bytes = make_layout(p->n, p->eta, n_walkers, n_shadows, with_grad != 0, p->precision == SO_PREC_MIXED).total;
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
    ProbPlan P;
    const so_status sv = plan_problem(p, phi, n_walkers, Q, bits, n_shadows, overlap, pair_out, status,
                                      static_cast<char *>(workspace), workspace_bytes, &P);
    if (sv != SO_OK) return sv;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (enqueue_prep(P, st) != hipSuccess) return SO_ERR_HIP;
    if (fused_ok(P.n, P.eta)) {
        hipEvent_t ea = nullptr;
        if (prof_begin(st, &ea) != hipSuccess) return SO_ERR_HIP;
        if (launch_pair(P.n, P.eta, P.mix, P.Xf, P.Cf, P.W, P.S, P.tab, P.pairs, P.fbc, P.fbl, P.L.fb_cap, P.wst,
                        P.match, st) != hipSuccess)
            return SO_ERR_HIP;
        if (prof_end(st, ea, PROF_PAIR, P.W * P.S) != hipSuccess) return SO_ERR_HIP;
    } else if (enqueue_two_kernel(P, st) != hipSuccess) {
        return SO_ERR_HIP;
    }
    if (enqueue_finish(P, st) != hipSuccess) return SO_ERR_HIP;
    return SO_OK;
}

so_status shadow_overlap_noalloc(const so_params *p, const so_c64 *phi, int64_t n_walkers, const double *Q,
                                 const uint64_t *bits, int64_t n_shadows, so_c64 *overlap, so_c64 *pair_out,
                                 int32_t *status, void *stream) {
    // every argument check of shadow_overlap comes before the first HIP call
    int K;
    if (!params_ok(p, &K) || !phi || !Q || !bits || !overlap || n_walkers < 1 || n_shadows < 1 ||
        n_walkers > (int64_t)INT32_MAX || n_shadows > (int64_t)INT32_MAX)
        return SO_ERR_ARG;
    size_t need = 0;
    const so_status sv = so_workspace_size(p, n_walkers, n_shadows, 0, &need);
    if (sv != SO_OK) return sv;
    if (need > (size_t)SO_NOALLOC_SCRATCH_BYTES) return SO_ERR_WORKSPACE;
    void *ptr = nullptr;
    if (scratch_address(&ptr) != hipSuccess) return SO_ERR_HIP;
    // the same kernels as shadow_overlap, on the scratch array: every region
    // that must start at zero (the queue counter) or hold statuses is written
    // by the kernels themselves, so no memset is needed
    return shadow_overlap(p, phi, n_walkers, Q, bits, n_shadows, overlap, pair_out, status, ptr,
                          (size_t)SO_NOALLOC_SCRATCH_BYTES, stream);
}

so_status shadow_overlap_grad(const so_params *p, const so_c64 *phi, int64_t n_walkers, const double *Q,
                              const uint64_t *bits, int64_t n_shadows, so_c64 *overlap, so_c64 *dlog,
                              so_c64 *green, int32_t *status, void *workspace, size_t workspace_bytes,
                              void *stream) {
    int K;
    if (!params_ok(p, &K) || !phi || !Q || !bits || !overlap || !dlog || n_walkers < 1 || n_shadows < 1)
        return SO_ERR_ARG;
    if (!so_supported(p->n, p->eta) || !grad_ok(p->n, p->eta)) return SO_ERR_UNSUPPORTED;
    if (p->precision != SO_PREC_FP64) return SO_ERR_UNSUPPORTED;
    if (n_walkers > (int64_t)INT32_MAX || n_shadows > (int64_t)INT32_MAX) return SO_ERR_ARG;
    const int n = p->n, eta = p->eta, d = 2 * n, NE = n - eta, T = so_tiles(n);
    const int64_t W = n_walkers, S = n_shadows;
    Layout L = make_layout(n, eta, W, S, true);
    if (!workspace || workspace_bytes < L.total) return SO_ERR_WORKSPACE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(workspace);
    double *Xa = reinterpret_cast<double *>(ws + L.off_X);
    double *Ca = reinterpret_cast<double *>(ws + L.off_C);
    int32_t *wst = status ? status : reinterpret_cast<int32_t *>(ws + L.off_stat);
    so_u64 *fbc = reinterpret_cast<so_u64 *>(ws + L.off_fbc);
    double2 *Fp = reinterpret_cast<double2 *>(ws + L.off_F);
    double2 *Op = reinterpret_cast<double2 *>(ws + L.off_O);
    double2 *Qf = reinterpret_cast<double2 *>(ws + L.off_QF);
    double2 *Rf = reinterpret_cast<double2 *>(ws + L.off_RF);
    double2 *Ld = reinterpret_cast<double2 *>(ws + L.off_LD);
    NodeTab tab;
    build_nodetab(p, K, &tab);
    RedTab rt;
    std::memset(&rt, 0, sizeof(rt));
    for (int j = 0; j < tab.Ke; ++j) { rt.e[j] = tab.e[j]; rt.v[j] = tab.v[j]; }

    // Phi = Qf R: the pairs are evaluated at Qf and k_grad_walker carries
    // S, D and G back to Phi, so no node Pfaffian depends on the walker norm
    hipLaunchKernelGGL(k_walker_prep, dim3((unsigned)W), dim3(64), 0, st, n, eta,
                       reinterpret_cast<const double2 *>(phi), Xa, wst, fbc, Ld, Qf, Rf);
    if (hipGetLastError() != hipSuccess) return SO_ERR_HIP;
    hipLaunchKernelGGL(k_shadow_prep, dim3((unsigned)S), dim3(256), (size_t)d * d * sizeof(double), st, n, Q,
                       bits, Ca);
    if (hipGetLastError() != hipSuccess) return SO_ERR_HIP;
    const int spw = (int)((S + L.Gy - 1) / L.Gy);
    hipEvent_t ea = nullptr;
    if (prof_begin(st, &ea) != hipSuccess) return SO_ERR_HIP;
    const dim3 grid((unsigned)W, (unsigned)L.Gy);
    const size_t lds = grad_lds(T, n, NE).total;
    const double2 *Xc = reinterpret_cast<const double2 *>(Xa);
    const double2 *Cc = reinterpret_cast<const double2 *>(Ca);
#define SO_GRAD_LAUNCH(TT, NN)                                                                              \
    hipLaunchKernelGGL((k_grad_pair<TT, NN>), grid, dim3(128), lds, st, n, eta, Xc, Cc, S, spw, rt, Fp, Op, wst)
    switch (T * 16 + NE) {
        case 16 + 2: SO_GRAD_LAUNCH(1, 2); break;
        case 16 + 4: SO_GRAD_LAUNCH(1, 4); break;
        case 16 + 6: SO_GRAD_LAUNCH(1, 6); break;
        case 32 + 2: SO_GRAD_LAUNCH(2, 2); break;
        case 32 + 4: SO_GRAD_LAUNCH(2, 4); break;
        case 32 + 6: SO_GRAD_LAUNCH(2, 6); break;
        case 32 + 8: SO_GRAD_LAUNCH(2, 8); break;
        default: return SO_ERR_UNSUPPORTED;
    }
#undef SO_GRAD_LAUNCH
    if (hipGetLastError() != hipSuccess) return SO_ERR_HIP;
    if (prof_end(st, ea, PROF_GRAD, W * S) != hipSuccess) return SO_ERR_HIP;
    hipLaunchKernelGGL(k_grad_walker, dim3((unsigned)W), dim3(64), 0, st, n, eta, static_cast<const double2 *>(Qf),
                       Xa, Fp, Op, L.Gy, S, reinterpret_cast<double2 *>(overlap), reinterpret_cast<double2 *>(dlog),
                       reinterpret_cast<double2 *>(green), wst, (p->flags & SO_FLAG_LOG_OUTPUT) ? 1 : 0,
                       static_cast<const double2 *>(Rf), static_cast<const double2 *>(Ld));
    if (hipGetLastError() != hipSuccess) return SO_ERR_HIP;
    return SO_OK;
}

so_status so_rdm1_workspace_size(int n, int64_t n_shadows, size_t *bytes) {
    if (!bytes || n < 2 || n > SO_NMAX_SUPPORTED || n_shadows < 1) return SO_ERR_ARG;
    *bytes = rdm_plan(n, n_shadows).bytes;
    return SO_OK;
}

so_status so_rdm1(int n, const double *Q, const uint64_t *bits, int64_t n_shadows, int trial, so_c64 *rdm,
                  double *majorana, void *workspace, size_t workspace_bytes, void *stream) {
    if (!Q || !bits || !rdm || n < 2 || n > SO_NMAX_SUPPORTED || n_shadows < 1) return SO_ERR_ARG;
    const RdmPlan r = rdm_plan(n, n_shadows);
    if (!workspace || workspace_bytes < r.bytes) return SO_ERR_WORKSPACE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    double *part = static_cast<double *>(workspace);
    double *Xsum = part + (size_t)r.blocks * r.DP * r.DP;
    hipEvent_t ea = nullptr;
    if (prof_begin(st, &ea) != hipSuccess) return SO_ERR_HIP;
    switch (r.T) {
        case 1: hipLaunchKernelGGL(k_rdm_partial<1>, dim3((unsigned)r.blocks), dim3(256), 0, st, n, Q, bits, n_shadows, r.spb, part); break;
        case 2: hipLaunchKernelGGL(k_rdm_partial<2>, dim3((unsigned)r.blocks), dim3(256), 0, st, n, Q, bits, n_shadows, r.spb, part); break;
        case 3: hipLaunchKernelGGL(k_rdm_partial<3>, dim3((unsigned)r.blocks), dim3(256), 0, st, n, Q, bits, n_shadows, r.spb, part); break;
        default: return SO_ERR_UNSUPPORTED;
    }
    if (hipGetLastError() != hipSuccess) return SO_ERR_HIP;
    if (prof_end(st, ea, PROF_RDM, n_shadows) != hipSuccess) return SO_ERR_HIP;
    const int dp2 = r.DP * r.DP;
    hipLaunchKernelGGL(k_rdm_sum, dim3((unsigned)((dp2 + 63) / 64)), dim3(1024), 0, st, dp2, (int)r.blocks, part, Xsum);
    if (hipGetLastError() != hipSuccess) return SO_ERR_HIP;
    hipLaunchKernelGGL(k_rdm_out, dim3(1), dim3(256), 0, st, n, r.DP, Xsum, (2.0 * n - 1.0) / (double)n_shadows,
                       trial ? 2.0 : 1.0, majorana, reinterpret_cast<double2 *>(rdm));
    return hipGetLastError() == hipSuccess ? SO_OK : SO_ERR_HIP;
}

so_status so_force_bias(const so_c64 *green, int64_t n_walkers, int n, const double *L, int64_t n_gamma,
                        double dt, so_c64 *xbar, void *stream) {
    if (!green || !L || !xbar || n_walkers < 1 || n_gamma < 1 || n < 1 || n > SO_NMAX || !(dt >= 0.0))
        return SO_ERR_ARG;
    if (n_walkers > (int64_t)INT32_MAX) return SO_ERR_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_force_bias, dim3((unsigned)n_walkers), dim3(256), 0, st,
                       reinterpret_cast<const double2 *>(green), n, L, n_gamma, std::sqrt(dt),
                       reinterpret_cast<double2 *>(xbar));
    return hipGetLastError() == hipSuccess ? SO_OK : SO_ERR_HIP;
}

so_status so_vce_walkers(const so_vce_dims *dims, const so_c64 *phi_alpha, const so_c64 *phi_beta,
                         int64_t n_walkers, so_c64 *active_phi, so_c64 *prefactor, void *stream) {
    VceDims v;
    if (!vce_dims_ok(dims, &v) || !phi_alpha || !phi_beta || !active_phi || !prefactor || n_walkers < 1 ||
        n_walkers > (int64_t)INT32_MAX)
        return SO_ERR_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return launch_vce_prep(v, phi_alpha, phi_beta, n_walkers, reinterpret_cast<double2 *>(active_phi),
                           reinterpret_cast<double2 *>(prefactor), st) == hipSuccess
               ? SO_OK
               : SO_ERR_HIP;
}

so_status so_vce_workspace_size(const so_params *p, const so_vce_dims *dims, int64_t n_walkers,
                                int64_t n_shadows, size_t *bytes) {
    VceDims v;
    if (!bytes || !p || !vce_dims_ok(dims, &v) || p->n != 2 * v.na || p->eta != v.nal + v.nbe) return SO_ERR_ARG;
    size_t base = 0;
    const so_status sv = so_workspace_size(p, n_walkers, n_shadows, 0, &base);
    if (sv != SO_OK) return sv;
    *bytes = align_up(base) + vce_extra_bytes(n_walkers, p->n, p->eta);
    return SO_OK;
}

so_status so_vce_overlap(const so_params *p, const so_vce_dims *dims, const so_c64 *phi_alpha,
                         const so_c64 *phi_beta, int64_t n_walkers, const double *Q, const uint64_t *bits,
                         int64_t n_shadows, so_c64 *overlap, so_c64 *prefactor, int32_t *status,
                         void *workspace, size_t workspace_bytes, void *stream) {
    VceDims v;
    // every check of shadow_overlap is made here, before anything is enqueued
    if (!phi_alpha || !phi_beta || !overlap || !Q || !bits || !vce_dims_ok(dims, &v) || n_walkers < 1 ||
        n_shadows < 1 || n_walkers > (int64_t)INT32_MAX || n_shadows > (int64_t)INT32_MAX)
        return SO_ERR_ARG;
    size_t need = 0;
    const so_status sv = so_vce_workspace_size(p, dims, n_walkers, n_shadows, &need);
    if (sv != SO_OK) return sv;
    if (!workspace || workspace_bytes < need) return SO_ERR_WORKSPACE;
    size_t base = 0;
    (void)so_workspace_size(p, n_walkers, n_shadows, 0, &base);
    char *ws = static_cast<char *>(workspace);
    double2 *act = reinterpret_cast<double2 *>(ws + align_up(base));
    double2 *pref = prefactor ? reinterpret_cast<double2 *>(prefactor)
                              : reinterpret_cast<double2 *>(ws + align_up(base) +
                                                            align_up((size_t)n_walkers * p->n * p->eta * sizeof(double2)));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (launch_vce_prep(v, phi_alpha, phi_beta, n_walkers, act, pref, st) != hipSuccess) return SO_ERR_HIP;
    const so_status so = shadow_overlap(p, reinterpret_cast<const so_c64 *>(act), n_walkers, Q, bits, n_shadows,
                                        overlap, nullptr, status, workspace, base, stream);
    if (so != SO_OK) return so;
    hipLaunchKernelGGL(k_vce_scale, dim3((unsigned)((n_walkers + 255) / 256)), dim3(256), 0, st, n_walkers, pref,
                       reinterpret_cast<double2 *>(overlap), (p->flags & SO_FLAG_LOG_OUTPUT) ? 1 : 0);
    return hipGetLastError() == hipSuccess ? SO_OK : SO_ERR_HIP;
}

so_status so_local_energy_workspace_size(const so_params *p, int64_t n_walkers, int64_t n_shadows, int n_gamma,
                                         size_t *bytes) {
    int K;
    if (!bytes || !energy_args_ok(p, n_walkers, n_shadows, n_gamma, &K)) return SO_ERR_ARG;
    if (!so_supported(p->n, p->eta) || p->n > SO_EN_NMAX || p->precision != SO_PREC_FP64) return SO_ERR_UNSUPPORTED;
    *bytes = energy_layout(p->n, n_walkers, n_shadows).total;
    return SO_OK;
}

so_status so_local_energy(const so_params *p, const so_c64 *phi, int64_t n_walkers, const double *Q,
                          const uint64_t *bits, int64_t n_shadows, const so_c64 *t, const double *L, int n_gamma,
                          so_c64 *overlap, so_c64 *numerator, so_c64 *energy, so_c64 *pair_overlap,
                          so_c64 *pair_numerator, int32_t *status, void *workspace, size_t workspace_bytes,
                          void *stream) {
    int K;
    if (!phi || !Q || !bits || !t || (n_gamma > 0 && !L) || !energy_args_ok(p, n_walkers, n_shadows, n_gamma, &K))
        return SO_ERR_ARG;
    if (!overlap && !numerator && !energy && !pair_overlap && !pair_numerator) return SO_ERR_ARG;
    if (p->flags & SO_FLAG_LOG_OUTPUT) return SO_ERR_UNSUPPORTED;
    if (!so_supported(p->n, p->eta) || p->n > SO_EN_NMAX || p->precision != SO_PREC_FP64) return SO_ERR_UNSUPPORTED;
    const int n = p->n, eta = p->eta, d = 2 * n, T = so_tiles(n);
    const int64_t W = n_walkers, S = n_shadows;
    const EnLayout Lo = energy_layout(n, W, S);
    if (!workspace || workspace_bytes < Lo.total) return SO_ERR_WORKSPACE;
    char *ws = static_cast<char *>(workspace);
    double *Xa = reinterpret_cast<double *>(ws + Lo.off_X);
    double *Ca = reinterpret_cast<double *>(ws + Lo.off_C);
    double *Vt = reinterpret_cast<double *>(ws + Lo.off_V);
    double *K2 = reinterpret_cast<double *>(ws + Lo.off_K2);
    double2 *Kt = reinterpret_cast<double2 *>(ws + Lo.off_Kt);
    double *Ms = reinterpret_cast<double *>(ws + Lo.off_M);
    double2 *op = pair_overlap ? reinterpret_cast<double2 *>(pair_overlap) : reinterpret_cast<double2 *>(ws + Lo.off_o);
    double2 *ep = pair_numerator ? reinterpret_cast<double2 *>(pair_numerator)
                                 : reinterpret_cast<double2 *>(ws + Lo.off_e);
    int32_t *wst = status ? status : reinterpret_cast<int32_t *>(ws + Lo.off_stat);
    double2 *Xr = reinterpret_cast<double2 *>(ws + Lo.off_Xr);
    double *Cr = reinterpret_cast<double *>(ws + Lo.off_Cr);
    double2 *Ld = reinterpret_cast<double2 *>(ws + Lo.off_LD);
    // n - eta + 1 nodes off the roots of unity, whatever p->nodes asks for
    EnTab tab;
    energy_nodetab(p, &tab);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // the pairs run at each walker's orthonormal factor (Phi = Qf R); the
    // reduction applies det R to S_w and N_w (E_w does not depend on it)
    hipLaunchKernelGGL(k_walker_prep, dim3((unsigned)W), dim3(64), 0, st, n, eta,
                       reinterpret_cast<const double2 *>(phi), Xa, wst, static_cast<so_u64 *>(nullptr), Ld);
    if (hipGetLastError() != hipSuccess) return SO_ERR_HIP;
    hipLaunchKernelGGL(k_shadow_prep, dim3((unsigned)S), dim3(256), (size_t)d * d * sizeof(double), st, n, Q, bits, Ca);
    if (hipGetLastError() != hipSuccess) return SO_ERR_HIP;
    const int n4 = n * n * n * n;
    hipLaunchKernelGGL(k_energy_v, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, st, n, n_gamma, L, Vt);
    if (hipGetLastError() != hipSuccess) return SO_ERR_HIP;
    hipLaunchKernelGGL(k_energy_small, dim3(1), dim3(256), 0, st, n, n_gamma, L,
                       reinterpret_cast<const double2 *>(t), K2, Kt);
    if (hipGetLastError() != hipSuccess) return SO_ERR_HIP;
    if (T == 1) {
        hipLaunchKernelGGL(k_energy_shadow<1>, dim3((unsigned)S), dim3(256), 0, st, n, Ca, Vt, K2, Ms, Cr);
        hipLaunchKernelGGL(k_energy_walker<1>, dim3((unsigned)W), dim3(256), 0, st, n, eta, Xa, Xr);
    } else if (T == 2) {
        hipLaunchKernelGGL(k_energy_shadow<2>, dim3((unsigned)S), dim3(256), 0, st, n, Ca, Vt, K2, Ms, Cr);
        hipLaunchKernelGGL(k_energy_walker<2>, dim3((unsigned)W), dim3(256), 0, st, n, eta, Xa, Xr);
    } else {
        hipLaunchKernelGGL(k_energy_shadow<3>, dim3((unsigned)S), dim3(256), 0, st, n, Ca, Vt, K2, Ms, Cr);
        hipLaunchKernelGGL(k_energy_walker<3>, dim3((unsigned)W), dim3(256), 0, st, n, eta, Xa, Xr);
    }
    if (hipGetLastError() != hipSuccess) return SO_ERR_HIP;
    hipEvent_t ea = nullptr;
    if (prof_begin(st, &ea) != hipSuccess) return SO_ERR_HIP;
    const dim3 grid((unsigned)S, (unsigned)W);
    const size_t lds = energy_lds_bytes(n, eta);
    if (T == 1) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_energy_pair<1>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_energy_pair<1>, grid, dim3(SO_EN_THREADS), lds, st, n, eta, Xr, Cr, Ms, Vt, Kt, tab, S,
                           op, ep, wst);
    } else if (T == 2) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_energy_pair<2>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_energy_pair<2>, grid, dim3(SO_EN_THREADS), lds, st, n, eta, Xr, Cr, Ms, Vt, Kt, tab, S,
                           op, ep, wst);
    } else {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_energy_pair<3>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_energy_pair<3>, grid, dim3(SO_EN_THREADS), lds, st, n, eta, Xr, Cr, Ms, Vt, Kt, tab, S,
                           op, ep, wst);
    }
    if (hipGetLastError() != hipSuccess) return SO_ERR_HIP;
    if (prof_end(st, ea, PROF_ENERGY, W * S) != hipSuccess) return SO_ERR_HIP;
    hipLaunchKernelGGL(k_energy_reduce, dim3((unsigned)W), dim3(256), 0, st, S, op, ep,
                       reinterpret_cast<double2 *>(overlap), reinterpret_cast<double2 *>(numerator),
                       reinterpret_cast<double2 *>(energy), wst, static_cast<const double2 *>(Ld),
                       (pair_overlap || pair_numerator) ? 1 : 0);
    return hipGetLastError() == hipSuccess ? SO_OK : SO_ERR_HIP;
}

so_status so_batch_workspace_size(const so_problem *probs, int n_probs, size_t *bytes) {
    if (!probs || !bytes || n_probs < 1 || n_probs > kBatchMax) return SO_ERR_ARG;
    for (int k = 0; k < n_probs; ++k) {
        if (!problem_ok(probs[k])) return SO_ERR_ARG;
        if (!so_supported(probs[k].params.n, probs[k].params.eta)) return SO_ERR_UNSUPPORTED;
    }
    size_t offs[kBatchMax + 1];
    *bytes = batch_layout(probs, n_probs, offs);
    return SO_OK;
}

so_status shadow_overlap_batched(const so_problem *probs, int n_probs, void *workspace, size_t workspace_bytes,
                                 void *stream) {
    size_t need = 0;
    so_status sv = so_batch_workspace_size(probs, n_probs, &need);
    if (sv != SO_OK) return sv;
    if (!workspace || workspace_bytes < need) return SO_ERR_WORKSPACE;
    size_t offs[kBatchMax + 1];
    batch_layout(probs, n_probs, offs);
    char *ws = static_cast<char *>(workspace);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    ProbPlan plans[kBatchMax];
    for (int k = 0; k < n_probs; ++k) {
        const so_problem &pr = probs[k];
        sv = plan_problem(&pr.params, pr.phi, pr.n_walkers, pr.Q, pr.bits, pr.n_shadows, pr.overlap, pr.pair_out,
                          pr.status, ws + offs[k], offs[k + 1] - offs[k], &plans[k]);
        if (sv != SO_OK) return sv;
    }
    for (int k = 0; k < n_probs; ++k)
        if (enqueue_prep(plans[k], st) != hipSuccess) return SO_ERR_HIP;
    // fused problems in longest-processing-time order, one launch
    // per formation precision
    int order[kBatchMax], nf = 0;
    double cost[kBatchMax];
    for (int k = 0; k < n_probs; ++k)
        if (fused_ok(plans[k].n, plans[k].eta)) {
            cost[k] = pair_cost(plans[k].n, plans[k].eta) * (double)plans[k].W * (double)plans[k].S;
            order[nf++] = k;
        }
    for (int a = 1; a < nf; ++a)
        for (int b = a; b > 0 && cost[order[b]] > cost[order[b - 1]]; --b) std::swap(order[b], order[b - 1]);
    // one launch per formation precision, or, with SO_FLAG_BATCH_BY_LEVEL, one
    // per precision and register level (pair_class_level)
    bool by_level = false;
    for (int k = 0; k < n_probs; ++k) by_level = by_level || (probs[k].params.flags & SO_FLAG_BATCH_BY_LEVEL);
    for (int prec = 0; prec < 2; ++prec)
    for (int lev = 0; lev < (by_level ? 3 : 1); ++lev) {
        int ix[kBatchMax], nj = 0, wpc = 0;
        for (int a = 0; a < nf; ++a)
            if (plans[order[a]].mix == (prec == 1) &&
                (!by_level || pair_class_level(so_tiles(plans[order[a]].n), plans[order[a]].n - plans[order[a]].eta,
                                               plans[order[a]].mix) == lev)) {
                ix[nj++] = order[a];
                if (probs[order[a]].waves_per_cu > wpc) wpc = probs[order[a]].waves_per_cu;
            }
        if (!nj) continue;
        const BatchRegion rg = batch_region(ws + offs[n_probs] + (size_t)prec * batch_region_bytes());
        if (launch_batch(plans, probs, ix, nj, 0, wpc, kBatchRounds, rg, st) != hipSuccess) return SO_ERR_HIP;
    }
    for (int k = 0; k < n_probs; ++k)
        if (!fused_ok(plans[k].n, plans[k].eta) && enqueue_two_kernel(plans[k], st) != hipSuccess) return SO_ERR_HIP;
    for (int k = 0; k < n_probs; ++k)
        if (enqueue_finish(plans[k], st) != hipSuccess) return SO_ERR_HIP;
    return SO_OK;
}

so_status so_autotune(so_problem *prob, void *workspace, size_t workspace_bytes, void *stream) {
    if (!prob) return SO_ERR_ARG;
    size_t need = 0;
    so_status sv = so_batch_workspace_size(prob, 1, &need);
    if (sv != SO_OK) return sv;
    if (!workspace || workspace_bytes < need) return SO_ERR_WORKSPACE;
    size_t offs[2];
    batch_layout(prob, 1, offs);
    char *ws = static_cast<char *>(workspace);
    const BatchRegion rg = batch_region(ws + offs[1]);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    ProbPlan P;
    // pair values go to the workspace: the caller's outputs are not touched
    sv = plan_problem(&prob->params, prob->phi, prob->n_walkers, prob->Q, prob->bits, prob->n_shadows,
                      prob->overlap, nullptr, nullptr, ws, offs[1], &P);
    if (sv != SO_OK) return sv;
    if (!fused_ok(P.n, P.eta)) {
        prob->shadows_per_item = 0;
        prob->waves_per_cu = 0;
        return SO_OK;
    }
    if (enqueue_prep(P, st) != hipSuccess) return SO_ERR_HIP;
    const int nb = node_batch(P.n - P.eta);
    // a sample of about 2^21 pairs: enough to fill the machine for a few ms
    int64_t Ss = ((int64_t)1 << 21) / P.W;
    if (Ss < 8 * nb) Ss = 8 * nb;
    if (Ss > P.S) Ss = P.S;
    const int mults[5] = {1, 2, 4, 8, 16};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SO_ERR_HIP;
    float best = 1e30f;
    int best_spw = nb * kPairBatchesPerWave;
    so_problem trial = *prob;
    const int ix[1] = {0};
    for (int mi = 0; mi < 5; ++mi) {
        trial.shadows_per_item = nb * mults[mi];
        float tmin = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
            if (hipEventRecord(e0, st) != hipSuccess) return SO_ERR_HIP;
            if (launch_batch(&P, &trial, ix, 1, Ss, 0, 1, rg, st) != hipSuccess) return SO_ERR_HIP;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return SO_ERR_HIP;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return SO_ERR_HIP;
            if (ms < tmin) tmin = ms;
        }
        if (tmin < best) {
            best = tmin;
            best_spw = trial.shadows_per_item;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    prob->shadows_per_item = best_spw;
    prob->waves_per_cu = 0;
    return SO_OK;
}

so_status so_fallback_count(const so_params *p, int64_t n_walkers, int64_t n_shadows, const void *workspace,
                            size_t workspace_bytes, int64_t *count, void *stream) {
    int K;
    if (!count || !params_ok(p, &K) || n_walkers < 1 || n_shadows < 1) return SO_ERR_ARG;
    if (!so_supported(p->n, p->eta)) return SO_ERR_UNSUPPORTED;
    const Layout L = make_layout(p->n, p->eta, n_walkers, n_shadows, false, p->precision == SO_PREC_MIXED);
    if (!workspace || workspace_bytes < L.total) return SO_ERR_WORKSPACE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    so_u64 v = 0;
    if (hipMemcpyAsync(&v, static_cast<const char *>(workspace) + L.off_fbc, sizeof(v), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return SO_ERR_HIP;
    *count = (int64_t)v;
    return SO_OK;
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
