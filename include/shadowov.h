/*
 * shadowov.h -- C ABI of the MI355X (gfx950) matchgate-shadow overlap library.
 *
 * The library estimates, for every AFQMC walker Slater determinant phi_w and
 * every matchgate shadow (Q_s, b_s), the single-shadow overlap estimate
 * o_ws of <Psi_T|phi_w>, and the shadow average S_w = (1/S) sum_s o_ws
 * (Zhao et al., arXiv:2506.22408, section "Classical shadows and the
 * evaluation of overlaps": eqs. a_mat, b_mat, the interpolation of
 * Pf(A(z)) at the nodes and the estimator o_p).  It also gives the
 * holomorphic derivative d log S_w / d Phi_w and the mixed Green's function
 * G_w (section "Force bias and local energy", eqs. force_bias_diff and
 * Pfaffian_der).
 *
 * Conventions (fixed readings of the paper):
 *   - o_ws = 2 <0|rho_hat_s|phi_w>, so that S_w estimates <Psi_T|phi_w>
 *     for the measured state |Psi> = (|0> + |Psi_T>)/sqrt2; the paper's o_p
 *     omits the factor 2 (SO_FLAG_PAPER_NORM reproduces it literally);
 *   - W (not W^*) and W^T (not W^dagger) in B = W M_phi Q^T C_b Q M_phi^T W^T;
 *   - the selected rows are the first Majorana of each occupied orbital and
 *     both Majoranas of each empty orbital, in increasing order;
 *   - Majoranas gamma_{2j-1} = a_j + a_j^dag, gamma_{2j} = -i(a_j - a_j^dag);
 *     U_Q^dag gamma_mu U_Q = sum_nu Q_{mu nu} gamma_nu; bit j-1 of b_s is b_j.
 *
 * Memory: every array argument of shadow_overlap / shadow_overlap_grad is a
 * DEVICE pointer owned by the caller.  The library never allocates device
 * memory: scratch space is the caller's `workspace` (size from
 * so_workspace_size).  All work is enqueued on `stream` (a hipStream_t;
 * NULL = the default stream); the calls return without synchronising.
 * Arguments are validated on the host before anything is enqueued; a
 * failed check returns an error code and enqueues nothing.  Numerical
 * conditions are reported per walker in the optional `status` array.
 * Calls that share a workspace must not overlap in time.
 */
#ifndef SHADOWOV_H
#define SHADOWOV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Interleaved complex128 (re, im), 16 bytes. */
typedef struct {
    double re;
    double im;
} so_c64;

typedef enum {
    SO_OK = 0,
    SO_ERR_ARG = -1,         /* invalid argument: sizes, eta, null pointer, flags */
    SO_ERR_UNSUPPORTED = -2, /* (n, eta) outside the compiled kernel sizes */
    SO_ERR_HIP = -3,         /* a HIP runtime call (launch) failed */
    SO_ERR_WORKSPACE = -4    /* workspace pointer null or smaller than required */
} so_status;

/* Interpolation nodes for Pf(A(z)).  UNIT: z_k = exp(2 pi i k / K) (default;
 * a DFT, condition number 1).  CHEBYSHEV: z_k = cos((2k+1) pi / (2K)) as
 * printed in the paper (ill-conditioned for large n).  The estimator is one
 * linear functional of the coefficients of Pf(A(z)), so its value does not
 * depend on the nodes: so_node_weights gives the named family's nodes and
 * weights, while the kernels evaluate Pf(B + c J) = z^{-m/2} Pf(A(z)),
 * c = 1/z, a polynomial of degree n - eta in c, at the n - eta + 1 points
 * c_j = exp(2 pi i (j + 1/3) / (n - eta + 1)) of the unit circle (as well
 * conditioned as the roots of unity, and off +-1 and +-i, where the pair
 * matrices of signed-permutation shadows are often exactly singular). */
enum { SO_NODES_UNIT = 0, SO_NODES_CHEBYSHEV = 1 };

/* Arithmetic of the pair formation B = X C' X^T (eq. b_mat).  FP64:
 * everything in FP64.  MIXED: X_w and C'_s are rounded to single precision
 * and B is formed on the FP32 matrix cores with FP32 accumulation, then
 * widened; pivoting, the Pfaffians, the node weights and the reduction over
 * shadows stay FP64, and pairs flagged for the full-size path are redone in
 * FP64 there.  The rounding of B (relative ~1e-7) reaches o_ws amplified by
 * the conditioning of its Pfaffians: typically a few 1e-7 relative, 1e-5 for
 * the worst pairs of Haar-random shadows at n = 24, and S_w (an average over
 * shadows) within ~1e-6 of |S_w| + mean |o_ws|.  shadow_overlap and
 * shadow_overlap_batched accept both; shadow_overlap_grad only FP64
 * (SO_ERR_UNSUPPORTED otherwise).  MIXED adds 4 (W + S) DP^2 bytes of
 * workspace (DP = 16 ceil(2n / 16)). */
enum { SO_PREC_FP64 = 0, SO_PREC_MIXED = 1 };

#define SO_FLAG_PAPER_NORM 1u /* omit the factor 2 (paper's o_p as printed) */
#define SO_FLAG_LOG_OUTPUT 2u /* overlap[w] receives log S_w = log|S_w| + i Arg S_w
                                 (principal branch) instead of S_w; S_w == 0 sets
                                 SO_WSTAT_ZERO.  shadow_overlap, shadow_overlap_grad,
                                 shadow_overlap_batched, so_vce_overlap */
#define SO_FLAG_BATCH_BY_LEVEL 4u /* shadow_overlap_batched: if any problem sets it,
                                     the fused problems go in one launch per
                                     register level instead of one (ignored by
                                     the other calls) */
#define SO_FLAG_SIGNED_PERM 8u /* shadow_overlap: every Q_s is a signed permutation
                                  (the paper's shadow ensemble).  With FP64
                                  formation and n = 8T (n = 8, 16, 24) the pair
                                  kernel then forms U = C'X^T as a signed gather
                                  instead of a matrix product, same values bit
                                  for bit; a shadow that is not a signed
                                  permutation gives NaN pairs (its walkers get
                                  SO_WSTAT_NONFINITE).  Ignored elsewhere. */

typedef struct {
    int n;          /* modes = qubits = spin orbitals; see so_max_n() */
    int eta;        /* electrons in the walkers: even, 2 <= eta <= n */
    int n_nodes;    /* K interpolation nodes; 0 means n + 1; must be >= n - eta/2 + 1 */
    int nodes;      /* SO_NODES_UNIT or SO_NODES_CHEBYSHEV */
    int precision;  /* SO_PREC_FP64 or SO_PREC_MIXED */
    unsigned flags; /* SO_FLAG_* */
} so_params;

/* Per-walker status bits written to the optional `status` array. */
#define SO_WSTAT_RANK 1      /* Phi_w is rank-deficient: outputs for w are NaN */
#define SO_WSTAT_NONFINITE 2 /* a non-finite value reached S_w */
#define SO_WSTAT_ZERO 4      /* sum_s o_ws == 0: log and gradient undefined (NaN) */
#define SO_WSTAT_FALLBACK_LOST 8 /* reserved, never set: every pair that the
                                    elimination flags reaches the full-size path
                                    (through its queue, or through a scan of the
                                    pair values when the queue is full) */
#define SO_WSTAT_SINGULAR 16 /* shadow_overlap_grad: a node matrix B + c J of some
                                pair was exactly singular, where the derivative by
                                inverses is undefined: dlog and green for w are
                                not reliable */

/* Largest supported n (and the supported (n, eta) pairs are those with
 * m = 2n - eta in the compiled set; see so_supported). */
int so_max_n(void);

/* 1 if kernels are compiled for (n, eta), else 0.  Host only. */
int so_supported(int n, int eta);

/* Bytes of device workspace needed by one call with these sizes.
 * with_grad: 0 for shadow_overlap, 1 for shadow_overlap_grad.
 * Host only; returns SO_ERR_ARG / SO_ERR_UNSUPPORTED on bad parameters. */
so_status so_workspace_size(const so_params *p, int64_t n_walkers, int64_t n_shadows,
                            int with_grad, size_t *bytes);

/* Host copies of the K nodes z_k and weights w_k that the kernels use, with
 * o = sum_k w_k Pf(A(z_k)) (section "Classical shadows and the evaluation of
 * overlaps": interpolation at the nodes, then the estimator o_p).  `nodes`
 * and `weights` are HOST arrays of at least K entries; K is returned in
 * *n_nodes.  Host only (no GPU needed). */
so_status so_node_weights(const so_params *p, so_c64 *nodes, so_c64 *weights, int *n_nodes);

/* Shadow-averaged overlaps.
 *   phi       [n_walkers][n][eta] complex128, row-major (Phi_{pj} of the walker
 *             |phi> = prod_j (sum_p Phi_pj a_p^dag)|0>, column 1 leftmost);
 *             need not be orthonormal but must have full column rank
 *   Q         [n_shadows][2n][2n] float64 row-major, each in SO(2n) (trusted)
 *   bits      [n_shadows] uint64, bit j-1 = b_j of the measured bitstring
 *   overlap   [n_walkers] complex128 out: S_w = (1/S) sum_s o_ws
 *   pair_out  [n_walkers][n_shadows] complex128 out (o_ws), or NULL
 *   status    [n_walkers] int32 out (SO_WSTAT_* bits), or NULL
 *   workspace device scratch of at least so_workspace_size(p, W, S, 0) bytes
 *   stream    hipStream_t or NULL
 * Sizes: n_walkers >= 1, n_shadows >= 1.  Deterministic: the reduction over
 * shadows has a fixed order, so repeated calls give identical bits. */
so_status shadow_overlap(const so_params *p, const so_c64 *phi, int64_t n_walkers,
                         const double *Q, const uint64_t *bits, int64_t n_shadows,
                         so_c64 *overlap, so_c64 *pair_out, int32_t *status,
                         void *workspace, size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and results as shadow_overlap (the same kernels, bit for bit),
 * with the scratch space in a library-owned static device array of
 * SO_NOALLOC_SCRATCH_BYTES per GPU instead of a caller workspace.  The
 * caller still passes the inputs and outputs (device pointers, as in
 * shadow_overlap).  No hipMalloc, hipFree or other allocating call is made;
 * the first call on a device looks up the array's device address
 * (hipGetSymbolAddress) and keeps it.  Problems whose workspace
 * (so_workspace_size with_grad = 0) exceeds the array return
 * SO_ERR_WORKSPACE before anything is enqueued; e.g. n = 16, eta = 8 fits
 * about W x S = 256 x 5,000.  Every call on one GPU uses that GPU's one
 * array, which keeps the last call's contents (the kernels clear what must
 * start at zero): calls that overlap in time on one GPU, on any streams or
 * threads, race and must be serialised by the caller. */
#define SO_NOALLOC_SCRATCH_BYTES (64u << 20)
so_status shadow_overlap_noalloc(const so_params *p, const so_c64 *phi, int64_t n_walkers,
                                 const double *Q, const uint64_t *bits, int64_t n_shadows,
                                 so_c64 *overlap, so_c64 *pair_out, int32_t *status, void *stream);

/* Overlaps and their first derivative (section "Force bias and local
 * energy": d Pf = Pf/2 Tr(A^{-1} dA), eq. Pfaffian_der, applied through
 * A(z) = C_0^(s) + z B and B(Phi)).
 *   overlap   [n_walkers] complex128 out: S_w
 *   dlog      [n_walkers][n][eta] complex128 out: D_w = d log S_w / d Phi_w,
 *             the holomorphic derivative (S_w is a polynomial in Phi_w)
 *   green     [n_walkers][n][n] complex128 out, or NULL: mixed Green's function
 *             G_pq = <Psi_T|a_p^dag a_q|phi>/<Psi_T|phi> = (D_w Phi_w^T)_pq
 *   other arguments as in shadow_overlap (workspace from with_grad = 1).
 * Walkers with S_w == 0 get SO_WSTAT_ZERO and NaN derivatives.  The pairs are
 * evaluated at each walker's orthonormal factor Q_w (Phi_w = Q_w R_w, a
 * Householder QR) and carried back: S_w = det R_w S(Q_w), D_w = D(Q_w) R_w^{-T},
 * G_w = G(Q_w); so walkers of any norm a double holds keep full accuracy, and
 * with SO_FLAG_LOG_OUTPUT log S_w stays finite where S_w itself is not.
 * Supported shapes: n - eta even with 2 <= n - eta <= 8 and n <= 16 (the
 * paper's N = 16, eta = 8 included); others return SO_ERR_UNSUPPORTED.
 * Deterministic (fixed reduction order). */
so_status shadow_overlap_grad(const so_params *p, const so_c64 *phi, int64_t n_walkers,
                              const double *Q, const uint64_t *bits, int64_t n_shadows,
                              so_c64 *overlap, so_c64 *dlog, so_c64 *green, int32_t *status,
                              void *workspace, size_t workspace_bytes, void *stream);

/* One problem of a batch: the arguments of shadow_overlap, plus two tuning
 * knobs for problems on the fused pair kernel (n - eta even, 2..12):
 *   shadows_per_item  shadows per work item (one workgroup) of the batch
 *                     launch (rounded up to a multiple of the node batch
 *                     64/(ne+1)); 0 = library default
 *   waves_per_cu      reserved (the hardware dispatcher schedules the items);
 *                     so_autotune writes 0
 * so_autotune fills both. */
typedef struct {
    so_params params;
    const so_c64 *phi;
    int64_t n_walkers;
    const double *Q;
    const uint64_t *bits;
    int64_t n_shadows;
    so_c64 *overlap;
    so_c64 *pair_out;
    int32_t *status;
    int shadows_per_item;
    int waves_per_cu;
} so_problem;

/* Workspace bytes for shadow_overlap_batched over these problems (1..16). */
so_status so_batch_workspace_size(const so_problem *probs, int n_probs, size_t *bytes);

/* Several independent problems -- e.g. walker and shadow sets of several
 * geometries with different orbital counts -- in one call: the overlaps of
 * shadow_overlap for each, bit for bit the same values.  All problems on the
 * fused pair kernel with one formation precision share ONE launch, whatever
 * their (n, eta): its workgroups take work items (walker, shadow range) of
 * every problem, the costliest problem first, with the items of walkers
 * w = x (mod 8) on XCD x of the MI355X so that each XCD keeps its walkers'
 * matrices in its L2.  Problems of other shapes use the two-kernel path
 * inside the same call.  The one launch runs every class at the register
 * allocation of the heaviest, so light classes lose occupancy: on the paper's
 * four reaction-path geometries (n = 8..20) it takes 386 ms against 359 ms as
 * separate calls.  With SO_FLAG_BATCH_BY_LEVEL the problems go instead in one
 * launch per register level (two there, 368 ms); the values are the same bits
 * either way.  Everything is enqueued on `stream` with no
 * allocation, no memset and no host synchronisation, so the call may be
 * captured into a hipGraph and replayed (the workspace and outputs must then
 * stay fixed). */
so_status shadow_overlap_batched(const so_problem *probs, int n_probs, void *workspace, size_t workspace_bytes,
                                 void *stream);

/* Autotuner: times the batch launch of this problem alone on a sample of its
 * own inputs (about 2^21 pairs) over shadows_per_item in {1, 2, 4, 8, 16}
 * node batches, and writes the fastest into *prob (zeros for problems on the
 * two-kernel path).  Synchronises the stream (not capturable); the caller's
 * outputs are not written.  Workspace: so_batch_workspace_size(prob, 1). */
so_status so_autotune(so_problem *prob, void *workspace, size_t workspace_bytes, void *stream);

/* One-particle reduced density matrix from the shadows (Supp. "Reduced
 * Density Matrices": eq. local_fermionic_ob_exp for a product of two
 * Majoranas, whose channel factor is C(2n,2)/C(n,1) = 2n - 1, and eqs.
 * majorana_op, 1rdm_off_diagonal, 1rdm_diagonal for the fermionic elements).
 *   n          modes, 2 <= n <= so_max_n()
 *   Q, bits    [n_shadows][2n][2n] float64 and [n_shadows] uint64 (device),
 *              as in shadow_overlap
 *   trial      0: the matrix of the measured state; 1: of the trial state
 *              when the shadows are of (|0> + |Psi_T>)/sqrt2 (twice the
 *              measured state's: a number-conserving operator has no vacuum
 *              or cross term)
 *   rdm        [n][n] complex128 out (device): rdm[p][q] = <a_p^dag a_q>,
 *              modes 0-based (mode p <-> Majoranas 2p, 2p+1); its trace is the
 *              particle number
 *   majorana   [2n][2n] float64 out (device) or NULL: M[mu][nu] =
 *              (2n - 1)/S sum_s C'_s[mu][nu], the estimate of -i<gamma_mu gamma_nu>
 *              (mu != nu), zero diagonal
 *   workspace  so_rdm1_workspace_size(n, n_shadows) bytes (device)
 * Deterministic (fixed reduction order); enqueued on `stream`; no
 * allocation or host synchronisation. */
so_status so_rdm1_workspace_size(int n, int64_t n_shadows, size_t *bytes);
so_status so_rdm1(int n, const double *Q, const uint64_t *bits, int64_t n_shadows, int trial, so_c64 *rdm,
                  double *majorana, void *workspace, size_t workspace_bytes, void *stream);

/* Virtual correlation energy (section "Virtual correlation energy", eq.
 * vce_overlap; Supp. "Virtual Correlation Energy Derivation"): overlaps of
 * full-space walkers with the trial state |Xi_c^a Xi_c^b> (x) |Psi_T,a> (x)
 * |0_v>, whose frozen core fills spatial orbitals 0..n_core-1 of each spin,
 * whose active part |Psi_T,a> (the state the shadows are of) lives on the
 * active orbitals n_core..n_core+n_active-1, and whose virtual orbitals
 * (the rest of the n_basis) are empty.  The 2 n_active active modes are
 * ordered alpha orbitals first, then beta; the trial state's creation order
 * is core alpha, core beta, active alpha, active beta, as in the paper's
 * first determinant. */
typedef struct {
    int n_basis;   /* N_B spatial orbitals of the full space */
    int n_core;    /* frozen doubly occupied core orbitals, >= 0 */
    int n_active;  /* active spatial orbitals, 1..12 (n = 2 n_active modes) */
    int n_alpha;   /* active alpha electrons, 0..n_active */
    int n_beta;    /* active beta electrons, 0..n_active (n_alpha + n_beta >= 1) */
} so_vce_dims;

/* The per-walker prologue: from the full-space walker (alpha and beta
 * orbital blocks) to the active-space walker phi~_a and the prefactor c_w
 * with <Psi_T|phi_w> = c_w <Psi_T,a|phi~_a,w>.  The paper's c_w is
 * det(Sigma^a) det(Sigma^b) det(R^a) det(R^b) / (det(U^dag) det(V)), from
 * an SVD of each spin's core rows and a QR of its projected active rows;
 * the kernel gets the same value from Householder reflections (an LQ
 * factorisation of the core rows, then a QR), one wave per walker.
 *   phi_alpha  [n_walkers][n_basis][n_core + n_alpha] complex128 (device),
 *              row-major: orbital coefficients, core rows first
 *   phi_beta   [n_walkers][n_basis][n_core + n_beta]  complex128 (device)
 *   active_phi [n_walkers][2 n_active][n_alpha + n_beta] complex128 out
 *              (device): diag(Q^a, Q^b), orthonormal columns, alpha first
 *   prefactor  [n_walkers] complex128 out (device)
 * Only the core and active rows are read.  A core block (or projected
 * active block) with an exactly zero row (column) norm gives c_w = 0 and
 * an orthonormal phi~_a; non-finite inputs propagate.  Limits: the matrices
 * of one spin, (n_core + n_active)(n_core + max(n_alpha, n_beta)) complex
 * entries plus the reflectors, fit 64 KiB of LDS (n_core <= 57 at the
 * paper's (8e, 8o)); otherwise SO_ERR_ARG.  Enqueued on `stream`; no
 * allocation. */
so_status so_vce_walkers(const so_vce_dims *dims, const so_c64 *phi_alpha, const so_c64 *phi_beta,
                         int64_t n_walkers, so_c64 *active_phi, so_c64 *prefactor, void *stream);

/* Workspace of so_vce_overlap: that of shadow_overlap for (n, eta) =
 * (2 n_active, n_alpha + n_beta), plus the active walkers and prefactors. */
so_status so_vce_workspace_size(const so_params *p, const so_vce_dims *dims, int64_t n_walkers,
                                int64_t n_shadows, size_t *bytes);

/* Full-space overlaps: the prologue above, shadow_overlap on the active
 * walkers (p->n must be 2 n_active and p->eta n_alpha + n_beta), then
 * overlap[w] = c_w S_w.  prefactor [n_walkers] (device) receives c_w, or
 * NULL; status as in shadow_overlap.  All arguments are checked before
 * anything is enqueued. */
so_status so_vce_overlap(const so_params *p, const so_vce_dims *dims, const so_c64 *phi_alpha,
                         const so_c64 *phi_beta, int64_t n_walkers, const double *Q, const uint64_t *bits,
                         int64_t n_shadows, so_c64 *overlap, so_c64 *prefactor, int32_t *status,
                         void *workspace, size_t workspace_bytes, void *stream);

/* Local energy E_L = <Psi_T|H|phi_w> / <Psi_T|phi_w> (section "Force bias
 * and local energy": eqs. local_energy, ham_cholesky_decom, energy_tb_diff,
 * Pfaffian_der, Pfaffian_2nd_der) for
 *   H = sum_pq t_pq a_p^dag a_q + 1/2 sum_g Lhat_g^2,  Lhat_g = sum_pq L^g_pq a_p^dag a_q
 * (the paper's H = v_0 - 1/2 sum_g v_g^2 with v_g = i Lhat_g), from the
 * first and second derivatives of the node Pfaffians as the walker moves
 * along e^{lambda Lhat}.  The node matrices must be invertible, and
 * z = -1 is a root of every pair's Pfaffian when n - eta is odd; this entry
 * point therefore uses its own nodes, whatever p->nodes and p->n_nodes say:
 * Pf(C_0 + z B) = z^{eta/2} R(z) with deg R = n - eta for every walker along
 * e^{lambda Lhat}, so n - eta + 1 nodes z_k = exp(2 pi i (k + 1/3) /
 * (n - eta + 1)), which avoid +-1 and +-i, determine the estimator and its
 * derivatives.
 *   phi, Q, bits  as in shadow_overlap (device)
 *   t        [n][n] complex128 (device), any one-body matrix
 *   L        [n*n][n_gamma] float64 (device), L[p n + q][g] = L^g_pq, each L^g
 *            real symmetric (the kernel relies on it); NULL if n_gamma = 0
 *   overlap  [n_walkers] complex128 out (device) or NULL: S_w
 *   numerator [n_walkers] complex128 out or NULL: the shadow estimate of
 *            <Psi_T|H|phi_w>, N_w = (1/S) sum_s e_ws
 *   energy   [n_walkers] complex128 out or NULL: N_w / S_w
 *   pair_overlap, pair_numerator  [n_walkers][n_shadows] complex128 out or
 *            NULL: the single-shadow terms o_ws and e_ws of those averages
 *   status   [n_walkers] int32 out or NULL: SO_WSTAT_RANK (S_w, N_w, E_w
 *            are then NaN) / _NONFINITE, and SO_WSTAT_SINGULAR if a node
 *            matrix of some pair was exactly singular (the energy of that
 *            pair is undefined: N_w and E_w are then NaN, S_w is kept)
 * The pairs are evaluated at each walker's orthonormal factor Q_w (Phi_w =
 * Q_w R_w, a Householder QR) and S_w, N_w and the single-shadow terms are
 * multiplied by det R_w; E_w, which does not depend on it, is taken before,
 * so it stays finite for walkers whose S_w and N_w leave the double range
 * (those are flagged SO_WSTAT_NONFINITE).
 * Supported: n <= 24, FP64 (SO_ERR_UNSUPPORTED otherwise); n_walkers <=
 * 65535.  One 256-thread workgroup per pair; deterministic (fixed
 * reduction order); no allocation; enqueued on `stream`. */
so_status so_local_energy_workspace_size(const so_params *p, int64_t n_walkers, int64_t n_shadows, int n_gamma,
                                         size_t *bytes);
so_status so_local_energy(const so_params *p, const so_c64 *phi, int64_t n_walkers, const double *Q,
                          const uint64_t *bits, int64_t n_shadows, const so_c64 *t, const double *L, int n_gamma,
                          so_c64 *overlap, so_c64 *numerator, so_c64 *energy, so_c64 *pair_overlap,
                          so_c64 *pair_numerator, int32_t *status, void *workspace, size_t workspace_bytes,
                          void *stream);

/* Force bias of every walker ("Force bias and local energy", eq. force_bias,
 * with the Cholesky vectors L^gamma of eq. cholesky_vec):
 *   xbar[w][gamma] = -sqrt(dt) i sum_pq L[p n + q][gamma] G_w[p][q].
 *   green   [n_walkers][n][n] complex128 (device), e.g. from shadow_overlap_grad
 *   L       [n n][n_gamma] float64 (device), real
 *   xbar    [n_walkers][n_gamma] complex128 out (device)
 * n <= 32, dt >= 0.  Enqueued on `stream`; the caller owns all memory. */
so_status so_force_bias(const so_c64 *green, int64_t n_walkers, int n, const double *L, int64_t n_gamma,
                        double dt, so_c64 *xbar, void *stream);

/* Diagnostics: the number of walker x shadow pairs that the last
 * shadow_overlap call with these arguments and this workspace sent to the
 * full-size path (the elimination of B_KK met a zero pivot or growth beyond
 * its bound; such pairs are evaluated as Pf(B + c J) at the full size, which
 * needs no block of B to be invertible).  Synchronises `stream`, then copies
 * the counter from the workspace.  Host; SO_ERR_ARG / _UNSUPPORTED /
 * _WORKSPACE as for so_workspace_size and a too small workspace. */
so_status so_fallback_count(const so_params *p, int64_t n_walkers, int64_t n_shadows, const void *workspace,
                            size_t workspace_bytes, int64_t *count, void *stream);

/* Kernel timing for benchmarks (not for the hot path of an application).
 * so_profile_enable(1) makes every later shadow_overlap call bracket each
 * launch of its node-Pfaffian kernel (kind 0), of its formation kernel
 * (kind 1) and of its fused pair kernel (kind 2; formation, elimination and
 * node Pfaffians in one launch, used when n - eta is even, 2..12), and
 * every shadow_overlap_grad call its per-pair adjoint kernel (kind 3), with
 * HIP events recorded on the call's stream.  so_profile_read
 * waits for the recorded events of one kind, returns their summed duration
 * in milliseconds, the number of launches and the number of walker x shadow
 * pairs those launches processed, and forgets them.  Kind 4 is so_rdm1's
 * contraction kernel (units: shadows), kind 5 the VCE prologue kernel
 * (units: walkers) and kind 6 so_local_energy's pair kernel (units: pairs).  Host only; events are
 * created with hipEventCreate while enabled. */
so_status so_profile_enable(int on);
so_status so_profile_read(int kind, double *ms, int64_t *launches, int64_t *pairs);

/* Static description of a status code. */
const char *so_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* SHADOWOV_H */
