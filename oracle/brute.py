"""Dense 2^n brute force of the matchgate-shadow overlap estimator.

TEST INFRASTRUCTURE ONLY (see the ``oracle`` package docstring).

This is the plain definition, written out with no Pfaffians and no Wick
contractions, for n <= 8:

* Majorana operators by Jordan-Wigner, gamma_{2j-1} = a_j + a_j^dag and
  gamma_{2j} = -i (a_j - a_j^dag) (Supp. "Reduced Density Matrices"), mode 1
  the most significant qubit.
* The Gaussian unitary of a shadow, U_Q = exp(1/4 sum h_{mu nu} gamma_mu
  gamma_nu) with Q = exp(h), satisfies U_Q^dag gamma_mu U_Q = sum_nu Q_{mu nu}
  gamma_nu; the snapshot is sigma = U_Q^dag |b><b| U_Q (its covariance is
  Q^T C_b Q, the product in eq. b_mat).
* The inverse matchgate channel multiplies the grade-2x Majorana components of
  sigma by C(2N,2x)/C(N,x) (the factors of the estimator o_p):
  rho_hat = sum_S mu_{|S|/2} 2^{-n} Tr(gamma_S^dag sigma) gamma_S.
* For |Psi> = (|0> + |Psi_T>)/sqrt2 (section "Classical shadows and the
  evaluation of overlaps"), <Psi_T|phi> = 2 <0|rho|phi>, so a single shadow
  gives the estimate o = 2 <0|rho_hat|phi>.
"""
from __future__ import annotations

from math import comb

import numpy as np
import scipy.linalg as sla


def _bit(x, n, j):
    return (x >> (n - 1 - j)) & 1


def majorana_action(n: int):
    """For each 0-based Majorana mu: (flip mask, phase vector ph) with
    gamma_mu |x> = ph[x] |x ^ flip>."""
    dim = 1 << n
    xs = np.arange(dim)
    out = []
    for j in range(n):
        parity = np.zeros(dim, dtype=np.int64)
        for k in range(j):
            parity ^= (xs >> (n - 1 - k)) & 1
        sgn = 1.0 - 2.0 * parity
        occ = (xs >> (n - 1 - j)) & 1
        flip = 1 << (n - 1 - j)
        out.append((flip, sgn.astype(np.complex128)))                    # a + a^dag
        out.append((flip, 1j * (1.0 - 2.0 * occ) * sgn))                 # -i (a - a^dag)
    return out


def majoranas_dense(n: int):
    dim = 1 << n
    mats = []
    for flip, ph in majorana_action(n):
        M = np.zeros((dim, dim), np.complex128)
        M[np.arange(dim) ^ flip, np.arange(dim)] = ph
        mats.append(M)
    return mats


def annihilators_dense(n: int):
    g = majoranas_dense(n)
    return [(g[2 * j] + 1j * g[2 * j + 1]) / 2 for j in range(n)]


def slater_state(phi) -> np.ndarray:
    """|phi> = prod_j (sum_k Phi_kj a_k^dag) |0>, column 1 leftmost."""
    phi = np.asarray(phi, np.complex128)
    n, eta = phi.shape
    a = annihilators_dense(n)
    v = np.zeros(1 << n, np.complex128)
    v[0] = 1.0
    for j in reversed(range(eta)):
        v = sum(phi[k, j] * (a[k].conj().T @ v) for k in range(n))
    return v


def gaussian_unitary(Q) -> np.ndarray:
    """U_Q with U_Q^dag gamma_mu U_Q = sum_nu Q_{mu nu} gamma_nu, Q in SO(2n)."""
    Q = np.asarray(Q, np.float64)
    d = Q.shape[0]
    n = d // 2
    h = sla.logm(Q)
    h = np.real(h)
    h = (h - h.T) / 2
    g = majoranas_dense(n)
    H = sum(h[m, v] * (g[m] @ g[v]) for m in range(d) for v in range(d) if h[m, v] != 0.0) / 4
    U = sla.expm(H)
    for mu in range(d):
        lhs = U.conj().T @ g[mu] @ U
        rhs = sum(Q[mu, v] * g[v] for v in range(d))
        if not np.allclose(lhs, rhs, atol=1e-9):
            raise ValueError("U_Q does not realise Q (logarithm failed)")
    return U


def snapshot(Q, bits: int) -> np.ndarray:
    """sigma = U_Q^dag |b><b| U_Q; bit j-1 of ``bits`` is b_j."""
    Q = np.asarray(Q)
    n = Q.shape[0] // 2
    idx = sum(((int(bits) >> j) & 1) << (n - 1 - j) for j in range(n))
    U = gaussian_unitary(Q)
    row = U[idx, :]
    return np.outer(row.conj(), row)


def channel_inverse_overlap(sigma, phi_vec, n: int) -> complex:
    """<0| rho_hat |phi> with rho_hat the inverse matchgate channel applied to
    sigma, enumerating every even Majorana monomial gamma_S (4^n/2 of them)."""
    dim = 1 << n
    xs = np.arange(dim)
    act = majorana_action(n)
    mu_fac = [comb(2 * n, 2 * r) / comb(n, r) for r in range(n + 1)]
    total = 0.0 + 0.0j
    # depth-first over subsets S = {mu_1 < mu_2 < ...}; gamma_S = gamma_{S'} gamma_mu
    # with mu the largest element, so ph_S(x) = ph_mu(x) ph_{S'}(x ^ flip_mu).
    stack = [(0, np.ones(dim, np.complex128), 0, 0)]     # (flip, ph, size, next mu)
    while stack:
        flip, ph, size, start = stack.pop()
        if size % 2 == 0:
            coef = np.sum(np.conj(ph) * sigma[xs ^ flip, xs]) / dim
            if coef != 0 and phi_vec[flip] != 0:
                total += mu_fac[size // 2] * coef * ph[flip] * phi_vec[flip]
        for mu in range(start, 2 * n):
            f_mu, ph_mu = act[mu]
            stack.append((flip ^ f_mu, ph_mu * ph[xs ^ f_mu], size + 1, mu + 1))
    return total


def overlap_pair(phi, Q, bits: int) -> complex:
    """o = 2 <0|rho_hat|phi> for one walker and one shadow (n <= 8)."""
    phi = np.asarray(phi, np.complex128)
    n = phi.shape[0]
    return 2.0 * channel_inverse_overlap(snapshot(Q, bits), slater_state(phi), n)


def mixed_one_body(phi, Q, bits: int) -> np.ndarray:
    """N_pq = 2 <0|rho_hat a_p^dag a_q|phi> for one shadow (n <= 6)."""
    phi = np.asarray(phi, np.complex128)
    n = phi.shape[0]
    sigma = snapshot(Q, bits)
    a = annihilators_dense(n)
    v = slater_state(phi)
    N = np.zeros((n, n), np.complex128)
    for p in range(n):
        for q in range(n):
            N[p, q] = 2.0 * channel_inverse_overlap(sigma, a[p].conj().T @ (a[q] @ v), n)
    return N
