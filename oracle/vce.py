"""Virtual correlation energy (VCE): the full-space overlap from the active one.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; see ``oracle/__init__.py``).

Follows Supp. "Virtual Correlation Energy Derivation" and eq. vce_overlap of
section "Virtual correlation energy", step by step.  The trial state is
|Xi_c^a> (x) |Xi_c^b> (x) |Psi_T,a> (x) |0_v^a> (x) |0_v^b>.  Its core
determinants fill spatial orbitals 0..N_c-1 of each spin, the active space is
orbitals N_c..N_c+N_a-1, and the rest are virtual.  For a full-space walker
with alpha orbitals phi^a [N_B, N_c + n_alpha] and beta orbitals
phi^b [N_B, N_c + n_beta]:

* Xi_c^dag phi_c, the core rows of phi, has the SVD U_c Sigma_c V_c^dag
  (full SVD: V = [V_c, V_c'] square unitary);
* phi_a V_c' = Q R (QR), and the active walker of that spin is Q;
* U = diag(U_c^a, U_c^b, I, I) and V = [[V_c^a, 0, V_c^a', 0],
  [0, V_c^b, 0, V_c^b']] are the paper's block matrices, column order
  included;
* <Psi_T|phi> = det(Sigma^a) det(Sigma^b) det(R^a) det(R^b)
  <Psi_T,a|phi~_a> / (det(U^dag) det(V)).

The active walker phi~_a is the 2 N_a x (n_alpha + n_beta) matrix
diag(Q^a, Q^b).  Its modes are alpha orbitals 0..N_a-1, then beta orbitals
N_a..2N_a-1, and its columns list the alpha electrons first.  The sign
convention is that of the paper's first determinant: its rows are ordered
(Xi^a, Xi^b, chi^a, chi^b) and its columns (phi^a, phi^b).
"""
from __future__ import annotations

import numpy as np


def _spin_factor(phi, n_core: int, n_active: int):
    """One spin: (U_c, Sigma_c, V, Q, R) of the derivation, V = [V_c, V_c']."""
    phi = np.asarray(phi, np.complex128)
    ne = phi.shape[1]
    core = phi[:n_core, :]                          # Xi_c^dag phi_c
    act = phi[n_core:n_core + n_active, :]          # phi_a
    if n_core > 0:
        Uc, sig, Vh = np.linalg.svd(core, full_matrices=True)
        V = Vh.conj().T
    else:
        Uc, sig, V = np.zeros((0, 0), np.complex128), np.zeros(0), np.eye(ne, dtype=np.complex128)
    Vp = V[:, n_core:]                              # V_c': the added orthonormal columns
    Q, R = np.linalg.qr(act @ Vp)                   # phi_a V_c' = Q R
    return Uc, sig, V, Q, R


def active_walker(phi_alpha, phi_beta, n_core: int, n_active: int):
    """(phi~_a [2 N_a, n_alpha + n_beta], prefactor) for one full-space walker,
    where prefactor = det(Sigma^a) det(Sigma^b) det(R^a) det(R^b) /
    (det(U^dag) det(V)), so that <Psi_T|phi> = prefactor <Psi_T,a|phi~_a>."""
    na_ = np.asarray(phi_alpha).shape[1] - n_core
    nb_ = np.asarray(phi_beta).shape[1] - n_core
    Uca, siga, Va, Qa, Ra = _spin_factor(phi_alpha, n_core, n_active)
    Ucb, sigb, Vb, Qb, Rb = _spin_factor(phi_beta, n_core, n_active)
    # U = diag(U_c^a, U_c^b, I, I): det(U^dag) = conj(det U_c^a) conj(det U_c^b)
    det_Udag = np.conj(np.linalg.det(Uca) if n_core else 1.0) * np.conj(np.linalg.det(Ucb) if n_core else 1.0)
    # V in the paper's column order (V_c^a, V_c^b, V_c^a', V_c^b')
    ea, eb = n_core + na_, n_core + nb_
    Vfull = np.zeros((ea + eb, ea + eb), np.complex128)
    Vfull[:ea, :n_core] = Va[:, :n_core]
    Vfull[ea:, n_core:2 * n_core] = Vb[:, :n_core]
    Vfull[:ea, 2 * n_core:2 * n_core + na_] = Va[:, n_core:]
    Vfull[ea:, 2 * n_core + na_:] = Vb[:, n_core:]
    pref = (np.prod(siga) * np.prod(sigb) * np.linalg.det(Ra) * np.linalg.det(Rb)
            / (det_Udag * np.linalg.det(Vfull)))
    act = np.zeros((2 * n_active, na_ + nb_), np.complex128)
    act[:n_active, :na_] = Qa
    act[n_active:, na_:] = Qb
    return act, complex(pref)


def active_walkers(phi_alpha, phi_beta, n_core: int, n_active: int):
    """Batched :func:`active_walker`: phi_alpha [W, N_B, N_c + n_alpha],
    phi_beta [W, N_B, N_c + n_beta] -> (phi~_a [W, 2 N_a, eta], prefactor [W])."""
    phi_alpha = np.asarray(phi_alpha, np.complex128)
    phi_beta = np.asarray(phi_beta, np.complex128)
    outs = [active_walker(phi_alpha[w], phi_beta[w], n_core, n_active) for w in range(phi_alpha.shape[0])]
    return np.stack([o[0] for o in outs]), np.array([o[1] for o in outs], np.complex128)


def full_space_overlap(phi_alpha, phi_beta, n_core: int, n_active: int, ci):
    """The plain definition, Supp. "Virtual Correlation Energy Derivation"
    (first determinant): sum_i c_i^* det(T_i^dag Phi) over the active
    determinants i, in the full spin-orbital basis (alpha orbitals 0..N_B-1,
    then beta).  The columns of T_i are the core orbitals of each spin, then
    the occupied active orbitals of each spin, in the paper's order
    (Xi^a, Xi^b, chi^a, chi^b).  Phi = diag(phi^a, phi^b).
    ``ci`` maps (alpha occupation tuple, beta occupation tuple) of active
    orbitals (0-based within the active space) to the coefficient c_i of the
    ket |Psi_T,a>."""
    pa = np.asarray(phi_alpha, np.complex128)
    pb = np.asarray(phi_beta, np.complex128)
    NB = pa.shape[0]
    ea, eb = pa.shape[1], pb.shape[1]
    Phi = np.zeros((2 * NB, ea + eb), np.complex128)
    Phi[:NB, :ea] = pa
    Phi[NB:, ea:] = pb
    total = 0.0 + 0.0j
    for (occ_a, occ_b), c in ci.items():
        cols = ([p for p in range(n_core)] + [NB + p for p in range(n_core)]
                + [n_core + p for p in occ_a] + [NB + n_core + p for p in occ_b])
        T = np.zeros((2 * NB, len(cols)), np.complex128)
        for j, r in enumerate(cols):
            T[r, j] = 1.0
        total += np.conj(c) * np.linalg.det(T.conj().T @ Phi)
    return total


def active_space_overlap(act, n_active: int, ci):
    """<Psi_T,a|phi~_a> = sum_i c_i^* det(phi~_a[occupied rows]) with the
    active modes ordered alpha (0..N_a-1) then beta (N_a..2N_a-1)."""
    act = np.asarray(act, np.complex128)
    total = 0.0 + 0.0j
    for (occ_a, occ_b), c in ci.items():
        rows = list(occ_a) + [n_active + p for p in occ_b]
        total += np.conj(c) * np.linalg.det(act[rows, :])
    return total


def vce_overlap(phi_alpha, phi_beta, n_core: int, n_active: int, Q, bits, K=None, family="unit", nthreads=0):
    """Shadow estimate of the full-space overlap <Psi_T|phi_w> (eq. vce_overlap):
    prefactor_w times the shadow average S_w of the active walker phi~_a
    (section "Classical shadows and the evaluation of overlaps").  Returns
    (overlap [W], prefactor [W], phi~_a [W, 2 N_a, eta])."""
    from . import overlap
    act, pref = active_walkers(phi_alpha, phi_beta, n_core, n_active)
    return pref * overlap(act, Q, bits, K=K, family=family, nthreads=nthreads), pref, act
