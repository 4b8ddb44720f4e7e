"""CPU oracle for the matchgate-shadow overlap estimator (arXiv:2506.22408).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct FP64
reference that the HIP library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the product package never does, and the two share no code.

Parts
-----
* ``shadow_oracle.c`` (built to ``liboracle.so``): the Pfaffian route of the
  paper, step by step, in plain C99 ``double complex`` with OpenMP over pairs.
* :func:`node_weights`: interpolation nodes and the node weights that fold the
  polynomial interpolation, the inverse-channel factors C(2N,2x)/C(N,x) and the
  prefactor of the estimator o_p into one vector (section "Classical shadows
  and the evaluation of overlaps"), computed at 50 digits with mpmath.
* :mod:`oracle.brute`: the plain definition o = 2<0|rho_hat|phi> on dense
  2^n state vectors (n <= 8).
* :mod:`oracle.closed_form`: the exact value for signed-permutation shadows
  (a weighted sum of eta x eta minors), usable up to n ~ 20.
* :mod:`oracle.vce`: the virtual-correlation-energy prologue (full-space
  walker -> active walker and prefactor, Supp. "Virtual Correlation Energy
  Derivation") and the plain full-space determinant expansion it is pinned to.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction
from math import comb

import mpmath
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "shadow_oracle.c")
# ORACLE_SANITIZE=1 selects a build with AddressSanitizer and UBSan (run the
# process with the gcc ASan runtime preloaded; tests/test_sanitizers.py does)
_SANITIZE = os.environ.get("ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "liboracle_asan.so" if _SANITIZE else "liboracle.so")
_lib = None

NODE_FAMILIES = ("unit", "chebyshev")


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (plain -O2, no fast-math), or the
    sanitized ``liboracle_asan.so`` when ORACLE_SANITIZE=1."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        opt = (["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                "-fno-omit-frame-pointer"] if _SANITIZE else ["-O2"])
        cmd = ["gcc", "-std=c99", *opt, "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        c = ctypes
        P = c.c_void_p
        lib.or_pfaffian.argtypes = [c.c_int, P, P]
        lib.or_covariance.argtypes = [c.c_int, P, c.c_uint64, P]
        lib.or_covariance.restype = None
        lib.or_complement.argtypes = [c.c_int, c.c_int, P, P]
        lib.or_xmatrix.argtypes = [c.c_int, c.c_int, P, P, P, P]
        lib.or_pair_perp.argtypes = [c.c_int, c.c_int, c.c_int, P, P, P, P, P, c.c_uint64, P, P]
        lib.or_pair.argtypes = [c.c_int, c.c_int, c.c_int, P, P, P, P, c.c_uint64, P, P]
        lib.or_overlap_pairs.argtypes = [c.c_int, c.c_int, c.c_int, P, P, P, c.c_long, P, P, c.c_long,
                                         P, P, c.c_long, P, P, P, c.c_int]
        lib.or_pair_grad.argtypes = [c.c_int, c.c_int, c.c_int, P, P, P, P, c.c_uint64, P, P]
        lib.or_grad_walkers.argtypes = [c.c_int, c.c_int, c.c_int, P, P, P, c.c_long, P, P, c.c_long,
                                        P, P, P, c.c_int]
        lib.or_kmatrix.argtypes = [c.c_int, P, P]
        lib.or_kmatrix.restype = None
        lib.or_energy_pairs.argtypes = [c.c_int, c.c_int, c.c_int, P, P, P, c.c_long, P, P, c.c_long,
                                        P, P, c.c_long, P, P, c.c_int, P, P, P, c.c_int]
        for f in ("or_pfaffian", "or_complement", "or_xmatrix", "or_pair_perp", "or_pair",
                  "or_overlap_pairs", "or_pair_grad", "or_grad_walkers", "or_energy_pairs"):
            getattr(lib, f).restype = c.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# node weights
# --------------------------------------------------------------------------
def channel_factor(n: int, x: int) -> Fraction:
    """Inverse matchgate-channel factor C(2N,2x)/C(N,x) of the estimator o_p."""
    return Fraction(comb(2 * n, 2 * x), comb(n, x))


def node_weights(n: int, eta: int, K: int | None = None, family: str = "unit"):
    """Nodes z_k and weights w_k with o = sum_k w_k Pf(A(z_k)).

    The Pfaffian Pf(A(z)) = sum_x c_x z^x is a polynomial of degree
    l = N - floor(eta/2); o = i^{eta/2} / 2^{N - eta/2} * 2 * sum_{x<=l} c_x
    C(2N,2x)/C(N,x) (estimator o_p, with the factor 2 that turns
    <0|rho_hat|phi> into <Psi_T|phi> for |Psi> = (|0> + |Psi_T>)/sqrt2).
    The coefficients come from interpolation at the nodes, so the whole map
    p -> o is one linear functional w.

    family "unit": z_k = exp(2 pi i k/K); interpolation is a DFT.
    family "chebyshev": z_k = cos((2k+1) pi / (2K)) as printed in the paper;
    the Vandermonde system is solved at 50 digits.
    The weights are exact (to 50 digits) for the FP64-rounded nodes.
    """
    if eta < 1 or eta % 2 or eta > n:
        raise ValueError("eta must be even with 2 <= eta <= n")
    ell = n - eta // 2
    if K is None:
        K = n + 1
    if K < ell + 1:
        raise ValueError(f"need at least {ell + 1} nodes")
    with mpmath.workdps(60):
        pref = 2 * mpmath.mpc(0, 1) ** (eta // 2) / mpmath.mpf(2) ** (n - eta // 2)
        mu = [mpmath.mpf(channel_factor(n, x).numerator) / channel_factor(n, x).denominator
              if x <= ell else mpmath.mpf(0) for x in range(K)]
        if family == "unit":
            zs = [mpmath.exp(2j * mpmath.pi * k / K) for k in range(K)]
        elif family == "chebyshev":
            zs = [mpmath.cos((2 * k + 1) * mpmath.pi / (2 * K)) for k in range(K)]
        else:
            raise ValueError(f"unknown node family {family!r}")
        zr = [complex(z) for z in zs]          # the FP64 nodes actually used
        zm = [mpmath.mpc(z.real, z.imag) for z in zr]
        # w = pref * V^{-T} mu with V_{kx} = z_k^x
        VT = mpmath.matrix(K, K)
        for k in range(K):
            for x in range(K):
                VT[x, k] = zm[k] ** x
        w = mpmath.lu_solve(VT, mpmath.matrix(mu))
        wts = [complex(pref * w[k]) for k in range(K)]
    return np.array(zr, dtype=np.complex128), np.array(wts, dtype=np.complex128)


# --------------------------------------------------------------------------
# thin wrappers over the C routines
# --------------------------------------------------------------------------
def pfaffian(A) -> complex:
    """Pfaffian of a complex skew-symmetric matrix (Parlett-Reid, pivoted)."""
    A = _c128(A)
    m = A.shape[0]
    out = np.zeros(1, np.complex128)
    st = _load().or_pfaffian(m, _ptr(A), _ptr(out))
    if st:
        raise RuntimeError(f"or_pfaffian failed ({st})")
    return complex(out[0])


def covariance(Q, bits: int) -> np.ndarray:
    Q = _f64(Q)
    d = Q.shape[0]
    out = np.zeros((d, d))
    _load().or_covariance(d // 2, _ptr(Q), ctypes.c_uint64(int(bits)), _ptr(out))
    return out


def complement(phi) -> np.ndarray:
    phi = _c128(phi)
    n, eta = phi.shape
    out = np.zeros((n, max(n - eta, 1)), np.complex128)
    st = _load().or_complement(n, eta, _ptr(phi), _ptr(out))
    if st:
        raise np.linalg.LinAlgError("rank-deficient walker")
    return out[:, : n - eta]


def xmatrix(phi, perp=None) -> np.ndarray:
    phi = _c128(phi)
    n, eta = phi.shape
    perp = complement(phi) if perp is None else _c128(perp)
    X = np.zeros((2 * n - eta, 2 * n), np.complex128)
    st = _load().or_xmatrix(n, eta, _ptr(phi), _ptr(_c128(perp if perp.size else np.zeros((n, 1)))),
                            _ptr(X), None)
    if st:
        raise np.linalg.LinAlgError("singular [Phi | Phi_perp]")
    return X


def pair(phi, Q, bits: int, K=None, family="unit", perp=None, return_nodes=False):
    """One walker x shadow estimate o (and optionally the K Pfaffian values)."""
    phi = _c128(phi)
    n, eta = phi.shape
    z, w = node_weights(n, eta, K, family)
    Kk = len(z)
    Q = _f64(Q)
    o = np.zeros(1, np.complex128)
    nodes_out = np.zeros(Kk, np.complex128)
    lib = _load()
    if perp is None:
        st = lib.or_pair(n, eta, Kk, _ptr(z), _ptr(w), _ptr(phi), _ptr(Q), ctypes.c_uint64(int(bits)),
                         _ptr(o), _ptr(nodes_out))
    else:
        perp = _c128(perp)
        if perp.size == 0:
            perp = np.zeros((n, 1), np.complex128)
        st = lib.or_pair_perp(n, eta, Kk, _ptr(z), _ptr(w), _ptr(phi), _ptr(perp), _ptr(Q),
                              ctypes.c_uint64(int(bits)), _ptr(o), _ptr(nodes_out))
    if st:
        raise np.linalg.LinAlgError(f"oracle pair failed ({st})")
    return (complex(o[0]), nodes_out) if return_nodes else complex(o[0])


def overlap_pairs(phi, Q, bits, K=None, family="unit", pairs=None, nthreads=0, return_nodes=False):
    """Per-pair estimates o_ws.

    phi [W,n,eta] complex, Q [S,2n,2n] real, bits [S] uint64.  With
    ``pairs=None`` returns a [W,S] array; otherwise ``pairs`` is a (P,2) array
    of (walker, shadow) indices and a [P] array is returned.
    """
    phi = _c128(phi)
    Q = _f64(Q)
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    W, n, eta = phi.shape
    S = Q.shape[0]
    z, w = node_weights(n, eta, K, family)
    Kk = len(z)
    if pairs is None:
        npairs = W * S
        pw = ps = None
    else:
        pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
        npairs = pairs.shape[0]
        pw = np.ascontiguousarray(pairs[:, 0], dtype=np.int64)
        ps = np.ascontiguousarray(pairs[:, 1], dtype=np.int64)
    out = np.zeros(npairs, np.complex128)
    status = np.zeros(npairs, np.int32)
    nodes_out = np.zeros((npairs, Kk), np.complex128) if return_nodes else None
    _load().or_overlap_pairs(n, eta, Kk, _ptr(z), _ptr(w), _ptr(phi), W, _ptr(Q), _ptr(bits), S,
                             None if pw is None else _ptr(pw), None if ps is None else _ptr(ps), npairs,
                             _ptr(out), None if nodes_out is None else _ptr(nodes_out), _ptr(status),
                             int(nthreads))
    if status.any():
        raise np.linalg.LinAlgError(f"oracle failed on {int((status != 0).sum())} pairs")
    if pairs is None:
        out = out.reshape(W, S)
        if return_nodes:
            nodes_out = nodes_out.reshape(W, S, Kk)
    return (out, nodes_out) if return_nodes else out


def overlap(phi, Q, bits, K=None, family="unit", nthreads=0) -> np.ndarray:
    """S_w = (1/S) sum_s o_ws, the shadow estimate of <Psi_T|phi_w>."""
    return overlap_pairs(phi, Q, bits, K, family, nthreads=nthreads).mean(axis=1)


def grad(phi, Q, bits, K=None, family="unit", nthreads=0):
    """Per walker: S_w, D_w = d log S_w / d Phi_w (holomorphic, n x eta) and
    the mixed Green's function G_w = D_w Phi_w^T (G_pq = <a_p^dag a_q>).

    Eq. Pfaffian_der needs every node matrix A(z_k) to be invertible.  For a
    signed-permutation shadow that maps both Majoranas of a mode onto one
    mode, Pf(A(z)) has exact roots at z = +-1, and the unit-circle nodes
    include z = 1: use family="chebyshev" (the paper's nodes, never +-1) for
    that ensemble."""
    phi = _c128(phi)
    Q = _f64(Q)
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    W, n, eta = phi.shape
    S = Q.shape[0]
    z, w = node_weights(n, eta, K, family)
    osum = np.zeros(W, np.complex128)
    gsum = np.zeros((W, n, eta), np.complex128)
    status = np.zeros(W, np.int32)
    _load().or_grad_walkers(n, eta, len(z), _ptr(z), _ptr(w), _ptr(phi), W, _ptr(Q), _ptr(bits), S,
                            _ptr(osum), _ptr(gsum), _ptr(status), int(nthreads))
    if status.any():
        raise np.linalg.LinAlgError(f"oracle grad failed on {int((status != 0).sum())} walkers")
    D = gsum / osum[:, None, None]
    G = D @ np.transpose(phi, (0, 2, 1))
    return osum / S, D, G


def kmatrix(L) -> np.ndarray:
    """Majorana matrix K of a one-body operator Lhat = sum_pq L_pq a_p^dag a_q
    acting by commutation, [Lhat, gamma_rho] = sum_sigma K[rho, sigma]
    gamma_sigma (0-based Majoranas 2r, 2r+1 of mode r)."""
    L = _c128(L)
    n = L.shape[0]
    Km = np.zeros((2 * n, 2 * n), np.complex128)
    _load().or_kmatrix(n, _ptr(L), _ptr(Km))
    return Km


def energy_pairs(phi, Q, bits, t, L, K=None, family="chebyshev", pairs=None, nthreads=0):
    """Per-pair overlap estimates o_ws and local-energy numerators e_ws
    ("Force bias and local energy": eqs. local_energy, ham_cholesky_decom,
    energy_tb_diff, Pfaffian_der, Pfaffian_2nd_der).

    H = sum_pq t_pq a_p^dag a_q + 1/2 sum_g Lhat_g^2, Lhat_g = sum_pq
    L[p n + q, g] a_p^dag a_q; e_ws is the single-shadow estimate of
    <Psi_T|H|phi_w>, from the first and second derivatives of the node
    Pfaffians along e^{lambda Lhat}.  t [n, n] complex, L [n*n, n_gamma] real.
    Returns (o, e), each [W, S] (or [P] for a (P, 2) list of pairs).

    The default nodes are the paper's Chebyshev nodes.  The roots of unity
    include z = -1, which for odd n - eta is a root of Pf(C_0 + z B) for
    every walker and shadow: there the second-derivative formula multiplies
    a vanishing Pfaffian by two diverging inverses and loses all accuracy."""
    phi = _c128(phi)
    Q = _f64(Q)
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    t = _c128(t)
    L = _f64(L).reshape(phi.shape[1] ** 2, -1)
    W, n, eta = phi.shape
    S = Q.shape[0]
    ng = L.shape[1]
    z, w = node_weights(n, eta, K, family)
    if pairs is None:
        npairs, pw, ps = W * S, None, None
    else:
        pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
        npairs = pairs.shape[0]
        pw = np.ascontiguousarray(pairs[:, 0])
        ps = np.ascontiguousarray(pairs[:, 1])
    o = np.zeros(npairs, np.complex128)
    e = np.zeros(npairs, np.complex128)
    status = np.zeros(npairs, np.int32)
    _load().or_energy_pairs(n, eta, len(z), _ptr(z), _ptr(w), _ptr(phi), W, _ptr(Q), _ptr(bits), S,
                            None if pw is None else _ptr(pw), None if ps is None else _ptr(ps), npairs,
                            _ptr(t), _ptr(L), ng, _ptr(o), _ptr(e), _ptr(status), int(nthreads))
    if status.any():
        raise np.linalg.LinAlgError(f"oracle energy failed on {int((status != 0).sum())} pairs")
    if pairs is None:
        o, e = o.reshape(W, S), e.reshape(W, S)
    return o, e


def local_energy(phi, Q, bits, t, L, K=None, family="chebyshev", nthreads=0):
    """Per walker: S_w, the numerator N_w = (1/S) sum_s e_ws and the local
    energy E_L = N_w / S_w (eq. local_energy)."""
    o, e = energy_pairs(phi, Q, bits, t, L, K, family, nthreads=nthreads)
    Sw, Nw = o.mean(axis=1), e.mean(axis=1)
    return Sw, Nw, Nw / Sw


def force_bias(G, L, dt: float = 0.01) -> np.ndarray:
    """x_bar_gamma = -sqrt(dt) <v_gamma> with v_gamma = i sum_pq L^gamma_pq a_p^dag a_q
    (eqs. force_bias and cholesky_vec): -sqrt(dt) * i * sum_pq L[pq, gamma] G_pq."""
    G = np.asarray(G)
    W, n, _ = G.shape
    return -np.sqrt(dt) * 1j * (G.reshape(W, n * n) @ np.asarray(L).reshape(n * n, -1))


def rdm1(Q, bits, weights=None, trial: bool = False):
    """One-particle reduced density matrix from matchgate shadows
    (Supp. "Reduced Density Matrices").

    For a Majorana product of |S| = 2 operators the estimator of eq.
    local_fermionic_ob_exp is C(2n,2)/C(n,1) pf(i C'_s|_S) = (2n - 1) i C'_s[mu][nu]
    per shadow, with C'_s = Q_s^T C_b Q_s the shadow covariance, so
    <gamma_mu gamma_nu> (mu != nu) is estimated by i M[mu][nu] with
    M = (2n - 1) sum_s w_s C'_s (weights w_s, default 1/S).  The fermionic
    elements follow from gamma_{2j-1} = a_j + a_j^dag, gamma_{2j} = -i (a_j - a_j^dag)
    (eqs. majorana_op, 1rdm_off_diagonal, 1rdm_diagonal), written here 0-based
    (mode p <-> Majoranas 2p, 2p+1):
        <a_p^dag a_q> = 1/4 (<g_2p g_2q> + i <g_2p g_2q+1> - i <g_2p+1 g_2q> + <g_2p+1 g_2q+1>),  p != q
        <a_p^dag a_p> = 1/2 (1 + i <g_2p g_2p+1>).
    With trial=True the shadows are taken to be of (|0> + |Psi_T>)/sqrt2 and
    the result is the trial state's matrix, twice the measured state's (a
    number-conserving operator has no vacuum or cross term).

    Returns (G [n, n] complex128 with G[p, q] = <a_p^dag a_q>, M [2n, 2n] real).
    """
    Q = _f64(Q)
    bits = np.asarray(bits, dtype=np.uint64).reshape(-1)
    S, d, _ = Q.shape
    n = d // 2
    w = np.full(S, 1.0 / S) if weights is None else np.asarray(weights, np.float64)
    Cbar = np.zeros((d, d))
    for s in range(S):
        Cbar += w[s] * covariance(Q[s], int(bits[s]))
    M = (2 * n - 1) * Cbar
    np.fill_diagonal(M, 0.0)
    g2 = 1j * M                        # <gamma_mu gamma_nu>, mu != nu
    G = np.zeros((n, n), np.complex128)
    for p in range(n):
        for q in range(n):
            if p == q:
                G[p, p] = 0.5 * (1.0 + 1j * g2[2 * p, 2 * p + 1])
            else:
                G[p, q] = 0.25 * (g2[2 * p, 2 * q] + 1j * g2[2 * p, 2 * q + 1]
                                  - 1j * g2[2 * p + 1, 2 * q] + g2[2 * p + 1, 2 * q + 1])
    if trial:
        G = 2.0 * G
    return G, M
