"""Exact estimator for signed-permutation shadows (a weighted sum of minors).

TEST INFRASTRUCTURE ONLY (see the ``oracle`` package docstring).

The paper's shadows use random signed permutation matrices Q (section
"Classical shadows and the evaluation of overlaps").  For such Q,
U_Q^dag gamma_mu U_Q = s_mu gamma_{pi(mu)}, so the snapshot factorises:

    sigma = prod_j (1 - i beta_j s_{2j} s_{2j+1} gamma_{pi(2j)} gamma_{pi(2j+1)}) / 2

(0-based Majoranas, beta_j = (-1)^{b_j}, using |b><b| = prod_j (1 - i beta_j
gamma_{2j} gamma_{2j+1})/2).  Expanding the product, each subset T of modes
gives one Majorana monomial of grade 2|T|, which the inverse channel scales by
C(2n,2|T|)/C(n,|T|).  Hence

    o = 2^{1-n} sum_T mu_{|T|} prod_{j in T} (-i beta_j s_{2j} s_{2j+1})
        <0| prod_{j in T} gamma_{pi(2j)} gamma_{pi(2j+1)} |phi>,

and <0|Gamma|phi> = ph * <x|phi> with <x|phi> = det Phi[occupied(x), :].
Cost O(2^n eta^3): exact at the paper's n = 16 on the paper's own ensemble.
"""
from __future__ import annotations

from math import comb

import numpy as np


def random_signed_permutation(rng, n: int):
    """Uniform signed permutation of 2n Majoranas with det = +1.
    Returns (Q, perm, signs) with Q[mu, perm[mu]] = signs[mu]."""
    d = 2 * n
    perm = rng.permutation(d)
    signs = rng.choice([-1.0, 1.0], size=d)
    Q = np.zeros((d, d))
    Q[np.arange(d), perm] = signs
    if np.linalg.det(Q) < 0:
        signs[0] = -signs[0]
        Q[0, perm[0]] = signs[0]
    return Q, perm, signs


def _apply_majorana(mu: int, n: int, x: int):
    """gamma_mu |x> = ph |x'> (Jordan-Wigner, mode 0 most significant)."""
    j = mu // 2
    pos = n - 1 - j
    parity = bin(x >> (pos + 1)).count("1") & 1
    sgn = -1.0 if parity else 1.0
    occ = (x >> pos) & 1
    x2 = x ^ (1 << pos)
    if mu % 2 == 0:
        return sgn + 0j, x2
    return 1j * (1.0 - 2.0 * occ) * sgn, x2


def overlap_pair(phi, perm, signs, bits: int) -> complex:
    """Exact o for one walker and one signed-permutation shadow."""
    phi = np.asarray(phi, np.complex128)
    n, eta = phi.shape
    beta = [1.0 - 2.0 * ((int(bits) >> j) & 1) for j in range(n)]
    mu_fac = [comb(2 * n, 2 * r) / comb(n, r) for r in range(n + 1)]
    pair_mask = []
    for j in range(n):
        m = 0
        for mu in (perm[2 * j], perm[2 * j + 1]):
            m ^= 1 << (n - 1 - mu // 2)
        pair_mask.append(m)
    total = 0.0 + 0.0j
    for T in range(1 << n):
        flip = 0
        for j in range(n):
            if (T >> j) & 1:
                flip ^= pair_mask[j]
        if bin(flip).count("1") != eta:
            continue
        # apply Gamma_T = prod_{j in T, increasing} gamma_{pi(2j)} gamma_{pi(2j+1)}
        # to the basis state |flip> (right to left); it must land on |0>
        ph, x = 1.0 + 0j, flip
        coef = 1.0 + 0j
        js = [j for j in range(n) if (T >> j) & 1]
        for j in reversed(js):
            f, x = _apply_majorana(int(perm[2 * j + 1]), n, x)
            ph *= f
            f, x = _apply_majorana(int(perm[2 * j]), n, x)
            ph *= f
        for j in js:
            coef *= -1j * beta[j] * signs[2 * j] * signs[2 * j + 1]
        assert x == 0
        occ = [k for k in range(n) if (flip >> (n - 1 - k)) & 1]
        amp = np.linalg.det(phi[occ, :])
        total += mu_fac[len(js)] * coef * ph * amp
    return 2.0 ** (1 - n) * total
