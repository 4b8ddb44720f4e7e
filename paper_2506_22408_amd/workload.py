"""Seeded synthetic inputs shaped like the paper's post-processing workload.

This module only draws random inputs; it holds none of the estimator's
arithmetic, so both the HIP path and the CPU oracle can be fed from it.

The paper's data (measured matchgate shadows, VQE trial states, walkers of
the Ni-complex runs) is not available, so every workload is synthetic with
the paper's shapes: an (8,8) active space on N = 16 qubits, eta = 8
electrons, 1,280 walkers and tens of thousands of shadows (sections
"Computational details" and "HPC post-processing time").

Recipe (numpy ``default_rng(seed)``, PCG64, drawn in this order):
  walkers  Phi = reduced QR of (Z1 + i Z2), Z i.i.d. N(0,1)      [W,n,eta] c128
  shadows  Q   = Haar SO(2n): QR of a Gaussian, column signs fixed by
                 sign(diag R), first column negated if det < 0    [S,2n,2n] f64
           or (perm workloads) uniform signed permutations with det = +1,
                 the paper's ensemble                             [S,2n,2n] f64
  bits     b   = n-1 uniform bits, the last bit set to their parity
                 (uniform over even-parity strings); bit j is b_{j+1} [S] u64
  L        Cholesky-like vectors, N(0, 0.1^2), symmetrised per index pair
                                                                  [n*n, n_gamma]
  t        (local-energy workloads) one-body matrix, N(0, 0.1^2),
           symmetrised, drawn after L                             [n, n] c128

Full-space walkers for the virtual-correlation-energy path (make_vce), drawn
after nothing else from their own seed: alpha, then beta orbitals, each the
reduced QR of (Z1 + i Z2) of shape [W, N_B, N_c + n_spin]; then Q and b of
the active space (n = 2 N_a modes) as above.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def walkers(rng, W: int, n: int, eta: int, orthonormal: bool = True) -> np.ndarray:
    Z = rng.standard_normal((W, n, eta)) + 1j * rng.standard_normal((W, n, eta))
    if not orthonormal:
        return np.ascontiguousarray(Z)
    Qm, _ = np.linalg.qr(Z)
    return np.ascontiguousarray(Qm)


def haar_so(rng, S: int, d: int, chunk: int = 4096) -> np.ndarray:
    out = np.empty((S, d, d))
    for s0 in range(0, S, chunk):
        s1 = min(S, s0 + chunk)
        Z = rng.standard_normal((s1 - s0, d, d))
        Qm, R = np.linalg.qr(Z)
        sgn = np.sign(np.diagonal(R, axis1=1, axis2=2))
        sgn[sgn == 0] = 1.0
        Qm = Qm * sgn[:, None, :]
        neg = np.linalg.det(Qm) < 0
        Qm[neg, :, 0] *= -1.0
        out[s0:s1] = Qm
    return out


def signed_permutations(rng, S: int, d: int) -> np.ndarray:
    """Uniform signed permutations of d Majoranas with det = +1, the paper's
    shadow ensemble: Q[mu, pi(mu)] = s_mu with a uniform permutation pi and
    uniform signs, the first sign flipped where the determinant is -1."""
    perm = np.argsort(rng.random((S, d)), axis=1)
    signs = rng.choice(np.array([-1.0, 1.0]), size=(S, d))
    out = np.zeros((S, d, d))
    rows = np.arange(d)
    for s in range(S):
        out[s, rows, perm[s]] = signs[s]
    neg = np.linalg.det(out) < 0
    out[neg, 0, :] *= -1.0
    return out


def even_bits(rng, S: int, n: int) -> np.ndarray:
    b = rng.integers(0, 2, size=(S, n - 1), dtype=np.uint64)
    par = b.sum(axis=1) % 2
    words = np.zeros(S, dtype=np.uint64)
    for j in range(n - 1):
        words |= b[:, j] << np.uint64(j)
    words |= par.astype(np.uint64) << np.uint64(n - 1)
    return words


def cholesky_like(rng, n: int, n_gamma: int, scale: float = 0.1) -> np.ndarray:
    L = rng.standard_normal((n, n, n_gamma)) * scale
    L = 0.5 * (L + L.transpose(1, 0, 2))
    return np.ascontiguousarray(L.reshape(n * n, n_gamma))


@dataclass
class Workload:
    name: str
    n: int
    eta: int
    phi: np.ndarray
    Q: np.ndarray
    bits: np.ndarray
    L: np.ndarray | None = None
    t: np.ndarray | None = None

    @property
    def W(self) -> int:
        return self.phi.shape[0]

    @property
    def S(self) -> int:
        return self.Q.shape[0]


def one_body(rng, n: int, scale: float = 0.1) -> np.ndarray:
    h = rng.standard_normal((n, n)) * scale
    return np.ascontiguousarray(0.5 * (h + h.T)).astype(np.complex128)


def make(name: str, n: int, eta: int, W: int, S: int, seed: int, n_gamma: int = 0,
         orthonormal: bool = True, with_t: bool = False, shadows: str = "haar") -> Workload:
    """shadows: "haar" (Haar SO(2n)) or "perm" (signed permutations, the paper's ensemble)."""
    rng = np.random.default_rng(seed)
    phi = walkers(rng, W, n, eta, orthonormal)
    if shadows == "haar":
        Q = haar_so(rng, S, 2 * n)
    elif shadows == "perm":
        Q = signed_permutations(rng, S, 2 * n)
    else:
        raise ValueError(f"unknown shadow ensemble {shadows!r}")
    bits = even_bits(rng, S, n)
    L = cholesky_like(rng, n, n_gamma) if n_gamma else None
    t = one_body(rng, n) if with_t else None
    return Workload(name, n, eta, phi, Q, bits, L, t)


# The five workloads: small plain, paper-sized, uneven batch, gradient, precision.
CONFIGS = {
    "small_n8": dict(n=8, eta=4, W=16, S=64, seed=1),
    "paper_n16": dict(n=16, eta=8, W=1024, S=10000, seed=2),
    "grad_n16": dict(n=16, eta=8, W=1024, S=10000, seed=4, n_gamma=200),
    "precision_n24": dict(n=24, eta=12, W=2048, S=50000, seed=5),
    "energy_n16": dict(n=16, eta=8, W=128, S=1000, seed=7, n_gamma=200, with_t=True),
    "energy_n24": dict(n=24, eta=12, W=64, S=200, seed=3, n_gamma=200, with_t=True),
    # the paper's own shadow ensemble (random signed permutations) at the paper's size
    "perm_n16": dict(n=16, eta=8, W=1024, S=10000, seed=9, shadows="perm"),
}
UNEVEN = [dict(n=8, eta=4, W=4096, S=2000, seed=30),
          dict(n=12, eta=6, W=2048, S=5000, seed=31),
          dict(n=16, eta=8, W=1024, S=10000, seed=32),
          dict(n=20, eta=10, W=512, S=20000, seed=33)]


def config(name: str, W: int | None = None, S: int | None = None) -> Workload:
    """A named workload; W/S override truncate it (same seed, same prefix of
    walkers is NOT guaranteed when W changes, since draws are sequential)."""
    c = dict(CONFIGS[name])
    if W is not None:
        c["W"] = W
    if S is not None:
        c["S"] = S
    return make(name, **c)


@dataclass
class VceWorkload:
    """Full-space walkers (alpha and beta orbital blocks over N_B spatial
    orbitals: core 0..N_c-1, active N_c..N_c+N_a-1, then virtual) and the
    shadows of the 2 N_a-mode active space."""
    name: str
    n_basis: int
    n_core: int
    n_active: int
    n_alpha: int
    n_beta: int
    phi_alpha: np.ndarray
    phi_beta: np.ndarray
    Q: np.ndarray
    bits: np.ndarray

    @property
    def n(self) -> int:
        return 2 * self.n_active

    @property
    def eta(self) -> int:
        return self.n_alpha + self.n_beta

    @property
    def W(self) -> int:
        return self.phi_alpha.shape[0]

    @property
    def S(self) -> int:
        return self.Q.shape[0]


def make_vce(name: str, n_basis: int, n_core: int, n_active: int, n_alpha: int, n_beta: int, W: int, S: int,
             seed: int, orthonormal: bool = True) -> VceWorkload:
    rng = np.random.default_rng(seed)
    pa = walkers(rng, W, n_basis, n_core + n_alpha, orthonormal)
    pb = walkers(rng, W, n_basis, n_core + n_beta, orthonormal)
    n = 2 * n_active
    Q = haar_so(rng, S, 2 * n)
    bits = even_bits(rng, S, n)
    return VceWorkload(name, n_basis, n_core, n_active, n_alpha, n_beta, pa, pb, Q, bits)


# N_B = 130 spatial orbitals and the (8e, 8o) active space are the paper's; it
# gives no core count, and 46 doubly occupied core orbitals is a stand-in.
VCE_CONFIGS = {
    "vce_n16": dict(n_basis=130, n_core=46, n_active=8, n_alpha=4, n_beta=4, W=1024, S=10000, seed=6),
}


def vce_config(name: str, W: int | None = None, S: int | None = None) -> VceWorkload:
    c = dict(VCE_CONFIGS[name])
    if W is not None:
        c["W"] = W
    if S is not None:
        c["S"] = S
    return make_vce(name, **c)
