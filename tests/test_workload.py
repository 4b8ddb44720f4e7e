"""The seeded input generator produces what its recipe states."""
import numpy as np

from paper_2506_22408_amd import workload as wl


def test_haar_so_is_special_orthogonal():
    rng = np.random.default_rng(0)
    Q = wl.haar_so(rng, 50, 32)
    eye = np.eye(32)
    assert np.abs(np.einsum("sij,sik->sjk", Q, Q) - eye).max() < 1e-12
    assert np.allclose(np.linalg.det(Q), 1.0)


def test_bits_even_parity_and_range():
    rng = np.random.default_rng(1)
    b = wl.even_bits(rng, 1000, 16)
    assert b.dtype == np.uint64
    assert np.all(b < (1 << 16))
    assert all(bin(int(v)).count("1") % 2 == 0 for v in b)
    # every bit position is used
    assert all(((b >> np.uint64(j)) & np.uint64(1)).any() for j in range(16))


def test_walkers_orthonormal():
    rng = np.random.default_rng(2)
    phi = wl.walkers(rng, 20, 16, 8)
    gram = np.einsum("wpi,wpj->wij", phi.conj(), phi)
    assert np.abs(gram - np.eye(8)).max() < 1e-12


def test_seeded_reproducible():
    a = wl.make("x", 8, 4, 4, 6, seed=3, n_gamma=5)
    b = wl.make("x", 8, 4, 4, 6, seed=3, n_gamma=5)
    assert np.array_equal(a.phi, b.phi) and np.array_equal(a.Q, b.Q)
    assert np.array_equal(a.bits, b.bits) and np.array_equal(a.L, b.L)
    assert np.allclose(a.L.reshape(8, 8, 5), a.L.reshape(8, 8, 5).transpose(1, 0, 2))
