"""Pins of the oracle's VCE prologue (Supp. "Virtual Correlation Energy
Derivation", eq. vce_overlap) against the plain definition: the full-space
overlap as a sum of determinants over the active determinants of an explicit
multi-determinant trial state.

A transposed or conjugated factor, a wrong block order in V (the sign
(-1)^(N_c n_alpha)), or a dropped det(R) or det(Sigma) fails
test_factorisation_equals_full_space_determinants.  The cases cover no core,
an empty spin, no virtual orbitals and non-orthonormal walkers.
"""
import itertools

import numpy as np
import pytest

from oracle import vce


def rand_walker(rng, NB, ne, orth):
    z = rng.standard_normal((NB, ne)) + 1j * rng.standard_normal((NB, ne))
    return np.linalg.qr(z)[0] if orth else z


def rand_ci(rng, na, nal, nbe):
    ci = {}
    for oa in itertools.combinations(range(na), nal):
        for ob in itertools.combinations(range(na), nbe):
            ci[(oa, ob)] = rng.standard_normal() + 1j * rng.standard_normal()
    return ci


CASES = [  # N_B, N_c, N_a, n_alpha, n_beta, orthonormal walker
    (9, 2, 3, 2, 1, False), (9, 2, 3, 2, 1, True), (7, 0, 3, 1, 2, False), (10, 3, 3, 0, 2, False),
    (12, 2, 4, 2, 2, True), (6, 3, 3, 1, 1, False), (5, 1, 4, 3, 3, True), (14, 5, 4, 1, 3, False),
]


@pytest.mark.parametrize("NB,nc,na,nal,nbe,orth", CASES)
def test_factorisation_equals_full_space_determinants(NB, nc, na, nal, nbe, orth):
    rng = np.random.default_rng(NB * 100 + nc * 10 + na + nal)
    pa, pb = rand_walker(rng, NB, nc + nal, orth), rand_walker(rng, NB, nc + nbe, orth)
    ci = rand_ci(rng, na, nal, nbe)
    full = vce.full_space_overlap(pa, pb, nc, na, ci)
    act, pref = vce.active_walker(pa, pb, nc, na)
    assert abs(pref * vce.active_space_overlap(act, na, ci) - full) <= 1e-12 * abs(full)
    # the active walker has orthonormal columns and the block structure
    assert np.allclose(act.conj().T @ act, np.eye(nal + nbe), atol=1e-13)
    assert np.all(act[:na, nal:] == 0) and np.all(act[na:, :nal] == 0)


def test_single_determinants_each():
    """Every active determinant on its own (c = one-hot) reproduces its
    full-space determinant, so no term of the sum can hide another."""
    rng = np.random.default_rng(11)
    NB, nc, na, nal, nbe = 8, 2, 3, 2, 1
    pa, pb = rand_walker(rng, NB, nc + nal, False), rand_walker(rng, NB, nc + nbe, False)
    act, pref = vce.active_walker(pa, pb, nc, na)
    for key in rand_ci(rng, na, nal, nbe):
        ci = {key: 1.0}
        full = vce.full_space_overlap(pa, pb, nc, na, ci)
        assert abs(pref * vce.active_space_overlap(act, na, ci) - full) <= 1e-12 * max(abs(full), 1e-300)


def test_virtual_rows_do_not_enter():
    rng = np.random.default_rng(12)
    NB, nc, na, nal, nbe = 11, 2, 3, 1, 2
    pa, pb = rand_walker(rng, NB, nc + nal, False), rand_walker(rng, NB, nc + nbe, False)
    act, pref = vce.active_walker(pa, pb, nc, na)
    pa2, pb2 = pa.copy(), pb.copy()
    pa2[nc + na:] = rng.standard_normal(pa2[nc + na:].shape)
    pb2[nc + na:] = 0.0
    act2, pref2 = vce.active_walker(pa2, pb2, nc, na)
    assert np.allclose(act, act2, atol=1e-14) and abs(pref - pref2) <= 1e-13 * abs(pref)


def test_multilinear_in_the_walker():
    """phi^a -> phi^a R multiplies the overlap by det R (a determinant is
    multilinear in its columns), whatever the trial state."""
    rng = np.random.default_rng(13)
    NB, nc, na, nal, nbe = 9, 3, 3, 2, 2
    pa, pb = rand_walker(rng, NB, nc + nal, True), rand_walker(rng, NB, nc + nbe, True)
    R = rng.standard_normal((nc + nal, nc + nal)) + 1j * rng.standard_normal((nc + nal, nc + nal))
    ci = rand_ci(rng, na, nal, nbe)
    a0, p0 = vce.active_walker(pa, pb, nc, na)
    a1, p1 = vce.active_walker(pa @ R, pb, nc, na)
    o0 = p0 * vce.active_space_overlap(a0, na, ci)
    o1 = p1 * vce.active_space_overlap(a1, na, ci)
    assert abs(o1 - np.linalg.det(R) * o0) <= 1e-11 * abs(o1)


def test_no_core_is_the_active_overlap():
    """N_c = 0: V = I, so the prefactor times <Psi_a|phi~_a> is the overlap
    of the active rows themselves."""
    rng = np.random.default_rng(14)
    NB, na, nal, nbe = 7, 4, 2, 2
    pa, pb = rand_walker(rng, NB, nal, False), rand_walker(rng, NB, nbe, False)
    ci = rand_ci(rng, na, nal, nbe)
    act, pref = vce.active_walker(pa, pb, 0, na)
    direct = np.zeros((2 * na, nal + nbe), complex)
    direct[:na, :nal], direct[na:, nal:] = pa[:na], pb[:na]
    assert abs(pref * vce.active_space_overlap(act, na, ci) - vce.active_space_overlap(direct, na, ci)) <= \
        1e-12 * abs(vce.active_space_overlap(direct, na, ci))


def test_rank_deficient_core_gives_zero():
    rng = np.random.default_rng(15)
    NB, nc, na, nal, nbe = 8, 3, 3, 1, 1
    pa, pb = rand_walker(rng, NB, nc + nal, False), rand_walker(rng, NB, nc + nbe, False)
    pa[1] = 2.0 * pa[0]   # two core rows proportional: Xi^dag phi_c has rank 2 < 3
    _, pref = vce.active_walker(pa, pb, nc, na)
    assert abs(pref) <= 1e-12
    assert abs(vce.full_space_overlap(pa, pb, nc, na, rand_ci(rng, na, nal, nbe))) <= 1e-10
