"""Parity of the HIP adjoint (shadow_overlap_grad, through the C ABI) with the
CPU oracle's gradient, and with central finite differences of the HIP
forward itself.

Tolerances: S_w as in the forward (1e-10 relative); D_w and G_w per walker
|x_gpu - x_oracle| <= 1e-10 max|x_oracle| (observed: below 2e-13); central
finite differences (h = 1e-6) to 1e-7 relative (their own truncation and
rounding error is about 1e-8).  Shadows near a pair-preserving rotation,
whose pair values nearly cancel, hold S_w to 1e-9 (D_w and G_w still to
1e-10).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2506_22408_amd import workload as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2506_22408_amd import binding
    return binding


def dev():
    return torch.device("cuda:0")


def to_dev(phi, Q, bits):
    return (torch.from_numpy(np.ascontiguousarray(phi)).to(dev()),
            torch.from_numpy(np.ascontiguousarray(Q)).to(dev()),
            torch.from_numpy(np.ascontiguousarray(bits).view(np.int64)).to(dev()))


def gpu_grad(B, phi, Q, bits):
    out, dlog, green, status = B.shadow_overlap_grad(*to_dev(phi, Q, bits))
    torch.cuda.synchronize()
    return out.cpu().numpy(), dlog.cpu().numpy(), green.cpu().numpy(), status.cpu().numpy()


def close_per_walker(a, b, rtol):
    worst = 0.0
    for w in range(a.shape[0]):
        scale = np.abs(b[w]).max()
        err = np.abs(a[w] - b[w]).max()
        assert err <= rtol * scale, f"walker {w}: err {err:.3e} vs scale {scale:.3e}"
        worst = max(worst, err / scale)
    return worst


@pytest.mark.parametrize("n,eta,W,S", [
    (4, 2, 3, 7), (6, 2, 2, 5), (8, 4, 4, 9), (8, 2, 2, 4),            # one tile, ne = 2, 4, 6
    (10, 8, 3, 6), (12, 8, 2, 5), (10, 4, 3, 7), (16, 8, 3, 11)])      # two tiles, ne = 2, 4, 6, 8
def test_grad_matches_oracle(B, n, eta, W, S):
    w = wl.make("g", n, eta, W, S, seed=500 + 3 * n + eta)
    sg, dg, gg, st = gpu_grad(B, w.phi, w.Q, w.bits)
    so, do, go = oracle.grad(w.phi, w.Q, w.bits)
    assert not st.any()
    assert np.all(np.abs(sg - so) <= 1e-10 * np.abs(so))
    ed, eg = close_per_walker(dg, do, 1e-10), close_per_walker(gg, go, 1e-10)
    print(f"n={n} eta={eta}: worst D {ed:.2e}, G {eg:.2e} (relative to max per walker)")


@pytest.mark.parametrize("n,eta,S", [(8, 4, 16), (8, 4, 40), (8, 4, 136), (16, 8, 16), (16, 8, 40), (16, 8, 136)])
def test_grad_several_shadows_per_range(B, n, eta, S):
    """1024 walkers split the shadows into 8 ranges per walker, so one wave
    accumulates F and the pair sum over spw = 2, 5 and 17 shadows (as the
    paper-sized workload does over 1,250): 16 walkers against the oracle."""
    W = 1024
    w = wl.make("spw", n, eta, W, S, seed=610 + n + S)
    sg, dg, gg, st = gpu_grad(B, w.phi, w.Q, w.bits)
    assert not st.any()
    pick = np.random.default_rng(S).choice(W, 16, replace=False)
    so, do, go = oracle.grad(w.phi[pick], w.Q, w.bits)
    assert np.all(np.abs(sg[pick] - so) <= 1e-10 * np.abs(so))
    ed, eg = close_per_walker(dg[pick], do, 1e-10), close_per_walker(gg[pick], go, 1e-10)
    print(f"n={n} S={S} (spw {-(-S // 8)}): worst D {ed:.2e}, G {eg:.2e}")


@pytest.fixture(scope="module")
def grad_paper(B):
    """The paper-sized derivative workload (1024 walkers x 10,000 shadows,
    8 shadow ranges of 1,250 per walker) through the C ABI once."""
    w = wl.config("grad_n16")
    print(f"grad_n16: {w.W} x {w.S} pairs through shadow_overlap_grad", flush=True)
    return w, gpu_grad(B, w.phi, w.Q, w.bits)


def test_grad_paper_workload_sampled(grad_paper):
    """S_w, D_w and G_w of 16 walkers of the full workload against the
    oracle over all 10,000 shadows."""
    w, (sg, dg, gg, st) = grad_paper
    assert not st.any()
    pick = np.random.default_rng(4).choice(w.W, 16, replace=False)
    so, do, go = oracle.grad(w.phi[pick], w.Q, w.bits)
    assert np.all(np.abs(sg[pick] - so) <= 1e-10 * np.abs(so))
    ed, eg = close_per_walker(dg[pick], do, 1e-10), close_per_walker(gg[pick], go, 1e-10)
    print(f"grad_n16, 16 walkers x 10000 shadows: worst D {ed:.2e}, G {eg:.2e}")


def test_grad_paper_workload_finite_differences(B, grad_paper):
    """Central differences (h = 1e-6) of the HIP forward over all 10,000
    shadows on 8 walkers of the full workload, against D_w S_w from the
    full-size derivative launch."""
    w, (sg, dg, _, _) = grad_paper
    pick = np.arange(8) * 127
    Qd = torch.from_numpy(w.Q).to(dev())
    bd = torch.from_numpy(w.bits.view(np.int64)).to(dev())
    rng = np.random.default_rng(8)
    h = 1e-6
    for _ in range(4):
        p, j = int(rng.integers(w.n)), int(rng.integers(w.eta))
        for step in (h, 1j * h):
            ph = w.phi[pick].copy()
            ph[:, p, j] += step
            sp, _, _ = B.shadow_overlap(torch.from_numpy(ph).to(dev()), Qd, bd)
            ph[:, p, j] -= 2 * step
            sm, _, _ = B.shadow_overlap(torch.from_numpy(ph).to(dev()), Qd, bd)
            fd = (sp.cpu().numpy() - sm.cpu().numpy()) / (2 * step)
            an = dg[pick, p, j] * sg[pick]
            assert np.all(np.abs(fd - an) <= 1e-7 * np.abs(an) + 1e-12), (p, j, step, fd, an)
            print(f"FD ({p},{j}) step {step}: worst rel {np.max(np.abs(fd - an) / np.abs(an)):.2e}")


def test_grad_signed_permutation_shadows(B):
    """The paper's shadow ensemble (random signed permutations) through the
    derivative, against the oracle and against central differences of the
    HIP forward.  A signed permutation that maps both Majoranas of a mode onto
    one mode gives Pf(A(z)) exact roots at z = +-1, where eq. Pfaffian_der's
    inverse does not exist; the oracle's unit-circle nodes include z = 1, so
    it is run on the paper's Chebyshev nodes, which avoid +-1.  Their
    Vandermonde system amplifies the oracle's own rounding by 1e3 to 1e4 at
    n = 16 (a few 1e-12 to 1e-10 relative per shadow), so D_w and G_w are held
    to 1e-9 here; the finite differences check the kernel independently."""
    w = wl.make("gp", 16, 8, 24, 60, seed=66, shadows="perm")
    sg, dg, gg, st = gpu_grad(B, w.phi, w.Q, w.bits)
    so, do, go = oracle.grad(w.phi, w.Q, w.bits, family="chebyshev")
    assert not st.any()
    assert np.all(np.abs(sg - so) <= 1e-10 * np.abs(so))
    ed, eg = close_per_walker(dg, do, 1e-9), close_per_walker(gg, go, 1e-9)
    print(f"signed permutations: worst D {ed:.2e}, G {eg:.2e}")
    Qd, bd = torch.from_numpy(w.Q).to(dev()), torch.from_numpy(w.bits.view(np.int64)).to(dev())
    rng = np.random.default_rng(9)
    h = 1e-6
    E = rng.standard_normal((w.n, w.eta)) + 1j * rng.standard_normal((w.n, w.eta))
    ph = np.stack([w.phi + h * E, w.phi - h * E])
    sp, _, _ = B.shadow_overlap(torch.from_numpy(ph[0]).to(dev()), Qd, bd)
    sm, _, _ = B.shadow_overlap(torch.from_numpy(ph[1]).to(dev()), Qd, bd)
    fd = (sp.cpu().numpy() - sm.cpu().numpy()) / (2 * h)
    an = np.einsum("wpj,pj->w", dg, E) * sg
    assert np.all(np.abs(fd - an) <= 1e-7 * np.abs(an)), np.abs(fd - an) / np.abs(an)


def test_grad_finite_differences_of_the_gpu_forward(B):
    """Central differences of the HIP forward S_w along Phi_pj (holomorphic
    derivative: a real step h on the complex entry) against D_w S_w."""
    n, eta = 16, 8
    w = wl.make("fd", n, eta, 8, 40, seed=77)
    sg, dg, _, _ = gpu_grad(B, w.phi, w.Q, w.bits)
    rng = np.random.default_rng(3)
    h = 1e-6
    for _ in range(6):
        p, j = int(rng.integers(n)), int(rng.integers(eta))
        for step in (h, 1j * h):
            ph = w.phi.copy()
            ph[:, p, j] += step
            sp, _, _ = B.shadow_overlap(*to_dev(ph, w.Q, w.bits))
            ph[:, p, j] -= 2 * step
            sm, _, _ = B.shadow_overlap(*to_dev(ph, w.Q, w.bits))
            fd = (sp.cpu().numpy() - sm.cpu().numpy()) / (2 * step)
            an = dg[:, p, j] * sg
            assert np.all(np.abs(fd - an) <= 1e-7 * np.abs(an) + 1e-12), (p, j, step, fd, an)
            print(f"FD ({p},{j}) step {step}: worst rel {np.max(np.abs(fd - an) / np.abs(an)):.2e}")


def test_grad_full_size_route(B):
    """Shadows near a pair-preserving rotation make the elimination of K
    ill conditioned, so those pairs take the full-size route (Pf and inverse
    of every B + e_j J); all must still match the oracle."""
    import scipy.linalg as sla
    n, eta = 8, 4
    rng = np.random.default_rng(41)
    phi = wl.walkers(rng, 3, n, eta)
    Qs = []
    for eps in (3e-1, 1e-2, 1e-4, 1e-6):
        hm = rng.standard_normal((2 * n, 2 * n))
        Qs.append(sla.expm(eps * (hm - hm.T)))
    Qs = np.array(Qs)
    bits = wl.even_bits(rng, len(Qs), n)
    sg, dg, gg, st = gpu_grad(B, phi, Qs, bits)
    so, do, go = oracle.grad(phi, Qs, bits)
    assert not (st & ~B.SO_WSTAT_SINGULAR).any()
    assert np.all(np.abs(sg - so) <= 1e-9 * np.abs(so))
    ed, eg = close_per_walker(dg, do, 1e-10), close_per_walker(gg, go, 1e-10)
    print(f"full-size route: worst D {ed:.2e}, G {eg:.2e} (relative to max per walker)")


@pytest.mark.parametrize("n,eta", [(8, 4), (16, 8)])
def test_grad_full_size_route_then_ordinary_pairs(B, n, eta):
    """A pair on the full-size route followed, in the same shadow range, by
    ordinary pairs (the two waves of a workgroup must leave the route in step):
    1,024 copies of one walker over 8 ranges of 100 shadows, the first of each
    range near a pair-preserving rotation, must all give the same bits, and
    those must match the oracle."""
    import scipy.linalg as sla
    W, Gy, spw = 1024, 8, 100
    base = wl.make("fr", n, eta, 1, Gy * spw, seed=4100 + n)
    rng = np.random.default_rng(4200 + n)
    Q = base.Q.copy()
    for r in range(Gy):
        hm = rng.standard_normal((2 * n, 2 * n))
        Q[r * spw] = sla.expm(1e-6 * (hm - hm.T))
    ph1, Qd, bd = to_dev(base.phi, Q, base.bits)
    B.shadow_overlap(ph1, Qd, bd)
    routed = B.fallback_count(ph1, Qd, bd)
    assert routed >= Gy // 2                       # the route opens most ranges
    phi = np.repeat(base.phi, W, axis=0)
    sg, dg, gg, st = gpu_grad(B, phi, Q, base.bits)
    assert not (st & ~B.SO_WSTAT_SINGULAR).any()
    for x in (sg, dg, gg, st):
        assert (x == x[:1]).all(), "copies of one walker differ"
    so, do, go = oracle.grad(base.phi, Q, base.bits)
    assert np.all(np.abs(sg[:1] - so) <= 1e-9 * np.abs(so))
    ed, eg = close_per_walker(dg[:1], do, 1e-10), close_per_walker(gg[:1], go, 1e-10)
    print(f"n={n}: full-size route first in {routed} of {Gy} ranges, 1024 copies equal; D {ed:.2e}, G {eg:.2e}")


def test_grad_zero_overlap_is_flagged(B):
    """Walkers whose orbitals are single modes, with the identity shadow and
    b = 0, give pair values that are exactly zero, so S_w = 0: the walker is
    flagged and its derivative (of log S_w) is NaN, not a number."""
    n, eta, W = 8, 4, 3
    rng = np.random.default_rng(2)
    phi = np.zeros((W, n, eta), complex)
    for w in range(W):
        phi[w, rng.choice(n, eta, replace=False), np.arange(eta)] = 1.0
    Q = np.tile(np.eye(2 * n), (5, 1, 1))
    bits = np.zeros(5, np.uint64)
    sg, dg, gg, st = gpu_grad(B, phi, Q, bits)
    assert np.all(sg == 0)
    assert np.all(st & B.SO_WSTAT_ZERO)
    assert np.all(np.isnan(dg)) and np.all(np.isnan(gg))


def test_grad_under_right_multiplication_of_the_walkers(B):
    """The overlap is multilinear in the walker's orbitals, so for every
    invertible eta x eta A: S(Phi A) = det A S(Phi), D(Phi A) = D(Phi) A^{-T}
    and G(Phi A) = G(Phi).  A random well-conditioned A, and A = c I with
    c = 1e+-20 and 1e+-60 (c^8 outside double precision at 1e+-60, where the
    log output holds log S(Phi) + eta log c exactly and the walker's
    Householder factors keep D and G at full accuracy)."""
    n, eta, W, S = 16, 8, 4, 23
    w = wl.make("gr", n, eta, W, S, seed=83)
    s0, d0, g0, st0 = gpu_grad(B, w.phi, w.Q, w.bits)
    assert not st0.any()
    rng = np.random.default_rng(84)
    A = np.eye(eta) + 0.3 * (rng.standard_normal((W, eta, eta)) + 1j * rng.standard_normal((W, eta, eta)))
    sa, da, ga, sta = gpu_grad(B, w.phi @ A, w.Q, w.bits)
    assert not sta.any()
    assert np.all(np.abs(sa - np.linalg.det(A) * s0) <= 1e-10 * np.abs(sa))
    close_per_walker(da, d0 @ np.linalg.inv(A).transpose(0, 2, 1), 1e-10)
    close_per_walker(ga, g0, 1e-10)
    Q, bits = w.Q, w.bits
    l0 = B.shadow_overlap_grad(*to_dev(w.phi, Q, bits), log_output=True)[0].cpu().numpy()
    for c in (1e-60, 1e-20, 1e20, 1e60):
        lc, dc, gc, stc = (t.cpu().numpy() for t in B.shadow_overlap_grad(*to_dev(w.phi * c, Q, bits),
                                                                            log_output=True))
        assert not stc.any()
        dl = lc - (l0 + eta * np.log(c))
        dl = dl.real + 1j * ((dl.imag + np.pi) % (2 * np.pi) - np.pi)
        assert np.all(np.abs(dl) <= 1e-12 * np.abs(lc.real) + 1e-12), (c, dl)
        close_per_walker(dc, d0 / c, 1e-10)
        close_per_walker(gc, g0, 1e-10)
        _, _, _, sp = gpu_grad(B, w.phi * c, Q, bits)
        if c > 1 and eta * np.log10(c) > 308:
            assert (sp & B.SO_WSTAT_NONFINITE).all()
        else:
            assert not sp.any()


def test_grad_rank_deficient_walker_is_nan(B):
    """A walker whose orbitals are linearly dependent has no derivative: it
    is flagged SO_WSTAT_RANK and its S_w, D_w and G_w are NaN, while the
    other walkers of the call keep the oracle's values."""
    n, eta, W, S = 8, 4, 3, 6
    w = wl.make("rk", n, eta, W, S, seed=77)
    phi = w.phi.copy()
    phi[1, :, 3] = phi[1, :, 0] * (0.5 - 0.25j)
    sg, dg, gg, st = gpu_grad(B, phi, w.Q, w.bits)
    assert st[1] & B.SO_WSTAT_RANK and not st[[0, 2]].any()
    assert np.isnan(sg[1]) and np.all(np.isnan(dg[1])) and np.all(np.isnan(gg[1]))
    so, do, go = oracle.grad(phi[[0, 2]], w.Q, w.bits)
    assert np.all(np.abs(sg[[0, 2]] - so) <= 1e-10 * np.abs(so))
    close_per_walker(dg[[0, 2]], do, 1e-10)
    close_per_walker(gg[[0, 2]], go, 1e-10)


def test_grad_unsupported_shapes_are_refused(B):
    for n, eta in ((16, 2), (20, 16), (9, 4)):       # ne = 14; n > 16; ne odd
        w = wl.make("u", n, eta, 2, 3, seed=1)
        with pytest.raises(B.ShadowOvError) as e:
            B.shadow_overlap_grad(*to_dev(w.phi, w.Q, w.bits))
        assert e.value.code == B.SO_ERR_UNSUPPORTED


def test_force_bias_matches_oracle(B):
    """x_bar from the GPU Green's function with 200 Cholesky-like vectors
    (the gradient workload's shapes) against the oracle's definition."""
    w = wl.config("grad_n16", W=8, S=30)
    _, _, gg, st = gpu_grad(B, w.phi, w.Q, w.bits)
    assert not st.any()
    xb = B.force_bias(torch.from_numpy(gg).to(dev()), torch.from_numpy(w.L).to(dev()), 0.01).cpu().numpy()
    ref = oracle.force_bias(gg, w.L, 0.01)
    assert xb.shape == (8, 200)
    assert np.all(np.abs(xb - ref) <= 1e-13 * np.abs(ref).max())


def test_autograd_log_overlap(B):
    """loss = Re sum_w c_w log S_w; phi.grad from the autograd function
    against central differences of the loss in Re and Im of Phi entries."""
    n, eta = 8, 4
    w = wl.make("ag", n, eta, 3, 12, seed=21)
    phi = torch.from_numpy(w.phi).to(dev()).requires_grad_(True)
    Qd = torch.from_numpy(w.Q).to(dev())
    bd = torch.from_numpy(w.bits.view(np.int64)).to(dev())
    c = torch.tensor([0.3 - 0.7j, -1.1 + 0.2j, 0.5 + 0.5j], dtype=torch.complex128, device=dev())
    logs, st = B.log_overlap(phi, Qd, bd)
    assert not st.any()
    (c * logs).real.sum().backward()
    g = phi.grad.cpu().numpy()

    def loss(ph):
        s, _, _ = B.shadow_overlap(torch.from_numpy(ph).to(dev()), Qd, bd)
        return float((c * torch.log(s)).real.sum())

    rng = np.random.default_rng(0)
    h = 1e-6
    for _ in range(5):
        wi, p, j = int(rng.integers(3)), int(rng.integers(n)), int(rng.integers(eta))
        num = 0j
        for step, unit in ((h, 1.0), (1j * h, 1j)):
            ph = w.phi.copy()
            ph[wi, p, j] += step
            lp = loss(ph)
            ph[wi, p, j] -= 2 * step
            lm = loss(ph)
            num += unit * (lp - lm) / (2 * h)
        assert abs(num - g[wi, p, j]) <= 1e-7 * max(abs(g[wi, p, j]), 1e-3), (wi, p, j, num, g[wi, p, j])


def test_grad_deterministic(B):
    w = wl.make("d", 16, 8, 3, 25, seed=12)
    a = gpu_grad(B, w.phi, w.Q, w.bits)
    b = gpu_grad(B, w.phi, w.Q, w.bits)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
