"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerance (FP64 path): per pair |o_gpu - o_oracle| <= 1e-10 * max(|o_oracle|,
1e-3 * median|o_oracle|), i.e. 1e-10 relative except for pairs whose value is
a thousand times below the typical one, which are held to 1e-13 of the typical
magnitude (their relative error is dominated by cancellation in the node sum,
identical in both implementations up to rounding).  Walker averages:
|S_gpu - S_oracle| <= 1e-10 |S_oracle|.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import closed_form
from paper_2506_22408_amd import workload as wl

pytestmark = pytest.mark.gpu

RTOL = 1e-10


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


def gpu_overlap(B, phi, Q, bits, **kw):
    t = to_dev(phi, Q, bits)
    out, pairs, status = B.shadow_overlap(*t, return_pairs=True, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy(), pairs.cpu().numpy(), status.cpu().numpy()


def assert_pairs_close(og, oo, rtol=RTOL, what=""):
    scale = np.median(np.abs(oo))
    bound = rtol * np.maximum(np.abs(oo), 1e-3 * scale)
    err = np.abs(og - oo)
    bad = err > bound
    worst = np.max(err / np.maximum(np.abs(oo), 1e-3 * scale))
    assert not bad.any(), f"{what}: {bad.sum()} of {bad.size} pairs out of tolerance, worst rel {worst:.3e}"
    return worst


def assert_walkers_close(sg, so, rtol=RTOL, what=""):
    rel = np.abs(sg - so) / np.abs(so)
    assert np.all(rel <= rtol), f"{what}: worst rel {rel.max():.3e}"
    return rel.max()


def test_small_workload_all_pairs(B):
    w = wl.config("small_n8")
    sg, pg, st = gpu_overlap(B, w.phi, w.Q, w.bits)
    po = oracle.overlap_pairs(w.phi, w.Q, w.bits)
    print(f"small_n8 pairs worst rel {assert_pairs_close(pg, po, what='small_n8'):.2e}")
    assert_walkers_close(sg, po.mean(axis=1), what="small_n8 S_w")
    assert not st.any()


@pytest.mark.parametrize("n,eta,W,S", [
    # two-kernel path (ne = n - eta odd, 0 or above 12)
    (2, 2, 3, 4), (5, 4, 2, 7), (8, 8, 2, 3), (16, 2, 2, 3), (17, 2, 2, 5), (21, 8, 2, 3),
    (18, 2, 2, 3), (20, 4, 2, 3), (24, 10, 2, 3), (24, 8, 2, 3),
    # fused pair kernel, every (tiles, ne) instance; S ragged against the node batches
    (4, 2, 3, 5), (6, 2, 5, 9), (8, 2, 3, 7), (10, 4, 4, 11), (12, 6, 3, 13), (12, 8, 3, 10), (16, 14, 2, 5),
    (16, 8, 5, 33), (18, 16, 2, 4), (20, 16, 2, 5), (22, 16, 2, 4), (24, 16, 2, 9),
    # ne = 10 and 12: node Pfaffians per 16-lane row (batches of 5 and 4 pairs)
    (14, 4, 2, 6), (12, 2, 3, 11), (16, 4, 2, 9), (14, 2, 2, 5), (20, 10, 3, 9), (18, 8, 2, 7),
    (24, 12, 3, 10), (22, 10, 2, 5)])
def test_sizes_and_ragged_shapes(B, n, eta, W, S):
    """Every compiled size class: m = 2n - eta from 2 to 46, both paths."""
    w = wl.make("t", n, eta, W, S, seed=1000 + 7 * n + eta, orthonormal=(n % 2 == 0))
    sg, pg, st = gpu_overlap(B, w.phi, w.Q, w.bits)
    po = oracle.overlap_pairs(w.phi, w.Q, w.bits)
    print(f"n={n} eta={eta} m={2 * n - eta}: worst rel {assert_pairs_close(pg, po, what=f'n{n}e{eta}'):.2e}")
    assert_walkers_close(sg, po.mean(axis=1), what="S_w")
    assert not st.any()


def test_chebyshev_nodes_and_custom_node_count(B):
    w = wl.make("t", 10, 4, 3, 8, seed=77)
    for kw in (dict(nodes="chebyshev"), dict(n_nodes=14), dict(nodes="chebyshev", n_nodes=12)):
        _, pg, _ = gpu_overlap(B, w.phi, w.Q, w.bits, **kw)
        po = oracle.overlap_pairs(w.phi, w.Q, w.bits, K=kw.get("n_nodes") or None,
                                  family=kw.get("nodes", "unit"))
        assert_pairs_close(pg, po, rtol=1e-9 if kw.get("nodes") == "chebyshev" else RTOL, what=str(kw))


def test_paper_norm_flag(B):
    w = wl.make("t", 8, 4, 2, 5, seed=5)
    _, p1, _ = gpu_overlap(B, w.phi, w.Q, w.bits)
    _, p2, _ = gpu_overlap(B, w.phi, w.Q, w.bits, paper_norm=True)
    assert np.allclose(p2 * 2, p1, rtol=1e-14, atol=0)


def test_signed_permutation_closed_form_paper_size(B):
    """N = 16, eta = 8 on the paper's own ensemble: exact closed form."""
    rng = np.random.default_rng(160)
    phi = wl.walkers(rng, 2, 16, 8)
    Qs, refs, bl = [], [], []
    for _ in range(3):
        Q, perm, signs = closed_form.random_signed_permutation(rng, 16)
        b = int(wl.even_bits(rng, 1, 16)[0])
        Qs.append(Q)
        bl.append(b)
        refs.append([closed_form.overlap_pair(phi[i], perm, signs, b) for i in range(2)])
    _, pg, _ = gpu_overlap(B, phi, np.array(Qs), np.array(bl, np.uint64))
    ref = np.array(refs).T
    assert_pairs_close(pg, ref, rtol=1e-10, what="closed form")


def test_paper_sized_workload_sampled(B):
    """The full N = 16 workload (1024 walkers x 10,000 shadows) exactly as the
    benchmark runs it: the oracle checks every walker on the first 1,000
    shadows, every shadow of 16 walkers, and 512 random pairs."""
    w = wl.config("paper_n16")
    sg, pg, st = gpu_overlap(B, w.phi, w.Q, w.bits)
    assert not st.any()
    po_first = oracle.overlap_pairs(w.phi, w.Q[:1000], w.bits[:1000])
    worst = assert_pairs_close(pg[:, :1000], po_first, what="paper_n16 first 1000 shadows")
    rng = np.random.default_rng(9)
    ws = rng.choice(w.W, 16, replace=False)
    po_w = oracle.overlap_pairs(w.phi[ws], w.Q, w.bits)
    worst = max(worst, assert_pairs_close(pg[ws], po_w, what="paper_n16 walkers"))
    assert_walkers_close(sg[ws], po_w.mean(axis=1), what="paper_n16 S_w")
    pairs = np.stack([rng.integers(0, w.W, 512), rng.integers(0, w.S, 512)], axis=1)
    po = oracle.overlap_pairs(w.phi, w.Q, w.bits, pairs=pairs)
    worst = max(worst, assert_pairs_close(pg[pairs[:, 0], pairs[:, 1]], po, what="paper_n16 sample"))
    print(f"paper_n16 worst rel {worst:.2e}")
    # S_w must be the mean of the pair estimates the kernel wrote
    assert np.allclose(sg, pg.mean(axis=1), rtol=1e-12, atol=0)


def test_determinism(B):
    w = wl.make("t", 16, 8, 7, 45, seed=3)
    a = gpu_overlap(B, w.phi, w.Q, w.bits)
    b = gpu_overlap(B, w.phi, w.Q, w.bits)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_edge_cases(B):
    n, eta = 8, 4
    rng = np.random.default_rng(4)
    phi = wl.walkers(rng, 4, n, eta)
    Q = wl.haar_so(rng, 3, 2 * n)
    bits = wl.even_bits(rng, 3, n)
    # single walker, single shadow
    sg, pg, _ = gpu_overlap(B, phi[:1], Q[:1], bits[:1])
    assert_pairs_close(pg, oracle.overlap_pairs(phi[:1], Q[:1], bits[:1]), what="1x1")
    # pair-preserving shadows give exactly (to rounding) zero
    Qi = np.stack([np.eye(2 * n), np.kron(np.eye(n), [[np.cos(.4), np.sin(.4)], [-np.sin(.4), np.cos(.4)]])])
    _, pz, _ = gpu_overlap(B, phi, Qi, np.array([0, 0b1001], np.uint64))
    assert np.abs(pz).max() < 1e-13
    # non-orthonormal walker with full rank is fine
    phi2 = phi.copy()
    phi2[1] = phi2[1] @ np.array([[2.0, 0.5, 0, 0], [0, 1, 0, 0], [0, 0, 3, 1j], [0, 0, 0, 0.7]])
    _, pg2, st2 = gpu_overlap(B, phi2, Q, bits)
    assert_pairs_close(pg2, oracle.overlap_pairs(phi2, Q, bits), what="non-orthonormal")
    assert not st2.any()
    # rank-deficient walker: flagged, NaN, the other walkers unaffected
    phi3 = phi.copy()
    phi3[2][:, 3] = phi3[2][:, 1]
    sg3, pg3, st3 = gpu_overlap(B, phi3, Q, bits)
    assert st3[2] & B.SO_WSTAT_RANK and np.isnan(sg3[2]) and np.isnan(pg3[2]).all()
    assert not st3[[0, 1, 3]].any()
    assert_pairs_close(pg3[[0, 1, 3]], oracle.overlap_pairs(phi3[[0, 1, 3]], Q, bits), what="others")
    # non-finite input
    phi4 = phi.copy()
    phi4[0, 0, 0] = np.nan
    sg4, _, st4 = gpu_overlap(B, phi4, Q, bits)
    assert st4[0] & B.SO_WSTAT_NONFINITE and not np.isfinite(sg4[0])
    # a non-finite shadow reaches every walker
    Q5 = Q.copy()
    Q5[1, 0, 0] = np.nan
    sg5, _, st5 = gpu_overlap(B, phi, Q5, bits)
    assert np.all(st5 & B.SO_WSTAT_NONFINITE) and not np.isfinite(sg5).any()


def test_gpu_multilinearity_full_size(B):
    """o(Phi R) = det(R) o at the paper's size, on every pair of a slice."""
    w = wl.make("t", 16, 8, 8, 200, seed=8)
    rng = np.random.default_rng(1)
    R = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    _, p1, _ = gpu_overlap(B, w.phi, w.Q, w.bits)
    _, p2, _ = gpu_overlap(B, w.phi @ R, w.Q, w.bits)
    assert_pairs_close(p2, np.linalg.det(R) * p1, rtol=1e-9, what="multilinearity")


def test_error_paths_through_binding(B):
    w = wl.make("t", 8, 4, 2, 3, seed=2)
    phi, Q, bits = to_dev(w.phi, w.Q, w.bits)
    with pytest.raises(B.ShadowOvError) as e:
        B.shadow_overlap(phi[:, :, :3], Q, bits)          # odd eta
    assert e.value.code == B.SO_ERR_ARG
    small = torch.empty(16, dtype=torch.uint8, device=dev())
    with pytest.raises(B.ShadowOvError) as e:
        B.shadow_overlap(phi, Q, bits, workspace=small)
    assert e.value.code == B.SO_ERR_WORKSPACE
    with pytest.raises(B.ShadowOvError):
        B.shadow_overlap(phi, Q, bits, n_nodes=3)          # too few nodes for the degree


def test_occupied_elimination_growth_and_fallback(B):
    """Shadows close to a pair-preserving rotation make the occupied block
    B_OO nearly singular: mild cases stay on the elimination path, strong
    ones (growth above the threshold, or an exactly zero pivot) go through
    the full-size path; all must match the oracle."""
    import scipy.linalg as sla
    n, eta = 16, 8
    rng = np.random.default_rng(31)
    phi = wl.walkers(rng, 3, n, eta)
    Qs = []
    for eps in (3e-1, 1e-1, 1e-2, 1e-3, 1e-5, 1e-7, 0.0):
        h = rng.standard_normal((2 * n, 2 * n))
        Qs.append(sla.expm(eps * (h - h.T)))
    Qs = np.array(Qs)
    bits = wl.even_bits(rng, len(Qs), n)
    sg, pg, st = gpu_overlap(B, phi, Qs, bits)
    po = oracle.overlap_pairs(phi, Qs, bits)
    assert not st.any()
    scale = np.median(np.abs(po[:, :3]))      # the well-conditioned shadows set the scale
    err = np.abs(pg - po)
    assert np.all(err <= 1e-10 * np.maximum(np.abs(po), 1e-3 * scale)), err / np.maximum(np.abs(po), 1e-3 * scale)


def hf_walkers(rng, W, n, eta):
    """Walkers whose orbitals are single modes (Hartree-Fock-like)."""
    phi = np.zeros((W, n, eta), complex)
    for w in range(W):
        phi[w, rng.choice(n, eta, replace=False), np.arange(eta)] = 1.0
    return phi


@pytest.mark.parametrize("n,eta", [(8, 4), (9, 4)])     # fused pair kernel; two-kernel path
def test_fallback_queue_overflow_still_exact(B, n, eta):
    """Single-mode walkers with the identity shadow and b = 0 make the
    occupied rows of B exactly zero, so every pair meets a zero pivot and
    needs the full-size path: 4,800 pairs against a queue of 4,096.  The
    pairs the queue cannot hold are marked in the pair array and found by
    the full-size kernel's scan, so every pair is exact (the overlap of a
    pair-preserving shadow is zero) and no walker is flagged."""
    W, S = 48, 100
    phi = hf_walkers(np.random.default_rng(5), W, n, eta)
    Q = np.broadcast_to(np.eye(2 * n), (S, 2 * n, 2 * n)).copy()
    bits = np.zeros(S, np.uint64)
    t = to_dev(phi, Q, bits)
    out, pairs, st = B.shadow_overlap(*t, return_pairs=True)
    cnt = B.fallback_count(*t)
    pg, st = pairs.cpu().numpy(), st.cpu().numpy()
    print(f"n={n}: {cnt} of {W * S} pairs on the full-size path")
    assert cnt == W * S
    assert not st.any()
    assert np.abs(pg).max() < 1e-13


@pytest.mark.parametrize("n,eta", [(8, 4), (9, 4)])
def test_fallback_overflow_hf_walkers_signed_permutations(B, n, eta):
    """Single-mode walkers with signed-permutation shadows (the first steps
    of an AFQMC run on the paper's ensemble): many pairs need the full-size
    path, more than its queue holds; every pair against the oracle, a few
    against the closed form."""
    W, S = 64, 128
    rng = np.random.default_rng(7 + n)
    phi = hf_walkers(rng, W, n, eta)
    Qs, perms, signs = [], [], []
    for _ in range(S):
        Q, pm, sg = closed_form.random_signed_permutation(rng, n)
        Qs.append(Q), perms.append(pm), signs.append(sg)
    Q = np.array(Qs)
    bits = wl.even_bits(rng, S, n)
    t = to_dev(phi, Q, bits)
    out, pairs, st = B.shadow_overlap(*t, return_pairs=True)
    cnt = B.fallback_count(*t)
    sg_, pg, st = out.cpu().numpy(), pairs.cpu().numpy(), st.cpu().numpy()
    po = oracle.overlap_pairs(phi, Q, bits)
    print(f"n={n}: {cnt} of {W * S} pairs on the full-size path")
    assert cnt > 4096
    assert not st.any()
    scale = np.abs(po).max()
    assert np.all(np.abs(pg - po) <= 1e-10 * np.maximum(np.abs(po), 1e-3 * scale))
    for k in range(6):
        w_, s_ = int(rng.integers(W)), int(rng.integers(S))
        ref = closed_form.overlap_pair(phi[w_], perms[s_], signs[s_], int(bits[s_]))
        assert abs(pg[w_, s_] - ref) <= 1e-10 * max(abs(ref), 1e-3 * scale)
    so = po.mean(axis=1)
    assert np.all(np.abs(sg_ - so) <= 1e-10 * np.maximum(np.abs(so), 1e-3 * scale))


@pytest.mark.parametrize("n,eta,W,S", [(8, 4, 5, 37), (16, 8, 6, 41), (16, 4, 3, 19), (24, 12, 3, 11), (12, 6, 3, 9)])
def test_signed_perm_formation_same_bits(B, n, eta, W, S):
    """SO_FLAG_SIGNED_PERM: for signed-permutation shadows the gather formation
    (n = 8T) gives the bits of the matrix-core formation, whose sums have one
    nonzero term; other n ignore the flag."""
    rng = np.random.default_rng(80 + n + eta)
    phi = wl.walkers(rng, W, n, eta)
    Q = wl.signed_permutations(rng, S, 2 * n)
    bits = wl.even_bits(rng, S, n)
    t = to_dev(phi, Q, bits)
    o1, p1, s1 = B.shadow_overlap(*t, return_pairs=True)
    o2, p2, s2 = B.shadow_overlap(*t, return_pairs=True, signed_perm=True)
    torch.cuda.synchronize()
    assert torch.equal(p1, p2) and torch.equal(o1, o2) and torch.equal(s1, s2)
    po = oracle.overlap_pairs(phi, Q, bits)
    assert_pairs_close(p2.cpu().numpy(), po, what=f"signed-perm formation n={n}")


def test_signed_perm_flag_with_other_shadows_is_loud(B):
    """A shadow that is not a signed permutation under SO_FLAG_SIGNED_PERM
    gives NaN pair values and SO_WSTAT_NONFINITE; the mixed precision mode
    ignores the flag."""
    n, eta, W = 16, 8, 4
    rng = np.random.default_rng(88)
    phi = wl.walkers(rng, W, n, eta)
    Q = np.concatenate([wl.signed_permutations(rng, 5, 2 * n), wl.haar_so(rng, 1, 2 * n)])
    bits = wl.even_bits(rng, 6, n)
    t = to_dev(phi, Q, bits)
    _, pairs, st = B.shadow_overlap(*t, return_pairs=True, signed_perm=True)
    pg, st = pairs.cpu().numpy(), st.cpu().numpy()
    assert np.isnan(pg[:, 5]).all() and np.isfinite(pg[:, :5]).all()
    assert (st & B.SO_WSTAT_NONFINITE).all()
    om, _, sm = B.shadow_overlap(*t, precision="mixed", signed_perm=True)
    om2, _, _ = B.shadow_overlap(*t, precision="mixed")
    torch.cuda.synchronize()
    assert torch.equal(om, om2) and not sm.any()


def test_single_mode_walkers_signed_permutations_paper_size(B):
    """Single-mode (Hartree-Fock-like) walkers on the paper's signed-permutation
    ensemble at the paper's size (n = 16, eta = 8, 1024 walkers x 10,000
    shadows): most pairs meet a zero pivot in the reduced elimination and take
    the full-size path, far more than its queue holds.  1,000 sampled pairs
    against the oracle, 100 of them against the closed form, and S_w of 8
    walkers over all shadows against the oracle.  Many of these pairs are
    exactly zero, so the floor of the pair tolerance is taken from the nonzero
    ones."""
    n, eta, W, S = 16, 8, 1024, 10000
    rng = np.random.default_rng(1616)
    phi = hf_walkers(rng, W, n, eta)
    Q = wl.signed_permutations(rng, S, 2 * n)
    bits = wl.even_bits(rng, S, n)
    t = to_dev(phi, Q, bits)
    print("single-mode walkers x signed permutations: inputs ready", flush=True)
    out, pairs, st = B.shadow_overlap(*t, return_pairs=True)
    cnt = B.fallback_count(*t)
    assert not st.cpu().numpy().any()
    assert cnt > W * S // 2
    sw, ss = rng.integers(0, W, 1000), rng.integers(0, S, 1000)
    pg = pairs[torch.from_numpy(sw).to(dev()), torch.from_numpy(ss).to(dev())].cpu().numpy()
    sg = out.cpu().numpy()
    del pairs
    po = oracle.overlap_pairs(phi, Q, bits, pairs=np.stack([sw, ss], 1))
    nz = np.abs(po)[np.abs(po) > 0]
    floor = 1e-3 * np.median(nz)
    rel = np.abs(pg - po) / np.maximum(np.abs(po), floor)
    assert rel.max() <= RTOL, f"worst sampled pair rel {rel.max():.3e}"
    for k in range(100):
        perm = np.argmax(np.abs(Q[ss[k]]), axis=1)
        signs = Q[ss[k]][np.arange(2 * n), perm]
        ref = closed_form.overlap_pair(phi[sw[k]], perm, signs, int(bits[ss[k]]))
        assert abs(pg[k] - ref) <= RTOL * max(abs(ref), floor)
    pick = np.arange(8) * 127
    so = oracle.overlap(phi[pick], Q, bits)
    assert np.all(np.abs(sg[pick] - so) <= RTOL * np.maximum(np.abs(so), floor))
    print(f"{cnt} of {W * S} pairs on the full-size path ({cnt / (W * S):.2f}); worst sampled pair rel {rel.max():.2e}")


def test_signed_permutation_paper_workload(B):
    """The paper's own shadow ensemble at the paper's size: 1024 walkers x
    10,000 random signed permutations (n = 16, eta = 8).  2,000 sampled pairs
    against the oracle, 8 against the closed form, and S_w of 8 walkers over
    all shadows; the count of full-size pairs is reported."""
    w = wl.config("perm_n16")
    t = to_dev(w.phi, w.Q, w.bits)
    print(f"perm_n16: {w.W} x {w.S} pairs", flush=True)
    out, pairs, st = B.shadow_overlap(*t, return_pairs=True)
    cnt = B.fallback_count(*t)
    assert not st.cpu().numpy().any()
    rng = np.random.default_rng(16)
    sw, ss = rng.integers(0, w.W, 2000), rng.integers(0, w.S, 2000)
    pg = pairs[torch.from_numpy(sw).to(dev()), torch.from_numpy(ss).to(dev())].cpu().numpy()
    sg = out.cpu().numpy()
    del pairs
    po = oracle.overlap_pairs(w.phi, w.Q, w.bits, pairs=np.stack([sw, ss], 1))
    worst = assert_pairs_close(pg, po, what="perm_n16 sampled pairs")
    for k in range(8):
        Q = w.Q[ss[k]]
        perm = np.argmax(np.abs(Q), axis=1)
        signs = Q[np.arange(Q.shape[0]), perm]
        ref = closed_form.overlap_pair(w.phi[sw[k]], perm, signs, int(w.bits[ss[k]]))
        assert abs(pg[k] - ref) <= RTOL * max(abs(ref), 1e-3 * np.median(np.abs(po)))
    pick = np.arange(8) * 101
    so = oracle.overlap(w.phi[pick], w.Q, w.bits)
    assert_walkers_close(sg[pick], so, what="perm_n16 S_w")
    print(f"perm_n16: worst sampled pair rel err {worst:.2e}; {cnt} of {w.W * w.S} pairs on the full-size path")


