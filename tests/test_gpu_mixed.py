"""Mixed precision (precision="mixed", through the C ABI): B = X C' X^T is
formed on the single-precision matrix cores with single-precision
accumulation, everything after it in FP64.

Tolerances.  Rounding X_w and C'_s to single precision and accumulating in
single precision perturbs B by ~1e-7 relative; the perturbation reaches a pair
value o_ws multiplied by the conditioning of its node Pfaffians, and relative
to the scale of the terms that o_ws sums, not to o_ws itself when those
cancel.  Per pair the tests hold the median relative error to 1e-6 and every
error to 1e-4 |o_ws| + 1e-6 mean_s |o_ws|; per walker
|S_w - S_w^oracle| <= 1e-6 mean_s |o_ws| (the scale of the shadow sum).  The
pairs that the elimination flags go through the full-size path in FP64.
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


def run(B, w, precision):
    out, pairs, st = B.shadow_overlap(*to_dev(w.phi, w.Q, w.bits), precision=precision, return_pairs=True)
    torch.cuda.synchronize()
    return out.cpu().numpy(), pairs.cpu().numpy(), st.cpu().numpy()


def check_mixed(S_gpu, P_gpu, P_ref):
    d = np.abs(P_gpu - P_ref)
    rel = d / np.abs(P_ref)
    scale = np.abs(P_ref).mean(axis=1)
    assert np.median(rel) <= 1e-6, f"median pair error {np.median(rel):.2e}"
    bound = 1e-4 * np.abs(P_ref) + 1e-6 * scale[:, None]
    assert np.all(d <= bound), f"largest pair error {(d / bound).max():.2f} x the bound"
    S_ref = P_ref.mean(axis=1)
    err = np.abs(S_gpu - S_ref)
    assert np.all(err <= 1e-6 * scale), f"walker error {(err / scale).max():.2e} of mean |o|"
    return rel


@pytest.mark.parametrize("n,eta,W,S", [
    (8, 4, 5, 40), (6, 2, 4, 33),                      # one tile, fused (ne = 4)
    (16, 8, 6, 70), (12, 6, 4, 50), (10, 4, 3, 41),    # two tiles, fused (ne = 8, 6, 6)
    (24, 16, 3, 30), (20, 14, 2, 17),                  # three tiles, fused (ne = 8, 6)
    (24, 12, 4, 60), (20, 10, 3, 40), (16, 4, 2, 21),  # fused, row-mapped nodes (ne = 12, 10, 12)
    (11, 4, 3, 21), (18, 2, 2, 9),                     # two-kernel path (ne = 7, 16)
])
def test_mixed_matches_oracle(B, n, eta, W, S):
    w = wl.make("mx", n, eta, W, S, seed=1000 + 7 * n + eta)
    Sg, Pg, st = run(B, w, "mixed")
    assert not st.any()
    Pref = oracle.overlap_pairs(w.phi, w.Q, w.bits)
    check_mixed(Sg, Pg, Pref)


@pytest.mark.parametrize("n,eta", [(16, 8), (24, 12)])
def test_mixed_really_rounds(B, n, eta):
    """The mixed results differ from the FP64 path by single-precision
    rounding (not by zero: the single-precision kernels ran) and stay within
    the mixed tolerance of it."""
    w = wl.make("mr", n, eta, 4, 40, seed=77 + n)
    S64, P64, st64 = run(B, w, "fp64")
    Smx, Pmx, stmx = run(B, w, "mixed")
    assert not st64.any() and not stmx.any()
    rel = np.abs(Pmx - P64) / np.abs(P64)
    assert np.median(rel) > 1e-10
    check_mixed(Smx, Pmx, P64)


def test_mixed_deterministic(B):
    w = wl.make("md", 16, 8, 3, 50, seed=5)
    a = run(B, w, "mixed")
    b = run(B, w, "mixed")
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_mixed_full_size_route(B):
    """Shadows near a pair-preserving rotation send pairs to the full-size
    path (FP64 there); the mixed results still meet the tolerance."""
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
    out, pairs, st = B.shadow_overlap(*to_dev(phi, Qs, bits), precision="mixed", return_pairs=True)
    torch.cuda.synchronize()
    assert not st.cpu().numpy().any()
    check_mixed(out.cpu().numpy(), pairs.cpu().numpy(), oracle.overlap_pairs(phi, Qs, bits))


def test_mixed_batched_matches_single_calls(B):
    """A batch holding FP64 and mixed problems of the same kernel classes:
    each result is bit for bit the single call's in its own precision."""
    shapes = [(16, 8, 4, 45, "mixed"), (16, 8, 3, 29, "fp64"), (8, 4, 5, 23, "mixed"), (24, 12, 2, 17, "mixed")]
    ws = [wl.make(f"b{k}", n, eta, W, S, seed=1300 + k) for k, (n, eta, W, S, _) in enumerate(shapes)]
    probs = []
    for w, sh in zip(ws, shapes):
        phi, Q, bits = to_dev(w.phi, w.Q, w.bits)
        probs.append(dict(phi=phi, Q=Q, bits=bits, precision=sh[4], return_pairs=True))
    bt = B.Batch(probs)
    bt.run()
    torch.cuda.synchronize()
    for k, (pr, sh) in enumerate(zip(probs, shapes)):
        out, pairs, st = B.shadow_overlap(pr["phi"], pr["Q"], pr["bits"], precision=sh[4], return_pairs=True)
        torch.cuda.synchronize()
        assert np.array_equal(bt.overlap[k].cpu().numpy(), out.cpu().numpy())
        assert np.array_equal(bt.pairs[k].cpu().numpy(), pairs.cpu().numpy())
        assert not st.cpu().numpy().any()


def test_mixed_gradient_is_refused(B):
    w = wl.make("g", 8, 4, 2, 3, seed=1)
    with pytest.raises(B.ShadowOvError) as e:
        B.shadow_overlap_grad(*to_dev(w.phi, w.Q, w.bits), precision="mixed")
    assert e.value.code == B.SO_ERR_UNSUPPORTED


def test_mixed_precision_workload_sampled(B):
    """The n = 24, eta = 12 workload at full size (2048 walkers x 50,000
    shadows) in the mixed mode, checked against the oracle on 1,000 sampled
    pairs (and against the FP64 path on the same pairs)."""
    w = wl.config("precision_n24")
    phi, Q, bits = to_dev(w.phi, w.Q, w.bits)
    outs = {}
    for prec in ("mixed", "fp64"):
        o, pairs, st = B.shadow_overlap(phi, Q, bits, precision=prec, return_pairs=True)
        torch.cuda.synchronize()
        assert not st.cpu().numpy().any()
        rng = np.random.default_rng(24)
        sw = rng.integers(0, w.W, 1000)
        ss = rng.integers(0, w.S, 1000)
        outs[prec] = pairs[torch.from_numpy(sw).to(dev()), torch.from_numpy(ss).to(dev())].cpu().numpy()
        del pairs
    ref = oracle.overlap_pairs(w.phi, w.Q, w.bits, pairs=np.stack([sw, ss], 1))
    assert np.all(np.abs(outs["fp64"] - ref) <= 1e-10 * np.abs(ref))
    d = np.abs(outs["mixed"] - ref)
    assert np.median(d / np.abs(ref)) <= 1e-6
    assert np.all(d <= 1e-4 * np.abs(ref) + 1e-6 * np.abs(ref).mean())
