"""Batched problems (shadow_overlap_batched through the C ABI): a miniature of
the uneven reaction-path workload (N = 8, 12, 16, 20 qubits, eta = N/2, one
problem per geometry) must give exactly the bits of separate shadow_overlap
calls (same kernels, same node tables, same fixed-order reduction), whatever
the tuning knobs, also when captured into a graph and replayed; and the
values of the oracle, on every pair of the miniature and on sampled pairs of
the full-size workload (tolerance as for single calls: 1e-10 per pair
relative to max(|o|, 1e-3 median |o|), 1e-10 per walker)."""
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


def dev_problem(w, **kw):
    d = dict(phi=torch.from_numpy(np.ascontiguousarray(w.phi)).to(dev()),
             Q=torch.from_numpy(np.ascontiguousarray(w.Q)).to(dev()),
             bits=torch.from_numpy(np.ascontiguousarray(w.bits).view(np.int64)).to(dev()),
             return_pairs=True)
    d.update(kw)
    return d


def mini_uneven():
    """n = 8, 12, 16, 20 (eta = n/2): fused kernel classes (1, 4), (2, 6),
    (2, 8) and (3, 10); a second (2, 8) problem so that one launch
    serves two problems; and a problem on the two-kernel path (ne = 5)."""
    shapes = [(8, 4, 9, 23), (12, 6, 6, 31), (16, 8, 5, 45), (20, 10, 3, 17), (16, 8, 4, 29), (9, 4, 3, 11)]
    return [wl.make(f"u{k}", n, eta, W, S, seed=900 + k) for k, (n, eta, W, S) in enumerate(shapes)]


def single(B, pr):
    out, pairs, st = B.shadow_overlap(pr["phi"], pr["Q"], pr["bits"], return_pairs=True)
    torch.cuda.synchronize()
    return out.cpu().numpy(), pairs.cpu().numpy(), st.cpu().numpy()


def batch_results(bt):
    torch.cuda.synchronize()
    return [(bt.overlap[k].cpu().numpy(), bt.pairs[k].cpu().numpy(), bt.status[k].cpu().numpy())
            for k in range(bt.n)]


def assert_same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_batched_matches_individual_calls(B):
    probs = [dev_problem(w) for w in mini_uneven()]
    bt = B.Batch(probs)
    bt.run()
    got = batch_results(bt)
    for k, pr in enumerate(probs):
        assert_same(got[k], single(B, pr))
        assert not got[k][2].any()


def test_one_launch_per_level_gives_the_same_bits(B):
    """SO_FLAG_BATCH_BY_LEVEL (one launch per register level) changes only the
    grouping of the work items, not any pair's arithmetic."""
    ws = mini_uneven()
    one = batch_results(_run(B.Batch([dev_problem(w) for w in ws])))
    lev = batch_results(_run(B.Batch([dev_problem(w) for w in ws], by_level=True)))
    for a, b in zip(lev, one):
        assert_same(a, b)
    mixed = [dev_problem(w, precision="mixed") for w in ws]
    for a, b in zip(batch_results(_run(B.Batch(mixed, by_level=True))), batch_results(_run(B.Batch(mixed)))):
        assert_same(a, b)


def test_tuning_knobs_do_not_change_results(B):
    ws = mini_uneven()
    ref = batch_results(_run(B.Batch([dev_problem(w) for w in ws])))
    for spi, wpc in ((7, 4), (28, 16), (56, 2)):
        got = batch_results(_run(B.Batch([dev_problem(w, shadows_per_item=spi, waves_per_cu=wpc) for w in ws])))
        for a, b in zip(got, ref):
            assert_same(a, b)


def _run(bt):
    bt.run()
    return bt


def test_autotune_returns_valid_knobs(B):
    ws = mini_uneven()
    bt = B.Batch([dev_problem(w) for w in ws])
    knobs = bt.autotune()
    for w, (spi, wpc) in zip(ws, knobs):
        ne = w.n - w.eta
        if ne % 2 == 0 and 2 <= ne <= 12:
            nb = 64 // (ne + 1) if ne <= 8 else 1         # node batch of the fused kernel
            assert spi % nb == 0 and spi // nb in (1, 2, 4, 8, 16) and wpc == 0
        else:
            assert (spi, wpc) == (0, 0)
    bt.run()
    for k, got in enumerate(batch_results(bt)):
        assert_same(got, single(B, dict(phi=bt.keep[3 * k], Q=bt.keep[3 * k + 1], bits=bt.keep[3 * k + 2])))


def test_graph_capture_and_replay(B):
    ws = mini_uneven()
    probs = [dev_problem(w) for w in ws]
    bt = B.Batch(probs)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bt.run()
    torch.cuda.current_stream().wait_stream(side)
    eager = batch_results(bt)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bt.run()
    other = mini_uneven()[2]
    for rep in range(3):
        for k in range(bt.n):                      # scribble over the outputs first
            bt.overlap[k].fill_(0)
            bt.pairs[k].fill_(0)
        g.replay()
        for a, b in zip(batch_results(bt), eager):
            assert_same(a, b)
        single(B, dev_problem(other))              # eager work between replays
    # the graph reads its inputs at replay time: change a walker in place
    bt.keep[0][0].mul_(1.5)
    g.replay()
    got = batch_results(bt)
    ref0 = single(B, dict(phi=bt.keep[0], Q=bt.keep[1], bits=bt.keep[2]))
    assert_same(got[0], ref0)
    for a, b in zip(got[1:], eager[1:]):
        assert_same(a, b)


def assert_oracle_pairs(pg, po, what):
    scale = np.median(np.abs(po))
    rel = np.abs(pg - po) / np.maximum(np.abs(po), 1e-3 * scale)
    assert rel.max() <= 1e-10, f"{what}: worst rel {rel.max():.3e}"
    return rel.max()


def test_batched_matches_oracle(B):
    ws = mini_uneven()
    bt = B.Batch([dev_problem(w) for w in ws])
    bt.run()
    for k, (w, (og, pg, st)) in enumerate(zip(ws, batch_results(bt))):
        po = oracle.overlap_pairs(w.phi, w.Q, w.bits)
        worst = assert_oracle_pairs(pg, po, f"problem {k} (n={w.n})")
        so = po.mean(axis=1)
        assert np.all(np.abs(og - so) <= 1e-10 * np.abs(so))
        assert not st.any()
        print(f"problem {k} (n={w.n}, eta={w.eta}): worst pair rel err {worst:.2e}")


def test_uneven_full_size_sampled(B):
    """The four reaction-path geometries at full size (3.89e7 pairs) in one
    batched call; 1,000 sampled pairs per geometry against the oracle."""
    ws = [wl.make(f"uneven{k}", **c) for k, c in enumerate(wl.UNEVEN)]
    print("uneven: inputs ready", flush=True)
    bt = B.Batch([dev_problem(w) for w in ws])
    bt.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(33)
    for k, w in enumerate(ws):
        assert not bt.status[k].cpu().numpy().any()
        sw, ss = rng.integers(0, w.W, 1000), rng.integers(0, w.S, 1000)
        pg = bt.pairs[k][torch.from_numpy(sw).to(dev()), torch.from_numpy(ss).to(dev())].cpu().numpy()
        po = oracle.overlap_pairs(w.phi, w.Q, w.bits, pairs=np.stack([sw, ss], 1))
        worst = assert_oracle_pairs(pg, po, f"geometry n={w.n}")
        print(f"uneven n={w.n}: {w.W} x {w.S}, worst sampled pair rel err {worst:.2e}")
