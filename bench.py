#!/usr/bin/env python3
"""Benchmark: walker x shadow overlaps per second on one MI355X.

One step = one call of the whole hot path (walker prep, shadow prep, pair
formation, elimination and node Pfaffians, reduction over shadows) on the
paper-sized workload: N = 16 qubits, eta = 8 electrons, 1,024 walkers, 10,000
Haar SO(32) shadows with even-parity bitstrings, n + 1 = 17 interpolation
nodes, FP64; seeded synthetic inputs already resident in HBM.

Prints one JSON line.  ``roofline`` is for the dominant kernel, timed with
HIP events around each of its launches on the stream it runs on.  When n - eta
is even and at most 12 (the paper's N = 16, eta = 8 included) that is the
fused pair kernel ``k_pair``, whose algorithmic flops per pair are the
method's formation plus Pfaffian count, 16 n^2 m + 8 n m^2 + K (4/3) m^3
(m = 2n - eta, K = n + 1; 485k at N = 16); otherwise the node-Pfaffian kernel
with K (4/3) m^3.  The peak is the FP64 peak (vector and matrix alike 78.6
TFLOP/s).  ``cpu_baseline`` times the FP64 CPU oracle on a bounded sample of
the same workload.

Further legs (each can be skipped): ``mixed`` (the same workload with the
single-precision formation), ``precision_n24`` (FP64 and mixed on the n = 24
workload with sampled pair errors against the oracle), ``grad`` (derivative
and force bias, with its own oracle baseline), ``rdm1`` (density matrix from
the shadows, HBM-bound), ``vce`` (full-space overlaps through the
virtual-correlation-energy prologue), ``energy`` (local energies from the
second Pfaffian derivatives, with its own oracle baseline), ``perm`` (the
main workload's size on random signed-permutation shadows, with the number
of pairs that took the full-size path) and ``uneven``
(four geometries in one batched call, graph-replayed, FP64 and mixed,
beside the same call in one launch per register level and beside separate
calls).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "walker×shadow overlaps/sec at n=16 (batched/mixed vs plain FP64); grad evals/s"
PEAK_FP64_TFLOPS = 78.6     # 256 CU x 2.4 GHz x 128 FP64 flop/clk (vector and matrix alike)
CSRC = os.path.join(ROOT, "paper_2506_22408_amd", "csrc")


def pfaffian_flops_per_pair(n, eta, K):
    m = 2 * n - eta
    return K * (4.0 / 3.0) * m ** 3


def formation_flops_per_pair(n, eta):
    m = 2 * n - eta
    return 16.0 * n * n * m + 8.0 * n * m * m


def source_digest():
    """Digest of every HIP source: stored traffic figures are used only for
    the exact kernel code they were measured on."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def traffic_for_current_kernel(kernel, workload):
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic_{workload}.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_digest") != source_digest():
        return None        # counters were taken on another version of the kernel
    return t.get("bytes_per_launch")


def cpu_baseline(w, target_s=24.0):
    """The oracle on all walkers x the first few shadows.  The pilot (two
    shadows) overestimates the per-pair time about twofold, so target_s = 24
    gives a sample of roughly 10-15 s."""
    import numpy as np

    import oracle
    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    t = time.perf_counter()
    oracle.overlap_pairs(w.phi, w.Q[:2], w.bits[:2], nthreads=nthreads)
    pilot = max(time.perf_counter() - t, 1e-3) / (2 * w.W)
    s = int(max(1, min(w.S, target_s / (pilot * w.W))))
    t = time.perf_counter()
    oracle.overlap_pairs(w.phi, w.Q[:s], w.bits[:s], nthreads=nthreads)
    dt = time.perf_counter() - t
    return {"value": w.W * s / dt, "unit": "overlaps/s", "cores": nthreads, "kind": "oracle",
            "sample": f"all {w.W} walkers x first {s} of {w.S} shadows ({w.W * s} pairs, {dt:.1f} s)"}


def grad_executed_flops_per_pair(n, eta):
    """FP64 flops per pair that k_grad_pair executes in its own formulation
    (each operation counted once, although both waves form P): complex
    multiply-add = 8 flops, FP64 MFMA 16x16x4 = 2048.
      formation  (T^2 + T(T+1)/2) 4T MFMAs (U = C' Xall^T, then the upper tiles of P)
      elimination of K  rank-2 updates of the n x (n + 2ne) rows and the
                 2ne x 2ne trailing block, 2 and 3 complex products per entry
      back substitution  2ne + n right-hand sides through the n/2 pivot steps
      B_KK^{-1}  -W D W^T, n/2 terms of 2.5 complex products per entry
      nodes      ne + 1 pencil Pfaffians (ne^3/3 complex MACs) and
                 Gauss-Jordan inverses of [M_j | I] (2 ne^3 complex MACs)
      A_p, Z, Z', Abar  3 ne^2 (ne+1), 4 n ne^2 and 2 n^2 ne complex MACs
      F          T^2 4T + 2T 4T ceil(m/16) MFMAs."""
    T = -(-2 * n // 16)
    ne, KK = n - eta, 4 * T
    m, WR, KE = n + ne, n + 2 * ne, ne + 1
    nt2 = ne * (2 * ne - 1)
    TM = -(-m // 16)
    mfma = 2048.0
    form = (T * T + T * (T + 1) // 2) * KK * mfma
    elim = sum(max(0, n - k - 2) * max(0, WR - k - 2) * 16.0 + nt2 * 24.0 for k in range(0, n, 2))
    back = (2 * ne + n) * sum(16.0 * k for k in range(0, n, 2))
    binv = n * n * (n // 2) * 20.0
    nodes = KE * (8.0 * ne ** 3 / 3 + 16.0 * ne ** 3)
    asm = 8.0 * (3 * ne * ne * KE + 4 * n * ne * ne + 2 * n * n * ne)
    fmat = (T * T * KK + 2 * T * KK * TM) * mfma
    return form + elim + back + binv + nodes + asm + fmat


def grad_leg(args, B, wl, torch, np):
    """The derivative workload (N = 16, eta = 8, 1,024 walkers x 10,000
    shadows, 200 Cholesky-like vectors): one step = shadow_overlap_grad
    (S_w, d log S_w / d Phi_w, G_w) plus the force bias.  Reported as walker x
    shadow adjoint contributions per second, with walkers per second."""
    g = wl.config("grad_n16")
    dev = torch.device("cuda:0")
    phi = torch.from_numpy(g.phi).to(dev)
    Q = torch.from_numpy(g.Q).to(dev)
    bits = torch.from_numpy(g.bits.view(np.int64)).to(dev)
    L = torch.from_numpy(g.L).to(dev)
    B.shadow_overlap_grad(phi, Q, bits)
    torch.cuda.synchronize()
    B.profile_enable(True)
    B.profile_read(B.PROF_GRAD)
    t0 = time.perf_counter()
    for _ in range(args.grad_steps):
        out, dlog, green, status = B.shadow_overlap_grad(phi, Q, bits)
        xbar = B.force_bias(green, L, 0.01)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gms, glaunch, gpairs = B.profile_read(B.PROF_GRAD)
    B.profile_enable(False)
    if int(status.abs().sum()) != 0 or not bool(torch.isfinite(xbar.real).all()):
        raise RuntimeError("derivative run reported a numerical status")
    per = (t1 - t0) / args.grad_steps
    # algorithmic flops per pair: the forward count plus the adjoint by node
    # inverses, K 8 m^3, and the product of the adjoint with C' X^T, 16 n m^2
    K, m = g.n + 1, 2 * g.n - g.eta
    fl = (formation_flops_per_pair(g.n, g.eta) + pfaffian_flops_per_pair(g.n, g.eta, K) + K * 8.0 * m ** 3
          + 16.0 * g.n * m * m)
    kern_s = gms / 1e3 / glaunch
    achieved = fl * (gpairs / glaunch) / kern_s / 1e12
    flx = grad_executed_flops_per_pair(g.n, g.eta)
    executed = flx * (gpairs / glaunch) / kern_s / 1e12
    return {"metric": "grad evals/s", "value": g.W * g.S / per, "unit": "walker x shadow adjoint contributions/s",
            "walkers_per_s": g.W / per, "ms_per_step": per * 1e3, "steps": args.grad_steps,
            "config": {"workload": "grad_n16", "n": g.n, "eta": g.eta, "walkers": g.W, "shadows": g.S,
                       "n_gamma": g.L.shape[1]},
            "kernels": {"k_grad_pair": {"ms_per_step": gms / args.grad_steps}},
            "roofline": {"bound": "alu", "kernel": "k_grad_pair", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "flops_per_pair": fl,
                         "executed_flops_per_pair": flx, "executed_tflops": executed,
                         "executed_frac": executed / PEAK_FP64_TFLOPS,
                         "avg_launch_ms": kern_s * 1e3, "pairs_per_launch": gpairs / glaunch}}


def perm_leg(args, B, wl, torch, np):
    """The paper's shadow ensemble at the main workload's size: N = 16,
    eta = 8, 1,024 walkers x 10,000 random signed-permutation shadows.  The
    pairs whose elimination is flagged go through the full-size path in the
    same call; their number is reported."""
    w = wl.config("perm_n16")
    dev = torch.device("cuda:0")
    phi = torch.from_numpy(w.phi).to(dev)
    Q = torch.from_numpy(w.Q).to(dev)
    bits = torch.from_numpy(w.bits.view(np.int64)).to(dev)
    B.shadow_overlap(phi, Q, bits)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.perm_steps):
        out, _, status = B.shadow_overlap(phi, Q, bits)
    torch.cuda.synchronize()
    per = (time.perf_counter() - t0) / args.perm_steps
    flagged = B.fallback_count(phi, Q, bits)
    if int(status.abs().sum()) != 0 or not bool(torch.isfinite(out.real).all()):
        raise RuntimeError("signed-permutation run reported a numerical status")
    # the same with the gather formation (SO_FLAG_SIGNED_PERM), same bits
    out_g, _, _ = B.shadow_overlap(phi, Q, bits, signed_perm=True)
    torch.cuda.synchronize()
    if not torch.equal(out_g, out):
        raise RuntimeError("gather formation changed the overlaps")
    t0 = time.perf_counter()
    for _ in range(args.perm_steps):
        B.shadow_overlap(phi, Q, bits, signed_perm=True)
    torch.cuda.synchronize()
    per_g = (time.perf_counter() - t0) / args.perm_steps
    return {"metric": "walker x shadow overlaps/s, signed-permutation shadows", "value": w.W * w.S / per,
            "unit": "overlaps/s", "ms_per_step": per * 1e3, "steps": args.perm_steps,
            "full_size_path_pairs": flagged, "full_size_path_frac": flagged / (w.W * w.S),
            "gather_formation": {"value": w.W * w.S / per_g, "ms_per_step": per_g * 1e3,
                                 "flag": "SO_FLAG_SIGNED_PERM"},
            "config": {"workload": "perm_n16", "n": w.n, "eta": w.eta, "walkers": w.W, "shadows": w.S,
                       "shadow_family": "random signed permutations"}}


def uneven_leg(args, B, wl, torch, np):
    """Four reaction-path geometries (N = 8, 12, 16, 20, eta = N/2, walkers
    4096/2048/1024/512, shadows 2000/5000/10000/20000) in one batched call,
    autotuned, captured into a graph and replayed: total walker x shadow
    overlaps per second.  The same four problems as separate plain calls are
    timed beside it."""
    dev = torch.device("cuda:0")
    probs = []
    for c in wl.UNEVEN:
        w = wl.make("uneven", c["n"], c["eta"], c["W"], c["S"], seed=c["seed"])
        probs.append(dict(phi=torch.from_numpy(w.phi).to(dev), Q=torch.from_numpy(w.Q).to(dev),
                          bits=torch.from_numpy(w.bits.view(np.int64)).to(dev)))
    pairs = sum(c["W"] * c["S"] for c in wl.UNEVEN)
    bt = B.Batch(probs)
    knobs = bt.autotune()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bt.run()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bt.run()
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.uneven_steps):
        g.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / args.uneven_steps
    for pr in probs:
        B.shadow_overlap(pr["phi"], pr["Q"], pr["bits"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.uneven_steps):
        for pr in probs:
            B.shadow_overlap(pr["phi"], pr["Q"], pr["bits"])
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / args.uneven_steps
    for st in bt.status:
        if int(st.abs().sum()) != 0:
            raise RuntimeError("uneven batch reported a numerical status")
    # the same batch in one launch per register level (SO_FLAG_BATCH_BY_LEVEL)
    bl = B.Batch(probs, by_level=True)
    for k in range(bt.n):
        bl.arr[k].shadows_per_item = bt.arr[k].shadows_per_item
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bl.run()
    torch.cuda.current_stream().wait_stream(side)
    gl = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gl):
        bl.run()
    gl.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.uneven_steps):
        gl.replay()
    torch.cuda.synchronize()
    t_level = (time.perf_counter() - t0) / args.uneven_steps
    del gl, bl
    # the same batch with the single-precision formation, autotuned and replayed
    bm = B.Batch([dict(pr, precision="mixed") for pr in probs])
    bm.autotune()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bm.run()
    torch.cuda.current_stream().wait_stream(side)
    gm = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gm):
        bm.run()
    gm.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.uneven_steps):
        gm.replay()
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / args.uneven_steps
    return {"metric": "walker x shadow overlaps/s, uneven batch", "value": pairs / t_graph, "unit": "overlaps/s",
            "ms_per_step": t_graph * 1e3, "steps": args.uneven_steps, "pairs_per_step": pairs,
            "plain_calls": {"value": pairs / t_plain, "ms_per_step": t_plain * 1e3},
            "per_level_graph": {"value": pairs / t_level, "ms_per_step": t_level * 1e3,
                                "launches": "one per register level (2 here) instead of 1"},
            "mixed_graph": {"value": pairs / t_mixed, "ms_per_step": t_mixed * 1e3},
            "tuning": [{"n": c["n"], "shadows_per_item": k[0], "waves_per_cu": k[1]}
                       for c, k in zip(wl.UNEVEN, knobs)],
            "config": {"workload": "uneven_4_geometries", "n": [c["n"] for c in wl.UNEVEN],
                       "walkers": [c["W"] for c in wl.UNEVEN], "shadows": [c["S"] for c in wl.UNEVEN],
                       "graph": True}}


def mixed_n16_leg(args, B, torch, phi, Q, bits, pairs_per_step, out64):
    """The main workload with the formation in single precision (precision
    "mixed"): overlaps per second, and the largest |S_w - S_w^FP64| / |S_w|."""
    B.shadow_overlap(phi, Q, bits, precision="mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out, _, status = B.shadow_overlap(phi, Q, bits, precision="mixed")
    torch.cuda.synchronize()
    per = (time.perf_counter() - t0) / args.steps
    if int(status.abs().sum()) != 0:
        raise RuntimeError("mixed-precision run reported a numerical status")
    rel = ((out - out64).abs() / out64.abs()).max().item()
    return {"value": pairs_per_step / per, "unit": "overlaps/s", "ms_per_step": per * 1e3, "steps": args.steps,
            "precision": "mixed", "max_rel_diff_S_w_vs_fp64": rel}


def precision_leg(args, B, wl, torch, np):
    """The precision workload (N = 24, eta = 12, 2,048 walkers x 50,000 Haar
    SO(48) shadows): one step in FP64 and in the mixed mode, and the relative
    pair error of both against the FP64 oracle on a seeded sample of pairs
    (--precision-sample pairs; 1% of the workload is 1,024,000)."""
    import oracle
    w = wl.config("precision_n24")
    dev = torch.device("cuda:0")
    phi = torch.from_numpy(w.phi).to(dev)
    Q = torch.from_numpy(w.Q).to(dev)
    bits = torch.from_numpy(w.bits.view(np.int64)).to(dev)
    res = {"metric": "walker x shadow overlaps/s, n=24", "unit": "overlaps/s",
           "config": {"workload": "precision_n24", "n": w.n, "eta": w.eta, "walkers": w.W, "shadows": w.S,
                      "nodes": w.n + 1}}
    rng = np.random.default_rng(2024)
    ns = int(min(args.precision_sample, w.W * w.S))
    flat = rng.choice(w.W * w.S, size=ns, replace=False)
    sw, ss = flat // w.S, flat % w.S
    sample = {}
    for prec in ("fp64", "mixed"):
        B.shadow_overlap(phi, Q, bits, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.precision_steps):
            out, _, status = B.shadow_overlap(phi, Q, bits, precision=prec)
        torch.cuda.synchronize()
        per = (time.perf_counter() - t0) / args.precision_steps
        if int(status.abs().sum()) != 0:
            raise RuntimeError(f"n=24 {prec} run reported a numerical status")
        res[prec] = {"value": w.W * w.S / per, "ms_per_step": per * 1e3, "steps": args.precision_steps}
        _, pairs, _ = B.shadow_overlap(phi, Q, bits, precision=prec, return_pairs=True)
        sample[prec] = pairs[torch.from_numpy(sw).to(dev), torch.from_numpy(ss).to(dev)].cpu().numpy()
        del pairs
        torch.cuda.empty_cache()
    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    ref = np.empty(ns, np.complex128)
    chunk = 20000
    t0 = time.perf_counter()
    for a in range(0, ns, chunk):
        b = min(ns, a + chunk)
        ref[a:b] = oracle.overlap_pairs(w.phi, w.Q, w.bits, pairs=np.stack([sw[a:b], ss[a:b]], 1),
                                        nthreads=nthreads)
        if ns > chunk:
            print(f"precision leg: oracle {b}/{ns} pairs, {time.perf_counter() - t0:.0f} s", file=sys.stderr,
                  flush=True)
    scale = float(np.abs(ref).mean())
    for prec in ("fp64", "mixed"):
        err = np.abs(sample[prec] - ref)
        rel = err / np.abs(ref)
        res[prec]["pair_rel_err"] = {"median": float(np.median(rel)), "p99": float(np.quantile(rel, 0.99)),
                                     "max": float(rel.max()), "frac_le_1e-6": float(np.mean(rel <= 1e-6)),
                                     "max_err_over_mean_abs_o": float(err.max() / scale)}
    res["sample"] = f"{ns} pairs drawn uniformly without replacement (seed 2024) of {w.W * w.S}"
    res["value"] = res["mixed"]["value"]
    res["speedup_mixed_vs_fp64"] = res["mixed"]["value"] / res["fp64"]["value"]
    return res


def rdm_leg(args, B, wl, torch, np, Q16, bits16):
    """The one-particle density matrix from the shadows (so_rdm1): the
    10,000 shadows of the main workload and the 50,000 of the n = 24 one.
    Bound by HBM: the kernel reads every element of Q once, so the achieved
    bandwidth is 8 (2n)^2 S bytes over the reduction kernel's time."""
    out = {}
    dev = torch.device("cuda:0")
    cases = [("paper_n16", Q16, bits16)]
    w24 = wl.config("precision_n24")
    cases.append(("precision_n24", torch.from_numpy(w24.Q).to(dev), torch.from_numpy(w24.bits.view(np.int64)).to(dev)))
    for name, Q, bits in cases:
        S, d = Q.shape[0], Q.shape[1]
        B.rdm1(Q, bits)
        torch.cuda.synchronize()
        B.profile_enable(True)
        B.profile_read(B.PROF_RDM)
        t0 = time.perf_counter()
        for _ in range(args.rdm_steps):
            G, _ = B.rdm1(Q, bits)
        torch.cuda.synchronize()
        per = (time.perf_counter() - t0) / args.rdm_steps
        ms, launches, _ = B.profile_read(B.PROF_RDM)
        B.profile_enable(False)
        kern_s = ms / 1e3 / launches
        qbytes = 8.0 * d * d * S
        out[name] = {"ms_per_call": per * 1e3, "kernel_ms": kern_s * 1e3, "shadows": S, "n": d // 2,
                     "particle_number_trial": float(torch.trace(G).real),
                     "roofline": {"bound": "hbm", "kernel": "k_rdm_partial", "achieved": qbytes / kern_s / 1e9,
                                  "peak": 8000.0, "unit": "GB/s", "frac": qbytes / kern_s / 1e9 / 8000.0}}
    return {"metric": "one-particle density matrix from shadows", "steps": args.rdm_steps, "cases": out}


def vce_leg(args, B, wl, torch, np):
    """Full-space overlaps through the virtual-correlation-energy prologue
    (so_vce_overlap): N_B = 130 spatial orbitals, 46 core, the (8e, 8o)
    active space, 1,024 walkers x 10,000 shadows.  One step = the prologue
    kernel (active walkers and prefactors), the active-space overlap path and
    the prefactor scaling.  The prologue reads the core and active rows of
    each spin once, (N_c + N_a)(N_c + n_spin) complex entries, and writes the
    active walker and the prefactor; its achieved bandwidth is those bytes
    over its launch time (it is latency-bound: a chain of reflections per
    walker)."""
    dev = torch.device("cuda:0")
    w = wl.vce_config("vce_n16")
    pa = torch.from_numpy(w.phi_alpha).to(dev)
    pb = torch.from_numpy(w.phi_beta).to(dev)
    Q = torch.from_numpy(w.Q).to(dev)
    bits = torch.from_numpy(w.bits.view(np.int64)).to(dev)
    B.vce_overlap(pa, pb, w.n_core, w.n_active, Q, bits)
    torch.cuda.synchronize()
    B.profile_enable(True)
    for k in (B.PROF_VCE, B.PROF_PAIR):
        B.profile_read(k)
    t0 = time.perf_counter()
    for _ in range(args.vce_steps):
        o, pref, st = B.vce_overlap(pa, pb, w.n_core, w.n_active, Q, bits)
    torch.cuda.synchronize()
    per = (time.perf_counter() - t0) / args.vce_steps
    ms_v, l_v, units_v = B.profile_read(B.PROF_VCE)
    ms_p, l_p, _ = B.profile_read(B.PROF_PAIR)
    B.profile_enable(False)
    if int(st.abs().sum()) != 0 or not bool(torch.isfinite(o.real).all()):
        raise RuntimeError("VCE run reported a numerical status")
    nc, na = w.n_core, w.n_active
    per_walker = 16 * ((nc + na) * (nc + w.n_alpha) + (nc + na) * (nc + w.n_beta) + 2 * na * w.eta + 1)
    pro_s = ms_v / 1e3 / l_v
    gbs = per_walker * (units_v / l_v) / pro_s / 1e9
    return {"metric": "full-space (VCE) walker×shadow overlaps/s", "value": w.W * w.S / per, "unit": "overlaps/s",
            "steps": args.vce_steps, "ms_per_step": per * 1e3,
            "config": {"workload": "vce_n16", "n_basis": w.n_basis, "n_core": nc, "n_active": na,
                       "n_alpha": w.n_alpha, "n_beta": w.n_beta, "walkers": w.W, "shadows": w.S},
            "prologue": {"kernel": "k_vce_prep", "ms": pro_s * 1e3, "walkers_per_s": (units_v / l_v) / pro_s,
                         "bytes_per_walker": per_walker,
                         "roofline": {"bound": "latency", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                                      "frac": gbs / 8000.0}},
            "k_pair_ms": ms_p / l_p if l_p else None,
            "prologue_share": pro_s / per}


def energy_flops_per_pair(n, eta, K):
    """FP64 flops per walker x shadow pair of the local-energy kernel's own
    formulation (complex multiply-add = 8, real x complex = 4): formation, and
    per node the Pfaffian elimination (m^3/3 complex MACs) with X carried as
    right-hand sides and the back substitution (m^2 d together), X^T A^{-1} X,
    C' Yt and the W blocks, the two traces, and the
    n^4 contraction with V (the block sums sum_sp V Z^(sp) and sum_sp V Yt^(sp),
    eight real x complex products, and the square term's one: 36 flops per
    (p, q, r, s))."""
    m, d = 2 * n - eta, 2 * n
    node = (8 * m ** 3 / 3 + 8 * m * m * d + 8 * m * d * d + 4 * d ** 3 + 4 * d ** 3
            + 36 * n ** 4 + 12 * d * d)
    return 8 * m * d * d + 8 * m * m * d + K * node


def energy_leg(args, B, wl, torch, np):
    """Local energies (so_local_energy) on n = 16, eta = 8, 128 walkers x
    1,000 shadows, 200 Cholesky-like vectors and a one-body matrix: per pair
    n - eta + 1 = 9 nodes, each with a Pfaffian, a solve and an n^4
    contraction.  Value = walker x shadow local-energy terms per second."""
    dev = torch.device("cuda:0")
    w = wl.config("energy_n16")
    ts = [torch.from_numpy(x).to(dev) for x in (w.phi, w.Q, w.bits.view(np.int64), w.t, w.L)]
    S_, N_, E_, st = B.local_energy(*ts)
    torch.cuda.synchronize()
    B.profile_enable(True)
    B.profile_read(B.PROF_ENERGY)
    t0 = time.perf_counter()
    for _ in range(args.energy_steps):
        S_, N_, E_, st = B.local_energy(*ts)
    torch.cuda.synchronize()
    per = (time.perf_counter() - t0) / args.energy_steps
    ms, launches, units = B.profile_read(B.PROF_ENERGY)
    B.profile_enable(False)
    if int(st.abs().sum()) != 0 or not bool(torch.isfinite(E_.real).all()):
        raise RuntimeError("local-energy run reported a numerical status")
    # the algorithmic count takes the paper's K = n + 1 nodes (as the main
    # roofline does); the kernel evaluates n - eta + 1 (executed_frac)
    K, Kx = w.n + 1, w.n - w.eta + 1
    fl = energy_flops_per_pair(w.n, w.eta, K)
    flx = energy_flops_per_pair(w.n, w.eta, Kx)
    kern_s = ms / 1e3 / launches
    achieved = fl * (units / launches) / kern_s / 1e12
    executed = flx * (units / launches) / kern_s / 1e12
    rec = {"metric": "walker×shadow local-energy terms/s", "value": w.W * w.S / per, "unit": "pairs/s",
           "steps": args.energy_steps, "ms_per_step": per * 1e3, "dtype": "f64",
           "config": {"workload": "energy_n16", "n": w.n, "eta": w.eta, "walkers": w.W, "shadows": w.S,
                      "n_gamma": w.L.shape[1], "nodes_algorithmic": K, "nodes_executed": Kx,
                      "node_family": "unit circle, a third of a step off the roots of unity"},
           "mean_energy_real": float(E_.real.mean()),
           "roofline": {"bound": "alu", "kernel": "k_energy_pair", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                        "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "flops_per_pair": fl,
                        "executed_tflops": executed, "executed_frac": executed / PEAK_FP64_TFLOPS,
                        "avg_launch_ms": kern_s * 1e3, "pairs_per_launch": units / launches}}
    # context: the same call at 24 modes (three 16-column tiles), timed on the
    # pair kernel's own launches
    w24 = wl.config("energy_n24")
    t24 = [torch.from_numpy(x).to(dev) for x in (w24.phi, w24.Q, w24.bits.view(np.int64), w24.t, w24.L)]
    B.local_energy(*t24)
    torch.cuda.synchronize()
    B.profile_enable(True)
    B.profile_read(B.PROF_ENERGY)
    for _ in range(2):
        S_, N_, E_, st = B.local_energy(*t24)
    torch.cuda.synchronize()
    ms24, l24, u24 = B.profile_read(B.PROF_ENERGY)
    B.profile_enable(False)
    if int(st.abs().sum()) != 0 or not bool(torch.isfinite(E_.real).all()):
        raise RuntimeError("local-energy run at 24 modes reported a numerical status")
    rec["n24"] = {"workload": "energy_n24", "n": w24.n, "eta": w24.eta, "walkers": w24.W, "shadows": w24.S,
                  "n_gamma": w24.L.shape[1], "nodes_executed": w24.n - w24.eta + 1,
                  "pair_kernel_ms": ms24 / l24, "pairs_per_s": (u24 / l24) / (ms24 / l24 / 1e3)}
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_energy_baseline(w, np)
    return rec


def cpu_energy_baseline(w, np, target_s=10.0):
    """The oracle's local-energy route (per Cholesky vector, eq.
    Pfaffian_2nd_der with m x m products) on the first pairs of the same
    workload (walker-major), sized from a 16-pair pilot to about target_s
    seconds on all host threads."""
    import oracle
    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    allp = np.stack([np.arange(w.W * w.S) // w.S, np.arange(w.W * w.S) % w.S], 1)
    t = time.perf_counter()
    oracle.energy_pairs(w.phi, w.Q, w.bits, w.t, w.L, pairs=allp[:16], nthreads=nthreads)
    pilot = max(time.perf_counter() - t, 1e-3) / 16
    npairs = int(max(16, min(len(allp), target_s / pilot)))
    t = time.perf_counter()
    oracle.energy_pairs(w.phi, w.Q, w.bits, w.t, w.L, pairs=allp[:npairs], nthreads=nthreads)
    dt = time.perf_counter() - t
    return {"value": npairs / dt, "unit": "pairs/s", "cores": nthreads, "kind": "oracle",
            "sample": f"the first {npairs} walker x shadow pairs of energy_n16 ({dt:.1f} s)"}


def cpu_grad_baseline(wl, target_s=15.0):
    """The oracle's gradient on 16 walkers (one per host thread on the GPU
    host) x the first s shadows, s sized from a 64-shadow pilot to about
    target_s seconds."""
    import oracle
    g = wl.config("grad_n16")
    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    Wb, sp = 16, 64
    t = time.perf_counter()
    oracle.grad(g.phi[:Wb], g.Q[:sp], g.bits[:sp], nthreads=nthreads)
    pilot = max(time.perf_counter() - t, 1e-3) / (sp * Wb)
    s = int(max(sp, min(g.S, target_s / (pilot * Wb))))
    t = time.perf_counter()
    oracle.grad(g.phi[:Wb], g.Q[:s], g.bits[:s], nthreads=nthreads)
    dt = time.perf_counter() - t
    return {"value": Wb * s / dt, "unit": "walker x shadow adjoint contributions/s", "cores": nthreads,
            "kind": "oracle", "sample": f"{Wb} walkers x first {s} of {g.S} shadows ({Wb * s} pairs, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="paper_n16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-grad", action="store_true", help="skip the derivative leg")
    ap.add_argument("--grad-steps", type=int, default=2)
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-batch leg")
    ap.add_argument("--no-perm", action="store_true", help="skip the signed-permutation leg")
    ap.add_argument("--perm-steps", type=int, default=3)
    ap.add_argument("--uneven-steps", type=int, default=3)
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision legs")
    ap.add_argument("--no-rdm", action="store_true", help="skip the density-matrix leg")
    ap.add_argument("--rdm-steps", type=int, default=5)
    ap.add_argument("--no-vce", action="store_true", help="skip the full-space (VCE) leg")
    ap.add_argument("--no-energy", action="store_true", help="skip the local-energy leg")
    ap.add_argument("--energy-steps", type=int, default=2)
    ap.add_argument("--vce-steps", type=int, default=3)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES bytes device to device, three times (scales the HBM counters)")
    ap.add_argument("--precision-steps", type=int, default=2)
    ap.add_argument("--precision-sample", type=int, default=2000,
                    help="pairs of the n=24 workload checked against the oracle")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this benchmark measures one MI355X only; multi-GPU runs are not part of it "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world})", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "copies": 3}), flush=True)
        return

    from paper_2506_22408_amd import binding as B
    from paper_2506_22408_amd import workload as wl

    w = wl.config(args.workload)
    K = w.n + 1
    dev = torch.device("cuda:0")
    phi = torch.from_numpy(w.phi).to(dev)
    Q = torch.from_numpy(w.Q).to(dev)
    bits = torch.from_numpy(w.bits.view(np.int64)).to(dev)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        B.shadow_overlap(phi, Q, bits)
    torch.cuda.synchronize()

    kinds = {B.PROF_PAIR: "k_pair", B.PROF_PFAFF: "k_nodes", B.PROF_FORM: "k_form_mfma"}
    B.profile_enable(True)
    for k in kinds:
        B.profile_read(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out, _, status = B.shadow_overlap(phi, Q, bits)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {k: B.profile_read(k) for k in kinds}     # (ms, launches, pairs)
    B.profile_enable(False)
    if int(status.abs().sum()) != 0 or not bool(torch.isfinite(out.real).all()):
        raise RuntimeError("benchmark run reported a numerical status")

    elapsed = t1 - t0
    pairs_per_step = w.W * w.S
    value = pairs_per_step * args.steps / elapsed
    pf_flops = pfaffian_flops_per_pair(w.n, w.eta, K)
    fm_flops = formation_flops_per_pair(w.n, w.eta)
    flops = {B.PROF_PAIR: pf_flops + fm_flops, B.PROF_PFAFF: pf_flops, B.PROF_FORM: fm_flops}
    kernels = {}
    for k, name in kinds.items():
        ms, launches, pairs = prof[k]
        if launches:
            kernels[name] = {"ms_per_step": ms / args.steps, "launches_per_step": launches / args.steps,
                             "tflops": flops[k] * pairs / (ms / 1e3) / 1e12}
    dom = max((k for k in kinds if prof[k][1]), key=lambda k: prof[k][0])
    ms, launches, pairs = prof[dom]
    avg_s = ms / 1e3 / launches
    achieved = flops[dom] * (pairs / launches) / avg_s / 1e12
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "overlaps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Haar SO(2n) shadows, even-parity bits, QR-orthonormal Gaussian walkers)",
        "config": {"workload": args.workload, "n": w.n, "eta": w.eta, "walkers": w.W, "shadows": w.S,
                   "nodes": K, "node_family": "unit", "precision": "fp64"},
        "roofline": {
            "bound": "alu",
            "kernel": kinds[dom],
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": traffic_for_current_kernel(kinds[dom], args.workload),
            "flops_per_pair": flops[dom],
            "pairs_per_launch": pairs / launches,
            "avg_launch_ms": avg_s * 1e3,
            "launches": launches,
        },
        "kernels": kernels,
        "path": {"flops_per_pair": pf_flops + fm_flops, "tflops": (pf_flops + fm_flops) * value / 1e12,
                 "frac": (pf_flops + fm_flops) * value / 1e12 / PEAK_FP64_TFLOPS},
    }
    t_start = time.perf_counter()

    def leg(key, fn, *a):
        rec[key] = fn(*a)
        print(f"bench: {key} leg done ({time.perf_counter() - t_start:.0f} s)", file=sys.stderr, flush=True)

    print(f"bench: main leg done, {rec['ms_per_step']:.1f} ms per step", file=sys.stderr, flush=True)
    if not args.no_mixed:
        leg("mixed", mixed_n16_leg, args, B, torch, phi, Q, bits, pairs_per_step, out)
        leg("precision_n24", precision_leg, args, B, wl, torch, np)
    if not args.no_grad:
        leg("grad", grad_leg, args, B, wl, torch, np)
    if not args.no_rdm:
        leg("rdm1", rdm_leg, args, B, wl, torch, np, Q, bits)
    if not args.no_vce:
        leg("vce", vce_leg, args, B, wl, torch, np)
    if not args.no_energy:
        leg("energy", energy_leg, args, B, wl, torch, np)
    if not args.no_perm:
        leg("perm", perm_leg, args, B, wl, torch, np)
    if not args.no_uneven:
        leg("uneven", uneven_leg, args, B, wl, torch, np)
    if not args.no_cpu_baseline:
        leg("cpu_baseline", cpu_baseline, w)
        if "grad" in rec:
            rec["grad"]["cpu_baseline"] = cpu_grad_baseline(wl)
            print("bench: grad cpu baseline done", file=sys.stderr, flush=True)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
