"""The allocation-free entry point (shadow_overlap_noalloc, through the C
ABI) against shadow_overlap: the same kernels on the library's static
scratch array, so the results must be bit for bit those of the workspace
call.  Two calls in a row, the second smaller, check that the array's
leftover contents from the first do not leak into the second; a problem
larger than the array is refused before anything runs."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2506_22408_amd import workload as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2506_22408_amd import binding
    return binding


def dev():
    return torch.device("cuda:0")


def to_dev(w):
    return (torch.from_numpy(np.ascontiguousarray(w.phi)).to(dev()),
            torch.from_numpy(np.ascontiguousarray(w.Q)).to(dev()),
            torch.from_numpy(np.ascontiguousarray(w.bits).view(np.int64)).to(dev()))


def noalloc(B, phi, Q, bits, precision="fp64"):
    """One call through the C ABI with caller-owned outputs."""
    W, n, eta = phi.shape
    S = Q.shape[0]
    out = torch.full((W,), complex(7.0, -7.0), dtype=torch.complex128, device=dev())
    pairs = torch.full((W, S), complex(3.0, 3.0), dtype=torch.complex128, device=dev())
    status = torch.full((W,), -1, dtype=torch.int32, device=dev())
    p = B.make_params(n, eta, precision=precision)
    st = B.lib.shadow_overlap_noalloc(ctypes.byref(p), ctypes.c_void_p(phi.data_ptr()), W,
                                      ctypes.c_void_p(Q.data_ptr()), ctypes.c_void_p(bits.data_ptr()), S,
                                      ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(pairs.data_ptr()),
                                      ctypes.c_void_p(status.data_ptr()),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == B.SO_OK, B.status_string(st)
    torch.cuda.synchronize()
    return out.cpu().numpy(), pairs.cpu().numpy(), status.cpu().numpy()


def reference(B, phi, Q, bits, precision="fp64"):
    out, pairs, status = B.shadow_overlap(phi, Q, bits, precision=precision, return_pairs=True)
    torch.cuda.synchronize()
    return out.cpu().numpy(), pairs.cpu().numpy(), status.cpu().numpy()


@pytest.mark.parametrize("first,second", [
    ((16, 8, 96, 400), (16, 8, 40, 130)),     # fused pair kernel, paper's (n, eta)
    ((12, 6, 50, 300), (8, 4, 13, 21)),       # two fused kernel classes
    ((9, 4, 30, 70), (9, 4, 7, 11)),          # two-kernel path (n - eta odd)
])
def test_noalloc_matches_workspace_call(B, first, second):
    for k, (n, eta, W, S) in enumerate((first, second)):
        w = wl.make(f"na{k}", n, eta, W, S, seed=4200 + 10 * n + k)
        phi, Q, bits = to_dev(w)
        got = noalloc(B, phi, Q, bits)
        ref = reference(B, phi, Q, bits)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
        assert not got[2].any()


def test_noalloc_flagged_pairs_and_mixed(B):
    """Pairs that need the full-size path (their queue counter lives in the
    scratch array and must start at zero on every call), then a mixed call."""
    n, eta, W, S = 8, 4, 20, 30
    rng = np.random.default_rng(3)
    phi = np.zeros((W, n, eta), complex)
    for k in range(W):
        phi[k, rng.choice(n, eta, replace=False), np.arange(eta)] = 1.0
    Q = np.tile(np.eye(2 * n), (S, 1, 1))
    bits = np.zeros(S, np.uint64)
    t = (torch.from_numpy(phi).to(dev()), torch.from_numpy(Q).to(dev()),
         torch.from_numpy(bits.view(np.int64)).to(dev()))
    for _ in range(2):
        got = noalloc(B, *t)
        ref = reference(B, *t)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
    w = wl.make("nam", 16, 8, 12, 50, seed=77)
    phi, Q, bits = to_dev(w)
    got = noalloc(B, phi, Q, bits, precision="mixed")
    ref = reference(B, phi, Q, bits, precision="mixed")
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_noalloc_refuses_oversized_problem(B):
    n, eta, W, S = 16, 8, 1024, 10000
    p = B.make_params(n, eta)
    need = B.workspace_size(p, W, S)
    assert need > B.NOALLOC_SCRATCH_BYTES
    phi = torch.zeros((W, n, eta), dtype=torch.complex128, device=dev())
    Q = torch.zeros((S, 2 * n, 2 * n), dtype=torch.float64, device=dev())
    bits = torch.zeros(S, dtype=torch.int64, device=dev())
    out = torch.full((W,), 5.0, dtype=torch.complex128, device=dev())
    status = torch.zeros(W, dtype=torch.int32, device=dev())
    st = B.lib.shadow_overlap_noalloc(ctypes.byref(p), ctypes.c_void_p(phi.data_ptr()), W,
                                      ctypes.c_void_p(Q.data_ptr()), ctypes.c_void_p(bits.data_ptr()), S,
                                      ctypes.c_void_p(out.data_ptr()), None, ctypes.c_void_p(status.data_ptr()),
                                      None)
    assert st == B.SO_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert torch.all(out == 5.0)          # nothing was enqueued
