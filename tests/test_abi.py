"""Host-side checks of the C ABI: the library loads without a GPU, exports
every function the header declares, validates arguments before touching the
device, and computes node weights equal to the oracle's (independent code)."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2506_22408_amd import binding as B


def test_exports_every_declared_function():
    names = B.header_functions()
    assert {"shadow_overlap", "shadow_overlap_grad", "so_workspace_size", "so_node_weights",
            "so_status_string", "so_max_n", "so_supported"} <= set(names)
    for nm in names:
        assert hasattr(B.lib, nm), nm


def test_status_strings():
    for code in (0, -1, -2, -3, -4):
        assert B.status_string(code)
    assert B.status_string(-99) == "unknown status"


@pytest.mark.parametrize("n,eta,fam", [(8, 4, "unit"), (16, 8, "unit"), (24, 12, "unit"), (20, 10, "unit"),
                                       (6, 2, "unit"), (8, 4, "chebyshev"), (16, 8, "chebyshev"),
                                       (24, 12, "chebyshev")])
def test_node_weights_match_oracle(n, eta, fam):
    z, w = B.node_weights(B.make_params(n, eta, 0, fam))
    zo, wo = oracle.node_weights(n, eta, None, fam)
    assert len(z) == n + 1
    assert np.abs(z - zo).max() < 1e-15
    scale = np.abs(wo).max()
    assert np.abs(w - wo).max() <= 1e-14 * scale


def test_node_weights_paper_norm_and_custom_K():
    z, w = B.node_weights(B.make_params(16, 8, 0, "unit", paper_norm=True))
    _, wo = oracle.node_weights(16, 8)
    assert np.allclose(w * 2, wo, rtol=1e-14, atol=0)
    z, w = B.node_weights(B.make_params(16, 8, 20))
    zo, wo = oracle.node_weights(16, 8, 20)
    assert len(w) == 20 and np.abs(w - wo).max() <= 1e-14 * np.abs(wo).max()


def test_workspace_and_support_queries():
    assert B.lib.so_max_n() >= 24
    assert B.lib.so_supported(16, 8) == 1
    assert B.lib.so_supported(24, 12) == 1
    assert B.lib.so_supported(16, 7) == 0
    assert B.lib.so_supported(8, 10) == 0
    nb = B.workspace_size(B.make_params(16, 8), 1024, 10000)
    assert nb > 1024 * 10000 * 16
    with pytest.raises(B.ShadowOvError) as e:
        B.workspace_size(B.make_params(16, 7), 4, 4)
    assert e.value.code == B.SO_ERR_ARG
    with pytest.raises(B.ShadowOvError):
        B.workspace_size(B.make_params(16, 8, n_nodes=5), 4, 4)    # fewer nodes than the degree needs


@pytest.mark.parametrize("bad", [
    dict(n=16, eta=7), dict(n=16, eta=0), dict(n=4, eta=6), dict(n=1, eta=2), dict(n=40, eta=8),
])
def test_invalid_params_rejected_before_launch(bad):
    """Validation happens on the host before any HIP call (no GPU here)."""
    p = B.make_params(bad["n"], bad["eta"])
    dummy = ctypes.c_void_p(0x1000)   # never dereferenced: the call must fail first
    st = B.lib.shadow_overlap(ctypes.byref(p), dummy, 4, dummy, dummy, 4, dummy, None, None, dummy, 1 << 30, None)
    assert st in (B.SO_ERR_ARG, B.SO_ERR_UNSUPPORTED)


def test_null_pointers_and_small_workspace_rejected():
    p = B.make_params(8, 4)
    d = ctypes.c_void_p(0x1000)
    assert B.lib.shadow_overlap(ctypes.byref(p), None, 4, d, d, 4, d, None, None, d, 1 << 30, None) == B.SO_ERR_ARG
    assert B.lib.shadow_overlap(ctypes.byref(p), d, 0, d, d, 4, d, None, None, d, 1 << 30, None) == B.SO_ERR_ARG
    assert B.lib.shadow_overlap(ctypes.byref(p), d, 4, d, d, 4, d, None, None, d, 16, None) == B.SO_ERR_WORKSPACE
    assert B.lib.shadow_overlap(ctypes.byref(p), d, 4, d, d, 4, d, None, None, None, 1 << 30, None) == B.SO_ERR_WORKSPACE
    bad = B.SoParams(8, 4, 0, 7, 0, 0)       # unknown node family
    assert B.lib.shadow_overlap(ctypes.byref(bad), d, 4, d, d, 4, d, None, None, d, 1 << 30, None) == B.SO_ERR_ARG
    bad = B.SoParams(8, 4, 0, 0, 0, 1 << 5)  # unknown flag
    assert B.lib.shadow_overlap(ctypes.byref(bad), d, 4, d, d, 4, d, None, None, d, 1 << 30, None) == B.SO_ERR_ARG


def test_host_queries_every_shape():
    """Every host-side query over every (n, eta) the library names: workspace
    sizes of each entry point, node weights of both families, batch layouts,
    and the argument checks of the entry points that need a device (they
    must fail before any HIP call).  Run against the host-sanitized build
    this sweeps the layout and table code for memory errors."""
    d = ctypes.c_void_p(0x1000)
    nb = ctypes.c_size_t(0)
    for n in range(2, 25):
        for eta in range(2, n + 1, 2):
            for fam in ("unit", "chebyshev"):
                for prec in ("fp64", "mixed"):
                    p = B.make_params(n, eta, 0, fam, prec)
                    for grad in (0, 1):
                        assert B.lib.so_workspace_size(ctypes.byref(p), 7, 13, grad, ctypes.byref(nb)) == B.SO_OK
                    z, w = B.node_weights(p)
                    assert len(z) == n + 1 and np.all(np.isfinite(w))
            p = B.make_params(n, eta)
            st = B.lib.so_local_energy_workspace_size(ctypes.byref(p), 5, 9, 3, ctypes.byref(nb))
            assert st == B.SO_OK
            probs = (B.SoProblem * 2)()
            for k in range(2):
                probs[k].params = p
                probs[k].phi, probs[k].Q, probs[k].bits, probs[k].overlap = 0x1000, 0x1000, 0x1000, 0x1000
                probs[k].n_walkers, probs[k].n_shadows = 3 + k, 11 + k
            assert B.lib.so_batch_workspace_size(probs, 2, ctypes.byref(nb)) == B.SO_OK
            # entry points that would launch: refused before any HIP call
            assert B.lib.shadow_overlap(ctypes.byref(p), d, 4, d, d, 4, d, None, None, None, 0, None) == \
                B.SO_ERR_WORKSPACE
            cnt = ctypes.c_int64(0)
            assert B.lib.so_fallback_count(ctypes.byref(p), 4, 4, None, 0, ctypes.byref(cnt), None) == \
                B.SO_ERR_WORKSPACE
    big = B.make_params(16, 8)
    assert B.lib.shadow_overlap_noalloc(ctypes.byref(big), d, 1024, d, d, 10000, d, None, None, None) == \
        B.SO_ERR_WORKSPACE
    assert B.lib.shadow_overlap_noalloc(ctypes.byref(big), None, 4, d, d, 4, d, None, None, None) == B.SO_ERR_ARG
