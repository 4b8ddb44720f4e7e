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
