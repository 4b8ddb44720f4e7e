"""ctypes binding of ``libshadowov.so`` (declared in ``include/shadowov.h``).

Argument marshalling only: every step of the estimator runs in the HIP
kernels.  PyTorch supplies device memory (tensors, the workspace) and the
current HIP stream.  There is no CPU fallback: if the library is missing the
import of this module fails.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libshadowov.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "shadowov.h")

SO_OK, SO_ERR_ARG, SO_ERR_UNSUPPORTED, SO_ERR_HIP, SO_ERR_WORKSPACE = 0, -1, -2, -3, -4
SO_NODES = {"unit": 0, "chebyshev": 1}
SO_PREC = {"fp64": 0, "mixed": 1}
SO_FLAG_PAPER_NORM = 1
SO_FLAG_LOG_OUTPUT = 2
SO_FLAG_BATCH_BY_LEVEL = 4
SO_FLAG_SIGNED_PERM = 8
SO_WSTAT_RANK, SO_WSTAT_NONFINITE, SO_WSTAT_ZERO, SO_WSTAT_FALLBACK_LOST, SO_WSTAT_SINGULAR = 1, 2, 4, 8, 16


class ShadowOvError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {status_string(code)} ({code})")
        self.code = code


class SoParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("eta", ctypes.c_int), ("n_nodes", ctypes.c_int),
                ("nodes", ctypes.c_int), ("precision", ctypes.c_int), ("flags", ctypes.c_uint)]


class SoC64(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class SoVceDims(ctypes.Structure):
    _fields_ = [("n_basis", ctypes.c_int), ("n_core", ctypes.c_int), ("n_active", ctypes.c_int),
                ("n_alpha", ctypes.c_int), ("n_beta", ctypes.c_int)]


class SoProblem(ctypes.Structure):
    _fields_ = [("params", SoParams), ("phi", ctypes.c_void_p), ("n_walkers", ctypes.c_int64),
                ("Q", ctypes.c_void_p), ("bits", ctypes.c_void_p), ("n_shadows", ctypes.c_int64),
                ("overlap", ctypes.c_void_p), ("pair_out", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("shadows_per_item", ctypes.c_int), ("waves_per_cu", ctypes.c_int)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    c = ctypes
    P = c.c_void_p
    lib.so_max_n.restype = c.c_int
    lib.so_supported.argtypes = [c.c_int, c.c_int]
    lib.so_supported.restype = c.c_int
    lib.so_workspace_size.argtypes = [c.POINTER(SoParams), c.c_int64, c.c_int64, c.c_int, c.POINTER(c.c_size_t)]
    lib.so_workspace_size.restype = c.c_int
    lib.so_node_weights.argtypes = [c.POINTER(SoParams), c.POINTER(SoC64), c.POINTER(SoC64), c.POINTER(c.c_int)]
    lib.so_node_weights.restype = c.c_int
    lib.shadow_overlap.argtypes = [c.POINTER(SoParams), P, c.c_int64, P, P, c.c_int64, P, P, P, P, c.c_size_t, P]
    lib.shadow_overlap.restype = c.c_int
    lib.shadow_overlap_noalloc.argtypes = [c.POINTER(SoParams), P, c.c_int64, P, P, c.c_int64, P, P, P, P]
    lib.shadow_overlap_noalloc.restype = c.c_int
    lib.shadow_overlap_grad.argtypes = [c.POINTER(SoParams), P, c.c_int64, P, P, c.c_int64, P, P, P, P, P,
                                        c.c_size_t, P]
    lib.shadow_overlap_grad.restype = c.c_int
    lib.so_batch_workspace_size.argtypes = [c.POINTER(SoProblem), c.c_int, c.POINTER(c.c_size_t)]
    lib.so_batch_workspace_size.restype = c.c_int
    lib.shadow_overlap_batched.argtypes = [c.POINTER(SoProblem), c.c_int, P, c.c_size_t, P]
    lib.shadow_overlap_batched.restype = c.c_int
    lib.so_autotune.argtypes = [c.POINTER(SoProblem), P, c.c_size_t, P]
    lib.so_autotune.restype = c.c_int
    lib.so_force_bias.argtypes = [c.c_void_p, c.c_int64, c.c_int, c.c_void_p, c.c_int64, c.c_double, c.c_void_p,
                                  c.c_void_p]
    lib.so_force_bias.restype = c.c_int
    lib.so_rdm1_workspace_size.argtypes = [c.c_int, c.c_int64, c.POINTER(c.c_size_t)]
    lib.so_rdm1_workspace_size.restype = c.c_int
    lib.so_rdm1.argtypes = [c.c_int, P, P, c.c_int64, c.c_int, P, P, P, c.c_size_t, P]
    lib.so_rdm1.restype = c.c_int
    lib.so_vce_walkers.argtypes = [c.POINTER(SoVceDims), P, P, c.c_int64, P, P, P]
    lib.so_vce_walkers.restype = c.c_int
    lib.so_vce_workspace_size.argtypes = [c.POINTER(SoParams), c.POINTER(SoVceDims), c.c_int64, c.c_int64,
                                          c.POINTER(c.c_size_t)]
    lib.so_vce_workspace_size.restype = c.c_int
    lib.so_vce_overlap.argtypes = [c.POINTER(SoParams), c.POINTER(SoVceDims), P, P, c.c_int64, P, P, c.c_int64,
                                   P, P, P, P, c.c_size_t, P]
    lib.so_vce_overlap.restype = c.c_int
    lib.so_local_energy_workspace_size.argtypes = [c.POINTER(SoParams), c.c_int64, c.c_int64, c.c_int,
                                                   c.POINTER(c.c_size_t)]
    lib.so_local_energy_workspace_size.restype = c.c_int
    lib.so_local_energy.argtypes = [c.POINTER(SoParams), P, c.c_int64, P, P, c.c_int64, P, P, c.c_int, P, P, P, P,
                                    P, P, P, c.c_size_t, P]
    lib.so_local_energy.restype = c.c_int
    lib.so_fallback_count.argtypes = [c.POINTER(SoParams), c.c_int64, c.c_int64, P, c.c_size_t,
                                      c.POINTER(c.c_int64), P]
    lib.so_fallback_count.restype = c.c_int
    lib.so_profile_enable.argtypes = [c.c_int]
    lib.so_profile_enable.restype = c.c_int
    lib.so_profile_read.argtypes = [c.c_int, c.POINTER(c.c_double), c.POINTER(c.c_int64), c.POINTER(c.c_int64)]
    lib.so_profile_read.restype = c.c_int
    lib.so_status_string.argtypes = [c.c_int]
    lib.so_status_string.restype = c.c_char_p
    return lib


lib = _load()


def header_functions() -> list[str]:
    """Names of the functions that include/shadowov.h declares."""
    text = open(HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:so_status|int|const char\s*\*)\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def status_string(code: int) -> str:
    return lib.so_status_string(int(code)).decode()


def make_params(n: int, eta: int, n_nodes: int = 0, nodes: str = "unit", precision: str = "fp64",
                paper_norm: bool = False, log_output: bool = False) -> SoParams:
    flags = (SO_FLAG_PAPER_NORM if paper_norm else 0) | (SO_FLAG_LOG_OUTPUT if log_output else 0)
    return SoParams(int(n), int(eta), int(n_nodes), SO_NODES[nodes], SO_PREC[precision], flags)


def workspace_size(p: SoParams, W: int, S: int, with_grad: bool = False) -> int:
    out = ctypes.c_size_t(0)
    st = lib.so_workspace_size(ctypes.byref(p), int(W), int(S), int(with_grad), ctypes.byref(out))
    if st != SO_OK:
        raise ShadowOvError(st, "so_workspace_size")
    return int(out.value)


def node_weights(p: SoParams):
    """Host copy of the nodes and weights the kernels use (complex128 numpy)."""
    import numpy as np
    z = (SoC64 * 64)()
    w = (SoC64 * 64)()
    K = ctypes.c_int(0)
    st = lib.so_node_weights(ctypes.byref(p), z, w, ctypes.byref(K))
    if st != SO_OK:
        raise ShadowOvError(st, "so_node_weights")
    k = K.value
    return (np.array([complex(z[i].re, z[i].im) for i in range(k)]),
            np.array([complex(w[i].re, w[i].im) for i in range(k)]))


PROF_PFAFF, PROF_FORM, PROF_PAIR, PROF_GRAD, PROF_RDM, PROF_VCE, PROF_ENERGY = 0, 1, 2, 3, 4, 5, 6


def profile_enable(on: bool = True) -> None:
    lib.so_profile_enable(1 if on else 0)


def profile_read(kind: int = PROF_PFAFF):
    """(milliseconds, launches, pairs) of the timed launches of one kernel kind."""
    ms = ctypes.c_double(0)
    n = ctypes.c_int64(0)
    u = ctypes.c_int64(0)
    st = lib.so_profile_read(int(kind), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(u))
    if st != SO_OK:
        raise ShadowOvError(st, "so_profile_read")
    return ms.value, n.value, u.value


def _dev_ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_inputs(phi, Q, bits):
    if not (phi.is_cuda and Q.is_cuda and bits.is_cuda):
        raise ValueError("phi, Q and bits must be device tensors")
    if phi.dtype != torch.complex128 or Q.dtype != torch.float64:
        raise TypeError("phi must be complex128 and Q float64")
    if bits.dtype not in (torch.int64, torch.uint64):
        raise TypeError("bits must be int64/uint64")
    if phi.dim() != 3 or Q.dim() != 3 or bits.dim() != 1:
        raise ValueError("phi [W,n,eta], Q [S,2n,2n], bits [S]")
    W, n, eta = phi.shape
    S = Q.shape[0]
    if Q.shape[1:] != (2 * n, 2 * n) or bits.shape[0] != S:
        raise ValueError("shape mismatch between phi, Q and bits")
    return W, n, eta, S


_ws_cache: dict = {}


def _workspace(nbytes: int, device) -> torch.Tensor:
    key = (str(device), nbytes)
    t = _ws_cache.get(key)
    if t is None:
        _ws_cache.clear()
        t = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
        _ws_cache[key] = t
    return t


def shadow_overlap(phi: torch.Tensor, Q: torch.Tensor, bits: torch.Tensor, *, n_nodes: int = 0,
                   nodes: str = "unit", precision: str = "fp64", paper_norm: bool = False,
                   log_output: bool = False, return_pairs: bool = False, signed_perm: bool = False,
                   workspace: torch.Tensor | None = None):
    """S_w = (1/S) sum_s o_ws for every walker (complex128 [W]; log S_w with
    ``log_output``); with ``return_pairs`` also the [W,S] pair estimates.
    ``signed_perm`` declares every Q_s a signed permutation (SO_FLAG_SIGNED_PERM).
    Returns (overlap, pairs or None, status int32 [W])."""
    W, n, eta, S = _check_inputs(phi, Q, bits)
    phi, Q, bits = phi.contiguous(), Q.contiguous(), bits.contiguous()
    p = make_params(n, eta, n_nodes, nodes, precision, paper_norm, log_output)
    if signed_perm:
        p.flags |= SO_FLAG_SIGNED_PERM
    nbytes = workspace_size(p, W, S)
    ws = workspace if workspace is not None else _workspace(nbytes, phi.device)
    out = torch.empty(W, dtype=torch.complex128, device=phi.device)
    pairs = torch.empty((W, S), dtype=torch.complex128, device=phi.device) if return_pairs else None
    status = torch.zeros(W, dtype=torch.int32, device=phi.device)
    stream = torch.cuda.current_stream(phi.device).cuda_stream
    st = lib.shadow_overlap(ctypes.byref(p), _dev_ptr(phi), W, _dev_ptr(Q), _dev_ptr(bits), S, _dev_ptr(out),
                            _dev_ptr(pairs), _dev_ptr(status), _dev_ptr(ws), ws.numel(),
                            ctypes.c_void_p(stream))
    if st != SO_OK:
        raise ShadowOvError(st, "shadow_overlap")
    return out, pairs, status


NOALLOC_SCRATCH_BYTES = 64 << 20   # SO_NOALLOC_SCRATCH_BYTES


def shadow_overlap_noalloc(phi: torch.Tensor, Q: torch.Tensor, bits: torch.Tensor, overlap: torch.Tensor,
                           status: torch.Tensor, pairs: torch.Tensor | None = None, *, n_nodes: int = 0,
                           nodes: str = "unit", precision: str = "fp64", paper_norm: bool = False,
                           log_output: bool = False) -> None:
    """shadow_overlap on the library's own scratch array: the caller passes
    every output (overlap complex128 [W], status int32 [W], optionally pairs
    [W, S]); nothing is allocated."""
    W, n, eta, S = _check_inputs(phi, Q, bits)
    for t, shape, dt in ((overlap, (W,), torch.complex128), (status, (W,), torch.int32)):
        if t.shape != shape or t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise ValueError("overlap must be complex128 [W] and status int32 [W], contiguous, on the device")
    if pairs is not None and (pairs.shape != (W, S) or pairs.dtype != torch.complex128 or not pairs.is_contiguous()):
        raise ValueError("pairs must be complex128 [W, S], contiguous")
    p = make_params(n, eta, n_nodes, nodes, precision, paper_norm, log_output)
    stream = torch.cuda.current_stream(phi.device).cuda_stream
    st = lib.shadow_overlap_noalloc(ctypes.byref(p), _dev_ptr(phi.contiguous()), W, _dev_ptr(Q.contiguous()),
                                    _dev_ptr(bits.contiguous()), S, _dev_ptr(overlap), _dev_ptr(pairs),
                                    _dev_ptr(status), ctypes.c_void_p(stream))
    if st != SO_OK:
        raise ShadowOvError(st, "shadow_overlap_noalloc")


def fallback_count(phi: torch.Tensor, Q: torch.Tensor, bits: torch.Tensor, *, n_nodes: int = 0,
                   nodes: str = "unit", precision: str = "fp64", workspace: torch.Tensor | None = None) -> int:
    """Pairs that the last shadow_overlap call with these shapes (and this
    workspace: by default the cached one) sent to the full-size path."""
    W, n, eta, S = _check_inputs(phi, Q, bits)
    p = make_params(n, eta, n_nodes, nodes, precision)
    ws = workspace if workspace is not None else _workspace(workspace_size(p, W, S), phi.device)
    out = ctypes.c_int64(0)
    stream = torch.cuda.current_stream(phi.device).cuda_stream
    st = lib.so_fallback_count(ctypes.byref(p), W, S, _dev_ptr(ws), ws.numel(), ctypes.byref(out),
                               ctypes.c_void_p(stream))
    if st != SO_OK:
        raise ShadowOvError(st, "so_fallback_count")
    return int(out.value)


def shadow_overlap_grad(phi: torch.Tensor, Q: torch.Tensor, bits: torch.Tensor, *, n_nodes: int = 0,
                        nodes: str = "unit", precision: str = "fp64", paper_norm: bool = False,
                        log_output: bool = False, with_green: bool = True,
                        workspace: torch.Tensor | None = None):
    """S_w, D_w = d log S_w / d Phi_w (holomorphic) and G_w = D_w Phi_w^T.
    Returns (overlap [W], dlog [W,n,eta], green [W,n,n] or None, status [W])."""
    W, n, eta, S = _check_inputs(phi, Q, bits)
    phi, Q, bits = phi.contiguous(), Q.contiguous(), bits.contiguous()
    p = make_params(n, eta, n_nodes, nodes, precision, paper_norm, log_output)
    nbytes = workspace_size(p, W, S, with_grad=True)
    ws = workspace if workspace is not None else _workspace(nbytes, phi.device)
    out = torch.empty(W, dtype=torch.complex128, device=phi.device)
    dlog = torch.empty((W, n, eta), dtype=torch.complex128, device=phi.device)
    green = torch.empty((W, n, n), dtype=torch.complex128, device=phi.device) if with_green else None
    status = torch.zeros(W, dtype=torch.int32, device=phi.device)
    stream = torch.cuda.current_stream(phi.device).cuda_stream
    st = lib.shadow_overlap_grad(ctypes.byref(p), _dev_ptr(phi), W, _dev_ptr(Q), _dev_ptr(bits), S,
                                 _dev_ptr(out), _dev_ptr(dlog), _dev_ptr(green), _dev_ptr(status),
                                 _dev_ptr(ws), ws.numel(), ctypes.c_void_p(stream))
    if st != SO_OK:
        raise ShadowOvError(st, "shadow_overlap_grad")
    return out, dlog, green, status


def force_bias(green: torch.Tensor, L: torch.Tensor, dt: float = 0.01) -> torch.Tensor:
    """xbar [W, n_gamma] = -sqrt(dt) i sum_pq L[pq, gamma] G[w, p, q] (so_force_bias)."""
    if green.dtype != torch.complex128 or L.dtype != torch.float64:
        raise TypeError("green must be complex128 and L float64")
    if not green.is_cuda or not L.is_cuda:
        raise ValueError("green and L must be device tensors")
    W, n, n2 = green.shape
    if n2 != n or L.dim() != 2 or L.shape[0] != n * n:
        raise ValueError("green must be [W, n, n] and L [n*n, n_gamma]")
    green, L = green.contiguous(), L.contiguous()
    xbar = torch.empty((W, L.shape[1]), dtype=torch.complex128, device=green.device)
    stream = torch.cuda.current_stream(green.device).cuda_stream
    st = lib.so_force_bias(_dev_ptr(green), W, n, _dev_ptr(L), L.shape[1], float(dt), _dev_ptr(xbar),
                           ctypes.c_void_p(stream))
    if st != SO_OK:
        raise ShadowOvError(st, "so_force_bias")
    return xbar


def rdm1(Q: torch.Tensor, bits: torch.Tensor, *, trial: bool = True, with_majorana: bool = False,
         workspace: torch.Tensor | None = None):
    """One-particle density matrix <a_p^dag a_q> [n, n] complex128 from the
    shadows (so_rdm1); with ``trial`` the shadows are taken to be of
    (|0> + |Psi_T>)/sqrt2 and the trial state's matrix is returned.  Returns
    (rdm, majorana [2n, 2n] float64 or None); the particle number is the
    trace of rdm."""
    if Q.dtype != torch.float64 or bits.dtype not in (torch.int64, torch.uint64):
        raise TypeError("Q must be float64 and bits 64-bit integers")
    if not Q.is_cuda or not bits.is_cuda:
        raise ValueError("Q and bits must be device tensors")
    if Q.dim() != 3 or Q.shape[1] != Q.shape[2] or Q.shape[1] % 2 or bits.shape != (Q.shape[0],):
        raise ValueError("Q must be [S, 2n, 2n] and bits [S]")
    S, n = Q.shape[0], Q.shape[1] // 2
    Q, bits = Q.contiguous(), bits.contiguous()
    nbytes = ctypes.c_size_t(0)
    st = lib.so_rdm1_workspace_size(n, S, ctypes.byref(nbytes))
    if st != SO_OK:
        raise ShadowOvError(st, "so_rdm1_workspace_size")
    ws = workspace if workspace is not None else _workspace(int(nbytes.value), Q.device)
    rdm = torch.empty((n, n), dtype=torch.complex128, device=Q.device)
    maj = torch.empty((2 * n, 2 * n), dtype=torch.float64, device=Q.device) if with_majorana else None
    stream = torch.cuda.current_stream(Q.device).cuda_stream
    st = lib.so_rdm1(n, _dev_ptr(Q), _dev_ptr(bits), S, int(bool(trial)), _dev_ptr(rdm), _dev_ptr(maj),
                     _dev_ptr(ws), ws.numel(), ctypes.c_void_p(stream))
    if st != SO_OK:
        raise ShadowOvError(st, "so_rdm1")
    return rdm, maj


def local_energy(phi: torch.Tensor, Q: torch.Tensor, bits: torch.Tensor, t: torch.Tensor, L: torch.Tensor, *,
                 paper_norm: bool = False, return_pairs: bool = False, workspace: torch.Tensor | None = None):
    """Local energies E_L = N_w / S_w (so_local_energy) for H = sum t_pq a_p^dag a_q
    + 1/2 sum_g Lhat_g^2, with t [n, n] complex128 and L [n*n, n_gamma] float64
    (each L^g real symmetric).  Returns (overlap [W], numerator [W],
    energy [W], status int32 [W]), and with ``return_pairs`` also the
    single-shadow terms (o [W, S], e [W, S])."""
    W, n, eta, S = _check_inputs(phi, Q, bits)
    if not (t.is_cuda and L.is_cuda) or t.dtype != torch.complex128 or L.dtype != torch.float64:
        raise TypeError("t must be complex128 and L float64, on the device")
    if t.shape != (n, n) or L.dim() != 2 or L.shape[0] != n * n:
        raise ValueError("t must be [n, n] and L [n*n, n_gamma]")
    phi, Q, bits, t, L = phi.contiguous(), Q.contiguous(), bits.contiguous(), t.contiguous(), L.contiguous()
    ng = L.shape[1]
    p = make_params(n, eta, 0, "unit", "fp64", paper_norm)   # the library picks the energy's own nodes
    nbytes = ctypes.c_size_t(0)
    st = lib.so_local_energy_workspace_size(ctypes.byref(p), W, S, ng, ctypes.byref(nbytes))
    if st != SO_OK:
        raise ShadowOvError(st, "so_local_energy_workspace_size")
    ws = workspace if workspace is not None else _workspace(int(nbytes.value), phi.device)
    out = [torch.empty(W, dtype=torch.complex128, device=phi.device) for _ in range(3)]
    pairs = ([torch.empty((W, S), dtype=torch.complex128, device=phi.device) for _ in range(2)]
             if return_pairs else [None, None])
    status = torch.zeros(W, dtype=torch.int32, device=phi.device)
    stream = torch.cuda.current_stream(phi.device).cuda_stream
    st = lib.so_local_energy(ctypes.byref(p), _dev_ptr(phi), W, _dev_ptr(Q), _dev_ptr(bits), S, _dev_ptr(t),
                             _dev_ptr(L) if ng else None, ng, _dev_ptr(out[0]), _dev_ptr(out[1]), _dev_ptr(out[2]),
                             _dev_ptr(pairs[0]), _dev_ptr(pairs[1]), _dev_ptr(status), _dev_ptr(ws), ws.numel(),
                             ctypes.c_void_p(stream))
    if st != SO_OK:
        raise ShadowOvError(st, "so_local_energy")
    if return_pairs:
        return out[0], out[1], out[2], status, pairs[0], pairs[1]
    return out[0], out[1], out[2], status


def _vce_inputs(phi_alpha, phi_beta, n_core, n_active):
    for t in (phi_alpha, phi_beta):
        if not t.is_cuda or t.dtype != torch.complex128 or t.dim() != 3:
            raise TypeError("phi_alpha and phi_beta must be complex128 device tensors [W, N_B, N_c + n_spin]")
    W, NB, ea = phi_alpha.shape
    if phi_beta.shape[0] != W or phi_beta.shape[1] != NB:
        raise ValueError("phi_alpha and phi_beta must share W and N_B")
    d = SoVceDims(NB, int(n_core), int(n_active), ea - int(n_core), phi_beta.shape[2] - int(n_core))
    return W, d, phi_alpha.contiguous(), phi_beta.contiguous()


def vce_walkers(phi_alpha: torch.Tensor, phi_beta: torch.Tensor, n_core: int, n_active: int):
    """Active-space walkers and prefactors of full-space walkers (so_vce_walkers).
    Returns (active_phi [W, 2 n_active, n_alpha + n_beta], prefactor [W])."""
    W, d, pa, pb = _vce_inputs(phi_alpha, phi_beta, n_core, n_active)
    act = torch.empty((W, 2 * d.n_active, d.n_alpha + d.n_beta), dtype=torch.complex128, device=pa.device)
    pref = torch.empty(W, dtype=torch.complex128, device=pa.device)
    stream = torch.cuda.current_stream(pa.device).cuda_stream
    st = lib.so_vce_walkers(ctypes.byref(d), _dev_ptr(pa), _dev_ptr(pb), W, _dev_ptr(act), _dev_ptr(pref),
                            ctypes.c_void_p(stream))
    if st != SO_OK:
        raise ShadowOvError(st, "so_vce_walkers")
    return act, pref


def vce_overlap(phi_alpha: torch.Tensor, phi_beta: torch.Tensor, n_core: int, n_active: int, Q: torch.Tensor,
                bits: torch.Tensor, *, n_nodes: int = 0, nodes: str = "unit", precision: str = "fp64",
                paper_norm: bool = False, log_output: bool = False, workspace: torch.Tensor | None = None):
    """Full-space overlaps <Psi_T|phi_w> = c_w S_w(phi~_a) (so_vce_overlap; their
    principal logarithm with ``log_output``).  Returns (overlap [W],
    prefactor [W], status int32 [W])."""
    W, d, pa, pb = _vce_inputs(phi_alpha, phi_beta, n_core, n_active)
    if not (Q.is_cuda and bits.is_cuda) or Q.dtype != torch.float64 or bits.dtype not in (torch.int64, torch.uint64):
        raise TypeError("Q must be float64 and bits 64-bit integers, on the device")
    S = Q.shape[0]
    Q, bits = Q.contiguous(), bits.contiguous()
    p = make_params(2 * d.n_active, d.n_alpha + d.n_beta, n_nodes, nodes, precision, paper_norm, log_output)
    nbytes = ctypes.c_size_t(0)
    st = lib.so_vce_workspace_size(ctypes.byref(p), ctypes.byref(d), W, S, ctypes.byref(nbytes))
    if st != SO_OK:
        raise ShadowOvError(st, "so_vce_workspace_size")
    ws = workspace if workspace is not None else _workspace(int(nbytes.value), pa.device)
    out = torch.empty(W, dtype=torch.complex128, device=pa.device)
    pref = torch.empty(W, dtype=torch.complex128, device=pa.device)
    status = torch.zeros(W, dtype=torch.int32, device=pa.device)
    stream = torch.cuda.current_stream(pa.device).cuda_stream
    st = lib.so_vce_overlap(ctypes.byref(p), ctypes.byref(d), _dev_ptr(pa), _dev_ptr(pb), W, _dev_ptr(Q),
                            _dev_ptr(bits), S, _dev_ptr(out), _dev_ptr(pref), _dev_ptr(status), _dev_ptr(ws),
                            ws.numel(), ctypes.c_void_p(stream))
    if st != SO_OK:
        raise ShadowOvError(st, "so_vce_overlap")
    return out, pref, status


class ShadowLogOverlap(torch.autograd.Function):
    """log S_w(Phi_w) for every walker, differentiable in Phi.  S_w is a
    polynomial (holomorphic) in Phi_w, so the backward pass is PyTorch's
    conjugate-Wirtinger rule for a holomorphic map: grad_phi = conj(D_w) grad_out,
    with D_w = d log S_w / d Phi_w from shadow_overlap_grad."""

    @staticmethod
    def forward(ctx, phi, Q, bits, n_nodes=0, nodes="unit"):
        logS, dlog, _, status = shadow_overlap_grad(phi.detach(), Q, bits, n_nodes=n_nodes, nodes=nodes,
                                                    log_output=True, with_green=False)
        ctx.save_for_backward(dlog)
        ctx.mark_non_differentiable(status)
        return logS, status

    @staticmethod
    def backward(ctx, grad_out, grad_status):
        (dlog,) = ctx.saved_tensors
        return torch.conj(dlog) * grad_out[:, None, None], None, None, None, None


def log_overlap(phi, Q, bits, **kw):
    """(log S_w [W], status [W]) with autograd support in phi."""
    return ShadowLogOverlap.apply(phi, Q, bits, kw.get("n_nodes", 0), kw.get("nodes", "unit"))


class Batch:
    """A batch of problems for shadow_overlap_batched with every output and
    the workspace allocated up front, so that ``run`` allocates nothing and
    may be captured into a graph.  ``problems`` is a list of dicts with keys
    phi, Q, bits (device tensors) and optionally n_nodes, nodes, precision,
    paper_norm, return_pairs, shadows_per_item, waves_per_cu.  After ``run`` (and a
    synchronisation) ``overlap[k]``, ``status[k]`` and ``pairs[k]`` hold
    problem k's results.  ``by_level`` sets SO_FLAG_BATCH_BY_LEVEL (one launch
    per register level instead of one)."""

    def __init__(self, problems, by_level: bool = False):
        if not 1 <= len(problems) <= 16:
            raise ValueError("1 to 16 problems")
        self.keep, self.overlap, self.status, self.pairs = [], [], [], []
        arr = (SoProblem * len(problems))()
        dev = None
        for k, pr in enumerate(problems):
            phi, Q, bits = pr["phi"].contiguous(), pr["Q"].contiguous(), pr["bits"].contiguous()
            W, n, eta, S = _check_inputs(phi, Q, bits)
            dev = phi.device
            out = torch.empty(W, dtype=torch.complex128, device=dev)
            st = torch.zeros(W, dtype=torch.int32, device=dev)
            pairs = torch.empty((W, S), dtype=torch.complex128, device=dev) if pr.get("return_pairs") else None
            self.keep += [phi, Q, bits]
            self.overlap.append(out)
            self.status.append(st)
            self.pairs.append(pairs)
            a = arr[k]
            a.params = make_params(n, eta, pr.get("n_nodes", 0), pr.get("nodes", "unit"),
                                   pr.get("precision", "fp64"), pr.get("paper_norm", False),
                                   pr.get("log_output", False))
            if by_level:
                a.params.flags |= SO_FLAG_BATCH_BY_LEVEL
            a.phi, a.n_walkers, a.Q, a.bits, a.n_shadows = phi.data_ptr(), W, Q.data_ptr(), bits.data_ptr(), S
            a.overlap, a.status = out.data_ptr(), st.data_ptr()
            a.pair_out = pairs.data_ptr() if pairs is not None else None
            a.shadows_per_item = int(pr.get("shadows_per_item", 0))
            a.waves_per_cu = int(pr.get("waves_per_cu", 0))
        self.arr, self.n = arr, len(problems)
        nbytes = ctypes.c_size_t(0)
        st = lib.so_batch_workspace_size(arr, self.n, ctypes.byref(nbytes))
        if st != SO_OK:
            raise ShadowOvError(st, "so_batch_workspace_size")
        self.workspace = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=dev)

    def run(self):
        stream = torch.cuda.current_stream(self.workspace.device).cuda_stream
        st = lib.shadow_overlap_batched(self.arr, self.n, _dev_ptr(self.workspace), self.workspace.numel(),
                                        ctypes.c_void_p(stream))
        if st != SO_OK:
            raise ShadowOvError(st, "shadow_overlap_batched")

    def autotune(self):
        """Run so_autotune on every problem and keep the chosen knobs; returns
        [(shadows_per_item, waves_per_cu)] per problem."""
        stream = torch.cuda.current_stream(self.workspace.device).cuda_stream
        out = []
        for k in range(self.n):
            one = (SoProblem * 1)(self.arr[k])
            nbytes = ctypes.c_size_t(0)
            st = lib.so_batch_workspace_size(one, 1, ctypes.byref(nbytes))
            if st != SO_OK:
                raise ShadowOvError(st, "so_batch_workspace_size")
            ws = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=self.workspace.device)
            st = lib.so_autotune(one, _dev_ptr(ws), ws.numel(), ctypes.c_void_p(stream))
            if st != SO_OK:
                raise ShadowOvError(st, "so_autotune")
            self.arr[k].shadows_per_item = one[0].shadows_per_item
            self.arr[k].waves_per_cu = one[0].waves_per_cu
            out.append((one[0].shadows_per_item, one[0].waves_per_cu))
        return out
