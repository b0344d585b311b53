"""Thin ctypes binding of libqsim_hip.so (the C-ABI declared in include/qsim.h).

Only argument marshalling lives here: every step of the simulation runs in the
library's HIP kernels.  PyTorch provides device memory and the stream: a
``State`` owns a ``torch.empty(2**n, dtype=complex128|complex64, device=cuda)``
buffer and passes its pointer and the current torch stream to the library.
There is no CPU fallback: if the library is missing or no GPU is present the
calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

from . import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsim_hip.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "qsim.h")

QS_C64, QS_C128 = 1, 2
QS_OK, QS_ERR_ARG, QS_ERR_DTYPE, QS_ERR_SIZE, QS_ERR_HIP, QS_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
_ERR_NAMES = {-1: "QS_ERR_ARG", -2: "QS_ERR_DTYPE", -3: "QS_ERR_SIZE", -4: "QS_ERR_HIP", -5: "QS_ERR_UNSUPPORTED"}


class QsimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class QaoaDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("p", ctypes.c_int), ("num_edges", ctypes.c_int),
                ("edges", ctypes.c_void_p), ("w", ctypes.c_void_p)]


class PoolDesc(ctypes.Structure):
    _fields_ = [("num_graphs", ctypes.c_int), ("sets_per_graph", ctypes.c_int), ("p", ctypes.c_int),
                ("n_qubits", ctypes.c_void_p), ("edge_offset", ctypes.c_void_p), ("edges", ctypes.c_void_p)]


class TrajOut(ctypes.Structure):
    _fields_ = [("z", ctypes.c_void_p), ("x", ctypes.c_void_p), ("fid", ctypes.c_void_p),
                ("prob_mean", ctypes.c_void_p), ("counts", ctypes.c_void_p), ("log", ctypes.c_void_p),
                ("log_cap", ctypes.c_int)]


_lib = None


def lib():
    """Load libqsim_hip.so once.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2001_10554_amd.build` "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        i, d, u64, i64, vp, sz = ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
        sigs = {
            "qs_state_create": [i, i, vp, sz, vp, vp],
            "qs_state_destroy": [vp],
            "qs_state_set_stream": [vp, vp],
            "qs_sync": [vp],
            "qs_init_basis": [vp, u64],
            "qs_init_uniform": [vp],
            "qs_init_random": [vp, u64],
            "qs_apply_1q": [vp, i, vp],
            "qs_apply_c1q": [vp, i, i, vp],
            "qs_apply_diag2": [vp, i, i, vp],
            "qs_apply_swap": [vp, i, i],
            "qs_apply_block": [vp, vp, i],
            "qs_apply_cut_phase": [vp, vp, vp, i, d],
            "qs_prob_one": [vp, i, vp],
            "qs_expect_z_all": [vp, vp],
            "qs_norm2": [vp, vp],
            "qs_expect_cut": [vp, vp, vp, i, vp],
            "qs_expect_diag": [vp, vp, vp],
            "qs_expect_pauli": [vp, u64, u64, vp],
            "qs_inner": [vp, vp, vp],
            "qs_sample": [vp, i64, u64, vp],
            "qs_qaoa_workspace_bytes": [vp, i, vp],
            "qs_qaoa_run": [vp, vp, i, vp, vp, vp, sz, vp],
            "qs_pool_workspace_bytes": [vp, vp],
            "qs_pool_run": [vp, vp, vp, vp, vp, sz, vp],
            "qs_traj_workspace_bytes": [i, i, i, i, vp],
            "qs_traj_run": [i, i, vp, i, u64, i, d, u64, vp, vp, sz, vp],
        }
        for name, args in sigs.items():
            f = getattr(L, name, None)
            if f is None:
                continue
            f.argtypes = args
            f.restype = ctypes.c_int
        L.qs_last_error.restype = ctypes.c_char_p
        L.qs_last_error.argtypes = []
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != QS_OK:
        raise QsimError(rc, lib().qs_last_error().decode())


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _u8(m) -> np.ndarray:
    m = np.asarray(m)
    if m.dtype == np.float64 and m.shape == (8,):
        return np.ascontiguousarray(m)
    return W.mat_to_u8(m) if m.size == 4 else np.ascontiguousarray(
        np.stack([np.asarray(m, np.complex128).real, np.asarray(m, np.complex128).imag], -1).reshape(-1))


def _ptr(a: np.ndarray) -> ctypes.c_void_p:
    return a.ctypes.data_as(ctypes.c_void_p)


def _edges(edges) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))


class State:
    """An n-qubit register in HBM (the paper's QubitRegister)."""

    def __init__(self, n: int, dtype=torch.complex128, device="cuda", stream=None, amps: torch.Tensor | None = None):
        self.n = n
        self.dtype = dtype
        code = QS_C128 if dtype == torch.complex128 else QS_C64
        if amps is None:
            amps = torch.empty(1 << n, dtype=dtype, device=device)
        self.amps = amps
        self._h = ctypes.c_void_p()
        check(lib().qs_state_create(n, code, ctypes.c_void_p(amps.data_ptr()), amps.numel() * amps.element_size(),
                                    ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().qs_state_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream=None):
        check(lib().qs_state_set_stream(self._h, ctypes.c_void_p(_stream_ptr(stream))))

    def sync(self):
        check(lib().qs_sync(self._h))

    # -- initialisation
    def init_basis(self, index: int):
        check(lib().qs_init_basis(self._h, index))
        return self

    def init_uniform(self):
        check(lib().qs_init_uniform(self._h))
        return self

    def init_random(self, seed: int):
        check(lib().qs_init_random(self._h, seed))
        return self

    # -- gates
    def apply_1q(self, q: int, m):
        u = _u8(m)
        check(lib().qs_apply_1q(self._h, q, _ptr(u)))

    def apply_c1q(self, c: int, t: int, m):
        u = _u8(m)
        check(lib().qs_apply_c1q(self._h, c, t, _ptr(u)))

    def apply_diag2(self, q0: int, q1: int, d):
        dd = np.ascontiguousarray(np.stack([np.asarray(d, np.complex128).real, np.asarray(d, np.complex128).imag], -1).reshape(-1))
        check(lib().qs_apply_diag2(self._h, q0, q1, _ptr(dd)))

    def apply_swap(self, a: int, b: int):
        check(lib().qs_apply_swap(self._h, a, b))

    def apply_block(self, gates: np.ndarray):
        g = np.ascontiguousarray(gates, dtype=W.GATE_DTYPE)
        check(lib().qs_apply_block(self._h, _ptr(g), len(g)))

    def apply_cut_phase(self, edges, gamma: float, w=None):
        e = _edges(edges)
        wa = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        check(lib().qs_apply_cut_phase(self._h, _ptr(e), None if wa is None else _ptr(wa), len(e), gamma))

    # -- read-outs (device tensors; reading them on the host synchronises)
    def _out(self, k, dtype=torch.float64):
        return torch.empty(k, dtype=dtype, device=self.amps.device)

    def prob_one(self, q: int) -> torch.Tensor:
        o = self._out(1)
        check(lib().qs_prob_one(self._h, q, ctypes.c_void_p(o.data_ptr())))
        return o

    def expect_z_all(self) -> torch.Tensor:
        o = self._out(self.n)
        check(lib().qs_expect_z_all(self._h, ctypes.c_void_p(o.data_ptr())))
        return o

    def norm2(self) -> torch.Tensor:
        o = self._out(1)
        check(lib().qs_norm2(self._h, ctypes.c_void_p(o.data_ptr())))
        return o

    def expect_cut(self, edges, w=None) -> torch.Tensor:
        e = _edges(edges)
        wa = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        o = self._out(1)
        check(lib().qs_expect_cut(self._h, _ptr(e), None if wa is None else _ptr(wa), len(e), ctypes.c_void_p(o.data_ptr())))
        return o

    def expect_diag(self, d: torch.Tensor) -> torch.Tensor:
        assert d.dtype == torch.float64 and d.is_cuda and d.numel() == 1 << self.n
        o = self._out(1)
        check(lib().qs_expect_diag(self._h, ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(o.data_ptr())))
        return o

    def expect_pauli(self, xmask: int, zmask: int) -> torch.Tensor:
        o = self._out(2)
        check(lib().qs_expect_pauli(self._h, xmask, zmask, ctypes.c_void_p(o.data_ptr())))
        return o

    def inner(self, other: "State") -> torch.Tensor:
        o = self._out(2)
        check(lib().qs_inner(self._h, other._h, ctypes.c_void_p(o.data_ptr())))
        return o

    def sample(self, shots: int, seed: int) -> torch.Tensor:
        o = self._out(max(shots, 1), torch.int64)
        check(lib().qs_sample(self._h, shots, seed, ctypes.c_void_p(o.data_ptr())))
        return o[:shots]


# ---------------------------------------------------------------- QAOA Max-Cut
class Qaoa:
    """QAOA Max-Cut instance on one graph: energies and adjoint gradients for
    batches of angle vectors [gamma_1..gamma_p, beta_1..beta_p] held on the GPU."""

    def __init__(self, n: int, edges, p: int, w=None, device="cuda"):
        self.n, self.p = n, p
        self._edges = _edges(edges)
        self._w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        self._desc = QaoaDesc(n, p, len(self._edges), self._edges.ctypes.data, None if self._w is None else self._w.ctypes.data)
        self.device = device
        self._ws = {}

    def workspace(self, with_grad: bool) -> torch.Tensor:
        if with_grad not in self._ws:
            nbytes = ctypes.c_size_t()
            check(lib().qs_qaoa_workspace_bytes(ctypes.byref(self._desc), int(with_grad), ctypes.byref(nbytes)))
            self._ws[with_grad] = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        return self._ws[with_grad]

    def run(self, angles: torch.Tensor, grad: bool = True, stream=None):
        """angles: float64 [B, 2p] or [2p] on the GPU.  Returns (E [B], grad [B, 2p] or None)."""
        a = angles.reshape(-1, 2 * self.p)
        assert a.dtype == torch.float64 and a.is_cuda
        a = a.contiguous()
        B = a.shape[0]
        E = torch.empty(B, dtype=torch.float64, device=a.device)
        G = torch.empty(B, 2 * self.p, dtype=torch.float64, device=a.device) if grad else None
        ws = self.workspace(grad)
        check(lib().qs_qaoa_run(ctypes.byref(self._desc), ctypes.c_void_p(a.data_ptr()), B, ctypes.c_void_p(E.data_ptr()),
                                ctypes.c_void_p(G.data_ptr()) if grad else None, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                ctypes.c_void_p(_stream_ptr(stream))))
        return E, G


class Pool:
    """A pool of QAOA Max-Cut circuits: graph g (with its own qubit count) times
    sets_per_graph angle vectors, circuit c = g * sets_per_graph + a.  One call
    evaluates every <C> and (optionally) every adjoint gradient; the launch
    sequence is captured into a hipGraph on the first call and replayed after."""

    def __init__(self, graphs, n_qubits, sets_per_graph: int, p: int, device="cuda", grad: bool = True, ws_bytes: int | None = None):
        self.n_qubits = np.ascontiguousarray(n_qubits, dtype=np.int32)
        self.edges = np.ascontiguousarray(np.concatenate([_edges(e) for e in graphs]).reshape(-1), dtype=np.int32)
        self.offsets = np.ascontiguousarray(np.concatenate([[0], np.cumsum([len(_edges(e)) for e in graphs])]), dtype=np.int32)
        self.sets, self.p = sets_per_graph, p
        self.count = len(graphs) * sets_per_graph
        self._desc = PoolDesc(len(graphs), sets_per_graph, p, self.n_qubits.ctypes.data, self.offsets.ctypes.data, self.edges.ctypes.data)
        if ws_bytes is None:
            nbytes = ctypes.c_size_t()
            check(lib().qs_pool_workspace_bytes(ctypes.byref(self._desc), ctypes.byref(nbytes)))
            ws_bytes = nbytes.value
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=device)
        self.angles = torch.zeros(self.count, 2 * p, dtype=torch.float64, device=device)
        self.E = torch.empty(self.count, dtype=torch.float64, device=device)
        self.G = torch.empty(self.count, 2 * p, dtype=torch.float64, device=device) if grad else None

    def run(self, angles: torch.Tensor | None = None, stream=None):
        """Copy `angles` [count, 2p] into the pool's device buffer (if given) and
        evaluate; returns (E, G) device tensors owned by the pool."""
        if angles is not None:
            self.angles.copy_(angles.reshape(self.count, 2 * self.p))
        check(lib().qs_pool_run(ctypes.byref(self._desc), ctypes.c_void_p(self.angles.data_ptr()), ctypes.c_void_p(self.E.data_ptr()),
                                ctypes.c_void_p(self.G.data_ptr()) if self.G is not None else None,
                                ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), ctypes.c_void_p(_stream_ptr(stream))))
        return self.E, self.G


def traj_run(n: int, gates: np.ndarray, basis_index: int, n_traj: int, p: float, seed: int, dtype=torch.complex128,
             log_cap: int = 0, prob_mean: bool = True, device="cuda", stream=None) -> dict:
    """Noise trajectories with stochastic Pauli insertion.  Returns device tensors:
    z, x [n_traj, n]; fid [n_traj]; counts [n_traj]; prob_mean [2^n]; log [n_traj, log_cap]."""
    g = np.ascontiguousarray(gates, dtype=W.GATE_DTYPE)
    code = QS_C128 if dtype == torch.complex128 else QS_C64
    nbytes = ctypes.c_size_t()
    check(lib().qs_traj_workspace_bytes(n, code, len(g), n_traj, ctypes.byref(nbytes)))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
    f64 = dict(dtype=torch.float64, device=device)
    res = {"z": torch.empty(n_traj, n, **f64), "x": torch.empty(n_traj, n, **f64), "fid": torch.empty(n_traj, **f64),
           "counts": torch.empty(n_traj, dtype=torch.int32, device=device)}
    if prob_mean:
        res["prob_mean"] = torch.empty(1 << n, **f64)
    if log_cap:
        res["log"] = torch.zeros(n_traj, log_cap, dtype=torch.int32, device=device)
    out = TrajOut(res["z"].data_ptr(), res["x"].data_ptr(), res["fid"].data_ptr(),
                  res["prob_mean"].data_ptr() if prob_mean else None, res["counts"].data_ptr(),
                  res["log"].data_ptr() if log_cap else None, log_cap)
    check(lib().qs_traj_run(n, code, _ptr(g), len(g), basis_index, n_traj, p, seed, ctypes.byref(out),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(_stream_ptr(stream))))
    # ws is released to torch's caching allocator in stream order: later work
    # on this stream cannot overwrite it before the kernels above have run.
    return res


class QAOAEnergy(torch.autograd.Function):
    """E(theta) = <psi(theta)|C|psi(theta)> with the adjoint gradient as backward."""

    @staticmethod
    def forward(ctx, angles: torch.Tensor, problem: Qaoa):
        E, G = problem.run(angles.detach(), grad=True)
        ctx.save_for_backward(G)
        ctx.shape = angles.shape
        return E.reshape(angles.shape[:-1]) if angles.dim() > 1 else E[0]

    @staticmethod
    def backward(ctx, gE):
        (G,) = ctx.saved_tensors
        g = gE.reshape(-1, 1) * G
        return g.reshape(ctx.shape), None
