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
import math
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

from . import gates as G
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


class PsoSwarm(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("pos", "vel", "pbest", "pbest_val", "gbest", "gbest_val", "E")]


class PsoParams(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("phi_p", ctypes.c_double), ("phi_g", ctypes.c_double), ("attract", ctypes.c_int)]


class TrajOut(ctypes.Structure):
    _fields_ = [("z", ctypes.c_void_p), ("x", ctypes.c_void_p), ("fid", ctypes.c_void_p),
                ("prob_mean", ctypes.c_void_p), ("counts", ctypes.c_void_p), ("log", ctypes.c_void_p),
                ("log_cap", ctypes.c_int), ("diag", ctypes.c_void_p), ("diag_val", ctypes.c_void_p)]


class Noise(ctypes.Structure):
    _fields_ = [("p_depol", ctypes.c_double), ("T1", ctypes.c_double), ("T2", ctypes.c_double)]


_lib = None
_exiting = False


def _mark_exit():
    global _exiting
    _exiting = True


import atexit  # noqa: E402

atexit.register(_mark_exit)  # no library calls from finalisers once the interpreter is shutting down


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
            "qs_apply_kq": [vp, vp, i, vp],
            "qs_collapse": [vp, i, i, vp],
            "qs_measure": [vp, i, u64, vp, vp],
            "qs_apply_block": [vp, vp, i],
            "qs_block_passes": [i, i, vp, i, vp],
            "qs_apply_cut_phase": [vp, vp, vp, i, d],
            "qs_prob_one": [vp, i, vp],
            "qs_expect_z_all": [vp, vp],
            "qs_norm2": [vp, vp],
            "qs_expect_cut": [vp, vp, vp, i, vp],
            "qs_expect_diag": [vp, vp, vp],
            "qs_expect_pauli": [vp, u64, u64, vp],
            "qs_inner": [vp, vp, vp],
            "qs_sample": [vp, i64, u64, vp],
            "qs_sample_noalloc": [i, i, vp, sz, i64, u64, vp, vp],
            "qs_qaoa_workspace_bytes": [vp, i, vp],
            "qs_qaoa_run": [vp, vp, i, vp, vp, vp, sz, vp],
            "qs_pool_workspace_bytes": [vp, vp],
            "qs_pool_run": [vp, vp, vp, vp, vp, sz, vp],
            "qs_pool_release": [vp, vp, vp, vp, vp, sz],
            "qs_pool_circuit_bytes": [vp, i, vp],
            "qs_cut_max": [vp, vp, vp, vp, vp],
            "qs_pso_init": [vp, u64, vp, vp],
            "qs_pso_step": [vp, vp, i, i, u64, vp, vp, vp],
            "qs_pso_run": [vp, vp, i, u64, vp, vp, vp, sz, vp],
            "qs_traj_workspace_bytes": [i, i, i, i, vp],
            "qs_traj_run": [i, i, vp, i, u64, i, d, u64, vp, vp, sz, vp],
            "qs_traj_run_noise": [i, i, vp, i, u64, i, vp, u64, vp, vp, sz, vp],
            "qs_traj_noise_workspace_bytes": [i, i, vp, i, i, vp],
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


def _begin(stream=None):
    """The stream a call runs on.  A stream other than the current one first
    waits for the current stream's queued work (the call's inputs may be
    produced there); allocate the call's buffers under it."""
    cur = torch.cuda.current_stream()
    if stream is None or stream == cur:
        return cur
    stream.wait_stream(cur)
    return stream


def _finish(s, outputs=()):
    """After a call queued on stream s: the current stream waits for it, so its
    readers see the outputs, and the outputs are marked as used there (the
    caching allocator then keeps them until that stream's work is done)."""
    cur = torch.cuda.current_stream()
    if s != cur:
        cur.wait_stream(s)
        for t in outputs:
            if t is not None:
                t.record_stream(cur)


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
        self._stream = stream if stream is not None else torch.cuda.current_stream()
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
        self._stream = stream if stream is not None else torch.cuda.current_stream()
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

    def apply_kq(self, qubits, m):
        """Dense k-qubit matrix m (2^k x 2^k, row = output), 1 <= k <= 5; bit j
        of its row/column index is the value of qubits[j]."""
        qs = np.ascontiguousarray(qubits, dtype=np.int32)
        mm = np.ascontiguousarray(np.asarray(m, dtype=np.complex128))
        with torch.cuda.stream(self._stream):  # the matrix is copied and then read on the state's stream
            u = torch.view_as_real(torch.from_numpy(mm)).reshape(-1).to(self.amps.device)
        check(lib().qs_apply_kq(self._h, _ptr(qs), len(qs), ctypes.c_void_p(u.data_ptr())))
        u.record_stream(self._stream)  # not reused before the gate has run

    def collapse(self, q: int, outcome: int) -> torch.Tensor:
        """Project qubit q onto `outcome` and renormalise; returns P(outcome) (device)."""
        o = self._out(1)
        check(lib().qs_collapse(self._h, q, outcome, ctypes.c_void_p(o.data_ptr())))
        return self._done(o)

    def measure(self, q: int, seed: int):
        """Born-rule measurement of qubit q (decided on the device); returns
        (outcome int32 [1], its probability float64 [1]) device tensors."""
        out = self._out(1, torch.int32)
        pr = self._out(1)
        check(lib().qs_measure(self._h, q, seed, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(pr.data_ptr())))
        return self._done(out, pr)

    # -- named gates (matrices from the gates module; every one runs the C-ABI gate kernels)
    def h(self, q): self.apply_1q(q, G.H); return self
    def x(self, q): self.apply_1q(q, G.X); return self
    def y(self, q): self.apply_1q(q, G.Y); return self
    def z(self, q): self.apply_1q(q, G.Z); return self
    def s(self, q): self.apply_1q(q, G.S); return self
    def sdg(self, q): self.apply_1q(q, G.SDG); return self
    def t(self, q): self.apply_1q(q, G.T); return self
    def tdg(self, q): self.apply_1q(q, G.TDG); return self
    def sx(self, q): self.apply_1q(q, G.SX); return self
    def rx(self, q, theta): self.apply_1q(q, G.rx(theta)); return self
    def ry(self, q, theta): self.apply_1q(q, G.ry(theta)); return self
    def rz(self, q, theta): self.apply_1q(q, G.rz(theta)); return self
    def phase(self, q, phi): self.apply_1q(q, G.phase(phi)); return self
    def u3(self, q, theta, phi, lam): self.apply_1q(q, G.u3(theta, phi, lam)); return self
    def cnot(self, c, t): self.apply_c1q(c, t, G.X); return self
    def cy(self, c, t): self.apply_c1q(c, t, G.Y); return self
    def cz(self, a, b): self.apply_diag2(a, b, G.CZ_DIAG); return self
    def cphase(self, a, b, phi): self.apply_diag2(a, b, G.cphase_diag(phi)); return self
    def crx(self, c, t, theta): self.apply_c1q(c, t, G.rx(theta)); return self
    def swap(self, a, b): self.apply_swap(a, b); return self
    def iswap(self, a, b): self.apply_kq([a, b], G.ISWAP); return self
    def toffoli(self, c0, c1, t): self.apply_kq([c0, c1, t], G.TOFFOLI); return self
    def fredkin(self, c, a, b): self.apply_kq([c, a, b], G.FREDKIN); return self

    def apply_block(self, gates: np.ndarray):
        g = np.ascontiguousarray(gates, dtype=W.GATE_DTYPE)
        check(lib().qs_apply_block(self._h, _ptr(g), len(g)))

    def apply_cut_phase(self, edges, gamma: float, w=None):
        e = _edges(edges)
        wa = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        check(lib().qs_apply_cut_phase(self._h, _ptr(e), None if wa is None else _ptr(wa), len(e), gamma))

    # -- read-outs (device tensors; reading them on the host synchronises)
    def _out(self, k, dtype=torch.float64):
        """Output buffer allocated on the state's stream; _done makes the
        current stream wait for the call that fills it."""
        with torch.cuda.stream(self._stream):
            return torch.empty(k, dtype=dtype, device=self.amps.device)

    def _done(self, *outs):
        _finish(self._stream, outs)
        return outs[0] if len(outs) == 1 else outs

    def prob_one(self, q: int) -> torch.Tensor:
        o = self._out(1)
        check(lib().qs_prob_one(self._h, q, ctypes.c_void_p(o.data_ptr())))
        return self._done(o)

    def expect_z_all(self) -> torch.Tensor:
        o = self._out(self.n)
        check(lib().qs_expect_z_all(self._h, ctypes.c_void_p(o.data_ptr())))
        return self._done(o)

    def norm2(self) -> torch.Tensor:
        o = self._out(1)
        check(lib().qs_norm2(self._h, ctypes.c_void_p(o.data_ptr())))
        return self._done(o)

    def expect_cut(self, edges, w=None) -> torch.Tensor:
        e = _edges(edges)
        wa = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        o = self._out(1)
        check(lib().qs_expect_cut(self._h, _ptr(e), None if wa is None else _ptr(wa), len(e), ctypes.c_void_p(o.data_ptr())))
        return self._done(o)

    def expect_diag(self, d: torch.Tensor) -> torch.Tensor:
        assert d.dtype == torch.float64 and d.is_cuda and d.numel() == 1 << self.n
        o = self._out(1)
        check(lib().qs_expect_diag(self._h, ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(o.data_ptr())))
        return self._done(o)

    def expect_pauli(self, xmask: int, zmask: int) -> torch.Tensor:
        o = self._out(2)
        check(lib().qs_expect_pauli(self._h, xmask, zmask, ctypes.c_void_p(o.data_ptr())))
        return self._done(o)

    def inner(self, other: "State") -> torch.Tensor:
        o = self._out(2)
        check(lib().qs_inner(self._h, other._h, ctypes.c_void_p(o.data_ptr())))
        return self._done(o)

    def sample(self, shots: int, seed: int) -> torch.Tensor:
        o = self._out(max(shots, 1), torch.int64)
        check(lib().qs_sample(self._h, shots, seed, ctypes.c_void_p(o.data_ptr())))
        return self._done(o)[:shots]


def sample_noalloc(amps: torch.Tensor, shots: int, seed: int, stream=None) -> torch.Tensor:
    """qs_sample on a register tensor without a state handle (the library's
    fixed device array holds the partial sums).  Calls that overlap on one
    device race; the output tensor is allocated here, the call itself
    allocates nothing."""
    n = amps.numel().bit_length() - 1
    code = QS_C128 if amps.dtype == torch.complex128 else QS_C64
    s = _begin(stream)
    with torch.cuda.stream(s):
        o = torch.empty(max(shots, 1), dtype=torch.int64, device=amps.device)
    check(lib().qs_sample_noalloc(n, code, ctypes.c_void_p(amps.data_ptr()), amps.numel() * amps.element_size(), shots, seed,
                                  ctypes.c_void_p(o.data_ptr()), ctypes.c_void_p(s.cuda_stream)))
    _finish(s, (o,))
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
        s = _begin(stream)
        with torch.cuda.stream(s):
            a = a.contiguous()
            B = a.shape[0]
            E = torch.empty(B, dtype=torch.float64, device=a.device)
            G = torch.empty(B, 2 * self.p, dtype=torch.float64, device=a.device) if grad else None
        ws = self.workspace(grad)
        if s != torch.cuda.current_stream():
            ws.record_stream(s)  # the cached workspace is also used on s
        check(lib().qs_qaoa_run(ctypes.byref(self._desc), ctypes.c_void_p(a.data_ptr()), B, ctypes.c_void_p(E.data_ptr()),
                                ctypes.c_void_p(G.data_ptr()) if grad else None, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                ctypes.c_void_p(s.cuda_stream)))
        _finish(s, (E, G))
        return E, G


class Pool:
    """A pool of QAOA Max-Cut circuits: graph g (with its own qubit count) times
    sets_per_graph angle vectors, circuit c = g * sets_per_graph + a.  One call
    evaluates every <C> and (optionally) every adjoint gradient; the launch
    sequence is captured into a hipGraph on the first call and replayed after."""

    def __init__(self, graphs, n_qubits, sets_per_graph: int, p: int, device="cuda", grad: bool = True, ws_bytes: int | None = None,
                 ws_circuits: int | None = None):
        self.n_qubits = np.ascontiguousarray(n_qubits, dtype=np.int32)
        self.edges = np.ascontiguousarray(np.concatenate([_edges(e) for e in graphs]).reshape(-1), dtype=np.int32)
        self.offsets = np.ascontiguousarray(np.concatenate([[0], np.cumsum([len(_edges(e)) for e in graphs])]), dtype=np.int32)
        self.sets, self.p = sets_per_graph, p
        self.count = len(graphs) * sets_per_graph
        self._desc = PoolDesc(len(graphs), sets_per_graph, p, self.n_qubits.ctypes.data, self.offsets.ctypes.data, self.edges.ctypes.data)
        if ws_bytes is None and ws_circuits is not None:  # room for this many circuits of the largest size per launch
            nbytes = ctypes.c_size_t()
            check(lib().qs_pool_circuit_bytes(ctypes.byref(self._desc), int(grad), ctypes.byref(nbytes)))
            ws_bytes = nbytes.value * ws_circuits
        if ws_bytes is None:
            nbytes = ctypes.c_size_t()
            check(lib().qs_pool_workspace_bytes(ctypes.byref(self._desc), ctypes.byref(nbytes)))
            ws_bytes = nbytes.value
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=device)
        self.angles = torch.zeros(self.count, 2 * p, dtype=torch.float64, device=device)
        self.E = torch.empty(self.count, dtype=torch.float64, device=device)
        self.G = torch.empty(self.count, 2 * p, dtype=torch.float64, device=device) if grad else None

    def _plan_args(self):
        return (ctypes.byref(self._desc), ctypes.c_void_p(self.angles.data_ptr()), ctypes.c_void_p(self.E.data_ptr()),
                ctypes.c_void_p(self.G.data_ptr()) if self.G is not None else None, ctypes.c_void_p(self.ws.data_ptr()),
                self.ws.numel())

    def release(self):
        """Free the library's plan for this pool (captured graph, device tables)."""
        if getattr(self, "ws", None) is not None:
            check(lib().qs_pool_release(*self._plan_args()))

    def __del__(self):
        if _exiting:
            return
        try:
            self.release()
        except Exception:
            pass

    def run(self, angles: torch.Tensor | None = None, stream=None):
        """Copy `angles` [count, 2p] into the pool's device buffer (if given) and
        evaluate; returns (E, G) device tensors owned by the pool."""
        s = _begin(stream)
        if s != torch.cuda.current_stream():
            for t in (self.angles, self.E, self.G, self.ws):
                if t is not None:
                    t.record_stream(s)
        if angles is not None:
            with torch.cuda.stream(s):
                self.angles.copy_(angles.reshape(self.count, 2 * self.p))
        check(lib().qs_pool_run(ctypes.byref(self._desc), ctypes.c_void_p(self.angles.data_ptr()), ctypes.c_void_p(self.E.data_ptr()),
                                ctypes.c_void_p(self.G.data_ptr()) if self.G is not None else None,
                                ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), ctypes.c_void_p(s.cuda_stream)))
        _finish(s)
        return self.E, self.G


def block_passes(n: int, gates: np.ndarray, dtype=torch.complex128) -> int:
    """Read+write passes of the state that State.apply_block takes for this
    gate list (host-side planning only)."""
    g = np.ascontiguousarray(gates, dtype=W.GATE_DTYPE)
    out = ctypes.c_int(-1)
    check(lib().qs_block_passes(n, QS_C128 if dtype == torch.complex128 else QS_C64, _ptr(g), len(g), ctypes.byref(out)))
    return out.value


def cut_max(graphs, n_qubits, w=None, device="cuda", stream=None):
    """Exact Max-Cut value of each graph (and the smallest maximising
    bipartition): float64 [G] and uint64-as-int64 [G] device tensors."""
    nq = np.ascontiguousarray(n_qubits, dtype=np.int32)
    es = [_edges(e) for e in graphs]
    off = np.ascontiguousarray(np.concatenate([[0], np.cumsum([len(e) for e in es])]), dtype=np.int32)
    edges = np.ascontiguousarray(np.concatenate(es).reshape(-1), dtype=np.int32)
    desc = PoolDesc(len(es), 1, 1, nq.ctypes.data, off.ctypes.data, edges.ctypes.data)
    warr = None if w is None else np.ascontiguousarray(np.concatenate([np.asarray(x, np.float64) for x in w]))
    mx = torch.empty(len(es), dtype=torch.float64, device=device)
    arg = torch.empty(len(es), dtype=torch.int64, device=device)
    check(lib().qs_cut_max(ctypes.byref(desc), None if warr is None else _ptr(warr), ctypes.c_void_p(mx.data_ptr()),
                           ctypes.c_void_p(arg.data_ptr()), ctypes.c_void_p(_stream_ptr(stream))))
    return mx, arg


class Swarm:
    """Particle swarm over a Pool (graph g's swarm = its sets_per_graph angle
    vectors); the pool's angle and energy buffers are the swarm's positions
    and evaluations.  All state is device tensors."""

    def __init__(self, pool: Pool, omega=0.66, phi_p=1.6, phi_g=0.62, attract=1):
        self.pool = pool
        G, R, D = len(pool.n_qubits), pool.sets, 2 * pool.p
        f64 = dict(dtype=torch.float64, device=pool.angles.device)
        self.pos, self.E = pool.angles, pool.E
        self.vel = torch.empty(G, R, D, **f64)
        self.pbest = torch.empty(G, R, D, **f64)
        self.pbest_val = torch.empty(G, R, **f64)
        self.gbest = torch.empty(G, D, **f64)
        self.gbest_val = torch.empty(G, **f64)
        self.G, self.R, self.D = G, R, D
        self.params = PsoParams(omega, phi_p, phi_g, attract)
        self._sw = PsoSwarm(*[t.data_ptr() for t in (self.pos, self.vel, self.pbest, self.pbest_val, self.gbest,
                                                     self.gbest_val, self.E)])

    def init(self, seed: int, stream=None):
        check(lib().qs_pso_init(ctypes.byref(self.pool._desc), seed, ctypes.byref(self._sw), ctypes.c_void_p(_stream_ptr(stream))))

    def step(self, rnd: int, seed: int, move: bool = True, history: torch.Tensor | None = None, stream=None):
        check(lib().qs_pso_step(ctypes.byref(self.pool._desc), ctypes.byref(self.params), rnd, int(move), seed,
                                ctypes.byref(self._sw), None if history is None else ctypes.c_void_p(history.data_ptr()),
                                ctypes.c_void_p(_stream_ptr(stream))))

    def run(self, rounds: int, seed: int, stream=None) -> torch.Tensor:
        """Whole run on the device; returns the global-best history [rounds, G]."""
        hist = torch.empty(rounds, self.G, dtype=torch.float64, device=self.pos.device)
        check(lib().qs_pso_run(ctypes.byref(self.pool._desc), ctypes.byref(self.params), rounds, seed, ctypes.byref(self._sw),
                               ctypes.c_void_p(hist.data_ptr()), ctypes.c_void_p(self.pool.ws.data_ptr()), self.pool.ws.numel(),
                               ctypes.c_void_p(_stream_ptr(stream))))
        return hist


def traj_run(n: int, gates: np.ndarray, basis_index: int, n_traj: int, p: float, seed: int, dtype=torch.complex128,
             log_cap: int = 0, prob_mean: bool = True, device="cuda", stream=None, T1: float = math.inf, T2: float = math.inf,
             diag: torch.Tensor | None = None, readouts=("z", "x", "fid")) -> dict:
    """Noise trajectories with stochastic Pauli insertion (probability p per
    touched qubit) and stochastic noise gates (kind 5, timescales T1, T2).
    Returns device tensors: z, x [n_traj, n]; fid [n_traj]; counts [n_traj];
    prob_mean [2^n]; log [n_traj, log_cap]; diag [n_traj] (per-trajectory
    expectation of the diagonal observable `diag`, a float64 [2^n] device tensor).
    `readouts` names which of z, x, fid are computed (the others are absent
    from the result; <X_q> costs a read of every state per qubit)."""
    bad = set(readouts) - {"z", "x", "fid"}
    if bad:
        raise ValueError(f"unknown read-outs {sorted(bad)}")
    g = np.ascontiguousarray(gates, dtype=W.GATE_DTYPE)
    code = QS_C128 if dtype == torch.complex128 else QS_C64
    nbytes = ctypes.c_size_t()
    check(lib().qs_traj_noise_workspace_bytes(n, code, _ptr(g), len(g), n_traj, ctypes.byref(nbytes)))
    s = _begin(stream)
    with torch.cuda.stream(s):  # workspace and outputs belong to the stream the kernels run on
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
        f64 = dict(dtype=torch.float64, device=device)
        res = {k: torch.empty((n_traj, n) if k != "fid" else (n_traj,), **f64) for k in ("z", "x", "fid") if k in readouts}
        res["counts"] = torch.empty(n_traj, dtype=torch.int32, device=device)
        if prob_mean:
            res["prob_mean"] = torch.empty(1 << n, **f64)
        if log_cap:
            res["log"] = torch.zeros(n_traj, log_cap, dtype=torch.int32, device=device)
        if diag is not None:
            assert diag.dtype == torch.float64 and diag.is_cuda and diag.numel() == 1 << n
            res["diag"] = torch.empty(n_traj, **f64)
    opt = lambda k: res[k].data_ptr() if k in res else None  # noqa: E731
    out = TrajOut(opt("z"), opt("x"), opt("fid"),
                  res["prob_mean"].data_ptr() if prob_mean else None, res["counts"].data_ptr(),
                  res["log"].data_ptr() if log_cap else None, log_cap,
                  diag.data_ptr() if diag is not None else None, res["diag"].data_ptr() if diag is not None else None)
    if math.isinf(T1) and math.isinf(T2) and not np.any(g["kind"] == W.G_NOISE):
        check(lib().qs_traj_run(n, code, _ptr(g), len(g), basis_index, n_traj, p, seed, ctypes.byref(out),
                                ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(s.cuda_stream)))
    else:
        nz = Noise(p, T1, T2)
        check(lib().qs_traj_run_noise(n, code, _ptr(g), len(g), basis_index, n_traj, ctypes.byref(nz), seed, ctypes.byref(out),
                                      ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(s.cuda_stream)))
    # ws was allocated on s and goes back to the caching allocator in s's
    # order, so later work cannot overwrite it before the kernels above ran.
    _finish(s, tuple(res.values()))
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
