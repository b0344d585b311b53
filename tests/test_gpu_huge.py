"""Registers whose gate launches need more than 2^31 work-items: a 33-qubit
complex128 and a 34-qubit complex64 register (128 GiB each).  A HIP grid holds
fewer than 2^32 work-items, so these kernels run as several launch pieces;
every gate family that can exceed one piece is checked here.

The oracle cannot hold these registers, but each gate couples only the 2^k
amplitudes of a group that differ in the gate's qubits (eq. 3 and its
controlled and k-qubit forms).  For every gate, 2^14 random groups are read
back before and after the kernel, packed into a small register (group member
on the low qubits, sample on the high ones) and pushed through the oracle's
gate.  Amplitudes of a random normalised register are ~2^{-n/2}, so errors are
measured relative to the largest sampled amplitude.
"""
import numpy as np
import pytest

import oracle
from paper_2001_10554_amd import workloads as W
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu

K = 1 << 14


def _groups(rng, n, bits):
    """[2^k, K] global indices: member m of sample s has bit j of m on qubit bits[j]."""
    base = rng.integers(0, 1 << (n - len(bits)), size=K, dtype=np.int64)
    for b in sorted(bits):
        base = ((base >> b) << (b + 1)) | (base & ((1 << b) - 1))
    out = []
    for m in range(1 << len(bits)):
        idx = base.copy()
        for j, b in enumerate(bits):
            if (m >> j) & 1:
                idx |= 1 << b
        out.append(idx)
    return np.stack(out)


def _check(s, rng, n, bits, gpu_op, oracle_op, rel):
    import torch
    idx = _groups(rng, n, bits)
    t = torch.from_numpy(idx.reshape(-1)).cuda()
    before = s.amps[t].cpu().numpy().astype(np.complex128).reshape(idx.shape)
    gpu_op()
    after = s.amps[t].cpu().numpy().astype(np.complex128).reshape(idx.shape)
    buf = np.ascontiguousarray(before.T).reshape(-1)  # index = sample * 2^k + member
    oracle_op(buf)
    want = buf.reshape(K, -1).T
    scale = np.max(np.abs(before))
    err = np.max(np.abs(after - want)) / scale
    assert err < rel, (bits, err)


def _run(n, dtype, rel, ops):
    require_gpu()
    import torch

    from paper_2001_10554_amd.qsim import State
    bytes_needed = (1 << n) * (16 if dtype == torch.complex128 else 8)
    free, _ = torch.cuda.mem_get_info()
    if free < bytes_needed + (4 << 30):
        pytest.skip(f"needs {bytes_needed >> 30} GiB of free device memory")
    rng = np.random.default_rng(n)
    s = State(n, dtype).init_random(n)
    assert abs(s.norm2().item() - 1.0) < (1e-12 if dtype == torch.complex128 else 1e-5)
    try:
        for bits, gpu_op, oracle_op in ops(s, rng):
            print(f"n={n} {dtype} gate on {bits}", flush=True)
            _check(s, rng, n, bits, gpu_op, oracle_op, rel)
        assert abs(s.norm2().item() - 1.0) < (1e-11 if dtype == torch.complex128 else 1e-4)
    finally:
        del s
        torch.cuda.empty_cache()


def _ops(n, c128):
    """(qubits, GPU call, oracle call on the packed register) for every
    launch family; the comments give the number of launch pieces."""
    g = np.random.default_rng(7)
    m = [W.haar_2x2(g) for _ in range(4)]
    d = np.exp(1j * g.uniform(0, 2 * np.pi, 4))
    u3, _ = np.linalg.qr(g.standard_normal((8, 8)) + 1j * g.standard_normal((8, 8)))
    u1, _ = np.linalg.qr(g.standard_normal((2, 2)) + 1j * g.standard_normal((2, 2)))
    hi = n - 1
    line = 3 if c128 else 4  # controls below this bit sit inside a 128-byte line

    def ops(s, rng):
        yield [0], lambda: s.apply_1q(0, m[0]), lambda b: oracle.apply_1q(b, 0, m[0])        # lane kernel
        yield [hi], lambda: s.apply_1q(hi, m[1]), lambda b: oracle.apply_1q(b, 0, m[1])      # pair kernel
        c = line - 1
        yield [4, c], lambda: s.apply_c1q(c, 4, m[2]), lambda b: oracle.apply_c1q(b, 1, 0, m[2])          # controlled lane kernel
        yield [20, 0], lambda: s.apply_c1q(0, 20, W.PAULI_X), lambda b: oracle.apply_c1q(b, 1, 0, W.PAULI_X)  # controlled pair kernel
        yield [hi, 9], lambda: s.apply_c1q(9, hi, m[3]), lambda b: oracle.apply_c1q(b, 1, 0, m[3])        # control-1 quads
        yield [5, hi], lambda: s.apply_diag2(5, hi, d), lambda b: oracle.apply_diag2(b, 0, 1, d)
        yield [2, hi - 1], lambda: s.apply_swap(2, hi - 1), lambda b: oracle.apply_swap(b, 0, 1)
        yield [3], lambda: s.apply_kq([3], u1), lambda b: oracle.apply_kq(b, [0], u1)
        yield [1, 20, hi], lambda: s.apply_kq([1, 20, hi], u3), lambda b: oracle.apply_kq(b, [0, 1, 2], u3)
    return ops


def test_33q_c128_launch_pieces():
    import torch
    _run(33, torch.complex128, 1e-13, _ops(33, True))


def test_34q_c64_launch_pieces():
    import torch
    _run(34, torch.complex64, 1e-6, _ops(34, False))
