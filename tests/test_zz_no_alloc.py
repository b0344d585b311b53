"""qs_sample_noalloc, the allocation-free sampling entry point, through the C-ABI: its draws must
equal qs_sample's on the same register bit for bit (the same kernels, with the
partial sums in the library's fixed device array instead of the handle's
scratch).  Two calls in a row, the second on a smaller register, so stale
contents of the shared array from the first call would show."""
import ctypes

import numpy as np
import pytest

from paper_2001_10554_amd import workloads as W
from gpu_util import record, require_gpu

pytestmark = pytest.mark.gpu


def _noalloc(s, shots, seed):
    import torch
    from paper_2001_10554_amd.qsim import QS_C128, QS_C64, check, lib
    f = lib().qs_sample_noalloc
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64, ctypes.c_uint64,
                  ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    out = torch.full((shots,), -1, dtype=torch.int64, device="cuda")
    code = QS_C128 if s.dtype == torch.complex128 else QS_C64
    check(f(s.n, code, ctypes.c_void_p(s.amps.data_ptr()), s.amps.numel() * s.amps.element_size(), shots, seed,
            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return out


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_noalloc_sample_matches_handle_sample(dt):
    require_gpu()
    import torch
    from paper_2001_10554_amd.qsim import State
    dtype = torch.complex128 if dt == "c128" else torch.complex64
    for n, shots, seed in ((24, 1 << 16, 3), (13, 5000, 4)):  # the second call is smaller
        s = State(n, dtype).init_random(n)
        s.apply_1q(n - 1, W.haar_list(n, 1)[0])
        want = s.sample(shots, seed).cpu().numpy()
        got = _noalloc(s, shots, seed).cpu().numpy()
        record(f"n={n}: draws differing from qs_sample", int(np.count_nonzero(got != want)), 0)


def test_noalloc_rejects_bad_arguments():
    require_gpu()
    import torch
    from paper_2001_10554_amd.qsim import QS_ERR_ARG, QS_ERR_DTYPE, QS_ERR_SIZE, lib
    f = lib().qs_sample_noalloc
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64, ctypes.c_uint64,
                  ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    buf = torch.zeros(16, dtype=torch.complex128, device="cuda")
    out = torch.empty(4, dtype=torch.int64, device="cuda")
    p, o = ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(out.data_ptr())
    assert f(35, 2, p, 1 << 40, 4, 1, o, None) == QS_ERR_SIZE   # above the c128 limit
    assert f(5, 2, p, 256, 4, 1, o, None) == QS_ERR_SIZE        # buffer smaller than 2^5 amplitudes
    assert f(4, 3, p, 256, 4, 1, o, None) == QS_ERR_DTYPE
    assert f(4, 2, None, 256, 4, 1, o, None) == QS_ERR_ARG
    assert f(4, 2, p, 256, 4, 1, None, None) == QS_ERR_ARG
    assert f(4, 2, p, 256, -1, 1, o, None) == QS_ERR_ARG
