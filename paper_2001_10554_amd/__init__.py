"""MI355X-native state-vector simulator (hot path of arXiv 2001.10554, Intel
Quantum Simulator): one-qubit and controlled gates on a 2^n-amplitude register
in HBM, fused gate blocks, read-outs, QAOA Max-Cut with adjoint gradients, a
pool of uneven circuits and noise trajectories — all in hand-written HIP
kernels for gfx950 behind the C-ABI of ``include/qsim.h``.

Importing the package is cheap: the HIP library (and torch) are loaded on
first use of the binding, ``paper_2001_10554_amd.qsim``.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "qsim"]


def __getattr__(name):
    import importlib
    if name in ("qsim", "State", "QsimError", "lib"):
        mod = importlib.import_module(".qsim", __name__)
        return mod if name == "qsim" else getattr(mod, name)
    raise AttributeError(name)
