"""The C-ABI library builds, loads and exports every symbol include/qsim.h declares.

Runs without a GPU: only loading and symbol lookup, no compute calls.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qsim.h")
LIB = os.path.join(ROOT, "paper_2001_10554_amd", "libqsim_hip.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(qs_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["qs_state_create", "qs_state_destroy", "qs_init_basis", "qs_init_uniform", "qs_init_random",
                     "qs_apply_1q", "qs_apply_c1q", "qs_apply_block", "qs_apply_cut_phase", "qs_prob_one",
                     "qs_expect_z_all", "qs_expect_cut", "qs_expect_diag", "qs_expect_pauli", "qs_norm2", "qs_inner",
                     "qs_sample", "qs_qaoa_run", "qs_pool_run", "qs_traj_run", "qs_sync", "qs_last_error"]:
        assert required in names


@pytest.fixture(scope="module")
def built_lib():
    if not os.path.exists(LIB):
        from paper_2001_10554_amd import build
        build.build(verbose=False)
    import torch  # noqa: F401  (same HIP runtime as the binding uses)
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(built_lib):
    missing = [n for n in declared_functions() if not hasattr(built_lib, n)]
    assert not missing, f"declared in qsim.h but not exported: {missing}"


def test_only_qs_symbols_exported():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    syms = [l.split()[-1] for l in out.splitlines() if " T " in l]
    assert syms and all(s.startswith("qs_") for s in syms), [s for s in syms if not s.startswith("qs_")]


def test_last_error_initially_empty(built_lib):
    # a fresh process: the message is per thread and earlier tests may have set it
    import subprocess
    import sys
    code = ("import ctypes, torch; L = ctypes.CDLL(%r); f = L.qs_last_error; "
            "f.restype = ctypes.c_char_p; print(repr(f()))" % LIB)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, check=True).stdout
    assert out.strip() == "b''"


def test_binding_names_match_header():
    from paper_2001_10554_amd import qsim
    src = open(qsim.__file__).read()
    for n in declared_functions():
        assert f'"{n}"' in src or n == "qs_last_error", n


def test_gate_record_layout_matches_header():
    # qs_gate: int32 kind, q0, q1, pad, then double u[8] (80 bytes)
    from paper_2001_10554_amd import workloads as W
    dt = W.GATE_DTYPE
    assert dt.itemsize == 80
    assert [dt.fields[k][1] for k in ("kind", "q0", "q1", "pad", "u")] == [0, 4, 8, 12, 16]
    assert "80 bytes" in open(HEADER).read()
