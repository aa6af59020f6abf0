"""The C ABI library without a GPU: it loads, exports every function the
header declares, and its host-side checks and sizes behave (no kernel runs)."""
import ctypes
import re
import subprocess

import numpy as np
import pytest

from paper_2603_12292_amd import _lib


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    declared = _lib.declared_symbols()
    assert len(declared) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", lib._name], capture_output=True, text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if re.search(r"\sT\s", ln)}
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    for s in declared:
        assert getattr(lib, s) is not None


def test_binding_covers_the_header():
    bound = {name for name, _, _ in _lib.SIGNATURES}
    assert set(_lib.declared_symbols()) == bound


def test_abi_version_matches_header(lib):
    with open(_lib.HEADER) as f:
        m = re.search(r"#define BEAGLE_ABI_VERSION (\d+)", f.read())
    assert lib.beagle_abi_version() == int(m.group(1)) == _lib.ABI_VERSION


def test_constants_match_header():
    with open(_lib.HEADER) as f:
        text = f.read()
    for name, value in (("BEAGLE_FIT_MSE", _lib.FIT_MSE), ("BEAGLE_FIT_CORR", _lib.FIT_CORR),
                        ("BEAGLE_TUNE_AUTO", _lib.TUNE_AUTO), ("BEAGLE_TUNE_WIDE", _lib.TUNE_WIDE),
                        ("BEAGLE_TUNE_NARROW", _lib.TUNE_NARROW), ("BEAGLE_E_INVALID_ARG", _lib.E_INVALID_ARG),
                        ("BEAGLE_E_NOMEM", _lib.E_NOMEM), ("BEAGLE_E_UNSUPPORTED", _lib.E_UNSUPPORTED)):
        m = re.search(name + r"\s*=\s*(-?\d+)", text)
        assert m and int(m.group(1)) == value, name


def _structs(N=10, L=7, M=1000, D=3):
    # fake device addresses: only the sizes are read by the calls below
    P = _lib.Programs(0x1000, N * L, 0x2000, 0x3000, 0x4000, 2 * N, 0x5000, 0x6000, N)
    Dd = _lib.Dataset(0x7000, 0x8000, M, D)
    return P, Dd


def test_null_context_is_rejected(lib):
    P, D = _structs()
    rc = lib.beagle_eval(None, ctypes.byref(P), ctypes.byref(D), _lib.FIT_MSE, None, None, None)
    assert rc == _lib.E_INVALID_ARG
    assert b"ctx" in lib.beagle_last_error()
    assert lib.beagle_eval_batched(None, None, None, 1, 0, None, None, None) == _lib.E_INVALID_ARG
    assert lib.beagle_ctx_set_tuning(None, 0) == _lib.E_INVALID_ARG


def test_workspace_size_is_host_logic(lib):
    P, D = _structs()
    out = ctypes.c_size_t()
    assert lib.beagle_eval_workspace_size(ctypes.byref(P), ctypes.byref(D), _lib.FIT_MSE, ctypes.byref(out)) == 0
    mse = out.value
    assert lib.beagle_eval_workspace_size(ctypes.byref(P), ctypes.byref(D), _lib.FIT_CORR, ctypes.byref(out)) == 0
    corr = out.value
    # correlation keeps three partial sums per (chunk, program), MSE one
    assert corr > mse > 0
    # the case buffers grow with M (cases padded to 2048) and D
    P2, D2 = _structs(M=100_000, D=5)
    assert lib.beagle_eval_workspace_size(ctypes.byref(P2), ctypes.byref(D2), _lib.FIT_MSE, ctypes.byref(out)) == 0
    assert out.value > mse + 5 * 4 * 98_000


@pytest.mark.parametrize("field,value,code", [("D", 0, _lib.E_UNSUPPORTED), ("D", 17, _lib.E_UNSUPPORTED),
                                              ("M", 0, _lib.E_INVALID_ARG)])
def test_workspace_size_rejects_bad_data(lib, field, value, code):
    P, D = _structs()
    setattr(D, field, value)
    out = ctypes.c_size_t()
    assert lib.beagle_eval_workspace_size(ctypes.byref(P), ctypes.byref(D), _lib.FIT_MSE, ctypes.byref(out)) == code


def test_correlation_needs_two_cases(lib):
    P, D = _structs(M=1)
    out = ctypes.c_size_t()
    assert lib.beagle_eval_workspace_size(ctypes.byref(P), ctypes.byref(D), _lib.FIT_CORR,
                                          ctypes.byref(out)) == _lib.E_INVALID_ARG
    assert lib.beagle_eval_workspace_size(ctypes.byref(P), ctypes.byref(D), _lib.FIT_MSE, ctypes.byref(out)) == 0


def test_unknown_kind(lib):
    P, D = _structs()
    out = ctypes.c_size_t()
    assert lib.beagle_eval_workspace_size(ctypes.byref(P), ctypes.byref(D), 5, ctypes.byref(out)) == \
        _lib.E_INVALID_ARG
    assert np.isfinite(float(out.value))
