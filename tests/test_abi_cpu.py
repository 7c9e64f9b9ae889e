"""C ABI checks that need no GPU: the library loads, exports every function
include/sap.h declares, and validates options host-side."""

import ctypes
import os
import re

import pytest

from paper_1509_07919_amd import sap as binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "sap.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sap_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libsap.so is not built (run __graft_entry__.build())")
    return binding.load_library()


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(binding.EXPORTED)


def ws(lib, **kw):
    opt = binding.make_options(**kw)
    out = ctypes.c_size_t(0)
    rc = lib.sap_workspace_bytes(ctypes.byref(opt), ctypes.byref(out))
    return rc, out.value, lib.sap_last_error().decode()


@pytest.mark.parametrize("kw,msg", [
    (dict(n=0, k=0, p=1), "N must be"),
    (dict(n=100, k=100, p=1), "K must be < N"),
    (dict(n=1000, k=256, p=1), "K must be in"),
    (dict(n=100, k=2, p=0), "P must be"),
    (dict(n=100, k=2, p=101), "P must be"),
    (dict(n=100, k=10, p=6, mode="coupled"), "floor(N/P) >= 2K"),
])
def test_invalid_options(lib, kw, msg):
    rc, _, err = ws(lib, **kw)
    assert rc == binding.SAP_ERR_INVALID and msg in err


def test_workspace_size_accounts_for_layout(lib):
    rc, b64, _ = ws(lib, n=200_000, k=50, p=64, mode="coupled", factor_prec="fp64")
    assert rc == 0
    rc, b32, _ = ws(lib, n=200_000, k=50, p=64, mode="coupled", factor_prec="fp32")
    rc2, badj, _ = ws(lib, n=200_000, k=50, p=64, mode="coupled", factor_prec="fp32",
                      adjoint=True)
    assert rc == rc2 == 0
    cs = 51
    # two factor arrays, N*(K+1) each, dominate; the adjoint adds two more
    assert b64 >= 2 * 8 * 200_000 * cs and b32 >= 2 * 4 * 200_000 * cs
    assert badj - b32 >= 2 * 4 * 200_000 * cs
    rc, bd, _ = ws(lib, n=200_000, k=50, p=64, mode="decoupled", factor_prec="fp64")
    assert bd < b64                                  # no interface matrices


def test_sweep_chunks_must_be_non_negative(lib):
    opt = binding.make_options(n=100, k=2, p=2)
    opt.sweep_chunks = -1
    out = ctypes.c_size_t(0)
    assert lib.sap_workspace_bytes(ctypes.byref(opt), ctypes.byref(out)) == -1


def test_chunked_sweeps_need_transfer_storage(lib):
    # splitting every block's sweep into chains adds K x K transfer matrices
    rc1, one, _ = ws(lib, n=200_000, k=50, p=64, mode="coupled", factor_prec="fp64",
                     sweep_chunks=1)
    rc8, eight, _ = ws(lib, n=200_000, k=50, p=64, mode="coupled", factor_prec="fp64",
                       sweep_chunks=8)
    assert rc1 == rc8 == 0
    assert eight - one >= 2 * 8 * 64 * 7 * 50 * 50


def test_null_handle_calls_fail_cleanly(lib):
    assert lib.sap_factor(None, None, None) == binding.SAP_ERR_INVALID
    assert lib.sap_solve(None, None, None, 1e-10, 10, None, None) == binding.SAP_ERR_INVALID
    assert lib.sap_destroy(None) == 0


def test_workspace_too_small_is_nospace(lib):
    """sap_create checks the workspace size before it touches the device:
    a too-small workspace returns SAP_ERR_NOSPACE and no handle."""
    opt = binding.make_options(n=20_000, k=10, p=8, mode="coupled")
    need = ctypes.c_size_t(0)
    assert lib.sap_workspace_bytes(ctypes.byref(opt), ctypes.byref(need)) == 0
    h = ctypes.c_void_p(1234)
    fake = ctypes.c_void_p(1 << 20)               # 256-byte aligned, never dereferenced
    rc = lib.sap_create(ctypes.byref(opt), fake, need.value - 1, ctypes.byref(h))
    assert rc == binding.SAP_ERR_NOSPACE
    assert "workspace too small" in lib.sap_last_error().decode()
    assert not h.value
    rc = lib.sap_create(ctypes.byref(opt), ctypes.c_void_p((1 << 20) + 8), need.value,
                        ctypes.byref(h))
    assert rc == binding.SAP_ERR_INVALID and "aligned" in lib.sap_last_error().decode()
