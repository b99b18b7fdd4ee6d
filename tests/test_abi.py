"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every entry point include/gn.h declares, and the binding refuses to
run without it (no CPU fallback)."""
import ctypes
import os

import pytest

from paper_2509_14185_amd import gn


def _lib_or_skip():
    if not os.path.exists(gn.LIB_PATH):
        pytest.skip("libgn.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(gn.LIB_PATH)


def test_header_declares_the_hot_path_calls():
    names = set(gn.exported_names())
    for required in ["gn_create", "gn_set_points", "gn_residual", "gn_jacobian", "gn_gram", "gn_solve",
                     "gn_step", "gn_vjp", "gn_eval", "gn_destroy"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _lib_or_skip()
    missing = [n for n in gn.exported_names() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_without_device():
    lib = gn.load()
    assert lib.gn_status_string(gn.GN_ENOTPD) == b"matrix not positive definite"
    assert lib.gn_status_string(gn.GN_EINVAL) == b"invalid argument"


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(gn, "_lib", None)
    monkeypatch.setattr(gn, "LIB_PATH", "/nonexistent/libgn.so")
    with pytest.raises(RuntimeError):
        gn.load()
