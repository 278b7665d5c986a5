"""The C-ABI library loads and exports every entry point include/tok.h
declares (host-only calls; no GPU work)."""
import ctypes
import os
import re

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tok.h")
LIB = os.path.join(ROOT, "paper_2602_03529_amd", "libtok.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(tok_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libtok.so not built: run python -m paper_2602_03529_amd.build")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ["tok_encode", "tok_quantize", "tok_drop", "tok_decode", "tok_model_create",
                 "tok_workspace_size", "tok_weight_count", "tok_backward", "tok_select_similar",
                 "tok_packetize", "tok_reassemble", "tok_residual_compress", "tok_residual_apply",
                 "tok_gop_blend"]:
        assert need in names, names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_weight_count_matches_the_parameter_table(lib):
    lib.tok_weight_count.restype = ctypes.c_size_t
    assert lib.tok_weight_count() == synth.param_count() == 2225929


def test_status_strings(lib):
    lib.tok_status_str.restype = ctypes.c_char_p
    assert lib.tok_status_str(0) == b"ok"
    assert lib.tok_status_str(-2) == b"invalid shape"


def test_create_rejects_bad_blob(lib):
    lib.tok_model_create.restype = ctypes.c_int
    h = ctypes.c_void_p()
    buf = (ctypes.c_float * 10)()
    assert lib.tok_model_create(buf, 10, 1, 0, ctypes.byref(h)) == -1  # TOK_EINVAL, before any HIP call
    lib.tok_last_error.restype = ctypes.c_char_p
    assert b"expected 2225929" in lib.tok_last_error()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2602_03529_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.lib()
