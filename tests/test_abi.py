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
                 "tok_gop_blend", "tok_decode_blend", "tok_decode_residual"]:
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


def test_decode_residual_rejects_bad_arguments_before_any_device_work(lib):
    """Host-side checks of tok_decode_residual: null pointers, misaligned
    buffers, a bad latent shape and a too-small residual workspace are
    reported before the model is used or anything is launched (the handle
    here is a zeroed host buffer standing in for a model)."""
    f = lib.tok_decode_residual
    f.restype = ctypes.c_int
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    f.argtypes = [vp, vp, i32, i32, i32, i32, vp, ctypes.c_float, vp, vp, vp, vp, sz, vp, vp, sz, vp, sz, vp]
    lib.tok_last_error.restype = ctypes.c_char_p
    fake = ctypes.create_string_buffer(1 << 16)
    buf = ctypes.create_string_buffer((1 << 12) + 256)
    base = (ctypes.addressof(buf) + 255) & ~255  # 256-byte aligned host addresses
    a = lambda off: ctypes.c_void_p(base + off)

    def call(model=fake, x=a(0), r=a(256), idx=a(512), val=a(768), co=a(1024), rws=a(1280), rws_bytes=1 << 20,
             shape=(1, 2, 4, 4)):
        return f(model, a(1536), *shape, x, 0.1, a(1792), r, idx, val, 16, co, a(2048), 1 << 20, rws, rws_bytes,
                 None)
    assert call(model=None) == -1 and b"null" in lib.tok_last_error()
    assert call(x=None) == -1
    assert call(rws=None) == -1
    assert call(x=a(4)) == -1 and b"aligned" in lib.tok_last_error()
    assert call(r=a(264)) == -1 and b"aligned" in lib.tok_last_error()
    assert call(co=a(1028)) == -1 and b"aligned" in lib.tok_last_error()
    assert call(shape=(1, 0, 4, 4)) == -2
    assert call(shape=(70000, 2, 4, 4)) == -2
    assert call(rws_bytes=1) == -7 and b"workspace" in lib.tok_last_error()
