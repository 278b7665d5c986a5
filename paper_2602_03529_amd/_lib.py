"""ctypes loader for libtok.so: argument types of every entry point of
include/tok.h.  Importing this module fails loudly if the library has not
been built; there is no fallback implementation."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtok.so")

TOK_OK = 0
TOK_F32, TOK_BF16, TOK_FP8_E4M3 = 0, 1, 2
TOK_DROP_NONE, TOK_DROP_BERNOULLI, TOK_DROP_ROWS, TOK_DROP_EXTERNAL, TOK_DROP_SIMILARITY = 0, 1, 2, 3, 4
TOK_WS_ENCODE, TOK_WS_DECODE, TOK_WS_ROUNDTRIP, TOK_WS_STREAM = 1, 2, 3, 16


class DropDesc(C.Structure):
    """Mirror of tok_drop_desc."""
    _fields_ = [("mode", C.c_int), ("rate", C.c_float), ("seed", C.c_uint64), ("clip_id0", C.c_uint64),
                ("protect_iframe", C.c_int), ("ext_keep", C.c_void_p)]


class Request(C.Structure):
    """Mirror of tok_request."""
    _fields_ = [("T", C.c_int), ("H", C.c_int), ("W", C.c_int), ("pixels", C.c_void_p), ("drop", DropDesc)]


class Result(C.Structure):
    """Mirror of tok_result."""
    _fields_ = [("ticket", C.c_uint64), ("status", C.c_int), ("T2", C.c_int), ("H2", C.c_int), ("W2", C.c_int),
                ("codes", C.c_void_p), ("idx", C.c_void_p), ("keep", C.c_void_p), ("xhat", C.c_void_p),
                ("queue_ms", C.c_double), ("run_ms", C.c_double), ("total_ms", C.c_double),
                ("batch_size", C.c_int)]


class TokError(RuntimeError):
    def __init__(self, fn, status, detail):
        super().__init__("%s failed: status %d (%s)" % (fn, status, detail))
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libtok.so is not built (%s); run python -m paper_2602_03529_amd.build" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    vp, sz, i32, f32p = C.c_void_p, C.c_size_t, C.c_int, C.c_void_p
    L.tok_weight_count.restype = sz
    L.tok_weight_count.argtypes = []
    L.tok_model_create.restype = i32
    L.tok_model_create.argtypes = [vp, sz, i32, i32, C.POINTER(vp)]
    L.tok_model_destroy.restype = None
    L.tok_model_destroy.argtypes = [vp]
    L.tok_workspace_size.restype = i32
    L.tok_workspace_size.argtypes = [vp, i32, i32, i32, i32, i32, C.POINTER(sz)]
    L.tok_encode.restype = i32
    L.tok_encode.argtypes = [vp, vp, i32, i32, i32, i32, f32p, f32p, vp, C.POINTER(DropDesc), vp, vp, sz, vp]
    L.tok_quantize.restype = i32
    L.tok_quantize.argtypes = [vp, sz, vp, vp, vp]
    L.tok_drop.restype = i32
    L.tok_drop.argtypes = [C.POINTER(DropDesc), vp, vp, i32, i32, i32, i32, vp]
    L.tok_decode.restype = i32
    L.tok_select_workspace_size.restype = i32
    L.tok_select_workspace_size.argtypes = [i32, i32, i32, i32, C.POINTER(sz)]
    L.tok_select_similar.restype = i32
    L.tok_select_similar.argtypes = [C.c_float, vp, vp, i32, i32, i32, i32, vp, sz, vp]
    L.tok_select_scratch_bytes.restype = i32
    L.tok_select_scratch_bytes.argtypes = [C.POINTER(sz)]
    L.tok_select_similar_noalloc.restype = i32
    L.tok_select_similar_noalloc.argtypes = [C.c_float, vp, vp, i32, i32, i32, i32, vp]
    L.tok_packets_max_bytes.restype = i32
    L.tok_packets_max_bytes.argtypes = [i32, i32, i32, i32, C.POINTER(sz)]
    L.tok_packetize.restype = i32
    L.tok_packetize.argtypes = [vp, vp, i32, i32, i32, i32, vp, sz, vp, vp]
    L.tok_reassemble.restype = i32
    L.tok_reassemble.argtypes = [vp, sz, vp, sz, i32, i32, i32, i32, vp, vp, vp]
    L.tok_residual_workspace_size.restype = i32
    L.tok_residual_workspace_size.argtypes = [i32, i32, i32, C.POINTER(sz)]
    L.tok_residual_compress.restype = i32
    L.tok_residual_compress.argtypes = [vp, vp, i32, i32, i32, i32, C.c_float, vp, vp, vp, sz, vp, vp, sz, vp]
    L.tok_residual_apply.restype = i32
    L.tok_residual_apply.argtypes = [vp, vp, i32, i32, i32, i32, vp]
    L.tok_gop_blend.restype = i32
    L.tok_gop_blend.argtypes = [vp, i32, vp, i32, i32, i32, i32, i32, vp]
    L.tok_decode_blend.restype = i32
    L.tok_decode_blend.argtypes = [vp, vp, i32, i32, i32, i32, vp, i32, i32, vp, vp, sz, vp]
    L.tok_decode_residual.restype = i32
    L.tok_decode_residual.argtypes = [vp, vp, i32, i32, i32, i32, vp, C.c_float, vp, vp, vp, vp, sz, vp, vp, sz, vp,
                                      sz, vp]
    L.tok_decode.argtypes = [vp, vp, i32, i32, i32, i32, vp, vp, sz, vp]
    L.tok_model_set_weights.restype = i32
    L.tok_model_set_weights.argtypes = [vp, vp, vp]
    L.tok_train_workspace_size.restype = i32
    L.tok_train_workspace_size.argtypes = [vp, i32, i32, i32, i32, C.POINTER(sz)]
    L.tok_train_workspace_min_size.restype = i32
    L.tok_train_workspace_min_size.argtypes = [vp, i32, i32, i32, i32, C.POINTER(sz)]
    L.tok_train_forward.restype = i32
    L.tok_train_forward.argtypes = [vp, vp, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    L.tok_backward.restype = i32
    L.tok_backward.argtypes = [vp, vp, i32, i32, i32, i32, vp, vp, vp, vp, sz, vp]
    L.tok_conv3d_wgrad_workspace_size.restype = i32
    L.tok_conv3d_wgrad_workspace_size.argtypes = [i32, i32, i32, i32, i32, i32, i32, i32, C.POINTER(sz)]
    L.tok_conv3d_wgrad.restype = i32
    L.tok_conv3d_wgrad.argtypes = [i32, i32, vp, i32, i32, i32, i32, i32, vp, i32, i32, i32, i32, vp, vp, vp, sz, vp]
    L.tok_backward_outputs.restype = i32
    L.tok_backward_outputs.argtypes = [vp, vp, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    L.tok_train_codes.restype = i32
    L.tok_train_codes.argtypes = [vp, i32, i32, i32, i32, vp, vp, sz, vp]
    L.tok_op_act_pack.restype = i32
    L.tok_op_act_pack.argtypes = [i32, vp, i32, i32, i32, vp, vp]
    L.tok_op_act_unpack.restype = i32
    L.tok_op_act_unpack.argtypes = [i32, vp, i32, i32, i32, vp, vp]
    L.tok_op_conv3d_workspace_size.restype = i32
    L.tok_op_conv3d_workspace_size.argtypes = [i32, i32, i32, i32, i32, i32, i32, i32, C.POINTER(sz)]
    L.tok_op_conv3d_fwd.restype = i32
    L.tok_op_conv3d_fwd.argtypes = [i32, i32, vp, i32, i32, i32, i32, i32, vp, vp, vp, vp, i32, vp, sz, vp]
    L.tok_op_conv3d_dgrad.restype = i32
    L.tok_op_conv3d_dgrad.argtypes = [i32, i32, vp, i32, i32, i32, i32, i32, vp, vp, i32, vp, sz, vp]
    L.tok_op_conv3d_wgrad.restype = i32
    L.tok_op_conv3d_wgrad.argtypes = [i32, i32, vp, i32, i32, i32, i32, i32, vp, i32, vp, vp, vp, sz, vp]
    L.tok_op_gn_workspace_size.restype = i32
    L.tok_op_gn_workspace_size.argtypes = [i32, i32, i32, C.POINTER(sz)]
    L.tok_op_gn_stats.restype = i32
    L.tok_op_gn_stats.argtypes = [i32, vp, i32, i32, C.c_float, vp, vp, sz, vp]
    L.tok_op_gn_apply.restype = i32
    L.tok_op_gn_apply.argtypes = [i32, vp, i32, i32, vp, vp, vp, vp, vp, sz, vp]
    L.tok_op_gn_bwd.restype = i32
    L.tok_op_gn_bwd.argtypes = [i32, vp, vp, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.tok_op_fsq_ste_bwd.restype = i32
    L.tok_op_fsq_ste_bwd.argtypes = [vp, vp, vp, vp, sz, vp, vp]
    L.tok_profile_begin.restype = i32
    L.tok_profile_begin.argtypes = [vp]
    L.tok_profile_end.restype = i32
    L.tok_profile_end.argtypes = [vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_int)]
    L.tok_kernel_name.restype = C.c_char_p
    L.tok_kernel_name.argtypes = [i32]
    L.tok_server_request_bytes.restype = i32
    L.tok_server_request_bytes.argtypes = [vp, i32, i32, i32, C.POINTER(sz)]
    L.tok_server_create.restype = i32
    L.tok_server_create.argtypes = [vp, sz, i32, i32, C.POINTER(vp)]
    L.tok_server_submit.restype = i32
    L.tok_server_submit.argtypes = [vp, C.POINTER(Request), C.POINTER(C.c_uint64)]
    L.tok_server_wait.restype = i32
    L.tok_server_wait.argtypes = [vp, C.c_uint64, i32, C.POINTER(Result)]
    L.tok_server_copy_result.restype = i32
    L.tok_server_copy_result.argtypes = [vp, C.c_uint64, vp, vp, vp, vp, vp]
    L.tok_server_release.restype = i32
    L.tok_server_release.argtypes = [vp, C.c_uint64]
    L.tok_server_stats.restype = i32
    L.tok_server_stats.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(sz), C.POINTER(sz)]
    L.tok_server_destroy.restype = None
    L.tok_server_destroy.argtypes = [vp]
    L.tok_status_str.restype = C.c_char_p
    L.tok_status_str.argtypes = [i32]
    L.tok_last_error.restype = C.c_char_p
    L.tok_last_error.argtypes = []
    _lib = L
    return L


def check(fn, status):
    if status != TOK_OK:
        L = lib()
        detail = L.tok_status_str(status).decode() + ": " + L.tok_last_error().decode()
        raise TokError(fn, status, detail)
