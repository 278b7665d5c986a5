"""Thin PyTorch binding of libtok.so: the C-ABI entry points with torch
tensors for device memory and torch's current HIP stream.  Argument
marshalling only; every step of the tokenizer runs in the library's kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

PRECISIONS = {"f32": L.TOK_F32, "bf16": L.TOK_BF16, "fp8": L.TOK_FP8_E4M3}


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need(t, dtype, shape, name):
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s cuda tensor of shape %s, got %s %s" %
                         (name, dtype, tuple(shape), t.dtype, tuple(t.shape)))


def latent_shape(T, H, W):
    return (T - 1) // 4 + 1, H // 4, W // 4


@dataclass
class Drop:
    """Token-drop request (tok_drop_desc)."""
    mode: int = L.TOK_DROP_NONE
    rate: float = 0.0
    seed: int = 0
    clip_id0: int = 0
    protect_iframe: bool = False
    ext_keep: torch.Tensor | None = None

    def desc(self):
        return L.DropDesc(int(self.mode), float(self.rate), int(self.seed) & (2**64 - 1),
                          int(self.clip_id0) & (2**64 - 1), int(bool(self.protect_iframe)),
                          None if self.ext_keep is None else self.ext_keep.data_ptr())


def weight_count() -> int:
    return int(L.lib().tok_weight_count())


class TokModel:
    """A tok_model: weights packed on one device in one precision."""

    def __init__(self, weights_flat: np.ndarray, precision: str = "bf16", device: int = 0):
        w = np.ascontiguousarray(weights_flat, dtype=np.float32)
        self.lib = L.lib()
        self.device = device
        self.precision = precision
        h = C.c_void_p()
        L.check("tok_model_create", self.lib.tok_model_create(
            w.ctypes.data_as(C.c_void_p), w.size, PRECISIONS[precision], device, C.byref(h)))
        self.handle = h
        self._ws = None

    def close(self):
        if self.handle:
            self.lib.tok_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_size(self, N, T, H, W, what=L.TOK_WS_ROUNDTRIP, stream=False) -> int:
        """Workspace bytes; stream=True sizes it for causal temporal chunking."""
        if stream:
            what |= L.TOK_WS_STREAM
        n = C.c_size_t()
        L.check("tok_workspace_size", self.lib.tok_workspace_size(self.handle, N, T, H, W, what, C.byref(n)))
        return int(n.value)

    def workspace(self, N, T, H, W, what=L.TOK_WS_ROUNDTRIP):
        """A cached uint8 device tensor large enough for (N, T, H, W)."""
        need = self.workspace_size(N, T, H, W, what)
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device="cuda:%d" % self.device)
        return self._ws

    def encode(self, x: torch.Tensor, drop: Drop | None = None, z=True, keep=True, out=None, ws=None):
        """x: uint8 (N,T,H,W,3) -> dict(z, codes, idx, keep)."""
        N, T, H, W, _ = x.shape
        _need(x, torch.uint8, (N, T, H, W, 3), "x")
        T2, H2, W2 = latent_shape(T, H, W)
        dev = x.device
        o = out or {}
        zt = o.get("z") if o.get("z") is not None else (torch.empty((N, T2, H2, W2, 6), dtype=torch.float32, device=dev) if z else None)
        codes = o.get("codes") if o.get("codes") is not None else torch.empty((N, T2, H2, W2, 6), dtype=torch.float32, device=dev)
        idx = o.get("idx") if o.get("idx") is not None else torch.empty((N, T2, H2, W2), dtype=torch.int32, device=dev)
        kp = o.get("keep") if o.get("keep") is not None else (torch.empty((N, T2, H2, W2), dtype=torch.uint8, device=dev) if keep else None)
        if ws is None:
            ws = self.workspace(N, T, H, W)
        d = drop.desc() if drop is not None else None
        L.check("tok_encode", self.lib.tok_encode(
            self.handle, _ptr(x), N, T, H, W, _ptr(zt), _ptr(codes), _ptr(idx),
            C.byref(d) if d is not None else None, _ptr(kp), _ptr(ws), ws.numel(), _stream(dev)))
        return dict(z=zt, codes=codes, idx=idx, keep=kp)

    def decode(self, codes: torch.Tensor, out=None, ws=None, prev: torch.Tensor | None = None, blend_n: int = 2):
        """codes: float32 (N,T2,H2,W2,6) -> x_hat float32 (N,4(T2-1)+1,4H2,4W2,3).
        With prev (N,T_prev,4H2,4W2,3), the previous GoP's reconstruction, the
        first blend_n frames are blended with its last ones (Sec. 4.2, Eq. 2)
        inside the decoder's last conv."""
        N, T2, H2, W2, _ = codes.shape
        _need(codes, torch.float32, (N, T2, H2, W2, 6), "codes")
        T, H, W = 4 * (T2 - 1) + 1, 4 * H2, 4 * W2
        xh = out if out is not None else torch.empty((N, T, H, W, 3), dtype=torch.float32, device=codes.device)
        if ws is None:
            ws = self.workspace(N, T, H, W, L.TOK_WS_DECODE if self.precision == "fp8" else L.TOK_WS_ROUNDTRIP)
        if prev is None:
            L.check("tok_decode", self.lib.tok_decode(self.handle, _ptr(codes), N, T2, H2, W2, _ptr(xh), _ptr(ws),
                                                      ws.numel(), _stream(codes.device)))
        else:
            Tp = prev.shape[1]
            _need(prev, torch.float32, (N, Tp, H, W, 3), "prev")
            L.check("tok_decode_blend", self.lib.tok_decode_blend(
                self.handle, _ptr(codes), N, T2, H2, W2, _ptr(prev), Tp, int(blend_n), _ptr(xh), _ptr(ws), ws.numel(),
                _stream(codes.device)))
        return xh

    def decode_residual(self, codes: torch.Tensor, x: torch.Tensor, theta: float, capacity=None, out=None, ws=None):
        """decode, then the pixel residual layer (Sec. 4.3, Eq. 4) of source
        clips x uint8 (N,T,H,W,3) against the decoded clips, with the residual
        sums formed by the decoder's last conv as it writes each frame:
        dict(xhat, r (N,H,W,3), index, value, clip_offsets [N+1]), equal to
        decode then residual_compress."""
        N, T2, H2, W2, _ = codes.shape
        _need(codes, torch.float32, (N, T2, H2, W2, 6), "codes")
        T, H, W = 4 * (T2 - 1) + 1, 4 * H2, 4 * W2
        _need(x, torch.uint8, (N, T, H, W, 3), "x")
        dev = codes.device
        xh = out if out is not None else torch.empty((N, T, H, W, 3), dtype=torch.float32, device=dev)
        if ws is None:
            ws = self.workspace(N, T, H, W, L.TOK_WS_DECODE if self.precision == "fp8" else L.TOK_WS_ROUNDTRIP)
        cap = N * H * W * 3 if capacity is None else int(capacity)
        r = torch.empty((N, H, W, 3), dtype=torch.float32, device=dev)
        index = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        value = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
        co = torch.empty(N + 1, dtype=torch.uint64, device=dev)
        b = C.c_size_t()
        L.check("tok_residual_workspace_size", self.lib.tok_residual_workspace_size(N, H, W, C.byref(b)))
        rws = torch.empty(int(b.value), dtype=torch.uint8, device=dev)
        L.check("tok_decode_residual", self.lib.tok_decode_residual(
            self.handle, _ptr(codes), N, T2, H2, W2, _ptr(x), float(theta), _ptr(xh), _ptr(r), _ptr(index),
            _ptr(value), cap, _ptr(co), _ptr(ws), ws.numel(), _ptr(rws), rws.numel(), _stream(dev)))
        return dict(xhat=xh, r=r, index=index, value=value, clip_offsets=co)


    # ---- training step (tok_train_forward / tok_backward) -----------------
    def set_weights(self, w: torch.Tensor):
        """Replace the parameters by a device float32 blob (canonical order) and repack."""
        _need(w, torch.float32, (weight_count(),), "weights")
        L.check("tok_model_set_weights", self.lib.tok_model_set_weights(self.handle, _ptr(w), _stream(w.device)))

    def train_workspace_size(self, N, T, H, W, recompute=False) -> int:
        """Training workspace bytes.  The default size keeps every residual
        block's interior on the tape; recompute=True gives the smallest one,
        with which the backward recomputes them (same gradients, bit for bit)."""
        n = C.c_size_t()
        if recompute:
            L.check("tok_train_workspace_min_size",
                    self.lib.tok_train_workspace_min_size(self.handle, N, T, H, W, C.byref(n)))
        else:
            L.check("tok_train_workspace_size", self.lib.tok_train_workspace_size(self.handle, N, T, H, W, C.byref(n)))
        return int(n.value)

    def train_forward(self, x: torch.Tensor, keep: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                      xhat=False, z=False, idx=False):
        """Loss of the training objective on uint8 clips x (N,T,H,W,3).  Returns
        dict(loss=float32 (3,) {L, l1 term, commitment mean}, ws=the workspace
        holding the tape, and the requested optional outputs)."""
        N, T, H, W, _ = x.shape
        _need(x, torch.uint8, (N, T, H, W, 3), "x")
        T2, H2, W2 = latent_shape(T, H, W)
        dev = x.device
        if keep is not None:
            _need(keep, torch.uint8, (N, T2, H2, W2), "keep")
        if ws is None:
            ws = torch.empty(self.train_workspace_size(N, T, H, W), dtype=torch.uint8, device=dev)
        loss = torch.empty(3, dtype=torch.float32, device=dev)
        out = dict(loss=loss, ws=ws)
        out["xhat"] = torch.empty((N, T, H, W, 3), dtype=torch.float32, device=dev) if xhat else None
        out["z"] = torch.empty((N, T2, H2, W2, 6), dtype=torch.float32, device=dev) if z else None
        out["idx"] = torch.empty((N, T2, H2, W2), dtype=torch.int32, device=dev) if idx else None
        L.check("tok_train_forward", self.lib.tok_train_forward(
            self.handle, _ptr(x), N, T, H, W, _ptr(keep), _ptr(loss), _ptr(out["xhat"]), _ptr(out["z"]),
            _ptr(out["idx"]), _ptr(ws), ws.numel(), _stream(dev)))
        return out

    def backward(self, x: torch.Tensor, ws: torch.Tensor, gloss: torch.Tensor | None = None,
                 dweights: torch.Tensor | None = None, dx=False):
        """Gradients of the last train_forward on (x, ws): dict(dweights, dx)."""
        N, T, H, W, _ = x.shape
        _need(x, torch.uint8, (N, T, H, W, 3), "x")
        dev = x.device
        if gloss is not None:
            _need(gloss, torch.float32, (1,), "gloss")
        if dweights is None:
            dweights = torch.empty(weight_count(), dtype=torch.float32, device=dev)
        dxt = torch.empty((N, T, H, W, 3), dtype=torch.float32, device=dev) if dx else None
        L.check("tok_backward", self.lib.tok_backward(
            self.handle, _ptr(x), N, T, H, W, _ptr(gloss), _ptr(dweights), _ptr(dxt), _ptr(ws), ws.numel(),
            _stream(dev)))
        return dict(dweights=dweights, dx=dxt)


    def backward_outputs(self, x: torch.Tensor, ws: torch.Tensor, gxhat: torch.Tensor,
                         gcodes: torch.Tensor | None = None, gz: torch.Tensor | None = None,
                         dweights: torch.Tensor | None = None, dx=False):
        """Gradients of <gxhat, x_hat> + <gcodes, keep c> + <gz, z> for the last
        train_forward on (x, ws) (tok_backward_outputs): dict(dweights, dx)."""
        N, T, H, W, _ = x.shape
        _need(x, torch.uint8, (N, T, H, W, 3), "x")
        T2, H2, W2 = latent_shape(T, H, W)
        dev = x.device
        _need(gxhat, torch.float32, (N, T, H, W, 3), "gxhat")
        for t, nm in ((gcodes, "gcodes"), (gz, "gz")):
            if t is not None:
                _need(t, torch.float32, (N, T2, H2, W2, 6), nm)
        if dweights is None:
            dweights = torch.empty(weight_count(), dtype=torch.float32, device=dev)
        dxt = torch.empty((N, T, H, W, 3), dtype=torch.float32, device=dev) if dx else None
        L.check("tok_backward_outputs", self.lib.tok_backward_outputs(
            self.handle, _ptr(x), N, T, H, W, _ptr(gxhat), _ptr(gcodes), _ptr(gz), _ptr(dweights), _ptr(dxt),
            _ptr(ws), ws.numel(), _stream(dev)))
        return dict(dweights=dweights, dx=dxt)

    def train_codes(self, x_shape, ws: torch.Tensor) -> torch.Tensor:
        """The zero-filled codes keep * c the last train_forward on ws decoded."""
        N, T, H, W = x_shape[:4]
        T2, H2, W2 = latent_shape(T, H, W)
        codes = torch.empty((N, T2, H2, W2, 6), dtype=torch.float32, device=ws.device)
        L.check("tok_train_codes", self.lib.tok_train_codes(self.handle, N, T, H, W, _ptr(codes), _ptr(ws),
                                                            ws.numel(), _stream(ws.device)))
        return codes


def conv3d_wgrad(x: torch.Tensor, dy: torch.Tensor, shape_x, shape_y, Cin: int, Cout: int, view: int,
                 precision: str = "bf16", with_bias: bool = True):
    """tok_conv3d_wgrad on chunked-layout device tensors x, dy (float32 or
    bfloat16 storage); shape_x = (N, Ti, Hi, Wi), shape_y = (N, To, Ho, Wo).
    Returns (dw float32 (Cout, Cin, 3, 3, 3), db float32 (Cout) or None)."""
    N, Ti, Hi, Wi = shape_x
    _, To, Ho, Wo = shape_y
    prec = PRECISIONS[precision]
    dev = x.device
    n = C.c_size_t()
    lb = L.lib()
    L.check("tok_conv3d_wgrad_workspace_size", lb.tok_conv3d_wgrad_workspace_size(
        prec, view, N, To, Ho, Wo, Cin, Cout, C.byref(n)))
    ws = torch.empty(int(n.value), dtype=torch.uint8, device=dev)
    dw = torch.empty((Cout, Cin, 3, 3, 3), dtype=torch.float32, device=dev)
    db = torch.empty(Cout, dtype=torch.float32, device=dev) if with_bias else None
    L.check("tok_conv3d_wgrad", lb.tok_conv3d_wgrad(
        prec, view, _ptr(x), N, Ti, Hi, Wi, Cin, _ptr(dy), To, Ho, Wo, Cout, _ptr(dw), _ptr(db), _ptr(ws),
        ws.numel(), _stream(dev)))
    return dw, db


def _load_params(model, params):
    """Make the model hold `params` (repacking only when they changed)."""
    key = (params.data_ptr(), params._version)
    if getattr(model, "_params_key", None) != key:
        model.set_weights(params.detach())
        model._params_key = key


class TokenizerLoss(torch.autograd.Function):
    """L(params) of the training objective with the library's hand-written
    backward: forward runs tok_train_forward (after loading `params` into the
    model when they changed), backward runs tok_backward with the incoming
    gradient as its scale.  Each call keeps its own tape (workspace) until its
    backward has run; the backward recomputes block interiors with the
    weights of its own forward (reloaded if another call changed the model's
    weights in between; autograd rejects params modified in place)."""

    @staticmethod
    def forward(ctx, params, model, x, keep):
        _load_params(model, params)
        out = model.train_forward(x, keep)
        ctx.save_for_backward(params)
        ctx.model, ctx.x, ctx.ws = model, x, out["ws"]
        model.last_loss = out["loss"]
        return out["loss"][0].clone()

    @staticmethod
    def backward(ctx, gout):
        (params,) = ctx.saved_tensors
        _load_params(ctx.model, params)
        g = gout.detach().reshape(1).to(torch.float32).contiguous()
        res = ctx.model.backward(ctx.x, ctx.ws, gloss=g)
        ctx.ws = None
        return res["dweights"], None, None, None


def tokenizer_loss(model: "TokModel", params: torch.Tensor, x: torch.Tensor, keep: torch.Tensor | None = None):
    """Differentiable training loss; params: float32 (weight_count(),) cuda tensor."""
    return TokenizerLoss.apply(params, model, x, keep)


class Tokenizer(torch.autograd.Function):
    """The codec as one differentiable stage (Sec. 4.1 gradient interface):
    forward returns (x_hat, keep * c, z) of tok_train_forward for `params`;
    backward takes the gradients of those three outputs from whatever loss the
    caller computes and runs tok_backward_outputs (straight-through
    quantiser), returning the parameter gradient.  The tape lives in the
    call's own workspace until its backward has run."""

    @staticmethod
    def forward(ctx, params, model, x, keep):
        _load_params(model, params)
        out = model.train_forward(x, keep, xhat=True, z=True)
        codes = model.train_codes(tuple(x.shape), out["ws"])
        ctx.save_for_backward(params)
        ctx.model, ctx.x, ctx.ws = model, x, out["ws"]
        return out["xhat"], codes, out["z"]

    @staticmethod
    def backward(ctx, gxhat, gcodes, gz):
        (params,) = ctx.saved_tensors
        _load_params(ctx.model, params)
        x = ctx.x
        N, T, H, W, _ = x.shape
        if gxhat is None:
            gxhat = torch.zeros((N, T, H, W, 3), dtype=torch.float32, device=x.device)
        prep = (lambda g: None if g is None else g.detach().to(torch.float32).contiguous())
        res = ctx.model.backward_outputs(x, ctx.ws, prep(gxhat), prep(gcodes), prep(gz))
        ctx.ws = None
        return res["dweights"], None, None, None


def tokenizer(model: "TokModel", params: torch.Tensor, x: torch.Tensor, keep: torch.Tensor | None = None):
    """(x_hat, zero-filled codes, z) as differentiable functions of params."""
    return Tokenizer.apply(params, model, x, keep)


# ---------------------------------------------------------------------------
# Per-operation entry points (tok_op_*) and their autograd wrappers.
# Activations are torch tensors in the library's chunked layout
# (N, T, ceil(C/CH), H, W, CH) of float32 (CH = 16) or bfloat16 (CH = 32).
# ---------------------------------------------------------------------------
_OP_DTYPES = {"f32": torch.float32, "bf16": torch.bfloat16}


def _prec_of(t: torch.Tensor) -> str:
    for k, v in _OP_DTYPES.items():
        if t.dtype == v:
            return k
    raise ValueError("activations are float32 or bfloat16, got %s" % t.dtype)


def act_shape(N, T, H, W, C, precision):
    ch = 32 if precision == "bf16" else 16
    return (N, T, (C + ch - 1) // ch, H, W, ch)


def act_pack(x: torch.Tensor, precision: str = "bf16") -> torch.Tensor:
    """Dense float32 (N, T, H, W, C) -> chunked activations (tok_op_act_pack)."""
    assert x.dtype == torch.float32 and x.dim() == 5 and x.is_cuda and x.is_contiguous()
    N, T, H, W, Cc = x.shape
    out = torch.empty(act_shape(N, T, H, W, Cc, precision), dtype=_OP_DTYPES[precision], device=x.device)
    L.check("tok_op_act_pack", L.lib().tok_op_act_pack(PRECISIONS[precision], _ptr(x), N * T, H * W, Cc,
                                                       _ptr(out), _stream(x.device)))
    return out


def act_unpack(a: torch.Tensor, C_: int) -> torch.Tensor:
    """Chunked activations (N, T, chunks, H, W, CH) -> dense float32 (N, T, H, W, C)."""
    assert a.dim() == 6 and a.is_cuda and a.is_contiguous()
    N, T, _, H, W, _ = a.shape
    out = torch.empty((N, T, H, W, C_), dtype=torch.float32, device=a.device)
    L.check("tok_op_act_unpack", L.lib().tok_op_act_unpack(PRECISIONS[_prec_of(a)], _ptr(a), N * T, H * W, C_,
                                                           _ptr(out), _stream(a.device)))
    return out


def _view_out(view, Ti, Hi, Wi):
    if view == 0:
        return Ti, Hi, Wi
    if view == 1:
        return (Ti - 1) // 2 + 1, Hi // 2, Wi // 2
    return 2 * Ti - 1, 2 * Hi, 2 * Wi


def _conv_ws(precision, view, N, Ti, Hi, Wi, Cin, Cout, dev):
    n = C.c_size_t()
    L.check("tok_op_conv3d_workspace_size", L.lib().tok_op_conv3d_workspace_size(
        PRECISIONS[precision], view, N, Ti, Hi, Wi, Cin, Cout, C.byref(n)))
    return torch.empty(int(n.value), dtype=torch.uint8, device=dev)


def conv3d_fwd(x, w, b, view, shape_x, Cin, Cout, precision, resid=None):
    """tok_op_conv3d_fwd.  x: chunked activations, or uint8 pixels (N,T,H,W,3)
    when Cin = 3; returns chunked y, or dense float32 (N,To,Ho,Wo,3) when Cout = 3."""
    N, Ti, Hi, Wi = shape_x
    To, Ho, Wo = _view_out(view, Ti, Hi, Wi)
    dev = w.device
    if Cout == 3:
        y = torch.empty((N, To, Ho, Wo, 3), dtype=torch.float32, device=dev)
    else:
        y = torch.empty(act_shape(N, To, Ho, Wo, Cout, precision), dtype=_OP_DTYPES[precision], device=dev)
    ws = _conv_ws(precision, view, N, Ti, Hi, Wi, Cin, Cout, dev)
    L.check("tok_op_conv3d_fwd", L.lib().tok_op_conv3d_fwd(
        PRECISIONS[precision], view, _ptr(x), N, Ti, Hi, Wi, Cin, _ptr(w), _ptr(b), _ptr(resid), _ptr(y), Cout,
        _ptr(ws), ws.numel(), _stream(dev)))
    return y


def conv3d_dgrad(dy, w, view, shape_x, Cin, Cout, precision):
    """tok_op_conv3d_dgrad: dx (chunked, or dense float32 (N,T,H,W,3) when Cin = 3)."""
    N, Ti, Hi, Wi = shape_x
    dev = w.device
    if Cin == 3:
        dx = torch.empty((N, Ti, Hi, Wi, 3), dtype=torch.float32, device=dev)
    else:
        dx = torch.empty(act_shape(N, Ti, Hi, Wi, Cin, precision), dtype=_OP_DTYPES[precision], device=dev)
    ws = _conv_ws(precision, view, N, Ti, Hi, Wi, Cin, Cout, dev)
    L.check("tok_op_conv3d_dgrad", L.lib().tok_op_conv3d_dgrad(
        PRECISIONS[precision], view, _ptr(dy), N, Ti, Hi, Wi, Cin, _ptr(w), _ptr(dx), Cout, _ptr(ws), ws.numel(),
        _stream(dev)))
    return dx


def conv3d_wgrad_op(x, dy, view, shape_x, Cin, Cout, precision, with_bias=True):
    """tok_op_conv3d_wgrad: (dw float32 (Cout, Cin, 3, 3, 3), db float32 (Cout) or None)."""
    N, Ti, Hi, Wi = shape_x
    dev = dy.device
    dw = torch.empty((Cout, Cin, 3, 3, 3), dtype=torch.float32, device=dev)
    db = torch.empty(Cout, dtype=torch.float32, device=dev) if with_bias else None
    ws = _conv_ws(precision, view, N, Ti, Hi, Wi, Cin, Cout, dev)
    L.check("tok_op_conv3d_wgrad", L.lib().tok_op_conv3d_wgrad(
        PRECISIONS[precision], view, _ptr(x), N, Ti, Hi, Wi, Cin, _ptr(dy), Cout, _ptr(dw), _ptr(db), _ptr(ws),
        ws.numel(), _stream(dev)))
    return dw, db


def _gn_ws(precision, frames, HW, dev):
    n = C.c_size_t()
    L.check("tok_op_gn_workspace_size", L.lib().tok_op_gn_workspace_size(PRECISIONS[precision], frames, HW,
                                                                         C.byref(n)))
    return torch.empty(int(n.value), dtype=torch.uint8, device=dev)


def _gn_dims(x):
    N, T, _, H, W, _ = x.shape
    return N * T, H * W


def gn_stats(x, eps=1e-6):
    """tok_op_gn_stats: (mean, rstd) float32 (frames, 32, 2) of a 64-channel chunked tensor."""
    precision = _prec_of(x)
    frames, HW = _gn_dims(x)
    mr = torch.empty((frames, 32, 2), dtype=torch.float32, device=x.device)
    ws = _gn_ws(precision, frames, HW, x.device)
    L.check("tok_op_gn_stats", L.lib().tok_op_gn_stats(PRECISIONS[precision], _ptr(x), frames, HW, float(eps),
                                                       _ptr(mr), _ptr(ws), ws.numel(), _stream(x.device)))
    return mr


def gn_apply(x, mr, gamma, beta):
    """tok_op_gn_apply: SiLU(GroupNorm(x)) in x's layout."""
    precision = _prec_of(x)
    frames, HW = _gn_dims(x)
    y = torch.empty_like(x)
    ws = _gn_ws(precision, frames, HW, x.device)
    L.check("tok_op_gn_apply", L.lib().tok_op_gn_apply(PRECISIONS[precision], _ptr(x), frames, HW, _ptr(mr),
                                                       _ptr(gamma), _ptr(beta), _ptr(y), _ptr(ws), ws.numel(),
                                                       _stream(x.device)))
    return y


def gn_bwd(x, dy, mr, gamma, beta, resid=None):
    """tok_op_gn_bwd: (dx, dgamma, dbeta)."""
    precision = _prec_of(x)
    frames, HW = _gn_dims(x)
    dx = torch.empty_like(x)
    dg = torch.empty(64, dtype=torch.float32, device=x.device)
    dbt = torch.empty(64, dtype=torch.float32, device=x.device)
    ws = _gn_ws(precision, frames, HW, x.device)
    L.check("tok_op_gn_bwd", L.lib().tok_op_gn_bwd(PRECISIONS[precision], _ptr(x), _ptr(dy), frames, HW, _ptr(mr),
                                                   _ptr(gamma), _ptr(beta), _ptr(resid), _ptr(dx), _ptr(dg),
                                                   _ptr(dbt), _ptr(ws), ws.numel(), _stream(x.device)))
    return dx, dg, dbt


def fsq_ste_bwd(z, gcodes, keep=None, gz_in=None):
    """tok_op_fsq_ste_bwd: dL/dz of the straight-through quantiser."""
    n = z.numel() // 6
    gz = torch.empty_like(z)
    L.check("tok_op_fsq_ste_bwd", L.lib().tok_op_fsq_ste_bwd(_ptr(z), _ptr(keep), _ptr(gcodes), _ptr(gz_in), n,
                                                             _ptr(gz), _stream(z.device)))
    return gz


class Conv3dFn(torch.autograd.Function):
    """Causal 3x3x3 conv with the library's adjoint kernels (tok_op_conv3d_*)."""

    @staticmethod
    def forward(ctx, x, w, b, view, shape_x, Cin, Cout, precision, resid=None):
        w = w.detach().contiguous()
        b = None if b is None else b.detach().contiguous()
        y = conv3d_fwd(x.detach(), w, b, view, shape_x, Cin, Cout, precision,
                       None if resid is None else resid.detach())
        ctx.save_for_backward(x, w)
        ctx.cfg = (view, tuple(shape_x), Cin, Cout, precision, b is not None, resid is not None)
        return y

    @staticmethod
    def backward(ctx, gy):
        x, w = ctx.saved_tensors
        view, shape_x, Cin, Cout, precision, has_b, has_r = ctx.cfg
        gy = gy.contiguous()
        dx = None
        if ctx.needs_input_grad[0] and Cin != 3:
            dx = conv3d_dgrad(gy, w, view, shape_x, Cin, Cout, precision)
        dw, db = conv3d_wgrad_op(x, gy, view, shape_x, Cin, Cout, precision, with_bias=has_b)
        return dx, dw, db, None, None, None, None, None, (gy if has_r else None)


class GroupNormSiLUFn(torch.autograd.Function):
    """SiLU(GroupNorm(32)(x)) per frame on 64-channel chunked activations."""

    @staticmethod
    def forward(ctx, x, gamma, beta, eps=1e-6):
        x = x.detach()
        gamma, beta = gamma.detach().contiguous(), beta.detach().contiguous()
        mr = gn_stats(x, eps)
        ctx.save_for_backward(x, mr, gamma, beta)
        return gn_apply(x, mr, gamma, beta)

    @staticmethod
    def backward(ctx, gy):
        x, mr, gamma, beta = ctx.saved_tensors
        dx, dg, db = gn_bwd(x, gy.contiguous(), mr, gamma, beta)
        return dx, dg, db, None


class FsqSTEFn(torch.autograd.Function):
    """keep * FSQ(z) with the straight-through gradient (tok_quantize,
    tok_drop with an external mask, tok_op_fsq_ste_bwd)."""

    @staticmethod
    def forward(ctx, z, keep=None):
        z = z.detach().contiguous()
        codes, _ = quantize(z)
        if keep is not None:
            N, T2, H2, W2, _ = codes.shape
            drop(codes, Drop(mode=L.TOK_DROP_EXTERNAL, ext_keep=keep), keep=False)
        ctx.save_for_backward(z, keep)
        return codes

    @staticmethod
    def backward(ctx, gc):
        z, keep = ctx.saved_tensors
        return fsq_ste_bwd(z, gc.contiguous(), keep), None


KERNEL_IDS = 24


class Profile:
    """Context manager: per-kernel HIP-event timing of the model's launches."""

    def __init__(self, model: "TokModel"):
        self.model = model
        self.ms = {}
        self.count = {}

    def __enter__(self):
        L.check("tok_profile_begin", self.model.lib.tok_profile_begin(self.model.handle))
        return self

    def __exit__(self, *exc):
        ms = (C.c_double * KERNEL_IDS)()
        cnt = (C.c_int * KERNEL_IDS)()
        L.check("tok_profile_end", self.model.lib.tok_profile_end(self.model.handle, KERNEL_IDS, ms, cnt))
        for k in range(KERNEL_IDS):
            name = self.model.lib.tok_kernel_name(k).decode()
            self.ms[name] = ms[k]
            self.count[name] = cnt[k]
        return False


def quantize(z: torch.Tensor):
    """FSQ of float32 (..., 6) latents -> (codes, idx)."""
    assert z.dtype == torch.float32 and z.shape[-1] == 6 and z.is_cuda and z.is_contiguous()
    n = z.numel() // 6
    codes = torch.empty_like(z)
    idx = torch.empty(z.shape[:-1], dtype=torch.int32, device=z.device)
    L.check("tok_quantize", L.lib().tok_quantize(_ptr(z), n, _ptr(codes), _ptr(idx), _stream(z.device)))
    return codes, idx


def drop(codes: torch.Tensor | None, d: Drop, shape=None, keep=True):
    """Zero-fill codes (N,T2,H2,W2,6) in place by the mask of `d`; returns keep."""
    if codes is not None:
        N, T2, H2, W2, _ = codes.shape
        dev = codes.device
    else:
        N, T2, H2, W2 = shape
        dev = torch.device("cuda")
    kp = torch.empty((N, T2, H2, W2), dtype=torch.uint8, device=dev) if keep else None
    desc = d.desc()
    L.check("tok_drop", L.lib().tok_drop(C.byref(desc), _ptr(codes), _ptr(kp), N, T2, H2, W2, _stream(dev)))
    return kp


def select_workspace_size(N: int, T2: int, H2: int, W2: int) -> int:
    b = C.c_size_t()
    L.check("tok_select_workspace_size", L.lib().tok_select_workspace_size(N, T2, H2, W2, C.byref(b)))
    return int(b.value)


def select_similar(codes: torch.Tensor, rate: float, keep=True, ws=None):
    """Similarity-based token selection (Sec. 4.3, Eq. 3) on codes
    (N,T2,H2,W2,6) in place; returns keep (N,T2,H2,W2) uint8 or None."""
    N, T2, H2, W2, _ = codes.shape
    _need(codes, torch.float32, (N, T2, H2, W2, 6), "codes")
    dev = codes.device
    kp = torch.empty((N, T2, H2, W2), dtype=torch.uint8, device=dev) if keep else None
    if ws is None:
        ws = torch.empty(select_workspace_size(N, T2, H2, W2), dtype=torch.uint8, device=dev)
    L.check("tok_select_similar", L.lib().tok_select_similar(float(rate), _ptr(codes), _ptr(kp), N, T2, H2, W2,
                                                             _ptr(ws), ws.numel(), _stream(dev)))
    return kp


def select_scratch_bytes() -> int:
    b = C.c_size_t()
    L.check("tok_select_scratch_bytes", L.lib().tok_select_scratch_bytes(C.byref(b)))
    return int(b.value)


def select_similar_noalloc(codes: torch.Tensor, rate: float, keep=True):
    """select_similar on the library's static per-GPU scratch (no workspace,
    no device allocation by the library); calls on one GPU must not overlap."""
    N, T2, H2, W2, _ = codes.shape
    _need(codes, torch.float32, (N, T2, H2, W2, 6), "codes")
    dev = codes.device
    kp = torch.empty((N, T2, H2, W2), dtype=torch.uint8, device=dev) if keep else None
    L.check("tok_select_similar_noalloc",
            L.lib().tok_select_similar_noalloc(float(rate), _ptr(codes), _ptr(kp), N, T2, H2, W2, _stream(dev)))
    return kp


def packetize(idx: torch.Tensor, keep: torch.Tensor | None = None):
    """Row packets (Sec. 6.2) of FSQ indices (N,T2,H2,W2) int32 under keep:
    returns (buf uint8 of the worst-case length, offsets uint64 [N T2 H2 + 1];
    offsets[-1] is the stream's length)."""
    N, T2, H2, W2 = idx.shape
    _need(idx, torch.int32, (N, T2, H2, W2), "idx")
    if keep is not None:
        _need(keep, torch.uint8, (N, T2, H2, W2), "keep")
    dev = idx.device
    b = C.c_size_t()
    L.check("tok_packets_max_bytes", L.lib().tok_packets_max_bytes(N, T2, H2, W2, C.byref(b)))
    buf = torch.empty(int(b.value), dtype=torch.uint8, device=dev)
    offs = torch.empty(N * T2 * H2 + 1, dtype=torch.uint64, device=dev)
    L.check("tok_packetize", L.lib().tok_packetize(_ptr(idx), _ptr(keep), N, T2, H2, W2, _ptr(buf), buf.numel(),
                                                   _ptr(offs), _stream(dev)))
    return buf, offs


def reassemble(buf: torch.Tensor, offsets: torch.Tensor, shape, keep=True, nbytes=None):
    """Receiver (Sec. 6.2): codes (N,T2,H2,W2,6) float32 and keep from the
    packets of buf starting at `offsets` (uint64, any order)."""
    N, T2, H2, W2 = shape
    dev = buf.device
    assert buf.dtype == torch.uint8 and buf.is_contiguous()
    assert offsets.dtype == torch.uint64 and offsets.is_contiguous() and offsets.device == dev
    codes = torch.empty((N, T2, H2, W2, 6), dtype=torch.float32, device=dev)
    kp = torch.empty((N, T2, H2, W2), dtype=torch.uint8, device=dev) if keep else None
    nb = buf.numel() if nbytes is None else min(int(nbytes), buf.numel())
    L.check("tok_reassemble", L.lib().tok_reassemble(_ptr(buf), nb, _ptr(offsets), offsets.numel(), N, T2, H2, W2,
                                                     _ptr(codes), _ptr(kp), _stream(dev)))
    return codes, kp


def residual_compress(x: torch.Tensor, xhat: torch.Tensor, theta: float, capacity=None, ws=None):
    """Pixel residual layer (Sec. 4.3, Eq. 4): dict(r (N,H,W,3), index, value,
    clip_offsets [N+1]) for clips x uint8 and reconstructions xhat float32."""
    N, T, H, W, _ = x.shape
    _need(x, torch.uint8, (N, T, H, W, 3), "x")
    _need(xhat, torch.float32, (N, T, H, W, 3), "xhat")
    dev = x.device
    cap = N * H * W * 3 if capacity is None else int(capacity)
    r = torch.empty((N, H, W, 3), dtype=torch.float32, device=dev)
    index = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    value = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
    co = torch.empty(N + 1, dtype=torch.uint64, device=dev)
    if ws is None:
        b = C.c_size_t()
        L.check("tok_residual_workspace_size", L.lib().tok_residual_workspace_size(N, H, W, C.byref(b)))
        ws = torch.empty(int(b.value), dtype=torch.uint8, device=dev)
    L.check("tok_residual_compress", L.lib().tok_residual_compress(
        _ptr(x), _ptr(xhat), N, T, H, W, float(theta), _ptr(r), _ptr(index), _ptr(value), cap, _ptr(co), _ptr(ws),
        ws.numel(), _stream(dev)))
    return dict(r=r, index=index, value=value, clip_offsets=co)


def residual_apply(r: torch.Tensor, xhat: torch.Tensor):
    """xhat (N,T,H,W,3) += r (N,H,W,3) for every frame, in place."""
    N, T, H, W, _ = xhat.shape
    _need(xhat, torch.float32, (N, T, H, W, 3), "xhat")
    _need(r, torch.float32, (N, H, W, 3), "r")
    L.check("tok_residual_apply", L.lib().tok_residual_apply(_ptr(r), _ptr(xhat), N, T, H, W, _stream(xhat.device)))
    return xhat


def gop_blend(prev: torch.Tensor, xhat: torch.Tensor, n: int = 2):
    """GoP-boundary blending (Sec. 4.2, Eq. 2) of xhat's first n frames with
    prev's last n, in place."""
    N, T, H, W, _ = xhat.shape
    _need(xhat, torch.float32, (N, T, H, W, 3), "xhat")
    Tp = prev.shape[1]
    _need(prev, torch.float32, (N, Tp, H, W, 3), "prev")
    L.check("tok_gop_blend", L.lib().tok_gop_blend(_ptr(prev), Tp, _ptr(xhat), N, T, H, W, int(n),
                                                   _stream(xhat.device)))
    return xhat


class GopStream:
    """Decodes consecutive GoPs of a stream with boundary blending (Sec. 4.2,
    Eq. 2): each GoP's first n frames are blended, inside the decoder, with
    the last n frames of the previous GoP's output, which the stream keeps."""

    def __init__(self, model: TokModel, n: int = 2):
        self.model, self.n, self.tail = model, int(n), None

    def decode(self, codes: torch.Tensor, ws=None) -> torch.Tensor:
        if self.tail is not None and self.tail.shape[0] != codes.shape[0]:
            raise ValueError("batch size changed within a stream")
        xh = self.model.decode(codes, ws=ws, prev=self.tail, blend_n=self.n)
        self.tail = xh[:, xh.shape[1] - self.n:].contiguous()
        return xh

    def reset(self):
        self.tail = None


class TokServer:
    """tok_server: streaming request loop with continuous batching under an HBM budget."""

    def __init__(self, model: TokModel, budget_bytes: int, slots: int = 4, max_batch: int = 4):
        self.model = model
        self.lib = model.lib
        h = C.c_void_p()
        L.check("tok_server_create", self.lib.tok_server_create(model.handle, int(budget_bytes), slots, max_batch,
                                                                 C.byref(h)))
        self.handle = h
        self._pixels = {}

    def request_bytes(self, T, H, W) -> int:
        n = C.c_size_t()
        L.check("tok_server_request_bytes", self.lib.tok_server_request_bytes(self.model.handle, T, H, W,
                                                                               C.byref(n)))
        return int(n.value)

    def submit(self, pixels: torch.Tensor, drop: Drop | None = None) -> int:
        """pixels: host uint8 (T,H,W,3), ideally pinned; kept alive until the request is released."""
        assert pixels.dtype == torch.uint8 and not pixels.is_cuda and pixels.is_contiguous()
        T, H, W, _ = pixels.shape
        d = (drop or Drop()).desc()
        req = L.Request(T, H, W, pixels.data_ptr(), d)
        t = C.c_uint64()
        L.check("tok_server_submit", self.lib.tok_server_submit(self.handle, C.byref(req), C.byref(t)))
        self._pixels[t.value] = pixels
        return int(t.value)

    def wait(self, ticket: int, timeout_ms: int = -1):
        """Result metadata (dict) once done, or None on time-out."""
        r = L.Result()
        rc = self.lib.tok_server_wait(self.handle, ticket, timeout_ms, C.byref(r))
        if rc > 0:
            return None
        L.check("tok_server_wait", rc)
        return dict(ticket=r.ticket, status=r.status, latent=(r.T2, r.H2, r.W2), queue_ms=r.queue_ms,
                    run_ms=r.run_ms, total_ms=r.total_ms, batch_size=r.batch_size)

    def fetch(self, ticket: int, T: int, H: int, W: int):
        """Copy a finished request's results into new device tensors."""
        T2, H2, W2 = latent_shape(T, H, W)
        dev = torch.device("cuda:%d" % self.model.device)
        codes = torch.empty((T2, H2, W2, 6), dtype=torch.float32, device=dev)
        idx = torch.empty((T2, H2, W2), dtype=torch.int32, device=dev)
        keep = torch.empty((T2, H2, W2), dtype=torch.uint8, device=dev)
        xhat = torch.empty((T, H, W, 3), dtype=torch.float32, device=dev)
        L.check("tok_server_copy_result", self.lib.tok_server_copy_result(
            self.handle, ticket, _ptr(codes), _ptr(idx), _ptr(keep), _ptr(xhat), _stream(dev)))
        return dict(codes=codes, idx=idx, keep=keep, xhat=xhat)

    def release(self, ticket: int):
        L.check("tok_server_release", self.lib.tok_server_release(self.handle, ticket))
        self._pixels.pop(ticket, None)

    def stats(self):
        q, r, f = C.c_int(), C.c_int(), C.c_int()
        u, p = C.c_size_t(), C.c_size_t()
        L.check("tok_server_stats", self.lib.tok_server_stats(self.handle, C.byref(q), C.byref(r), C.byref(f),
                                                              C.byref(u), C.byref(p)))
        return dict(queued=q.value, running=r.value, finished=f.value, bytes_in_use=u.value, bytes_peak=p.value)

    def close(self):
        if self.handle:
            self.lib.tok_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
