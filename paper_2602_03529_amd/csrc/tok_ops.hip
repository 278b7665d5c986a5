// C ABI of the per-operation entry points (tok_op_*; contract in
// include/tok.h): the causal 3x3x3 convolution and its two adjoints,
// GroupNorm(32)+SiLU forward and backward, the straight-through quantiser
// adjoint, and layout conversion.  They run the same kernels as the fused
// encode / decode / training paths, on caller tensors and a caller workspace.
#include <algorithm>
#include <string>

#include "tok.h"
#include "tok_model.h"

using namespace tok;

namespace {

bool op_prec(tok_precision p, int* P) {
  if (p == TOK_F32) { *P = P_F32; return true; }
  if (p == TOK_BF16) { *P = P_BF16; return true; }
  return false;
}
int chan_chunk(int P) { return P == P_BF16 ? 32 : 16; }
size_t elem_bytes(int P) { return P == P_BF16 ? 2 : 4; }
bool al16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Output shape of a view; false if the input shape does not fit it.
bool view_out(int view, int Ti, int Hi, int Wi, int* To, int* Ho, int* Wo) {
  if (Ti < 1 || Hi < 1 || Wi < 1) return false;
  if (view == 0) { *To = Ti; *Ho = Hi; *Wo = Wi; return true; }
  if (view == 1) {
    if (Ti % 2 != 1 || Hi % 2 != 0 || Wi % 2 != 0) return false;
    *To = (Ti - 1) / 2 + 1; *Ho = Hi / 2; *Wo = Wi / 2;
    return true;
  }
  if (view == 2) { *To = 2 * Ti - 1; *Ho = 2 * Hi; *Wo = 2 * Wi; return true; }
  return false;
}

// The channel configurations the kernels implement: 3-channel tensors only as
// the first layer's pixels (Cin = 3 -> Cout = 64, stride 1) or the last
// layer's RGB output (Cout = 3, stride 1); otherwise whole 64-channel tiles.
bool op_channels(int view, int Cin, int Cout) {
  if (Cin == 3) return view == 0 && Cout == 64;
  if (Cout == 3) return view == 0 && Cin % 64 == 0;
  return Cin % 64 == 0 && Cout % 64 == 0 && Cin > 0 && Cout > 0;
}

// Workspace carve-up of the conv ops (every part 256-byte aligned).
struct ConvOpWs {
  size_t pk, zeros, stats, tmp, wp, wbp, total;
  int splits, nt, ntT;
};

int fwd_mode(int view, int Cin) {
  if (view == 0) return Cin == 3 ? CM_I2C : CM_S1;
  return view == 1 ? CM_S2 : CM_UPF;
}
int wgrad_view_mode(int view) { return view == 0 ? CM_S1 : (view == 1 ? CM_S2 : CM_UP); }
// input-gradient conv of a view: polyphase for stride 2, and for the upsampling view in fp32
int adj_op_mode(int P, int view) {
  if (view == 1) return CM_S2T;
  if (view == 2 && P == P_F32) return CM_UPT;
  return CM_S1T;
}

ConvOpWs conv_op_ws(int P, int view, int N, int Ti, int Hi, int Wi, int Cin, int Cout) {
  int To, Ho, Wo;
  view_out(view, Ti, Hi, Wi, &To, &Ho, &Wo);
  ConvOpWs w{};
  const size_t es = elem_bytes(P);
  const size_t pf = packed_conv_elems(Cout, Cin, P, fwd_mode(view, Cin), &w.nt);
  const size_t pa = packed_conv_elems(Cout, Cin, P, adj_op_mode(P, view), &w.ntT);
  w.pk = align256(std::max(pf, pa) * es);
  w.zeros = align256((size_t)std::max(Cin, Cout) * 4);
  const size_t tiles = (size_t)cdiv(Ho, 8) * cdiv(Wo, 64);
  w.stats = Cin == 3 ? align256((size_t)N * To * tiles * 32 * sizeof(float4)) : 0;
  // fine-resolution temporaries of the adjoints and one-chunk copies of 3-channel operands
  size_t tmp = 0;
  if (view == 2 && adj_op_mode(P, view) == CM_S1T) tmp = (size_t)N * To * Ho * Wo * cdiv(Cin, chan_chunk(P)) * kChunkBytes;
  if (Cout == 3) tmp = (size_t)N * To * Ho * Wo * kChunkBytes;
  if (Cin == 3) tmp = (size_t)N * Ti * Hi * Wi * kChunkBytes;
  w.tmp = align256(tmp);
  const int wm = wgrad_view_mode(view);
  const int per = wgrad_blocks_per_split(P, wm, Cout, Cin);
  const int items = wgrad_items(P, wm, Cout, Cin, N, To, Ho, Wo);
  w.splits = std::max(1, std::min(items, std::max(1, 2048 / per)));
  w.wp = align256((size_t)w.splits * wgrad_partial_taps(P, wm) * Cout * Cin * 4);
  w.wbp = align256((size_t)w.splits * wgrad_bias_parts(P, wm) * Cout * 4);
  w.total = w.pk + w.zeros + w.stats + w.tmp + w.wp + w.wbp;
  return w;
}

struct ConvOpArgs {
  int P, view, N, Ti, Hi, Wi, Cin, Cout, To, Ho, Wo;
  ConvOpWs w;
  char* ws;
};

tok_status conv_op_check(tok_precision prec, int view, int N, int Ti, int Hi, int Wi, int Cin, int Cout, void* ws,
                         size_t ws_bytes, ConvOpArgs* a) {
  if (!op_prec(prec, &a->P)) return fail(TOK_EUNSUPPORTED, "per-op convolutions take TOK_F32 or TOK_BF16");
  if (view < 0 || view > 2) return fail(TOK_EINVAL, "view must be 0 (stride 1), 1 (stride 2) or 2 (upsample x2)");
  if (N < 1 || !view_out(view, Ti, Hi, Wi, &a->To, &a->Ho, &a->Wo))
    return fail(TOK_ESHAPE, "input shape does not fit the view (stride 2 needs odd T and even H, W)");
  if (!op_channels(view, Cin, Cout))
    return fail(TOK_EUNSUPPORTED, "channels: multiples of 64, or 3 -> 64 / 64k -> 3 at stride 1");
  if ((long long)N * a->To > 65535 || (long long)N * Ti > 65535) return fail(TOK_ESHAPE, "N T above 65535");
  a->view = view; a->N = N; a->Ti = Ti; a->Hi = Hi; a->Wi = Wi; a->Cin = Cin; a->Cout = Cout;
  a->w = conv_op_ws(a->P, view, N, Ti, Hi, Wi, Cin, Cout);
  if (!ws) return fail(TOK_EINVAL, "null workspace");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(TOK_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < a->w.total) return fail(TOK_EWORKSPACE, "workspace needs " + std::to_string(a->w.total) + " bytes");
  a->ws = static_cast<char*>(ws);
  return TOK_OK;
}

char* ws_pk(const ConvOpArgs& a) { return a.ws; }
float* ws_zeros(const ConvOpArgs& a) { return reinterpret_cast<float*>(a.ws + a.w.pk); }
float4* ws_stats(const ConvOpArgs& a) { return reinterpret_cast<float4*>(a.ws + a.w.pk + a.w.zeros); }
char* ws_tmp(const ConvOpArgs& a) { return a.ws + a.w.pk + a.w.zeros + a.w.stats; }
float* ws_wp(const ConvOpArgs& a) { return reinterpret_cast<float*>(ws_tmp(a) + a.w.tmp); }
float* ws_wbp(const ConvOpArgs& a) { return reinterpret_cast<float*>(ws_tmp(a) + a.w.tmp + a.w.wp); }

// One conv launch on whole clips (input buffer frames = computed frames' source).
hipError_t run_conv(const ConvOpArgs& o, int mode, const void* wpk, const float* bias, int nt, int Cin, int Cout,
                    const void* in, int in_kind, int Ti, int Hi, int Wi, void* out, int out_kind, int To, int Ho,
                    int Wo, const void* resid, float4* stats, hipStream_t s) {
  const int CH = chan_chunk(o.P);
  ConvLaunch a;
  std::memset(&a, 0, sizeof(a));
  a.in = in;
  a.N = o.N; a.Ti = Ti; a.Hi = Hi; a.Wi = Wi;
  a.gi0 = 0;
  a.in_chunks = mode == CM_I2C ? kI2cK / CH : cdiv(Cin, CH);
  a.Cin = Cin;
  a.wpk = wpk;
  a.bias = bias;
  a.Cout = Cout;
  a.nt = nt;
  a.cout_tiles = cdiv(Cout, nt);
  a.out = out;
  a.resid = resid;
  a.To = To; a.Ho = Ho; a.Wo = Wo;
  a.To_buf = To; a.out_f0 = 0; a.go0 = 0;
  a.out_chunks = cdiv(Cout, CH);
  a.stats = stats;
  int th, tw;
  conv_tile(mode, &th, &tw);
  a.tiles_h = cdiv(Ho, th);
  a.tiles_w = cdiv(Wo, tw);
  a.mode = mode; a.in_kind = in_kind; a.out_kind = out_kind; a.prec = o.P;
  return launch_conv(a, s);
}

}  // namespace

extern "C" {

tok_status tok_op_act_pack(tok_precision prec, const float* src, int frames, int HW, int C, void* dst,
                           hipStream_t s) {
  int P;
  if (!op_prec(prec, &P)) return fail(TOK_EUNSUPPORTED, "layout conversion takes TOK_F32 or TOK_BF16");
  if (!src || !dst) return fail(TOK_EINVAL, "null argument");
  if (frames < 0 || HW < 0 || C < 1) return fail(TOK_ESHAPE, "bad shape");
  if (!al16(dst)) return fail(TOK_EINVAL, "dst must be 16-byte aligned");
  TOK_HIP(launch_act_pack(src, frames, HW, C, P, dst, s));
  return TOK_OK;
}

tok_status tok_op_act_unpack(tok_precision prec, const void* src, int frames, int HW, int C, float* dst,
                             hipStream_t s) {
  int P;
  if (!op_prec(prec, &P)) return fail(TOK_EUNSUPPORTED, "layout conversion takes TOK_F32 or TOK_BF16");
  if (!src || !dst) return fail(TOK_EINVAL, "null argument");
  if (frames < 0 || HW < 0 || C < 1) return fail(TOK_ESHAPE, "bad shape");
  if (!al16(src)) return fail(TOK_EINVAL, "src must be 16-byte aligned");
  TOK_HIP(launch_act_unpack(src, frames, HW, C, P, dst, s));
  return TOK_OK;
}

tok_status tok_op_conv3d_workspace_size(tok_precision prec, int view, int N, int Ti, int Hi, int Wi, int Cin,
                                        int Cout, size_t* bytes) {
  if (!bytes) return fail(TOK_EINVAL, "null argument");
  ConvOpArgs a;
  char dummy alignas(256)[1];
  const tok_status st = conv_op_check(prec, view, N, Ti, Hi, Wi, Cin, Cout, dummy, ~(size_t)0, &a);
  if (st != TOK_OK) return st;
  *bytes = a.w.total;
  return TOK_OK;
}

tok_status tok_op_conv3d_fwd(tok_precision prec, int view, const void* x, int N, int Ti, int Hi, int Wi, int Cin,
                             const float* w, const float* b, const void* resid, void* y, int Cout, void* ws,
                             size_t ws_bytes, hipStream_t s) {
  if (!x || !w || !y) return fail(TOK_EINVAL, "null argument");
  ConvOpArgs a;
  TOK_TRY(conv_op_check(prec, view, N, Ti, Hi, Wi, Cin, Cout, ws, ws_bytes, &a));
  if (resid && (view != 0 || Cout == 3)) return fail(TOK_EUNSUPPORTED, "a residual needs stride 1 and 64k outputs");
  if ((Cin != 3 && !al16(x)) || !al16(y) || (resid && !al16(resid)))
    return fail(TOK_EINVAL, "activations must be 16-byte aligned");
  const int mode = fwd_mode(view, Cin);
  TOK_HIP(launch_pack_weights(w, Cout, Cin, a.P, mode, ws_pk(a), nullptr, s));
  const float* bias = b;
  if (!bias) {
    TOK_HIP(launch_fill_zero(ws_zeros(a), (size_t)Cout, s));
    bias = ws_zeros(a);
  }
  const int in_kind = Cin == 3 ? IN_U8 : IN_ACT;
  const int out_kind = Cout == 3 ? OUT_RGB32 : OUT_ACT;
  float4* stats = Cin == 3 ? ws_stats(a) : nullptr;  // the first-layer kernel always writes GN partials
  TOK_HIP(run_conv(a, mode, ws_pk(a), bias, a.w.nt, Cin, Cout, x, in_kind, Ti, Hi, Wi, y, out_kind, a.To, a.Ho, a.Wo,
                   resid, stats, s));
  return TOK_OK;
}

tok_status tok_op_conv3d_dgrad(tok_precision prec, int view, const void* dy, int N, int Ti, int Hi, int Wi, int Cin,
                               const float* w, void* dx, int Cout, void* ws, size_t ws_bytes, hipStream_t s) {
  if (!dy || !w || !dx) return fail(TOK_EINVAL, "null argument");
  ConvOpArgs a;
  TOK_TRY(conv_op_check(prec, view, N, Ti, Hi, Wi, Cin, Cout, ws, ws_bytes, &a));
  if ((Cout != 3 && !al16(dy)) || (Cin != 3 && !al16(dx))) return fail(TOK_EINVAL, "activations must be 16-byte aligned");
  const int CH = chan_chunk(a.P);
  TOK_HIP(launch_pack_weights(w, Cout, Cin, a.P, adj_op_mode(a.P, view), ws_pk(a), nullptr, s));
  TOK_HIP(launch_fill_zero(ws_zeros(a), (size_t)Cin, s));
  const int out_kind = Cin == 3 ? OUT_RGB32 : OUT_ACT;
  const void* g = dy;
  if (Cout == 3) {
    // dense RGB gradient -> one-chunk activations
    TOK_HIP(launch_rgb_to_chunk(static_cast<const float*>(dy), (size_t)N * a.To * a.Ho * a.Wo, a.P, ws_tmp(a), s));
    g = ws_tmp(a);
  }
  if (view == 0) {
    TOK_HIP(run_conv(a, CM_S1T, ws_pk(a), ws_zeros(a), a.w.ntT, Cout, Cin, g, IN_ACT, Ti, Hi, Wi, dx, out_kind, Ti,
                     Hi, Wi, nullptr, nullptr, s));
  } else if (view == 1) {
    // stride 2: the polyphase adjoint, coarse gradient in, fine gradient out
    TOK_HIP(run_conv(a, CM_S2T, ws_pk(a), ws_zeros(a), a.w.ntT, Cout, Cin, g, IN_ACT, a.To, a.Ho, a.Wo, dx, OUT_ACT,
                     Ti, Hi, Wi, nullptr, nullptr, s));
  } else if (adj_op_mode(a.P, view) == CM_UPT) {
    // upsampling view, fp32: the polyphase adjoint, fine gradient in, source gradient out
    TOK_HIP(run_conv(a, CM_UPT, ws_pk(a), ws_zeros(a), a.w.ntT, Cout, Cin, g, IN_ACT, a.To, a.Ho, a.Wo, dx, OUT_ACT,
                     Ti, Hi, Wi, nullptr, nullptr, s));
  } else {
    // upsample then stride-1 conv: the stride-1 adjoint at the fine resolution, then the upsample adjoint
    TOK_HIP(run_conv(a, CM_S1T, ws_pk(a), ws_zeros(a), a.w.ntT, Cout, Cin, g, IN_ACT, a.To, a.Ho, a.Wo, ws_tmp(a),
                     OUT_ACT, a.To, a.Ho, a.Wo, nullptr, nullptr, s));
    TOK_HIP(launch_up_adjoint(ws_tmp(a), dx, N, Ti, Hi, Wi, cdiv(Cin, CH), a.P, s));
  }
  return TOK_OK;
}

tok_status tok_op_conv3d_wgrad(tok_precision prec, int view, const void* x, int N, int Ti, int Hi, int Wi, int Cin,
                               const void* dy, int Cout, float* dw, float* db, void* ws, size_t ws_bytes,
                               hipStream_t s) {
  if (!x || !dy || !dw) return fail(TOK_EINVAL, "null argument");
  ConvOpArgs a;
  TOK_TRY(conv_op_check(prec, view, N, Ti, Hi, Wi, Cin, Cout, ws, ws_bytes, &a));
  if ((Cin != 3 && !al16(x)) || (Cout != 3 && !al16(dy))) return fail(TOK_EINVAL, "activations must be 16-byte aligned");
  const int CH = chan_chunk(a.P);
  const void* xa = x;
  const void* ga = dy;
  if (Cin == 3) {
    TOK_HIP(launch_u8_to_chunked(static_cast<const uint8_t*>(x), (size_t)N * Ti * Hi * Wi, a.P, ws_tmp(a), s));
    xa = ws_tmp(a);
  }
  if (Cout == 3) {
    TOK_HIP(launch_rgb_to_chunk(static_cast<const float*>(dy), (size_t)N * a.To * a.Ho * a.Wo, a.P, ws_tmp(a), s));
    ga = ws_tmp(a);
  }
  WgradLaunch g;
  std::memset(&g, 0, sizeof(g));
  g.x = xa; g.N = N; g.Ti = Ti; g.Hi = Hi; g.Wi = Wi; g.x_chunks = cdiv(Cin, CH);
  g.dy = ga; g.To = a.To; g.Ho = a.Ho; g.Wo = a.Wo; g.dy_chunks = cdiv(Cout, CH);
  g.Cout = Cout; g.Cin = Cin; g.view = wgrad_view_mode(view); g.prec = a.P; g.splits = a.w.splits;
  g.partial = ws_wp(a);
  g.bpartial = ws_wbp(a);
  TOK_HIP(launch_wgrad(g, s));
  TOK_HIP(launch_wgrad_reduce(g, dw, db, s));
  return TOK_OK;
}

// ---- GroupNorm(32) + SiLU -------------------------------------------------

namespace {
struct GnOpWs { size_t stats, sc, gnp, fsum, m12, total; };
GnOpWs gn_op_ws(int P, int frames, int HW) {
  GnOpWs w;
  w.stats = align256((size_t)frames * gn_op_tiles(HW) * 32 * sizeof(float4));
  w.sc = align256((size_t)frames * 64 * 4) * 2;
  w.gnp = align256(gn_bwd_partial_floats(frames, HW, P) * 4);
  w.fsum = align256((size_t)frames * 64 * 8);
  w.m12 = align256((size_t)frames * 32 * 8);
  w.total = w.stats + w.sc + w.gnp + w.fsum + w.m12;
  return w;
}
tok_status gn_op_check(tok_precision prec, int frames, int HW, void* ws, size_t ws_bytes, int* P, GnOpWs* w) {
  if (!op_prec(prec, P)) return fail(TOK_EUNSUPPORTED, "GroupNorm ops take TOK_F32 or TOK_BF16");
  if (frames < 1 || HW < 1 || frames * (64 / chan_chunk(*P)) > 65535) return fail(TOK_ESHAPE, "bad shape");
  *w = gn_op_ws(*P, frames, HW);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(TOK_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < w->total) return fail(TOK_EWORKSPACE, "workspace needs " + std::to_string(w->total) + " bytes");
  return TOK_OK;
}
}  // namespace

tok_status tok_op_gn_workspace_size(tok_precision prec, int frames, int HW, size_t* bytes) {
  int P;
  if (!bytes) return fail(TOK_EINVAL, "null argument");
  if (!op_prec(prec, &P)) return fail(TOK_EUNSUPPORTED, "GroupNorm ops take TOK_F32 or TOK_BF16");
  if (frames < 1 || HW < 1) return fail(TOK_ESHAPE, "bad shape");
  *bytes = gn_op_ws(P, frames, HW).total;
  return TOK_OK;
}

tok_status tok_op_gn_stats(tok_precision prec, const void* x, int frames, int HW, float eps, float* mean_rstd,
                           void* ws, size_t ws_bytes, hipStream_t s) {
  int P;
  GnOpWs w;
  TOK_TRY(gn_op_check(prec, frames, HW, ws, ws_bytes, &P, &w));
  if (!x || !mean_rstd) return fail(TOK_EINVAL, "null argument");
  if (!al16(x) || (reinterpret_cast<uintptr_t>(mean_rstd) & 7)) return fail(TOK_EINVAL, "misaligned argument");
  if (!(eps >= 0.f)) return fail(TOK_EINVAL, "eps must be >= 0");
  float4* st = static_cast<float4*>(ws);
  TOK_HIP(launch_gn_partials(x, frames, HW, P, st, s));
  TOK_HIP(launch_gn_finalize(st, frames, gn_op_tiles(HW), nullptr, nullptr, eps, nullptr, nullptr,
                             reinterpret_cast<float2*>(mean_rstd), s));
  return TOK_OK;
}

tok_status tok_op_gn_apply(tok_precision prec, const void* x, int frames, int HW, const float* mean_rstd,
                           const float* gamma, const float* beta, void* y, void* ws, size_t ws_bytes, hipStream_t s) {
  int P;
  GnOpWs w;
  TOK_TRY(gn_op_check(prec, frames, HW, ws, ws_bytes, &P, &w));
  if (!x || !mean_rstd || !gamma || !beta || !y) return fail(TOK_EINVAL, "null argument");
  if (!al16(x) || !al16(y) || (reinterpret_cast<uintptr_t>(mean_rstd) & 7)) return fail(TOK_EINVAL, "misaligned argument");
  float* sc = reinterpret_cast<float*>(static_cast<char*>(ws) + w.stats);
  float* sh = sc + align256((size_t)frames * 64 * 4) / 4;
  TOK_HIP(launch_gn_affine(reinterpret_cast<const float2*>(mean_rstd), gamma, beta, frames, sc, sh, s));
  TOK_HIP(launch_gn_act(x, 1, 0, y, 1, 0, P, frames, 1, HW, sc, sh, s));
  return TOK_OK;
}

tok_status tok_op_gn_bwd(tok_precision prec, const void* x, const void* dy, int frames, int HW,
                         const float* mean_rstd, const float* gamma, const float* beta, const void* resid, void* dx,
                         float* dgamma, float* dbeta, void* ws, size_t ws_bytes, hipStream_t s) {
  int P;
  GnOpWs w;
  TOK_TRY(gn_op_check(prec, frames, HW, ws, ws_bytes, &P, &w));
  if (!x || !dy || !mean_rstd || !gamma || !beta || !dx || !dgamma || !dbeta) return fail(TOK_EINVAL, "null argument");
  if (!al16(x) || !al16(dy) || !al16(dx) || (resid && !al16(resid))) return fail(TOK_EINVAL, "misaligned argument");
  char* b = static_cast<char*>(ws) + w.stats + w.sc;
  float* gnp = reinterpret_cast<float*>(b);
  float2* fsum = reinterpret_cast<float2*>(b + w.gnp);
  float2* m12 = reinterpret_cast<float2*>(b + w.gnp + w.fsum);
  TOK_HIP(launch_gn_bwd(x, dy, reinterpret_cast<const float2*>(mean_rstd), gamma, beta, resid, dx, frames, HW, P, gnp,
                        fsum, m12, dgamma, dbeta, s));
  return TOK_OK;
}

tok_status tok_op_fsq_ste_bwd(const float* z, const uint8_t* keep, const float* gcodes, const float* gz_in,
                              size_t n_tokens, float* gz, hipStream_t s) {
  if (n_tokens && (!z || !gz)) return fail(TOK_EINVAL, "null argument");
  TOK_HIP(launch_fsq_ste(z, keep, gcodes, nullptr, gz_in, n_tokens, make_fsq_const(), gz, s));
  return TOK_OK;
}

}  // extern "C"
