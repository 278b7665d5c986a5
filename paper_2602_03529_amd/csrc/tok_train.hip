// C ABI of the training step: tok_train_workspace_size, tok_train_forward,
// tok_backward (see include/tok.h for the contract).
//
// The forward pass runs the tokenizer on whole clips and keeps a tape of the
// block-boundary activations (the input and output of every residual block
// and of every other layer), the GroupNorm statistics, the latent and the
// mask.  The backward pass walks the layers in reverse:
//   * a 3x3x3 conv's input gradient is the adjoint conv (anti-causal,
//     flipped, channel-transposed; conv3d.hip CM_S1T) on the output gradient,
//     after zero insertion for the stride-2 convs and followed by the
//     upsample adjoint for the upsampling convs;
//   * its weight and bias gradients come from the deterministic split-K
//     weight-gradient kernel (fp32 MFMA);
//   * each residual block takes its interior (GroupNorm_a+SiLU output,
//     conv_a output, GroupNorm_b+SiLU output) from the tape when the
//     workspace holds it, else recomputes it from its tape input (per-block
//     checkpointing), then back-propagates through conv_b, GroupNorm_b+SiLU,
//     conv_a, GroupNorm_a+SiLU and the skip;
//   * FSQ passes the decoder gradient straight through (masked tokens pass
//     none) and adds the commitment term's gradient.
#include <algorithm>
#include <string>

#include "tok.h"
#include "tok_model.h"

using namespace tok;

namespace {

constexpr int kWgradTargetBlocks = 2048;

// Workspace layout of one training step.
struct TrainPlan {
  Dims d;
  size_t npos, ntok;
  size_t l0, l1, l2, px;
  // level 0 (64 channels): tape, then work buffers (S and C adjacent: together
  // they are one 128-channel level-0 buffer)
  size_t H0, E1, E2, U1, R1, R2, S, C, S2, GA, GB, GX;
  size_t D1, U2, G1a, G1b;  // level 1 (128 channels)
  size_t D2, P, G2a, G2b;   // level 2 (128 channels)
  size_t Z, DEC, GZ, GDEC, KEEP, XHAT;
  size_t SC, SH, MR;        // per norm: N*T*64 scale, shift; N*T*32 (mean, rstd)
  bool keep_rb;             // residual-block interiors kept on the tape (no recompute)
  size_t RBI;               // [4 blocks][3] level-0 interior buffers when keep_rb
  size_t STATS, WP, WBP, GNP, FSUM, M12, L1P, CMP, O6P, LOSS;
  size_t total;
};

struct WgradShape { int layer, view, Ti, Hi, Wi, To, Ho, Wo; };

int wgrad_splits(int prec, int view, int Cout, int Cin, int N, int To, int Ho, int Wo) {
  const int per = wgrad_blocks_per_split(prec, view, Cout, Cin);
  const int items = wgrad_items(prec, view, Cout, Cin, N, To, Ho, Wo);
  return std::max(1, std::min(items, std::max(1, kWgradTargetBlocks / per)));
}

std::vector<WgradShape> wgrad_shapes(const Dims& d) {
  std::vector<WgradShape> v;
  const int rb[8] = {L_E_RB1_A, L_E_RB1_B, L_E_RB2_A, L_E_RB2_B, L_D_RB1_A, L_D_RB1_B, L_D_RB2_A, L_D_RB2_B};
  for (int l : rb) v.push_back({l, CM_S1, d.T, d.H, d.W, d.T, d.H, d.W});
  v.push_back({L_CONV_IN, CM_S1, d.T, d.H, d.W, d.T, d.H, d.W});
  v.push_back({L_CONV_OUT, CM_S1, d.T, d.H, d.W, d.T, d.H, d.W});
  v.push_back({L_DOWN1, CM_S2, d.T, d.H, d.W, d.T1, d.H1, d.W1});
  v.push_back({L_DOWN2, CM_S2, d.T1, d.H1, d.W1, d.T2, d.H2, d.W2});
  v.push_back({L_UP2, CM_UP, d.T2, d.H2, d.W2, d.T1, d.H1, d.W1});
  v.push_back({L_UP1, CM_UP, d.T1, d.H1, d.W1, d.T, d.H, d.W});
  return v;
}

TrainPlan make_train_plan(const Dims& d, int prec, bool keep_rb) {
  const size_t es = prec == P_BF16 ? 2 : 4;
  TrainPlan p;
  p.d = d;
  p.keep_rb = keep_rb;
  p.npos = (size_t)d.N * d.T * d.H * d.W;
  p.ntok = (size_t)d.N * d.T2 * d.H2 * d.W2;
  p.l0 = align256(p.npos * 64 * es);
  p.l1 = align256((size_t)d.N * d.T1 * d.H1 * d.W1 * 128 * es);
  p.l2 = align256(p.ntok * 128 * es);
  p.px = align256(p.npos * kChunkBytes);
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t r = o; o += align256(bytes); return r; };
  p.H0 = take(p.l0); p.E1 = take(p.l0); p.E2 = take(p.l0); p.U1 = take(p.l0); p.R1 = take(p.l0); p.R2 = take(p.l0);
  p.S = take(p.l0); p.C = take(p.l0); p.S2 = take(p.l0); p.GA = take(p.l0); p.GB = take(p.l0);
  p.GX = take(p.px);
  p.D1 = take(p.l1); p.U2 = take(p.l1); p.G1a = take(p.l1); p.G1b = take(p.l1);
  p.D2 = take(p.l2); p.P = take(p.l2); p.G2a = take(p.l2); p.G2b = take(p.l2);
  p.Z = take(p.ntok * 6 * 4); p.DEC = take(p.ntok * 6 * 4); p.GZ = take(p.ntok * 6 * 4);
  p.GDEC = take(p.ntok * 6 * 4); p.KEEP = take(p.ntok); p.XHAT = take(p.npos * 3 * 4);
  const size_t frames = (size_t)d.N * d.T;
  p.SC = take(N_COUNT * frames * 64 * 4); p.SH = take(N_COUNT * frames * 64 * 4);
  p.MR = take(N_COUNT * frames * 32 * 8);
  const size_t tiles0 = (size_t)cdiv(d.H, 8) * cdiv(d.W, 64);
  p.STATS = take(frames * tiles0 * 32 * sizeof(float4));
  size_t wp = 0, wbp = 0;
  for (const WgradShape& w : wgrad_shapes(d)) {
    const ConvSpec& c = kConv[w.layer];
    const size_t sp = wgrad_splits(prec, w.view, c.cout, c.cin, d.N, w.To, w.Ho, w.Wo);
    wp = std::max(wp, sp * wgrad_partial_taps(prec, w.view) * c.cout * c.cin);
    wbp = std::max(wbp, sp * wgrad_bias_parts(prec, w.view) * c.cout);
  }
  p.WP = take(wp * 4); p.WBP = take(wbp * 4);
  p.GNP = take(gn_bwd_partial_floats((int)frames, d.H * d.W, prec) * 4);
  p.FSUM = take(frames * 64 * 8); p.M12 = take(frames * 32 * 8);
  p.L1P = take((size_t)l1_blocks(p.npos) * 4); p.CMP = take((size_t)fsq_blocks(p.ntok) * 4);
  p.O6P = take(outer6_partial_floats(p.ntok) * 4);
  p.LOSS = take(4 * 4);
  p.RBI = keep_rb ? take(12 * p.l0) : 0;
  p.total = o;
  return p;
}

struct TrainCtx {
  tok_model* m;
  TrainPlan p;
  char* base;
  hipStream_t s;
  int CH;
  template <class T = void> T* at(size_t off) const { return reinterpret_cast<T*>(base + off); }
  float* sc(int norm) const { return at<float>(p.SC) + (size_t)norm * p.d.N * p.d.T * 64; }
  float* sh(int norm) const { return at<float>(p.SH) + (size_t)norm * p.d.N * p.d.T * 64; }
  float2* mr(int norm) const { return at<float2>(p.MR) + (size_t)norm * p.d.N * p.d.T * 32; }
};

// One conv launch on whole clips.
tok_status tconv(const TrainCtx& c, int kid, int mode, const void* wpk, const float* bias, int nt, int Cin, int Cout,
                 const void* in, int in_kind, int Ti, int Hi, int Wi, void* out, int out_kind, int To, int Ho, int Wo,
                 const void* resid, float4* stats) {
  ConvLaunch a;
  std::memset(&a, 0, sizeof(a));
  a.in = in;
  a.N = c.p.d.N; a.Ti = Ti; a.Hi = Hi; a.Wi = Wi;
  a.gi0 = 0;
  a.in_chunks = mode == CM_I2C ? kI2cK / c.CH : cdiv(Cin, c.CH);
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
  a.out_chunks = cdiv(Cout, c.CH);
  a.stats = stats;
  int th, tw;
  conv_tile(mode, &th, &tw);
  a.tiles_h = cdiv(Ho, th);
  a.tiles_w = cdiv(Wo, tw);
  a.mode = mode; a.in_kind = in_kind; a.out_kind = out_kind; a.prec = c.m->prec;
  Timed tm(c.m, kid, c.s);
  const hipError_t e = launch_conv(a, c.s);
  if (e != hipSuccess) return fail(TOK_EDEVICE, "conv (kernel id " + std::to_string(kid) + "): " + hipGetErrorString(e));
  return TOK_OK;
}

// Forward conv of layer l.
tok_status fwd(const TrainCtx& c, int l, const void* in, int in_kind, int Ti, int Hi, int Wi, void* out,
               int out_kind, int To, int Ho, int Wo, const void* resid, bool stats) {
  const tok_model* m = c.m;
  return tconv(c, l, conv_mode(l), m->wpk[l], m->bias[l], m->nt[l], kConv[l].cin, kConv[l].cout, in, in_kind, Ti,
               Hi, Wi, out, out_kind, To, Ho, Wo, resid, stats ? c.at<float4>(c.p.STATS) : nullptr);
}

// Input gradient of layer l's stride-1 conv (after zero insertion for the
// stride-2 ones, before the upsample adjoint for the upsampling ones).
tok_status adj(const TrainCtx& c, int l, const void* gy, int T, int H, int W, void* gx, int out_kind) {
  const tok_model* m = c.m;
  return tconv(c, K_DGRAD, CM_S1T, m->wpkT[l], m->zeros, m->ntT[l], kConv[l].cout, kConv[l].cin, gy, IN_ACT, T, H, W,
               gx, out_kind, T, H, W, nullptr, nullptr);
}

// Input gradient of layer l's stride-2 conv: coarse gradient (Tc, Hc, Wc) in,
// fine gradient (2 Tc - 1, 2 Hc, 2 Wc) out, in polyphase form.
tok_status adj_s2(const TrainCtx& c, int l, const void* gy, int Tc, int Hc, int Wc, void* gx) {
  const tok_model* m = c.m;
  return tconv(c, K_DGRAD, CM_S2T, m->wpkT[l], m->zeros, m->ntT[l], kConv[l].cout, kConv[l].cin, gy, IN_ACT, Tc, Hc,
               Wc, gx, OUT_ACT, 2 * Tc - 1, 2 * Hc, 2 * Wc, nullptr, nullptr);
}

// Input gradient of layer l's upsampling conv in polyphase form (fp32 models):
// fine gradient (Tf, Hf, Wf) in, source gradient ((Tf + 1) / 2, Hf / 2, Wf / 2) out.
tok_status adj_up(const TrainCtx& c, int l, const void* gy, int Tf, int Hf, int Wf, void* gx) {
  const tok_model* m = c.m;
  return tconv(c, K_DGRAD, CM_UPT, m->wpkT[l], m->zeros, m->ntT[l], kConv[l].cout, kConv[l].cin, gy, IN_ACT, Tf, Hf,
               Wf, gx, OUT_ACT, (Tf + 1) / 2, Hf / 2, Wf / 2, nullptr, nullptr);
}

tok_status wgrad(const TrainCtx& c, int l, int view, const void* x, int Ti, int Hi, int Wi, const void* dy, int To,
                 int Ho, int Wo, float* dweights) {
  const ConvSpec& cs = kConv[l];
  WgradLaunch a;
  std::memset(&a, 0, sizeof(a));
  a.x = x; a.N = c.p.d.N; a.Ti = Ti; a.Hi = Hi; a.Wi = Wi; a.x_chunks = cdiv(cs.cin, c.CH);
  a.dy = dy; a.To = To; a.Ho = Ho; a.Wo = Wo; a.dy_chunks = cdiv(cs.cout, c.CH);
  a.Cout = cs.cout; a.Cin = cs.cin; a.view = view; a.prec = c.m->prec;
  a.splits = wgrad_splits(c.m->prec, view, cs.cout, cs.cin, c.p.d.N, To, Ho, Wo);
  a.partial = c.at<float>(c.p.WP);
  a.bpartial = c.at<float>(c.p.WBP);
  Timed tm(c.m, K_WGRAD, c.s);
  hipError_t e = launch_wgrad(a, c.s);
  if (e == hipSuccess)
    e = launch_wgrad_reduce(a, dweights + c.m->w_off[l], dweights + c.m->b_off[l], c.s);
  if (e != hipSuccess) return fail(TOK_EDEVICE, "wgrad layer " + std::to_string(l) + ": " + hipGetErrorString(e));
  return TOK_OK;
}

tok_status gn_final(const TrainCtx& c, int norm) {
  const Dims& d = c.p.d;
  Timed tm(c.m, K_GN_FINAL, c.s);
  TOK_HIP(launch_gn_finalize(c.at<float4>(c.p.STATS), d.N * d.T, cdiv(d.H, 8) * cdiv(d.W, 64), c.m->gamma[norm],
                             c.m->beta[norm], kGnEps, c.sc(norm), c.sh(norm), c.mr(norm), c.s));
  return TOK_OK;
}

tok_status gn_act(const TrainCtx& c, int norm, const void* in, void* out) {
  const Dims& d = c.p.d;
  Timed tm(c.m, K_GN_ACT, c.s);
  TOK_HIP(launch_gn_act(in, d.T, 0, out, d.T, 0, c.m->prec, d.N, d.T, d.H * d.W, c.sc(norm), c.sh(norm), c.s));
  return TOK_OK;
}

tok_status gn_bwd(const TrainCtx& c, int norm, const void* x, const void* g, const void* resid, void* dx,
                  float* dweights) {
  const Dims& d = c.p.d;
  Timed tm(c.m, K_GN_BWD, c.s);
  TOK_HIP(launch_gn_bwd(x, g, c.mr(norm), c.m->gamma[norm], c.m->beta[norm], resid, dx, d.N * d.T, d.H * d.W,
                        c.m->prec, c.at<float>(c.p.GNP), c.at<float2>(c.p.FSUM), c.at<float2>(c.p.M12),
                        dweights + c.m->g_off[norm], dweights + c.m->be_off[norm], c.s));
  return TOK_OK;
}

// Interior buffer k (0: GroupNorm_a+SiLU output, 1: conv_a output, 2:
// GroupNorm_b+SiLU output) of the residual block whose first conv is la.
void* rb_interior(const TrainCtx& c, int la, int k) {
  const int rb = la == L_E_RB1_A ? 0 : (la == L_E_RB2_A ? 1 : (la == L_D_RB1_A ? 2 : 3));
  return c.at(c.p.RBI + (size_t)(rb * 3 + k) * c.p.l0);
}

// Residual block forward, out of place: Y = X + conv_b(silu(gn_b(conv_a(silu(gn_a X))))).
// On entry the stats buffer holds X's per-tile GroupNorm partials.  The
// interior goes to the tape when it is kept, else to work buffers.
tok_status rb_forward(const TrainCtx& c, int la, int na, const void* X, void* Y, bool out_stats) {
  const Dims& d = c.p.d;
  void* S = c.p.keep_rb ? rb_interior(c, la, 0) : c.at(c.p.S);
  void* C = c.p.keep_rb ? rb_interior(c, la, 1) : c.at(c.p.C);
  void* S2 = c.p.keep_rb ? rb_interior(c, la, 2) : S;
  TOK_TRY(gn_final(c, na));
  TOK_TRY(gn_act(c, na, X, S));
  TOK_TRY(fwd(c, la, S, IN_ACT, d.T, d.H, d.W, C, OUT_ACT, d.T, d.H, d.W, nullptr, true));
  TOK_TRY(gn_final(c, na + 1));
  TOK_TRY(gn_act(c, na + 1, C, S2));
  return fwd(c, la + 1, S2, IN_ACT, d.T, d.H, d.W, Y, OUT_ACT, d.T, d.H, d.W, X, out_stats);
}

// Residual block backward.  GB holds dL/dY on entry and dL/dX on exit.
tok_status rb_backward(const TrainCtx& c, int la, int na, const void* X, float* dweights) {
  const Dims& d = c.p.d;
  void* S = c.at(c.p.S);
  void* C = c.at(c.p.C);
  void* S2 = c.at(c.p.S2);
  void* GA = c.at(c.p.GA);
  void* GB = c.at(c.p.GB);
  const int lb = la + 1, nb = na + 1;
  // the interior: from the tape, or recomputed from the block input and the forward's statistics
  const void* Si = S;
  const void* Ci = C;
  const void* S2i = S2;
  if (c.p.keep_rb) {
    Si = rb_interior(c, la, 0);
    Ci = rb_interior(c, la, 1);
    S2i = rb_interior(c, la, 2);
  } else {
    TOK_TRY(gn_act(c, na, X, S));
    TOK_TRY(fwd(c, la, S, IN_ACT, d.T, d.H, d.W, C, OUT_ACT, d.T, d.H, d.W, nullptr, false));
    TOK_TRY(gn_act(c, nb, C, S2));
  }
  // conv_b
  TOK_TRY(wgrad(c, lb, CM_S1, S2i, d.T, d.H, d.W, GB, d.T, d.H, d.W, dweights));
  TOK_TRY(adj(c, lb, GB, d.T, d.H, d.W, GA, OUT_ACT));
  // GroupNorm_b + SiLU (in place on GA)
  TOK_TRY(gn_bwd(c, nb, Ci, GA, nullptr, GA, dweights));
  // conv_a
  TOK_TRY(wgrad(c, la, CM_S1, Si, d.T, d.H, d.W, GA, d.T, d.H, d.W, dweights));
  TOK_TRY(adj(c, la, GA, d.T, d.H, d.W, C, OUT_ACT));
  // GroupNorm_a + SiLU, plus the skip path
  return gn_bwd(c, na, X, C, GB, GB, dweights);
}

bool check_ws(const tok_model* m, int N, int T, int H, int W, size_t ws_bytes, TrainPlan* p, tok_status* st) {
  if (m->prec == P_FP8) {
    *st = fail(TOK_EUNSUPPORTED, "training needs an f32 or bf16 model");
    return false;
  }
  Dims d;
  if (!make_dims(N, T, H, W, &d)) {
    *st = fail(TOK_ESHAPE, "need N>=1, T%4==1, H%4==0, W%4==0");
    return false;
  }
  // a workspace that holds the residual-block interiors keeps them; a
  // smaller one (at least the checkpointing size) makes the backward recompute them
  *p = make_train_plan(d, m->prec, true);
  if (p->total <= ws_bytes) return true;
  *p = make_train_plan(d, m->prec, false);
  if (p->total > ws_bytes) {
    *st = fail(TOK_EWORKSPACE, "training workspace needs " + std::to_string(p->total) + " bytes");
    return false;
  }
  return true;
}

}  // namespace

extern "C" {

tok_status tok_train_workspace_size(const tok_model* m, int N, int T, int H, int W, size_t* bytes) {
  if (!m || !bytes) return fail(TOK_EINVAL, "null argument");
  if (m->prec == P_FP8) return fail(TOK_EUNSUPPORTED, "training needs an f32 or bf16 model");
  Dims d;
  if (!make_dims(N, T, H, W, &d)) return fail(TOK_ESHAPE, "need N>=1, T%4==1, H%4==0, W%4==0");
  *bytes = make_train_plan(d, m->prec, true).total;
  return TOK_OK;
}

tok_status tok_train_workspace_min_size(const tok_model* m, int N, int T, int H, int W, size_t* bytes) {
  if (!m || !bytes) return fail(TOK_EINVAL, "null argument");
  if (m->prec == P_FP8) return fail(TOK_EUNSUPPORTED, "training needs an f32 or bf16 model");
  Dims d;
  if (!make_dims(N, T, H, W, &d)) return fail(TOK_ESHAPE, "need N>=1, T%4==1, H%4==0, W%4==0");
  *bytes = make_train_plan(d, m->prec, false).total;
  return TOK_OK;
}

tok_status tok_train_forward(tok_model* m, const uint8_t* x, int N, int T, int H, int W, const uint8_t* keep,
                             float* loss, float* xhat, float* z, int32_t* idx, void* ws, size_t ws_bytes,
                             hipStream_t s) {
  if (!m || !x || !loss || !ws) return fail(TOK_EINVAL, "null argument");
  TrainPlan p;
  tok_status st;
  if (!check_ws(m, N, T, H, W, ws_bytes, &p, &st)) return st;
  const TrainCtx c{m, p, static_cast<char*>(ws), s, m->prec == P_BF16 ? 32 : 16};
  const Dims& d = p.d;
  // encoder
  TOK_TRY(fwd(c, L_CONV_IN, x, IN_U8, T, H, W, c.at(p.H0), OUT_ACT, T, H, W, nullptr, true));
  TOK_TRY(rb_forward(c, L_E_RB1_A, N_E_RB1_A, c.at(p.H0), c.at(p.E1), true));
  TOK_TRY(rb_forward(c, L_E_RB2_A, N_E_RB2_A, c.at(p.E1), c.at(p.E2), false));
  TOK_TRY(fwd(c, L_DOWN1, c.at(p.E2), IN_ACT, T, H, W, c.at(p.D1), OUT_ACT, d.T1, d.H1, d.W1, nullptr, false));
  TOK_TRY(fwd(c, L_DOWN2, c.at(p.D1), IN_ACT, d.T1, d.H1, d.W1, c.at(p.D2), OUT_ACT, d.T2, d.H2, d.W2, nullptr,
              false));
  DropArgs da;
  std::memset(&da, 0, sizeof(da));
  if (keep) {
    da.mode = TOK_DROP_EXTERNAL;
    da.ext_keep = keep;
  }
  const FsqConst fc = make_fsq_const();
  {
    Timed tm(m, L_PROJ, s);
    TOK_HIP(launch_proj_fsq(c.at(p.D2), m->prec, N, d.T2, 0, d.T2, d.T2, 0, d.H2, d.W2, 128 / c.CH, m->w1x1[L_PROJ],
                            m->bias[L_PROJ], fc, da, c.at<float>(p.Z), c.at<float>(p.DEC), idx,
                            c.at<uint8_t>(p.KEEP), s));
  }
  // decoder
  {
    Timed tm(m, L_PROJ_IN, s);
    TOK_HIP(launch_proj_in(c.at<float>(p.DEC), N, d.T2, 0, d.T2, d.H2 * d.W2, m->w1x1[L_PROJ_IN], m->bias[L_PROJ_IN],
                           m->prec, c.at(p.P), 128 / c.CH, d.T2, 0, s));
  }
  TOK_TRY(fwd(c, L_UP2, c.at(p.P), IN_ACT, d.T2, d.H2, d.W2, c.at(p.U2), OUT_ACT, d.T1, d.H1, d.W1, nullptr, false));
  TOK_TRY(fwd(c, L_UP1, c.at(p.U2), IN_ACT, d.T1, d.H1, d.W1, c.at(p.U1), OUT_ACT, T, H, W, nullptr, true));
  TOK_TRY(rb_forward(c, L_D_RB1_A, N_D_RB1_A, c.at(p.U1), c.at(p.R1), true));
  TOK_TRY(rb_forward(c, L_D_RB2_A, N_D_RB2_A, c.at(p.R1), c.at(p.R2), false));
  TOK_TRY(fwd(c, L_CONV_OUT, c.at(p.R2), IN_ACT, T, H, W, c.at(p.XHAT), OUT_RGB32, T, H, W, nullptr, false));
  // loss
  {
    Timed tm(m, K_BWD_MISC, s);
    TOK_HIP(launch_l1(c.at<float>(p.XHAT), x, p.npos, m->prec, nullptr, nullptr, c.at<float>(p.L1P), s));
    TOK_HIP(launch_fsq_bwd(c.at<float>(p.Z), c.at<uint8_t>(p.KEEP), nullptr, p.ntok, fc, 0.f, nullptr, nullptr,
                           c.at<float>(p.CMP), s));
    TOK_HIP(launch_loss_final(c.at<float>(p.L1P), l1_blocks(p.npos), c.at<float>(p.CMP), fsq_blocks(p.ntok),
                              1.0f / (float)(p.npos * 3), 1.0f / (float)(p.ntok * 6), kCommitWeight,
                              c.at<float>(p.LOSS), s));
  }
  TOK_HIP(hipMemcpyAsync(loss, c.at(p.LOSS), 3 * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (xhat) TOK_HIP(hipMemcpyAsync(xhat, c.at(p.XHAT), p.npos * 3 * 4, hipMemcpyDeviceToDevice, s));
  if (z) TOK_HIP(hipMemcpyAsync(z, c.at(p.Z), p.ntok * 6 * 4, hipMemcpyDeviceToDevice, s));
  return TOK_OK;
}

}  // extern "C"

namespace {

// Where the backward pass starts: the library's own objective (scaled by
// gloss), or gradients of the forward's outputs that come from the caller.
struct Seeds {
  bool own_loss;
  const float* gloss;   // own loss: device scalar or null (1)
  const float* gxhat;   // caller: dL/dx_hat (N,T,H,W,3)
  const float* gcodes;  // caller: dL/d(keep * c) (N,T2,H2,W2,6) or null
  const float* gz;      // caller: dL/dz (N,T2,H2,W2,6) or null
};

tok_status backward_impl(tok_model* m, const uint8_t* x, int N, int T, int H, int W, const Seeds& sd,
                         float* dweights, float* dx, void* ws, size_t ws_bytes, hipStream_t s) {
  if (!m || !x || !dweights || !ws) return fail(TOK_EINVAL, "null argument");
  TrainPlan p;
  tok_status st;
  if (!check_ws(m, N, T, H, W, ws_bytes, &p, &st)) return st;
  const TrainCtx c{m, p, static_cast<char*>(ws), s, m->prec == P_BF16 ? 32 : 16};
  const Dims& d = p.d;
  const int wide_chunks = 128 / c.CH;
  void* GB = c.at(p.GB);
  void* WIDE = c.at(p.S);  // S and C together: a 128-channel level-0 buffer
  const FsqConst fc = make_fsq_const();
  // seed: dL/dx_hat
  {
    Timed tm(m, K_BWD_MISC, s);
    if (sd.own_loss)
      TOK_HIP(launch_l1(c.at<float>(p.XHAT), x, p.npos, m->prec, sd.gloss, c.at(p.GX), c.at<float>(p.L1P), s));
    else
      TOK_HIP(launch_rgb_to_chunk(sd.gxhat, p.npos, m->prec, c.at(p.GX), s));
  }
  // conv_out, decoder residual blocks
  TOK_TRY(wgrad(c, L_CONV_OUT, CM_S1, c.at(p.R2), T, H, W, c.at(p.GX), T, H, W, dweights));
  TOK_TRY(adj(c, L_CONV_OUT, c.at(p.GX), T, H, W, GB, OUT_ACT));
  TOK_TRY(rb_backward(c, L_D_RB2_A, N_D_RB2_A, c.at(p.R1), dweights));
  TOK_TRY(rb_backward(c, L_D_RB1_A, N_D_RB1_A, c.at(p.U1), dweights));
  // up1: conv on the upsampled level-1 activations
  TOK_TRY(wgrad(c, L_UP1, CM_UP, c.at(p.U2), d.T1, d.H1, d.W1, GB, T, H, W, dweights));
  if (adj_mode(L_UP1, m->prec) == CM_UPT) {
    TOK_TRY(adj_up(c, L_UP1, GB, T, H, W, c.at(p.G1a)));
  } else {
    TOK_TRY(adj(c, L_UP1, GB, T, H, W, WIDE, OUT_ACT));
    Timed tm(m, K_BWD_MISC, s);
    TOK_HIP(launch_up_adjoint(WIDE, c.at(p.G1a), N, d.T1, d.H1, d.W1, wide_chunks, m->prec, s));
  }
  // up2
  TOK_TRY(wgrad(c, L_UP2, CM_UP, c.at(p.P), d.T2, d.H2, d.W2, c.at(p.G1a), d.T1, d.H1, d.W1, dweights));
  if (adj_mode(L_UP2, m->prec) == CM_UPT) {
    TOK_TRY(adj_up(c, L_UP2, c.at(p.G1a), d.T1, d.H1, d.W1, c.at(p.G2a)));
  } else {
    TOK_TRY(adj(c, L_UP2, c.at(p.G1a), d.T1, d.H1, d.W1, c.at(p.G1b), OUT_ACT));
    Timed tm(m, K_BWD_MISC, s);
    TOK_HIP(launch_up_adjoint(c.at(p.G1b), c.at(p.G2a), N, d.T2, d.H2, d.W2, wide_chunks, m->prec, s));
  }
  {
    Timed tm(m, K_BWD_MISC, s);
    // proj_in (6 -> 128), FSQ straight-through + commitment, proj (128 -> 6)
    const int HW2 = d.H2 * d.W2;
    TOK_HIP(launch_outer6(c.at<float>(p.DEC), c.at(p.G2a), p.ntok, HW2, m->prec, c.at<float>(p.O6P), 1,
                          dweights + m->w_off[L_PROJ_IN], dweights + m->b_off[L_PROJ_IN], s));
    TOK_HIP(launch_proj6(c.at(p.G2a), p.ntok, HW2, m->w1x1T[L_PROJ_IN], c.at<float>(p.GDEC), m->prec, s));
    if (sd.own_loss)
      TOK_HIP(launch_fsq_bwd(c.at<float>(p.Z), c.at<uint8_t>(p.KEEP), c.at<float>(p.GDEC), p.ntok, fc,
                             2.0f * kCommitWeight / (float)(p.ntok * 6), sd.gloss, c.at<float>(p.GZ),
                             c.at<float>(p.CMP), s));
    else
      TOK_HIP(launch_fsq_ste(c.at<float>(p.Z), c.at<uint8_t>(p.KEEP), c.at<float>(p.GDEC), sd.gcodes, sd.gz, p.ntok,
                             fc, c.at<float>(p.GZ), s));
    TOK_HIP(launch_outer6(c.at<float>(p.GZ), c.at(p.D2), p.ntok, HW2, m->prec, c.at<float>(p.O6P), 0,
                          dweights + m->w_off[L_PROJ], dweights + m->b_off[L_PROJ], s));
    TOK_HIP(launch_proj_in(c.at<float>(p.GZ), N, d.T2, 0, d.T2, HW2, m->w1x1T[L_PROJ], m->zeros, m->prec,
                           c.at(p.G2b), 128 / c.CH, d.T2, 0, s));
  }
  // down2: stride-2 conv = stride-1 conv then subsampling
  TOK_TRY(wgrad(c, L_DOWN2, CM_S2, c.at(p.D1), d.T1, d.H1, d.W1, c.at(p.G2b), d.T2, d.H2, d.W2, dweights));
  TOK_TRY(adj_s2(c, L_DOWN2, c.at(p.G2b), d.T2, d.H2, d.W2, c.at(p.G1b)));
  // down1
  TOK_TRY(wgrad(c, L_DOWN1, CM_S2, c.at(p.E2), T, H, W, c.at(p.G1b), d.T1, d.H1, d.W1, dweights));
  TOK_TRY(adj_s2(c, L_DOWN1, c.at(p.G1b), d.T1, d.H1, d.W1, GB));
  // encoder residual blocks, conv_in
  TOK_TRY(rb_backward(c, L_E_RB2_A, N_E_RB2_A, c.at(p.E1), dweights));
  TOK_TRY(rb_backward(c, L_E_RB1_A, N_E_RB1_A, c.at(p.H0), dweights));
  {
    Timed tm(m, K_BWD_MISC, s);
    TOK_HIP(launch_u8_to_chunked(x, p.npos, m->prec, c.at(p.GX), s));
  }
  TOK_TRY(wgrad(c, L_CONV_IN, CM_S1, c.at(p.GX), T, H, W, GB, T, H, W, dweights));
  if (dx) TOK_TRY(adj(c, L_CONV_IN, GB, T, H, W, dx, OUT_RGB32));
  return TOK_OK;
}

}  // namespace

extern "C" {

tok_status tok_backward(tok_model* m, const uint8_t* x, int N, int T, int H, int W, const float* gloss,
                        float* dweights, float* dx, void* ws, size_t ws_bytes, hipStream_t s) {
  const Seeds sd{true, gloss, nullptr, nullptr, nullptr};
  return backward_impl(m, x, N, T, H, W, sd, dweights, dx, ws, ws_bytes, s);
}

tok_status tok_backward_outputs(tok_model* m, const uint8_t* x, int N, int T, int H, int W, const float* gxhat,
                                const float* gcodes, const float* gz, float* dweights, float* dx, void* ws,
                                size_t ws_bytes, hipStream_t s) {
  if (!gxhat) return fail(TOK_EINVAL, "null gxhat");
  const Seeds sd{false, nullptr, gxhat, gcodes, gz};
  return backward_impl(m, x, N, T, H, W, sd, dweights, dx, ws, ws_bytes, s);
}

tok_status tok_train_codes(tok_model* m, int N, int T, int H, int W, float* codes, const void* ws, size_t ws_bytes,
                           hipStream_t s) {
  if (!m || !codes || !ws) return fail(TOK_EINVAL, "null argument");
  TrainPlan p;
  tok_status st;
  if (!check_ws(m, N, T, H, W, ws_bytes, &p, &st)) return st;
  TOK_HIP(hipMemcpyAsync(codes, static_cast<const char*>(ws) + p.DEC, p.ntok * 6 * 4, hipMemcpyDeviceToDevice, s));
  return TOK_OK;
}

namespace {
bool wgrad_op_shape(int view, int N, int Ti, int Hi, int Wi, int To, int Ho, int Wo) {
  if (N < 1 || Ti < 1 || Hi < 1 || Wi < 1) return false;
  if (view == CM_S1) return To == Ti && Ho == Hi && Wo == Wi;
  if (view == CM_S2) return Ti % 2 == 1 && Hi % 2 == 0 && Wi % 2 == 0 && To == (Ti - 1) / 2 + 1 && Ho == Hi / 2 &&
                            Wo == Wi / 2;
  if (view == CM_UP) return To == 2 * Ti - 1 && Ho == 2 * Hi && Wo == 2 * Wi;
  return false;
}
int view_mode(int view) { return view == 0 ? CM_S1 : (view == 1 ? CM_S2 : (view == 2 ? CM_UP : -1)); }
size_t wgrad_op_bytes(int P, int mode, int N, int To, int Ho, int Wo, int Cin, int Cout, int* splits) {
  *splits = wgrad_splits(P, mode, Cout, Cin, N, To, Ho, Wo);
  return align256((size_t)*splits * wgrad_partial_taps(P, mode) * Cout * Cin * 4) +
         align256((size_t)*splits * wgrad_bias_parts(P, mode) * Cout * 4);
}
}  // namespace

tok_status tok_conv3d_wgrad_workspace_size(tok_precision prec, int view, int N, int To, int Ho, int Wo, int Cin,
                                           int Cout, size_t* bytes) {
  if (!bytes || (prec != TOK_F32 && prec != TOK_BF16) || view_mode(view) < 0 || Cin < 1 || Cout < 1)
    return fail(TOK_EINVAL, "bad argument");
  int sp;
  *bytes = wgrad_op_bytes(prec == TOK_BF16 ? P_BF16 : P_F32, view_mode(view), N, To, Ho, Wo, Cin, Cout, &sp);
  return TOK_OK;
}

tok_status tok_conv3d_wgrad(tok_precision prec, int view, const void* x, int N, int Ti, int Hi, int Wi, int Cin,
                            const void* dy, int To, int Ho, int Wo, int Cout, float* dw, float* db, void* ws,
                            size_t ws_bytes, hipStream_t s) {
  if (!x || !dy || !dw || !ws || (prec != TOK_F32 && prec != TOK_BF16) || view_mode(view) < 0 || Cin < 1 ||
      Cout < 1)
    return fail(TOK_EINVAL, "bad argument");
  const int mode = view_mode(view);
  if (!wgrad_op_shape(mode, N, Ti, Hi, Wi, To, Ho, Wo)) return fail(TOK_ESHAPE, "input / output shapes do not match the view");
  const int P = prec == TOK_BF16 ? P_BF16 : P_F32, CH = P == P_BF16 ? 32 : 16;
  int sp;
  const size_t need = wgrad_op_bytes(P, mode, N, To, Ho, Wo, Cin, Cout, &sp);
  if (need > ws_bytes) return fail(TOK_EWORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
  WgradLaunch a;
  std::memset(&a, 0, sizeof(a));
  a.x = x; a.N = N; a.Ti = Ti; a.Hi = Hi; a.Wi = Wi; a.x_chunks = cdiv(Cin, CH);
  a.dy = dy; a.To = To; a.Ho = Ho; a.Wo = Wo; a.dy_chunks = cdiv(Cout, CH);
  a.Cout = Cout; a.Cin = Cin; a.view = mode; a.prec = P; a.splits = sp;
  a.partial = static_cast<float*>(ws);
  a.bpartial = reinterpret_cast<float*>(static_cast<char*>(ws) +
                                       align256((size_t)sp * wgrad_partial_taps(P, mode) * Cout * Cin * 4));
  TOK_HIP(launch_wgrad(a, s));
  TOK_HIP(launch_wgrad_reduce(a, dw, db, s));
  return TOK_OK;
}

}  // extern "C"
