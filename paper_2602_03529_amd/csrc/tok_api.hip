// C ABI of libtok.so: model packing, workspace planning and the launch
// sequences of encode / decode (see include/tok.h for the contract).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "tok.h"
#include "tok_model.h"

using namespace tok;

namespace {
thread_local std::string g_err;
}  // namespace

tok_status tok::fail(tok_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

FsqConst tok::make_fsq_const() {
  const int levels[6] = {8, 8, 8, 5, 5, 5};
  FsqConst f;
  int basis = 1;
  for (int c = 0; c < 6; ++c) {
    const double L = levels[c];
    const double h = (L - 1.0) * (1.0 - 1e-3) / 2.0;
    const double o = (levels[c] % 2 == 0) ? 0.5 : 0.0;
    const double d = std::floor(L / 2.0);
    f.h[c] = (float)h;
    f.o[c] = (float)o;
    f.s[c] = (float)std::atanh(o / h);
    f.d[c] = (float)d;
    f.inv_d[c] = (float)(1.0 / d);
    f.basis[c] = basis;
    basis *= levels[c];
  }
  return f;
}

namespace {

struct BlobItem { int is_conv; int id; };  // conv layer or norm
// module order: conv_in, rb1(gn_a, a, gn_b, b), rb2, down1, down2, proj, proj_in, up2, up1, rb1, rb2, conv_out
const BlobItem kOrder[] = {
    {1, L_CONV_IN},
    {0, N_E_RB1_A}, {1, L_E_RB1_A}, {0, N_E_RB1_B}, {1, L_E_RB1_B},
    {0, N_E_RB2_A}, {1, L_E_RB2_A}, {0, N_E_RB2_B}, {1, L_E_RB2_B},
    {1, L_DOWN1}, {1, L_DOWN2}, {1, L_PROJ}, {1, L_PROJ_IN}, {1, L_UP2}, {1, L_UP1},
    {0, N_D_RB1_A}, {1, L_D_RB1_A}, {0, N_D_RB1_B}, {1, L_D_RB1_B},
    {0, N_D_RB2_A}, {1, L_D_RB2_A}, {0, N_D_RB2_B}, {1, L_D_RB2_B},
    {1, L_CONV_OUT}};

size_t blob_count() {
  size_t n = 0;
  for (const auto& it : kOrder) {
    if (it.is_conv) {
      const ConvSpec& c = kConv[it.id];
      n += (size_t)c.cout * c.cin * c.k * c.k * c.k + c.cout;
    } else {
      n += 2 * 64;
    }
  }
  return n;
}

}  // namespace

namespace {

// Workspace plan for processing a clip in causal temporal chunks of CL latent
// frames (CL = T2: the whole clip at once).  Chunk [L0, L1) of latent frames
// covers level-0 frames [max(4 L0 - 3, 0), 4 L1 - 4], level-1 frames
// [max(2 L0 - 1, 0), 2 L1 - 2] and latent frames [L0, L1 - 1].  Every layer's
// input buffer keeps the last frames of the previous chunk in front of the
// current ones (2 for a stride-1 conv, 1 for a stride-2 or upsampling conv),
// which is all a causal k=3 layer reads from the past, so chunked and
// whole-clip processing compute the same values.
constexpr int kCache0 = 2, kCache1 = 1, kCache2 = 1;

struct Plan {
  int CL, F0max, F1max, Tb0, Tb1, Tb2;
  size_t l0, l0c, cache, l1, l2, stats, scsh;
  size_t off_l0a, off_l0b, off_l0c, off_cache, off_l1, off_l2, off_stats, off_sc, off_sh, total;
};

// The four residual-block convs of one level-0 stack share the scratch
// buffers B (conv input, with cache frames) and C (first conv output); when
// chunking, each conv's input cache is saved after it runs and restored before
// it runs in the next chunk, from its own slot of 2 frames per clip.
constexpr int kRbCaches = 4;

Plan make_plan(const Dims& d, int prec, int CL) {
  const size_t es = prec == P_BF16 ? 2 : 4;
  Plan p;
  p.CL = CL;
  p.F0max = CL >= d.T2 ? d.T : 4 * CL;
  p.F1max = CL >= d.T2 ? d.T1 : 2 * CL;
  p.Tb0 = kCache0 + p.F0max;
  p.Tb1 = kCache1 + p.F1max;
  p.Tb2 = kCache2 + CL;
  p.l0 = align256((size_t)d.N * p.Tb0 * d.H * d.W * 64 * es);
  p.l0c = align256((size_t)d.N * p.F0max * d.H * d.W * 64 * es);
  p.cache = CL >= d.T2 ? 0 : align256((size_t)kRbCaches * d.N * kCache0 * d.H * d.W * 64 * es);
  p.l1 = align256((size_t)d.N * p.Tb1 * d.H1 * d.W1 * 128 * es);
  p.l2 = align256((size_t)d.N * p.Tb2 * d.H2 * d.W2 * 128 * es);
  const size_t tiles0 = (size_t)cdiv(d.H, 8) * cdiv(d.W, 64);
  p.stats = align256((size_t)d.N * p.F0max * tiles0 * 32 * sizeof(float4));
  p.scsh = align256((size_t)d.N * p.F0max * 64 * sizeof(float));
  size_t o = 0;
  p.off_l0a = o; o += p.l0;
  p.off_l0b = o; o += p.l0;
  p.off_l0c = o; o += p.l0c;
  p.off_cache = o; o += p.cache;
  p.off_l1 = o; o += p.l1;
  p.off_l2 = o; o += p.l2;
  p.off_stats = o; o += p.stats;
  p.off_sc = o; o += p.scsh;
  p.off_sh = o; o += p.scsh;
  p.total = o;
  return p;
}

// Largest chunk size whose plan fits ws_bytes: the whole clip, else one
// latent frame per chunk; 0 if neither fits.
int choose_chunk(const Dims& d, int prec, size_t ws_bytes, Plan* out) {
  Plan p = make_plan(d, prec, d.T2);
  if (p.total <= ws_bytes) { *out = p; return d.T2; }
  p = make_plan(d, prec, 1);
  if (p.total <= ws_bytes) { *out = p; return 1; }
  *out = p;
  return 0;
}

struct Ws {
  char* base;
  Plan p;
  void* l0a() const { return base + p.off_l0a; }
  void* l0b() const { return base + p.off_l0b; }
  void* l0c() const { return base + p.off_l0c; }
  char* cache(int k) const { return base + p.off_cache + (size_t)k * (p.cache / kRbCaches); }
  void* l1() const { return base + p.off_l1; }
  void* l2() const { return base + p.off_l2; }
  float4* stats() const { return reinterpret_cast<float4*>(base + p.off_stats); }
  float* sc() const { return reinterpret_cast<float*>(base + p.off_sc); }
  float* sh() const { return reinterpret_cast<float*>(base + p.off_sh); }
};

// A window of frames in a buffer: Tb frames per clip, buffer frame 0 is
// global frame g0, the current chunk occupies [first, first + count).
struct Win {
  int Tb, g0, first, count;
};

// GoP-boundary blending fused into C_out's epilogue (tok_decode_blend).
struct Blend {
  const float* prev;
  int Tp, n;
};

// Pixel-residual sums accumulated by C_out as it writes each frame
// (tok_decode_residual): source clip x (T frames) and the (N, H, W, 3) sums.
struct ResAcc {
  const uint8_t* x;
  float* sum;
  int T;
};

const char* kKernelNames[K_IDS] = {
    "enc.conv_in", "enc.rb1.a", "enc.rb1.b", "enc.rb2.a", "enc.rb2.b", "enc.down1", "enc.down2",
    "enc.proj+fsq+drop", "dec.proj_in", "dec.up2", "dec.up1", "dec.rb1.a", "dec.rb1.b", "dec.rb2.a",
    "dec.rb2.b", "dec.conv_out", "gn_finalize", "gn_silu", "bwd.dgrad", "bwd.wgrad", "bwd.gn_silu",
    "bwd.other", "select.similarity", "dec.residual"};

// Conv launch: reads the whole input buffer `iw` (its frames are addressed
// through their global numbers) and writes the window `ow` of the output.
tok_status conv(const tok_model* m, int layer, int mode, const void* in, int in_kind, int N, const Win& iw, int Hi,
                int Wi, int Cin, void* out, int out_kind, const Win& ow, int Ho, int Wo, const void* resid,
                float4* stats, hipStream_t s, const uint8_t* in_scale = nullptr, uint8_t* out_scale = nullptr,
                const Blend* blend = nullptr, const ResAcc* racc = nullptr) {
  ConvLaunch a;
  std::memset(&a, 0, sizeof(a));
  if (blend) {
    a.blend_prev = blend->prev;
    a.blend_Tp = blend->Tp;
    a.blend_n = blend->n;
  }
  if (racc) {
    a.rs_x = racc->x;
    a.rs_sum = racc->sum;
    a.rs_T = racc->T;
  }
  const int CH = m->prec == P_BF16 ? 32 : (m->prec == P_FP8 ? 64 : 16);  // input chunking
  const int CHo = out_kind == OUT_FP8 ? 64 : (m->prec == P_F32 ? 16 : 32);
  a.in = in;
  a.N = N; a.Ti = iw.Tb; a.Hi = Hi; a.Wi = Wi;
  a.gi0 = iw.g0;
  a.in_chunks = mode == CM_I2C ? kI2cK / CH : cdiv(Cin, CH);
  a.Cin = Cin;
  a.wpk = m->wpk[layer];
  a.bias = m->bias[layer];
  a.Cout = kConv[layer].cout;
  a.nt = m->nt[layer];
  a.cout_tiles = cdiv(a.Cout, a.nt);
  a.out = out;
  a.resid = resid;
  a.To = ow.count; a.Ho = Ho; a.Wo = Wo;
  a.To_buf = ow.Tb; a.out_f0 = ow.first; a.go0 = ow.g0 + ow.first;
  a.out_chunks = cdiv(a.Cout, CHo);
  a.stats = stats;
  a.in_scale = in_scale;
  a.out_scale = out_scale;
  a.wscale = m->wscale[layer];
  int th, tw;
  conv_tile(mode, &th, &tw);
  a.tiles_h = cdiv(Ho, th);
  a.tiles_w = cdiv(Wo, tw);
  a.mode = mode; a.in_kind = in_kind; a.out_kind = out_kind; a.prec = m->prec;
  Timed tm(m, layer, s);
  const hipError_t e = launch_conv(a, s);
  if (e != hipSuccess) return fail(TOK_EDEVICE, std::string("conv layer ") + std::to_string(layer) + ": " + hipGetErrorString(e));
  return TOK_OK;
}

// GroupNorm `norm` + SiLU of the chunk frames of level-0 buffer `in` (whose
// per-tile statistics the producing conv left in the stats buffer) into the
// same frames of `out`.
tok_status gn_silu(const tok_model* m, int norm, const Ws& w, int N, const void* in, const Win& iw, void* out,
                   const Win& ow, int Ho, int Wo, hipStream_t s) {
  const int tiles = cdiv(Ho, 8) * cdiv(Wo, 64);
  {
    Timed tm(m, K_GN_FINAL, s);
    const hipError_t e = launch_gn_finalize(w.stats(), N * iw.count, tiles, m->gamma[norm], m->beta[norm], kGnEps,
                                            w.sc(), w.sh(), nullptr, s);
    if (e != hipSuccess) return fail(TOK_EDEVICE, std::string("gn_finalize: ") + hipGetErrorString(e));
  }
  Timed tm(m, K_GN_ACT, s);
  const hipError_t e = launch_gn_act(in, iw.Tb, iw.first, out, ow.Tb, ow.first, m->prec, N, iw.count, Ho * Wo,
                                     w.sc(), w.sh(), s);
  if (e != hipSuccess) return fail(TOK_EDEVICE, std::string("gn_act: ") + hipGetErrorString(e));
  return TOK_OK;
}


// Copy `frames` frames per clip between a buffer window position and a cache
// slot (dir > 0: buffer -> cache, else cache -> buffer).
tok_status cache_copy(char* buf, int Tb, int first, char* cache, int frames, int N, size_t frame_bytes, int dir,
                      hipStream_t s) {
  for (int n = 0; n < N; ++n) {
    char* b = buf + ((size_t)n * Tb + first) * frame_bytes;
    char* c = cache + (size_t)n * frames * frame_bytes;
    TOK_HIP(hipMemcpyAsync(dir > 0 ? c : b, dir > 0 ? b : c, (size_t)frames * frame_bytes, hipMemcpyDeviceToDevice,
                           s));
  }
  return TOK_OK;
}

// Two residual blocks at level 0 on the chunk window `win`, in place on
// buffer A; B holds each conv's input (cache frames in front of the chunk),
// C the first conv's output (chunk frames only).  Entry: A holds the block
// input and the stats buffer its GroupNorm partials.
//   B = silu(gn_a(A)); C = conv_a(B) (+stats); B = silu(gn_b(C)); A = A + conv_b(B) (+stats)
// `chunked`: restore / save each conv's input cache around it.
tok_status resblocks(const tok_model* m, int first_layer, int first_norm, const Ws& w, const Dims& d,
                     const Win& win, bool last_stats, bool chunked, int chunk_index, hipStream_t s) {
  const int N = d.N, H = d.H, W = d.W;
  const size_t fb = (size_t)H * W * 64 * (m->prec == P_BF16 ? 2 : 4);
  const Win cw{w.p.F0max, win.g0 + win.first, 0, win.count};  // C: chunk frames only
  char* B = static_cast<char*>(w.l0b());
  auto restore = [&](int k) -> tok_status {
    if (!chunked || chunk_index == 0) return TOK_OK;
    return cache_copy(B, win.Tb, win.first - kCache0, w.cache(k), kCache0, N, fb, -1, s);
  };
  auto save = [&](int k) -> tok_status {
    if (!chunked) return TOK_OK;
    return cache_copy(B, win.Tb, win.first + win.count - kCache0, w.cache(k), kCache0, N, fb, +1, s);
  };
  for (int r = 0; r < 2; ++r) {
    const int la = first_layer + 2 * r, lb = la + 1;
    const int na = first_norm + 2 * r, nb = na + 1;
    TOK_TRY(gn_silu(m, na, w, N, w.l0a(), win, w.l0b(), win, H, W, s));
    TOK_TRY(restore(2 * r));
    TOK_TRY(conv(m, la, CM_S1, w.l0b(), IN_ACT, N, win, H, W, 64, w.l0c(), OUT_ACT, cw, H, W, nullptr, w.stats(), s));
    TOK_TRY(save(2 * r));
    TOK_TRY(gn_silu(m, nb, w, N, w.l0c(), cw, w.l0b(), win, H, W, s));
    TOK_TRY(restore(2 * r + 1));
    const bool stats = (r == 0) || last_stats;
    TOK_TRY(conv(m, lb, CM_S1, w.l0b(), IN_ACT, N, win, H, W, 64, w.l0a(), OUT_ACT, win, H, W, w.l0a(),
                 stats ? w.stats() : nullptr, s));
    TOK_TRY(save(2 * r + 1));
  }
  return TOK_OK;
}

// Move the last `cache` frames of the chunk window to the front of the buffer
// (frames first + count - cache .. first + count - 1 -> first - cache ..),
// ready for the next chunk.  Frame by frame in increasing order, which is safe
// for overlapping ranges because the destination precedes the source.
tok_status shift_cache(void* buf, const Win& win, int N, size_t frame_bytes, int cache, hipStream_t s) {
  char* b = static_cast<char*>(buf);
  for (int n = 0; n < N; ++n)
    for (int j = 0; j < cache; ++j) {
      const int src = win.first + win.count - cache + j, dst = win.first - cache + j;
      if (src == dst) continue;
      char* clip = b + (size_t)n * win.Tb * frame_bytes;
      TOK_HIP(hipMemcpyAsync(clip + (size_t)dst * frame_bytes, clip + (size_t)src * frame_bytes, frame_bytes,
                             hipMemcpyDeviceToDevice, s));
    }
  return TOK_OK;
}

struct ChunkWins {
  Win l0, l1, l2;  // level-0, level-1, level-2 windows of chunk [L0, L1)
};

ChunkWins chunk_windows(const Plan& p, int L0, int L1) {
  const int a0 = std::max(4 * L0 - 3, 0), b0 = 4 * L1 - 4;
  const int a1 = std::max(2 * L0 - 1, 0), b1 = 2 * L1 - 2;
  ChunkWins c;
  c.l0 = Win{p.Tb0, a0 - kCache0, kCache0, b0 - a0 + 1};
  c.l1 = Win{p.Tb1, a1 - kCache1, kCache1, b1 - a1 + 1};
  c.l2 = Win{p.Tb2, L0 - kCache2, kCache2, L1 - L0};
  return c;
}

bool valid_drop(const tok_drop_desc* dd) {
  return !dd || (dd->mode >= 0 && dd->mode <= TOK_DROP_SIMILARITY && (dd->mode != TOK_DROP_EXTERNAL || dd->ext_keep));
}

bool is_similarity(const tok_drop_desc* dd) { return dd && dd->mode == TOK_DROP_SIMILARITY; }

// Drop count of the similarity selection: min(ceil(rate * n_p), n_p), rate
// clamped to [0, 1] (NaN counts as 0), evaluated in double.
long long similarity_drop_count(float rate, long long n_p) {
  double r = rate;
  if (!(r >= 0.0)) r = 0.0;
  if (r > 1.0) r = 1.0;
  const long long d = (long long)std::ceil(r * (double)n_p);
  return d < n_p ? d : n_p;
}

DropArgs make_drop(const tok_drop_desc* dd) {
  DropArgs a;
  std::memset(&a, 0, sizeof(a));
  if (!dd || dd->mode == TOK_DROP_SIMILARITY) return a;  // selected after FSQ, not per token
  a.mode = dd->mode;
  double r = dd->rate;
  if (!(r >= 0.0)) r = 0.0;
  if (r > 1.0) r = 1.0;
  a.thr = (uint32_t)std::floor(r * 16777216.0);
  a.seed = dd->seed;
  a.clip_id0 = dd->clip_id0;
  a.protect_iframe = dd->protect_iframe;
  a.ext_keep = dd->ext_keep;
  return a;
}

}  // namespace

namespace {

// Layout of the model's device allocation (bytes), computed from the layer table.
// An fp8 model holds the decoder only (packed e4m3 kernels with per-channel
// scales) and no adjoint kernels; f32 / bf16 models hold everything.
struct ModelLayout {
  size_t blob, wpk[L_COUNT], wpkT[L_COUNT], wsc[L_COUNT], w1T[L_COUNT], zeros, total;
  int nt[L_COUNT], ntT[L_COUNT];
  bool has[L_COUNT], hasT;
};

ModelLayout model_layout(int P) {
  const size_t es = P == P_BF16 ? 2 : (P == P_FP8 ? 1 : 4);
  ModelLayout L;
  std::memset(&L, 0, sizeof(L));
  L.hasT = P != P_FP8;
  size_t off = 0;
  L.blob = off;
  off = align256(off + blob_count() * 4);
  for (int l = 0; l < L_COUNT; ++l) {
    const ConvSpec& c = kConv[l];
    L.has[l] = P != P_FP8 || is_decoder_layer(l);
    if (c.k == 3) {
      if (L.has[l]) {
        L.wpk[l] = off;
        off = align256(off + packed_conv_elems(c.cout, c.cin, P, conv_mode(l), &L.nt[l]) * es);
      }
      if (P == P_FP8 && L.has[l]) {
        L.wsc[l] = off;
        off = align256(off + (size_t)c.cout * 4);
      }
      if (L.hasT) {
        L.wpkT[l] = off;
        off = align256(off + packed_conv_elems(c.cout, c.cin, P, adj_mode(l, P), &L.ntT[l]) * es);
      }
    } else {
      L.w1T[l] = off;
      off = align256(off + (size_t)c.cout * c.cin * 4);
    }
  }
  L.zeros = off;
  off = align256(off + 128 * 4);
  L.total = off;
  return L;
}

// Packs every kernel of the model from its blob (stream-ordered).
tok_status repack(tok_model* m, hipStream_t s) {
  for (int l = 0; l < L_COUNT; ++l) {
    const ConvSpec& c = kConv[l];
    const float* w = m->blob + m->w_off[l];
    if (c.k == 3) {
      if (m->wpk[l]) TOK_HIP(launch_pack_weights(w, c.cout, c.cin, m->prec, conv_mode(l), m->wpk[l], m->wscale[l], s));
      if (m->wpkT[l]) TOK_HIP(launch_pack_weights(w, c.cout, c.cin, m->prec, adj_mode(l, m->prec), m->wpkT[l], nullptr, s));
    } else {
      TOK_HIP(launch_transpose(w, c.cout, c.cin, m->w1x1T[l], s));
    }
  }
  return TOK_OK;
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// fp8 decoder (whole clips).  MX-FP8 activations feed every conv; the
// residual stream and the GroupNorm inputs stay bf16:
//   P  = proj_in(codes)                      MX-FP8, level 2
//   U2 = up2(P)                              MX-FP8, level 1
//   A  = up1(U2)                             bf16 (+ GN partials), level 0
//   RB: S = silu(gn_a A) (MX-FP8); C = conv_a(S) (bf16 + GN partials);
//       S = silu(gn_b C); A = A + conv_b(S)  (bf16, + GN partials)
//   last RB: R2 = A + conv_b(S) written as MX-FP8 (into C's space)
//   x_hat = conv_out(R2)
// ---------------------------------------------------------------------------
struct Fp8Plan {
  size_t P, Psc, U2, U2sc, A, S, Ssc, C, Csc, stats, sc, sh, total;
};

Fp8Plan make_fp8_plan(const Dims& d) {
  Fp8Plan p;
  const size_t n0 = (size_t)d.N * d.T * d.H * d.W, n1 = (size_t)d.N * d.T1 * d.H1 * d.W1;
  const size_t n2 = (size_t)d.N * d.T2 * d.H2 * d.W2;
  size_t o = 0;
  auto take = [&](size_t b) { const size_t r = o; o += align256(b); return r; };
  p.P = take(n2 * 128); p.Psc = take(n2 * 4);
  p.U2 = take(n1 * 128); p.U2sc = take(n1 * 4);
  p.A = take(n0 * 128);
  p.S = take(n0 * 64); p.Ssc = take(n0 * 2);
  p.C = take(n0 * 128); p.Csc = take(n0 * 2);
  p.stats = take((size_t)d.N * d.T * cdiv(d.H, 8) * cdiv(d.W, 64) * 32 * sizeof(float4));
  p.sc = take((size_t)d.N * d.T * 64 * 4); p.sh = take((size_t)d.N * d.T * 64 * 4);
  p.total = o;
  return p;
}

tok_status decode_fp8(tok_model* m, const float* codes, const Dims& d, float* xhat, void* ws, size_t ws_bytes,
                      hipStream_t s, const Blend* blend) {
  const Fp8Plan p = make_fp8_plan(d);
  if (p.total > ws_bytes)
    return fail(TOK_EWORKSPACE, "fp8 decode workspace needs " + std::to_string(p.total) + " bytes");
  char* b = static_cast<char*>(ws);
  auto at = [&](size_t off) { return b + off; };
  auto u8 = [&](size_t off) { return reinterpret_cast<uint8_t*>(b + off); };
  float4* stats = reinterpret_cast<float4*>(at(p.stats));
  float* sc = reinterpret_cast<float*>(at(p.sc));
  float* sh = reinterpret_cast<float*>(at(p.sh));
  const int N = d.N, T = d.T, H = d.H, W = d.W;
  const Win w0{T, 0, 0, T}, w1{d.T1, 0, 0, d.T1}, w2{d.T2, 0, 0, d.T2};
  {
    Timed tm(m, L_PROJ_IN, s);
    TOK_HIP(launch_proj_in_fp8(codes, N, d.T2, 0, d.T2, d.H2 * d.W2, m->w1x1[L_PROJ_IN], m->bias[L_PROJ_IN],
                               u8(p.P), u8(p.Psc), d.T2, 0, s));
  }
  TOK_TRY(conv(m, L_UP2, CM_UPF, at(p.P), IN_ACT, N, w2, d.H2, d.W2, 128, at(p.U2), OUT_FP8, w1, d.H1, d.W1, nullptr,
               nullptr, s, u8(p.Psc), u8(p.U2sc)));
  TOK_TRY(conv(m, L_UP1, CM_UPF, at(p.U2), IN_ACT, N, w1, d.H1, d.W1, 128, at(p.A), OUT_ACT, w0, H, W, nullptr, stats,
               s, u8(p.U2sc)));
  const int tiles = cdiv(H, 8) * cdiv(W, 64);
  auto gn = [&](int norm, const void* in) -> tok_status {
    {
      Timed tm(m, K_GN_FINAL, s);
      TOK_HIP(launch_gn_finalize(stats, N * T, tiles, m->gamma[norm], m->beta[norm], kGnEps, sc, sh, nullptr, s));
    }
    Timed tm(m, K_GN_ACT, s);
    TOK_HIP(launch_gn_act_fp8(in, T, 0, u8(p.S), u8(p.Ssc), T, 0, N, T, H * W, sc, sh, s));
    return TOK_OK;
  };
  for (int r = 0; r < 2; ++r) {
    const int la = L_D_RB1_A + 2 * r, na = N_D_RB1_A + 2 * r;
    TOK_TRY(gn(na, at(p.A)));
    TOK_TRY(conv(m, la, CM_S1, at(p.S), IN_ACT, N, w0, H, W, 64, at(p.C), OUT_ACT, w0, H, W, nullptr, stats, s,
                 u8(p.Ssc)));
    TOK_TRY(gn(na + 1, at(p.C)));
    if (r == 0)
      TOK_TRY(conv(m, la + 1, CM_S1, at(p.S), IN_ACT, N, w0, H, W, 64, at(p.A), OUT_ACT, w0, H, W, at(p.A), stats, s,
                   u8(p.Ssc)));
    else
      TOK_TRY(conv(m, la + 1, CM_S1, at(p.S), IN_ACT, N, w0, H, W, 64, at(p.C), OUT_FP8, w0, H, W, at(p.A), nullptr,
                   s, u8(p.Ssc), u8(p.Csc)));
  }
  TOK_TRY(conv(m, L_CONV_OUT, CM_S1, at(p.C), IN_ACT, N, w0, H, W, 64, xhat, OUT_RGB32, w0, H, W, nullptr, nullptr, s,
               u8(p.Csc)));
  // GoP blending as its own pass after the fp8 last layer (the walk with the blend measured slower)
  if (blend) TOK_HIP(launch_blend(blend->prev, blend->Tp, xhat, N, T, H, W, blend->n, s));
  return TOK_OK;
}

}  // namespace

extern "C" {

size_t tok_weight_count(void) { return blob_count(); }

const char* tok_status_str(tok_status s) {
  switch (s) {
    case TOK_OK: return "ok";
    case TOK_EINVAL: return "invalid argument";
    case TOK_ESHAPE: return "invalid shape";
    case TOK_ENOMEM: return "out of device memory";
    case TOK_EDEVICE: return "device error";
    case TOK_EBUDGET: return "over memory budget";
    case TOK_EUNSUPPORTED: return "unsupported";
    case TOK_EWORKSPACE: return "workspace too small";
  }
  return "unknown status";
}

const char* tok_last_error(void) { return g_err.c_str(); }

const char* tok_kernel_name(int k) { return (k >= 0 && k < K_IDS) ? kKernelNames[k] : "unknown"; }

tok_status tok_profile_begin(tok_model* m) {
  if (!m) return fail(TOK_EINVAL, "null model");
  m->profiling = true;
  return TOK_OK;
}

tok_status tok_profile_end(tok_model* m, int n_ids, double* ms, int* count) {
  if (!m) return fail(TOK_EINVAL, "null model");
  m->profiling = false;
  for (int k = 0; k < n_ids; ++k) {
    if (ms) ms[k] = 0.0;
    if (count) count[k] = 0;
  }
  tok_status st = TOK_OK;
  for (auto& r : m->prof) {
    float t = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
      st = fail(TOK_EDEVICE, "event timing failed");
    } else if (r.id >= 0 && r.id < n_ids) {
      if (ms) ms[r.id] += t;
      if (count) count[r.id] += 1;
    }
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  m->prof.clear();
  return st;
}

tok_status tok_model_create(const float* host_weights, size_t n_floats, tok_precision prec, int device,
                            tok_model** out) {
  if (!host_weights || !out) return fail(TOK_EINVAL, "null argument");
  if (n_floats != blob_count()) return fail(TOK_EINVAL, "weight blob has " + std::to_string(n_floats) +
                                                           " floats, expected " + std::to_string(blob_count()));
  if (prec != TOK_F32 && prec != TOK_BF16 && prec != TOK_FP8_E4M3) return fail(TOK_EUNSUPPORTED, "unknown precision");
  const int P = prec == TOK_BF16 ? P_BF16 : (prec == TOK_FP8_E4M3 ? P_FP8 : P_F32);
  const ModelLayout L = model_layout(P);

  tok_model* m = new (std::nothrow) tok_model;
  if (!m) return fail(TOK_ENOMEM, "host allocation failed");
  m->device = device;
  m->prec = P;
  // blob offsets of every tensor, in canonical order
  size_t cur = 0;
  for (const auto& it : kOrder) {
    if (it.is_conv) {
      const ConvSpec& c = kConv[it.id];
      m->w_off[it.id] = cur;
      cur += (size_t)c.cout * c.cin * c.k * c.k * c.k;
      m->b_off[it.id] = cur;
      cur += c.cout;
    } else {
      m->g_off[it.id] = cur; cur += 64;
      m->be_off[it.id] = cur; cur += 64;
    }
  }

  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) {
    delete m;
    return fail(TOK_EDEVICE, "cannot select device " + std::to_string(device));
  }
  tok_status st = TOK_OK;
  if (hipMalloc(&m->mem, L.total) != hipSuccess) {
    m->mem = nullptr;
    st = fail(TOK_ENOMEM, "hipMalloc of model weights failed");
  }
  if (st == TOK_OK) {
    char* base = static_cast<char*>(m->mem);
    m->blob = reinterpret_cast<float*>(base + L.blob);
    for (int l = 0; l < L_COUNT; ++l) {
      if (kConv[l].k == 3) {
        m->wpk[l] = L.has[l] ? base + L.wpk[l] : nullptr;
        m->wpkT[l] = L.hasT ? base + L.wpkT[l] : nullptr;
        m->wscale[l] = P == P_FP8 && L.has[l] ? reinterpret_cast<float*>(base + L.wsc[l]) : nullptr;
        m->nt[l] = L.nt[l];
        m->ntT[l] = L.ntT[l];
      } else {
        m->w1x1[l] = m->blob + m->w_off[l];
        m->w1x1T[l] = reinterpret_cast<float*>(base + L.w1T[l]);
      }
      m->bias[l] = m->blob + m->b_off[l];
    }
    for (int n = 0; n < N_COUNT; ++n) {
      m->gamma[n] = m->blob + m->g_off[n];
      m->beta[n] = m->blob + m->be_off[n];
    }
    m->zeros = reinterpret_cast<const float*>(base + L.zeros);
    hipError_t e = hipMemset(base + L.zeros, 0, 128 * 4);
    if (e == hipSuccess) e = hipMemcpy(m->blob, host_weights, n_floats * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) st = fail(TOK_EDEVICE, std::string("weight upload: ") + hipGetErrorString(e));
    if (st == TOK_OK) st = repack(m, nullptr);
    if (st == TOK_OK) {
      e = hipDeviceSynchronize();
      if (e != hipSuccess) st = fail(TOK_EDEVICE, std::string("weight packing: ") + hipGetErrorString(e));
    }
  }
  if (st != TOK_OK) {
    if (m->mem) hipFree(m->mem);
    delete m;
    hipSetDevice(prev);
    return st;
  }
  hipSetDevice(prev);
  *out = m;
  return TOK_OK;
}

tok_status tok_model_set_weights(tok_model* m, const float* weights, hipStream_t s) {
  if (!m || !weights) return fail(TOK_EINVAL, "null argument");
  TOK_HIP(hipMemcpyAsync(m->blob, weights, blob_count() * 4, hipMemcpyDeviceToDevice, s));
  return repack(m, s);
}

void tok_model_destroy(tok_model* m) {
  if (!m) return;
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(m->device);
  hipFree(m->mem);
  hipSetDevice(prev);
  delete m;
}

tok_status tok_workspace_size(const tok_model* m, int N, int T, int H, int W, int what, size_t* bytes) {
  if (!m || !bytes) return fail(TOK_EINVAL, "null argument");
  const int kind = what & ~TOK_WS_STREAM;
  if (kind < TOK_WS_ENCODE || kind > TOK_WS_ROUNDTRIP) return fail(TOK_EINVAL, "bad workspace kind");
  Dims d;
  if (!make_dims(N, T, H, W, &d)) return fail(TOK_ESHAPE, "need N>=1, T%4==1, H%4==0, W%4==0");
  if (m->prec == P_FP8) {
    if (kind != TOK_WS_DECODE || (what & TOK_WS_STREAM))
      return fail(TOK_EUNSUPPORTED, "fp8 models decode whole clips only");
    *bytes = make_fp8_plan(d).total;
    return TOK_OK;
  }
  *bytes = make_plan(d, m->prec, (what & TOK_WS_STREAM) ? 1 : d.T2).total;
  if (kind & TOK_WS_ENCODE) *bytes = std::max(*bytes, similarity_ws_bytes(N, d.T2, d.H2, d.W2));
  return TOK_OK;
}

tok_status tok_encode(tok_model* m, const uint8_t* x, int N, int T, int H, int W, float* z, float* codes,
                      int32_t* idx, const tok_drop_desc* drop, uint8_t* keep, void* ws, size_t ws_bytes,
                      hipStream_t s) {
  if (!m || !x || !ws) return fail(TOK_EINVAL, "null argument");
  if (!valid_drop(drop)) return fail(TOK_EINVAL, "bad drop descriptor");
  if (m->prec == P_FP8) return fail(TOK_EUNSUPPORTED, "fp8 models hold the decoder only");
  Dims d;
  if (!make_dims(N, T, H, W, &d)) return fail(TOK_ESHAPE, "need N>=1, T%4==1, H%4==0, W%4==0");
  Plan p;
  if (!choose_chunk(d, m->prec, ws_bytes, &p))
    return fail(TOK_EWORKSPACE, "workspace needs " + std::to_string(p.total) + " bytes");
  if (is_similarity(drop)) {
    if (!codes) return fail(TOK_EINVAL, "similarity-based selection needs the codes output");
    if (ws_bytes < similarity_ws_bytes(N, d.T2, d.H2, d.W2))
      return fail(TOK_EWORKSPACE, "workspace too small for the similarity selection");
    if ((reinterpret_cast<uintptr_t>(codes) & 7) || (reinterpret_cast<uintptr_t>(ws) & 15))
      return fail(TOK_EINVAL, "similarity selection needs 8-byte aligned codes and a 16-byte aligned workspace");
    if ((long long)d.T2 * d.H2 * d.W2 > 0x7fffffffLL || N > 65535)
      return fail(TOK_ESHAPE, "similarity selection needs N <= 65535 and under 2^31 tokens per clip");
  }
  Ws w{static_cast<char*>(ws), p};
  const FsqConst fc = make_fsq_const();
  const DropArgs da = make_drop(drop);
  const int CH = m->prec == P_BF16 ? 32 : 16;
  const size_t es = m->prec == P_BF16 ? 2 : 4;
  const size_t f0b = (size_t)H * W * 64 * es, f1b = (size_t)d.H1 * d.W1 * 128 * es;
  const Win pix{T, 0, 0, T};  // the uint8 clip: every frame resident
  const bool chunked = p.CL < d.T2;
  for (int L0 = 0; L0 < d.T2; L0 += p.CL) {
    const int L1 = std::min(L0 + p.CL, d.T2);
    const ChunkWins c = chunk_windows(p, L0, L1);
    TOK_TRY(conv(m, L_CONV_IN, conv_mode(L_CONV_IN), x, IN_U8, N, pix, H, W, 3, w.l0a(), OUT_ACT, c.l0, H, W, nullptr, w.stats(), s));
    TOK_TRY(resblocks(m, L_E_RB1_A, N_E_RB1_A, w, d, c.l0, false, chunked, L0, s));
    TOK_TRY(conv(m, L_DOWN1, CM_S2, w.l0a(), IN_ACT, N, c.l0, H, W, 64, w.l1(), OUT_ACT, c.l1, d.H1, d.W1, nullptr,
                 nullptr, s));
    const Win l2e{p.Tb2, L0, 0, L1 - L0};  // encoder latent activations: no cache needed
    TOK_TRY(conv(m, L_DOWN2, CM_S2, w.l1(), IN_ACT, N, c.l1, d.H1, d.W1, 128, w.l2(), OUT_ACT, l2e, d.H2, d.W2,
                 nullptr, nullptr, s));
    {
      Timed tm(m, L_PROJ, s);
      TOK_HIP(launch_proj_fsq(w.l2(), m->prec, N, p.Tb2, 0, L1 - L0, d.T2, L0, d.H2, d.W2, 128 / CH,
                              m->w1x1[L_PROJ], m->bias[L_PROJ], fc, da, z, codes, idx, keep, s));
    }
    if (L1 < d.T2) {
      TOK_TRY(shift_cache(w.l0a(), c.l0, N, f0b, kCache0, s));
      TOK_TRY(shift_cache(w.l1(), c.l1, N, f1b, kCache1, s));
    }
  }
  if (is_similarity(drop)) {
    // the activations are dead: the selection reuses the workspace from its start
    Timed tm(m, K_SELECT, s);
    TOK_HIP(launch_similarity_drop(codes, keep, N, d.T2, d.H2, d.W2,
                                   similarity_drop_count(drop->rate, (long long)(d.T2 - 1) * d.H2 * d.W2), ws, s));
  }
  return TOK_OK;
}

tok_status tok_quantize(const float* z, size_t n_tokens, float* codes, int32_t* idx, hipStream_t s) {
  if (n_tokens && !z) return fail(TOK_EINVAL, "null z");
  const FsqConst fc = make_fsq_const();
  TOK_HIP(launch_quantize(z, n_tokens, fc, codes, idx, s));
  return TOK_OK;
}

tok_status tok_drop(const tok_drop_desc* drop, float* codes, uint8_t* keep, int N, int T2, int H2, int W2,
                    hipStream_t s) {
  if (!drop || !valid_drop(drop)) return fail(TOK_EINVAL, "bad drop descriptor");
  if (is_similarity(drop)) return fail(TOK_EINVAL, "similarity-based selection needs scratch: tok_select_similar");
  if (N < 1 || T2 < 1 || H2 < 1 || W2 < 1) return fail(TOK_ESHAPE, "bad latent shape");
  if (!codes && !keep) return TOK_OK;
  TOK_HIP(launch_drop(make_drop(drop), codes, keep, N, T2, H2, W2, s));
  return TOK_OK;
}

tok_status tok_select_workspace_size(int N, int T2, int H2, int W2, size_t* bytes) {
  if (!bytes) return fail(TOK_EINVAL, "null argument");
  if (N < 1 || T2 < 1 || H2 < 1 || W2 < 1) return fail(TOK_ESHAPE, "bad latent shape");
  *bytes = similarity_ws_bytes(N, T2, H2, W2);
  return TOK_OK;
}

tok_status tok_select_similar(float rate, float* codes, uint8_t* keep, int N, int T2, int H2, int W2, void* ws,
                              size_t ws_bytes, hipStream_t s) {
  if (!codes || !ws) return fail(TOK_EINVAL, "null argument");
  if (N < 1 || T2 < 1 || H2 < 1 || W2 < 1) return fail(TOK_ESHAPE, "bad latent shape");
  if (N > 65535 || (long long)T2 * H2 * W2 > 0x7fffffffLL)
    return fail(TOK_ESHAPE, "need N <= 65535 and under 2^31 tokens per clip");
  if (ws_bytes < similarity_ws_bytes(N, T2, H2, W2)) return fail(TOK_EWORKSPACE, "workspace too small");
  if ((reinterpret_cast<uintptr_t>(codes) & 7) || (reinterpret_cast<uintptr_t>(ws) & 15))
    return fail(TOK_EINVAL, "codes must be 8-byte and ws 16-byte aligned");
  TOK_HIP(launch_similarity_drop(codes, keep, N, T2, H2, W2,
                                 similarity_drop_count(rate, (long long)(T2 - 1) * H2 * W2), ws, s));
  return TOK_OK;
}

tok_status tok_select_similar_noalloc(float rate, float* codes, uint8_t* keep, int N, int T2, int H2, int W2,
                                      hipStream_t s) {
  if (!codes) return fail(TOK_EINVAL, "null codes");
  if (N < 1 || T2 < 1 || H2 < 1 || W2 < 1) return fail(TOK_ESHAPE, "bad latent shape");
  if (N > 65535 || (long long)T2 * H2 * W2 > 0x7fffffffLL)
    return fail(TOK_ESHAPE, "need N <= 65535 and under 2^31 tokens per clip");
  const size_t need = similarity_ws_bytes(N, T2, H2, W2);
  if (need > kSimilarityScratchBytes)
    return fail(TOK_EWORKSPACE, "selection needs " + std::to_string(need) + " bytes of scratch, the static scratch holds " +
                                    std::to_string(kSimilarityScratchBytes));
  if (reinterpret_cast<uintptr_t>(codes) & 7) return fail(TOK_EINVAL, "codes must be 8-byte aligned");
  void* ws = nullptr;
  TOK_HIP(similarity_scratch(&ws));
  TOK_HIP(launch_similarity_drop(codes, keep, N, T2, H2, W2,
                                 similarity_drop_count(rate, (long long)(T2 - 1) * H2 * W2), ws, s));
  return TOK_OK;
}

tok_status tok_select_scratch_bytes(size_t* bytes) {
  if (!bytes) return fail(TOK_EINVAL, "null argument");
  *bytes = kSimilarityScratchBytes;
  return TOK_OK;
}

namespace {

tok_status decode_impl(tok_model* m, const float* codes, int N, int T2, int H2, int W2, float* xhat, void* ws,
                       size_t ws_bytes, hipStream_t s, const Blend* blend, const ResAcc* racc = nullptr) {
  if (!m || !codes || !xhat || !ws) return fail(TOK_EINVAL, "null argument");
  if (T2 < 1 || H2 < 1 || W2 < 1) return fail(TOK_ESHAPE, "bad latent shape");
  Dims d;
  if (!make_dims(N, 4 * (T2 - 1) + 1, 4 * H2, 4 * W2, &d)) return fail(TOK_ESHAPE, "bad latent shape");
  if (blend && (!blend->prev || blend->n < 1 || blend->n > d.T || blend->n > blend->Tp ||
                (reinterpret_cast<uintptr_t>(blend->prev) & 3)))
    return fail(TOK_EINVAL, "blend needs a 4-byte aligned prev and 1 <= n <= T, T_prev");
  if (blend && m->prec == P_FP8 &&
      ((reinterpret_cast<uintptr_t>(blend->prev) & 15) || (reinterpret_cast<uintptr_t>(xhat) & 15)))
    return fail(TOK_EINVAL, "fp8 blend (a separate pass) needs 16-byte aligned prev and xhat");
  if (m->prec == P_FP8) return decode_fp8(m, codes, d, xhat, ws, ws_bytes, s, blend);
  Plan p;
  if (!choose_chunk(d, m->prec, ws_bytes, &p))
    return fail(TOK_EWORKSPACE, "workspace needs " + std::to_string(p.total) + " bytes");
  Ws w{static_cast<char*>(ws), p};
  const int CH = m->prec == P_BF16 ? 32 : 16;
  const size_t es = m->prec == P_BF16 ? 2 : 4;
  const size_t f0b = (size_t)d.H * d.W * 64 * es, f1b = (size_t)d.H1 * d.W1 * 128 * es;
  const size_t f2b = (size_t)d.H2 * d.W2 * 128 * es;
  const bool chunked = p.CL < d.T2;
  for (int L0 = 0; L0 < d.T2; L0 += p.CL) {
    const int L1 = std::min(L0 + p.CL, d.T2);
    const ChunkWins c = chunk_windows(p, L0, L1);
    {
      Timed tm(m, L_PROJ_IN, s);
      TOK_HIP(launch_proj_in(codes, N, d.T2, L0, L1 - L0, H2 * W2, m->w1x1[L_PROJ_IN], m->bias[L_PROJ_IN], m->prec,
                             w.l2(), 128 / CH, p.Tb2, c.l2.first, s));
    }
    TOK_TRY(conv(m, L_UP2, CM_UPF, w.l2(), IN_ACT, N, c.l2, d.H2, d.W2, 128, w.l1(), OUT_ACT, c.l1, d.H1, d.W1,
                 nullptr, nullptr, s));
    TOK_TRY(conv(m, L_UP1, CM_UPF, w.l1(), IN_ACT, N, c.l1, d.H1, d.W1, 128, w.l0a(), OUT_ACT, c.l0, d.H, d.W,
                 nullptr, w.stats(), s));
    TOK_TRY(resblocks(m, L_D_RB1_A, N_D_RB1_A, w, d, c.l0, false, chunked, L0, s));
    const Win ow{d.T, 0, c.l0.g0 + c.l0.first, c.l0.count};
    TOK_TRY(conv(m, L_CONV_OUT, CM_S1, w.l0a(), IN_ACT, N, c.l0, d.H, d.W, 64, xhat, OUT_RGB32, ow, d.H, d.W, nullptr,
                 nullptr, s, nullptr, nullptr, blend, racc));
    if (L1 < d.T2) {
      TOK_TRY(shift_cache(w.l2(), c.l2, N, f2b, kCache2, s));
      TOK_TRY(shift_cache(w.l1(), c.l1, N, f1b, kCache1, s));
      TOK_TRY(shift_cache(w.l0a(), c.l0, N, f0b, kCache0, s));
    }
  }
  return TOK_OK;
}

}  // namespace

tok_status tok_decode(tok_model* m, const float* codes, int N, int T2, int H2, int W2, float* xhat, void* ws,
                      size_t ws_bytes, hipStream_t s) {
  return decode_impl(m, codes, N, T2, H2, W2, xhat, ws, ws_bytes, s, nullptr);
}

tok_status tok_decode_blend(tok_model* m, const float* codes, int N, int T2, int H2, int W2, const float* prev,
                            int T_prev, int n, float* xhat, void* ws, size_t ws_bytes, hipStream_t s) {
  const Blend b{prev, T_prev, n};
  return decode_impl(m, codes, N, T2, H2, W2, xhat, ws, ws_bytes, s, &b);
}

tok_status tok_decode_residual(tok_model* m, const float* codes, int N, int T2, int H2, int W2, const uint8_t* x,
                               float theta, float* xhat, float* r, uint32_t* index, float* value, size_t capacity,
                               uint64_t* clip_offsets, void* ws, size_t ws_bytes, void* rs_ws, size_t rs_ws_bytes,
                               hipStream_t s) {
  if (!m || !x || !r || !clip_offsets || !rs_ws || (capacity && (!index || !value))) return fail(TOK_EINVAL, "null argument");
  auto al = [](const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; };
  if (!al(x, 16) || !al(r, 16) || !al(clip_offsets, 8) || !al(rs_ws, 4) || !al(index, 4) || !al(value, 4))
    return fail(TOK_EINVAL, "x and r must be 16-byte, clip_offsets 8-byte, rs_ws, index and value 4-byte aligned");
  if (T2 < 1 || H2 < 1 || W2 < 1 || N < 1 || N > 65535 || (long long)N * 3 * (4 * H2) * (4 * W2) >= 0xffffffffLL)
    return fail(TOK_ESHAPE, "bad latent shape, or N H W 3 >= 2^32");
  const int T = 4 * (T2 - 1) + 1, H = 4 * H2, W = 4 * W2;
  if (rs_ws_bytes < residual_ws_bytes(N, H, W)) return fail(TOK_EWORKSPACE, "residual workspace too small");
  if (m->prec != P_BF16) {
    // (the fp32 last layer does not walk frames, and the fp8 walk with the sums measured slower than
    // decode then the standalone pass: that is what these models run)
    TOK_TRY(decode_impl(m, codes, N, T2, H2, W2, xhat, ws, ws_bytes, s, nullptr));
    Timed tm(m, K_RESID, s);
    TOK_HIP(launch_residual(x, xhat, N, T, H, W, theta, r, index, value, (long long)capacity,
                            reinterpret_cast<unsigned long long*>(clip_offsets), rs_ws, s));
    return TOK_OK;
  }
  const ResAcc ra{x, r, T};
  TOK_TRY(decode_impl(m, codes, N, T2, H2, W2, xhat, ws, ws_bytes, s, nullptr, &ra));
  Timed tm(m, K_RESID, s);
  TOK_HIP(launch_residual_sums(r, N, T, H, W, theta, index, value, (long long)capacity,
                               reinterpret_cast<unsigned long long*>(clip_offsets), rs_ws, s));
  return TOK_OK;
}

}  // extern "C"
