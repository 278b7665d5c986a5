// Internal interface between the C-ABI layer (tok_api.hip) and the kernel
// translation units (conv3d.hip, pointwise.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tok {

// Activations between layers use a channel-chunked layout:
//   [N][T][C / CH][H][W][CH]   with CH = 64 bytes / sizeof(element)
// so that one 64-byte chunk of one position is contiguous and a halo row of
// a chunk is one contiguous run of memory.
constexpr int kChunkBytes = 64;

// P_FP8: conv inputs and weights in fp8 e4m3 (OCP) on the scaled MFMA, fp32
// accumulate; see "MX-FP8 activations" below.
enum Prec { P_F32 = 0, P_BF16 = 1, P_FP8 = 2 };
// CM_UP: nearest x2 upsample folded into the halo addressing (27 taps);
// CM_UPF: the same operation in polyphase form (8 folded taps per output).
// CM_S1T: the adjoint (input gradient) of a stride-1 causal conv: anti-causal
// in time, spatially flipped, channels transposed; output frame 0 uses the
// temporal taps folded by the causal clamp (frame 0 is read three times).
// CM_I2C: the first layer (3 input channels, uint8 pixels): each output
// position's 27 taps x 3 channels are gathered in LDS into one K vector of 27
// taps x 4 (the 4th channel zero, so a tap is one 16-byte LDS read) padded to
// 128, and the layer runs as a single-tap product with ~7x fewer MFMAs than
// 27 taps of a 3-channel (padded) chunk.
// CM_S2T: the adjoint of a stride-2 causal conv, coarse gradient in, fine
// gradient out, in the polyphase form of CM_UPF (one wave per output phase,
// 2 x 2 x 2 source offsets per output; along each of t, h, w an output of
// parity 0 takes tap 1 from offset 0, parity 1 taps 2 and 0 from offsets 0
// and +1), instead of zero insertion and the dense stride-1 adjoint.
// CM_UPT: the adjoint of the upsampling conv, fine gradient in, source-resolution
// gradient out: a stride-2 conv over the fine gradient with 4 x 4 x 4 folded
// taps (along each dimension fine offsets -1, 0, +1, +2 around 2 s carry
// forward taps 2, 1 + 2, 0 + 1, 0; source frame 0 also collects the causal
// clamp), 8 instead of 27 Cin Cout MACs per fine position.
enum ConvMode { CM_S1 = 0, CM_S2 = 1, CM_UP = 2, CM_UPF = 3, CM_S1T = 4, CM_I2C = 5, CM_S2T = 6, CM_UPT = 7 };
constexpr int kI2cK = 128;  // 27 taps x 4 channels, padded to whole 32-element bf16 chunks
enum InKind { IN_ACT = 0, IN_U8 = 1 };
// OUT_ACT: chunked activations of the kernel's output precision (bf16 for
// P_FP8 kernels); OUT_FP8: MX-FP8 activations; OUT_RGB32: float NDHWC (3 ch).
enum OutKind { OUT_ACT = 0, OUT_RGB32 = 1, OUT_FP8 = 2 };

// MX-FP8 activations (the inputs of the P_FP8 convs): e4m3 values in the
// chunked layout with 64 channels per 64-byte chunk, plus a scale plane
// [N][T][C/64][H][W][2] of E8M0 bytes, one per (position, 32 channels): the
// value of an element is e4m3 * 2^(scale - 127).  The scale of a block is the
// smallest power of two that brings its largest magnitude to <= 448, so no
// element saturates.  The MFMA applies these scales itself (one per lane and
// 32-element K block).

// Weight gradient of a causal 3x3x3 conv (whole clips, no windows):
//   dW[o][i][kt][kh][kw] = sum over output positions p of dy[p][o] * x~[p + tap][i]
// where x~ is the conv's input seen through `view` (CM_S1 stride 1, CM_S2
// stride 2, CM_UP nearest x2 upsampled); with bpartial set, also the bias
// gradient db[o] = sum_p dy[p][o].  Each block reduces a share (split) of the
// output positions for one (temporal tap, 32 input channels, 64 output
// channels); partials [split][kt][9][Cout][Cin] and [split][Cout] are summed in
// split order by launch_wgrad_reduce into the canonical [Cout][Cin][3][3][3]
// layout, so the result does not depend on scheduling.
struct WgradLaunch {
  const void* x;      // chunked activations (Cin channels)
  int N, Ti, Hi, Wi, x_chunks;
  const void* dy;     // chunked gradients (Cout channels)
  int To, Ho, Wo, dy_chunks;
  int Cout, Cin;
  int view, prec;
  int splits;
  float* partial;     // [splits][taps][Cout][Cin], taps = wgrad_partial_taps(prec, view)
  float* bpartial;    // [splits][wgrad_bias_parts(prec, view)][Cout] or null
};
// Blocks per split, and work items (output tiles) shared among the splits,
// of the weight-gradient launch for these operands: bf16 operands with Cin
// and Cout multiples of 64 run on bf16 MFMA, everything else on fp32 MFMA.
int wgrad_blocks_per_split(int prec, int view, int Cout, int Cin);
int wgrad_items(int prec, int view, int Cout, int Cin, int N, int To, int Ho, int Wo);
// Partial sums per split: wgrad_partial_taps(...) x [Cout][Cin] floats of
// weights (27 taps, or 64 folded taps of the polyphase upsampling view) and
// wgrad_bias_parts(...) x [Cout] of bias.
int wgrad_partial_taps(int prec, int view);
int wgrad_bias_parts(int prec, int view);
hipError_t launch_wgrad(const WgradLaunch& a, hipStream_t s);
// Sums a launch's partials (in split order) into dw [Cout][Cin][3][3][3] and db.
hipError_t launch_wgrad_reduce(const WgradLaunch& a, float* dw, float* db, hipStream_t s);

// Frames are addressed in windows so that a clip can be processed in causal
// temporal chunks: a buffer holds Tb frames per clip, its frame 0 is global
// frame g0 of the clip, and a layer computes `count` output frames starting at
// buffer frame `first`.  Whole-clip processing is the window (T, 0, T, 0).
struct ConvLaunch {
  // input
  const void* in;        // IN_ACT: chunked activations; IN_U8: uint8 NDHWC (3 ch)
  int N, Ti, Hi, Wi;     // clips, input buffer frames per clip, spatial size
  int gi0;               // global frame index of input buffer frame 0
  int in_chunks;         // 64-byte chunks per input position
  int Cin;
  // weights (packed, see pack_conv_weights) and bias [Cout]
  const void* wpk;
  const float* bias;
  int Cout, cout_tiles, nt;  // nt = output channels per tile (64 or 16)
  // output
  void* out;             // OUT_ACT: chunked activations; OUT_RGB32: float NDHWC (3 ch)
  const void* resid;     // optional residual, same layout as out (may alias out)
  int To, Ho, Wo;        // output frames computed, spatial size
  int To_buf, out_f0;    // output buffer frames per clip, buffer frame of the first computed frame
  int go0;               // global frame index of the first computed frame
  int out_chunks;
  float4* stats;         // optional per-tile GroupNorm partials [N][To][tiles][32]
  int tiles_h, tiles_w;
  int mode, in_kind, out_kind, prec;
  // P_FP8 only: input scale plane, output scale plane (OUT_FP8), per-output-
  // channel weight scales [Cout]
  const uint8_t* in_scale;
  uint8_t* out_scale;
  const float* wscale;
  // OUT_RGB32 only: GoP-boundary blending (Sec. 4.2, Eq. 2) of global output
  // frames t < blend_n with frame blend_Tp - blend_n + t of blend_prev
  // (float NDHWC, blend_Tp frames per clip); null for none.
  const float* blend_prev;
  int blend_Tp, blend_n;
  // Frame-walking last layer only: pixel-residual sums (Sec. 4.3, Eq. 4) of
  // the frames written, sum_t (x_t / 127.5 - 1 - x_hat_t) per (n, h, w,
  // colour) in frame order (x_hat_t as stored, i.e. after blending), in fp32
  // into rs_sum (float (N, Ho, Wo, 3)); they start from rs_sum's contents
  // when go0 > 0 (a later chunk of the clip), else from 0.  rs_x is the
  // uint8 source (N, rs_T, Ho, Wo, 3), indexed by global frame.  Null: none.
  const uint8_t* rs_x;
  float* rs_sum;
  int rs_T;
};

// Tile geometry per mode (output rows x cols per workgroup).
inline void conv_tile(int mode, int* th, int* tw) {
  if (mode == CM_S2) { *th = 8; *tw = 32; }
  else if (mode == CM_UPT) { *th = 4; *tw = 32; }
  else { *th = 8; *tw = 64; }
}

hipError_t launch_conv(const ConvLaunch& a, hipStream_t s);

// Packing of a device-resident [Cout][Cin][3][3][3] float kernel into the
// layout the conv kernel streams through LDS (see conv3d.hip), on the device.
// packed_conv_elems returns the element count and the output-channel tile.
// For mode CM_S1T, (Cout, Cin) are the forward conv's; the packed kernel maps
// Cout-channel gradients to Cin-channel gradients.
size_t packed_conv_elems(int Cout, int Cin, int prec, int mode, int* nt_out);
// For P_FP8, wscale [Cout] receives the per-output-channel scales (largest
// magnitude of the channel's packed kernel / 448) and the packed values are
// e4m3(w / wscale); wscale is ignored otherwise.
hipError_t launch_pack_weights(const float* w, int Cout, int Cin, int prec, int mode, void* dst, float* wscale,
                               hipStream_t s);

// GroupNorm: merge per-tile partials of each (n, t) frame into per-channel
// scale/shift for the consumer's prologue.
// With mr set, also the (mean, rstd) of each (frame, group) for the backward;
// with gamma null only mr is written (scale, shift, beta unused).
hipError_t launch_gn_finalize(const float4* stats, int frames, int tiles, const float* gamma,
                              const float* beta, float eps, float* scale, float* shift, float2* mr,
                              hipStream_t s);

// y = silu(x * scale[n,f,c] + shift[n,f,c]) for f in [0, F): x is frame
// in_f0 + f of a level-0 buffer with in_Tb frames per clip, y frame out_f0 + f
// of one with out_Tb (64 channels, chunked layout); in place when the two
// coincide.  scale/shift are indexed by (n, f).
hipError_t launch_gn_act(const void* in, int in_Tb, int in_f0, void* out, int out_Tb, int out_f0, int prec, int N,
                         int F, int HW, const float* scale, const float* shift, hipStream_t s);
// The same from bf16 activations into MX-FP8 activations (out + out_scale).
hipError_t launch_gn_act_fp8(const void* in, int in_Tb, int in_f0, uint8_t* out, uint8_t* out_scale, int out_Tb,
                             int out_f0, int N, int F, int HW, const float* scale, const float* shift, hipStream_t s);

struct FsqConst {
  float h[6], o[6], s[6], inv_d[6], d[6];
  int basis[6];
};

struct DropArgs {
  int mode;
  uint32_t thr;        // floor(rate * 2^24)
  uint64_t seed;
  uint64_t clip_id0;
  int protect_iframe;
  const uint8_t* ext_keep;
};

// 1x1x1 projection 128 -> 6 on level-2 activations, FSQ, mask, zero fill.
// Reads frames [f0, f0+F) of an activation buffer of Tb frames per clip and
// writes latent frames [t0, t0+F) of dense (N, T2, H2, W2, .) outputs.
hipError_t launch_proj_fsq(const void* act, int prec, int N, int Tb, int f0, int F, int T2, int t0, int H2,
                           int W2, int in_chunks, const float* wp, const float* bp, const FsqConst& fc,
                           const DropArgs& d, float* z, float* codes, int32_t* idx, uint8_t* keep,
                           hipStream_t s);
hipError_t launch_quantize(const float* z, size_t n, const FsqConst& fc, float* codes,
                           int32_t* idx, hipStream_t s);
hipError_t launch_drop(const DropArgs& d, float* codes, uint8_t* keep, int N, int T2, int H2,
                       int W2, hipStream_t s);
// Similarity-based token selection (Sec. 4.3, Eq. 3): drops the D P tokens of
// each clip most similar to the co-located I token (ties to the lower index)
// from codes (N, T2, H2, W2, 6) in place and writes keep (or NULL).  ws holds
// similarity_ws_bytes(N, T2, H2, W2) bytes (unused when D is 0 or every P token).
size_t similarity_ws_bytes(int N, int T2, int H2, int W2);
// Bytes of the per-device static selection scratch (tok_select_similar_noalloc),
// and its address on the current device (taken once per device).
constexpr size_t kSimilarityScratchBytes = (size_t)32 << 20;
hipError_t similarity_scratch(void** ptr);
// Row packets of Sec. 6.2 (format in packets.hip): the sender writes packet
// offsets[g] .. offsets[g+1] of every row g and offsets[G] = stream length;
// the receiver zero-fills codes / keep and scatters the packets at offsets.
long long packets_max_bytes(int N, int T2, int H2, int W2);
hipError_t launch_packetize(const int32_t* idx, const uint8_t* keep, int N, int T2, int H2, int W2, uint8_t* out,
                            unsigned long long* offsets, hipStream_t s);
hipError_t launch_reassemble(const uint8_t* buf, unsigned long long bytes, const unsigned long long* offsets,
                             long long n_packets, int N, int T2, int H2, int W2, float* codes, uint8_t* keep,
                             hipStream_t s);
// Pixel residuals (Sec. 4.3, Eq. 4) and GoP blending (Sec. 4.2, Eq. 2), see enhance.hip.
size_t residual_ws_bytes(int N, int H, int W);
hipError_t launch_residual(const uint8_t* x, const float* xhat, int N, int T, int H, int W, float theta, float* rs,
                           uint32_t* index, float* value, long long capacity, unsigned long long* clip_off,
                           void* ws, hipStream_t s);
// The same from sums rs[n, h, w, c] = sum_t (x_t / 127.5 - 1 - x_hat_t) the
// decoder's last layer accumulated (rs becomes the thresholded mean).
hipError_t launch_residual_sums(float* rs, int N, int T, int H, int W, float theta, uint32_t* index, float* value,
                                long long capacity, unsigned long long* clip_off, void* ws, hipStream_t s);
hipError_t launch_residual_apply(const float* rs, float* xhat, int N, int T, int H, int W, hipStream_t s);
hipError_t launch_blend(const float* prev, int Tp, float* cur, int N, int T, int H, int W, int nb, hipStream_t s);
hipError_t launch_similarity_drop(float* codes, uint8_t* keep, int N, int T2, int H2, int W2, long long D, void* ws,
                                  hipStream_t s);
// 1x1x1 projection 6 -> 128: latent frames [t0, t0+F) of dense codes
// (N, T2, HW, 6) into buffer frames [f0, f0+F) of chunked activations with Tb
// frames per clip.
hipError_t launch_proj_in(const float* codes, int N, int T2, int t0, int F, int HW, const float* w,
                          const float* b, int prec, void* out, int out_chunks, int Tb, int f0, hipStream_t s);
// The same into MX-FP8 activations (128 channels: 2 chunks, 4 scales per position).
hipError_t launch_proj_in_fp8(const float* codes, int N, int T2, int t0, int F, int HW, const float* w,
                              const float* b, uint8_t* out, uint8_t* out_scale, int Tb, int f0, hipStream_t s);

// ---------------------------------------------------------------------------
// Backward pass (backward.hip).  Dense latent tensors are (N, T2, H2, W2, 6)
// float; activations and gradients use the chunked layout above.
// ---------------------------------------------------------------------------
int l1_blocks(size_t npos);
int fsq_blocks(size_t ntok);
size_t outer6_partial_floats(size_t ntok);
size_t gn_bwd_partial_floats(int frames, int HW, int prec);
// Partial sums of |x_hat - x| (x uint8, mapped to [-1, 1]) per 256 positions;
// with g set also the gradient seed gscale * sign(x_hat - x) / numel into a
// one-chunk activation buffer.  gscale: device scalar or null (1).
hipError_t launch_l1(const float* xhat, const uint8_t* x, size_t npos, int prec, const float* gscale, void* g,
                     float* partial, hipStream_t s);
hipError_t launch_u8_to_chunked(const uint8_t* x, size_t npos, int prec, void* out, hipStream_t s);
// Commitment partial sums; with gdec set also the straight-through adjoint gz.
hipError_t launch_fsq_bwd(const float* z, const uint8_t* keep, const float* gdec, size_t ntok, const FsqConst& fc,
                          float coef, const float* gscale, float* gz, float* partial, hipStream_t s);
hipError_t launch_loss_final(const float* l1p, int nl1, const float* cp, int nc, float inv_numel, float inv_m,
                             float commit_weight, float* loss, hipStream_t s);
// GroupNorm(32) + SiLU backward over `frames` frames of HW positions, 64
// channels: dx = d/dx of silu(gn(x)) applied to g, plus resid (nullable); dx
// may alias g or resid.  dgamma / dbeta receive the parameter gradients.
hipError_t launch_gn_bwd(const void* x, const void* g, const float2* mr, const float* gamma, const float* beta,
                         const void* resid, void* dx, int frames, int HW, int prec, float* partial, float2* fsum,
                         float2* m12, float* dgamma, float* dbeta, hipStream_t s);
// Adjoint of the nearest x2 upsample (time map t -> ceil(t / 2)).
hipError_t launch_up_adjoint(const void* fine, void* coarse, int N, int Tc, int Hc, int Wc, int chunks, int prec,
                             hipStream_t s);
// y[p][k] = sum_c w6[k][c] x[p][c] (128 chunked channels -> 6 dense).
hipError_t launch_proj6(const void* x, size_t ntok, int HW, const float* w6, float* y, int prec, hipStream_t s);
// 1x1x1 weight / bias gradients from dense a6 (6 wide) and chunked x (128).
hipError_t launch_outer6(const float* a6, const void* x, size_t ntok, int HW, int prec, float* partial,
                         int transposed, float* dw, float* db, hipStream_t s);
hipError_t launch_transpose(const float* in, int R, int C, float* out, hipStream_t s);

// ---------------------------------------------------------------------------
// Per-operation entry points (ops.hip).
// ---------------------------------------------------------------------------
// dense [frames][HW][C] float <-> chunked activations of prec (channels past C
// zero when packing, dropped when unpacking).
hipError_t launch_act_pack(const float* src, long long frames, int HW, int C, int prec, void* dst, hipStream_t s);
hipError_t launch_act_unpack(const void* src, long long frames, int HW, int C, int prec, float* dst, hipStream_t s);
// GroupNorm(32) per-tile partials of a 64-channel chunked tensor (the layout
// launch_gn_finalize merges), gn_op_tiles(HW) tiles per frame.
int gn_op_tiles(int HW);
hipError_t launch_gn_partials(const void* x, int frames, int HW, int prec, float4* stats, hipStream_t s);
// scale / shift [frames][64] from (mean, rstd) [frames][32] and the affine.
hipError_t launch_gn_affine(const float2* mr, const float* gamma, const float* beta, int frames, float* scale,
                            float* shift, hipStream_t s);
// g_z = g_z_in + keep (g_a + g_b) dz~/dz (straight-through quantiser); any
// input may be null.
hipError_t launch_fsq_ste(const float* z, const uint8_t* keep, const float* ga, const float* gb, const float* gzin,
                          size_t ntok, const FsqConst& fc, float* gz, hipStream_t s);
// dense float (npos, 3) -> one-chunk activations (channels 3.. zero).
hipError_t launch_rgb_to_chunk(const float* src, size_t npos, int prec, void* out, hipStream_t s);
hipError_t launch_fill_zero(float* p, size_t n, hipStream_t s);

}  // namespace tok
