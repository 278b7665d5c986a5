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

enum Prec { P_F32 = 0, P_BF16 = 1 };
// CM_UP: nearest x2 upsample folded into the halo addressing (27 taps);
// CM_UPF: the same operation in polyphase form (8 folded taps per output).
enum ConvMode { CM_S1 = 0, CM_S2 = 1, CM_UP = 2, CM_UPF = 3 };
enum InKind { IN_ACT = 0, IN_U8 = 1 };
enum OutKind { OUT_ACT = 0, OUT_RGB32 = 1 };

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
};

// Tile geometry per mode (output rows x cols per workgroup).
inline void conv_tile(int mode, int* th, int* tw) {
  if (mode == CM_S2) { *th = 4; *tw = 32; }
  else { *th = 8; *tw = 64; }
}

hipError_t launch_conv(const ConvLaunch& a, hipStream_t s);

// Host-side packing of a [Cout][Cin][3][3][3] float kernel into the layout the
// conv kernel streams through LDS (see conv3d.hip).  Returns element count.
size_t packed_conv_elems(int Cout, int Cin, int prec, int mode, int* nt_out);
void pack_conv_weights(const float* w, int Cout, int Cin, int prec, int mode, void* dst);

// GroupNorm: merge per-tile partials of each (n, t) frame into per-channel
// scale/shift for the consumer's prologue.
hipError_t launch_gn_finalize(const float4* stats, int frames, int tiles, const float* gamma,
                              const float* beta, float eps, float* scale, float* shift,
                              hipStream_t s);

// y = silu(x * scale[n,f,c] + shift[n,f,c]) for f in [0, F): x is frame
// in_f0 + f of a level-0 buffer with in_Tb frames per clip, y frame out_f0 + f
// of one with out_Tb (64 channels, chunked layout); in place when the two
// coincide.  scale/shift are indexed by (n, f).
hipError_t launch_gn_act(const void* in, int in_Tb, int in_f0, void* out, int out_Tb, int out_f0, int prec, int N,
                         int F, int HW, const float* scale, const float* shift, hipStream_t s);

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
// 1x1x1 projection 6 -> 128: latent frames [t0, t0+F) of dense codes
// (N, T2, HW, 6) into buffer frames [f0, f0+F) of chunked activations with Tb
// frames per clip.
hipError_t launch_proj_in(const float* codes, int N, int T2, int t0, int F, int HW, const float* w,
                          const float* b, int prec, void* out, int out_chunks, int Tb, int f0, hipStream_t s);

}  // namespace tok
