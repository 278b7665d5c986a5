// Causal 3x3x3 convolution as an implicit GEMM on CDNA4 matrix cores.
//
// Operation (the tokenizer's building block; causal in time so that a latent
// frame depends only on frames up to it, Sec. 4.3 I/P structure):
//   y[n,t,h,w,o] = b[o] + sum_{kt,kh,kw,i} W[o,i,kt,kh,kw] x~[n, s t + kt - 2, s h + kh - 1, s w + kw - 1, i]
// x~ repeats frame 0 for negative time indices and is 0 outside the frame.
// Three addressing modes share the kernel: stride 1, stride 2 in t/h/w, and a
// nearest x2 upsample of the input (time index ceil(u/2), spatial floor(./2))
// folded into the halo addressing.
//
// Mapping to MFMA (GEMM D = A x B):
//   A = weights   (rows: 16 output channels,  K: input channels of one tap)
//   B = activations (K: input channels,     cols: 16 output positions)
// so each lane of the 16x16 accumulator holds one output position and four
// consecutive output channels, which is what the NDHWC-style store and the
// GroupNorm statistics want.
//
// Workgroup = 4 waves.  A workgroup owns one output frame (n, t), a TH x TW
// spatial tile and nt output channels.  The K loop runs over the 3 temporal
// taps x the 64-byte input-channel chunks; per step it stages into LDS
//   * the spatial halo of one input frame / chunk, and
//   * the 9 spatial taps of packed weights for that (kt, chunk),
// both with direct global->LDS loads (no VGPR staging),
// then every wave runs 9 taps x (its position blocks x channel blocks) MFMAs.
// 16-byte quads inside a 64-byte LDS row are XOR-swizzled by the row index so
// that the 16 lanes reading 16 consecutive rows hit distinct banks.
#include <utility>

#include "tok_internal.h"
#include "tok_device.h"

namespace tok {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = 4;

__host__ __device__ __forceinline__ int swz(int row) { return (row >> 1) & 3; }

template <int PREC> struct Op;
template <> struct Op<P_F32> { static constexpr int CH = 16; static constexpr int QE = 4; };
template <> struct Op<P_BF16> { static constexpr int CH = 32; static constexpr int QE = 8; };
template <> struct Op<P_FP8> { static constexpr int CH = 64; static constexpr int QE = 16; };

// Per mode: output tile TH x TW, halo HH x HW (rows x positions), position
// blocks per wave MB, weight tap-matrices per stage WT, temporal stages KTS.
template <int MODE> struct Geo;
template <> struct Geo<CM_S1> {
  static constexpr int WR = 2, TW = 64, TH = 8, HH = TH + 2, HW = TW + 2;
  static constexpr int MB = WR * TW / 16, WT = 9, KTS = 3;
};
// Stride 2: a stage is one kernel row kh of one (temporal tap, input chunk):
// the 8 input rows 2 i + kh - 1 the tile's output rows i read through it,
// columns de-interleaved by parity, and that row's 3 taps of weights.
template <> struct Geo<CM_S2> {
  static constexpr int WR = 2, TW = 32, TH = 8, HH = TH, HW = 2 * TW + 1;
  static constexpr int MB = WR * TW / 16, WT = 3, KTS = 3;
};
template <> struct Geo<CM_S1T> : Geo<CM_S1> {};
// im2col first layer: no halo staging (the MFMA operands are gathered from
// the normalised pixel tile), one tap, one stage per 32-wide (bf16) K chunk.
template <> struct Geo<CM_I2C> {
  static constexpr int WR = 2, TW = 64, TH = 8, HH = 1, HW = 1;
  static constexpr int MB = 8, WT = 1, KTS = 1;
};

// Polyphase upsample conv: wave w owns output phase (h & 1, w & 1) = (w >> 1, w & 1)
// of the tile, i.e. 4 source rows x 32 source columns = 8 blocks; a stage holds
// the 2 x 2 folded taps of all 4 phases.
template <> struct Geo<CM_UPF> {
  static constexpr int WR = 0, TW = 64, TH = 8, HH = TH / 2 + 2, HW = TW / 2 + 2;
  static constexpr int MB = (TH / 2) * (TW / 2 / 16), WT = 16, KTS = 2;
};
// The stride-2 adjoint runs on the polyphase path (coarse gradient as source).
template <> struct Geo<CM_S2T> : Geo<CM_UPF> {};
// The upsampling adjoint: stride 2 over the fine gradient, 4 x 4 spatial taps
// (halo columns de-interleaved by parity as for CM_S2), 4 temporal stages.
template <> struct Geo<CM_UPT> {
  static constexpr int WR = 1, TW = 32, TH = 4, HH = 2 * TH + 2, HW = 2 * TW + 2;
  static constexpr int MB = WR * TW / 16, WT = 16, KTS = 4;
};

// Stride-1 modes give each wave a 4 x 32 sub-tile (waves 2 x 2 over the 8 x 64
// workgroup tile): an activation operand loaded for halo row r then serves
// output rows r - kh for every kh, a third fewer LDS reads than 2 x 64 rows.

// Workgroups per CU the bf16 first-layer kernel is compiled for (three since
// its GroupNorm partials are reduced through LDS: 2 VGPRs spill, against 53
// with the shuffle trees).
constexpr int kI2cOcc = 3;

// Output-tile-local position of lane l16 in position block m of a wave.
template <int MODE>
__device__ __forceinline__ void out_local(int wave, int m, int l16, int* i, int* j) {
  using G = Geo<MODE>;
  if constexpr (MODE == CM_S1 || MODE == CM_S1T || MODE == CM_I2C) {
    *i = 4 * (wave >> 1) + (m >> 1);
    *j = 32 * (wave & 1) + 16 * (m & 1) + l16;
  } else if constexpr (MODE == CM_UPF || MODE == CM_S2T) {
    *i = 2 * (m >> 1) + (wave >> 1);
    *j = 2 * ((m & 1) * 16 + l16) + (wave & 1);
  } else {
    constexpr int BPR = G::TW / 16;
    *i = wave * G::WR + m / BPR;
    *j = (m % BPR) * 16 + l16;
  }
}

// LDS row (position) index of output-local (i, j) for tap (kh, kw).
template <int MODE>
__device__ __forceinline__ int act_row(int i, int j, int kh, int kw) {
  using G = Geo<MODE>;
  if constexpr (MODE == CM_S1 || MODE == CM_S1T) {
    return (i + kh) * G::HW + (j + kw);
  } else if constexpr (MODE == CM_S2 || MODE == CM_UPT) {
    const int c = 2 * j + kw;
    return (2 * i + kh) * G::HW + (c & 1) * (G::TW + 1) + (c >> 1);
  } else {
    return ((i + kh + 1) >> 1) * G::HW + ((j + kw + 1) >> 1);
  }
}

// Source (h, w) of halo row p.
template <int MODE>
__device__ __forceinline__ void halo_src(int p, int h0, int w0, int* hs, int* ws) {
  using G = Geo<MODE>;
  const int r = p / G::HW;
  const int pc = p - r * G::HW;
  if constexpr (MODE == CM_S1 || MODE == CM_S1T) {
    *hs = h0 - 1 + r;
    *ws = w0 - 1 + pc;
  } else if constexpr (MODE == CM_S2 || MODE == CM_UPT) {
    const int c = (pc < G::TW + 1) ? 2 * pc : 2 * (pc - (G::TW + 1)) + 1;
    *hs = MODE == CM_S2 ? 2 * (h0 + r) - 1 : 2 * h0 - 1 + r;  // stride 2: row of kernel row 0
    *ws = 2 * w0 - 1 + c;
  } else {  // CM_UPF / CM_S2T: source rows / columns of the tile
    *hs = (h0 >> 1) - 1 + r;
    *ws = (w0 >> 1) - 1 + pc;
  }
}

// 16-byte direct global->LDS load (global_load_lds_dwordx4): lane l of the
// wave writes LDS address lds_wave_base + 16 l.  lds_wave_base must be uniform.
__device__ __forceinline__ void lds_dma16(const uint4* g, uint4* lds_wave_base) {
  __builtin_amdgcn_global_load_lds(g, lds_wave_base, 16, 0, 0);
}

// The same through a buffer resource: base and size in scalar registers, one
// 32-bit byte offset per lane (offsets past the size read zeros).  Needs no
// per-slot 64-bit addresses, which register-tight kernels otherwise keep in
// spill slots and reload, each reload waiting for the transfers in flight.
__device__ __forceinline__ void lds_dma16_buf(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint4* lds_wave_base) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)lds_wave_base, 16, voff, 0, 0, 0);
}

template <int PREC>
__device__ __forceinline__ void mfma_quad(f32x4& acc, const uint4& wq, const uint4& aq) {
  if constexpr (PREC == P_BF16) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, wq),
                                                  __builtin_bit_cast(bf16x8, aq), acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(wq.x), __uint_as_float(aq.x), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(wq.y), __uint_as_float(aq.y), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(wq.z), __uint_as_float(aq.z), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(wq.w), __uint_as_float(aq.w), acc, 0, 0, 0);
  }
}

// Operands of the K = 128 fp8 MFMA.  Lane group g (lanes 16 g .. 16 g + 15)
// holds 32 bytes per row / column; the hardware applies E8M0 scale block s
// (the byte supplied by lane 16 s + row / column) to bytes 0-15 (s = 0, 1) or
// 16-31 (s = 2, 3) of lane groups 0 and 1 (even s) or 2 and 3 (odd s).  With
// two taps x 64 channels per MFMA, lane group g takes tap g >> 1 and, so that
// every scale block is one tap's 32-channel block, the channel quads h and
// 2 + h (h = g & 1) of its 64-channel row: block s then covers channels
// 32 (s >> 1) .. + 31 of tap s & 1.
__device__ __forceinline__ i32x8 ld_fp8_pair(const uint4* base, int row, int h) {
  const uint4 q0 = base[row * 4 + (h ^ swz(row))];
  const uint4 q1 = base[row * 4 + ((2 + h) ^ swz(row))];
  return i32x8{(int)q0.x, (int)q0.y, (int)q0.z, (int)q0.w, (int)q1.x, (int)q1.y, (int)q1.z, (int)q1.w};
}

// D += A x B on e4m3 operands with K = 128: A (weights) unscaled, B
// (activations) scaled by the E8M0 bytes sb (this lane's scale block).
__device__ __forceinline__ void mfma_fp8(f32x4& acc, const i32x8& w, const i32x8& x, int sb) {
  acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(w, x, acc, 0, 0, 0, 127, 0, sb);
}

// The K = 64 (one tap x 64 channels) fp8 MFMA, 32 x 32 output (measured with
// an in-bounds probe): lane l holds row / column l % 32 and 32 bytes of K; the
// E8M0 scale of lane half h = l / 32 covers bytes 16 h .. 16 h + 15 of both
// halves' lanes of that row / column; D register r of lane l is
// D[8 (r / 4) + 4 h + r % 4][l % 32].  With ld_fp8_pair (lane half h takes
// channel quads h and 2 + h) the scale of half h covers channels 32 h .. + 31,
// i.e. exactly one MX block.
typedef __attribute__((ext_vector_type(16))) float f32x16;
__device__ __forceinline__ void mfma_fp8_32(f32x16& acc, const i32x8& w, const i32x8& x, int sb) {
  acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(w, x, acc, 0, 0, 0, 127, 0, sb);
}

// Map a linear block index to a virtual tile index so that the blocks one XCD
// receives (hardware dispatches block b to XCD b % 8) are contiguous tiles.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, l = b >> 3;
  return x * q + min(x, r) + l;
}

template <int PREC, int MODE, int NB, int IN_KIND, int OUT_KIND, bool RESID, bool STATS>
__global__ void __launch_bounds__(kThreads, (MODE == CM_I2C && PREC == P_BF16) ? kI2cOcc
                                           : (MODE == CM_S1 && OUT_KIND == OUT_RGB32 && PREC != P_FP8) ? 3 : 2)
    conv3d_kernel(ConvLaunch a) {
  using G = Geo<MODE>;
  using O = Op<PREC>;
  constexpr bool F8 = PREC == P_FP8;
  constexpr int OPREC = F8 ? P_BF16 : PREC;  // precision of OUT_ACT stores and of the residual
  using OO = Op<OPREC>;
  constexpr int NT = NB * 16;           // output channels per workgroup
  constexpr int HALO = G::HH * G::HW;   // halo rows (positions)
  constexpr int MB = G::MB;             // position blocks per wave
  constexpr int HQ = HALO * 4;          // halo quads per stage
  constexpr int WQ = G::WT * NT * 4;    // weight quads per stage
  constexpr int NBUF = 1;               // LDS buffers (two workgroups per CU overlap staging and compute)
  static_assert(WQ % 64 == 0, "weight stage must be whole waves");
  static_assert(!F8 || IN_KIND == IN_ACT, "fp8: activations in");
  static_assert(OUT_KIND != OUT_FP8 || (F8 && !STATS && NB == 4), "fp8 output: fp8 kernels, no statistics");
  constexpr int SCN = F8 ? HALO : 1;      // fp8: two E8M0 bytes per halo row

  constexpr int PXN = MODE == CM_I2C ? 3 * (G::TH + 2) * (G::TW + 2) * 4 : 1;  // normalised pixel halo
  static_assert(MODE != CM_I2C || (IN_KIND == IN_U8 && !F8), "im2col: uint8 input");

  // 64 -> 3 last layer (bf16 / fp32): rows-as-taps path below, weights staged compactly
  constexpr bool RGBL = !F8 && MODE == CM_S1 && OUT_KIND == OUT_RGB32;
  constexpr int WQR = 27 * 4;  // its weight quads per stage: 9 taps x 3 colours x 4 quads
  __shared__ uint4 lds_a[NBUF][HQ];
  __shared__ uint4 lds_w[NBUF][RGBL ? 128 : WQ];
  __shared__ uint16_t lds_sc[SCN];
  // im2col pixel tile: fp32 values, or for bf16 their bf16 bits (4 channels =
  // 8 bytes a pixel, so an operand half is one 8-byte read, no conversion)
  constexpr bool PXH16 = MODE == CM_I2C && PREC == P_BF16;
  __shared__ __align__(16) float lds_px[PXH16 ? 1 : PXN];
  __shared__ __align__(16) uint16_t lds_pxh[PXH16 ? PXN : 1];
  __shared__ float lds_lut[MODE == CM_I2C ? 256 : 1];
  constexpr int WQI = MODE == CM_I2C ? NT * 4 * (kI2cK / O::CH) : 1;  // im2col: every stage's weights
  __shared__ uint4 lds_wi[WQI];
  __shared__ float red[kWaves][32];
  __shared__ float gmean[32];
  __shared__ float lds_bias[NT];
  __shared__ float lds_wsc[F8 ? NT : 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int l16 = lane & 15;
  const int g4 = lane >> 4;

  // ---- tile coordinates -------------------------------------------------
  const int nblocks = gridDim.x;
  int v = xcd_remap(blockIdx.x, nblocks);
  const int ct = v % a.cout_tiles; v /= a.cout_tiles;
  const int to = v % a.To; v /= a.To;
  const int tw = v % a.tiles_w; v /= a.tiles_w;
  const int th = v % a.tiles_h; v /= a.tiles_h;
  const int n = v;
  const int h0 = th * G::TH, w0 = tw * G::TW;

  // This tile's per-channel bias (fp8: and weight scale) in LDS.  The
  // epilogue reads them between its output stores; global reads there would
  // each wait for the preceding stores (the output is not known not to alias).
  if (tid < NT) {
    const int c = ct * NT + tid;
    lds_bias[tid] = c < a.Cout ? a.bias[c] : 0.f;
    if constexpr (F8) lds_wsc[tid] = c < a.Cout ? a.wscale[c] : 0.f;
  }
  __syncthreads();

  f32x4 acc[MB][NB];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[m][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  const size_t plane_in = (size_t)a.Hi * a.Wi;
  // Folded weights come in two sets, one per output-frame parity.
  const int tg = a.go0 + to;  // global output frame
  // Folded weight sets: per output-frame parity (CM_UPF); frame 0 vs later frames (CM_S1T).
  size_t wset = ct;
  if constexpr (MODE == CM_UPF) wset = (size_t)ct * 2 + (tg & 1);
  if constexpr (MODE == CM_S1T) wset = (size_t)ct * 2 + (tg == 0 ? 1 : 0);
  // stride-2 adjoint: output frame 0 (causal clamp), even, odd output frames
  if constexpr (MODE == CM_S2T) wset = (size_t)ct * 3 + (tg == 0 ? 0 : ((tg & 1) ? 2 : 1));
  // upsampling adjoint: source frame 0 (causal clamp) vs later frames
  if constexpr (MODE == CM_UPT) wset = (size_t)ct * 2 + (tg == 0 ? 0 : 1);
  const uint4* wbase = reinterpret_cast<const uint4*>(a.wpk) + wset * G::KTS * a.in_chunks * WQ;
  constexpr int KHS = MODE == CM_S2 ? 3 : 1;  // stride 2: one stage per kernel row
  const int spk = a.in_chunks * KHS;          // stages per temporal tap
  const int nstages = G::KTS * spk;           // stage = (temporal tap, input chunk[, kernel row])
  // Order of the temporal taps: the blocks of neighbouring output frames run
  // side by side (output frame is the fastest tile index after the channel
  // tile), so each block takes its taps in an order in which neighbours read
  // the same input frame in the same step and the second read is served by
  // L2.  Stride 1: step j reads the input frame congruent to j mod 3 (shared
  // by three neighbours); stride 2: even / odd output frames take taps
  // (2, 0, 1) / (0, 2, 1) (frame 2t shared by t, t + 1 in step 0, frame 2t + 2
  // by t + 1, t + 2 in step 1); upsampling: even / odd output frames (1, 0) /
  // (0, 1) (source frame j shared by 2j, 2j + 1 in step 0).  The order
  // depends on the global output frame only, so chunked and whole-clip runs
  // still sum in the same order.
  auto stage_of = [&](int j) {
    const int jt = j / spk, ck = j - jt * spk;  // (ck: chunk and kernel row)
    int kt = jt;
    if constexpr (MODE == CM_S1) kt = (jt + 5 - tg % 3) % 3;
    else if constexpr (MODE == CM_S1T) kt = (jt + 3 - tg % 3) % 3;
    else if constexpr (MODE == CM_S2) kt = jt == 2 ? 1 : ((tg & 1) ? 2 * jt : 2 - 2 * jt);
    else if constexpr (MODE == CM_UPF) kt = (tg & 1) ? jt : 1 - jt;
    else if constexpr (MODE == CM_S2T) kt = (tg & 1) ? jt : 1 - jt;  // frame j + 1 shared by 2 j, 2 j + 1 in step 0
    else if constexpr (MODE == CM_UPT) kt = (tg & 1) ? jt : (jt + 2) & 3;  // fine frames 2 s + 1, 2 s + 2 shared with s + 1
    return kt * spk + ck;
  };

  // Input buffer frame read by temporal tap kt (causal in global frame
  // numbers: frame 0 repeats for t < 0).
  auto src_frame = [&](int kt) {
    int g;
    if constexpr (MODE == CM_S1) g = max(tg + kt - 2, 0);
    else if constexpr (MODE == CM_S1T) g = tg + kt;  // gradient frames t, t+1, t+2 (past the end: none)
    else if constexpr (MODE == CM_S2T) {
      // output frame 2 j reads gradient frames j (forward tap 2) and j + 1 (tap 0), frame 2 j + 1 frame
      // j + 1 (tap 1) only; its second stage has no taps (reported as past the end)
      const int jt = tg >> 1;
      g = (tg & 1) ? (kt == 0 ? jt + 1 : a.gi0 + a.Ti) : jt + kt;
    }
    else if constexpr (MODE == CM_S2) g = max(2 * tg + kt - 2, 0);
    else if constexpr (MODE == CM_UPT) {
      // source frame s reads fine gradient frames 2 s - 1 .. 2 s + 2 (frame -1: none, reported as past the end)
      g = 2 * tg - 1 + kt;
      if (g < 0) g = a.gi0 + a.Ti;
    }
    else {
      // even output frame 2j reads source frames j-1 (clamped) and j; odd 2j+1 reads j and j+1
      const int jt = tg >> 1;
      g = (tg & 1) ? jt + kt : max(jt - 1 + kt, 0);
    }
    return g - a.gi0;
  };

  // Halo slots this thread's lanes fill are the same in every stage: keep
  // their in-frame quad offsets (or -1 for the zero padding) in registers.
  // Stride 2: the offset for kernel row 0 (kernel row kh reads kh rows
  // further down) and a mask of the kernel rows whose source row is inside
  // the frame.
  constexpr int NHS = (HQ + kThreads - 1) / kThreads;
  int hoff[NHS];
  int hmask[MODE == CM_S2 ? NHS : 1];
#pragma unroll
  for (int k = 0; k < NHS; ++k) {
    const int e = wave * 64 + k * kThreads + lane;
    hoff[k] = -1;
    if constexpr (MODE == CM_S2) hmask[k] = 0;
    if (e < HQ) {
      const int p = e >> 2;
      const int q = (e & 3) ^ swz(p);
      int hs, ws;
      halo_src<MODE>(p, h0, w0, &hs, &ws);
      if constexpr (MODE == CM_S2) {
        hoff[k] = (hs * a.Wi + ws) * 4 + q;
#pragma unroll
        for (int kh = 0; kh < 3; ++kh)
          if (hs + kh >= 0 && hs + kh < a.Hi && ws >= 0 && ws < a.Wi) hmask[k] |= 1 << kh;
      } else if (hs >= 0 && hs < a.Hi && ws >= 0 && ws < a.Wi) {
        hoff[k] = (hs * a.Wi + ws) * 4 + q;
      }
    }
  }
  // fp8: in-frame position of halo rows tid, tid + 256, ... (scale staging), -1 outside
  constexpr int NSR = F8 ? (HALO + kThreads - 1) / kThreads : 1;
  int soff[NSR];
#pragma unroll
  for (int k = 0; k < NSR; ++k) {
    soff[k] = -1;
    const int p = tid + k * kThreads;
    if (F8 && p < HALO) {
      int hs, ws;
      halo_src<MODE>(p, h0, w0, &hs, &ws);
      if (hs >= 0 && hs < a.Hi && ws >= 0 && ws < a.Wi) soff[k] = hs * a.Wi + ws;
    }
  }

  // Issue the global->LDS transfers of stage st into buffer buf: the 9 taps of
  // packed weights and the spatial halo, both as direct-to-LDS loads (lane l
  // of a wave writes 16 bytes at the wave's LDS base + 16 l).  Slot (p, pq) of
  // the halo holds logical quad pq ^ swz(p) of halo row p; rows outside the
  // frame are written as zeros (the conv's zero padding).
  auto issue_async = [&](int st, int buf) {
    // stage st = (kt, chunk ck[, kernel row kh]); its weights follow the
    // previous stage's in the packed layout (stride 2: a kernel row's 3 taps)
    const int kt = st / spk, ck = (st - kt * spk) / KHS, kh = st % KHS;
    const uint4* wsrc = wbase + (size_t)st * WQ;
    if constexpr (RGBL) {
      // compact: row 3 tap + c of LDS <- packed row 16 tap + c (quads as packed, i.e. swizzled by the packed row)
      const int e = wave * 64 + lane;
      if (wave < 2 && e < WQR) {
        const int r = e >> 2;
        lds_dma16(wsrc + ((r / 3) * NT + r % 3) * 4 + (e & 3), &lds_w[buf][wave * 64]);
      }
    } else {
#pragma unroll
      for (int base = wave * 64; base < WQ; base += kThreads) lds_dma16(wsrc + base + lane, &lds_w[buf][base]);
    }
    const uint4* src = reinterpret_cast<const uint4*>(a.in) +
                       (((size_t)n * a.Ti + src_frame(kt)) * a.in_chunks + ck) * plane_in * 4;
#pragma unroll
    for (int k = 0; k < NHS; ++k) {
      const int base = wave * 64 + k * kThreads;
      const int e = base + lane;
      if (e < HQ) {
        if constexpr (MODE == CM_S2) {
          if ((hmask[k] >> kh) & 1) lds_dma16(src + hoff[k] + kh * a.Wi * 4, &lds_a[buf][base]);
          else lds_a[buf][e] = make_uint4(0, 0, 0, 0);
        } else {
          if (hoff[k] >= 0) lds_dma16(src + hoff[k], &lds_a[buf][base]);
          else lds_a[buf][e] = make_uint4(0, 0, 0, 0);
        }
      }
    }
    if constexpr (F8) {
      // scale bytes of the halo rows (rows outside the frame: zeros with scale 2^0)
      const uint16_t* ssrc = reinterpret_cast<const uint16_t*>(a.in_scale) +
                             (((size_t)n * a.Ti + src_frame(kt)) * a.in_chunks + ck) * plane_in;
#pragma unroll
      for (int k = 0; k < NSR; ++k) {
        const int p = tid + k * kThreads;
        if (p < HALO) lds_sc[p] = soff[k] >= 0 ? ssrc[soff[k]] : (uint16_t)0x7F7F;
      }
    }
  };

  // im2col first layer.  Once per tile: the 3 causal input frames' pixel
  // halos (TH+2 x TW+2), normalised to x/127.5 - 1 (0 outside the frame), as
  // floats [frame][row][col][4].  Per stage (K chunk): weights by direct
  // load; each thread writes quad (tid & 3) of rows (tid >> 2) + 64 u, i.e.
  // QE consecutive K entries k = (kt*9 + kh*3 + kw)*3 + c of one position.
  constexpr int PXW = G::TW + 2, PXH = G::TH + 2;
  auto stage_px = [&]() {
    // The 3 x PXH row segments of PXW pixels (3 bytes each).  Thread t loads
    // dwords t, t + 256, ... of the segments' 4-byte-aligned byte ranges with
    // buffer loads over the pixel tensor (bytes before its start or past its
    // end read as zeros), all issued before the first is used; the bytes are
    // then normalised through a 256-entry table of x/127.5 - 1.
    constexpr int SEG = PXW * 3, NSEG = 3 * PXH, DWS = (SEG + 6) / 4, NDW = NSEG * DWS;
    constexpr int K = (NDW + kThreads - 1) / kThreads;
    lds_lut[tid] = (float)tid / 127.5f - 1.0f;  // (bf16: read back rounded to nearest even)
    const uint32_t nbytes = (uint32_t)((size_t)a.N * a.Ti * a.Hi * a.Wi * 3);  // < 2^31, checked on the host
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(a.in), (short)0, (int)nbytes, 0x00020000);
    uint32_t vw[K];
    long long sstart[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int d = tid + k * kThreads;
      const int seg = d / DWS, dw = d - seg * DWS;
      const int f = seg / PXH, r = seg - f * PXH;
      const int hs = h0 - 1 + r;
      const int g = max(a.go0 + to + f - 2, 0) - a.gi0;  // causal clamp of the input frame
      sstart[k] = ((((long long)n * a.Ti + g) * a.Hi + hs) * a.Wi + (w0 - 1)) * 3;
      const uint32_t off = (uint32_t)((sstart[k] & ~3LL) + 4 * dw);  // a negative start wraps past the end: zeros
      vw[k] = 0u;
      if (d < NDW && hs >= 0 && hs < a.Hi) vw[k] = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0);
    }
    __syncthreads();  // the table
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int d = tid + k * kThreads;
      if (d >= NDW) continue;
      const int seg = d / DWS, dw = d - seg * DWS;
      const int hs = h0 - 1 + (seg - (seg / PXH) * PXH);
      const bool row_ok = hs >= 0 && hs < a.Hi;
      const int shift = (int)(sstart[k] & 3);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int rel = 4 * dw + j - shift;  // byte of the segment
        if (rel < 0 || rel >= SEG) continue;
        const int c = rel / 3, ch = rel - 3 * c;
        const int ws = w0 - 1 + c;
        const bool ok = row_ok && ws >= 0 && ws < a.Wi;
        const float v = ok ? lds_lut[(vw[k] >> (8 * j)) & 255u] : 0.f;
        if constexpr (PXH16) lds_pxh[(seg * PXW + c) * 4 + ch] = (uint16_t)(pack_bf16(v, 0.f) & 0xffffu);
        else lds_px[(seg * PXW + c) * 4 + ch] = v;
      }
    }
    for (int p = tid; p < 3 * PXH * PXW; p += kThreads) {  // the 4th (zero) channel
      if constexpr (PXH16) lds_pxh[p * 4 + 3] = 0;
      else lds_px[p * 4 + 3] = 0.f;
    }
  };
  // The 9 spatial taps of one stage: every wave multiplies its MB position
  // blocks by the NB output-channel blocks.
  auto compute = [&](int buf) {
    if constexpr (F8) {
      // K = 128 per MFMA = two taps x 64 channels (see ld_fp8_pair): data of
      // tap 2 pr + (g4 >> 1), channel quads h, 2 + h; the scale this lane
      // supplies is that of tap 2 pr + (g4 & 1), 32-channel block g4 >> 1.
      const int h = g4 & 1, sblk = g4 >> 1;
      if constexpr (MODE == CM_UPF || MODE == CM_S2T) {
        const int ph = wave >> 1, pw = wave & 1;
#pragma unroll 1
        for (int pr = 0; pr < 2; ++pr) {
          const int tap = 2 * pr + (g4 >> 1), stap = 2 * pr + h;
          const int dh = tap >> 1, dw = tap & 1, sdh = stap >> 1, sdw = stap & 1;
          i32x8 wq[NB];
#pragma unroll
          for (int b = 0; b < NB; ++b) wq[b] = ld_fp8_pair(lds_w[buf], (wave * 4 + tap) * NT + b * 16 + l16, h);
#pragma unroll
          for (int m = 0; m < MB; ++m) {
            const int row = ((m >> 1) + dh + ph) * G::HW + ((m & 1) * 16 + l16 + dw + pw);
            const int srow = ((m >> 1) + sdh + ph) * G::HW + ((m & 1) * 16 + l16 + sdw + pw);
            const i32x8 aq = ld_fp8_pair(lds_a[buf], row, h);
            const int sb = (lds_sc[srow] >> (8 * sblk)) & 255;
#pragma unroll
            for (int b = 0; b < NB; ++b) mfma_fp8(acc[m][b], wq[b], aq, sb);
          }
        }
      } else {
#pragma unroll 1
        for (int pr = 0; pr < 5; ++pr) {
          const int tp = 2 * pr + (g4 >> 1);
          const bool tv = tp < 9;  // the 10th "tap" has zero weights (its data and scale: tap 8's)
          const int tap = tv ? tp : 8, stap = min(2 * pr + h, 8);
          const int kh = tap / 3, kw = tap % 3, skh = stap / 3, skw = stap % 3;
          i32x8 wq[NB];
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            wq[b] = ld_fp8_pair(lds_w[buf], tap * NT + b * 16 + l16, h);
            if (!tv) wq[b] = i32x8{0, 0, 0, 0, 0, 0, 0, 0};
          }
#pragma unroll
          for (int m = 0; m < MB; ++m) {
            int i, j;
            out_local<MODE>(wave, m, l16, &i, &j);
            const i32x8 aq = ld_fp8_pair(lds_a[buf], act_row<MODE>(i, j, kh, kw), h);
            const int sb = (lds_sc[act_row<MODE>(i, j, skh, skw)] >> (8 * sblk)) & 255;
#pragma unroll
            for (int b = 0; b < NB; ++b) mfma_fp8(acc[m][b], wq[b], aq, sb);
          }
        }
      }
      return;
    }
    if constexpr (MODE == CM_UPF || MODE == CM_S2T) {
      const int ph = wave >> 1, pw = wave & 1;
#pragma unroll
      for (int tap = 0; tap < 4; ++tap) {
        const int dh = tap >> 1, dw = tap & 1;
        uint4 wq[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int row = (wave * 4 + tap) * NT + b * 16 + l16;
          wq[b] = lds_w[buf][row * 4 + (g4 ^ swz(row))];
        }
#pragma unroll
        for (int m = 0; m < MB; ++m) {
          const int row = ((m >> 1) + dh + ph) * G::HW + ((m & 1) * 16 + l16 + dw + pw);
          const uint4 aq = lds_a[buf][row * 4 + (g4 ^ swz(row))];
#pragma unroll
          for (int b = 0; b < NB; ++b) mfma_quad<PREC>(acc[m][b], wq[b], aq);
        }
      }
      return;
    }
    if constexpr (MODE == CM_S1 || MODE == CM_S1T) {
      // per kw: the 6 halo rows x 2 column blocks this wave reads, reused for kh = 0, 1, 2
      static_assert(MB == 8, "4 x 32 wave tile");
      const int i0 = 4 * (wave >> 1), j0 = 32 * (wave & 1) + l16;
#pragma unroll 1
      for (int kw = 0; kw < 3; ++kw) {
        uint4 bq[6][2];
#pragma unroll
        for (int hr = 0; hr < 6; ++hr)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) {
            const int row = (i0 + hr) * G::HW + j0 + 16 * cb + kw;
            bq[hr][cb] = lds_a[buf][row * 4 + (g4 ^ swz(row))];
          }
#pragma unroll
        for (int kh = 0; kh < 3; ++kh) {
          uint4 wq[NB];
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const int row = (kh * 3 + kw) * NT + b * 16 + l16;
            wq[b] = lds_w[buf][row * 4 + (g4 ^ swz(row))];
          }
#pragma unroll
          for (int m = 0; m < MB; ++m) {
#pragma unroll
            for (int b = 0; b < NB; ++b) mfma_quad<PREC>(acc[m][b], wq[b], bq[(m >> 1) + kh][m & 1]);
          }
        }
      }
      return;
    }
    constexpr int BPR = G::TW / 16;
    if constexpr (MODE == CM_S2) {
      // the stage's kernel row: halo row i serves output row i, column 2 j + kw
#pragma unroll
      for (int kw = 0; kw < 3; ++kw) {
        uint4 wq[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int row = kw * NT + b * 16 + l16;
          wq[b] = lds_w[buf][row * 4 + (g4 ^ swz(row))];
        }
#pragma unroll
        for (int m = 0; m < MB; ++m) {
          const int i = wave * G::WR + m / BPR;
          const int c = 2 * ((m % BPR) * 16 + l16) + kw;
          const int row = i * G::HW + (c & 1) * (G::TW + 1) + (c >> 1);
          const uint4 aq = lds_a[buf][row * 4 + (g4 ^ swz(row))];
#pragma unroll
          for (int b = 0; b < NB; ++b) mfma_quad<PREC>(acc[m][b], wq[b], aq);
        }
      }
      return;
    }
    constexpr int KD = MODE == CM_UPT ? 4 : 3;  // spatial taps per dimension
#pragma unroll 1
    for (int kh = 0; kh < KD; ++kh) {
#pragma unroll
      for (int kw = 0; kw < KD; ++kw) {
        const int tap = kh * KD + kw;
        uint4 wq[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int row = tap * NT + b * 16 + l16;
          wq[b] = lds_w[buf][row * 4 + (g4 ^ swz(row))];
        }
#pragma unroll
        for (int m = 0; m < MB; ++m) {
          const int i = wave * G::WR + m / BPR;
          const int j = (m % BPR) * 16 + l16;
          const int row = act_row<MODE>(i, j, kh, kw);
          const uint4 aq = lds_a[buf][row * 4 + (g4 ^ swz(row))];
#pragma unroll
          for (int b = 0; b < NB; ++b) mfma_quad<PREC>(acc[m][b], wq[b], aq);
        }
      }
    }
  };

  // im2col first layer: K chunk st of a position is taps (st CH + 4 v) / 4 ..,
  // 4 channels each (the 4th zero); a lane's operand quad is read straight
  // from the normalised pixel tile (one 16-byte read per tap) and converted.
  auto compute_i2c = [&](int st) {
    constexpr int QE = O::QE, TPQ = QE / 4;
    uint4 wq[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int row = b * 16 + l16;
      wq[b] = lds_wi[st * WQ + row * 4 + (g4 ^ swz(row))];
    }
    int off[TPQ];
#pragma unroll
    for (int x = 0; x < TPQ; ++x) {
      const int tap = (st * O::CH + g4 * QE) / 4 + x;
      const int kt = tap / 9, kh = (tap / 3) % 3, kw = tap % 3;
      off[x] = tap < 27 ? ((kt * PXH + kh) * PXW + kw) * 4 : -1;
    }
    if constexpr (PXH16) {
      // this lane's 8 K entries = 2 taps x 4 channels = two 8-byte pixel reads
      static_assert(TPQ == 2, "bf16: two taps per operand");
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        int i, j;
        out_local<MODE>(wave, m, l16, &i, &j);
        const int base = (i * PXW + j) * 4;
        uint2 p0 = *reinterpret_cast<const uint2*>(&lds_pxh[base + max(off[0], 0)]);
        uint2 p1 = *reinterpret_cast<const uint2*>(&lds_pxh[base + max(off[1], 0)]);
        if (off[0] < 0) p0 = make_uint2(0, 0);  // K padding past tap 26
        if (off[1] < 0) p1 = make_uint2(0, 0);
        const uint4 aq = make_uint4(p0.x, p0.y, p1.x, p1.y);
#pragma unroll
        for (int b = 0; b < NB; ++b) mfma_quad<PREC>(acc[m][b], wq[b], aq);
      }
      return;
    }
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      int i, j;
      out_local<MODE>(wave, m, l16, &i, &j);
      const int base = (i * PXW + j) * 4;
      float v[QE];
#pragma unroll
      for (int x = 0; x < TPQ; ++x) {
        const float4 t4 = off[x] >= 0 ? *reinterpret_cast<const float4*>(&lds_px[base + off[x]])
                                      : make_float4(0.f, 0.f, 0.f, 0.f);
        v[4 * x] = t4.x;
        v[4 * x + 1] = t4.y;
        v[4 * x + 2] = t4.z;
        v[4 * x + 3] = t4.w;
      }
      uint4 aq;
      if constexpr (PREC == P_BF16)
        aq = make_uint4(pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3]), pack_bf16(v[4], v[5]), pack_bf16(v[6], v[7]));
      else
        aq = make_uint4(__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]), __float_as_uint(v[3]));
#pragma unroll
      for (int b = 0; b < NB; ++b) mfma_quad<PREC>(acc[m][b], wq[b], aq);
    }
  };

  // fp8 stride-1 64-channel convs: 32 x 32 x 64 MFMAs, one tap per
  // instruction.  Wave tile 4 rows x 32 columns: position block m = output
  // row i0 + m (32 positions), channel block c = 32 output channels.  Per kw
  // the wave loads halo rows i0 .. i0 + 5 once and reuses them for kh = 0..2
  // (output row m reads halo row m + kh).
  constexpr bool F8W = F8 && MODE == CM_S1 && NB == 4;
  if constexpr (F8W) {
    f32x16 a32[4][2];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) a32[m][c][r] = 0.f;
    const int hh = lane >> 5, p32 = lane & 31;
    const int i0 = 4 * (wave >> 1), j0 = 32 * (wave & 1) + p32;
    for (int st = 0; st < nstages; ++st) {
      __syncthreads();
      issue_async(stage_of(st), 0);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
#pragma unroll 1
      for (int kw = 0; kw < 3; ++kw) {
        i32x8 bq[6];
        int sq[6];
#pragma unroll
        for (int hr = 0; hr < 6; ++hr) {
          const int row = (i0 + hr) * G::HW + j0 + kw;
          bq[hr] = ld_fp8_pair(lds_a[0], row, hh);
          sq[hr] = (lds_sc[row] >> (8 * hh)) & 255;
        }
#pragma unroll
        for (int kh = 0; kh < 3; ++kh) {
          i32x8 wq[2];
#pragma unroll
          for (int c = 0; c < 2; ++c) wq[c] = ld_fp8_pair(lds_w[0], (kh * 3 + kw) * NT + c * 32 + p32, hh);
#pragma unroll
          for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int c = 0; c < 2; ++c) mfma_fp8_32(a32[m][c], wq[c], bq[m + kh], sq[m + kh]);
        }
      }
    }
    // ---- epilogue of the 32 x 32 layout: value r of (m, c) is channel
    // ct NT + 32 c + 8 (r / 4) + 4 hh + r % 4 at position (i0 + m, j0)
    const size_t plane_out = (size_t)a.Ho * a.Wo;
    const int ow = w0 + j0;
    if constexpr (OUT_KIND == OUT_FP8) {
      const int res_chunks = a.Cout / OO::CH;
      const size_t frame = (size_t)n * a.To_buf + a.out_f0 + to;
      // every residual value of this lane, loaded before the first store and
      // without branches (positions past the frame edge read a clamped,
      // in-frame address; their values are never stored)
      uint2 rres[RESID ? 4 : 1][2][4];
      if constexpr (RESID) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const size_t pos = (size_t)min(h0 + i0 + m, a.Ho - 1) * a.Wo + min(ow, a.Wo - 1);
#pragma unroll
          for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int c0 = ct * NT + 32 * c + 8 * q + 4 * hh;
              rres[m][c][q] = *reinterpret_cast<const uint2*>(
                  reinterpret_cast<const char*>(a.resid) +
                  ((frame * res_chunks + c0 / OO::CH) * plane_out + pos) * kChunkBytes + (c0 % OO::CH) * 2);
            }
        }
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int oh = h0 + i0 + m;
        const bool valid = (oh < a.Ho) && (ow < a.Wo);
        const size_t pos = (size_t)oh * a.Wo + ow;
        float v[2][16];
        float am[2] = {0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int lc = 32 * c + 8 * q + 4 * hh;
#pragma unroll
            for (int r = 0; r < 4; ++r) v[c][4 * q + r] = a32[m][c][4 * q + r] * lds_wsc[lc + r] + lds_bias[lc + r];
            if constexpr (RESID) {
              const uint2 rv = rres[m][c][q];
              v[c][4 * q] += bf16_lo(rv.x); v[c][4 * q + 1] += bf16_hi(rv.x);
              v[c][4 * q + 2] += bf16_lo(rv.y); v[c][4 * q + 3] += bf16_hi(rv.y);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) am[c] = fmaxf(am[c], fabsf(v[c][4 * q + r]));
          }
#pragma unroll
        for (int c = 0; c < 2; ++c) am[c] = fmaxf(am[c], __shfl_xor(am[c], 32));
        const int e0 = fp8_block_exp(am[0]), e1 = fp8_block_exp(am[1]);
        if (valid) {
          char* orow = reinterpret_cast<char*>(a.out) + ((frame * a.out_chunks + ct) * plane_out + pos) * kChunkBytes;
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const float f = ldexpf(1.0f, -(c == 0 ? e0 : e1));
#pragma unroll
            for (int q = 0; q < 4; ++q)
              *reinterpret_cast<uint32_t*>(orow + 32 * c + 8 * q + 4 * hh) =
                  pack_fp8x4(v[c][4 * q] * f, v[c][4 * q + 1] * f, v[c][4 * q + 2] * f, v[c][4 * q + 3] * f);
          }
          if (hh == 0)
            reinterpret_cast<uint16_t*>(a.out_scale)[(frame * a.out_chunks + ct) * plane_out + pos] =
                (uint16_t)((e0 + 127) | ((e1 + 127) << 8));
        }
      }
      return;
    } else {
      static_assert(OUT_KIND == OUT_ACT && OPREC == P_BF16, "fp8 convs store bf16 or fp8 activations");
      // group g = channel / 2 of the 32 GroupNorm groups; this lane's items
      // (c, q) hold groups 16 c + 4 q + 2 hh and + 1
      float s_lo[8], s_hi[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) s_lo[k] = s_hi[k] = 0.f;
      auto out_off = [&](int oh, int owp, int c, int q) {
        const int c0 = ct * NT + 32 * c + 8 * q + 4 * hh;
        const int chunk = c0 / OO::CH, within = c0 % OO::CH;
        return (((size_t)n * a.To_buf + a.out_f0 + to) * a.out_chunks + chunk) * plane_out * kChunkBytes +
               ((size_t)oh * a.Wo + owp) * kChunkBytes + (size_t)within * 2;
      };
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int oh = h0 + i0 + m;
        const bool valid = (oh < a.Ho) && (ow < a.Wo);
        // the row's residual values, loaded before its first store (one row
        // at a time: the statistics keep every output value in registers),
        // without branches: past the frame edge from a clamped in-frame address
        uint2 rres[2][4];
        if constexpr (RESID) {
#pragma unroll
          for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              rres[c][q] = *reinterpret_cast<const uint2*>(reinterpret_cast<const char*>(a.resid) +
                                                           out_off(min(oh, a.Ho - 1), min(ow, a.Wo - 1), c, q));
        }
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int lc = 32 * c + 8 * q + 4 * hh;
            float v4[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) v4[r] = a32[m][c][4 * q + r] * lds_wsc[lc + r] + lds_bias[lc + r];
            const size_t off = out_off(oh, ow, c, q);
            if (valid) {
              if constexpr (RESID) {
                const uint2 rv = rres[c][q];
                v4[0] += bf16_lo(rv.x); v4[1] += bf16_hi(rv.x);
                v4[2] += bf16_lo(rv.y); v4[3] += bf16_hi(rv.y);
              }
              const uint2 pv = make_uint2(pack_bf16(v4[0], v4[1]), pack_bf16(v4[2], v4[3]));
              *reinterpret_cast<uint2*>(reinterpret_cast<char*>(a.out) + off) = pv;
              v4[0] = bf16_lo(pv.x); v4[1] = bf16_hi(pv.x); v4[2] = bf16_lo(pv.y); v4[3] = bf16_hi(pv.y);
            }
            if constexpr (STATS) {
#pragma unroll
              for (int r = 0; r < 4; ++r) a32[m][c][4 * q + r] = valid ? v4[r] : 0.f;  // keep final values
              if (valid) {
                s_lo[4 * c + q] += v4[0] + v4[1];
                s_hi[4 * c + q] += v4[2] + v4[3];
              }
            }
          }
      }
      if constexpr (STATS) {
        const int vr = min(G::TH, a.Ho - h0), vc = min(G::TW, a.Wo - w0);
        const float cnt = 2.0f * (float)(vr * vc);
        // Group sums through LDS (the K loop's halo buffer): lane (wave, hh,
        // p32) puts its partials of groups 16 c + 4 q + 2 hh (+1) at row g,
        // column 32 wave + p32 (rows 136 floats apart, so that the readers
        // below hit distinct banks); thread t then adds 16 values of row t / 8
        // and three shuffles finish the row.  Fixed order: deterministic.
        float* red2 = reinterpret_cast<float*>(&lds_a[0][0]);
        static_assert(32 * 136 * 4 <= HQ * 16, "group partials fit the halo buffer");
        const int rg = tid >> 3, rp = tid & 7;
        auto row_total = [&]() {
          float t = 0.f;
#pragma unroll
          for (int u = 0; u < 16; ++u) t += red2[rg * 136 + u * 8 + rp];
          t += __shfl_xor(t, 1);
          t += __shfl_xor(t, 2);
          t += __shfl_xor(t, 4);
          return t;
        };
        __syncthreads();  // every wave is done with the K loop's LDS
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int g = 16 * (k >> 2) + 4 * (k & 3) + 2 * hh;
          red2[g * 136 + wave * 32 + p32] = s_lo[k];
          red2[(g + 1) * 136 + wave * 32 + p32] = s_hi[k];
        }
        __syncthreads();
        {
          const float t = row_total();
          if (rp == 0) gmean[rg] = t / cnt;
        }
        __syncthreads();  // gmean is set and every row is read
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int c = k >> 2, q = k & 3;
          const int g = 16 * c + 4 * q + 2 * hh;
          const float ma = gmean[g], mb = gmean[g + 1];
          float qa = 0.f, qb = 0.f;
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            if (h0 + i0 + m < a.Ho && ow < a.Wo) {
              const float d0 = a32[m][c][4 * q] - ma, d1 = a32[m][c][4 * q + 1] - ma;
              const float d2 = a32[m][c][4 * q + 2] - mb, d3 = a32[m][c][4 * q + 3] - mb;
              qa += d0 * d0 + d1 * d1;
              qb += d2 * d2 + d3 * d3;
            }
          }
          red2[g * 136 + wave * 32 + p32] = qa;
          red2[(g + 1) * 136 + wave * 32 + p32] = qb;
        }
        __syncthreads();
        {
          const float m2 = row_total();
          if (rp == 0) {
            const int tiles = a.tiles_h * a.tiles_w;
            a.stats[(((size_t)n * a.To + to) * tiles + (size_t)th * a.tiles_w + tw) * 32 + rg] =
                make_float4(cnt, gmean[rg], m2, 0.f);
          }
        }
      }
      return;
    }
  }

  // 64 -> 3 last layer (bf16 / fp32): the MFMA rows are (spatial tap, colour)
  // pairs instead of output channels, 27 of 2 x 16 rows, and the columns are
  // the halo positions.  Every stage (temporal tap, input chunk) accumulates
  //   D[(kh, kw, c)][p] += sum_i W[c, i, kt, kh, kw] x[i, frame(kt), p]
  // so the K loop needs 2 MFMAs per 16 halo positions instead of 9 taps x one
  // 16-row block of which 3 rows are used; the epilogue then forms
  //   y[c](i, j) = b[c] + sum_{kh, kw} D[(kh, kw, c)][(i + kh, j + kw)]
  // through LDS, one kh at a time.
  constexpr bool RGB = !F8 && MODE == CM_S1 && OUT_KIND == OUT_RGB32;
  if constexpr (RGB) {
    static_assert(NB == 1 && !RESID && !STATS, "3-channel output: one 16-row weight block, no residual or statistics");
    constexpr int PB = (HALO + 15) / 16;              // halo position blocks
    constexpr int KB = (PB + kWaves - 1) / kWaves;    // per wave: blocks wave, wave + 4, ...
    f32x4 ar[KB][2];
#pragma unroll
    for (int k = 0; k < KB; ++k) ar[k][0] = ar[k][1] = f32x4{0.f, 0.f, 0.f, 0.f};
    // this lane's A rows 16 rb + l16 = 3 tap + c (rows 27..31: zero): compact LDS row r, swizzled as packed row 16 tap + c
    int wrow[2], wswz[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const int r = 16 * rb + l16;
      wrow[rb] = r < 27 ? r : -1;
      wswz[rb] = swz((r / 3) * NT + r % 3);
    }
    for (int st = 0; st < nstages; ++st) {
      __syncthreads();
      issue_async(stage_of(st), 0);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
      uint4 wq[2];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        wq[rb] = lds_w[0][max(wrow[rb], 0) * 4 + (g4 ^ wswz[rb])];
        if (wrow[rb] < 0) wq[rb] = make_uint4(0, 0, 0, 0);
      }
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        const int pb = wave + kWaves * k;
        if (pb < PB) {  // uniform per wave
          const int p = pb * 16 + l16, pc = min(p, HALO - 1);
          uint4 aq = lds_a[0][pc * 4 + (g4 ^ swz(pc))];
          if (p >= HALO) aq = make_uint4(0, 0, 0, 0);
          mfma_quad<PREC>(ar[k][0], wq[0], aq);
          mfma_quad<PREC>(ar[k][1], wq[1], aq);
        }
      }
    }
    // epilogue: thread t owns output positions t and t + 256 of the tile; D
    // rows pass through the (then free) halo buffer
    float* lds_d = reinterpret_cast<float*>(&lds_a[0][0]);
    static_assert(9 * HALO * 4 <= HQ * 16, "one kh's D rows fit the halo buffer");
    constexpr int NPOS = G::TH * G::TW / kThreads;
    float o[NPOS][3];
#pragma unroll
    for (int u = 0; u < NPOS; ++u)
#pragma unroll
      for (int c = 0; c < 3; ++c) o[u][c] = lds_bias[c];
#pragma unroll
    for (int kh = 0; kh < 3; ++kh) {
      __syncthreads();  // the K loop's / previous pass's LDS reads are done
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        const int pb = wave + kWaves * k;
        const int p = pb * 16 + l16;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int R = 16 * rb + 4 * g4 + r - 9 * kh;  // row within this kh's 9 rows (kw, c)
            if (pb < PB && p < HALO && R >= 0 && R < 9) lds_d[R * HALO + p] = ar[k][rb][r];
          }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NPOS; ++u) {
        const int pos = tid + kThreads * u, i = pos / G::TW, j = pos % G::TW;
        const float* d = lds_d + (i + kh) * G::HW + j;
#pragma unroll
        for (int kw = 0; kw < 3; ++kw)
#pragma unroll
          for (int c = 0; c < 3; ++c) o[u][c] += d[(3 * kw + c) * HALO + kw];
      }
    }
    const size_t plane_out = (size_t)a.Ho * a.Wo;
#pragma unroll
    for (int u = 0; u < NPOS; ++u) {
      const int pos = tid + kThreads * u;
      const int oh = h0 + pos / G::TW, ow = w0 + pos % G::TW;
      if (oh >= a.Ho || ow >= a.Wo) continue;
      float* op = reinterpret_cast<float*>(a.out) +
                  (((size_t)n * a.To_buf + a.out_f0 + to) * plane_out + (size_t)oh * a.Wo + ow) * 3;
      if (a.blend_prev != nullptr && tg < a.blend_n) {
        // frame i = tg + 1 of the GoP: a_i prev[Tp - n + i] + (1 - a_i) x_hat, a_i = (n - i) / n
        const float al = (float)(a.blend_n - (tg + 1)) / (float)a.blend_n, be = 1.0f - al;
        const float* pp = a.blend_prev + (((size_t)n * a.blend_Tp + (a.blend_Tp - a.blend_n + tg)) * plane_out +
                                          (size_t)oh * a.Wo + ow) * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) o[u][c] = al * pp[c] + be * o[u][c];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) op[c] = o[u][c];
    }
    return;
  }

  if constexpr (MODE == CM_I2C) {
    // pixels and all the weights once, then every K chunk without further staging
    stage_px();
#pragma unroll
    for (int base = wave * 64; base < WQI; base += kThreads) lds_dma16(wbase + base + lane, &lds_wi[base]);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    for (int st = 0; st < nstages; ++st) compute_i2c(st);
  } else {
    for (int j = 0; j < nstages; ++j) {
      const int st = stage_of(j);
      if constexpr (MODE == CM_S1T || MODE == CM_S2T || MODE == CM_UPT) {
        if (src_frame(st / a.in_chunks) >= a.Ti) continue;  // beyond the last gradient frame (uniform per block)
      }
      __syncthreads();
      issue_async(st, 0);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // direct-to-LDS loads have landed
      __syncthreads();
      compute(0);
    }
  }

  // ---- epilogue: bias, residual, store, GroupNorm partials ---------------
  const size_t plane_out = (size_t)a.Ho * a.Wo;
  float s_lo[NB], s_hi[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) s_lo[b] = s_hi[b] = 0.f;

  if constexpr (OUT_KIND == OUT_FP8) {
    // MX-FP8 output: per position, one E8M0 scale per 32 channels (b = 0, 1
    // and b = 2, 3 of this tile), from the block maximum over the 4 lanes
    // (g4) that hold the position's channels.  Residual (bf16) added first.
    const int res_chunks = a.Cout / OO::CH;
    const size_t frame = (size_t)n * a.To_buf + a.out_f0 + to;
    // every residual value of this lane, loaded before the first store and
    // without branches (past the frame edge: a clamped in-frame address)
    uint2 rres[RESID ? MB : 1][NB];
    if constexpr (RESID) {
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        int i, j;
        out_local<MODE>(wave, m, l16, &i, &j);
        const size_t pos = (size_t)min(h0 + i, a.Ho - 1) * a.Wo + min(w0 + j, a.Wo - 1);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int c0 = ct * NT + b * 16 + 4 * g4;
          rres[m][b] = *reinterpret_cast<const uint2*>(
              reinterpret_cast<const char*>(a.resid) +
              ((frame * res_chunks + c0 / OO::CH) * plane_out + pos) * kChunkBytes + (c0 % OO::CH) * 2);
        }
      }
    }
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      int i, j;
      out_local<MODE>(wave, m, l16, &i, &j);
      const int oh = h0 + i, ow = w0 + j;
      const bool valid = (oh < a.Ho) && (ow < a.Wo);
      const size_t pos = (size_t)oh * a.Wo + ow;
      float v[NB][4];
      float am[2] = {0.f, 0.f};
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int lc = b * 16 + 4 * g4;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[b][r] = acc[m][b][r] * lds_wsc[lc + r] + lds_bias[lc + r];
        if constexpr (RESID) {
          const uint2 rv = rres[m][b];
          v[b][0] += bf16_lo(rv.x); v[b][1] += bf16_hi(rv.x);
          v[b][2] += bf16_lo(rv.y); v[b][3] += bf16_hi(rv.y);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) am[b >> 1] = fmaxf(am[b >> 1], fabsf(v[b][r]));
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        am[h] = fmaxf(am[h], __shfl_xor(am[h], 16));
        am[h] = fmaxf(am[h], __shfl_xor(am[h], 32));
      }
      const int e0 = fp8_block_exp(am[0]), e1 = fp8_block_exp(am[1]);
      const float inv0 = ldexpf(1.0f, -e0), inv1 = ldexpf(1.0f, -e1);
      if (valid) {
        char* orow = reinterpret_cast<char*>(a.out) + ((frame * a.out_chunks + ct) * plane_out + pos) * kChunkBytes;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const float f = b < 2 ? inv0 : inv1;
          *reinterpret_cast<uint32_t*>(orow + b * 16 + 4 * g4) =
              pack_fp8x4(v[b][0] * f, v[b][1] * f, v[b][2] * f, v[b][3] * f);
        }
        if (g4 == 0)
          reinterpret_cast<uint16_t*>(a.out_scale)[(frame * a.out_chunks + ct) * plane_out + pos] =
              (uint16_t)((e0 + 127) | ((e1 + 127) << 8));
      }
    }
    return;
  }

  // activation output: byte offset of this lane's 4 channels of block b at
  // position block m (the residual has the output's layout)
  // (a per-block base: frame, channel chunk and the lane's channels; plus the
  // position's 32-bit offset: a plane is below 2^31 bytes, checked on the host)
  size_t cbase[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int c0 = ct * NT + b * 16 + 4 * g4;
    const int chunk = c0 / OO::CH, within = c0 % OO::CH;
    cbase[b] = (((size_t)n * a.To_buf + a.out_f0 + to) * a.out_chunks + chunk) * plane_out * kChunkBytes +
               (size_t)within * (kChunkBytes / OO::CH);
  }
  auto act_off = [&](int oh, int ow, int b) {
    return cbase[b] + (size_t)(uint32_t)((oh * a.Wo + ow) * kChunkBytes);
  };
  // bf16 residual: every value of this lane loaded before the first store,
  // without branches (past the frame edge: a clamped in-frame address whose
  // value is never stored)
  constexpr bool RPRE = RESID && OUT_KIND == OUT_ACT && OPREC == P_BF16;
  uint2 rres[RPRE ? MB : 1][NB];
  if constexpr (RPRE) {
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      int i, j;
      out_local<MODE>(wave, m, l16, &i, &j);
      const int ohc = min(h0 + i, a.Ho - 1), owc = min(w0 + j, a.Wo - 1);
#pragma unroll
      for (int b = 0; b < NB; ++b)
        rres[m][b] = *reinterpret_cast<const uint2*>(reinterpret_cast<const char*>(a.resid) + act_off(ohc, owc, b));
    }
  }
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    int i, j;
    out_local<MODE>(wave, m, l16, &i, &j);
    const int oh = h0 + i, ow = w0 + j;
    const bool valid = (oh < a.Ho) && (ow < a.Wo);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int c0 = ct * NT + b * 16 + 4 * g4, lc = b * 16 + 4 * g4;
      float v4[4];
      // (bias and weight scale are 0 past Cout; fp8 still forces those values to 0)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if constexpr (F8) {
          const float y = acc[m][b][r] * lds_wsc[lc + r] + lds_bias[lc + r];
          v4[r] = (c0 + r) < a.Cout ? y : 0.f;
        } else {
          v4[r] = acc[m][b][r] + lds_bias[lc + r];
        }
      }
      if constexpr (OUT_KIND == OUT_ACT) {
        const size_t off = act_off(oh, ow, b);
        if constexpr (OPREC == P_BF16) {
          if (valid) {
            if constexpr (RESID) {
              const uint2 rv = rres[m][b];
              v4[0] += bf16_lo(rv.x); v4[1] += bf16_hi(rv.x);
              v4[2] += bf16_lo(rv.y); v4[3] += bf16_hi(rv.y);
            }
            const uint2 pv = make_uint2(pack_bf16(v4[0], v4[1]), pack_bf16(v4[2], v4[3]));
            *reinterpret_cast<uint2*>(reinterpret_cast<char*>(a.out) + off) = pv;
            // statistics of the stored (rounded) values
            v4[0] = bf16_lo(pv.x); v4[1] = bf16_hi(pv.x); v4[2] = bf16_lo(pv.y); v4[3] = bf16_hi(pv.y);
          }
        } else {
          if (valid) {
            if constexpr (RESID) {
              const float4 rv = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(a.resid) + off);
              v4[0] += rv.x; v4[1] += rv.y; v4[2] += rv.z; v4[3] += rv.w;
            }
            *reinterpret_cast<float4*>(reinterpret_cast<char*>(a.out) + off) = make_float4(v4[0], v4[1], v4[2], v4[3]);
          }
        }
      } else {
        if (valid) {
          float* op = reinterpret_cast<float*>(a.out) +
                      (((size_t)n * a.To_buf + a.out_f0 + to) * plane_out + (size_t)oh * a.Wo + ow) * 3;
          if (a.blend_prev != nullptr && tg < a.blend_n) {
            // frame i = tg + 1 of the GoP: a_i prev[Tp - n + i] + (1 - a_i) x_hat, a_i = (n - i) / n
            const float al = (float)(a.blend_n - (tg + 1)) / (float)a.blend_n, be = 1.0f - al;
            const float* pp = a.blend_prev + (((size_t)n * a.blend_Tp + (a.blend_Tp - a.blend_n + tg)) * plane_out +
                                              (size_t)oh * a.Wo + ow) * 3;
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (c0 + r < 3) v4[r] = al * pp[c0 + r] + be * v4[r];
          }
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (c0 + r < 3) op[c0 + r] = v4[r];
        }
      }
      if constexpr (STATS) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[m][b][r] = valid ? v4[r] : 0.f;  // keep final values
        if (valid) {
          s_lo[b] += v4[0] + v4[1];
          s_hi[b] += v4[2] + v4[3];
        }
      }
    }
  }

  if constexpr (STATS) {
    // Per-tile Welford partials (count, mean, M2) per group of 2 channels.
    // Requires nt == Cout == 64 (32 groups), checked on the host.
    const int vr = min(G::TH, a.Ho - h0), vc = min(G::TW, a.Wo - w0);
    const float cnt = 2.0f * (float)(vr * vc);
    // Group sums through LDS (a buffer the K loop no longer needs): lane
    // (wave, g4, l16) puts its partials of groups 8 b + 2 g4 (+1) at row g,
    // column 16 wave + l16 (rows 72 floats apart, so that the readers below
    // hit distinct banks); thread t then adds 8 values of row t / 8 and three
    // shuffles finish the row.  Fixed order: deterministic.
    float* red2;
    if constexpr (MODE == CM_I2C) {
      if constexpr (PXH16) red2 = reinterpret_cast<float*>(lds_pxh);
      else red2 = lds_px;
      static_assert(MODE != CM_I2C || 32 * 72 * 4 <= PXN * (PXH16 ? 2 : 4), "group partials fit the pixel tile");
    } else {
      red2 = reinterpret_cast<float*>(&lds_a[0][0]);
      static_assert(MODE == CM_I2C || 32 * 72 * 4 <= HQ * 16, "group partials fit the halo buffer");
    }
    const int rg = tid >> 3, rp = tid & 7;
    auto row_total = [&]() {
      float t = 0.f;
#pragma unroll
      for (int u = 0; u < 8; ++u) t += red2[rg * 72 + u * 8 + rp];
      t += __shfl_xor(t, 1);
      t += __shfl_xor(t, 2);
      t += __shfl_xor(t, 4);
      return t;
    };
    __syncthreads();  // every wave is done with the K loop's LDS
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      red2[(b * 8 + 2 * g4) * 72 + wave * 16 + l16] = s_lo[b];
      red2[(b * 8 + 2 * g4 + 1) * 72 + wave * 16 + l16] = s_hi[b];
    }
    __syncthreads();
    {
      const float t = row_total();
      if (rp == 0) gmean[rg] = t / cnt;
    }
    __syncthreads();  // gmean is set and every row is read
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const float ma = gmean[b * 8 + 2 * g4], mb = gmean[b * 8 + 2 * g4 + 1];
      float qa = 0.f, qb = 0.f;
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        int i, j;
        out_local<MODE>(wave, m, l16, &i, &j);
        if (h0 + i < a.Ho && w0 + j < a.Wo) {
          const float d0 = acc[m][b][0] - ma, d1 = acc[m][b][1] - ma;
          const float d2 = acc[m][b][2] - mb, d3 = acc[m][b][3] - mb;
          qa += d0 * d0 + d1 * d1;
          qb += d2 * d2 + d3 * d3;
        }
      }
      red2[(b * 8 + 2 * g4) * 72 + wave * 16 + l16] = qa;
      red2[(b * 8 + 2 * g4 + 1) * 72 + wave * 16 + l16] = qb;
    }
    __syncthreads();
    {
      const float m2 = row_total();
      if (rp == 0) {
        const int tiles = a.tiles_h * a.tiles_w;
        a.stats[(((size_t)n * a.To + to) * tiles + (size_t)th * a.tiles_w + tw) * 32 + rg] =
            make_float4(cnt, gmean[rg], m2, 0.f);
      }
    }
  }
}

template <int PREC, int MODE, int NB, int IN_KIND, int OUT_KIND, bool RESID, bool STATS>
hipError_t launch_one(const ConvLaunch& a, hipStream_t s) {
  const long long nb = (long long)a.N * a.To * a.tiles_h * a.tiles_w * a.cout_tiles;
  if (nb <= 0 || nb > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((conv3d_kernel<PREC, MODE, NB, IN_KIND, OUT_KIND, RESID, STATS>),
                     dim3((unsigned)nb), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// 64 -> 3 last layer (bf16 or MX-fp8 input), walking the frames of one
// spatial tile.  The workgroup owns an 8 x 64 output tile of one clip and
// stages every input frame's halo once (per 64-byte channel chunk), instead of
// once per temporal tap.  The MFMA rows are (colour c, temporal tap kt)
// pairs, row 4 c + kt (12 of 16 used), so for output position p of a wave's
// block the lane (l16 = p, g4 = c) receives
//   d[kt] = sum_{kh, kw, i} W[c, i, kt, kh, kw] x[i, f, p + (kh, kw)]
// for the frame f being staged; output frame t gathers d[0] of frame t - 2,
// d[1] of t - 1 and d[2] of t (causal clamp: frame 0 supplies every tap that
// would read before it).  Each lane keeps the three output frames still
// collecting taps in registers and stores a frame once its last tap is in.
// Per output frame the sum is d[0] + d[1] + d[2] in that order (bf16: on top
// of the bias; fp8: then scaled by the colour's weight scale and biased), on
// every frame window, so chunked and whole-clip decodes agree bit for bit.
// Wave w owns output rows 2 w, 2 w + 1 (8 blocks of 16 positions).
// bf16: K = 32 channels x one tap per MFMA (16x16x32).  fp8: K = 128 = two
// taps x 64 channels per MFMA (16x16x128 with the activations' E8M0 scales),
// taps paired as in the fp8 stride-1 conv (a tenth, zero-weight tap pads the
// last pair).
// ---------------------------------------------------------------------------
constexpr int kWalkHW = 66, kWalkHalo = 10 * kWalkHW, kWalkHQ = kWalkHalo * 4;

template <int PREC, bool RS, bool BL>
__global__ void __launch_bounds__(kThreads, 3) conv_rgb_walk_kernel(ConvLaunch a) {
  constexpr bool F8 = PREC == P_FP8;
  constexpr int NCK = F8 ? 1 : 2;  // input chunks (64 channels)
  __shared__ uint4 lds_h[kWalkHQ];
  __shared__ uint16_t lds_sc[F8 ? kWalkHalo : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, g4 = lane >> 4;
  int v = xcd_remap(blockIdx.x, gridDim.x);
  const int tw = v % a.tiles_w; v /= a.tiles_w;
  const int th = v % a.tiles_h; v /= a.tiles_h;
  const int n = v;
  const int h0 = th * 8, w0 = tw * 64;

  // this lane's weight operands: row l16 = (c, kt) of the packed stride-1
  // layout's 16-row tile [kt][chunk][tap][row c][quad ^ swz(16 tap + c)]
  const int wc = l16 >> 2, wkt = l16 & 3;
  const bool wrow = wc < 3 && wkt < 3;
  const uint4* wq = reinterpret_cast<const uint4*>(a.wpk);
  // the 81 used weight rows (kt, tap, c) of each chunk in LDS, compact row
  // (kt * 9 + tap) * 3 + c, each row's quads in their packed (swizzled) order
  __shared__ uint4 lds_w[NCK * 81 * 4];
  for (int e = tid; e < NCK * 81 * 4; e += kThreads) {
    const int ck = e / (81 * 4), r = (e >> 2) % 81, c = r % 3, kt = r / 27, tap = (r / 3) % 9;
    lds_w[e] = ck < a.in_chunks ? wq[((size_t)((kt * a.in_chunks + ck) * 9 + tap) * 16 + c) * 4 + (e & 3)]
                                : make_uint4(0, 0, 0, 0);
  }
  // LDS index of this lane's quad q of (chunk ck, tap): row (c, kt) = (wc, wkt)
  auto wslot = [&](int ck, int tap, int q) {
    return (ck * 81 + (wkt * 9 + tap) * 3 + wc) * 4 + (q ^ swz(tap * 16 + wc));
  };
  const float bias = g4 < 3 ? a.bias[g4] : 0.f;
  const float wsc = F8 && g4 < 3 ? a.wscale[g4] : 1.f;

  // halo slots this thread fills (the same in every stage): in-frame quad offset or -1
  constexpr int NHS = (kWalkHQ + kThreads - 1) / kThreads;
  int hoff[NHS];
#pragma unroll
  for (int k = 0; k < NHS; ++k) {
    const int e = wave * 64 + k * kThreads + lane;
    hoff[k] = -1;
    if (e < kWalkHQ) {
      const int p = e >> 2, q = (e & 3) ^ swz(p);
      const int hs = h0 - 1 + p / kWalkHW, ws = w0 - 1 + p % kWalkHW;
      if (hs >= 0 && hs < a.Hi && ws >= 0 && ws < a.Wi) hoff[k] = (hs * a.Wi + ws) * 4 + q;
    }
  }
  // fp8: in-frame position of halo rows tid, tid + 256, tid + 512 (-1 outside)
  constexpr int NSR = F8 ? (kWalkHalo + kThreads - 1) / kThreads : 1;
  int soff[NSR];
#pragma unroll
  for (int k = 0; k < NSR; ++k) {
    const int p = tid + k * kThreads;
    const int hs = h0 - 1 + p / kWalkHW, ws = w0 - 1 + p % kWalkHW;
    soff[k] = (F8 && p < kWalkHalo && hs >= 0 && hs < a.Hi && ws >= 0 && ws < a.Wi) ? hs * a.Wi + ws : -1;
  }
  const size_t plane_in = (size_t)a.Hi * a.Wi, plane_out = (size_t)a.Ho * a.Wo;

  // output frames t, t + 1, t + 2 still collecting taps (colour g4, 8 positions)
  const float init = F8 ? 0.f : bias;
  float o0[8], o1[8], o2[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) o0[m] = o1[m] = o2[m] = init;
  // pixel-residual sums of this lane's 8 positions (colour g4), carried over
  // from the clip's earlier chunks
  static_assert(!(RS || BL) || !F8, "residual sums and blending: bf16");
  const bool rs_on = RS && g4 < 3;
  float rsum[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    rsum[m] = 0.f;
    const int oh = h0 + 2 * wave + (m >> 2), ow = w0 + (m & 3) * 16 + l16;
    if (rs_on && a.go0 > 0 && oh < a.Ho && ow < a.Wo)
      rsum[m] = a.rs_sum[(((size_t)n * a.Ho + oh) * a.Wo + ow) * 3 + g4];
  }

  const int f_first = max(a.go0 - 2, 0), f_end = a.go0 + a.To;
  for (int fg = f_first; fg < f_end; ++fg) {
    // residual: the tile's source bytes of this frame, 8 rows x 192 bytes =
    // 384 dwords (row r, dword q: bytes 12 q .. of columns w0 + ..), loaded
    // before its stages so that they arrive while the halo transfers are
    // awaited; rows past the frame are skipped, bytes past the frame's end
    // read as zeros (columns past Wo are never used)
    constexpr int XDW = 8 * 48;
    uint32_t xd[2] = {0u, 0u};
    // blending: the tile's pixels of the previous GoP's frame that output
    // frame fg is blended with, 8 rows x 192 floats, likewise (rows past the
    // frame skipped, floats past its end read as zeros)
    constexpr int PDW = 8 * 192, PK = PDW / kThreads;
    const bool bl_f = BL && fg >= a.go0 && fg < a.blend_n;
    float pd[BL ? PK : 1];
#pragma unroll
    for (int k = 0; k < (BL ? PK : 1); ++k) pd[k] = 0.f;
    if (bl_f) {
      const __amdgpu_buffer_rsrc_t pr = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float*>(a.blend_prev + ((size_t)n * a.blend_Tp + (a.blend_Tp - a.blend_n + fg)) * plane_out * 3),
          (short)0, (int)(plane_out * 12), 0x00020000);
#pragma unroll
      for (int k = 0; k < (BL ? PK : 1); ++k) {
        const int dq = tid + k * kThreads, r = dq / 192, q = dq % 192;
        if (h0 + r < a.Ho)
          pd[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                pr, (int)(((((h0 + r) * a.Wo + w0) * 3) + q) * 4), 0, 0));
      }
    }
    if (RS && fg >= a.go0) {
      const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<uint8_t*>(a.rs_x + ((size_t)n * a.rs_T + fg) * plane_out * 3), (short)0, (int)(plane_out * 3),
          0x00020000);
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int dq = tid + k * kThreads, r = dq / 48, q = dq % 48;
        if (dq < XDW && h0 + r < a.Ho)
          xd[k] = __builtin_amdgcn_raw_buffer_load_b32(xr, (int)((((h0 + r) * a.Wo + w0) * 3) + 4 * q), 0, 0);
      }
    }
    f32x4 d[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) d[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ck = 0; ck < NCK; ++ck) {
      if (ck >= a.in_chunks) break;
      __syncthreads();  // every wave is done reading the previous stage
      const size_t fplane = ((size_t)n * a.Ti + (fg - a.gi0)) * a.in_chunks + ck;
      const uint4* src = reinterpret_cast<const uint4*>(a.in) + fplane * plane_in * 4;
      uint16_t sv[NSR];
      if constexpr (F8) {
        // scale bytes of the halo rows (outside the frame: zeros with scale 2^0)
        const uint16_t* ssrc = reinterpret_cast<const uint16_t*>(a.in_scale) + fplane * plane_in;
#pragma unroll
        for (int k = 0; k < NSR; ++k) sv[k] = soff[k] >= 0 ? ssrc[soff[k]] : (uint16_t)0x7F7F;
      }
#pragma unroll
      for (int k = 0; k < NHS; ++k) {
        const int base = wave * 64 + k * kThreads, e = base + lane;
        if (e < kWalkHQ) {
          if (hoff[k] < 0) lds_h[e] = make_uint4(0, 0, 0, 0);
          else if constexpr (RS)  // (the plane is below 2^31 bytes, checked on the host)
            lds_dma16_buf(__builtin_amdgcn_make_buffer_rsrc(const_cast<uint4*>(src), (short)0,
                                                            (int)(plane_in * 64), 0x00020000),
                          (uint32_t)hoff[k] * 16u, &lds_h[base]);
          else lds_dma16(src + hoff[k], &lds_h[base]);
        }
      }
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      if constexpr (F8) {
#pragma unroll
        for (int k = 0; k < NSR; ++k)
          if (tid + k * kThreads < kWalkHalo) lds_sc[tid + k * kThreads] = sv[k];
      }
      __syncthreads();
      if constexpr (F8) {
        // pair t: data of tap 2 t + (g4 >> 1) (quads h, 2 + h), scale of tap
        // 2 t + h, 32-channel block g4 >> 1 (tap 9 stands for tap 8)
        const int h = g4 & 1, sblk = g4 >> 1;
#pragma unroll 1
        for (int t = 0; t < 5; ++t) {
          const int tap = min(2 * t + (g4 >> 1), 8), stap = min(2 * t + h, 8);
          const int kh = tap / 3, kw = tap % 3, skh = stap / 3, skw = stap % 3;
          // weights of row (c, kt) = (wc, wkt), tap 2 t + (g4 >> 1); zero for the unused rows and the tenth tap
          i32x8 wv = i32x8{0, 0, 0, 0, 0, 0, 0, 0};
          if (wrow && 2 * t + (g4 >> 1) < 9) {
            const uint4 q0 = lds_w[wslot(0, tap, h)], q1 = lds_w[wslot(0, tap, 2 + h)];
            wv = i32x8{(int)q0.x, (int)q0.y, (int)q0.z, (int)q0.w, (int)q1.x, (int)q1.y, (int)q1.z, (int)q1.w};
          }
#pragma unroll
          for (int m = 0; m < 8; ++m) {
            const int i = 2 * wave + (m >> 2), j = (m & 3) * 16 + l16;
            const i32x8 aq = ld_fp8_pair(lds_h, (i + kh) * kWalkHW + j + kw, h);
            const int sb = (lds_sc[(i + skh) * kWalkHW + j + skw] >> (8 * sblk)) & 255;
            mfma_fp8(d[m], wv, aq, sb);
          }
        }
      } else {
        // halo row 2 w + hr serves output row r = hr - kh for kh = 0..2
#pragma unroll 1
        for (int hr = 0; hr < 4; ++hr)
#pragma unroll
          for (int kw = 0; kw < 3; ++kw) {
            uint4 bq[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
              const int p = (2 * wave + hr) * kWalkHW + cb * 16 + l16 + kw;
              bq[cb] = lds_h[p * 4 + (g4 ^ swz(p))];
            }
#pragma unroll
            for (int r = 0; r < 2; ++r) {
              const int kh = hr - r;
              if (kh < 0 || kh > 2) continue;
              uint4 wv = make_uint4(0, 0, 0, 0);
              if (wrow) wv = lds_w[wslot(ck, kh * 3 + kw, g4)];
#pragma unroll
              for (int cb = 0; cb < 4; ++cb)
                d[r * 4 + cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf16x8, wv), __builtin_bit_cast(bf16x8, bq[cb]), d[r * 4 + cb], 0, 0, 0);
            }
          }
      }
    }
    // residual: the source bytes through the (now unused) halo buffer; lane
    // (l16, g4) takes colour g4 of its 8 positions (byte m & 3 of xv[m >> 2])
    uint32_t xv[2] = {0u, 0u};
    float pv[BL ? 8 : 1];
    if ((RS && fg >= a.go0) || bl_f) {
      __syncthreads();  // every wave is done reading this frame's halo
      uint32_t* lx = reinterpret_cast<uint32_t*>(lds_h);
      float* lp = reinterpret_cast<float*>(lds_h) + 512;  // (after the residual's 1536 bytes)
      if (RS) {
#pragma unroll
        for (int k = 0; k < 2; ++k)
          if (tid + k * kThreads < XDW) lx[tid + k * kThreads] = xd[k];
      }
      if (BL) {
#pragma unroll
        for (int k = 0; k < (BL ? PK : 1); ++k) lp[tid + k * kThreads] = pd[k];
      }
      __syncthreads();
      const uint8_t* lb = reinterpret_cast<const uint8_t*>(lds_h);
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int e = (2 * wave + (m >> 2)) * 192 + ((m & 3) * 16 + l16) * 3 + min(g4, 2);
        if (RS) xv[m >> 2] |= (uint32_t)lb[e] << (8 * (m & 3));
        if constexpr (BL) pv[m] = lp[e];
      }
    }
    // taps of frame fg: d[m][kt] belongs to output frame fg + 2 - kt (frame 0: to
    // every output frame whose clamped tap reads it)
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      if (fg == 0) {
        o0[m] = ((o0[m] + d[m][0]) + d[m][1]) + d[m][2];
        o1[m] = (o1[m] + d[m][0]) + d[m][1];
        o2[m] = o2[m] + d[m][0];
      } else {
        o0[m] += d[m][2];
        o1[m] += d[m][1];
        o2[m] += d[m][0];
      }
    }
    // output frame fg is complete
    if (fg >= a.go0 && g4 < 3) {
      const int to = fg - a.go0;
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int oh = h0 + 2 * wave + (m >> 2), ow = w0 + (m & 3) * 16 + l16;
        if (oh >= a.Ho || ow >= a.Wo) continue;
        float y = F8 ? o0[m] * wsc + bias : o0[m];
        if constexpr (BL) {
          if (fg < a.blend_n) {
            // frame i = fg + 1 of the GoP: a_i prev[Tp - n + i] + (1 - a_i) x_hat, a_i = (n - i) / n
            const float al = (float)(a.blend_n - (fg + 1)) / (float)a.blend_n, be = 1.0f - al;
            y = al * pv[m] + be * y;
          }
        }
        reinterpret_cast<float*>(a.out)[(((size_t)n * a.To_buf + a.out_f0 + to) * plane_out + (size_t)oh * a.Wo + ow) * 3 +
                                        g4] = y;
        if (rs_on) rsum[m] += ((float)((xv[m >> 2] >> (8 * (m & 3))) & 255u) / 127.5f - 1.0f) - y;
      }
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      o0[m] = o1[m];
      o1[m] = o2[m];
      o2[m] = init;
    }
  }
  if (rs_on) {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int oh = h0 + 2 * wave + (m >> 2), ow = w0 + (m & 3) * 16 + l16;
      if (oh < a.Ho && ow < a.Wo) a.rs_sum[(((size_t)n * a.Ho + oh) * a.Wo + ow) * 3 + g4] = rsum[m];
    }
  }
}

// Launches the frame-walking last layer after checking what it assumes: 3
// output colours in one 16-row tile, at most 64 input channels, and every
// walked input frame (max(go0 - 2, 0) .. go0 + To - 1) inside the input buffer.
template <int PREC>
hipError_t launch_rgb_walk(const ConvLaunch& a, hipStream_t s) {
  if (a.Cout != 3 || a.nt != 16 || a.in_chunks > (PREC == P_FP8 ? 1 : 2) || a.gi0 > (a.go0 > 2 ? a.go0 - 2 : 0) ||
      a.go0 + a.To - a.gi0 > a.Ti)
    return hipErrorInvalidValue;
  if (a.rs_sum && (!a.rs_x || a.go0 + a.To > a.rs_T)) return hipErrorInvalidValue;  // residual sums: source frames
  const long long nb = (long long)a.N * a.tiles_h * a.tiles_w;
  if (nb <= 0 || nb > 0x7fffffffLL) return hipErrorInvalidValue;
  if (a.rs_sum) {
    // (residual sums: bf16 only, and not with blending; the fp8 variant measured slower than the separate pass)
    if constexpr (PREC != P_BF16) return hipErrorInvalidValue;
    else {
      if (a.blend_prev) return hipErrorInvalidValue;
      hipLaunchKernelGGL((conv_rgb_walk_kernel<PREC, true, false>), dim3((unsigned)nb), dim3(kThreads), 0, s, a);
    }
  } else if (a.blend_prev) {
    // (blending: bf16 only; the fp8 variant measured slower than the separate blend pass)
    if constexpr (PREC != P_BF16) return hipErrorInvalidValue;
    else hipLaunchKernelGGL((conv_rgb_walk_kernel<PREC, false, true>), dim3((unsigned)nb), dim3(kThreads), 0, s, a);
  } else {
    hipLaunchKernelGGL((conv_rgb_walk_kernel<PREC, false, false>), dim3((unsigned)nb), dim3(kThreads), 0, s, a);
  }
  return hipGetLastError();
}

template <int PREC>
hipError_t dispatch_prec(const ConvLaunch& a, hipStream_t s) {
  // The configurations the tokenizer uses.
  const bool res = a.resid != nullptr, st = a.stats != nullptr;
  if (a.in_kind == IN_U8) {
    if (a.mode == CM_I2C && a.nt == 64 && a.out_kind == OUT_ACT && !res && st)
      return launch_one<PREC, CM_I2C, 4, IN_U8, OUT_ACT, false, true>(a, s);
    return hipErrorInvalidValue;
  }
  if (a.out_kind == OUT_RGB32) {
    if (a.mode == CM_S1 && a.nt == 16 && !res && !st) {
      if constexpr (PREC == P_BF16) return launch_rgb_walk<P_BF16>(a, s);
      if (a.rs_sum) return hipErrorInvalidValue;  // residual sums: the frame-walking kernel only
      return launch_one<PREC, CM_S1, 1, IN_ACT, OUT_RGB32, false, false>(a, s);
    }
    if (a.mode == CM_S1T && a.nt == 16 && !res && !st)
      return launch_one<PREC, CM_S1T, 1, IN_ACT, OUT_RGB32, false, false>(a, s);
    return hipErrorInvalidValue;
  }
  if constexpr (PREC == P_F32) {
    // the upsampling adjoint: 32 output channels a workgroup
    if (a.mode == CM_UPT) {
      if (a.nt == 32 && a.out_kind == OUT_ACT && !res && !st)
        return launch_one<PREC, CM_UPT, 2, IN_ACT, OUT_ACT, false, false>(a, s);
      return hipErrorInvalidValue;
    }
  }
  if (a.mode == CM_S2) {
    if (!res && !st && a.nt == 128) return launch_one<PREC, CM_S2, 8, IN_ACT, OUT_ACT, false, false>(a, s);
    if (!res && !st && a.nt == 64) return launch_one<PREC, CM_S2, 4, IN_ACT, OUT_ACT, false, false>(a, s);
    return hipErrorInvalidValue;
  }
  if (a.nt != 64) return hipErrorInvalidValue;
  if (a.mode == CM_S1) {
    if (!res && st) return launch_one<PREC, CM_S1, 4, IN_ACT, OUT_ACT, false, true>(a, s);
    if (res && st) return launch_one<PREC, CM_S1, 4, IN_ACT, OUT_ACT, true, true>(a, s);
    if (res && !st) return launch_one<PREC, CM_S1, 4, IN_ACT, OUT_ACT, true, false>(a, s);
    if (!res && !st) return launch_one<PREC, CM_S1, 4, IN_ACT, OUT_ACT, false, false>(a, s);
    return hipErrorInvalidValue;
  }
  if (a.mode == CM_S1T) {
    if (!res && !st) return launch_one<PREC, CM_S1T, 4, IN_ACT, OUT_ACT, false, false>(a, s);
    return hipErrorInvalidValue;
  }
  if (a.mode == CM_S2T) {
    if (!res && !st) return launch_one<PREC, CM_S2T, 4, IN_ACT, OUT_ACT, false, false>(a, s);
    return hipErrorInvalidValue;
  }
  if (a.mode == CM_UPF) {
    if (!res && !st) return launch_one<PREC, CM_UPF, 4, IN_ACT, OUT_ACT, false, false>(a, s);
    if (!res && st) return launch_one<PREC, CM_UPF, 4, IN_ACT, OUT_ACT, false, true>(a, s);
    return hipErrorInvalidValue;
  }
  return hipErrorInvalidValue;
}


// ---------------------------------------------------------------------------
// Weight gradient of fp32 operands, stride 1 and stride 2 (the upsampling
// view: wgrad_up_kernel below).  Block = 256 threads (4 waves); block b
// handles temporal tap kt, a 32-channel slice of the input channels, a
// 64-channel slice of the output channels and a contiguous share of the
// (clip, frame, tile) items.  Per item it stages the output-gradient tile
// (TH x TW positions x 64 channels) and the input halo (32 channels) in LDS,
// then runs fp32 16x16x4 MFMAs with K = output positions: wave w accumulates
// output channels 16w..16w+15 x the 32 input channels x the 9 spatial taps
// (18 accumulator blocks).  Staging uses 16-byte loads, all of an item's
// issued before its first barrier (one load latency per item), and two
// blocks fit on a CU (76 KB of LDS at most), so one block's staging overlaps
// the other's MFMAs.
// ---------------------------------------------------------------------------
template <int VIEW> struct WGeo;
template <> struct WGeo<CM_S1> { static constexpr int TH = 2, TW = 64, HH = TH + 2, HW = TW + 2; };
template <> struct WGeo<CM_S2> { static constexpr int TH = 2, TW = 32, HH = 2 * TH + 1, HW = 2 * TW + 1; };

template <int VIEW>
__device__ __forceinline__ int wg_row(int r, int c, int kh, int kw) {
  using G = WGeo<VIEW>;
  if constexpr (VIEW == CM_S1) return (r + kh) * G::HW + c + kw;
  else return (2 * r + kh) * G::HW + 2 * c + kw;
}

template <int VIEW>
__global__ void __launch_bounds__(256, 2) wgrad_kernel(WgradLaunch a) {
  using G = WGeo<VIEW>;
  constexpr int CH = 16;                   // fp32 channels per 64-byte chunk
  constexpr int NPOS = G::TH * G::TW;      // output positions per item
  constexpr int HALO = G::HH * G::HW;
  constexpr int NDYQ = NPOS * 16;          // dy float4s per item (64 channels)
  constexpr int NXQ = HALO * 8;            // halo float4s per item (32 channels)
  constexpr int DYK = (NDYQ + 255) / 256, XK = (NXQ + 255) / 256;
  __shared__ float s_dy[NPOS][64 + 1];
  __shared__ float s_x[HALO][32 + 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, k4 = lane >> 4;
  const int ic_tiles = (a.Cin + 31) / 32, oc_tiles = (a.Cout + 63) / 64;
  int v = blockIdx.x;
  const int sp = v % a.splits; v /= a.splits;
  const int ot = v % oc_tiles; v /= oc_tiles;
  const int it = v % ic_tiles; v /= ic_tiles;
  const int kt = v;
  const int tiles_h = (a.Ho + G::TH - 1) / G::TH, tiles_w = (a.Wo + G::TW - 1) / G::TW;
  const long long items = (long long)a.N * a.To * tiles_h * tiles_w;
  const long long i0 = items * sp / a.splits, i1 = items * (sp + 1) / a.splits;

  f32x4 acc[9][2];
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[t][0] = acc[t][1] = f32x4{0.f, 0.f, 0.f, 0.f};
  // Blocks of temporal tap 0 and the first input-channel slice also sum the
  // output gradient per channel (the bias gradient), in item order.
  const bool bias_sum = a.bpartial && kt == 0 && it == 0;
  float bsum = 0.f;

  const size_t plane_x = (size_t)a.Hi * a.Wi, plane_y = (size_t)a.Ho * a.Wo;
  const float4* dyq = reinterpret_cast<const float4*>(a.dy);
  const float4* xq = reinterpret_cast<const float4*>(a.x);
  for (long long item = i0; item < i1; ++item) {
    long long u = item;
    const int tw = (int)(u % tiles_w); u /= tiles_w;
    const int th = (int)(u % tiles_h); u /= tiles_h;
    const int to = (int)(u % a.To); u /= a.To;
    const int n = (int)u;
    const int h0 = th * G::TH, w0 = tw * G::TW;
    int ts;
    if constexpr (VIEW == CM_S1) ts = max(to + kt - 2, 0);
    else ts = max(2 * to + kt - 2, 0);
    // all of the item's 16-byte loads first (zeros outside the frame and past
    // the stored channels); element e = (chunk, position, quad), quad fastest
    float4 vd[DYK], vx[XK];
#pragma unroll
    for (int k = 0; k < DYK; ++k) {
      const int e = tid + 256 * k;
      const int q = e & 3, p = (e >> 2) % NPOS, c4 = (e >> 2) / NPOS;
      const int oh = h0 + p / G::TW, ow = w0 + p % G::TW;
      const int ck = ot * 4 + c4;
      vd[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e < NDYQ && oh < a.Ho && ow < a.Wo && ck < a.dy_chunks)
        vd[k] = dyq[((((size_t)n * a.To + to) * a.dy_chunks + ck) * plane_y + (size_t)oh * a.Wo + ow) * 4 + q];
    }
#pragma unroll
    for (int k = 0; k < XK; ++k) {
      const int e = tid + 256 * k;
      const int q = e & 3, p = (e >> 2) % HALO, c2 = (e >> 2) / HALO;
      const int r = p / G::HW, c = p % G::HW;
      int hs, ws;
      if constexpr (VIEW == CM_S1) { hs = h0 - 1 + r; ws = w0 - 1 + c; }
      else { hs = 2 * h0 - 1 + r; ws = 2 * w0 - 1 + c; }
      const int ck = it * 2 + c2;
      vx[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e < NXQ && hs >= 0 && hs < a.Hi && ws >= 0 && ws < a.Wi && ck < a.x_chunks)
        vx[k] = xq[((((size_t)n * a.Ti + ts) * a.x_chunks + ck) * plane_x + (size_t)hs * a.Wi + ws) * 4 + q];
    }
    __syncthreads();  // the previous item's MFMAs are done with the tiles
#pragma unroll
    for (int k = 0; k < DYK; ++k) {
      const int e = tid + 256 * k;
      if (e < NDYQ) {
        const int q = e & 3, p = (e >> 2) % NPOS, c4 = (e >> 2) / NPOS;
        float* d = &s_dy[p][c4 * 16 + q * 4];
        d[0] = vd[k].x; d[1] = vd[k].y; d[2] = vd[k].z; d[3] = vd[k].w;
      }
    }
#pragma unroll
    for (int k = 0; k < XK; ++k) {
      const int e = tid + 256 * k;
      if (e < NXQ) {
        const int q = e & 3, p = (e >> 2) % HALO, c2 = (e >> 2) / HALO;
        float* d = &s_x[p][c2 * 16 + q * 4];
        d[0] = vx[k].x; d[1] = vx[k].y; d[2] = vx[k].z; d[3] = vx[k].w;
      }
    }
    __syncthreads();
    if (bias_sum && tid < 64) {
      for (int p = 0; p < NPOS; ++p) bsum += s_dy[p][tid];
    }
    // K = output positions, 4 per MFMA
#pragma unroll 2
    for (int k0 = 0; k0 < NPOS; k0 += 4) {
      const int p = k0 + k4;
      const int r = p / G::TW, c = p % G::TW;
      const float av = s_dy[p][wave * 16 + l16];
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const int row = wg_row<VIEW>(r, c, t / 3, t % 3);
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[t][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, s_x[row][b * 16 + l16], acc[t][b], 0, 0, 0);
      }
    }
  }
  // D block (o, i): lane holds o = 4*k4 + r (r = 0..3), i = l16
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int oc = ot * 64 + wave * 16 + 4 * k4 + r, icn = it * 32 + b * 16 + l16;
        if (oc < a.Cout && icn < a.Cin)
          a.partial[((((size_t)sp * 3 + kt) * 9 + t) * a.Cout + oc) * a.Cin + icn] = acc[t][b][r];
      }
  if (bias_sum && tid < 64 && ot * 64 + tid < a.Cout) a.bpartial[(size_t)sp * a.Cout + ot * 64 + tid] = bsum;
}

// ---------------------------------------------------------------------------
// Weight gradient of the upsampling conv (nearest x2 upsample, then the causal
// 3x3x3 conv), fp32, in polyphase form.  Along each of t, h, w an output of
// parity 0 reads, through the upsample, source offset -1 with tap 0 and offset
// 0 with taps 1 and 2; parity 1 reads offset 0 with taps 0 and 1 and offset +1
// with tap 2 (time: source frame ceil(u / 2), clamped at 0 like the conv's
// causal padding).  The gradient is therefore accumulated per output phase
// (pt, ph, pw) and source offset index (dt, dh, dw) in {0, 1}^3 -- 64 folded
// taps, each over 1/8 of the output positions, 8 Cin Cout MACs per output
// position instead of the dense view's 27 -- and the reduction unfolds them:
// dW[kt, kh, kw] = sum over phases of the folded tap (kt, kh, kw) falls on.
//   partial[split][fold][Cout][Cin], fold = ((((pt 2 + dt) 2 + ph) 2 + pw) 2 + dh) 2 + dw
//   bias partial[split][pt 2 + ph][Cout]
// Block = (pt, dt, ph, 32 input channels, 64 output channels, split).  An item
// is kUpTM source rows m (output rows 2 m + ph) x 64 output columns (32 source
// columns x both pw) of one output frame 2 j + pt; its positions are ordered
// (row, pw, column), so the 4 positions of an MFMA's K share their phase.
// Staging as in wgrad_kernel: every 16-byte load of an item issued before its
// first barrier; the source halo is kUpTM + 2 rows x 34 columns.
// ---------------------------------------------------------------------------
constexpr int kUpTM = 2;

__global__ void __launch_bounds__(256, 2) wgrad_up_kernel(WgradLaunch a) {
  constexpr int TM = kUpTM, NPOS = TM * 64, HR = TM + 2, HC = 34, HALO = HR * HC;
  constexpr int NDYQ = NPOS * 16;          // dy float4s per item (64 channels)
  constexpr int NXQ = HALO * 8;            // halo float4s per item (32 channels)
  constexpr int DYK = (NDYQ + 255) / 256, XK = (NXQ + 255) / 256;
  __shared__ float s_dy[NPOS][64 + 1];
  __shared__ float s_x[HALO][32 + 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, k4 = lane >> 4;
  const int ic_tiles = (a.Cin + 31) / 32, oc_tiles = (a.Cout + 63) / 64;
  int v = blockIdx.x;
  const int sp = v % a.splits; v /= a.splits;
  const int ot = v % oc_tiles; v /= oc_tiles;
  const int it = v % ic_tiles; v /= ic_tiles;
  const int ph = v & 1, dt = (v >> 1) & 1, pt = v >> 2;
  const int Tj = (a.To + 1 - pt) / 2;  // output frames 2 j + pt < To
  const int tiles_m = (a.Hi + TM - 1) / TM, tiles_w = (a.Wo + 63) / 64;
  const long long items = (long long)a.N * Tj * tiles_m * tiles_w;
  const long long i0 = items * sp / a.splits, i1 = items * (sp + 1) / a.splits;

  f32x4 acc[2][4][2];  // [pw][2 dh + dw][input-channel block]
#pragma unroll
  for (int pw = 0; pw < 2; ++pw)
#pragma unroll
    for (int f = 0; f < 4; ++f) acc[pw][f][0] = acc[pw][f][1] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bool bias_sum = a.bpartial && dt == 0 && it == 0;
  float bsum = 0.f;

  const size_t plane_x = (size_t)a.Hi * a.Wi, plane_y = (size_t)a.Ho * a.Wo;
  const float4* dyq = reinterpret_cast<const float4*>(a.dy);
  const float4* xq = reinterpret_cast<const float4*>(a.x);
  for (long long item = i0; item < i1; ++item) {
    long long u = item;
    const int tw = (int)(u % tiles_w); u /= tiles_w;
    const int tm = (int)(u % tiles_m); u /= tiles_m;
    const int j = (int)(u % Tj);
    const int n = (int)(u / Tj);
    const int to = 2 * j + pt;
    const int m0 = tm * TM, w0 = tw * 64, q0 = w0 >> 1;
    const int ts = max(j + dt - (pt ? 0 : 1), 0);  // source frame of temporal offset index dt
    float4 vd[DYK], vx[XK];
#pragma unroll
    for (int k = 0; k < DYK; ++k) {
      const int e = tid + 256 * k;
      const int q = e & 3, p = (e >> 2) % NPOS, c4 = (e >> 2) / NPOS;
      const int m = m0 + p / 64, ow = w0 + 2 * (p & 31) + ((p >> 5) & 1);
      const int ck = ot * 4 + c4;
      vd[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e < NDYQ && m < a.Hi && ow < a.Wo && ck < a.dy_chunks)
        vd[k] = dyq[((((size_t)n * a.To + to) * a.dy_chunks + ck) * plane_y + (size_t)(2 * m + ph) * a.Wo + ow) * 4 + q];
    }
#pragma unroll
    for (int k = 0; k < XK; ++k) {
      const int e = tid + 256 * k;
      const int q = e & 3, p = (e >> 2) % HALO, c2 = (e >> 2) / HALO;
      const int hs = m0 - 1 + p / HC, ws = q0 - 1 + p % HC;
      const int ck = it * 2 + c2;
      vx[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e < NXQ && hs >= 0 && hs < a.Hi && ws >= 0 && ws < a.Wi && ck < a.x_chunks)
        vx[k] = xq[((((size_t)n * a.Ti + ts) * a.x_chunks + ck) * plane_x + (size_t)hs * a.Wi + ws) * 4 + q];
    }
    __syncthreads();  // the previous item's MFMAs are done with the tiles
#pragma unroll
    for (int k = 0; k < DYK; ++k) {
      const int e = tid + 256 * k;
      if (e < NDYQ) {
        const int q = e & 3, p = (e >> 2) % NPOS, c4 = (e >> 2) / NPOS;
        float* d = &s_dy[p][c4 * 16 + q * 4];
        d[0] = vd[k].x; d[1] = vd[k].y; d[2] = vd[k].z; d[3] = vd[k].w;
      }
    }
#pragma unroll
    for (int k = 0; k < XK; ++k) {
      const int e = tid + 256 * k;
      if (e < NXQ) {
        const int q = e & 3, p = (e >> 2) % HALO, c2 = (e >> 2) / HALO;
        float* d = &s_x[p][c2 * 16 + q * 4];
        d[0] = vx[k].x; d[1] = vx[k].y; d[2] = vx[k].z; d[3] = vx[k].w;
      }
    }
    __syncthreads();
    if (bias_sum && tid < 64) {
      for (int p = 0; p < NPOS; ++p) bsum += s_dy[p][tid];
    }
    // K = 4 positions (r, pw, c0 + k4) per MFMA; source offset (dh, dw) of
    // phase (ph, pw) reads halo row r + ph + dh, column c + pw + dw
#pragma unroll
    for (int r = 0; r < TM; ++r)
#pragma unroll
      for (int pw = 0; pw < 2; ++pw)
#pragma unroll 2
        for (int c0 = 0; c0 < 32; c0 += 4) {
          const int c = c0 + k4;
          const float av = s_dy[r * 64 + pw * 32 + c][wave * 16 + l16];
#pragma unroll
          for (int f = 0; f < 4; ++f) {
            const int row = (r + ph + (f >> 1)) * HC + c + pw + (f & 1);
#pragma unroll
            for (int b = 0; b < 2; ++b)
              acc[pw][f][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, s_x[row][b * 16 + l16], acc[pw][f][b], 0, 0, 0);
          }
        }
  }
  // D block (o, i): lane holds o = 4 k4 + r (r = 0..3), i = l16
#pragma unroll
  for (int pw = 0; pw < 2; ++pw)
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int oc = ot * 64 + wave * 16 + 4 * k4 + r, icn = it * 32 + b * 16 + l16;
          const int fold = ((((pt * 2 + dt) * 2 + ph) * 2 + pw) * 2 + (f >> 1)) * 2 + (f & 1);
          if (oc < a.Cout && icn < a.Cin)
            a.partial[(((size_t)sp * 64 + fold) * a.Cout + oc) * a.Cin + icn] = acc[pw][f][b][r];
        }
  if (bias_sum && tid < 64 && ot * 64 + tid < a.Cout)
    a.bpartial[((size_t)sp * 4 + pt * 2 + ph) * a.Cout + ot * 64 + tid] = bsum;
}

// ---------------------------------------------------------------------------
// Weight gradient on bf16 MFMA (bf16 operands; channel counts are padded to
// 64-channel tiles, empty 16-channel blocks are skipped).
// D[o][i] += dy[p][o] x~[p + tap][i] with K = output positions: 16x16x32 bf16
// MFMAs, A = dy (rows o), B = x (columns i).  Block = (temporal tap, 64
// output channels, 64 input channels, split); wave w owns input channels
// 16w .. 16w+15 and all 64 output channels x 9 spatial taps (36 accumulator
// blocks).  An item is TH output rows x 64 columns of one output frame.  Both
// operands need K (positions) contiguous in LDS, so dy and the input halo are
// transposed while staged (8 x 8 register transposes, 16-byte LDS stores):
//   s_dy[o][p], p = r * 64 + c;   s_x[i][row][plane][col]
// with rows / columns of the conv's input as the tap sees it: stride 1 stores
// the halo directly; stride 2 stores the halo's even and odd columns in two
// planes.  The column read by tap kw is then offset by 0, 1 or 2 elements
// from a 16-byte boundary; offset reads take 5 dwords and realign them with
// byte shifts.
// The upsampling view (VIEW = CM_UPF) runs in polyphase form, as
// wgrad_up_kernel does for fp32: block = (pt, dt, ph, ...), an item is TH
// source rows m (output rows 2 m + ph) x 64 output columns of frame 2 j + pt,
// its positions ordered (row, pw, column) so that a K step of 32 positions is
// one (row, pw); the halo is the source's (TH + 2 rows x 34 columns), and
// accumulator t = 4 pw + 2 dh + dw holds folded tap (pw, dh, dw), written to
// the 64-tap partial layout (8 Cin Cout MACs per output position instead of 27).
// ---------------------------------------------------------------------------
template <int VIEW> struct WMGeo;
template <> struct WMGeo<CM_S1> { static constexpr int TH = 2, ROWS = 4, PLANES = 1, QB = 9; };
template <> struct WMGeo<CM_UPF> { static constexpr int TH = 2, ROWS = 4, PLANES = 1, QB = 5; };
template <> struct WMGeo<CM_S2> { static constexpr int TH = 1, ROWS = 3, PLANES = 2, QB = 9; };
constexpr int kWmCols = 80;   // halo columns per plane row: >= 66, multiple of 8, + 8 for the read window

template <int VIEW> struct WMLds {
  using G = WMGeo<VIEW>;
  static constexpr int NPOS = G::TH * 64;
  static constexpr int DYS = NPOS + 8;  // s_dy row stride (elements): 4 dwords mod 32 banks
  static constexpr int XR = G::ROWS * G::PLANES * kWmCols;
  static constexpr int XS = ((XR / 2 + 27) / 32) * 32 * 2 + 8;  // s_x channel stride: 4 dwords mod 32 banks
};

// 8 x 8 transpose of bf16: v[p] holds 8 channels of position p; w[c] receives
// 8 positions of channel c.
__device__ __forceinline__ void transpose8x8_bf16(const uint4* v, uint4* w) {
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    uint32_t d[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t a = (&v[2 * j].x)[c >> 1], b = (&v[2 * j + 1].x)[c >> 1];
      d[j] = (c & 1) ? ((a >> 16) | (b & 0xffff0000u)) : ((a & 0xffffu) | (b << 16));
    }
    w[c] = make_uint4(d[0], d[1], d[2], d[3]);
  }
}

// The same transpose, handing each w[c] to store(c, w[c]) as soon as it is
// formed (no 8-vector temporary).
template <typename F>
__device__ __forceinline__ void transpose8x8_bf16_store(const uint4* v, F store) {
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    uint32_t d[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t a = (&v[2 * j].x)[c >> 1], b = (&v[2 * j + 1].x)[c >> 1];
      d[j] = (c & 1) ? ((a >> 16) | (b & 0xffff0000u)) : ((a & 0xffffu) | (b << 16));
    }
    store(c, make_uint4(d[0], d[1], d[2], d[3]));
  }
}

// 16 bf16 from element offset e0 (a multiple of 8) of an LDS array: two
// aligned 16-byte reads, from which the 8 elements at offset 0, 1 or 2 are
// taken in registers (no unaligned LDS access).
struct Win16 { uint4 lo, hi; };
__device__ __forceinline__ Win16 ld16_bf16(const uint16_t* base, int e0) {
  const uint4* q = reinterpret_cast<const uint4*>(base + e0);
  return Win16{q[0], q[1]};
}
template <int MIS>
__device__ __forceinline__ uint4 win_at(const Win16& w) {
  if constexpr (MIS == 0) return w.lo;
  else if constexpr (MIS == 2) return make_uint4(w.lo.y, w.lo.z, w.lo.w, w.hi.x);
  else
    return make_uint4(__builtin_amdgcn_alignbyte(w.lo.y, w.lo.x, 2), __builtin_amdgcn_alignbyte(w.lo.z, w.lo.y, 2),
                      __builtin_amdgcn_alignbyte(w.lo.w, w.lo.z, 2), __builtin_amdgcn_alignbyte(w.hi.x, w.lo.w, 2));
}

template <int VIEW>
__global__ void __launch_bounds__(256, 2) wgrad_mfma_kernel(WgradLaunch a) {
  using G = WMGeo<VIEW>;
  using Lp = WMLds<VIEW>;
  constexpr int NPOS = Lp::NPOS, KS = NPOS / 32;
  __shared__ __align__(16) uint16_t s_dy[64 * Lp::DYS];
  __shared__ __align__(16) uint16_t s_x[64 * Lp::XS];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, g4 = lane >> 4;
  const int ic_tiles = (a.Cin + 63) / 64, oc_tiles = (a.Cout + 63) / 64;
  int v = blockIdx.x;
  const int sp = v % a.splits; v /= a.splits;
  const int ot = v % oc_tiles; v /= oc_tiles;
  const int it = v % ic_tiles; v /= ic_tiles;
  constexpr bool UPF = VIEW == CM_UPF;
  const int kt = v;                                       // dense views: temporal tap
  const int ph = v & 1, dt = (v >> 1) & 1, pt = v >> 2;   // polyphase: output phase / offset index
  const int Tj = UPF ? (a.To + 1 - pt) / 2 : a.To;        // output frames of the block
  const int tiles_h = UPF ? (a.Hi + G::TH - 1) / G::TH : (a.Ho + G::TH - 1) / G::TH, tiles_w = (a.Wo + 63) / 64;
  const int nob = min(4, (a.Cout - ot * 64 + 15) / 16);      // output-channel blocks holding channels
  const bool wave_cols = it * 64 + wave * 16 < a.Cin;          // this wave's input channels exist
  const int dy_ch = a.dy_chunks * 32, x_ch = a.x_chunks * 32;  // channels stored (zeros past Cout / Cin)
  const long long items = (long long)a.N * Tj * tiles_h * tiles_w;
  const long long i0 = items * sp / a.splits, i1 = items * (sp + 1) / a.splits;
  const bool bias_sum = a.bpartial && (UPF ? dt : kt) == 0 && it == 0;
  float bsum = 0.f;  // thread t: channel t >> 2, positions (t & 3) + 4 k of each item
  __shared__ float s_bias[4][64];

  f32x4 acc[4][9];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[b][t] = f32x4{0.f, 0.f, 0.f, 0.f};

  const size_t plane_x = (size_t)a.Hi * a.Wi, plane_y = (size_t)a.Ho * a.Wo;
  const uint4* dyq = reinterpret_cast<const uint4*>(a.dy);
  const uint4* xq = reinterpret_cast<const uint4*>(a.x);
  for (long long item = i0; item < i1; ++item) {
    long long u = item;
    const int tw = (int)(u % tiles_w); u /= tiles_w;
    const int th = (int)(u % tiles_h); u /= tiles_h;
    const int jt = (int)(u % Tj); u /= Tj;
    const int n = (int)u;
    const int to = UPF ? 2 * jt + pt : jt;
    const int h0 = th * G::TH, w0 = tw * 64;  // polyphase: h0 = first source row m0
    int ts;
    if constexpr (VIEW == CM_S1) ts = max(to + kt - 2, 0);
    else if constexpr (VIEW == CM_S2) ts = max(2 * to + kt - 2, 0);
    else ts = max(jt + dt - (pt ? 0 : 1), 0);
    // ---- staging: dy in blocks of 8 positions x 8 output channels (position
    // block fastest across lanes: their transposed 16-byte stores hit distinct
    // banks), the input halo in blocks of 8 columns (of one plane row) x 8
    // input channels.  Thread t owns blocks t and t + 256 of the NDY + NHX and
    // issues all their global loads before the barrier, so an item waits for
    // one load latency, overlapped with the other waves' previous compute.
    constexpr int QB = G::QB;  // column blocks holding the halo columns (66; polyphase 34)
    constexpr int NDY = (NPOS / 8) * 8, NHX = G::ROWS * G::PLANES * QB * 8;
    static_assert(NDY + NHX <= 512, "two staging blocks per thread");
    auto halo_block = [&](int hb, int* qb, int* cb, int* pl, int* hr) {
      *qb = hb % QB; hb /= QB;
      *cb = hb % 8; hb /= 8;
      *pl = hb % G::PLANES;
      *hr = hb / G::PLANES;
    };
    uint4 vv[2][8];
#pragma unroll
    for (int r2 = 0; r2 < 2; ++r2) {
      const int blk = tid + 256 * r2;
#pragma unroll
      for (int k = 0; k < 8; ++k) vv[r2][k] = make_uint4(0, 0, 0, 0);
      if (blk < NDY) {
        const int pb = blk % (NPOS / 8), cb = blk / (NPOS / 8);
        const int oc = ot * 64 + cb * 8;  // 8 channels inside one 32-channel chunk
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int p = pb * 8 + k;
          int oh = h0 + p / 64, ow = w0 + p % 64;
          if constexpr (UPF) { oh = 2 * (h0 + p / 64) + ph; ow = w0 + 2 * (p & 31) + ((p >> 5) & 1); }
          if (oh < a.Ho && ow < a.Wo && oc < dy_ch)
            vv[r2][k] = dyq[((((size_t)n * a.To + to) * a.dy_chunks + oc / 32) * plane_y + (size_t)oh * a.Wo + ow) * 4 +
                            (oc % 32) / 8];
        }
      } else if (blk < NDY + NHX) {
        int qb, cb, pl, hr;
        halo_block(blk - NDY, &qb, &cb, &pl, &hr);
        const int ic = it * 64 + cb * 8;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int q = qb * 8 + k;
          int hs, ws;
          if constexpr (VIEW == CM_S1) { hs = h0 - 1 + hr; ws = w0 - 1 + q; }
          else if constexpr (VIEW == CM_S2) { hs = 2 * h0 - 1 + hr; ws = 2 * w0 - 1 + 2 * q + pl; }
          else { hs = h0 - 1 + hr; ws = (w0 >> 1) - 1 + q; }  // source rows / columns
          if (q < (UPF ? 34 : 66) && hs >= 0 && hs < a.Hi && ws >= 0 && ws < a.Wi && ic < x_ch)
            vv[r2][k] = xq[((((size_t)n * a.Ti + ts) * a.x_chunks + ic / 32) * plane_x + (size_t)hs * a.Wi + ws) * 4 +
                           (ic % 32) / 8];
        }
      }
    }
    __syncthreads();  // every wave is done with the previous item's LDS tiles
#pragma unroll
    for (int r2 = 0; r2 < 2; ++r2) {
      const int blk = tid + 256 * r2;
      if (blk < NDY) {
        const int pb = blk % (NPOS / 8), cb = blk / (NPOS / 8);
        transpose8x8_bf16_store(vv[r2], [&](int k, const uint4& w) {
          *reinterpret_cast<uint4*>(&s_dy[(cb * 8 + k) * Lp::DYS + pb * 8]) = w;
        });
      } else if (blk < NDY + NHX) {
        int qb, cb, pl, hr;
        halo_block(blk - NDY, &qb, &cb, &pl, &hr);
        uint16_t* dst = &s_x[cb * 8 * Lp::XS + (hr * G::PLANES + pl) * kWmCols + qb * 8];
        transpose8x8_bf16_store(vv[r2], [&](int k, const uint4& w) {
          *reinterpret_cast<uint4*>(dst + k * Lp::XS) = w;
        });
      }
    }
    __syncthreads();
    if (bias_sum) {
      for (int p = tid & 3; p < NPOS; p += 4) bsum += __uint_as_float((uint32_t)s_dy[(tid >> 2) * Lp::DYS + p] << 16);
    }
    // ---- K loop over the item's positions, 32 per step ----
    const uint16_t* xrow = s_x + (wave * 16 + l16) * Lp::XS;
#pragma unroll 1
    for (int ks = 0; ks < (wave_cols ? KS : 0); ++ks) {
      const int pr = (ks * 32) / 64, pc = (ks * 32) % 64 + 8 * g4;  // this lane's 8 positions: row pr, cols pc..pc+7
      bf16x8 av[4];
#pragma unroll
      for (int b = 0; b < 4; ++b)
        av[b] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&s_dy[(b * 16 + l16) * Lp::DYS + ks * 32 + 8 * g4]));
      auto mma = [&](int t, const uint4& xv) {
        const bf16x8 bv = __builtin_bit_cast(bf16x8, xv);
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (b < nob) acc[b][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[b], bv, acc[b][t], 0, 0, 0);
      };
      if constexpr (UPF) {
        // K step ks = (row pr, phase pw); offset (dh, dw) reads halo row pr + ph + dh,
        // columns c + pw + dw of this lane's c = 8 g4 .. 8 g4 + 7
#pragma unroll
        for (int dh = 0; dh < 2; ++dh) {
          const Win16 w = ld16_bf16(xrow, (pr + ph + dh) * kWmCols + 8 * g4);
          if ((ks & 1) == 0) {
            mma(2 * dh + 0, win_at<0>(w));
            mma(2 * dh + 1, win_at<1>(w));
          } else {
            mma(4 + 2 * dh + 0, win_at<1>(w));
            mma(4 + 2 * dh + 1, win_at<2>(w));
          }
        }
        continue;
      }
#pragma unroll
      for (int kh = 0; kh < 3; ++kh) {
        if constexpr (VIEW == CM_S2) {
          // columns 2c + kw: kw = 0, 2 from the even plane (offset 0, 1), kw = 1 from the odd plane
          const int row = 2 * pr + kh;
          const Win16 ev = ld16_bf16(xrow, (row * 2 + 0) * kWmCols + pc);
          const Win16 od = ld16_bf16(xrow, (row * 2 + 1) * kWmCols + pc);
          mma(kh * 3 + 0, win_at<0>(ev));
          mma(kh * 3 + 1, win_at<0>(od));
          mma(kh * 3 + 2, win_at<1>(ev));
        } else {
          const Win16 w = ld16_bf16(xrow, (pr + kh) * kWmCols + pc);
          mma(kh * 3 + 0, win_at<0>(w));
          mma(kh * 3 + 1, win_at<1>(w));
          mma(kh * 3 + 2, win_at<2>(w));
        }
      }
    }
  }
  // D block (o, i): lane holds o = 16 b + 4 g4 + r, i = 16 wave + l16
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int t = 0; t < (UPF ? 8 : 9); ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int oc = ot * 64 + b * 16 + 4 * g4 + r, icn = it * 64 + wave * 16 + l16;
        // polyphase: folded tap ((((pt, dt), ph), pw = t / 4), dh, dw) of the 64
        const size_t slot = UPF ? (size_t)sp * 64 + (((((pt * 2 + dt) * 2 + ph) * 2 + (t >> 2)) * 2 + ((t >> 1) & 1)) * 2 +
                                                     (t & 1))
                                : ((size_t)sp * 3 + kt) * 9 + t;
        if (oc < a.Cout && icn < a.Cin) a.partial[(slot * a.Cout + oc) * a.Cin + icn] = acc[b][t][r];
      }
  if (bias_sum) {
    s_bias[tid & 3][tid >> 2] = bsum;
    __syncthreads();
    const size_t bslot = UPF ? (size_t)sp * 4 + pt * 2 + ph : (size_t)sp;
    if (tid < 64 && ot * 64 + tid < a.Cout)
      a.bpartial[bslot * a.Cout + ot * 64 + tid] = ((s_bias[0][tid] + s_bias[1][tid]) + s_bias[2][tid]) + s_bias[3][tid];
  }
}

// Sums the per-split partials in split order: weights into the canonical
// [o][i][kt][kh][kw] layout, then (elements past the weights) the bias.
// Thread e takes element e of a split's [kt][kh*3+kw][o][i] partial, so the
// loads of a wave are contiguous; only the one store per element is strided.
__global__ void __launch_bounds__(256) wgrad_reduce_kernel(const float* __restrict__ partial,
                                                            const float* __restrict__ bpartial, int splits, int Cout,
                                                            int Cin, float* __restrict__ dw, float* __restrict__ db) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)Cout * Cin * 27;
  if (e >= total) {
    const size_t o = e - total;
    if (o >= (size_t)Cout || !db) return;
    float acc = 0.f;
#pragma unroll 8
    for (int s = 0; s < splits; ++s) acc += bpartial[(size_t)s * Cout + o];
    db[o] = acc;
    return;
  }
  const int i = (int)(e % Cin);
  const size_t r = e / Cin;
  const int o = (int)(r % Cout), tap = (int)(r / Cout);  // tap = kt * 9 + kh * 3 + kw
  float acc = 0.f;
#pragma unroll 8
  for (int s = 0; s < splits; ++s) acc += partial[(size_t)s * total + e];
  dw[((size_t)o * Cin + i) * 27 + tap] = acc;
}

// The polyphase partials of wgrad_up_kernel unfolded into the canonical layout
// and summed in split order (per split: the 8 output phases in (pt, ph, pw)
// order); the bias over the 4 (pt, ph) partials of every split.
__global__ void __launch_bounds__(256) wgrad_reduce_up_kernel(const float* __restrict__ partial,
                                                               const float* __restrict__ bpartial, int splits,
                                                               int Cout, int Cin, float* __restrict__ dw,
                                                               float* __restrict__ db) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)Cout * Cin * 27;
  if (e >= total) {
    const size_t o = e - total;
    if (o >= (size_t)Cout || !db) return;
    float acc = 0.f;
    for (int s = 0; s < 4 * splits; ++s) acc += bpartial[(size_t)s * Cout + o];
    db[o] = acc;
    return;
  }
  const int i = (int)(e % Cin);
  const size_t r = e / Cin;
  const int o = (int)(r % Cout), tap = (int)(r / Cout);  // tap = kt * 9 + kh * 3 + kw
  const int kt = tap / 9, kh = (tap / 3) % 3, kw = tap % 3;
  // offset index of tap k for output parity p: p = 0 -> (0, 1, 1), p = 1 -> (0, 0, 1)
  auto off = [](int p, int k) { return p ? (k == 2 ? 1 : 0) : (k >= 1 ? 1 : 0); };
  const size_t fold_stride = (size_t)Cout * Cin, oi = (size_t)o * Cin + i;
  float acc = 0.f;
  for (int s = 0; s < splits; ++s)
#pragma unroll
    for (int ph8 = 0; ph8 < 8; ++ph8) {
      const int pt = ph8 >> 2, ph = (ph8 >> 1) & 1, pw = ph8 & 1;
      const int fold = ((((pt * 2 + off(pt, kt)) * 2 + ph) * 2 + pw) * 2 + off(ph, kh)) * 2 + off(pw, kw);
      acc += partial[((size_t)s * 64 + fold) * fold_stride + oi];
    }
  dw[((size_t)o * Cin + i) * 27 + tap] = acc;
}

}  // namespace

// fp8 decoder convs: MX-FP8 input, outputs bf16 (OUT_ACT), MX-FP8 or RGB.
hipError_t dispatch_fp8(const ConvLaunch& a, hipStream_t s) {
  const bool res = a.resid != nullptr, st = a.stats != nullptr;
  if (a.in_kind != IN_ACT || !a.in_scale || !a.wscale) return hipErrorInvalidValue;
  if (a.out_kind == OUT_RGB32) {
    if (a.mode == CM_S1 && a.nt == 16 && !res && !st) return launch_rgb_walk<P_FP8>(a, s);
    return hipErrorInvalidValue;
  }
  if (a.nt != 64 || a.Cout % 64 != 0) return hipErrorInvalidValue;
  if (a.out_kind == OUT_FP8) {
    if (!a.out_scale || st) return hipErrorInvalidValue;
    if (a.mode == CM_UPF && !res) return launch_one<P_FP8, CM_UPF, 4, IN_ACT, OUT_FP8, false, false>(a, s);
    if (a.mode == CM_S1 && res) return launch_one<P_FP8, CM_S1, 4, IN_ACT, OUT_FP8, true, false>(a, s);
    if (a.mode == CM_S1 && !res) return launch_one<P_FP8, CM_S1, 4, IN_ACT, OUT_FP8, false, false>(a, s);
    return hipErrorInvalidValue;
  }
  if (a.out_kind != OUT_ACT) return hipErrorInvalidValue;
  if (a.mode == CM_UPF && !res) {
    if (st) return launch_one<P_FP8, CM_UPF, 4, IN_ACT, OUT_ACT, false, true>(a, s);
    return launch_one<P_FP8, CM_UPF, 4, IN_ACT, OUT_ACT, false, false>(a, s);
  }
  if (a.mode == CM_S1) {
    if (!res && st) return launch_one<P_FP8, CM_S1, 4, IN_ACT, OUT_ACT, false, true>(a, s);
    if (res && st) return launch_one<P_FP8, CM_S1, 4, IN_ACT, OUT_ACT, true, true>(a, s);
    if (res && !st) return launch_one<P_FP8, CM_S1, 4, IN_ACT, OUT_ACT, true, false>(a, s);
    return launch_one<P_FP8, CM_S1, 4, IN_ACT, OUT_ACT, false, false>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_conv(const ConvLaunch& a, hipStream_t s) {
  // output positions are addressed with 32-bit offsets within a plane
  if ((size_t)a.Ho * a.Wo * kChunkBytes >= ((size_t)1 << 31)) return hipErrorInvalidValue;
  // the first layer reads its uint8 pixels with 32-bit buffer offsets
  if (a.in_kind == IN_U8 && (size_t)a.N * a.Ti * a.Hi * a.Wi * 3 >= ((size_t)1 << 31)) return hipErrorInvalidValue;
  if (a.stats && !(a.nt == 64 && a.Cout == 64 && a.cout_tiles == 1)) return hipErrorInvalidValue;
  // the epilogue reads the residual of every channel of its tile
  if (a.resid && (a.nt <= 0 || a.Cout % a.nt != 0)) return hipErrorInvalidValue;
  // the stride-2 adjoint maps a coarse gradient to its fine-resolution input shape
  if (a.mode == CM_S2T && (a.To != 2 * a.Ti - 1 || a.Ho != 2 * a.Hi || a.Wo != 2 * a.Wi || a.gi0 != 0))
    return hipErrorInvalidValue;
  // the upsampling adjoint maps a fine gradient to its source shape
  if (a.mode == CM_UPT && (a.Ti != 2 * a.To - 1 || a.Hi != 2 * a.Ho || a.Wi != 2 * a.Wo || a.gi0 != 0))
    return hipErrorInvalidValue;
  if (a.prec == P_BF16) return dispatch_prec<P_BF16>(a, s);
  if (a.prec == P_F32) return dispatch_prec<P_F32>(a, s);
  if (a.prec == P_FP8) return dispatch_fp8(a, s);
  return hipErrorInvalidValue;
}

namespace {
bool wgrad_uses_mfma_bf16(int prec, int Cout, int Cin) { (void)Cout; (void)Cin; return prec == P_BF16; }
}  // namespace

namespace {
bool wgrad_polyphase(int prec, int view) { (void)prec; return view == CM_UP; }
}  // namespace

int wgrad_partial_taps(int prec, int view) { return wgrad_polyphase(prec, view) ? 64 : 27; }
int wgrad_bias_parts(int prec, int view) { return wgrad_polyphase(prec, view) ? 4 : 1; }

int wgrad_blocks_per_split(int prec, int view, int Cout, int Cin) {
  if (wgrad_uses_mfma_bf16(prec, Cout, Cin))
    return (wgrad_polyphase(prec, view) ? 8 : 3) * ((Cin + 63) / 64) * ((Cout + 63) / 64);
  if (wgrad_polyphase(prec, view)) return 8 * ((Cin + 31) / 32) * ((Cout + 63) / 64);
  return 3 * ((Cin + 31) / 32) * ((Cout + 63) / 64);
}

int wgrad_items(int prec, int view, int Cout, int Cin, int N, int To, int Ho, int Wo) {
  int th, tw;
  if (wgrad_polyphase(prec, view)) {
    // items of one (pt, ph) class: TM source rows x 64 columns of the odd output frames
    const int tm = wgrad_uses_mfma_bf16(prec, Cout, Cin) ? WMGeo<CM_UPF>::TH : kUpTM;
    return N * (To / 2) * ((Ho / 2 + tm - 1) / tm) * ((Wo + 63) / 64);
  } else if (wgrad_uses_mfma_bf16(prec, Cout, Cin)) {
    th = view == CM_S2 ? WMGeo<CM_S2>::TH : WMGeo<CM_S1>::TH;
    tw = 64;
  } else if (view == CM_S2) {
    th = WGeo<CM_S2>::TH; tw = WGeo<CM_S2>::TW;
  } else {
    th = WGeo<CM_S1>::TH; tw = WGeo<CM_S1>::TW;
  }
  return N * To * ((Ho + th - 1) / th) * ((Wo + tw - 1) / tw);
}

hipError_t launch_wgrad(const WgradLaunch& a, hipStream_t s) {
  const long long nb = (long long)wgrad_blocks_per_split(a.prec, a.view, a.Cout, a.Cin) * a.splits;
  if (nb <= 0 || nb > 0x7fffffffLL || a.splits < 1) return hipErrorInvalidValue;
  const dim3 g((unsigned)nb), b(256);
  if (wgrad_uses_mfma_bf16(a.prec, a.Cout, a.Cin)) {
    if (a.view == CM_S1) hipLaunchKernelGGL(wgrad_mfma_kernel<CM_S1>, g, b, 0, s, a);
    else if (a.view == CM_S2) hipLaunchKernelGGL(wgrad_mfma_kernel<CM_S2>, g, b, 0, s, a);
    else if (a.view == CM_UP) {
      if (a.To != 2 * a.Ti - 1 || a.Ho != 2 * a.Hi || a.Wo != 2 * a.Wi) return hipErrorInvalidValue;
      hipLaunchKernelGGL(wgrad_mfma_kernel<CM_UPF>, g, b, 0, s, a);
    } else return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (a.prec != P_F32) return hipErrorInvalidValue;
  if (a.view == CM_S1) hipLaunchKernelGGL(wgrad_kernel<CM_S1>, g, b, 0, s, a);
  else if (a.view == CM_S2) hipLaunchKernelGGL(wgrad_kernel<CM_S2>, g, b, 0, s, a);
  else if (a.view == CM_UP) {
    if (a.To != 2 * a.Ti - 1 || a.Ho != 2 * a.Hi || a.Wo != 2 * a.Wi) return hipErrorInvalidValue;
    hipLaunchKernelGGL(wgrad_up_kernel, g, b, 0, s, a);
  } else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_wgrad_reduce(const WgradLaunch& a, float* dw, float* db, hipStream_t s) {
  const size_t total = (size_t)a.Cout * a.Cin * 27 + a.Cout;
  const dim3 g((unsigned)((total + 255) / 256)), b(256);
  if (wgrad_polyphase(a.prec, a.view))
    hipLaunchKernelGGL(wgrad_reduce_up_kernel, g, b, 0, s, a.partial, a.bpartial, a.splits, a.Cout, a.Cin, dw, db);
  else
    hipLaunchKernelGGL(wgrad_reduce_kernel, g, b, 0, s, a.partial, a.bpartial, a.splits, a.Cout, a.Cin, dw, db);
  return hipGetLastError();
}

// Packed weight layout, per output-channel tile ct (nt channels):
//   [ct][kt][chunk][kh*3+kw][o (nt)][quad 0..3][QE]   (quads XOR-swizzled by row)
// where row = tap * nt + o, and chunk covers CH input channels; channels
// beyond Cin / Cout are zero.  One (ct, kt, chunk) stage is 9 * nt * 64 bytes.
// Polyphase upsample layout (CM_UPF), per ct and output-frame parity pt:
//   [ct][pt][dt][chunk][phase][dh*2+dw][o][quad][QE], row = (phase*4 + tap) * nt + o,
// holding the folded kernel: along each of t, h, w a nearest-x2 upsample
// followed by a 3-tap kernel is, for output parity 0, tap 0 on source offset
// -1 and taps 1+2 on offset 0; for parity 1, taps 0+1 on offset 0 and tap 2 on
// offset +1.
// Stride-2 adjoint layout (CM_S2T), as CM_UPF's with three weight sets (output
// frame 0, even, odd output frames) and, per dimension, parity 0 holding tap 1
// on source offset 0 (offset -1: zero), parity 1 tap 2 on offset 0 and tap 0 on
// offset +1; in time, set 0 holds taps 0 + 1 + 2 on gradient frame 0 and tap 0
// on frame 1, set 1 tap 2 on frame j and tap 0 on frame j + 1, set 2 tap 1 on
// frame j + 1 (and nothing on its second stage).  Channels as in CM_S1T.
// Adjoint layout (CM_S1T), per adjoint output tile ct and weight set:
//   [ct][set][dt][chunk][kh*3+kw][o][quad][QE]
// with adjoint output channel o = forward input channel, adjoint input channel
// = forward output channel, gradient frame t + dt and spatial tap (dh, dw) =
// forward tap (2 - dh, 2 - dw).  Set 0 (output frames >= 1) uses forward tap
// kt = 2 - dt; set 1 (output frame 0, which the causal clamp reads for every
// t + kt <= 2) sums forward taps kt = 0 .. 2 - dt.
//
// The packing runs on the device (one thread per packed element), so packed
// weights can be refreshed from a device-resident parameter vector.
namespace {

struct PackGeom {
  int Cout, Cin;     // forward conv
  int CH, QE, nt, chunks, mode;
  int co;            // output channels of the packed kernel (Cin for the adjoint)
  int R;             // entries of the layout's leading dimensions per output-channel tile
};

__host__ __device__ inline int fold_lo(int parity, int d) { return parity == 0 ? (d == 0 ? 0 : 1) : (d == 0 ? 0 : 2); }
__host__ __device__ inline int fold_hi(int parity, int d) { return parity == 0 ? (d == 0 ? 0 : 2) : (d == 0 ? 1 : 2); }

__device__ float pack_value(const float* __restrict__ w, const PackGeom& g, size_t e) {
  const int x = (int)(e % g.QE); e /= g.QE;
  const int pq = (int)(e % 4); e /= 4;
  const int o = (int)(e % g.nt); e /= g.nt;
  auto W = [&](int co, int ci, int kt, int kh, int kw) -> float {
    return w[((((size_t)co * g.Cin + ci) * 3 + kt) * 3 + kh) * 3 + kw];
  };
  if (g.mode == CM_UPF) {
    const int tap = (int)(e % 4); e /= 4;
    const int phase = (int)(e % 4); e /= 4;
    const int ck = (int)(e % g.chunks); e /= g.chunks;
    const int dt = (int)(e % 2); e /= 2;
    const int pt = (int)(e % 2); e /= 2;
    const int ct = (int)e;
    const int row = (phase * 4 + tap) * g.nt + o;
    const int q = pq ^ swz(row);
    const int co = ct * g.nt + o, ci = ck * g.CH + q * g.QE + x;
    if (co >= g.Cout || ci >= g.Cin) return 0.f;
    const int ph = phase >> 1, pw = phase & 1, dh = tap >> 1, dw = tap & 1;
    float v = 0.f;
    for (int kt = fold_lo(pt, dt); kt <= fold_hi(pt, dt); ++kt)
      for (int kh = fold_lo(ph, dh); kh <= fold_hi(ph, dh); ++kh)
        for (int kw = fold_lo(pw, dw); kw <= fold_hi(pw, dw); ++kw) v += W(co, ci, kt, kh, kw);
    return v;
  }
  if (g.mode == CM_S2T) {
    const int tap = (int)(e % 4); e /= 4;
    const int phase = (int)(e % 4); e /= 4;
    const int ck = (int)(e % g.chunks); e /= g.chunks;
    const int dt = (int)(e % 2); e /= 2;
    const int set = (int)(e % 3); e /= 3;
    const int ct = (int)e;
    const int row = (phase * 4 + tap) * g.nt + o;
    const int q = pq ^ swz(row);
    const int oc = ct * g.nt + o, ic = ck * g.CH + q * g.QE + x;  // adjoint out / in channels
    if (oc >= g.Cin || ic >= g.Cout) return 0.f;
    // forward tap of parity p, source offset index d (offsets -1, 0 / 0, +1): -1 for none
    auto s2t = [](int p, int d) { return p == 0 ? (d == 0 ? -1 : 1) : (d == 0 ? 2 : 0); };
    const int kh = s2t(phase >> 1, tap >> 1), kw = s2t(phase & 1, tap & 1);
    if (kh < 0 || kw < 0) return 0.f;
    int k0, k1;  // forward temporal taps summed on this stage
    if (set == 0) { k0 = 0; k1 = dt == 0 ? 2 : 0; }
    else if (set == 1) { k0 = k1 = dt == 0 ? 2 : 0; }
    else { if (dt == 1) return 0.f; k0 = k1 = 1; }
    float v = 0.f;
    for (int kt = k0; kt <= k1; ++kt) v += W(ic, oc, kt, kh, kw);
    return v;
  }
  if (g.mode == CM_UPT) {
    // [ct][set 2][dt 4][chunk][dh*4+dw][o][quad][QE]
    const int tap = (int)(e % 16); e /= 16;
    const int ck = (int)(e % g.chunks); e /= g.chunks;
    const int dt = (int)(e % 4); e /= 4;
    const int set = (int)(e % 2); e /= 2;
    const int ct = (int)e;
    const int row = tap * g.nt + o;
    const int q = pq ^ swz(row);
    const int oc = ct * g.nt + o, ic = ck * g.CH + q * g.QE + x;  // adjoint out / in channels
    if (oc >= g.Cin || ic >= g.Cout) return 0.f;
    // forward taps folded onto fine offset d - 1 around 2 s: d = 0 -> 2, 1 -> 1..2, 2 -> 0..1, 3 -> 0
    auto lo = [](int d) { return d == 0 ? 2 : (d == 1 ? 1 : 0); };
    auto hi = [](int d) { return d <= 1 ? 2 : (d == 2 ? 1 : 0); };
    int t0 = lo(dt), t1 = hi(dt);
    if (set == 0) {  // source frame 0: fine frame dt - 1 collects every tap whose clamped source is 0
      if (dt == 0) return 0.f;
      t0 = 0; t1 = 3 - dt;
    }
    const int dh = tap >> 2, dw = tap & 3;
    float v = 0.f;
    for (int kt = t0; kt <= t1; ++kt)
      for (int kh = lo(dh); kh <= hi(dh); ++kh)
        for (int kw = lo(dw); kw <= hi(dw); ++kw) v += W(ic, oc, kt, kh, kw);
    return v;
  }
  if (g.mode == CM_I2C) {
    // [ct][chunk][o][quad][QE]: K index k = (kt*9 + kh*3 + kw)*4 + c, zero for c = 3 and past 108
    const int ck = (int)(e % g.chunks); e /= g.chunks;
    const int ct = (int)e;
    const int q = pq ^ swz(o);
    const int co = ct * g.nt + o, k = ck * g.CH + q * g.QE + x;
    if (co >= g.Cout || k >= 108 || (k & 3) == 3) return 0.f;
    const int tp = k >> 2;
    return W(co, k & 3, tp / 9, (tp / 3) % 3, tp % 3);
  }
  const int tap = (int)(e % 9); e /= 9;
  const int ck = (int)(e % g.chunks); e /= g.chunks;
  const int kt = (int)(e % 3); e /= 3;  // CM_S1T: gradient frame offset dt
  const int row = tap * g.nt + o;
  const int q = pq ^ swz(row);          // logical quad stored at physical quad pq
  if (g.mode == CM_S1T) {
    const int set = (int)(e % 2); e /= 2;
    const int ct = (int)e;
    const int oc = ct * g.nt + o, ic = ck * g.CH + q * g.QE + x;  // adjoint out / in channels
    if (oc >= g.Cin || ic >= g.Cout) return 0.f;
    const int dt = kt, kh = 2 - tap / 3, kw = 2 - tap % 3;
    float v = 0.f;
    for (int k = (set == 0 ? 2 - dt : 0); k <= 2 - dt; ++k) v += W(ic, oc, k, kh, kw);
    return v;
  }
  const int ct = (int)e;
  const int co = ct * g.nt + o, ci = ck * g.CH + q * g.QE + x;
  if (co >= g.Cout || ci >= g.Cin) return 0.f;
  return W(co, ci, kt, tap / 3, tap % 3);
}

// Per-output-channel fp8 scale: the largest magnitude of the channel's packed
// (possibly folded) kernel / 448, or 1 for an all-zero channel.  One block per
// output channel; its packed elements are, for outer index r (the layout's
// leading dimensions after the tile) and inner index q (quad, element):
//   e = ((ct R + r) nt + o) 4 QE + q.
__global__ void __launch_bounds__(256) wscale_kernel(const float* __restrict__ w, PackGeom g, int R,
                                                      float* __restrict__ scale) {
  __shared__ float red[256];
  const int c = blockIdx.x, ct = c / g.nt, o = c % g.nt;
  const int inner = 4 * g.QE;
  float m = 0.f;
  for (int j = threadIdx.x; j < R * inner; j += 256) {
    const int r = j / inner, q = j % inner;
    const size_t e = (((size_t)ct * R + r) * g.nt + o) * inner + q;
    m = fmaxf(m, fabsf(pack_value(w, g, e)));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) scale[c] = red[0] > 0.f ? red[0] / kFp8Max : 1.f;
}

// Round to nearest even, as the activations' hardware conversion does.
__device__ inline uint16_t bf16_bits_rne(float v) {
  uint32_t u = __float_as_uint(v);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <int PREC>
__global__ void __launch_bounds__(256) pack_kernel(const float* __restrict__ w, PackGeom g, size_t n, void* dst,
                                                    const float* __restrict__ wscale) {
  if constexpr (PREC == P_FP8) {
    // four consecutive elements (same output channel) per thread -> one 32-bit store
    const size_t e = ((size_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (e >= n) return;
    const size_t row = e / (4 * g.QE);  // (ct, r, o) flattened
    const int c = (int)(row / ((size_t)g.R * g.nt)) * g.nt + (int)(row % g.nt);
    float v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = pack_value(w, g, e + k);
    const float inv = c < g.co ? 1.0f / wscale[c] : 0.f;
    reinterpret_cast<uint32_t*>(dst)[e / 4] = pack_fp8x4(v[0] * inv, v[1] * inv, v[2] * inv, v[3] * inv);
  } else {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float v = pack_value(w, g, e);
    if constexpr (PREC == P_BF16) reinterpret_cast<uint16_t*>(dst)[e] = bf16_bits_rne(v);
    else reinterpret_cast<float*>(dst)[e] = v;
  }
}

PackGeom pack_geom(int Cout, int Cin, int prec, int mode, size_t* elems) {
  PackGeom g;
  g.Cout = Cout; g.Cin = Cin; g.mode = mode;
  g.CH = prec == P_BF16 ? 32 : (prec == P_FP8 ? 64 : 16);
  g.QE = g.CH / 4;
  const bool adj = mode == CM_S1T || mode == CM_S2T || mode == CM_UPT;
  const int co = adj ? Cin : Cout;   // the adjoints map Cout channels to Cin channels
  const int ci = adj ? Cout : Cin;
  g.co = co;
  // the upsampling adjoint: 32 channels a tile (LDS); stride 2: 128 when they
  // come in whole tiles (its stages are one kernel row, so 128 fit in LDS)
  g.nt = mode == CM_UPT ? 32 : (mode == CM_S2 && co % 128 == 0 ? 128 : (co >= 64 ? 64 : 16));
  g.chunks = (ci + g.CH - 1) / g.CH;
  if (mode == CM_I2C) g.chunks = kI2cK / g.CH;  // K = 27 taps x 4 channels, padded
  if (mode == CM_UPF) g.R = 2 * 2 * g.chunks * 16;
  else if (mode == CM_S2T) g.R = 3 * 2 * g.chunks * 16;
  else if (mode == CM_UPT) g.R = 2 * 4 * g.chunks * 16;
  else if (mode == CM_S1T) g.R = 2 * 3 * g.chunks * 9;
  else if (mode == CM_I2C) g.R = g.chunks;
  else g.R = 3 * g.chunks * 9;
  const size_t tiles = (size_t)((co + g.nt - 1) / g.nt);
  *elems = tiles * g.R * g.nt * g.CH;
  return g;
}

}  // namespace

size_t packed_conv_elems(int Cout, int Cin, int prec, int mode, int* nt_out) {
  size_t n;
  const PackGeom g = pack_geom(Cout, Cin, prec, mode, &n);
  if (nt_out) *nt_out = g.nt;
  return n;
}

hipError_t launch_pack_weights(const float* w, int Cout, int Cin, int prec, int mode, void* dst, float* wscale,
                               hipStream_t s) {
  size_t n;
  const PackGeom g = pack_geom(Cout, Cin, prec, mode, &n);
  if (prec == P_FP8) {
    if (!wscale || mode == CM_S1T || mode == CM_S2T || mode == CM_UPT) return hipErrorInvalidValue;
    hipLaunchKernelGGL(wscale_kernel, dim3(g.co), dim3(256), 0, s, w, g, g.R, wscale);
    hipLaunchKernelGGL(pack_kernel<P_FP8>, dim3((unsigned)((n / 4 + 255) / 256)), dim3(256), 0, s, w, g, n, dst,
                       (const float*)wscale);
  } else {
    const dim3 grid((unsigned)((n + 255) / 256));
    if (prec == P_BF16) hipLaunchKernelGGL(pack_kernel<P_BF16>, grid, dim3(256), 0, s, w, g, n, dst, nullptr);
    else hipLaunchKernelGGL(pack_kernel<P_F32>, grid, dim3(256), 0, s, w, g, n, dst, nullptr);
  }
  return hipGetLastError();
}

}  // namespace tok
