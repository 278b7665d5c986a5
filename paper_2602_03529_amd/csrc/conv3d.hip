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
#include "tok_internal.h"
#include "tok_device.h"

namespace tok {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = 4;

#ifndef TOK_SWZ_SHIFT
#define TOK_SWZ_SHIFT 1
#endif
__host__ __device__ __forceinline__ int swz(int row) { return (row >> TOK_SWZ_SHIFT) & 3; }

template <int PREC> struct Op;
template <> struct Op<P_F32> { static constexpr int CH = 16; static constexpr int QE = 4; };
template <> struct Op<P_BF16> { static constexpr int CH = 32; static constexpr int QE = 8; };

// Per mode: output tile TH x TW, halo HH x HW (rows x positions), position
// blocks per wave MB, weight tap-matrices per stage WT, temporal stages KTS.
template <int MODE> struct Geo;
template <> struct Geo<CM_S1> {
  static constexpr int WR = 2, TW = 64, TH = 8, HH = TH + 2, HW = TW + 2;
  static constexpr int MB = WR * TW / 16, WT = 9, KTS = 3;
};
template <> struct Geo<CM_S2> {
  static constexpr int WR = 1, TW = 32, TH = 4, HH = 2 * TH + 1, HW = 2 * TW + 1;
  static constexpr int MB = WR * TW / 16, WT = 9, KTS = 3;
};
template <> struct Geo<CM_UP> {
  static constexpr int WR = 2, TW = 64, TH = 8, HH = TH / 2 + 2, HW = TW / 2 + 2;
  static constexpr int MB = WR * TW / 16, WT = 9, KTS = 3;
};
// Polyphase upsample conv: wave w owns output phase (h & 1, w & 1) = (w >> 1, w & 1)
// of the tile, i.e. 4 source rows x 32 source columns = 8 blocks; a stage holds
// the 2 x 2 folded taps of all 4 phases.
template <> struct Geo<CM_UPF> {
  static constexpr int WR = 0, TW = 64, TH = 8, HH = TH / 2 + 2, HW = TW / 2 + 2;
  static constexpr int MB = (TH / 2) * (TW / 2 / 16), WT = 16, KTS = 2;
};

// Output-tile-local position of lane l16 in position block m of a wave.
template <int MODE>
__device__ __forceinline__ void out_local(int wave, int m, int l16, int* i, int* j) {
  using G = Geo<MODE>;
  if constexpr (MODE == CM_UPF) {
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
  if constexpr (MODE == CM_S1) {
    return (i + kh) * G::HW + (j + kw);
  } else if constexpr (MODE == CM_S2) {
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
  if constexpr (MODE == CM_S1) {
    *hs = h0 - 1 + r;
    *ws = w0 - 1 + pc;
  } else if constexpr (MODE == CM_S2) {
    const int c = (pc < G::TW + 1) ? 2 * pc : 2 * (pc - (G::TW + 1)) + 1;
    *hs = 2 * h0 - 1 + r;
    *ws = 2 * w0 - 1 + c;
  } else {  // CM_UP, CM_UPF: source rows / columns of the upsampled tile
    *hs = (h0 >> 1) - 1 + r;
    *ws = (w0 >> 1) - 1 + pc;
  }
}

// 16-byte direct global->LDS load (global_load_lds_dwordx4): lane l of the
// wave writes LDS address lds_wave_base + 16 l.  lds_wave_base must be uniform.
__device__ __forceinline__ void lds_dma16(const uint4* g, uint4* lds_wave_base) {
  __builtin_amdgcn_global_load_lds(g, lds_wave_base, 16, 0, 0);
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

// Map a linear block index to a virtual tile index so that the blocks one XCD
// receives (hardware dispatches block b to XCD b % 8) are contiguous tiles.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, l = b >> 3;
  return x * q + min(x, r) + l;
}

template <int PREC, int MODE, int NB, int IN_KIND, int OUT_KIND, bool RESID, bool STATS, bool DB>
__global__ void __launch_bounds__(kThreads, DB ? 1 : 2) conv3d_kernel(ConvLaunch a) {
  using G = Geo<MODE>;
  using O = Op<PREC>;
  constexpr int NT = NB * 16;           // output channels per workgroup
  constexpr int HALO = G::HH * G::HW;   // halo rows (positions)
  constexpr int MB = G::MB;             // position blocks per wave
  constexpr int HQ = HALO * 4;          // halo quads per stage
  constexpr int WQ = G::WT * NT * 4;    // weight quads per stage
  constexpr int NBUF = DB ? 2 : 1;      // LDS buffers (double buffering: 1 workgroup per CU)
  static_assert(WQ % 64 == 0, "weight stage must be whole waves");
  static_assert(!DB || IN_KIND == IN_ACT, "double buffering needs asynchronous staging");

  __shared__ uint4 lds_a[NBUF][HQ];
  __shared__ uint4 lds_w[NBUF][WQ];
  __shared__ float red[kWaves][32];
  __shared__ float gmean[32];

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

  f32x4 acc[MB][NB];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[m][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  const size_t plane_in = (size_t)a.Hi * a.Wi;
  // Folded weights come in two sets, one per output-frame parity.
  const int tg = a.go0 + to;  // global output frame
  const size_t wset = MODE == CM_UPF ? (size_t)ct * 2 + (tg & 1) : (size_t)ct;
  const uint4* wbase = reinterpret_cast<const uint4*>(a.wpk) + wset * G::KTS * a.in_chunks * WQ;
  const int nstages = G::KTS * a.in_chunks;  // stage = (temporal tap, input chunk)

  // Input buffer frame read by temporal tap kt (causal in global frame
  // numbers: frame 0 repeats for t < 0).
  auto src_frame = [&](int kt) {
    int g;
    if constexpr (MODE == CM_S1) g = max(tg + kt - 2, 0);
    else if constexpr (MODE == CM_S2) g = max(2 * tg + kt - 2, 0);
    else if constexpr (MODE == CM_UP) g = (max(tg + kt - 2, 0) + 1) >> 1;
    else {
      // even output frame 2j reads source frames j-1 (clamped) and j; odd 2j+1 reads j and j+1
      const int jt = tg >> 1;
      g = (tg & 1) ? jt + kt : max(jt - 1 + kt, 0);
    }
    return g - a.gi0;
  };

  // Halo slots this thread's lanes fill are the same in every stage: keep
  // their in-frame quad offsets (or -1 for the zero padding) in registers.
  constexpr int NHS = (HQ + kThreads - 1) / kThreads;
  int hoff[NHS];
#pragma unroll
  for (int k = 0; k < NHS; ++k) {
    const int e = wave * 64 + k * kThreads + lane;
    hoff[k] = -1;
    if (e < HQ) {
      const int p = e >> 2;
      const int q = (e & 3) ^ swz(p);
      int hs, ws;
      halo_src<MODE>(p, h0, w0, &hs, &ws);
      if (hs >= 0 && hs < a.Hi && ws >= 0 && ws < a.Wi) hoff[k] = (hs * a.Wi + ws) * 4 + q;
    }
  }

  // Issue the global->LDS transfers of stage st into buffer buf: the 9 taps of
  // packed weights and the spatial halo, both as direct-to-LDS loads (lane l
  // of a wave writes 16 bytes at the wave's LDS base + 16 l).  Slot (p, pq) of
  // the halo holds logical quad pq ^ swz(p) of halo row p; rows outside the
  // frame are written as zeros (the conv's zero padding).
  auto issue_async = [&](int st, int buf) {
    const int kt = st / a.in_chunks, ck = st - kt * a.in_chunks;
    const uint4* wsrc = wbase + (size_t)st * WQ;
#pragma unroll
    for (int base = wave * 64; base < WQ; base += kThreads) lds_dma16(wsrc + base + lane, &lds_w[buf][base]);
    const uint4* src = reinterpret_cast<const uint4*>(a.in) +
                       (((size_t)n * a.Ti + src_frame(kt)) * a.in_chunks + ck) * plane_in * 4;
#pragma unroll
    for (int k = 0; k < NHS; ++k) {
      const int base = wave * 64 + k * kThreads;
      const int e = base + lane;
      if (e < HQ) {
        if (hoff[k] >= 0) lds_dma16(src + hoff[k], &lds_a[buf][base]);
        else lds_a[buf][e] = make_uint4(0, 0, 0, 0);
      }
    }
  };

  // uint8 RGB input (first layer): x / 127.5 - 1 in channels 0..2 of quad 0,
  // zeros elsewhere; converted in registers, so staged synchronously.
  auto stage_u8 = [&](int st) {
    constexpr int NHQ = (HQ + kThreads - 1) / kThreads;
    const int kt = st / a.in_chunks;
    const uint4* wsrc = wbase + (size_t)st * WQ;
#pragma unroll
    for (int base = wave * 64; base < WQ; base += kThreads) lds_dma16(wsrc + base + lane, &lds_w[0][base]);
    const uint8_t* src = reinterpret_cast<const uint8_t*>(a.in) + ((size_t)n * a.Ti + src_frame(kt)) * plane_in * 3;
    uint32_t px[NHQ];
    uint32_t inb = 0;
#pragma unroll
    for (int k = 0; k < NHQ; ++k) {
      const int e = tid + k * kThreads;
      px[k] = 0;
      if (e < HQ && (e & 3) == 0) {
        int hs, ws;
        halo_src<MODE>(e >> 2, h0, w0, &hs, &ws);
        if (hs >= 0 && hs < a.Hi && ws >= 0 && ws < a.Wi) {
          const uint8_t* pp = src + ((size_t)hs * a.Wi + ws) * 3;
          px[k] = (uint32_t)pp[0] | ((uint32_t)pp[1] << 8) | ((uint32_t)pp[2] << 16);
          inb |= 1u << k;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NHQ; ++k) {
      const int e = tid + k * kThreads;
      if (e < HQ) {
        const int p = e >> 2, q = e & 3;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (inb & (1u << k)) {
          const float r = (float)(px[k] & 0xff) / 127.5f - 1.0f;
          const float g = (float)((px[k] >> 8) & 0xff) / 127.5f - 1.0f;
          const float bch = (float)((px[k] >> 16) & 0xff) / 127.5f - 1.0f;
          if constexpr (PREC == P_BF16) val = make_uint4(pack_bf16(r, g), pack_bf16(bch, 0.f), 0, 0);
          else val = make_uint4(__float_as_uint(r), __float_as_uint(g), __float_as_uint(bch), 0);
        }
        lds_a[0][p * 4 + (q ^ swz(p))] = val;
      }
    }
  };

  // The 9 spatial taps of one stage: every wave multiplies its MB position
  // blocks by the NB output-channel blocks.
  auto compute = [&](int buf) {
    if constexpr (MODE == CM_UPF) {
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
    constexpr int BPR = G::TW / 16;
#pragma unroll 1
    for (int kh = 0; kh < 3; ++kh) {
#pragma unroll
      for (int kw = 0; kw < 3; ++kw) {
        const int tap = kh * 3 + kw;
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

  if constexpr (DB) {
    issue_async(0, 0);
    for (int st = 0; st < nstages; ++st) {
      // stage st has landed in buffer st & 1, and every wave is done with
      // stage st - 1, whose buffer the next transfers overwrite
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
      if (st + 1 < nstages) issue_async(st + 1, (st + 1) & 1);
      compute(st & 1);
    }
  } else {
    for (int st = 0; st < nstages; ++st) {
      __syncthreads();
      if constexpr (IN_KIND == IN_ACT) issue_async(st, 0);
      else stage_u8(st);
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

#pragma unroll
  for (int m = 0; m < MB; ++m) {
    int i, j;
    out_local<MODE>(wave, m, l16, &i, &j);
    const int oh = h0 + i, ow = w0 + j;
    const bool valid = (oh < a.Ho) && (ow < a.Wo);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int c0 = ct * NT + b * 16 + 4 * g4;
      float v4[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) v4[r] = acc[m][b][r] + ((c0 + r) < a.Cout ? a.bias[c0 + r] : 0.f);
      if constexpr (OUT_KIND == OUT_ACT) {
        const int chunk = c0 / O::CH, within = c0 % O::CH;
        const size_t off = (((size_t)n * a.To_buf + a.out_f0 + to) * a.out_chunks + chunk) * plane_out * kChunkBytes +
                           ((size_t)oh * a.Wo + ow) * kChunkBytes + (size_t)within * (kChunkBytes / O::CH);
        if constexpr (PREC == P_BF16) {
          if (valid) {
            if constexpr (RESID) {
              const uint2 rv = *reinterpret_cast<const uint2*>(reinterpret_cast<const char*>(a.resid) + off);
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
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        s_lo[b] += __shfl_xor(s_lo[b], off);
        s_hi[b] += __shfl_xor(s_hi[b], off);
      }
      if (l16 == 0) {
        red[wave][b * 8 + 2 * g4] = s_lo[b];
        red[wave][b * 8 + 2 * g4 + 1] = s_hi[b];
      }
    }
    __syncthreads();
    if (tid < 32) gmean[tid] = (((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid]) / cnt;
    __syncthreads();
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
      s_lo[b] = qa;
      s_hi[b] = qb;
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        s_lo[b] += __shfl_xor(s_lo[b], off);
        s_hi[b] += __shfl_xor(s_hi[b], off);
      }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (l16 == 0) {
        red[wave][b * 8 + 2 * g4] = s_lo[b];
        red[wave][b * 8 + 2 * g4 + 1] = s_hi[b];
      }
    }
    __syncthreads();
    if (tid < 32) {
      const float m2 = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
      const int tiles = a.tiles_h * a.tiles_w;
      a.stats[(((size_t)n * a.To + to) * tiles + (size_t)th * a.tiles_w + tw) * 32 + tid] =
          make_float4(cnt, gmean[tid], m2, 0.f);
    }
  }
}

template <int PREC, int MODE, int NB, int IN_KIND, int OUT_KIND, bool RESID, bool STATS, bool DB = false>
hipError_t launch_one(const ConvLaunch& a, hipStream_t s) {
  const long long nb = (long long)a.N * a.To * a.tiles_h * a.tiles_w * a.cout_tiles;
  if (nb <= 0 || nb > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((conv3d_kernel<PREC, MODE, NB, IN_KIND, OUT_KIND, RESID, STATS, DB>),
                     dim3((unsigned)nb), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

#ifndef TOK_CONV_DB
#define TOK_CONV_DB 0
#endif
constexpr bool kDB = TOK_CONV_DB != 0;

template <int PREC>
hipError_t dispatch_prec(const ConvLaunch& a, hipStream_t s) {
  // The configurations the tokenizer uses.
  const bool res = a.resid != nullptr, st = a.stats != nullptr;
  if (a.in_kind == IN_U8) {
    if (a.mode == CM_S1 && a.nt == 64 && a.out_kind == OUT_ACT && !res && st)
      return launch_one<PREC, CM_S1, 4, IN_U8, OUT_ACT, false, true>(a, s);
    return hipErrorInvalidValue;
  }
  if (a.out_kind == OUT_RGB32) {
    if (a.mode == CM_S1 && a.nt == 16 && !res && !st)
      return launch_one<PREC, CM_S1, 1, IN_ACT, OUT_RGB32, false, false, kDB>(a, s);
    return hipErrorInvalidValue;
  }
  if (a.nt != 64) return hipErrorInvalidValue;
  if (a.mode == CM_S1) {
    if (!res && st) return launch_one<PREC, CM_S1, 4, IN_ACT, OUT_ACT, false, true, kDB>(a, s);
    if (res && st) return launch_one<PREC, CM_S1, 4, IN_ACT, OUT_ACT, true, true, kDB>(a, s);
    if (res && !st) return launch_one<PREC, CM_S1, 4, IN_ACT, OUT_ACT, true, false, kDB>(a, s);
    if (!res && !st) return launch_one<PREC, CM_S1, 4, IN_ACT, OUT_ACT, false, false, kDB>(a, s);
    return hipErrorInvalidValue;
  }
  if (a.mode == CM_S2) {
    if (!res && !st) return launch_one<PREC, CM_S2, 4, IN_ACT, OUT_ACT, false, false, kDB>(a, s);
    return hipErrorInvalidValue;
  }
  if (a.mode == CM_UP) {
    if (!res && !st) return launch_one<PREC, CM_UP, 4, IN_ACT, OUT_ACT, false, false, kDB>(a, s);
    if (!res && st) return launch_one<PREC, CM_UP, 4, IN_ACT, OUT_ACT, false, true, kDB>(a, s);
    return hipErrorInvalidValue;
  }
  if (a.mode == CM_UPF) {
    if (!res && !st) return launch_one<PREC, CM_UPF, 4, IN_ACT, OUT_ACT, false, false, kDB>(a, s);
    if (!res && st) return launch_one<PREC, CM_UPF, 4, IN_ACT, OUT_ACT, false, true, kDB>(a, s);
    return hipErrorInvalidValue;
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_conv(const ConvLaunch& a, hipStream_t s) {
  if (a.stats && !(a.nt == 64 && a.Cout == 64 && a.cout_tiles == 1)) return hipErrorInvalidValue;
  if (a.prec == P_BF16) return dispatch_prec<P_BF16>(a, s);
  if (a.prec == P_F32) return dispatch_prec<P_F32>(a, s);
  return hipErrorInvalidValue;
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
namespace {
int fold_lo(int parity, int d) { return parity == 0 ? (d == 0 ? 0 : 1) : (d == 0 ? 0 : 2); }
int fold_hi(int parity, int d) { return parity == 0 ? (d == 0 ? 0 : 2) : (d == 0 ? 1 : 2); }

void store_elem(void* dst, size_t e, float v, int prec) {
  if (prec == P_BF16) {
    uint32_t u;
    __builtin_memcpy(&u, &v, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    reinterpret_cast<uint16_t*>(dst)[e] = (uint16_t)(u >> 16);
  } else {
    reinterpret_cast<float*>(dst)[e] = v;
  }
}
}  // namespace

size_t packed_conv_elems(int Cout, int Cin, int prec, int mode, int* nt_out) {
  const int CH = prec == P_BF16 ? 32 : 16;
  const int nt = Cout >= 64 ? 64 : 16;
  const int tiles = (Cout + nt - 1) / nt;
  const int chunks = (Cin + CH - 1) / CH;
  if (nt_out) *nt_out = nt;
  if (mode == CM_UPF) return (size_t)tiles * 2 * 2 * chunks * 16 * nt * CH;
  return (size_t)tiles * 3 * chunks * 9 * nt * CH;
}

void pack_conv_weights(const float* w, int Cout, int Cin, int prec, int mode, void* dst) {
  const int CH = prec == P_BF16 ? 32 : 16;
  const int QE = CH / 4;
  int nt;
  packed_conv_elems(Cout, Cin, prec, mode, &nt);
  const int tiles = (Cout + nt - 1) / nt;
  const int chunks = (Cin + CH - 1) / CH;
  auto W = [&](int co, int ci, int kt, int kh, int kw) -> float {
    if (co >= Cout || ci >= Cin) return 0.f;
    return w[((((size_t)co * Cin + ci) * 3 + kt) * 3 + kh) * 3 + kw];
  };
  size_t e = 0;
  if (mode == CM_UPF) {
    for (int ct = 0; ct < tiles; ++ct)
      for (int pt = 0; pt < 2; ++pt)
        for (int dt = 0; dt < 2; ++dt)
          for (int ck = 0; ck < chunks; ++ck)
            for (int phase = 0; phase < 4; ++phase)
              for (int tap = 0; tap < 4; ++tap)
                for (int o = 0; o < nt; ++o)
                  for (int pq = 0; pq < 4; ++pq)
                    for (int x = 0; x < QE; ++x, ++e) {
                      const int row = (phase * 4 + tap) * nt + o;
                      const int q = pq ^ swz(row);
                      const int co = ct * nt + o, ci = ck * CH + q * QE + x;
                      const int ph = phase >> 1, pw = phase & 1, dh = tap >> 1, dw = tap & 1;
                      float v = 0.f;
                      for (int kt = fold_lo(pt, dt); kt <= fold_hi(pt, dt); ++kt)
                        for (int kh = fold_lo(ph, dh); kh <= fold_hi(ph, dh); ++kh)
                          for (int kw = fold_lo(pw, dw); kw <= fold_hi(pw, dw); ++kw) v += W(co, ci, kt, kh, kw);
                      store_elem(dst, e, v, prec);
                    }
    return;
  }
  for (int ct = 0; ct < tiles; ++ct)
    for (int kt = 0; kt < 3; ++kt)
      for (int ck = 0; ck < chunks; ++ck)
        for (int tap = 0; tap < 9; ++tap)
          for (int o = 0; o < nt; ++o)
            for (int pq = 0; pq < 4; ++pq)
              for (int x = 0; x < QE; ++x, ++e) {
                const int row = tap * nt + o;
                const int q = pq ^ swz(row);  // logical quad stored at physical quad pq
                store_elem(dst, e, W(ct * nt + o, ck * CH + q * QE + x, kt, tap / 3, tap % 3), prec);
              }
}

}  // namespace tok
