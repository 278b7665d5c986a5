// Memory-bound kernels of the tokenizer path: GroupNorm statistics merge,
// the 1x1x1 latent projections, finite scalar quantisation and token
// dropping with zero fill (Sec. 6.2: dropped and lost tokens are both zeros).
#include "tok_internal.h"
#include "tok_device.h"

namespace tok {

namespace {

// ---------------------------------------------------------------------------
// GroupNorm finalize.  One wave per (frame (n, t), group), four groups per
// block, eight blocks per frame.  Lane j of group g merges tiles j, j+64, ...
// with Chan's pairwise update, then the 64 lane results are merged in a fixed
// butterfly order, so the result is deterministic and independent of the
// launch order of the producing conv's workgroups.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void chan_merge(float& n, float& m, float& q, float nb, float mb, float qb) {
  if (nb == 0.f) return;
  if (n == 0.f) { n = nb; m = mb; q = qb; return; }
  const float tot = n + nb;
  const float d = mb - m;
  const float f = nb / tot;
  m = m + d * f;
  q = q + qb + d * d * n * f;
  n = tot;
}

__global__ void __launch_bounds__(256) gn_finalize_kernel(const float4* __restrict__ stats, int tiles,
                                                           const float* __restrict__ gamma,
                                                           const float* __restrict__ beta, float eps,
                                                           float* __restrict__ scale,
                                                           float* __restrict__ shift,
                                                           float2* __restrict__ mr) {
  const int frame = blockIdx.x >> 3;
  const int g = ((blockIdx.x & 7) << 2) + (threadIdx.x >> 6), j = threadIdx.x & 63;
  const float4* s = stats + (size_t)frame * tiles * 32;
  float n = 0.f, m = 0.f, q = 0.f;
#pragma unroll 4
  for (int t = j; t < tiles; t += 64) {
    const float4 p = s[(size_t)t * 32 + g];
    chan_merge(n, m, q, p.x, p.y, p.z);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const float nb = __shfl_xor(n, off), mb = __shfl_xor(m, off), qb = __shfl_xor(q, off);
    // lower lane keeps itself as the left operand: same order on every lane pair
    if ((j & off) == 0) chan_merge(n, m, q, nb, mb, qb);
    else {
      float n2 = nb, m2 = mb, q2 = qb;
      chan_merge(n2, m2, q2, n, m, q);
      n = n2; m = m2; q = q2;
    }
  }
  if (j < 2) {
    const int c = 2 * g + j;
    const float var = q / n;
    const float rstd = 1.0f / sqrtf(var + eps);
    if (mr && j == 0) mr[(size_t)frame * 32 + g] = make_float2(m, rstd);
    if (!gamma) return;  // statistics only
    const float sc = rstd * gamma[c];
    scale[(size_t)frame * 64 + c] = sc;
    shift[(size_t)frame * 64 + c] = beta[c] - m * sc;
  }
}

// ---------------------------------------------------------------------------
// GroupNorm apply + SiLU, elementwise over a level-0 tensor (64 channels).
// blockIdx.y = frame * chunks + chunk; every thread handles kItems 16-byte
// quads of that plane, kThreads apart, so each load / store instruction is
// fully coalesced and all quads of a thread share one channel set.
// ---------------------------------------------------------------------------
constexpr int kActItems = 4;

template <int PREC>
__global__ void __launch_bounds__(256) gn_act_kernel(const uint4* in, int in_Tb, int in_f0,
                                                      uint4* out, int out_Tb, int out_f0,  // may alias (in place)
                                                      int F, int HW, const float* __restrict__ scale,
                                                      const float* __restrict__ shift) {
  constexpr int CH = PREC == P_BF16 ? 32 : 16;
  constexpr int QE = CH / 4;
  constexpr int CHUNKS = 64 / CH;
  const int frame = blockIdx.y / CHUNKS, ck = blockIdx.y % CHUNKS;  // frame = n * F + f
  const int n = frame / F, f = frame % F;
  const size_t fi = ((size_t)n * in_Tb + in_f0 + f) * CHUNKS + ck;    // input (frame, chunk) plane
  const size_t fo = ((size_t)n * out_Tb + out_f0 + f) * CHUNKS + ck;  // output plane
  const size_t plane = (size_t)HW * 4;  // quads per (frame, chunk)
  const size_t q0 = (size_t)blockIdx.x * (256 * kActItems) + threadIdx.x;
  const int c0 = ck * CH + (threadIdx.x & 3) * QE;
  float sc[QE], sh[QE];
#pragma unroll
  for (int c = 0; c < QE; ++c) {
    sc[c] = scale[(size_t)frame * 64 + c0 + c];
    sh[c] = shift[(size_t)frame * 64 + c0 + c];
  }
  const uint4* src = in + fi * plane;
  uint4* dst = out + fo * plane;
  uint4 v[kActItems];
#pragma unroll
  for (int k = 0; k < kActItems; ++k) {
    const size_t q = q0 + (size_t)k * 256;
    if (q < plane) v[k] = src[q];
  }
#pragma unroll
  for (int k = 0; k < kActItems; ++k) {
    const size_t q = q0 + (size_t)k * 256;
    if (q >= plane) continue;
    uint32_t u[4] = {v[k].x, v[k].y, v[k].z, v[k].w};
    uint32_t o[4];
    if constexpr (PREC == P_BF16) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        o[j] = pack_bf16(silu_f(fmaf(bf16_lo(u[j]), sc[2 * j], sh[2 * j])),
                         silu_f(fmaf(bf16_hi(u[j]), sc[2 * j + 1], sh[2 * j + 1])));
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) o[j] = __float_as_uint(silu_f(fmaf(__uint_as_float(u[j]), sc[j], sh[j])));
    }
    dst[q] = make_uint4(o[0], o[1], o[2], o[3]);
  }
}

// ---------------------------------------------------------------------------
// FSQ (Mentzer et al.): b = tanh(z + s) h - o; q = rint(b) (half to even);
// codes = q / floor(L/2); idx = sum (q + floor(L/2)) * basis.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void fsq6(const float z[6], const FsqConst& fc, float codes[6], int* idx) {
  int id = 0;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const float b = tanhf(z[c] + fc.s[c]) * fc.h[c] - fc.o[c];
    const float q = rintf(b);
    codes[c] = q * fc.inv_d[c];
    id += ((int)q + (int)fc.d[c]) * fc.basis[c];
  }
  *idx = id;
}

__device__ __forceinline__ uint8_t keep_bit(const DropArgs& d, int n, int t, int h, int w, int T2, int H2,
                                            int W2) {
  if (d.mode == 0) return 1;
  if (d.protect_iframe && t == 0) return 1;
  const size_t tok = (((size_t)n * T2 + t) * H2 + h) * W2 + w;
  if (d.mode == 3) return d.ext_keep[tok] != 0;
  const uint64_t base = d.seed ^ ((d.clip_id0 + (uint64_t)n) * 0x9E3779B97F4A7C15ull);
  uint64_t key;
  if (d.mode == 1) key = ((uint64_t)t * H2 + h) * W2 + w;
  else key = 0x5A5A5A5A00000000ull | ((uint64_t)t * H2 + h);
  const uint32_t u = (uint32_t)(splitmix64(base ^ key) >> 40);
  return u >= d.thr ? 1 : 0;
}

// Level-2 activations (chunked, 128 ch) -> z (6) -> FSQ -> mask.  One thread
// per token; the 6 x 128 projection lives in LDS.
template <int PREC>
__global__ void __launch_bounds__(256) proj_fsq_kernel(const void* __restrict__ act, int N, int Tb, int f0, int F,
                                                        int T2, int t0, int H2, int W2, int in_chunks,
                                                        const float* __restrict__ wp, const float* __restrict__ bp,
                                                        FsqConst fc, DropArgs d, float* __restrict__ z,
                                                        float* __restrict__ codes, int32_t* __restrict__ idx,
                                                        uint8_t* __restrict__ keep) {
  constexpr int CH = PREC == P_BF16 ? 32 : 16;
  __shared__ float w[6 * 128];
  for (int e = threadIdx.x; e < 6 * 128; e += blockDim.x) w[e] = wp[e];
  __syncthreads();
  const size_t HW = (size_t)H2 * W2;
  const size_t ntok = (size_t)N * F * HW;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= ntok) return;
  const size_t nf = gid / HW, hw = gid % HW;
  const int n = (int)(nf / F), f = (int)(nf % F);
  const int t = t0 + f;                                   // global latent frame
  const size_t frame = (size_t)n * Tb + f0 + f;           // activation buffer frame
  const size_t tok = ((size_t)n * T2 + t) * HW + hw;      // dense output token
  float acc[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) acc[c] = bp[c];
  for (int ck = 0; ck < in_chunks; ++ck) {
    const char* base = reinterpret_cast<const char*>(act) + ((frame * in_chunks + ck) * HW + hw) * kChunkBytes;
#pragma unroll
    for (int qd = 0; qd < 4; ++qd) {
      const uint4 v = reinterpret_cast<const uint4*>(base)[qd];
      float x[8];
      int ne;
      if constexpr (PREC == P_BF16) {
        x[0] = bf16_lo(v.x); x[1] = bf16_hi(v.x); x[2] = bf16_lo(v.y); x[3] = bf16_hi(v.y);
        x[4] = bf16_lo(v.z); x[5] = bf16_hi(v.z); x[6] = bf16_lo(v.w); x[7] = bf16_hi(v.w);
        ne = 8;
      } else {
        x[0] = __uint_as_float(v.x); x[1] = __uint_as_float(v.y);
        x[2] = __uint_as_float(v.z); x[3] = __uint_as_float(v.w);
        ne = 4;
      }
      const int c0 = ck * CH + qd * ne;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if (e < ne) {
#pragma unroll
          for (int c = 0; c < 6; ++c) acc[c] = fmaf(w[c * 128 + c0 + e], x[e], acc[c]);
        }
      }
    }
  }
  float cd[6];
  int id;
  fsq6(acc, fc, cd, &id);
  const int h = (int)(hw / W2), ww = (int)(hw % W2);
  const uint8_t k = keep_bit(d, n, t, h, ww, T2, H2, W2);
  if (z) {
#pragma unroll
    for (int c = 0; c < 6; ++c) z[tok * 6 + c] = acc[c];
  }
  if (codes) {
#pragma unroll
    for (int c = 0; c < 6; ++c) codes[tok * 6 + c] = k ? cd[c] : 0.f;
  }
  if (idx) idx[tok] = id;
  if (keep) keep[tok] = k;
}

__global__ void __launch_bounds__(256) quantize_kernel(const float* __restrict__ z, size_t n, FsqConst fc,
                                                        float* __restrict__ codes, int32_t* __restrict__ idx) {
  const size_t tok = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tok >= n) return;
  float zz[6], cd[6];
  int id;
#pragma unroll
  for (int c = 0; c < 6; ++c) zz[c] = z[tok * 6 + c];
  fsq6(zz, fc, cd, &id);
  if (codes) {
#pragma unroll
    for (int c = 0; c < 6; ++c) codes[tok * 6 + c] = cd[c];
  }
  if (idx) idx[tok] = id;
}

__global__ void __launch_bounds__(256) drop_kernel(DropArgs d, float* __restrict__ codes,
                                                    uint8_t* __restrict__ keep, int N, int T2, int H2, int W2) {
  const size_t ntok = (size_t)N * T2 * H2 * W2;
  const size_t tok = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tok >= ntok) return;
  const int ww = (int)(tok % W2);
  size_t r = tok / W2;
  const int h = (int)(r % H2);
  r /= H2;
  const int t = (int)(r % T2);
  const int n = (int)(r / T2);
  const uint8_t k = keep_bit(d, n, t, h, ww, T2, H2, W2);
  if (keep) keep[tok] = k;
  if (codes && !k) {
#pragma unroll
    for (int c = 0; c < 6; ++c) codes[tok * 6 + c] = 0.f;
  }
}

// codes (6) -> 128 channels; one thread per (token, chunk) writes 64 bytes.
template <int PREC>
__global__ void __launch_bounds__(256) proj_in_kernel(const float* __restrict__ codes, int N, int T2, int t0, int F,
                                                       int HW, const float* __restrict__ wpin,
                                                       const float* __restrict__ bpin, void* __restrict__ out,
                                                       int out_chunks, int Tb, int f0) {
  constexpr int CH = PREC == P_BF16 ? 32 : 16;
  __shared__ float w[128 * 6];
  __shared__ float bsh[128];
  for (int e = threadIdx.x; e < 128 * 6; e += blockDim.x) w[e] = wpin[e];
  for (int e = threadIdx.x; e < 128; e += blockDim.x) bsh[e] = bpin[e];
  __syncthreads();
  const size_t ntok = (size_t)N * F * HW;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= ntok * out_chunks) return;
  const size_t lt = gid / out_chunks;  // (n, f, hw)
  const int ck = (int)(gid % out_chunks);
  const size_t nf = lt / HW, hw = lt % HW;
  const int n = (int)(nf / F), f = (int)(nf % F);
  const size_t tok = ((size_t)n * T2 + t0 + f) * HW + hw;  // dense input token
  const size_t frame = (size_t)n * Tb + f0 + f;            // output buffer frame
  float c6[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) c6[c] = codes[tok * 6 + c];
  float y[CH];
#pragma unroll
  for (int e = 0; e < CH; ++e) {
    const int o = ck * CH + e;
    float a = bsh[o];
#pragma unroll
    for (int c = 0; c < 6; ++c) a = fmaf(w[o * 6 + c], c6[c], a);
    y[e] = a;
  }
  uint4* dst = reinterpret_cast<uint4*>(reinterpret_cast<char*>(out) +
                                        ((frame * out_chunks + ck) * HW + hw) * kChunkBytes);
#pragma unroll
  for (int qd = 0; qd < 4; ++qd) {
    if constexpr (PREC == P_BF16) {
      dst[qd] = make_uint4(pack_bf16(y[qd * 8 + 0], y[qd * 8 + 1]), pack_bf16(y[qd * 8 + 2], y[qd * 8 + 3]),
                           pack_bf16(y[qd * 8 + 4], y[qd * 8 + 5]), pack_bf16(y[qd * 8 + 6], y[qd * 8 + 7]));
    } else {
      dst[qd] = make_uint4(__float_as_uint(y[qd * 4 + 0]), __float_as_uint(y[qd * 4 + 1]),
                           __float_as_uint(y[qd * 4 + 2]), __float_as_uint(y[qd * 4 + 3]));
    }
  }
}

// ---------------------------------------------------------------------------
// MX-FP8 producers.  One thread per (position, 32-channel block): compute the
// 32 values, take their largest magnitude, pick the block's E8M0 scale
// 2^e (smallest with max * 2^-e <= 448), and store 32 e4m3 bytes plus the
// scale byte.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void store_fp8_block(const float* v, uint8_t* dst, uint8_t* sdst) {
  float am = 0.f;
#pragma unroll
  for (int k = 0; k < 32; ++k) am = fmaxf(am, fabsf(v[k]));
  const int e = fp8_block_exp(am);
  const float f = ldexpf(1.0f, -e);
  uint32_t w[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) w[k] = pack_fp8x4(v[4 * k] * f, v[4 * k + 1] * f, v[4 * k + 2] * f, v[4 * k + 3] * f);
  reinterpret_cast<uint4*>(dst)[0] = make_uint4(w[0], w[1], w[2], w[3]);
  reinterpret_cast<uint4*>(dst)[1] = make_uint4(w[4], w[5], w[6], w[7]);
  *sdst = (uint8_t)(e + 127);
}

// y = silu(x * scale + shift): bf16 level-0 activations (64 channels, 2
// chunks of 32) -> MX-FP8 (1 chunk of 64 + 2 scale bytes per position).
// Eight lanes per position: lanes 0-3 hold the four 8-channel quads of input
// chunk 0 (output channels 0-31, the first MX block), lanes 4-7 those of chunk
// 1; a block's maximum is reduced over its 4 lanes by shuffles, and lane 0
// stores both scale bytes.  Each thread keeps its 8 channels' scale and shift
// in registers for kF8Items positions, 32 positions apart.
constexpr int kF8Items = 4;
__global__ void __launch_bounds__(256) gn_act_fp8_kernel(const uint4* __restrict__ in, int in_Tb, int in_f0,
                                                          uint8_t* __restrict__ out, uint8_t* __restrict__ osc,
                                                          int out_Tb, int out_f0, int F, int HW,
                                                          const float* __restrict__ scale,
                                                          const float* __restrict__ shift) {
  const int nf = blockIdx.y;  // (n, f)
  const int n = nf / F, f = nf % F;
  const int sub = threadIdx.x & 7, blk = sub >> 2, qq = sub & 3;
  const size_t fin = (size_t)n * in_Tb + in_f0 + f, fout = (size_t)n * out_Tb + out_f0 + f;
  const int c0 = blk * 32 + qq * 8;
  const float4* ps = reinterpret_cast<const float4*>(scale + (size_t)nf * 64 + c0);
  const float4* ph = reinterpret_cast<const float4*>(shift + (size_t)nf * 64 + c0);
  const float4 s0 = ps[0], s1 = ps[1], h0 = ph[0], h1 = ph[1];
  const float sc[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
  const float sh[8] = {h0.x, h0.y, h0.z, h0.w, h1.x, h1.y, h1.z, h1.w};
  const int p0 = blockIdx.x * (32 * kF8Items) + (threadIdx.x >> 3);
  const uint4* src = in + (fin * 2 + blk) * (size_t)HW * 4 + qq;
  uint4 u[kF8Items];
#pragma unroll
  for (int k = 0; k < kF8Items; ++k) {
    const int pos = p0 + 32 * k;
    u[k] = pos < HW ? src[(size_t)pos * 4] : make_uint4(0u, 0u, 0u, 0u);
  }
#pragma unroll
  for (int k = 0; k < kF8Items; ++k) {
    const int pos = p0 + 32 * k;
    const uint32_t w4[4] = {u[k].x, u[k].y, u[k].z, u[k].w};
    float v[8];
    float am = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      v[2 * j] = silu_f(bf16_lo(w4[j]) * sc[2 * j] + sh[2 * j]);
      v[2 * j + 1] = silu_f(bf16_hi(w4[j]) * sc[2 * j + 1] + sh[2 * j + 1]);
      am = fmaxf(am, fmaxf(fabsf(v[2 * j]), fabsf(v[2 * j + 1])));
    }
    am = fmaxf(am, __shfl_xor(am, 1));
    am = fmaxf(am, __shfl_xor(am, 2));
    const int e = fp8_block_exp(am);
    const int e_other = __shfl_xor(e, 4);  // the other block's exponent (lane 0: block 1's)
    const float fs = ldexpf(1.0f, -e);
    if (pos < HW) {
      const uint2 o = make_uint2(pack_fp8x4(v[0] * fs, v[1] * fs, v[2] * fs, v[3] * fs),
                                 pack_fp8x4(v[4] * fs, v[5] * fs, v[6] * fs, v[7] * fs));
      *reinterpret_cast<uint2*>(out + (fout * HW + pos) * kChunkBytes + c0) = o;
      if (sub == 0)
        reinterpret_cast<uint16_t*>(osc)[fout * HW + pos] = (uint16_t)((e + 127) | ((e_other + 127) << 8));
    }
  }
}

// codes (6) -> 128 channels of MX-FP8 (2 chunks, 4 scale bytes per position).
__global__ void __launch_bounds__(256) proj_in_fp8_kernel(const float* __restrict__ codes, int N, int T2, int t0,
                                                           int F, int HW, const float* __restrict__ wpin,
                                                           const float* __restrict__ bpin, uint8_t* __restrict__ out,
                                                           uint8_t* __restrict__ osc, int Tb, int f0) {
  __shared__ float w[128 * 6];
  __shared__ float bsh[128];
  for (int e = threadIdx.x; e < 128 * 6; e += blockDim.x) w[e] = wpin[e];
  for (int e = threadIdx.x; e < 128; e += blockDim.x) bsh[e] = bpin[e];
  __syncthreads();
  const size_t ntok = (size_t)N * F * HW;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= ntok * 4) return;
  const size_t lt = gid / 4;
  const int blk = (int)(gid % 4);  // 32-channel block: chunk blk / 2, half blk % 2
  const size_t nf = lt / HW, hw = lt % HW;
  const int n = (int)(nf / F), f = (int)(nf % F);
  const size_t tok = ((size_t)n * T2 + t0 + f) * HW + hw;
  const size_t frame = (size_t)n * Tb + f0 + f;
  float c6[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) c6[c] = codes[tok * 6 + c];
  float y[32];
#pragma unroll
  for (int e = 0; e < 32; ++e) {
    const int o = blk * 32 + e;
    float a = bsh[o];
#pragma unroll
    for (int c = 0; c < 6; ++c) a = fmaf(w[o * 6 + c], c6[c], a);
    y[e] = a;
  }
  const size_t ck = frame * 2 + blk / 2;
  store_fp8_block(y, out + (ck * HW + hw) * kChunkBytes + (blk % 2) * 32, osc + (ck * HW + hw) * 2 + (blk % 2));
}

inline unsigned blocks_for(size_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_gn_finalize(const float4* stats, int frames, int tiles, const float* gamma, const float* beta,
                              float eps, float* scale, float* shift, float2* mr, hipStream_t s) {
  if (frames < 1 || frames > (1 << 27)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gn_finalize_kernel, dim3(frames * 8), dim3(256), 0, s, stats, tiles, gamma, beta, eps, scale,
                     shift, mr);
  return hipGetLastError();
}

hipError_t launch_gn_act(const void* in, int in_Tb, int in_f0, void* out, int out_Tb, int out_f0, int prec, int N,
                         int F, int HW, const float* scale, const float* shift, hipStream_t s) {
  const int chunks = prec == P_BF16 ? 2 : 4;
  const long long frames = (long long)N * F;
  if (frames * chunks > 65535 || F < 1 || in_f0 < 0 || in_f0 + F > in_Tb || out_f0 < 0 || out_f0 + F > out_Tb)
    return hipErrorInvalidValue;
  const dim3 grid(blocks_for((size_t)HW * 4, 256 * kActItems), (unsigned)(frames * chunks));
  if (prec == P_BF16)
    hipLaunchKernelGGL(gn_act_kernel<P_BF16>, grid, dim3(256), 0, s, reinterpret_cast<const uint4*>(in), in_Tb, in_f0,
                       reinterpret_cast<uint4*>(out), out_Tb, out_f0, F, HW, scale, shift);
  else
    hipLaunchKernelGGL(gn_act_kernel<P_F32>, grid, dim3(256), 0, s, reinterpret_cast<const uint4*>(in), in_Tb, in_f0,
                       reinterpret_cast<uint4*>(out), out_Tb, out_f0, F, HW, scale, shift);
  return hipGetLastError();
}

hipError_t launch_gn_act_fp8(const void* in, int in_Tb, int in_f0, uint8_t* out, uint8_t* out_scale, int out_Tb,
                             int out_f0, int N, int F, int HW, const float* scale, const float* shift, hipStream_t s) {
  const long long frames = (long long)N * F;
  if (frames > 65535 || F < 1 || in_f0 < 0 || in_f0 + F > in_Tb || out_f0 < 0 || out_f0 + F > out_Tb)
    return hipErrorInvalidValue;
  const dim3 grid(blocks_for((size_t)HW, 32 * kF8Items), (unsigned)frames);
  hipLaunchKernelGGL(gn_act_fp8_kernel, grid, dim3(256), 0, s, reinterpret_cast<const uint4*>(in), in_Tb, in_f0, out,
                     out_scale, out_Tb, out_f0, F, HW, scale, shift);
  return hipGetLastError();
}

hipError_t launch_proj_in_fp8(const float* codes, int N, int T2, int t0, int F, int HW, const float* w, const float* b,
                              uint8_t* out, uint8_t* out_scale, int Tb, int f0, hipStream_t s) {
  const size_t n = (size_t)N * F * HW * 4;
  hipLaunchKernelGGL(proj_in_fp8_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, codes, N, T2, t0, F, HW, w, b, out,
                     out_scale, Tb, f0);
  return hipGetLastError();
}

hipError_t launch_proj_fsq(const void* act, int prec, int N, int Tb, int f0, int F, int T2, int t0, int H2, int W2,
                           int in_chunks, const float* wp, const float* bp, const FsqConst& fc, const DropArgs& d,
                           float* z, float* codes, int32_t* idx, uint8_t* keep, hipStream_t s) {
  const size_t ntok = (size_t)N * F * H2 * W2;
  if (prec == P_BF16)
    hipLaunchKernelGGL(proj_fsq_kernel<P_BF16>, dim3(blocks_for(ntok, 256)), dim3(256), 0, s, act, N, Tb, f0, F, T2,
                       t0, H2, W2, in_chunks, wp, bp, fc, d, z, codes, idx, keep);
  else
    hipLaunchKernelGGL(proj_fsq_kernel<P_F32>, dim3(blocks_for(ntok, 256)), dim3(256), 0, s, act, N, Tb, f0, F, T2,
                       t0, H2, W2, in_chunks, wp, bp, fc, d, z, codes, idx, keep);
  return hipGetLastError();
}

hipError_t launch_quantize(const float* z, size_t n, const FsqConst& fc, float* codes, int32_t* idx,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(quantize_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, z, n, fc, codes, idx);
  return hipGetLastError();
}

hipError_t launch_drop(const DropArgs& d, float* codes, uint8_t* keep, int N, int T2, int H2, int W2,
                       hipStream_t s) {
  const size_t ntok = (size_t)N * T2 * H2 * W2;
  hipLaunchKernelGGL(drop_kernel, dim3(blocks_for(ntok, 256)), dim3(256), 0, s, d, codes, keep, N, T2, H2, W2);
  return hipGetLastError();
}

hipError_t launch_proj_in(const float* codes, int N, int T2, int t0, int F, int HW, const float* w, const float* b,
                          int prec, void* out, int out_chunks, int Tb, int f0, hipStream_t s) {
  const size_t n = (size_t)N * F * HW * out_chunks;
  if (prec == P_BF16)
    hipLaunchKernelGGL(proj_in_kernel<P_BF16>, dim3(blocks_for(n, 256)), dim3(256), 0, s, codes, N, T2, t0, F, HW, w,
                       b, out, out_chunks, Tb, f0);
  else
    hipLaunchKernelGGL(proj_in_kernel<P_F32>, dim3(blocks_for(n, 256)), dim3(256), 0, s, codes, N, T2, t0, F, HW, w,
                       b, out, out_chunks, Tb, f0);
  return hipGetLastError();
}

}  // namespace tok
