// Memory-bound kernels of the training step's backward pass: the loss and its
// gradient seeds, the straight-through FSQ adjoint, GroupNorm+SiLU backward,
// the stride-2 / upsample adjoint helpers, the 1x1x1 projections' adjoints and
// deterministic reductions (fixed-order partial sums, no floating atomics).
//
// The objective (appendix Eq. 5 / Eq. 7, l1 pixel term; commitment term of
// the stand-in's quantiser):
//   L = mean |x_hat - x| + 0.1 * mean (z~ - sg(c))^2,   z~ = b / floor(l/2)
// with the decoder reading keep * c and a straight-through dc/dz~ = 1.
#include <algorithm>

#include "tok_internal.h"
#include "tok_device.h"

namespace tok {

namespace {

template <int PREC> struct E;
template <> struct E<P_F32> { static constexpr int CH = 16, QE = 4; };
template <> struct E<P_BF16> { static constexpr int CH = 32, QE = 8; };

template <int PREC>
__device__ __forceinline__ void load_quad(const void* base, size_t q, float* v) {
  const uint4 u = reinterpret_cast<const uint4*>(base)[q];
  if constexpr (PREC == P_BF16) {
    v[0] = bf16_lo(u.x); v[1] = bf16_hi(u.x); v[2] = bf16_lo(u.y); v[3] = bf16_hi(u.y);
    v[4] = bf16_lo(u.z); v[5] = bf16_hi(u.z); v[6] = bf16_lo(u.w); v[7] = bf16_hi(u.w);
  } else {
    v[0] = __uint_as_float(u.x); v[1] = __uint_as_float(u.y); v[2] = __uint_as_float(u.z); v[3] = __uint_as_float(u.w);
  }
}

template <int PREC>
__device__ __forceinline__ void store_quad(void* base, size_t q, const float* v) {
  uint4 u;
  if constexpr (PREC == P_BF16) {
    u = make_uint4(pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3]), pack_bf16(v[4], v[5]), pack_bf16(v[6], v[7]));
  } else {
    u = make_uint4(__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]), __float_as_uint(v[3]));
  }
  reinterpret_cast<uint4*>(base)[q] = u;
}

inline unsigned nblk(size_t n, int per) { return (unsigned)((n + per - 1) / per); }

// ---------------------------------------------------------------------------
// Loss terms and gradient seeds.  Per-block partial sums are reduced in a
// fixed order (no floating atomics), so loss and gradients are deterministic.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ float block_sum(float v, float* red) {
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int o = N / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  return red[0];
}

// l1 term: partial sums of |x_hat - x| per block of 256 positions; with g set,
// also the seed dL/dx_hat = gscale * sign(x_hat - x) / numel (sign(0) = 0)
// into channels 0..2 of a one-chunk activation buffer (other channels 0).
template <int PREC>
__global__ void __launch_bounds__(256) l1_kernel(const float* __restrict__ xhat, const uint8_t* __restrict__ x,
                                                  size_t npos, float inv_numel, const float* __restrict__ gscale,
                                                  void* __restrict__ g, float* __restrict__ partial) {
  constexpr int CH = E<PREC>::CH, QE = E<PREC>::QE;
  __shared__ float red[256];
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  float s = 0.f;
  if (p < npos) {
    const float u = inv_numel * (gscale ? *gscale : 1.f);
    float gv[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) gv[c] = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float d = xhat[p * 3 + c] - ((float)x[p * 3 + c] / 127.5f - 1.0f);
      s += fabsf(d);
      gv[c] = d > 0.f ? u : (d < 0.f ? -u : 0.f);
    }
    if (g) {
#pragma unroll
      for (int q = 0; q < 4; ++q) store_quad<PREC>(g, p * 4 + q, gv + q * QE);
    }
  }
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// uint8 pixels -> one-chunk activations x/127.5 - 1 in channels 0..2.
template <int PREC>
__global__ void __launch_bounds__(256) u8_to_chunked_kernel(const uint8_t* __restrict__ x, size_t npos,
                                                             void* __restrict__ out) {
  constexpr int CH = E<PREC>::CH, QE = E<PREC>::QE;
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= npos) return;
  float v[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) v[c] = c < 3 ? (float)x[p * 3 + c] / 127.5f - 1.0f : 0.f;
#pragma unroll
  for (int q = 0; q < 4; ++q) store_quad<PREC>(out, p * 4 + q, v + q * QE);
}

// Commitment term and the straight-through FSQ adjoint, per token:
//   z~ = b / floor(L/2),  c = rint(b) / floor(L/2),  b = tanh(z + s) h - o
//   partial sums of (z~ - c)^2;   with gdec set:
//   g_z~ = keep * g_dec + gscale * coef * (z~ - c),   g_z = g_z~ (h / floor(L/2)) (1 - tanh^2(z + s))
// (the decoder reads keep * c and dc/dz~ = 1).
__global__ void __launch_bounds__(256) fsq_bwd_kernel(const float* __restrict__ z, const uint8_t* __restrict__ keep,
                                                       const float* __restrict__ gdec, size_t ntok, FsqConst fc,
                                                       float coef, const float* __restrict__ gscale,
                                                       float* __restrict__ gz, float* __restrict__ partial) {
  __shared__ float red[256];
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  float s = 0.f;
  if (t < ntok) {
    const float k = keep ? (float)keep[t] : 1.f;
    const float cf = coef * (gscale ? *gscale : 1.f);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const float th = tanhf(z[t * 6 + c] + fc.s[c]);
      const float b = th * fc.h[c] - fc.o[c];
      const float d = b * fc.inv_d[c] - rintf(b) * fc.inv_d[c];
      s += d * d;
      if (gdec) gz[t * 6 + c] = (k * gdec[t * 6 + c] + cf * d) * fc.h[c] * fc.inv_d[c] * (1.f - th * th);
    }
  }
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// loss[0] = l1_sum * inv_numel + commit_weight * commit_sum / M, loss[1] = l1
// term, loss[2] = commitment mean; sums strided over 256 threads, then a tree.
__global__ void __launch_bounds__(256) loss_final_kernel(const float* __restrict__ l1p, int nl1,
                                                          const float* __restrict__ cp, int nc, float inv_numel,
                                                          float inv_m, float commit_weight, float* __restrict__ loss) {
  __shared__ float red[256];
  float a = 0.f, b = 0.f;
  for (int i = threadIdx.x; i < nl1; i += 256) a += l1p[i];
  for (int i = threadIdx.x; i < nc; i += 256) b += cp[i];
  a = block_sum<256>(a, red);
  __syncthreads();
  b = block_sum<256>(b, red);
  if (threadIdx.x == 0) {
    const float l1 = a * inv_numel, cm = b * inv_m;
    loss[0] = l1 + commit_weight * cm;
    loss[1] = l1;
    loss[2] = cm;
  }
}

// ---------------------------------------------------------------------------
// GroupNorm (per frame, 32 groups of 2 channels, 64 channels) + SiLU backward.
// With x^ = (x - mu) rstd, a = x^ gamma + beta, g_a = g * silu'(a):
//   dx = rstd (gamma g_a - m1 - x^ m2),  m1 = mean over the group of gamma g_a,
//   m2 = mean of gamma g_a x^;   dgamma = sum g_a x^,  dbeta = sum g_a.
// Because gamma is constant per channel, m1 and m2 follow from the per-channel
// sums A_c = sum g_a x^ and B_c = sum g_a, which are also dgamma and dbeta.
// Pass 1: per (frame, chunk, block, quad) partial sums of A and B; a block
// strides over the positions of its frame in a fixed order.
// ---------------------------------------------------------------------------
template <int PREC>
__device__ __forceinline__ void gn_bwd_elem(const float* xv, const float* gv, int c0, const float2* mr,
                                            const float* gamma, const float* beta, float* ga, float* xh) {
  constexpr int QE = E<PREC>::QE;
#pragma unroll
  for (int j = 0; j < QE; ++j) {
    const int c = c0 + j;
    const float2 m = mr[c >> 1];
    const float xhat = (xv[j] - m.x) * m.y;
    const float a = xhat * gamma[c] + beta[c];
    const float sg = 1.f / (1.f + __expf(-a));
    ga[j] = gv[j] * sg * (1.f + a * (1.f - sg));
    xh[j] = xhat;
  }
}

template <int PREC>
__global__ void __launch_bounds__(256) gn_bwd_stats_kernel(const void* __restrict__ x, const void* __restrict__ g,
                                                            const float2* __restrict__ mr, const float* __restrict__ gamma,
                                                            const float* __restrict__ beta, int HW,
                                                            float* __restrict__ partial) {
  constexpr int CH = E<PREC>::CH, QE = E<PREC>::QE, CHUNKS = 64 / CH, NV = 2 * QE;
  __shared__ float red[4][4][NV];
  const int fc = blockIdx.y, frame = fc / CHUNKS, ck = fc % CHUNKS, nxb = gridDim.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, quad = tid & 3;
  const int c0 = ck * CH + quad * QE;
  float acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.f;
  for (int pos = blockIdx.x * 64 + (tid >> 2); pos < HW; pos += 64 * nxb) {
    const size_t q = ((size_t)fc * HW + pos) * 4 + quad;
    float xv[QE], gv[QE], ga[QE], xh[QE];
    load_quad<PREC>(x, q, xv);
    load_quad<PREC>(g, q, gv);
    gn_bwd_elem<PREC>(xv, gv, c0, mr + (size_t)frame * 32, gamma, beta, ga, xh);
#pragma unroll
    for (int j = 0; j < QE; ++j) {
      acc[j] += ga[j] * xh[j];
      acc[QE + j] += ga[j];
    }
  }
  // reduce over the 16 position lanes of the wave that share this quad (lane bits 2..5)
#pragma unroll
  for (int i = 0; i < NV; ++i)
#pragma unroll
    for (int off = 4; off < 64; off <<= 1) acc[i] += __shfl_xor(acc[i], off);
  if (lane < 4) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wave][lane][i] = acc[i];
  }
  __syncthreads();
  if (tid < 4 * NV) {
    const int qd = tid / NV, i = tid % NV;
    const float v = ((red[0][qd][i] + red[1][qd][i]) + red[2][qd][i]) + red[3][qd][i];
    partial[(((size_t)fc * nxb + blockIdx.x) * 4 + qd) * NV + i] = v;
  }
}

// Pass 2a: per frame (one wave, lane = channel): A_c, B_c over the blocks,
// then m1, m2 per group of 2 channels.
template <int PREC>
__global__ void __launch_bounds__(64) gn_bwd_frame_kernel(const float* __restrict__ partial, int nxb, int HW,
                                                           const float* __restrict__ gamma, float2* __restrict__ fsum,
                                                           float2* __restrict__ m12) {
  constexpr int CH = E<PREC>::CH, QE = E<PREC>::QE, CHUNKS = 64 / CH, NV = 2 * QE;
  const int frame = blockIdx.x, c = threadIdx.x;
  const int ck = c / CH, quad = (c % CH) / QE, j = c % QE;
  const float* p = partial + ((size_t)(frame * CHUNKS + ck) * nxb * 4 + quad) * NV;
  float A = 0.f, B = 0.f;
  for (int b = 0; b < nxb; ++b) {
    A += p[(size_t)b * 4 * NV + j];
    B += p[(size_t)b * 4 * NV + QE + j];
  }
  fsum[(size_t)frame * 64 + c] = make_float2(A, B);
  const float gA = gamma[c] * A, gB = gamma[c] * B;
  const float oA = __shfl_xor(gA, 1), oB = __shfl_xor(gB, 1);
  if ((c & 1) == 0) {
    const float cnt = 2.f * (float)HW;
    m12[(size_t)frame * 32 + (c >> 1)] = make_float2((gB + oB) / cnt, (gA + oA) / cnt);
  }
}

// Pass 2b: dgamma, dbeta per channel, summed over frames in order.
__global__ void __launch_bounds__(64) gn_bwd_param_kernel(const float2* __restrict__ fsum, int frames,
                                                           float* __restrict__ dgamma, float* __restrict__ dbeta) {
  const int c = threadIdx.x;
  float a = 0.f, b = 0.f;
#pragma unroll 8
  for (int f = 0; f < frames; ++f) {
    const float2 v = fsum[(size_t)f * 64 + c];
    a += v.x;
    b += v.y;
  }
  dgamma[c] = a;
  dbeta[c] = b;
}

// Pass 3: dx = rstd (gamma g_a - m1 - x^ m2) (+ a residual gradient).  In
// place on g or on resid is allowed (each thread reads its elements first).
template <int PREC>
__global__ void __launch_bounds__(256) gn_bwd_apply_kernel(const void* __restrict__ x, const void* g,
                                                            const float2* __restrict__ mr, const float2* __restrict__ m12,
                                                            const float* __restrict__ gamma, const float* __restrict__ beta,
                                                            const void* resid, void* dx, int HW) {
  constexpr int CH = E<PREC>::CH, QE = E<PREC>::QE, CHUNKS = 64 / CH;
  const int fc = blockIdx.y, frame = fc / CHUNKS, ck = fc % CHUNKS;
  const int pos = blockIdx.x * 64 + (threadIdx.x >> 2), quad = threadIdx.x & 3;
  if (pos >= HW) return;
  const size_t q = ((size_t)fc * HW + pos) * 4 + quad;
  float xv[QE], gv[QE], ga[QE], xh[QE], out[QE], rv[QE];
  load_quad<PREC>(x, q, xv);
  load_quad<PREC>(g, q, gv);
  if (resid) load_quad<PREC>(resid, q, rv);
  const int c0 = ck * CH + quad * QE;
  const float2* mrf = mr + (size_t)frame * 32;
  gn_bwd_elem<PREC>(xv, gv, c0, mrf, gamma, beta, ga, xh);
#pragma unroll
  for (int j = 0; j < QE; ++j) {
    const int c = c0 + j;
    const float2 m = m12[(size_t)frame * 32 + (c >> 1)];
    out[j] = mrf[c >> 1].y * (gamma[c] * ga[j] - m.x - xh[j] * m.y) + (resid ? rv[j] : 0.f);
  }
  store_quad<PREC>(dx, q, out);
}

// ---------------------------------------------------------------------------
// Upsample adjoint: coarse[n, j, h, w] = sum of fine frames {2j-1, 2j} (just 0
// for j = 0) x the 2 x 2 pixels.  One thread per coarse 64-byte chunk position.
// ---------------------------------------------------------------------------
template <int PREC>
__global__ void __launch_bounds__(256) up_adjoint_kernel(const void* __restrict__ fine, void* __restrict__ coarse,
                                                          int N, int Tc, int Hc, int Wc, int chunks) {
  constexpr int QE = E<PREC>::QE;
  const size_t total = (size_t)N * Tc * chunks * Hc * Wc;
  const size_t gid = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= total) return;
  size_t r = gid;
  const int w = (int)(r % Wc); r /= Wc;
  const int h = (int)(r % Hc); r /= Hc;
  const int ck = (int)(r % chunks); r /= chunks;
  const int j = (int)(r % Tc);
  const int n = (int)(r / Tc);
  const int Tf = 2 * Tc - 1, Hf = 2 * Hc, Wf = 2 * Wc;
  float acc[4 * QE];
#pragma unroll
  for (int i = 0; i < 4 * QE; ++i) acc[i] = 0.f;
  for (int tf = (j == 0 ? 0 : 2 * j - 1); tf <= 2 * j; ++tf)
    for (int dh = 0; dh < 2; ++dh)
      for (int dw = 0; dw < 2; ++dw) {
        const size_t fq = ((((size_t)n * Tf + tf) * chunks + ck) * Hf + 2 * h + dh) * Wf + 2 * w + dw;
        float v[4 * QE];
#pragma unroll
        for (int q = 0; q < 4; ++q) load_quad<PREC>(fine, fq * 4 + q, v + q * QE);
#pragma unroll
        for (int i = 0; i < 4 * QE; ++i) acc[i] += v[i];
      }
#pragma unroll
  for (int q = 0; q < 4; ++q) store_quad<PREC>(coarse, gid * 4 + q, acc + q * QE);
}

// ---------------------------------------------------------------------------
// 1x1x1 projections' adjoints.  proj6: y[p][k] = sum_c w6[k][c] x[p][c] over
// 128 chunked channels (w6 = [6][128]).
// ---------------------------------------------------------------------------
template <int PREC>
__global__ void __launch_bounds__(256) proj6_kernel(const void* __restrict__ x, size_t ntok, int HW,
                                                     const float* __restrict__ w6, float* __restrict__ y) {
  constexpr int CH = E<PREC>::CH, QE = E<PREC>::QE, CHUNKS = 128 / CH;
  __shared__ float ws[6 * 128];
  for (int e = threadIdx.x; e < 6 * 128; e += 256) ws[e] = w6[e];
  __syncthreads();
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= ntok) return;
  const size_t frame = t / HW, hw = t % HW;
  float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int ck = 0; ck < CHUNKS; ++ck)
    for (int q = 0; q < 4; ++q) {
      float v[QE];
      load_quad<PREC>(x, ((frame * CHUNKS + ck) * HW + hw) * 4 + q, v);
#pragma unroll
      for (int j = 0; j < QE; ++j) {
        const int c = ck * CH + q * QE + j;
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[k] = fmaf(ws[k * 128 + c], v[j], acc[k]);
      }
    }
#pragma unroll
  for (int k = 0; k < 6; ++k) y[t * 6 + k] = acc[k];
}

// Partial sums for the 1x1x1 weight gradients over blocks of 64 tokens:
//   P[k][c] = sum a6[p][k] x[p][c],  A[k] = sum a6[p][k],  X[c] = sum x[p][c]
// (902 values per block), each summed over the block's tokens in order.
constexpr int kOuterCols = 6 * 128 + 6 + 128;

template <int PREC>
__global__ void __launch_bounds__(256) outer6_kernel(const float* __restrict__ a6, const void* __restrict__ x,
                                                      size_t ntok, int HW, float* __restrict__ partial) {
  constexpr int CH = E<PREC>::CH, CHUNKS = 128 / CH;
  __shared__ float s_a[64][6];
  __shared__ float s_x[64][129];
  const size_t t0 = (size_t)blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * 6; e += 256) {
    const size_t t = t0 + e / 6;
    s_a[e / 6][e % 6] = t < ntok ? a6[t * 6 + e % 6] : 0.f;
  }
  for (int e = threadIdx.x; e < 64 * 128; e += 256) {
    const int r = e / 128, c = e % 128;
    const size_t t = t0 + r;
    float v = 0.f;
    if (t < ntok) {
      const size_t frame = t / HW, hw = t % HW;
      const size_t off = ((frame * CHUNKS + c / CH) * HW + hw) * CH + c % CH;
      if constexpr (PREC == P_BF16) v = __uint_as_float((uint32_t)reinterpret_cast<const uint16_t*>(x)[off] << 16);
      else v = reinterpret_cast<const float*>(x)[off];
    }
    s_x[r][c] = v;
  }
  __syncthreads();
  float* out = partial + (size_t)blockIdx.x * kOuterCols;
  for (int o = threadIdx.x; o < kOuterCols; o += 256) {
    float s = 0.f;
    if (o < 768) {
      const int k = o / 128, c = o % 128;
      for (int r = 0; r < 64; ++r) s = fmaf(s_a[r][k], s_x[r][c], s);
    } else if (o < 774) {
      for (int r = 0; r < 64; ++r) s += s_a[r][o - 768];
    } else {
      for (int r = 0; r < 64; ++r) s += s_x[r][o - 774];
    }
    out[o] = s;
  }
}

// Sums the block partials in a fixed order: 64 columns per block, wave w
// sums rows w, w + 16, ... in order, then the 16 wave sums are added in wave
// order.  transposed = 0: dw[k][c] (a 128 -> 6 projection, whose bias
// gradient is A); transposed = 1: dw[c][k] (6 -> 128, bias gradient X).
__global__ void __launch_bounds__(1024) outer6_reduce_kernel(const float* __restrict__ partial, int rows,
                                                              int transposed, float* __restrict__ dw,
                                                              float* __restrict__ db) {
  __shared__ float part[16][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int o = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (o < kOuterCols) {
#pragma unroll 8
    for (int r = w; r < rows; r += 16) s += partial[(size_t)r * kOuterCols + o];
  }
  part[w][lane] = s;
  __syncthreads();
  if (w != 0 || o >= kOuterCols) return;
  s = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) s += part[k][lane];
  if (o < 768) {
    const int k = o / 128, c = o % 128;
    dw[transposed ? c * 6 + k : o] = s;
  } else if (o < 774) {
    if (!transposed) db[o - 768] = s;
  } else {
    if (transposed) db[o - 774] = s;
  }
}

// [R][C] -> [C][R] (the 1x1x1 weights' transposes used by the adjoints).
__global__ void transpose_kernel(const float* __restrict__ in, int R, int C, float* __restrict__ out) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= R * C) return;
  const int r = e / C, c = e % C;
  out[(size_t)c * R + r] = in[e];
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
#define TOK_PREC_LAUNCH(K, grid, block, ...)                                          \
  do {                                                                                \
    if (prec == P_BF16) hipLaunchKernelGGL(K<P_BF16>, grid, block, 0, s, __VA_ARGS__); \
    else hipLaunchKernelGGL(K<P_F32>, grid, block, 0, s, __VA_ARGS__);                \
  } while (0)

int l1_blocks(size_t npos) { return (int)nblk(npos, 256); }
int fsq_blocks(size_t ntok) { return (int)nblk(ntok, 256); }
int outer6_blocks(size_t ntok) { return (int)nblk(ntok, 64); }
size_t outer6_partial_floats(size_t ntok) { return (size_t)outer6_blocks(ntok) * kOuterCols; }

hipError_t launch_l1(const float* xhat, const uint8_t* x, size_t npos, int prec, const float* gscale, void* g,
                     float* partial, hipStream_t s) {
  if (npos == 0) return hipErrorInvalidValue;
  TOK_PREC_LAUNCH(l1_kernel, dim3(l1_blocks(npos)), dim3(256), xhat, x, npos, 1.0f / (float)(npos * 3), gscale, g,
                  partial);
  return hipGetLastError();
}

hipError_t launch_u8_to_chunked(const uint8_t* x, size_t npos, int prec, void* out, hipStream_t s) {
  TOK_PREC_LAUNCH(u8_to_chunked_kernel, dim3(nblk(npos, 256)), dim3(256), x, npos, out);
  return hipGetLastError();
}

hipError_t launch_fsq_bwd(const float* z, const uint8_t* keep, const float* gdec, size_t ntok, const FsqConst& fc,
                          float coef, const float* gscale, float* gz, float* partial, hipStream_t s) {
  if (ntok == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fsq_bwd_kernel, dim3(fsq_blocks(ntok)), dim3(256), 0, s, z, keep, gdec, ntok, fc, coef, gscale,
                     gz, partial);
  return hipGetLastError();
}

hipError_t launch_loss_final(const float* l1p, int nl1, const float* cp, int nc, float inv_numel, float inv_m,
                             float commit_weight, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, s, l1p, nl1, cp, nc, inv_numel, inv_m, commit_weight,
                     loss);
  return hipGetLastError();
}

int gn_bwd_blocks(int HW) { return std::min((HW + 63) / 64, 16); }
size_t gn_bwd_partial_floats(int frames, int HW, int prec) {
  const int QE = prec == P_BF16 ? 8 : 4, chunks = prec == P_BF16 ? 2 : 4;
  return (size_t)frames * chunks * gn_bwd_blocks(HW) * 4 * 2 * QE;
}

hipError_t launch_gn_bwd(const void* x, const void* g, const float2* mr, const float* gamma, const float* beta,
                         const void* resid, void* dx, int frames, int HW, int prec, float* partial, float2* fsum,
                         float2* m12, float* dgamma, float* dbeta, hipStream_t s) {
  const int chunks = prec == P_BF16 ? 2 : 4, nxb = gn_bwd_blocks(HW);
  if ((long long)frames * chunks > 65535 || frames < 1 || HW < 1) return hipErrorInvalidValue;
  TOK_PREC_LAUNCH(gn_bwd_stats_kernel, dim3(nxb, frames * chunks), dim3(256), x, g, mr, gamma, beta, HW, partial);
  TOK_PREC_LAUNCH(gn_bwd_frame_kernel, dim3(frames), dim3(64), partial, nxb, HW, gamma, fsum, m12);
  hipLaunchKernelGGL(gn_bwd_param_kernel, dim3(1), dim3(64), 0, s, fsum, frames, dgamma, dbeta);
  TOK_PREC_LAUNCH(gn_bwd_apply_kernel, dim3((HW + 63) / 64, frames * chunks), dim3(256), x, g, mr, m12, gamma, beta,
                  resid, dx, HW);
  return hipGetLastError();
}

hipError_t launch_up_adjoint(const void* fine, void* coarse, int N, int Tc, int Hc, int Wc, int chunks, int prec,
                             hipStream_t s) {
  const size_t total = (size_t)N * Tc * chunks * Hc * Wc;
  TOK_PREC_LAUNCH(up_adjoint_kernel, dim3(nblk(total, 256)), dim3(256), fine, coarse, N, Tc, Hc, Wc, chunks);
  return hipGetLastError();
}

hipError_t launch_proj6(const void* x, size_t ntok, int HW, const float* w6, float* y, int prec, hipStream_t s) {
  TOK_PREC_LAUNCH(proj6_kernel, dim3(nblk(ntok, 256)), dim3(256), x, ntok, HW, w6, y);
  return hipGetLastError();
}

hipError_t launch_outer6(const float* a6, const void* x, size_t ntok, int HW, int prec, float* partial,
                         int transposed, float* dw, float* db, hipStream_t s) {
  const int rows = outer6_blocks(ntok);
  TOK_PREC_LAUNCH(outer6_kernel, dim3(rows), dim3(256), a6, x, ntok, HW, partial);
  hipLaunchKernelGGL(outer6_reduce_kernel, dim3((kOuterCols + 63) / 64), dim3(1024), 0, s, partial, rows, transposed,
                     dw, db);
  return hipGetLastError();
}

hipError_t launch_transpose(const float* in, int R, int C, float* out, hipStream_t s) {
  hipLaunchKernelGGL(transpose_kernel, dim3((R * C + 255) / 256), dim3(256), 0, s, in, R, C, out);
  return hipGetLastError();
}

}  // namespace tok
