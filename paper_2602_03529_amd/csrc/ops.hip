// Small kernels behind the per-operation entry points (tok_ops.hip): layout
// conversion between dense channels-last tensors and the library's chunked
// activations, GroupNorm statistics of a whole tensor, the GroupNorm affine,
// and the straight-through quantiser adjoint for gradients that come from
// outside the library.  All memory-bound; none is on the encode / decode path.
#include "tok_internal.h"
#include "tok_device.h"

namespace tok {

namespace {

template <int PREC> struct OE;
template <> struct OE<P_F32> { static constexpr int CH = 16, QE = 4; };
template <> struct OE<P_BF16> { static constexpr int CH = 32, QE = 8; };

template <int PREC>
__device__ __forceinline__ void ld_quad(const void* base, size_t q, float* v) {
  const uint4 u = reinterpret_cast<const uint4*>(base)[q];
  if constexpr (PREC == P_BF16) {
    v[0] = bf16_lo(u.x); v[1] = bf16_hi(u.x); v[2] = bf16_lo(u.y); v[3] = bf16_hi(u.y);
    v[4] = bf16_lo(u.z); v[5] = bf16_hi(u.z); v[6] = bf16_lo(u.w); v[7] = bf16_hi(u.w);
  } else {
    v[0] = __uint_as_float(u.x); v[1] = __uint_as_float(u.y); v[2] = __uint_as_float(u.z); v[3] = __uint_as_float(u.w);
  }
}

template <int PREC>
__device__ __forceinline__ void st_quad(void* base, size_t q, const float* v) {
  uint4 u;
  if constexpr (PREC == P_BF16)
    u = make_uint4(pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3]), pack_bf16(v[4], v[5]), pack_bf16(v[6], v[7]));
  else
    u = make_uint4(__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]), __float_as_uint(v[3]));
  reinterpret_cast<uint4*>(base)[q] = u;
}

inline unsigned nb(size_t n, int per) { return (unsigned)((n + per - 1) / per); }

// dense [frames][HW][C] float -> chunked [frames][chunks][HW][CH] (channels
// past C zero).  One thread per 16-byte output quad.
template <int PREC>
__global__ void __launch_bounds__(256) act_pack_kernel(const float* __restrict__ src, long long frames, int HW, int C,
                                                        int chunks, void* __restrict__ dst) {
  constexpr int CH = OE<PREC>::CH, QE = OE<PREC>::QE;
  const size_t total = (size_t)frames * chunks * HW * 4;
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= total) return;
  const int quad = (int)(q & 3);
  size_t r = q >> 2;
  const int pos = (int)(r % HW); r /= HW;
  const int ck = (int)(r % chunks);
  const size_t f = r / chunks;
  const float* s = src + ((size_t)f * HW + pos) * C;
  float v[QE];
#pragma unroll
  for (int j = 0; j < QE; ++j) {
    const int c = ck * CH + quad * QE + j;
    v[j] = c < C ? s[c] : 0.f;
  }
  st_quad<PREC>(dst, q, v);
}

// chunked -> dense float (channels past C dropped).  One thread per input quad.
template <int PREC>
__global__ void __launch_bounds__(256) act_unpack_kernel(const void* __restrict__ src, long long frames, int HW, int C,
                                                          int chunks, float* __restrict__ dst) {
  constexpr int CH = OE<PREC>::CH, QE = OE<PREC>::QE;
  const size_t total = (size_t)frames * chunks * HW * 4;
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= total) return;
  const int quad = (int)(q & 3);
  size_t r = q >> 2;
  const int pos = (int)(r % HW); r /= HW;
  const int ck = (int)(r % chunks);
  const size_t f = r / chunks;
  float v[QE];
  ld_quad<PREC>(src, q, v);
  float* d = dst + ((size_t)f * HW + pos) * C;
#pragma unroll
  for (int j = 0; j < QE; ++j) {
    const int c = ck * CH + quad * QE + j;
    if (c < C) d[c] = v[j];
  }
}

// GroupNorm(32) partial statistics of a 64-channel chunked tensor: per frame
// and tile of kGnOpTile positions, per group (2 channels) the count, mean and
// sum of squared deviations (two passes over the tile, fixed reduction
// order), in the float4 layout the producing convs write:
// stats[(frame * tiles + tile) * 32 + group] = (count, mean, M2, 0).
constexpr int kGnOpTile = 1024;

template <int PREC>
__global__ void __launch_bounds__(256) gn_partial_kernel(const void* __restrict__ x, int HW, int tiles,
                                                          float4* __restrict__ stats) {
  constexpr int CH = OE<PREC>::CH, QE = OE<PREC>::QE, CHUNKS = 64 / CH, S = CHUNKS * 4, R = 256 / S, G = QE / 2;
  __shared__ float red[32][R + 1];
  __shared__ float gmean[32];
  const int tile = blockIdx.x, frame = blockIdx.y, tid = threadIdx.x;
  const int slot = tid % S, row = tid / S, ck = slot / 4, quad = slot % 4;
  const int g0 = (ck * CH + quad * QE) / 2;  // first group of this thread's channels
  const int p0 = tile * kGnOpTile, p1 = min(p0 + kGnOpTile, HW);
  const float cnt = 2.f * (float)(p1 - p0);
  float acc[G];
#pragma unroll
  for (int g = 0; g < G; ++g) acc[g] = 0.f;
  for (int p = p0 + row; p < p1; p += R) {
    float v[QE];
    ld_quad<PREC>(x, (((size_t)frame * CHUNKS + ck) * HW + p) * 4 + quad, v);
#pragma unroll
    for (int g = 0; g < G; ++g) acc[g] += v[2 * g] + v[2 * g + 1];
  }
#pragma unroll
  for (int g = 0; g < G; ++g) red[g0 + g][row] = acc[g];
  __syncthreads();
  if (tid < 32) {
    float s = 0.f;
    for (int r = 0; r < R; ++r) s += red[tid][r];
    gmean[tid] = s / cnt;
  }
  __syncthreads();
  float mu[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    mu[g] = gmean[g0 + g];
    acc[g] = 0.f;
  }
  for (int p = p0 + row; p < p1; p += R) {
    float v[QE];
    ld_quad<PREC>(x, (((size_t)frame * CHUNKS + ck) * HW + p) * 4 + quad, v);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const float a = v[2 * g] - mu[g], b = v[2 * g + 1] - mu[g];
      acc[g] += a * a + b * b;
    }
  }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < G; ++g) red[g0 + g][row] = acc[g];
  __syncthreads();
  if (tid < 32) {
    float s = 0.f;
    for (int r = 0; r < R; ++r) s += red[tid][r];
    stats[((size_t)frame * tiles + tile) * 32 + tid] = make_float4(cnt, gmean[tid], s, 0.f);
  }
}

// Per (frame, channel): scale = gamma rstd, shift = beta - mean scale.
__global__ void __launch_bounds__(64) gn_affine_kernel(const float2* __restrict__ mr, const float* __restrict__ gamma,
                                                        const float* __restrict__ beta, float* __restrict__ scale,
                                                        float* __restrict__ shift) {
  const int f = blockIdx.x, c = threadIdx.x;
  const float2 m = mr[(size_t)f * 32 + (c >> 1)];
  const float sc = m.y * gamma[c];
  scale[(size_t)f * 64 + c] = sc;
  shift[(size_t)f * 64 + c] = beta[c] - m.x * sc;
}

// Straight-through quantiser adjoint per token:
//   g_z = g_z_in + keep (g_a + g_b) (h / floor(L/2)) (1 - tanh^2(z + s))
// (any of keep, g_a, g_b, g_z_in may be null: 1, 0, 0, 0).
__global__ void __launch_bounds__(256) fsq_ste_kernel(const float* __restrict__ z, const uint8_t* __restrict__ keep,
                                                       const float* __restrict__ ga, const float* __restrict__ gb,
                                                       const float* __restrict__ gzin, size_t ntok, FsqConst fc,
                                                       float* __restrict__ gz) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= ntok) return;
  const float k = keep ? (float)keep[t] : 1.f;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const size_t e = t * 6 + c;
    const float th = tanhf(z[e] + fc.s[c]);
    const float g = (ga ? ga[e] : 0.f) + (gb ? gb[e] : 0.f);
    const float d = k * g * fc.h[c] * fc.inv_d[c] * (1.f - th * th);
    gz[e] = (gzin ? gzin[e] : 0.f) + d;
  }
}

// Dense float (npos, 3) -> one-chunk activations, channels 3.. zero.
template <int PREC>
__global__ void __launch_bounds__(256) rgb_to_chunk_kernel(const float* __restrict__ src, size_t npos,
                                                            void* __restrict__ out) {
  constexpr int CH = OE<PREC>::CH, QE = OE<PREC>::QE;
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= npos) return;
  float v[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) v[c] = c < 3 ? src[p * 3 + c] : 0.f;
#pragma unroll
  for (int q = 0; q < 4; ++q) st_quad<PREC>(out, p * 4 + q, v + q * QE);
}

__global__ void __launch_bounds__(256) fill_zero_kernel(float* __restrict__ p, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

}  // namespace

#define TOK_OPS_PREC(K, grid, ...)                                                         \
  do {                                                                                     \
    if (prec == P_BF16) hipLaunchKernelGGL(K<P_BF16>, grid, dim3(256), 0, s, __VA_ARGS__); \
    else hipLaunchKernelGGL(K<P_F32>, grid, dim3(256), 0, s, __VA_ARGS__);                 \
  } while (0)

hipError_t launch_act_pack(const float* src, long long frames, int HW, int C, int prec, void* dst, hipStream_t s) {
  const int chunks = (C + (prec == P_BF16 ? 32 : 16) - 1) / (prec == P_BF16 ? 32 : 16);
  const size_t total = (size_t)frames * chunks * HW * 4;
  if (!total) return hipSuccess;
  TOK_OPS_PREC(act_pack_kernel, dim3(nb(total, 256)), src, frames, HW, C, chunks, dst);
  return hipGetLastError();
}

hipError_t launch_act_unpack(const void* src, long long frames, int HW, int C, int prec, float* dst, hipStream_t s) {
  const int chunks = (C + (prec == P_BF16 ? 32 : 16) - 1) / (prec == P_BF16 ? 32 : 16);
  const size_t total = (size_t)frames * chunks * HW * 4;
  if (!total) return hipSuccess;
  TOK_OPS_PREC(act_unpack_kernel, dim3(nb(total, 256)), src, frames, HW, C, chunks, dst);
  return hipGetLastError();
}

int gn_op_tiles(int HW) { return (HW + kGnOpTile - 1) / kGnOpTile; }

hipError_t launch_gn_partials(const void* x, int frames, int HW, int prec, float4* stats, hipStream_t s) {
  if (frames < 1 || frames > 65535 || HW < 1) return hipErrorInvalidValue;
  TOK_OPS_PREC(gn_partial_kernel, dim3(gn_op_tiles(HW), frames), x, HW, gn_op_tiles(HW), stats);
  return hipGetLastError();
}

hipError_t launch_gn_affine(const float2* mr, const float* gamma, const float* beta, int frames, float* scale,
                            float* shift, hipStream_t s) {
  if (frames < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gn_affine_kernel, dim3(frames), dim3(64), 0, s, mr, gamma, beta, scale, shift);
  return hipGetLastError();
}

hipError_t launch_fsq_ste(const float* z, const uint8_t* keep, const float* ga, const float* gb, const float* gzin,
                          size_t ntok, const FsqConst& fc, float* gz, hipStream_t s) {
  if (!ntok) return hipSuccess;
  hipLaunchKernelGGL(fsq_ste_kernel, dim3(nb(ntok, 256)), dim3(256), 0, s, z, keep, ga, gb, gzin, ntok, fc, gz);
  return hipGetLastError();
}

hipError_t launch_rgb_to_chunk(const float* src, size_t npos, int prec, void* out, hipStream_t s) {
  if (!npos) return hipSuccess;
  TOK_OPS_PREC(rgb_to_chunk_kernel, dim3(nb(npos, 256)), src, npos, out);
  return hipGetLastError();
}

hipError_t launch_fill_zero(float* p, size_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(nb(n, 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

#undef TOK_OPS_PREC

}  // namespace tok
