// Pixel-level enhancement around the decoder: the residual layer of scalable
// coding (Sec. 4.3, Eq. 4) and GoP-boundary blending (Sec. 4.2, Eq. 2).
//
// Residual sender, per clip of T frames (the averaging window):
//   rs_mean_kernel     r = (1/T) sum_t (x_t - x_hat_t) per (h, w, c), fp32 sums in
//                      frame order; entries with |r| < theta become 0; writes
//                      the dense thresholded residual and each block's count
//                      of non-zero entries
//   rs_finish_kernel   the same from sums the decoder's last layer accumulated
//                      while writing x_hat (in place)
//   rs_scan_kernel     one workgroup: exclusive scan of the block counts
//   rs_compact_kernel  the non-zero entries of each clip as (flat index
//                      (h W + w) 3 + c, value) in increasing index order
// Receiver: rs_apply_kernel adds the averaged residual to every frame.
// All three sender kernels stream the frames once (HBM-bound).
#include "tok_internal.h"
#include "tok_device.h"

namespace tok {

namespace {

constexpr int kRsThreads = 256;
constexpr int kRsVec = 4;                         // consecutive entries per thread
constexpr int kRsBlock = kRsThreads * kRsVec;     // entries per block
constexpr int kScanThreads = 1024;

__device__ __forceinline__ float px(uint32_t u) { return (float)u / 127.5f - 1.0f; }

// r = sum / T with entries of magnitude below theta set to 0; returns the
// number of non-zero entries.
__device__ __forceinline__ int rs_mean4(float s[4], int T, float theta) {
  const float fT = (float)T;
  int nz = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float r = s[k] / fT;
    s[k] = fabsf(r) < theta ? 0.f : r;
    nz += s[k] != 0.f;
  }
  return nz;
}

// The block's count of non-zero entries (wave sums by shuffles, then the 4
// waves) into counts[slot].
__device__ __forceinline__ void rs_block_count(int nz, uint32_t* wsum, uint32_t* counts, size_t slot) {
  const int tid = threadIdx.x;
  int v = nz;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((tid & 63) == 0) wsum[tid >> 6] = (uint32_t)v;
  __syncthreads();
  if (tid == 0) counts[slot] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// grid (blocks per clip, N); E = H W 3 entries per frame (a multiple of 16).
// A thread owns 4 consecutive entries (a wave one contiguous 1 KB run of
// reconstructions per frame); four frames in flight.
__global__ void __launch_bounds__(kRsThreads) rs_mean_kernel(const uint8_t* __restrict__ x,
                                                              const float* __restrict__ xhat, int T, long long E,
                                                              float theta, float* __restrict__ rs,
                                                              uint32_t* __restrict__ counts) {
  __shared__ uint32_t wsum[kRsThreads / 64];
  const int n = blockIdx.y, tid = threadIdx.x;
  const long long e = ((long long)blockIdx.x * kRsThreads + tid) * kRsVec;
  int nz = 0;
  if (e < E) {
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    const size_t clip = (size_t)n * T * E;
#pragma unroll 4
    for (int t = 0; t < T; ++t) {
      const size_t o = clip + (size_t)t * E + e;
      const uint32_t u = *reinterpret_cast<const uint32_t*>(x + o);
      const float4 h = *reinterpret_cast<const float4*>(xhat + o);
      s0 += px(u & 255u) - h.x;
      s1 += px((u >> 8) & 255u) - h.y;
      s2 += px((u >> 16) & 255u) - h.z;
      s3 += px(u >> 24) - h.w;
    }
    float r[4] = {s0, s1, s2, s3};
    nz = rs_mean4(r, T, theta);
    *reinterpret_cast<float4*>(rs + (size_t)n * E + e) = make_float4(r[0], r[1], r[2], r[3]);
  }
  rs_block_count(nz, wsum, counts, (size_t)n * gridDim.x + blockIdx.x);
}

// Same grid as rs_mean_kernel: rs holds sum_t (x_t / 127.5 - 1 - x_hat_t)
// per entry (accumulated in frame order by the decoder's last layer) and is
// replaced by the thresholded mean.
__global__ void __launch_bounds__(kRsThreads) rs_finish_kernel(float* __restrict__ rs, int T, long long E,
                                                                float theta, uint32_t* __restrict__ counts) {
  __shared__ uint32_t wsum[kRsThreads / 64];
  const int n = blockIdx.y, tid = threadIdx.x;
  const long long e = ((long long)blockIdx.x * kRsThreads + tid) * kRsVec;
  int nz = 0;
  if (e < E) {
    float4* p = reinterpret_cast<float4*>(rs + (size_t)n * E + e);
    const float4 v = *p;
    float r[4] = {v.x, v.y, v.z, v.w};
    nz = rs_mean4(r, T, theta);
    *p = make_float4(r[0], r[1], r[2], r[3]);
  }
  rs_block_count(nz, wsum, counts, (size_t)n * gridDim.x + blockIdx.x);
}

// counts[0..B) -> exclusive prefix sums in place; counts[B] = total.
__global__ void __launch_bounds__(kScanThreads) rs_scan_kernel(uint32_t* __restrict__ counts, long long B) {
  __shared__ unsigned long long part[kScanThreads];
  const int t = threadIdx.x;
  const long long per = (B + kScanThreads - 1) / kScanThreads;
  const long long a = t * per, b = a + per < B ? a + per : B;
  unsigned long long sum = 0;
  for (long long i = a; i < b; ++i) sum += counts[i];
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    const unsigned long long v = t >= o ? part[t - o] : 0ull;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  unsigned long long run = part[t] - sum;
  for (long long i = a; i < b; ++i) {
    const uint32_t c = counts[i];
    counts[i] = (uint32_t)run;
    run += c;
  }
  if (t == kScanThreads - 1) counts[B] = (uint32_t)part[t];
}

// Same grid as rs_mean_kernel.  Entry k of the batch list goes to position k
// (positions >= capacity are not written); clip_off[n] = first entry of clip n.
__global__ void __launch_bounds__(kRsThreads) rs_compact_kernel(const float* __restrict__ rs, long long E,
                                                                 const uint32_t* __restrict__ offs,
                                                                 uint32_t* __restrict__ index,
                                                                 float* __restrict__ value, long long capacity,
                                                                 unsigned long long* __restrict__ clip_off, int N) {
  __shared__ uint32_t wbase[kRsThreads / 64];
  const int n = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const long long e = ((long long)blockIdx.x * kRsThreads + tid) * kRsVec;
  float rv[kRsVec] = {0.f, 0.f, 0.f, 0.f};
  if (e < E) {
    const float4 v = *reinterpret_cast<const float4*>(rs + (size_t)n * E + e);
    rv[0] = v.x;
    rv[1] = v.y;
    rv[2] = v.z;
    rv[3] = v.w;
  }
  int nz = 0;
#pragma unroll
  for (int k = 0; k < kRsVec; ++k) nz += rv[k] != 0.f;
  // exclusive prefix of nz over the block, in thread order
  int incl = nz;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wbase[wv] = (uint32_t)incl;
  __syncthreads();
  uint32_t before = 0;
  for (int q = 0; q < wv; ++q) before += wbase[q];
  const long long blk = (long long)n * gridDim.x + blockIdx.x;
  unsigned long long pos = (unsigned long long)offs[blk] + before + (uint32_t)(incl - nz);
  if (blockIdx.x == 0 && tid == 0) {
    clip_off[n] = offs[blk];
    if (n == N - 1) clip_off[N] = offs[(long long)N * gridDim.x];
  }
#pragma unroll
  for (int k = 0; k < kRsVec; ++k) {
    if (rv[k] != 0.f) {
      if ((long long)pos < capacity) {
        index[pos] = (uint32_t)(e + k);
        value[pos] = rv[k];
      }
      ++pos;
    }
  }
}

// x_hat[n, t] += r[n] for every frame t.
__global__ void __launch_bounds__(kRsThreads) rs_apply_kernel(const float* __restrict__ rs, float* __restrict__ xhat,
                                                               int T, long long E) {
  const int n = blockIdx.y;
  const long long e = ((long long)blockIdx.x * kRsThreads + threadIdx.x) * kRsVec;
  if (e >= E) return;
  const float4 r = *reinterpret_cast<const float4*>(rs + (size_t)n * E + e);
#pragma unroll 4
  for (int t = 0; t < T; ++t) {
    float4* p = reinterpret_cast<float4*>(xhat + ((size_t)n * T + t) * E + e);
    float4 v = *p;
    v.x += r.x;
    v.y += r.y;
    v.z += r.z;
    v.w += r.w;
    *p = v;
  }
}

// Frames i = 1..n of the current GoP: alpha_i prev[Tp - n + i] + (1 - alpha_i) cur[i],
// alpha_i = (n - i) / n.  grid (blocks per frame, nblend, N).
__global__ void __launch_bounds__(kRsThreads) blend_kernel(const float* __restrict__ prev, int Tp,
                                                            float* __restrict__ cur, int T, int nb, long long E) {
  const int i = blockIdx.y + 1, n = blockIdx.z;
  const long long e = ((long long)blockIdx.x * kRsThreads + threadIdx.x) * kRsVec;
  if (e >= E) return;
  const float a = (float)(nb - i) / (float)nb, b = 1.0f - a;
  const float4 p = *reinterpret_cast<const float4*>(prev + ((size_t)n * Tp + (Tp - nb + i - 1)) * E + e);
  float4* c = reinterpret_cast<float4*>(cur + ((size_t)n * T + (i - 1)) * E + e);
  float4 v = *c;
  v.x = a * p.x + b * v.x;
  v.y = a * p.y + b * v.y;
  v.z = a * p.z + b * v.z;
  v.w = a * p.w + b * v.w;
  *c = v;
}

}  // namespace

size_t residual_ws_bytes(int N, int H, int W) {
  const long long E = 3LL * H * W, bpc = (E + kRsBlock - 1) / kRsBlock;
  return (size_t)(N * bpc + 1) * sizeof(uint32_t);
}

hipError_t launch_residual(const uint8_t* x, const float* xhat, int N, int T, int H, int W, float theta, float* rs,
                           uint32_t* index, float* value, long long capacity, unsigned long long* clip_off,
                           void* ws, hipStream_t s) {
  const long long E = 3LL * H * W, bpc = (E + kRsBlock - 1) / kRsBlock;
  // entry counts and offsets are 32-bit: the whole batch's N E entries must fit
  if (N < 1 || N > 65535 || T < 1 || E < 16 || (E & 15) || bpc > 0x7fffffffLL || (long long)N * E >= 0xffffffffLL)
    return hipErrorInvalidValue;
  uint32_t* counts = static_cast<uint32_t*>(ws);
  const dim3 grid((unsigned)bpc, N);
  hipLaunchKernelGGL(rs_mean_kernel, grid, dim3(kRsThreads), 0, s, x, xhat, T, E, theta, rs, counts);
  hipLaunchKernelGGL(rs_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, counts, (long long)N * bpc);
  hipLaunchKernelGGL(rs_compact_kernel, grid, dim3(kRsThreads), 0, s, rs, E, counts, index, value, capacity,
                     clip_off, N);
  return hipGetLastError();
}

hipError_t launch_residual_sums(float* rs, int N, int T, int H, int W, float theta, uint32_t* index, float* value,
                                long long capacity, unsigned long long* clip_off, void* ws, hipStream_t s) {
  const long long E = 3LL * H * W, bpc = (E + kRsBlock - 1) / kRsBlock;
  if (N < 1 || N > 65535 || T < 1 || E < 16 || (E & 15) || bpc > 0x7fffffffLL || (long long)N * E >= 0xffffffffLL)
    return hipErrorInvalidValue;
  uint32_t* counts = static_cast<uint32_t*>(ws);
  const dim3 grid((unsigned)bpc, N);
  hipLaunchKernelGGL(rs_finish_kernel, grid, dim3(kRsThreads), 0, s, rs, T, E, theta, counts);
  hipLaunchKernelGGL(rs_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, counts, (long long)N * bpc);
  hipLaunchKernelGGL(rs_compact_kernel, grid, dim3(kRsThreads), 0, s, rs, E, counts, index, value, capacity,
                     clip_off, N);
  return hipGetLastError();
}

hipError_t launch_residual_apply(const float* rs, float* xhat, int N, int T, int H, int W, hipStream_t s) {
  const long long E = 3LL * H * W, bpc = (E + kRsBlock - 1) / kRsBlock;
  if (N < 1 || N > 65535 || T < 1 || E < 16 || (E & 15)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rs_apply_kernel, dim3((unsigned)bpc, N), dim3(kRsThreads), 0, s, rs, xhat, T, E);
  return hipGetLastError();
}

hipError_t launch_blend(const float* prev, int Tp, float* cur, int N, int T, int H, int W, int nb, hipStream_t s) {
  const long long E = 3LL * H * W, bpc = (E + kRsBlock - 1) / kRsBlock;
  if (N < 1 || N > 65535 || nb < 1 || nb > 65535 || nb > T || nb > Tp || E < 16 || (E & 15)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(blend_kernel, dim3((unsigned)bpc, nb, N), dim3(kRsThreads), 0, s, prev, Tp, cur, T, nb, E);
  return hipGetLastError();
}

}  // namespace tok
