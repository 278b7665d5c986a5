// Token-level kernels of scalable coding (Sec. 4.3): similarity-based token
// selection (Eq. 3).
//
// Per clip, the D P-frame tokens with the highest cosine similarity to the I
// token at the same spatial location are dropped (codes zero-filled, keep = 0),
// ties going to the lower token index.  The selection is an exact top-D over
// unique 64-bit keys, (similarity order key << 32) | (2^32 - 1 - token index),
// done as a radix select with 8-bit digits from the top:
//   sel_key_kernel    one 32-bit similarity key per P token, clears the histograms
//   sel_pass_kernel   x8: histogram of the next digit among the tokens that
//                     match the digits chosen so far; each workgroup first
//                     derives the previous pass's digit from its histogram
//   sel_apply_kernel  keep mask and zero fill against the D-th largest key
// No workgroup waits for another and no device-scope fence is needed: a
// histogram is read only by launches after the one that built it.
// Every count is an integer, so the result does not depend on the order in
// which workgroups run.
#include "tok_internal.h"
#include "tok_device.h"

#include <mutex>

namespace tok {

namespace {

constexpr int kSelThreads = 256;
constexpr int kSelItems = 8;  // keys per thread in a histogram pass
constexpr int kSelTile = kSelThreads * kSelItems;
constexpr int kSelKeyItems = 4;  // tokens per thread in the key kernel
constexpr int kSelPasses = 8;    // 8-bit digits of the 64-bit selection key

struct SelState {
  unsigned long long prefix;  // digits chosen so far (8 per finished pass)
  unsigned need;              // how many of the remaining candidates are still to drop
  unsigned pad;
};

struct SelWs {
  uint32_t* keys;  // [N][NP] similarity keys of the P tokens
  uint32_t* hist;  // [N][8][256] digit histograms
  SelState* st0;   // [N] state before pass 0 (need = D)
  SelState* st;    // [N][8] selection state after each pass
};

SelWs carve(void* ws, int N, long long NP) {
  char* p = static_cast<char*>(ws);
  auto take = [&](size_t bytes) {
    char* q = p;
    p += (bytes + 255) & ~(size_t)255;
    return q;
  };
  SelWs w;
  w.keys = reinterpret_cast<uint32_t*>(take((size_t)N * NP * 4));
  w.hist = reinterpret_cast<uint32_t*>(take((size_t)N * kSelPasses * 256 * 4));
  w.st0 = reinterpret_cast<SelState*>(take((size_t)N * sizeof(SelState)));
  w.st = reinterpret_cast<SelState*>(take((size_t)N * kSelPasses * sizeof(SelState)));
  return w;
}

// Exact order key of the cosine similarity S of Eq. 3 between a P token and
// the I token at the same location.  With v = 4 c (FSQ codes times 4 are
// integers in [-4, 4], |v|^2 <= 96), S orders as sign(dot) dot^2 / nn with
// nn = |v_P|^2 |v_I|^2 <= 9216: two different such fractions differ by at
// least 1 / 9216^2 > 2^-27, so floor(dot^2 2^30 / nn) keeps every strict
// order and every tie.  Returned biased to [0, 2^31] (S = 0, also for a
// zero norm, maps to 2^30).
__device__ __forceinline__ uint32_t sim_key(const float* p, const float* q) {
  const float2* p2 = reinterpret_cast<const float2*>(p);
  const float2* q2 = reinterpret_cast<const float2*>(q);
  int dot = 0, np = 0, nq = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float2 u = p2[c], v = q2[c];
    const int a0 = (int)rintf(4.f * u.x), a1 = (int)rintf(4.f * u.y);
    const int b0 = (int)rintf(4.f * v.x), b1 = (int)rintf(4.f * v.y);
    dot += a0 * b0 + a1 * b1;
    np += a0 * a0 + a1 * a1;
    nq += b0 * b0 + b1 * b1;
  }
  const uint64_t nn = (uint64_t)np * (uint64_t)nq;
  if (nn == 0 || dot == 0) return 1u << 30;
  const uint64_t mag = ((uint64_t)(dot * dot) << 30) / nn;  // <= 2^30 (Cauchy-Schwarz)
  return dot > 0 ? (uint32_t)((1u << 30) + mag) : (uint32_t)((1u << 30) - mag);
}

__device__ __forceinline__ uint64_t composite(uint32_t key, long long token) {
  return ((uint64_t)key << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)token);
}

// grid (ceil(NP / 1024), N).  Workgroup 0 of a clip also clears its
// histograms and sets the initial selection state (the pass kernels run after
// this one on the same stream).
__global__ void __launch_bounds__(kSelThreads) sel_key_kernel(const float* __restrict__ codes, SelWs w, int T2,
                                                               int HW, long long NP, unsigned D) {
  const int n = blockIdx.y, tid = threadIdx.x;
  if (blockIdx.x == 0) {
    for (int b = tid; b < kSelPasses * 256; b += kSelThreads) w.hist[(size_t)n * kSelPasses * 256 + b] = 0;
    if (tid == 0) w.st0[n] = SelState{0ull, D, 0u};
  }
  const float* clip = codes + (size_t)n * T2 * HW * 6;
#pragma unroll
  for (int k = 0; k < kSelKeyItems; ++k) {
    const long long j = ((long long)blockIdx.x * kSelKeyItems + k) * kSelThreads + tid;
    if (j < NP) {
      const long long i = j + HW;
      w.keys[(size_t)n * NP + j] = sim_key(clip + (size_t)i * 6, clip + (size_t)(j % HW) * 6);
    }
  }
}

// Adds one to hist[digit] for every lane with cand set.  A wave whose
// candidates all share one digit (common: equal codes give equal keys) makes
// a single LDS atomic.
__device__ __forceinline__ void wave_hist_add(uint32_t* hist, bool cand, unsigned dg, int lane) {
  const unsigned long long m = __ballot(cand);
  if (!m) return;
  const int first = __ffsll((long long)m) - 1;
  const unsigned d0 = __shfl(dg, first, 64);
  const unsigned long long same = __ballot(cand && dg == d0);
  if (same == m) {
    if (lane == first) atomicAdd(&hist[d0], (unsigned)__popcll(m));
  } else if (cand) {
    atomicAdd(&hist[dg], 1u);
  }
}

// Selection state after pass `pass` of clip n, from the state after the
// previous pass and that pass's finished histogram (wave 0 of the calling
// workgroup; lane 0 returns it).  Lane l holds bins 255-4l .. 252-4l
// (highest first); the digit is the bin where the running count from the top
// first reaches `need` (the candidates number at least `need`, so one does).
__device__ SelState next_state(const SelWs& w, int n, int pass, int lane) {
  const SelState prev = pass == 0 ? w.st0[n] : w.st[n * kSelPasses + pass - 1];
  const uint32_t* hist = w.hist + ((size_t)n * kSelPasses + pass) * 256;
  uint32_t c[4], sum = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    c[q] = hist[255 - 4 * lane - q];
    sum += c[q];
  }
  uint32_t incl = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  const unsigned need = prev.need;
  const unsigned long long m = __ballot(incl >= need);
  const int L = __ffsll((long long)m) - 1;
  uint32_t cum = incl - sum;
  int q = 0;
  for (; q < 3; ++q) {
    if (cum + c[q] >= need) break;
    cum += c[q];
  }
  SelState s;
  s.prefix = (prev.prefix << 8) | (unsigned long long)(255 - 4 * lane - q);
  s.need = need - cum;
  s.pad = 0;
  // broadcast lane L's result
  s.prefix = __shfl(s.prefix, L, 64);
  s.need = __shfl(s.need, L, 64);
  return s;
}

// grid (ceil(NP / kSelTile), N).  Pass p > 0 first derives the digit of pass
// p - 1 (every workgroup alike, from the histogram the previous launch
// finished) and stores the state, identically from every workgroup, for the
// next launch; no workgroup waits for another.
__global__ void __launch_bounds__(kSelThreads) sel_pass_kernel(SelWs w, long long NP, int HW, int pass) {
  __shared__ uint32_t wh[kSelThreads / 64][256];
  __shared__ unsigned long long s_prefix;
  const int n = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int b = tid; b < (kSelThreads / 64) * 256; b += kSelThreads) (&wh[0][0])[b] = 0;
  if (pass > 0 && wv == 0) {
    const SelState s = next_state(w, n, pass - 1, lane);
    if (lane == 0) {
      s_prefix = s.prefix;
      w.st[n * kSelPasses + pass - 1] = s;
    }
  }
  __syncthreads();
  const unsigned long long prefix = pass > 0 ? s_prefix : 0ull;
  const int shift = 56 - 8 * pass;
  const int hs = pass == 0 ? 0 : shift + 8;  // the chosen digits sit above bit hs
  const uint32_t* keys = w.keys + (size_t)n * NP;
#pragma unroll 4
  for (int k = 0; k < kSelItems; ++k) {
    const long long j = ((long long)blockIdx.x * kSelItems + k) * kSelThreads + tid;
    bool cand = j < NP;
    unsigned dg = 0;
    if (cand) {
      const uint64_t c = composite(keys[j], j + HW);
      cand = pass == 0 || (c >> hs) == prefix;
      dg = (unsigned)(c >> shift) & 255u;
    }
    wave_hist_add(wh[wv], cand, dg, lane);
  }
  __syncthreads();
  uint32_t tot = 0;
#pragma unroll
  for (int q = 0; q < kSelThreads / 64; ++q) tot += wh[q][tid];
  if (tot) atomicAdd(&w.hist[((size_t)n * kSelPasses + pass) * 256 + tid], tot);
}

enum { SEL_KEEP_ALL = 0, SEL_DROP_ALL_P = 1, SEL_THRESHOLD = 2 };

// grid (ceil(T2 HW / 1024), N): keep for every token of the clip, zero fill of
// the dropped ones, 4 tokens per thread.  Latent frame 0 (the I frame) is
// always kept.
__global__ void __launch_bounds__(kSelThreads) sel_apply_kernel(float* __restrict__ codes, uint8_t* __restrict__ keep,
                                                                 SelWs w, int T2, int HW, long long NP, int mode) {
  __shared__ unsigned long long s_thr;
  const int n = blockIdx.y, tid = threadIdx.x;
  if (mode == SEL_THRESHOLD) {
    // the D-th largest key: the digits of the first 7 passes and the last pass's histogram
    if (tid < 64) {
      const SelState s = next_state(w, n, kSelPasses - 1, tid);
      if (tid == 0) s_thr = s.prefix;
    }
    __syncthreads();
  }
  const long long per = (long long)T2 * HW;
#pragma unroll
  for (int k = 0; k < kSelKeyItems; ++k) {
    const long long i = ((long long)blockIdx.x * kSelKeyItems + k) * kSelThreads + tid;
    if (i >= per) break;
    bool drop = false;
    if (i >= HW) {
      if (mode == SEL_DROP_ALL_P) drop = true;
      else if (mode == SEL_THRESHOLD) drop = composite(w.keys[(size_t)n * NP + (i - HW)], i) >= s_thr;
    }
    if (keep) keep[(size_t)n * per + i] = drop ? 0 : 1;
    if (drop) {
      float2* c2 = reinterpret_cast<float2*>(codes + ((size_t)n * per + i) * 6);
      const float2 z = make_float2(0.f, 0.f);
      c2[0] = z;
      c2[1] = z;
      c2[2] = z;
    }
  }
}

}  // namespace

size_t similarity_ws_bytes(int N, int T2, int H2, int W2) {
  const long long NP = (long long)(T2 - 1) * H2 * W2;
  auto a = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return a((size_t)N * NP * 4) + a((size_t)N * kSelPasses * 256 * 4) + a((size_t)N * sizeof(SelState)) +
         a((size_t)N * kSelPasses * sizeof(SelState));
}

// Selection scratch for callers that cannot allocate: one array per GPU,
// held until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host the name is a stand-in, not a device address): each
// device's address comes from hipGetSymbolAddress, taken once per device
// with that device current.
namespace {
static __device__ __align__(256) unsigned char scratch[kSimilarityScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t similarity_scratch(void** ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_similarity_drop(float* codes, uint8_t* keep, int N, int T2, int H2, int W2, long long D, void* ws,
                                  hipStream_t s) {
  const long long HW = (long long)H2 * W2, NP = (long long)(T2 - 1) * HW;
  if (N < 1 || N > 65535 || T2 < 1 || HW < 1 || D < 0 || D > NP || (long long)T2 * HW > 0x7fffffffLL)
    return hipErrorInvalidValue;
  if ((reinterpret_cast<uintptr_t>(codes) & 7) != 0) return hipErrorInvalidValue;
  int mode = SEL_THRESHOLD;
  if (D == 0) mode = SEL_KEEP_ALL;
  if (D == NP) mode = SEL_DROP_ALL_P;
  SelWs w{};
  if (mode == SEL_THRESHOLD) {
    if (!ws) return hipErrorInvalidValue;
    w = carve(ws, N, NP);
    const long long kg = (NP + kSelKeyItems * kSelThreads - 1) / (kSelKeyItems * kSelThreads);
    hipLaunchKernelGGL(sel_key_kernel, dim3((unsigned)kg, N), dim3(kSelThreads), 0, s, codes, w, T2, (int)HW, NP,
                       (unsigned)D);
    const long long pg = (NP + kSelTile - 1) / kSelTile;
    for (int pass = 0; pass < kSelPasses; ++pass)
      hipLaunchKernelGGL(sel_pass_kernel, dim3((unsigned)pg, N), dim3(kSelThreads), 0, s, w, NP, (int)HW, pass);
  }
  const long long ag = ((long long)T2 * HW + kSelKeyItems * kSelThreads - 1) / (kSelKeyItems * kSelThreads);
  hipLaunchKernelGGL(sel_apply_kernel, dim3((unsigned)ag, N), dim3(kSelThreads), 0, s, codes, keep, w, T2, (int)HW,
                     NP, mode);
  return hipGetLastError();
}

}  // namespace tok
