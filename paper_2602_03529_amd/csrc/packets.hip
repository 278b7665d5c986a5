// Token packets of the streaming protocol (Sec. 6.2): one packet per row of a
// token matrix, header = row number + position mask, payload = the valid
// tokens; the receiver puts valid tokens back and zero-fills the rest.
//
// Wire format (little-endian, fields 4-byte aligned), rows of all clips of a
// batch numbered g = (n T2 + t') H2 + h':
//   u32 g | u8 mask[ceil(W2/8)] (bit w&7 of byte w>>3 = column w valid), zero
//   padding to a multiple of 4 | u16 FSQ index of each valid token by column,
//   plus one zero u16 if their count is odd.
// Packets follow each other in row order.
//
// Sender: pk_size_kernel (one wave per row: packet size) -> pk_scan_kernel (one
// workgroup: exclusive scan of the sizes into byte offsets) -> pk_write_kernel
// (one wave per row: header, mask from ballots, payload compacted by ballot
// prefix counts).  Receiver: rx_clear_kernel (codes and keep to zero) ->
// rx_scatter_kernel (one wave per received packet, byte loads only, so any
// offset is safe; packets that do not fit in the buffer or name a row outside
// the batch are skipped).
#include "tok_internal.h"
#include "tok_device.h"

namespace tok {

namespace {

constexpr int kPkThreads = 256;
constexpr int kPkRows = kPkThreads / 64;  // rows (one per wave) per workgroup
constexpr int kScanThreads = 1024;

__host__ __device__ inline int mask_field_bytes(int W2) { return 4 * (((W2 + 7) / 8 + 3) / 4); }
__host__ __device__ inline long long packet_size(int W2, int count) {
  return 4 + mask_field_bytes(W2) + 4 * ((count + 1) / 2);
}

__device__ __forceinline__ unsigned long long lanes_below(int lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// offsets[g] = size of packet g.
__global__ void __launch_bounds__(kPkThreads) pk_size_kernel(const uint8_t* __restrict__ keep, long long G, int W2,
                                                              unsigned long long* __restrict__ offsets) {
  const long long g = (long long)blockIdx.x * kPkRows + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (g >= G) return;
  int count = 0;
  for (int w0 = 0; w0 < W2; w0 += 64) {
    const int w = w0 + lane;
    const bool k = w < W2 && (keep == nullptr || keep[g * W2 + w] != 0);
    count += __popcll(__ballot(k));
  }
  if (lane == 0) offsets[g] = (unsigned long long)packet_size(W2, count);
}

// In place: offsets[0..G) sizes -> exclusive prefix sums, offsets[G] = total.
// One workgroup; thread t owns a contiguous run of ceil(G / 1024) entries.
__global__ void __launch_bounds__(kScanThreads) pk_scan_kernel(unsigned long long* __restrict__ offsets, long long G) {
  __shared__ unsigned long long part[kScanThreads];
  const int t = threadIdx.x;
  const long long per = (G + kScanThreads - 1) / kScanThreads;
  const long long a = t * per, b = a + per < G ? a + per : G;
  unsigned long long sum = 0;
  for (long long i = a; i < b; ++i) sum += offsets[i];
  part[t] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread sums
  for (int o = 1; o < kScanThreads; o <<= 1) {
    const unsigned long long v = t >= o ? part[t - o] : 0ull;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  unsigned long long run = part[t] - sum;
  for (long long i = a; i < b; ++i) {
    const unsigned long long sz = offsets[i];
    offsets[i] = run;
    run += sz;
  }
  if (t == kScanThreads - 1) offsets[G] = part[t];
}

__global__ void __launch_bounds__(kPkThreads) pk_write_kernel(const int32_t* __restrict__ idx,
                                                               const uint8_t* __restrict__ keep, long long G, int W2,
                                                               const unsigned long long* __restrict__ offsets,
                                                               uint8_t* __restrict__ out) {
  const long long g = (long long)blockIdx.x * kPkRows + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (g >= G) return;
  uint8_t* base = out + offsets[g];
  const int MB = mask_field_bytes(W2);
  uint16_t* pay = reinterpret_cast<uint16_t*>(base + 4 + MB);
  if (lane == 0) *reinterpret_cast<uint32_t*>(base) = (uint32_t)g;
  int count = 0;
  for (int w0 = 0; w0 < W2; w0 += 64) {
    const int w = w0 + lane;
    const bool k = w < W2 && (keep == nullptr || keep[g * W2 + w] != 0);
    const unsigned long long m = __ballot(k);
    // bytes w0/8 .. w0/8 + 7 of the mask field (columns beyond W2 are 0 bits;
    // bytes past the field belong to the payload and are not written here)
    const int byte = (w0 >> 3) + lane;
    if (lane < 8 && byte < MB) base[4 + byte] = (uint8_t)(m >> (8 * lane));
    if (k) pay[count + __popcll(m & lanes_below(lane))] = (uint16_t)idx[g * W2 + w];
    count += __popcll(m);
  }
  if (lane == 0 && (count & 1)) pay[count] = 0;
}

__global__ void __launch_bounds__(kPkThreads) rx_clear_kernel(float* __restrict__ codes, uint8_t* __restrict__ keep,
                                                               long long tokens) {
  const long long i = (long long)blockIdx.x * kPkThreads + threadIdx.x;
  if (i >= tokens) return;
  float2* c2 = reinterpret_cast<float2*>(codes + i * 6);
  const float2 z = make_float2(0.f, 0.f);
  c2[0] = z;
  c2[1] = z;
  c2[2] = z;
  if (keep) keep[i] = 0;
}

__device__ __forceinline__ uint32_t load_u8(const uint8_t* p) { return *p; }

// FSQ code of index v for levels (8, 8, 8, 5, 5, 5): digit_c = (v / beta_c) mod L_c,
// code_c = (digit_c - floor(L_c/2)) / floor(L_c/2); exact in fp32.
__device__ __forceinline__ void index_to_code(uint32_t v, float* c) {
  const uint32_t d0 = v % 8u, d1 = (v / 8u) % 8u, d2 = (v / 64u) % 8u;
  const uint32_t d3 = (v / 512u) % 5u, d4 = (v / 2560u) % 5u, d5 = (v / 12800u) % 5u;
  c[0] = ((float)d0 - 4.f) * 0.25f;
  c[1] = ((float)d1 - 4.f) * 0.25f;
  c[2] = ((float)d2 - 4.f) * 0.25f;
  c[3] = ((float)d3 - 2.f) * 0.5f;
  c[4] = ((float)d4 - 2.f) * 0.5f;
  c[5] = ((float)d5 - 2.f) * 0.5f;
}

__global__ void __launch_bounds__(kPkThreads) rx_scatter_kernel(const uint8_t* __restrict__ buf,
                                                                 unsigned long long bytes,
                                                                 const unsigned long long* __restrict__ offs,
                                                                 long long n_packets, long long G, int W2,
                                                                 float* __restrict__ codes,
                                                                 uint8_t* __restrict__ keep) {
  const long long p = (long long)blockIdx.x * kPkRows + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (p >= n_packets) return;
  const unsigned long long off = offs[p];
  const int MB = mask_field_bytes(W2);
  if (off > bytes || bytes - off < (unsigned long long)(4 + MB)) return;
  const uint8_t* base = buf + off;
  const uint32_t g = load_u8(base) | load_u8(base + 1) << 8 | load_u8(base + 2) << 16 | load_u8(base + 3) << 24;
  if ((long long)g >= G) return;
  // valid count (columns < W2 only), then the size check
  int count = 0;
  for (int w0 = 0; w0 < W2; w0 += 64) {
    const int w = w0 + lane;
    const bool k = w < W2 && ((load_u8(base + 4 + (w >> 3)) >> (w & 7)) & 1u);
    count += __popcll(__ballot(k));
  }
  if (bytes - off < (unsigned long long)packet_size(W2, count)) return;
  const uint8_t* pay = base + 4 + MB;
  int run = 0;
  for (int w0 = 0; w0 < W2; w0 += 64) {
    const int w = w0 + lane;
    const bool k = w < W2 && ((load_u8(base + 4 + (w >> 3)) >> (w & 7)) & 1u);
    const unsigned long long m = __ballot(k);
    if (k) {
      const int pos = run + __popcll(m & lanes_below(lane));
      const uint32_t v = load_u8(pay + 2 * pos) | load_u8(pay + 2 * pos + 1) << 8;
      float c[6];
      index_to_code(v, c);
      const long long tok = (long long)g * W2 + w;
      float2* c2 = reinterpret_cast<float2*>(codes + tok * 6);
      c2[0] = make_float2(c[0], c[1]);
      c2[1] = make_float2(c[2], c[3]);
      c2[2] = make_float2(c[4], c[5]);
      if (keep) keep[tok] = 1;
    }
    run += __popcll(m);
  }
}

}  // namespace

long long packets_max_bytes(int N, int T2, int H2, int W2) {
  return (long long)N * T2 * H2 * packet_size(W2, W2);
}

hipError_t launch_packetize(const int32_t* idx, const uint8_t* keep, int N, int T2, int H2, int W2, uint8_t* out,
                            unsigned long long* offsets, hipStream_t s) {
  const long long G = (long long)N * T2 * H2;
  if (G < 1 || W2 < 1) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)((G + kPkRows - 1) / kPkRows);
  hipLaunchKernelGGL(pk_size_kernel, dim3(grid), dim3(kPkThreads), 0, s, keep, G, W2, offsets);
  hipLaunchKernelGGL(pk_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, offsets, G);
  hipLaunchKernelGGL(pk_write_kernel, dim3(grid), dim3(kPkThreads), 0, s, idx, keep, G, W2, offsets, out);
  return hipGetLastError();
}

hipError_t launch_reassemble(const uint8_t* buf, unsigned long long bytes, const unsigned long long* offsets,
                             long long n_packets, int N, int T2, int H2, int W2, float* codes, uint8_t* keep,
                             hipStream_t s) {
  const long long G = (long long)N * T2 * H2, tokens = G * W2;
  if (G < 1 || W2 < 1 || n_packets < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rx_clear_kernel, dim3((unsigned)((tokens + kPkThreads - 1) / kPkThreads)), dim3(kPkThreads), 0,
                     s, codes, keep, tokens);
  if (n_packets > 0)
    hipLaunchKernelGGL(rx_scatter_kernel, dim3((unsigned)((n_packets + kPkRows - 1) / kPkRows)), dim3(kPkThreads), 0,
                       s, buf, bytes, offsets, n_packets, G, W2, codes, keep);
  return hipGetLastError();
}

}  // namespace tok
