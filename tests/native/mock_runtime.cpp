// Host-only stand-ins for the HIP runtime calls and tok_* compute entry
// points that the streaming server uses, so that the server's scheduling,
// arena and batching logic can be exercised on a machine without a GPU.
// "Device" memory is host memory; a stream is a FIFO whose work completes a
// configurable delay after it is recorded; kernels write a deterministic
// pattern derived from the clip's pixels so results can be checked.
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "tok.h"

namespace {
std::mutex g_mu;
std::atomic<long long> g_delay_us{200};
using Clock = std::chrono::steady_clock;
struct MockEvent { Clock::time_point ready; };
std::unordered_map<void*, MockEvent*> g_events;
std::atomic<int> g_fail_encodes{0};
}  // namespace

extern "C" void mock_set_delay_us(long long us) { g_delay_us = us; }
// The next n tok_encode calls fail with TOK_EDEVICE (a launch that fails).
extern "C" void mock_fail_next_encodes(int n) { g_fail_encodes = n; }

hipError_t hipMalloc(void** p, size_t n) { *p = std::malloc(n); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t) {
  std::memmove(dst, src, n);
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = reinterpret_cast<hipStream_t>(new int(0)); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { delete reinterpret_cast<int*>(s); return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  auto* m = new MockEvent{Clock::now()};
  *e = reinterpret_cast<hipEvent_t>(m);
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) { delete reinterpret_cast<MockEvent*>(e); return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  reinterpret_cast<MockEvent*>(e)->ready = Clock::now() + std::chrono::microseconds(g_delay_us.load());
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  return Clock::now() >= reinterpret_cast<MockEvent*>(e)->ready ? hipSuccess : hipErrorNotReady;
}

extern "C" {
tok_status tok_workspace_size(const tok_model*, int N, int T, int H, int W, int what, size_t* bytes) {
  // Shape-dependent sizes with the same structure as the real plan: a whole
  // clip grows with T, a streamed one does not.
  const size_t frame = (size_t)H * W * 64 * 2;
  const int T2 = (T - 1) / 4 + 1;
  const int frames = (what & TOK_WS_STREAM) ? 26 : (3 * T + 6);
  (void)T2;
  *bytes = (size_t)N * frames * frame;  // untouched by the stand-in kernels
  return TOK_OK;
}
tok_status tok_encode(tok_model*, const uint8_t* x, int N, int T, int H, int W, float* z, float* codes,
                      int32_t* idx, const tok_drop_desc*, uint8_t* keep, void*, size_t, hipStream_t) {
  if (g_fail_encodes.load() > 0) {
    --g_fail_encodes;
    return TOK_EDEVICE;
  }
  const size_t tok = (size_t)((T - 1) / 4 + 1) * (H / 4) * (W / 4);
  const size_t pix = (size_t)T * H * W * 3;
  for (int n = 0; n < N; ++n) {
    const float v = (float)x[(size_t)n * pix];  // clip's first pixel byte identifies it
    for (size_t i = 0; i < tok; ++i) {
      for (int c = 0; c < 6; ++c) codes[((size_t)n * tok + i) * 6 + c] = v + c;
      idx[(size_t)n * tok + i] = (int32_t)v;
    }
    if (keep) std::memset(keep + (size_t)n * tok, 1, tok);
    if (z) std::memset(z + (size_t)n * tok * 6, 0, tok * 6 * 4);
  }
  return TOK_OK;
}
tok_status tok_drop(const tok_drop_desc*, float*, uint8_t* keep, int N, int T2, int H2, int W2, hipStream_t) {
  if (keep) std::memset(keep, 1, (size_t)N * T2 * H2 * W2);
  return TOK_OK;
}
tok_status tok_select_similar(float, float*, uint8_t* keep, int N, int T2, int H2, int W2, void*, size_t,
                              hipStream_t) {
  if (keep) std::memset(keep, 1, (size_t)N * T2 * H2 * W2);
  return TOK_OK;
}
tok_status tok_decode(tok_model*, const float* codes, int N, int T2, int H2, int W2, float* xhat, void*, size_t,
                      hipStream_t) {
  const size_t tok = (size_t)T2 * H2 * W2;
  const size_t px = (size_t)(4 * (T2 - 1) + 1) * (4 * H2) * (4 * W2) * 3;
  for (int n = 0; n < N; ++n) xhat[(size_t)n * px] = codes[(size_t)n * tok * 6];  // first value marks the clip
  return TOK_OK;
}
}
