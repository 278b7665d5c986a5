// C ABI of the coding steps around the tokenizer: row packets and their
// reassembly (Sec. 6.2), the pixel-residual layer (Sec. 4.3, Eq. 4) and
// GoP-boundary blending (Sec. 4.2, Eq. 2).  Argument checks here, kernels in
// packets.hip and enhance.hip.
#include <string>

#include "tok.h"
#include "tok_model.h"

using namespace tok;

namespace {

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

bool latent_ok(int N, int T2, int H2, int W2) { return N >= 1 && T2 >= 1 && H2 >= 1 && W2 >= 1; }

bool pixels_ok(int N, int T, int H, int W) {
  return N >= 1 && N <= 65535 && T >= 1 && H >= 4 && W >= 4 && H % 4 == 0 && W % 4 == 0 &&
         (long long)N * 3 * H * W < 0xffffffffLL;
}

}  // namespace

tok_status tok_packets_max_bytes(int N, int T2, int H2, int W2, size_t* bytes) {
  if (!bytes) return fail(TOK_EINVAL, "null argument");
  if (!latent_ok(N, T2, H2, W2)) return fail(TOK_ESHAPE, "bad latent shape");
  *bytes = (size_t)packets_max_bytes(N, T2, H2, W2);
  return TOK_OK;
}

tok_status tok_packetize(const int32_t* idx, const uint8_t* keep, int N, int T2, int H2, int W2, uint8_t* out,
                         size_t out_bytes, uint64_t* offsets, hipStream_t s) {
  if (!idx || !out || !offsets) return fail(TOK_EINVAL, "null argument");
  if (!latent_ok(N, T2, H2, W2) || (long long)N * T2 * H2 > 0xffffffffLL)
    return fail(TOK_ESHAPE, "bad latent shape (at most 2^32 - 1 rows)");
  if (!aligned(out, 4) || !aligned(offsets, 8) || !aligned(idx, 4))
    return fail(TOK_EINVAL, "idx and out must be 4-byte, offsets 8-byte aligned");
  if (out_bytes < (size_t)packets_max_bytes(N, T2, H2, W2))
    return fail(TOK_EWORKSPACE, "out smaller than tok_packets_max_bytes");
  TOK_HIP(launch_packetize(idx, keep, N, T2, H2, W2, out, reinterpret_cast<unsigned long long*>(offsets), s));
  return TOK_OK;
}

tok_status tok_reassemble(const uint8_t* buf, size_t bytes, const uint64_t* offsets, size_t n_packets, int N, int T2,
                          int H2, int W2, float* codes, uint8_t* keep, hipStream_t s) {
  if (!codes || (n_packets && (!buf || !offsets))) return fail(TOK_EINVAL, "null argument");
  if (!latent_ok(N, T2, H2, W2) || (long long)N * T2 * H2 > 0xffffffffLL) return fail(TOK_ESHAPE, "bad latent shape");
  if (!aligned(codes, 8) || !aligned(offsets, 8)) return fail(TOK_EINVAL, "codes and offsets must be 8-byte aligned");
  TOK_HIP(launch_reassemble(buf, bytes, reinterpret_cast<const unsigned long long*>(offsets), (long long)n_packets, N,
                            T2, H2, W2, codes, keep, s));
  return TOK_OK;
}

tok_status tok_residual_workspace_size(int N, int H, int W, size_t* bytes) {
  if (!bytes) return fail(TOK_EINVAL, "null argument");
  if (!pixels_ok(N, 1, H, W)) return fail(TOK_ESHAPE, "need H, W multiples of 4 and N H W 3 < 2^32");
  *bytes = residual_ws_bytes(N, H, W);
  return TOK_OK;
}

tok_status tok_residual_compress(const uint8_t* x, const float* xhat, int N, int T, int H, int W, float theta,
                                 float* r, uint32_t* index, float* value, size_t capacity, uint64_t* clip_offsets,
                                 void* ws, size_t ws_bytes, hipStream_t s) {
  if (!x || !xhat || !r || !clip_offsets || !ws || (capacity && (!index || !value)))
    return fail(TOK_EINVAL, "null argument");
  if (!pixels_ok(N, T, H, W)) return fail(TOK_ESHAPE, "need H, W multiples of 4 and N H W 3 < 2^32");
  if (!aligned(x, 16) || !aligned(xhat, 16) || !aligned(r, 16) || !aligned(clip_offsets, 8) || !aligned(ws, 4) ||
      !aligned(index, 4) || !aligned(value, 4))
    return fail(TOK_EINVAL, "x, xhat and r must be 16-byte, clip_offsets 8-byte, ws, index and value 4-byte aligned");
  if (ws_bytes < residual_ws_bytes(N, H, W)) return fail(TOK_EWORKSPACE, "workspace too small");
  TOK_HIP(launch_residual(x, xhat, N, T, H, W, theta, r, index, value, (long long)capacity,
                          reinterpret_cast<unsigned long long*>(clip_offsets), ws, s));
  return TOK_OK;
}

tok_status tok_residual_apply(const float* r, float* xhat, int N, int T, int H, int W, hipStream_t s) {
  if (!r || !xhat) return fail(TOK_EINVAL, "null argument");
  if (!pixels_ok(N, T, H, W)) return fail(TOK_ESHAPE, "need H, W multiples of 4 and N H W 3 < 2^32");
  if (!aligned(r, 16) || !aligned(xhat, 16)) return fail(TOK_EINVAL, "r and xhat must be 16-byte aligned");
  TOK_HIP(launch_residual_apply(r, xhat, N, T, H, W, s));
  return TOK_OK;
}

tok_status tok_gop_blend(const float* prev, int T_prev, float* xhat, int N, int T, int H, int W, int n,
                         hipStream_t s) {
  if (!prev || !xhat) return fail(TOK_EINVAL, "null argument");
  if (!pixels_ok(N, T, H, W) || n < 1 || n > T || n > T_prev) return fail(TOK_ESHAPE, "need 1 <= n <= T, T_prev");
  if (!aligned(prev, 16) || !aligned(xhat, 16)) return fail(TOK_EINVAL, "prev and xhat must be 16-byte aligned");
  TOK_HIP(launch_blend(prev, T_prev, xhat, N, T, H, W, n, s));
  return TOK_OK;
}
