/*
 * tok.h - C ABI of the MI355X video-tokenizer library (libtok.so).
 *
 * The library implements the data-parallel hot path of the generative codec
 * of arXiv 2602.03529 ("Morphe"): the visual tokenizer's encoder f_phi,
 * finite scalar quantisation of the latent, token dropping with zero fill,
 * and the decoder g_theta (Sec. 2.4 defines f_phi / g_theta; Sec. 4.3 the
 * per-frame token matrices; Sec. 6.2 the zero fill of dropped and lost
 * tokens).  The paper does not publish the tokenizer's layer list, so the
 * network is a seeded stand-in of the same kind (causal 3-D convolutions,
 * GroupNorm+SiLU residual blocks, stride-2 down/up-sampling, FSQ):
 *
 *   encode: u8 -> x/127.5-1 -> conv 3->64 -> RB(64) x2 -> conv 64->128 /2
 *           -> conv 128->128 /2 -> 1x1 128->6 = z
 *   FSQ   : levels [8,8,8,5,5,5]: b = tanh(z+s)h - o, q = rint(b),
 *           codes = q / floor(L/2), idx = sum (q + floor(L/2)) * [1,8,64,512,2560,12800]
 *   drop  : codes *= keep (all 6 channels of a dropped token become 0)
 *   decode: 1x1 6->128 -> up x2 + conv 128->128 -> up x2 + conv 128->64
 *           -> RB(64) x2 -> conv 64->3 = x_hat
 *   RB(x) = x + conv(SiLU(GN(conv(SiLU(GN(x)))))), GN = GroupNorm(32) per frame.
 * All 3x3x3 convolutions are causal in time (two copies of frame 0 in front)
 * and zero-padded in space; the first latent frame depends on frame 0 only.
 *
 * Conventions
 *  - Every tensor argument is a DEVICE pointer unless marked "host".  The
 *    caller owns every tensor and the workspace; the library owns only the
 *    packed weights inside a tok_model.  No call allocates device memory
 *    except tok_model_create and tok_server_create.
 *  - Pixel and output tensors are dense NDHWC: x is uint8 (N,T,H,W,3),
 *    x_hat is float32 (N,T,H,W,3).  Latent tensors are dense float32
 *    (N,T2,H2,W2,6); idx is int32 (N,T2,H2,W2); keep is uint8 (N,T2,H2,W2).
 *    T2 = (T-1)/4 + 1, H2 = H/4, W2 = W/4.
 *  - Shapes: N >= 1, T >= 1 with T % 4 == 1, H and W positive multiples of 4.
 *    Violations return TOK_ESHAPE before anything is launched.
 *  - Every compute call is asynchronous on the given HIP stream; nothing
 *    synchronises the host.  Kernel faults surface as TOK_EDEVICE from a
 *    later call or from the caller's own synchronisation.
 *  - Results are deterministic (no floating-point atomics) and
 *    batch-invariant: a clip's outputs do not depend on the other clips of
 *    the batch.
 *  - Errors: every call returns a tok_status; nothing throws across the
 *    ABI.  tok_last_error() returns a thread-local description of the last
 *    failure.
 */
#ifndef TOK_H
#define TOK_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TOK_OK = 0,
  TOK_EINVAL = -1,        /* null pointer or invalid enum / argument */
  TOK_ESHAPE = -2,        /* tensor shape violates the constraints above */
  TOK_ENOMEM = -3,        /* device allocation failed (tok_model_create only) */
  TOK_EDEVICE = -4,       /* a HIP runtime call or kernel launch failed */
  TOK_EBUDGET = -5,       /* request can never fit the caller's memory budget */
  TOK_EUNSUPPORTED = -6,  /* precision / mode not available in this build */
  TOK_EWORKSPACE = -7     /* workspace smaller than tok_workspace_size */
} tok_status;

typedef enum {
  TOK_F32 = 0,       /* fp32 operands, fp32 MFMA, fp32 activations */
  TOK_BF16 = 1,      /* bf16 operands and activations, fp32 accumulate */
  TOK_FP8_E4M3 = 2   /* fp8 e4m3 operands, per-output-channel fp32 scales */
} tok_precision;

typedef enum {
  TOK_DROP_NONE = 0,       /* keep every token */
  TOK_DROP_BERNOULLI = 1,  /* token i = (t*H2 + h)*W2 + w of clip c dropped when
                              splitmix64(seed ^ c*0x9E3779B97F4A7C15 ^ i) >> 40
                              < floor(rate * 2^24) */
  TOK_DROP_ROWS = 2,       /* one draw per token-matrix row r = t*H2 + h with key
                              0x5A5A5A5A00000000 | r; a dropped row is a lost
                              packet of Sec. 6.2 and zeroes all W2 tokens */
  TOK_DROP_EXTERNAL = 3,   /* keep mask supplied by the caller (device, uint8) */
  TOK_DROP_SIMILARITY = 4  /* similarity-based token selection (Sec. 4.3, Eq. 3):
                              see tok_select_similar; only tok_encode and the
                              server take it (it needs the codes and scratch) */
} tok_drop_mode;

/* Token-drop request.  clip_id0: the hash id of clip 0 of the batch; clip n
 * uses clip_id0 + n, so a clip's mask does not depend on its batch-mates.
 * protect_iframe != 0 never drops latent frame 0 (the GoP's I frame). */
typedef struct {
  int mode;                  /* tok_drop_mode */
  float rate;                /* drop probability in [0, 1] (clamped) */
  uint64_t seed;
  uint64_t clip_id0;
  int protect_iframe;
  const uint8_t* ext_keep;   /* device (N,T2,H2,W2) for TOK_DROP_EXTERNAL, else NULL */
} tok_drop_desc;

typedef struct tok_model tok_model;

/* What a workspace is sized for.  TOK_WS_STREAM (or-ed in) sizes it for
 * causal temporal chunking: the clip is processed one latent frame (4 input
 * frames) at a time, each layer keeping the last 1-2 frames of its input, so
 * the workspace does not grow with T and the results are those of whole-clip
 * processing.  tok_encode / tok_decode process the whole clip at once when
 * the workspace they are given allows it, else in chunks. */
enum { TOK_WS_ENCODE = 1, TOK_WS_DECODE = 2, TOK_WS_ROUNDTRIP = 3, TOK_WS_STREAM = 16 };

/* Number of float32 values in the canonical weight blob (2,225,929): every
 * tensor in module order (encoder conv_in, rb1, rb2, down1, down2, proj;
 * decoder proj_in, up2, up1, rb1, rb2, conv_out), conv weights as
 * [Cout][Cin][kt][kh][kw] followed by the bias [Cout]; each residual block is
 * gn_a.gamma, gn_a.beta, a.w, a.b, gn_b.gamma, gn_b.beta, b.w, b.b. */
size_t tok_weight_count(void);

/* Copy the host float32 weight blob to `device`, convert it to `prec` and
 * pack it into the kernels' layouts.  *out receives the model handle.  The
 * model is read-only afterwards and may be used from several streams. */
tok_status tok_model_create(const float* host_weights, size_t n_floats, tok_precision prec,
                            int device, tok_model** out);
void tok_model_destroy(tok_model* model);

/* Bytes of device workspace that tok_encode / tok_decode need for a batch of
 * N clips of T x H x W pixels (`what` = TOK_WS_ENCODE / DECODE / ROUNDTRIP). */
tok_status tok_workspace_size(const tok_model* model, int N, int T, int H, int W, int what,
                              size_t* bytes);

/* Encoder f_phi followed by FSQ and the token mask, fused.
 * x: uint8 (N,T,H,W,3).  z: float32 pre-quantisation latent or NULL.
 * codes: float32 normalised codes, already multiplied by keep.  idx: int32
 * code indices (a dropped token keeps its true index).  drop: NULL = keep all;
 * TOK_DROP_SIMILARITY needs codes and runs tok_select_similar on them once
 * the whole batch is encoded, in the same workspace (tok_workspace_size
 * covers it).  keep: uint8 mask output or NULL.  ws: workspace of ws_bytes. */
tok_status tok_encode(tok_model* model, const uint8_t* x, int N, int T, int H, int W, float* z,
                      float* codes, int32_t* idx, const tok_drop_desc* drop, uint8_t* keep,
                      void* ws, size_t ws_bytes, hipStream_t stream);

/* FSQ alone on n_tokens float32 latent vectors z (n_tokens, 6):
 * codes (n_tokens, 6) float32, idx (n_tokens) int32.  Either output may be NULL. */
tok_status tok_quantize(const float* z, size_t n_tokens, float* codes, int32_t* idx,
                        hipStream_t stream);

/* Token dropping alone (Sec. 6.2 zero fill): builds keep (N,T2,H2,W2) from
 * `drop` and multiplies codes (N,T2,H2,W2,6) by it in place.  codes or keep
 * may be NULL (mask only / zero-fill only is not allowed: keep NULL means the
 * mask is not stored).  TOK_DROP_SIMILARITY is rejected (TOK_EINVAL): it
 * needs scratch memory, use tok_select_similar. */
tok_status tok_drop(const tok_drop_desc* drop, float* codes, uint8_t* keep, int N, int T2,
                    int H2, int W2, hipStream_t stream);

/* Similarity-based token selection (Sec. 4.3, Eq. 3).  Latent frame 0 of each
 * clip is its I-frame token matrix and is never dropped; the token of a later
 * (P) frame at (h, w) scores the cosine similarity of its FSQ code vector to
 * the I token at (h, w) (0 when either vector is zero).  Per clip, the
 * D = min(ceil(rate * N_P), N_P) most similar of the N_P = (T2-1) H2 W2 P
 * tokens are dropped, rate clamped to [0, 1]: the similarity threshold of
 * Sec. 4.3 is set by the bandwidth budget as a drop count.  Equal similarities
 * go to the lower token index i = (t H2 + h) W2 + w first, so the result is
 * unique.  Similarities are compared exactly (codes * 4 are integers, the
 * comparison is of rationals, not of rounded cosines).
 * codes: device float32 (N,T2,H2,W2,6), dropped tokens zero-filled in place.
 * keep: device uint8 (N,T2,H2,W2) output or NULL.  ws: device scratch of at
 * least tok_select_workspace_size bytes, 16-byte aligned; its contents are
 * not preserved.  codes must be 8-byte aligned.
 * Errors: TOK_EINVAL (null codes / ws), TOK_ESHAPE (N > 65535 or a clip of
 * 2^31 tokens or more), TOK_EWORKSPACE. */
tok_status tok_select_workspace_size(int N, int T2, int H2, int W2, size_t* bytes);
tok_status tok_select_similar(float rate, float* codes, uint8_t* keep, int N, int T2, int H2,
                              int W2, void* ws, size_t ws_bytes, hipStream_t stream);

/* tok_select_similar without a workspace argument and without any device
 * allocation, for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The selection's
 * scratch (order keys, digit histograms, selection state) is a static device
 * array of tok_select_scratch_bytes() bytes (32 MiB), one per GPU, held by
 * each GPU the library runs on until the process ends; the call uses the
 * array of the current device, so make the stream's device current.  Every
 * call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (several streams, several host threads) race and give wrong results;
 * serialise them.  Results equal tok_select_similar's bit for bit.  Batches
 * whose tok_select_workspace_size exceeds the array are rejected with
 * TOK_EWORKSPACE before anything is launched (e.g. 4 x 5 x 180 x 320 latents
 * need 3.7 MB, 2 x 9 x 270 x 480 need 8.3 MB).  Other errors as
 * tok_select_similar. */
tok_status tok_select_scratch_bytes(size_t* bytes);
tok_status tok_select_similar_noalloc(float rate, float* codes, uint8_t* keep, int N, int T2, int H2,
                                      int W2, hipStream_t stream);

/* ---- Token packets (Sec. 6.2) --------------------------------------------
 * The token matrices are sent row by row, one packet per row: a header with
 * the row number and a mask of the row's valid (not dropped) tokens, then the
 * valid tokens.  Rows of a batch are numbered g = (n T2 + t) H2 + h (for one
 * clip, the row of its token matrices).  Wire format, little-endian, every
 * field 4-byte aligned:
 *   u32 g
 *   u8  mask[ceil(W2/8)]   bit (w & 7) of byte (w >> 3) = 1: column w is valid
 *   u8  0 ...              padding to a multiple of 4 bytes
 *   u16 idx[count]         FSQ code index (< 64000) of each valid token, by column
 *   u16 0                  present when count is odd
 * Packets follow each other in row order with no gaps; every row gets a
 * packet, also one with no valid token. */

/* Upper bound of the stream length: every token valid. */
tok_status tok_packets_max_bytes(int N, int T2, int H2, int W2, size_t* bytes);

/* Sender.  idx: device int32 (N,T2,H2,W2) FSQ indices (tok_encode's idx), 4-byte aligned.
 * keep: device uint8 (N,T2,H2,W2) mask, or NULL for all valid.  out: device
 * buffer, 4-byte aligned, of out_bytes >= tok_packets_max_bytes bytes.
 * offsets: device uint64 [N T2 H2 + 1], receives each packet's byte offset in
 * out and, last, the stream's length.  Errors: TOK_EINVAL (null / misaligned
 * pointer), TOK_ESHAPE, TOK_EWORKSPACE (out too small). */
tok_status tok_packetize(const int32_t* idx, const uint8_t* keep, int N, int T2, int H2, int W2,
                         uint8_t* out, size_t out_bytes, uint64_t* offsets, hipStream_t stream);

/* Receiver.  buf: device bytes [bytes] holding the packets that arrived;
 * offsets: device uint64 [n_packets], where each starts in buf (any order).
 * codes: device float32 (N,T2,H2,W2,6), 8-byte aligned: every token is the
 * zero code vector except the valid tokens of the packets, which get the
 * code of their index.  keep: device uint8 (N,T2,H2,W2) or NULL: 1 exactly
 * at the tokens a packet delivered.  A packet whose row number is not below
 * N T2 H2 or which does not fit inside buf is skipped; a row must arrive at
 * most once (or its copies must be identical).  A lost packet and a row of
 * dropped tokens thus reach the decoder alike. */
tok_status tok_reassemble(const uint8_t* buf, size_t bytes, const uint64_t* offsets,
                          size_t n_packets, int N, int T2, int H2, int W2, float* codes,
                          uint8_t* keep, hipStream_t stream);

/* ---- Pixel residuals (Sec. 4.3, Eq. 4) -----------------------------------
 * Sender: x uint8 (N,T,H,W,3) clips (16-byte aligned), xhat float32
 * (N,T,H,W,3) their reconstructions (16-byte aligned), the averaging window
 * being a clip's T frames.  r: float32 (N,H,W,3) out, 16-byte aligned:
 * (1/T) sum_t (x_t/127.5 - 1 - xhat_t), sums in fp32 in frame order, with
 * every entry of magnitude below theta set to 0.  The non-zero entries of r
 * as a sparse list, clip by clip, each in increasing flat index
 * (h W + w) 3 + c: index (uint32) and value (float32) arrays of `capacity`
 * entries (entries past it are not written), clip_offsets uint64 [N + 1]:
 * clip n's entries are [clip_offsets[n], clip_offsets[n+1]) (the total may
 * exceed capacity; N H W 3 entries always fit).  ws: device scratch of
 * tok_residual_workspace_size bytes.  index, value and ws 4-byte aligned,
 * clip_offsets 8-byte aligned.  Needs H, W multiples of 4 and N H W 3 < 2^32. */
tok_status tok_residual_workspace_size(int N, int H, int W, size_t* bytes);
tok_status tok_residual_compress(const uint8_t* x, const float* xhat, int N, int T, int H, int W,
                                 float theta, float* r, uint32_t* index, float* value,
                                 size_t capacity, uint64_t* clip_offsets, void* ws,
                                 size_t ws_bytes, hipStream_t stream);
/* Receiver: xhat (N,T,H,W,3) += r (N,H,W,3) for every frame, in place. */
tok_status tok_residual_apply(const float* r, float* xhat, int N, int T, int H, int W,
                              hipStream_t stream);

/* ---- GoP-boundary blending (Sec. 4.2, Eq. 2) -----------------------------
 * xhat (N,T,H,W,3) is the current GoP's reconstruction, prev (N,T_prev,H,W,3)
 * the previous GoP's.  In place, frame i = 1..n (1-based) of xhat becomes
 * a_i prev[T_prev - n + i] + (1 - a_i) xhat[i] with a_i = (n - i) / n, in
 * fp32; later frames are untouched.  Needs 1 <= n <= T, T_prev; both buffers
 * 16-byte aligned. */
tok_status tok_gop_blend(const float* prev, int T_prev, float* xhat, int N, int T, int H, int W,
                         int n, hipStream_t stream);

/* tok_decode with the same blend fused into C_out's epilogue: the decoded
 * frames i = 1..n are written already blended with prev (N,T_prev,H,W,3,
 * float32, device), the previous GoP's reconstruction, so a stream of GoPs
 * is decoded and smoothed in one pass per GoP (overlapped-GoP streaming keeps
 * the last n frames of each output as the next call's prev, T_prev = n).
 * prev must not overlap xhat.  fp8 models blend in a separate pass after the
 * last layer (same arithmetic as tok_gop_blend) and need prev and xhat
 * 16-byte aligned.  Errors as tok_decode, plus TOK_EINVAL for a null or
 * misaligned prev or n outside 1..min(T, T_prev). */
tok_status tok_decode_blend(tok_model* model, const float* codes, int N, int T2, int H2, int W2,
                            const float* prev, int T_prev, int n, float* xhat, void* ws,
                            size_t ws_bytes, hipStream_t stream);

/* tok_decode followed by tok_residual_compress of the decoded clip (Sec. 4.3,
 * Eq. 4; the averaging window is the clip's T = 4(T2-1)+1 frames), with the
 * residual sums fused into C_out for bf16 models: as the last layer writes
 * each frame of x_hat it adds x_t/127.5 - 1 - x_hat_t, in fp32 and in frame
 * order, into r, so the separate pass over the T frames of x and x_hat is
 * not needed; then r becomes the thresholded mean and its non-zero entries
 * are listed.  Results equal tok_decode then tok_residual_compress bit for
 * bit (fp32 and fp8 models run exactly that).  x: uint8 (N,T,4 H2,4 W2,3)
 * source clips (device, 16-byte aligned); xhat, ws, ws_bytes as tok_decode;
 * r, index, value, capacity, clip_offsets as tok_residual_compress; rs_ws:
 * device scratch of tok_residual_workspace_size(N, 4 H2, 4 W2) bytes.
 * r's contents on entry are overwritten; r, xhat and x must not overlap.
 * Errors as tok_decode and tok_residual_compress. */
tok_status tok_decode_residual(tok_model* model, const float* codes, int N, int T2, int H2, int W2,
                               const uint8_t* x, float theta, float* xhat, float* r, uint32_t* index,
                               float* value, size_t capacity, uint64_t* clip_offsets, void* ws,
                               size_t ws_bytes, void* rs_ws, size_t rs_ws_bytes, hipStream_t stream);

/* Decoder g_theta: codes float32 (N,T2,H2,W2,6) -> x_hat float32
 * (N, 4(T2-1)+1, 4 H2, 4 W2, 3). */
tok_status tok_decode(tok_model* model, const float* codes, int N, int T2, int H2, int W2,
                      float* xhat, void* ws, size_t ws_bytes, hipStream_t stream);

/* Per-kernel timing.  Between tok_profile_begin and tok_profile_end every
 * kernel that tok_encode / tok_decode launch for `model` is bracketed by a
 * pair of HIP events recorded on the caller's stream.  tok_profile_end waits
 * for the last event, then writes for each kernel id k < n_ids the summed
 * duration ms[k] and the launch count count[k] (either may be NULL) and
 * frees the events.  Kernel ids: 0..15 the convolution layers in blob order
 * (conv_in, enc rb1.a, rb1.b, rb2.a, rb2.b, down1, down2, proj, proj_in, up2,
 * up1, dec rb1.a, rb1.b, rb2.a, rb2.b, conv_out; 7 and 8 are the fused
 * projection kernels), 16 GroupNorm finalize, 17 GroupNorm apply + SiLU,
 * and for tok_train_forward / tok_backward: 18 adjoint (input-gradient)
 * convolutions, 19 weight-gradient kernels, 20 GroupNorm+SiLU backward,
 * 21 other backward kernels, 22 similarity-based token selection (tok_encode
 * with TOK_DROP_SIMILARITY), 23 the residual layer of tok_decode_residual
 * (threshold, scan and compaction; for fp32 / fp8 models the whole separate
 * pass); tok_kernel_name(k) names them.
 * Profiling allocates events and is meant for measurement runs; do not
 * profile one model from several host threads at once. */
tok_status tok_profile_begin(tok_model* model);
tok_status tok_profile_end(tok_model* model, int n_ids, double* ms, int* count);
const char* tok_kernel_name(int k);

/* ---------------------------------------------------------------------------
 * Training step.  The codec is trained end to end and gradients flow through
 * the whole tokenizer (Sec. 4.1 gradient interface; Appendix, Eq. 5 l1 pixel
 * term, and Eq. 7 training on token-dropped latents).  Objective of the
 * stand-in:
 *   L = mean |x_hat - x| + 0.1 * mean (z~ - sg(c))^2
 * over the N*T*H*W*3 pixels and the M = N*T2*H2*W2*6 latent values, with
 * z~ = b / floor(L/2) the unrounded normalised code, c its FSQ code, the
 * decoder reading keep * c, the straight-through rule dc/dz~ = 1 and
 * sign(0) = 0 as the l1 subgradient.  tok_train_forward stores a tape of
 * block-boundary activations in the workspace; tok_backward recomputes each
 * residual block's interior from it (per-block checkpointing) and writes the
 * gradient of every parameter.
 * -------------------------------------------------------------------------*/

/* Replace the model's parameters by the device float32 blob `weights`
 * (canonical order, tok_weight_count() floats) and repack its kernels, on
 * `stream`.  Must not overlap with other work that uses the model. */
tok_status tok_model_set_weights(tok_model* model, const float* weights, hipStream_t stream);

/* Bytes of workspace for tok_train_forward + tok_backward on N clips of
 * T x H x W (whole clips; the tape lives in it between the two calls).  A
 * workspace of this size also keeps every residual block's interior
 * activations on the tape, so the backward does not recompute them. */
tok_status tok_train_workspace_size(const tok_model* model, int N, int T, int H, int W, size_t* bytes);

/* The smallest training workspace (per-block checkpointing): with fewer
 * bytes than tok_train_workspace_size the backward recomputes each residual
 * block's interior from the block input on the tape (same results, bit for
 * bit, for two more GroupNorm+SiLU passes and one conv per block).  The
 * forward and the backward of one step must get the same ws and ws_bytes. */
tok_status tok_train_workspace_min_size(const tok_model* model, int N, int T, int H, int W, size_t* bytes);

/* Forward pass of the objective.  x: uint8 (N,T,H,W,3).  keep: uint8
 * (N,T2,H2,W2) token mask (1 = kept) or NULL for all kept.  loss: device
 * float[3] receiving {L, l1 term, commitment mean}.  xhat, z (float32) and
 * idx (int32) are optional copies of the reconstruction, pre-quantisation
 * latent and code indices.  The tape stays valid in ws until the next call
 * that uses ws. */
tok_status tok_train_forward(tok_model* model, const uint8_t* x, int N, int T, int H, int W,
                             const uint8_t* keep, float* loss, float* xhat, float* z, int32_t* idx,
                             void* ws, size_t ws_bytes, hipStream_t stream);

/* Backward pass of the last tok_train_forward on the same x, shape and ws.
 * gloss: device float scalar dOut/dL (NULL = 1).  dweights: device float32
 * (tok_weight_count()) receiving dL/dparameters in canonical blob order
 * (every entry is written).  dx: optional float32 (N,T,H,W,3) receiving
 * dL/dx for the normalised input x/127.5 - 1. */
tok_status tok_backward(tok_model* model, const uint8_t* x, int N, int T, int H, int W,
                        const float* gloss, float* dweights, float* dx, void* ws, size_t ws_bytes,
                        hipStream_t stream);

/* Weight and bias gradient of one causal 3x3x3 convolution, the building
 * block tok_backward uses for every 3x3x3 layer:
 *   dw[o][i][kt][kh][kw] = sum over output positions p of dy[p][o] * x~[p + tap][i]
 *   db[o]                = sum over p of dy[p][o]
 * where x~ is the conv's input as the tap reads it (causal time clamp, zero
 * outside the frame).  view 0: stride 1 (To = Ti, Ho = Hi, Wo = Wi); view 1:
 * stride 2 (To = (Ti-1)/2+1, Ho = Hi/2, Wo = Wi/2); view 2: nearest x2
 * upsampled input (To = 2 Ti - 1, Ho = 2 Hi, Wo = 2 Wi).  x (N,Ti,Hi,Wi,Cin)
 * and dy (N,To,Ho,Wo,Cout) are device tensors of `prec` (TOK_F32 or
 * TOK_BF16) in the library's chunked activation layout
 * [N][T][ceil(C/CH)][H][W][CH], CH = 64 bytes / element size, channels past
 * C zero.  dw: float32 (Cout,Cin,3,3,3), db: float32 (Cout) or NULL.  Results
 * are deterministic (fixed-order reduction of per-split partials in ws). */
tok_status tok_conv3d_wgrad_workspace_size(tok_precision prec, int view, int N, int To, int Ho, int Wo, int Cin,
                                           int Cout, size_t* bytes);
tok_status tok_conv3d_wgrad(tok_precision prec, int view, const void* x, int N, int Ti, int Hi, int Wi, int Cin,
                            const void* dy, int To, int Ho, int Wo, int Cout, float* dw, float* db, void* ws,
                            size_t ws_bytes, hipStream_t stream);

/* Backward pass of the last tok_train_forward (same x, shape and ws) for
 * gradients of its outputs that come from the caller, e.g. a loss computed
 * outside the library: the codec is one differentiable stage of a larger
 * model (Sec. 4.1, the codec's internal gradient interface; Appendix Eq. 7,
 * gradients through the zero-filled decoder input).  Writes the gradient of
 *   <gxhat, x_hat> + <gcodes, keep * c> + <gz, z>
 * with respect to every parameter (dweights, canonical blob order, every
 * entry written) and, if dx is not NULL, to the normalised input
 * x/127.5 - 1 (float32 (N,T,H,W,3)).  x_hat is the reconstruction, keep * c
 * the zero-filled FSQ codes the decoder read (tok_train_codes), z the
 * pre-quantisation latent; the straight-through rule dc/dz~ = 1 applies and
 * dropped tokens pass no gradient from the decoder or from gcodes.  The
 * library's own loss terms do not enter.  gxhat: device float32 (N,T,H,W,3),
 * required; gcodes, gz: device float32 (N,T2,H2,W2,6) or NULL (zero).
 * Errors as tok_backward. */
tok_status tok_backward_outputs(tok_model* model, const uint8_t* x, int N, int T, int H, int W,
                                const float* gxhat, const float* gcodes, const float* gz,
                                float* dweights, float* dx, void* ws, size_t ws_bytes,
                                hipStream_t stream);

/* Copy the zero-filled codes keep * c (N,T2,H2,W2,6 float32) that the last
 * tok_train_forward on ws fed to the decoder. */
tok_status tok_train_codes(tok_model* model, int N, int T, int H, int W, float* codes,
                           const void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Per-operation entry points: the building blocks of the codec, each with its
 * adjoint, for torch.autograd.Function wrappers and for models that use the
 * codec's layers outside the fixed encode / decode graphs.  They run the same
 * kernels as tok_encode / tok_decode / tok_backward.
 *
 * prec is TOK_F32 or TOK_BF16 (TOK_EUNSUPPORTED otherwise).  Activations use
 * the library's chunked layout [N][T][ceil(C/CH)][H][W][CH] of prec, CH = 64
 * bytes / element size (16 fp32, 32 bf16), channels past C zero, 16-byte
 * aligned; tok_op_act_pack / tok_op_act_unpack convert from and to dense
 * channels-last float32.  Workspaces are device memory, 256-byte aligned, of
 * the size the matching *_workspace_size call returns; their contents are not
 * preserved.  Every call is asynchronous on `stream`; nothing allocates.
 * -------------------------------------------------------------------------*/

/* dense float32 [frames][HW][C] -> chunked activations of prec, and back
 * (frames = N T, HW = H W; channels past C are written as zero / dropped). */
tok_status tok_op_act_pack(tok_precision prec, const float* src, int frames, int HW, int C, void* dst,
                           hipStream_t stream);
tok_status tok_op_act_unpack(tok_precision prec, const void* src, int frames, int HW, int C,
                             float* dst, hipStream_t stream);

/* Causal 3x3x3 convolution (the encoder's and decoder's conv layers):
 *   y[n,t,h,w,o] = b[o] + sum over kt,kh,kw,i of w[o][i][kt][kh][kw] x~[n, s t + kt - 2,
 *                  s h + kh - 1, s w + kw - 1, i]   (+ resid[n,t,h,w,o])
 * with frame indices below 0 reading frame 0 (causal replicate padding) and
 * spatial indices outside the frame reading 0.  view 0: stride s = 1
 * (To,Ho,Wo = Ti,Hi,Wi); view 1: stride 2 in t, h, w (Ti odd, Hi and Wi even;
 * To = (Ti-1)/2+1, Ho = Hi/2, Wo = Wi/2: output frame 0 sees input frame 0
 * only); view 2: the input upsampled first by nearest x2 in h, w with time
 * map t -> ceil(t/2) (To = 2 Ti - 1, Ho = 2 Hi, Wo = 2 Wi), then stride 1.
 * w: device float32 [Cout][Cin][3][3][3]; b: device float32 [Cout] or NULL.
 * Channels: Cin and Cout multiples of 64 (chunked activations), or the first
 * layer Cin = 3 -> Cout = 64 at view 0, whose x is uint8 pixels (N,Ti,Hi,Wi,3)
 * normalised as x/127.5 - 1, or the last layer Cout = 3 at view 0, whose y
 * (and dy) is dense float32 (N,To,Ho,Wo,3).  resid: optional chunked tensor of
 * y's shape added to the output (view 0, Cout multiple of 64; it may alias y).
 * dgrad writes dx = J^T dy (dx of Cin = 3 is dense float32 (N,Ti,Hi,Wi,3), the
 * gradient for the normalised pixels); wgrad writes dw = dL/dw (same layout as
 * w, float32) and, if db is not NULL, db = dL/db, both deterministic.  Errors:
 * TOK_EINVAL (null / misaligned pointer, view outside 0..2), TOK_ESHAPE (shape
 * does not fit the view, N T above 65535), TOK_EUNSUPPORTED (channels or
 * precision), TOK_EWORKSPACE. */
tok_status tok_op_conv3d_workspace_size(tok_precision prec, int view, int N, int Ti, int Hi, int Wi,
                                        int Cin, int Cout, size_t* bytes);
tok_status tok_op_conv3d_fwd(tok_precision prec, int view, const void* x, int N, int Ti, int Hi,
                             int Wi, int Cin, const float* w, const float* b, const void* resid,
                             void* y, int Cout, void* ws, size_t ws_bytes, hipStream_t stream);
tok_status tok_op_conv3d_dgrad(tok_precision prec, int view, const void* dy, int N, int Ti, int Hi,
                               int Wi, int Cin, const float* w, void* dx, int Cout, void* ws,
                               size_t ws_bytes, hipStream_t stream);
tok_status tok_op_conv3d_wgrad(tok_precision prec, int view, const void* x, int N, int Ti, int Hi,
                               int Wi, int Cin, const void* dy, int Cout, float* dw, float* db,
                               void* ws, size_t ws_bytes, hipStream_t stream);

/* GroupNorm(32) with SiLU, per frame (the residual blocks' normalisation):
 * 64 channels in 32 groups of 2; the statistics of frame f and group g are
 * the mean and biased variance over the HW positions and the group's 2
 * channels.  x: chunked (frames = N T, HW = H W, 64 channels).
 * gn_stats: mean_rstd float32 [frames][32][2] = (mean, 1/sqrt(var + eps)).
 * gn_apply: y = SiLU((x - mean) rstd gamma[c] + beta[c]) (y may equal x).
 * gn_bwd:   dx = J^T dy of gn_apply at x (plus resid if not NULL; dx may
 *           alias dy or resid), dgamma[64] and dbeta[64] (written, not
 *           accumulated), deterministic.
 * gamma, beta: device float32 [64].  Errors: TOK_EINVAL, TOK_ESHAPE (frames
 * above 16383 (bf16: 32767) or empty), TOK_EUNSUPPORTED, TOK_EWORKSPACE. */
tok_status tok_op_gn_workspace_size(tok_precision prec, int frames, int HW, size_t* bytes);
tok_status tok_op_gn_stats(tok_precision prec, const void* x, int frames, int HW, float eps,
                           float* mean_rstd, void* ws, size_t ws_bytes, hipStream_t stream);
tok_status tok_op_gn_apply(tok_precision prec, const void* x, int frames, int HW,
                           const float* mean_rstd, const float* gamma, const float* beta, void* y,
                           void* ws, size_t ws_bytes, hipStream_t stream);
tok_status tok_op_gn_bwd(tok_precision prec, const void* x, const void* dy, int frames, int HW,
                         const float* mean_rstd, const float* gamma, const float* beta,
                         const void* resid, void* dx, float* dgamma, float* dbeta, void* ws,
                         size_t ws_bytes, hipStream_t stream);

/* Straight-through adjoint of FSQ (tok_quantize) on n_tokens latent vectors:
 *   gz = gz_in + keep * gcodes * (h / floor(L/2)) * (1 - tanh^2(z + s))
 * per channel (the rounding passes the gradient of the codes unchanged to
 * the unrounded b / floor(L/2), b = tanh(z + s) h - o).  z, gcodes, gz_in,
 * gz: device float32 (n_tokens, 6); keep: device uint8 (n_tokens) or NULL
 * (all kept); gcodes or gz_in may be NULL (zero).  gz may alias gz_in. */
tok_status tok_op_fsq_ste_bwd(const float* z, const uint8_t* keep, const float* gcodes,
                              const float* gz_in, size_t n_tokens, float* gz, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Streaming request loop (continuous batching under an HBM budget).
 *
 * The paper streams every 9-frame GoP through the codec in real time
 * (Sec. 7 codec wrapper: weights stay resident; Sec. 6: the sender encodes and
 * the receiver decodes continuously).  A tok_server owns one device arena of
 * `budget_bytes` (allocated once, at create) and `slots` HIP streams.  A
 * scheduler thread admits queued clips strictly oldest first, whenever a
 * stream slot is free and the clip's memory fits in the arena; the run of
 * consecutive queued clips of identical shape at the head of the queue (up to
 * `max_batch`) is admitted together as one batched launch.
 * Admitted work runs asynchronously and overlaps with work on the other
 * slots; memory returns to the arena when the client releases a result.
 * A clip's result does not depend on what it was batched with.
 * -------------------------------------------------------------------------*/
typedef struct tok_server tok_server;

typedef struct {
  int T, H, W;              /* clip shape (T % 4 == 1, H and W multiples of 4) */
  const uint8_t* pixels;    /* host (T,H,W,3) uint8; copied to the device at admission
                               (pinned memory makes the copy asynchronous) */
  tok_drop_desc drop;       /* per-clip token drop (NONE, BERNOULLI, ROWS or SIMILARITY); clip_id0 is
                               this clip's hash id */
} tok_request;

typedef struct {
  uint64_t ticket;
  tok_status status;        /* TOK_OK, or the error that ended the request */
  int T2, H2, W2;           /* latent grid */
  const float* codes;       /* device (T2,H2,W2,6), zero-filled by the drop mask */
  const int32_t* idx;       /* device (T2,H2,W2) */
  const uint8_t* keep;      /* device (T2,H2,W2) */
  const float* xhat;        /* device (T,H,W,3) reconstruction */
  double queue_ms;          /* submit -> admission */
  double run_ms;            /* admission -> completion observed by the scheduler */
  double total_ms;          /* submit -> completion */
  int batch_size;           /* clips in the launch this request ran in */
} tok_result;

/* Device bytes one clip of T x H x W occupies at least while admitted
 * (streaming workspace, pixels, latents and reconstruction).  The server runs
 * a launch on the whole-clip workspace when that takes at most a quarter of
 * the arena, else in causal temporal chunks. */
tok_status tok_server_request_bytes(const tok_model* model, int T, int H, int W, size_t* bytes);
tok_status tok_server_create(tok_model* model, size_t budget_bytes, int slots, int max_batch,
                             tok_server** out);
/* Queue a request; returns at once.  TOK_EBUDGET if the clip can never fit
 * the budget, TOK_ESHAPE for a bad shape (the request is not queued). */
tok_status tok_server_submit(tok_server* server, const tok_request* req, uint64_t* ticket);
/* Wait up to timeout_ms (negative: forever) for a request to finish.
 * TOK_OK with *out filled when done; TOK_EINVAL for an unknown ticket;
 * 1 (positive) when the time-out expired first. */
int tok_server_wait(tok_server* server, uint64_t ticket, int timeout_ms, tok_result* out);
/* Copy a finished request's results into caller buffers (device pointers,
 * any may be NULL; shapes as in tok_result), asynchronously on `stream`. */
tok_status tok_server_copy_result(tok_server* server, uint64_t ticket, float* codes, int32_t* idx,
                                  uint8_t* keep, float* xhat, hipStream_t stream);
/* Return a finished request's memory to the arena; its result pointers die. */
tok_status tok_server_release(tok_server* server, uint64_t ticket);
/* Counters: queued, running and finished requests, arena bytes in use and
 * the high-water mark. */
tok_status tok_server_stats(tok_server* server, int* queued, int* running, int* finished,
                            size_t* bytes_in_use, size_t* bytes_peak);
/* Waits for admitted work, fails queued requests, frees the arena. */
void tok_server_destroy(tok_server* server);

const char* tok_status_str(tok_status s);
const char* tok_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TOK_H */
