// Model state and launch helpers shared by the C-ABI translation units
// (tok_api.hip: inference, tok_train.hip: training step).  Not public.
#pragma once

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "tok.h"
#include "tok_internal.h"

namespace tok {

// Records `msg` as the calling thread's last error and returns s.
tok_status fail(tok_status s, const std::string& msg);

#define TOK_HIP(call)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return ::tok::fail(TOK_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

#define TOK_TRY(x)                 \
  do {                             \
    tok_status s_ = (x);           \
    if (s_ != TOK_OK) return s_;   \
  } while (0)

// ---------------------------------------------------------------------------
// Parameter table (canonical blob order, see tok_weight_count in tok.h)
// ---------------------------------------------------------------------------
enum LayerId {
  L_CONV_IN = 0, L_E_RB1_A, L_E_RB1_B, L_E_RB2_A, L_E_RB2_B, L_DOWN1, L_DOWN2, L_PROJ,
  L_PROJ_IN, L_UP2, L_UP1, L_D_RB1_A, L_D_RB1_B, L_D_RB2_A, L_D_RB2_B, L_CONV_OUT, L_COUNT
};
enum NormId { N_E_RB1_A = 0, N_E_RB1_B, N_E_RB2_A, N_E_RB2_B, N_D_RB1_A, N_D_RB1_B, N_D_RB2_A, N_D_RB2_B, N_COUNT };

struct ConvSpec { int cout, cin, k; };
inline constexpr ConvSpec kConv[L_COUNT] = {
    {64, 3, 3},   {64, 64, 3},  {64, 64, 3},  {64, 64, 3},  {64, 64, 3},  {128, 64, 3},
    {128, 128, 3}, {6, 128, 1}, {128, 6, 1},  {128, 128, 3}, {64, 128, 3}, {64, 64, 3},
    {64, 64, 3},  {64, 64, 3},  {64, 64, 3},  {3, 64, 3}};

// Layers of the decoder g_theta (the only ones an fp8 model holds).
inline bool is_decoder_layer(int l) { return l >= L_PROJ_IN; }

// Addressing mode of each 3x3x3 layer's forward conv.
inline int conv_mode(int l) {
  if (l == L_CONV_IN) return CM_I2C;
  if (l == L_DOWN1 || l == L_DOWN2) return CM_S2;
  if (l == L_UP2 || l == L_UP1) return CM_UPF;
  return CM_S1;
}

// Mode of each 3x3x3 layer's input-gradient conv (the packed adjoint kernel):
// polyphase for the strided layers, and for the upsampling layers in fp32
// (in bf16 the dense adjoint at the fine resolution is faster: the polyphase
// form stages twice the bytes per output of the strided forward conv).
inline int adj_mode(int l, int prec) {
  if (conv_mode(l) == CM_S2) return CM_S2T;
  if (conv_mode(l) == CM_UPF && prec == P_F32) return CM_UPT;
  return CM_S1T;
}

constexpr float kGnEps = 1e-6f;
constexpr float kCommitWeight = 0.1f;

FsqConst make_fsq_const();

// Kernel ids of the per-launch profile (tok_profile_end).
enum KernelId {
  K_GN_FINAL = 16, K_GN_ACT = 17, K_DGRAD = 18, K_WGRAD = 19, K_GN_BWD = 20, K_BWD_MISC = 21, K_SELECT = 22,
  K_RESID = 23, K_IDS = 24
};

inline int cdiv(int a, int b) { return (a + b - 1) / b; }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Dims {
  int N, T, H, W, T1, H1, W1, T2, H2, W2;
};

inline bool make_dims(int N, int T, int H, int W, Dims* d) {
  if (N < 1 || T < 1 || H < 4 || W < 4) return false;
  if ((T - 1) % 4 != 0 || H % 4 != 0 || W % 4 != 0) return false;
  d->N = N; d->T = T; d->H = H; d->W = W;
  d->T1 = (T - 1) / 2 + 1; d->H1 = H / 2; d->W1 = W / 2;
  d->T2 = (d->T1 - 1) / 2 + 1; d->H2 = H / 4; d->W2 = W / 4;
  return true;
}

}  // namespace tok

struct ProfRec {
  int id;
  hipEvent_t a, b;
};

// Device-resident model.  `blob` is the canonical fp32 parameter vector;
// biases, GroupNorm affines and the 1x1x1 weights are read from it in place,
// and the 3x3x3 kernels are packed from it on the device (forward layout and,
// for the backward, the adjoint layout).
struct tok_model {
  bool profiling = false;
  std::vector<ProfRec> prof;
  int device = 0;
  int prec = tok::P_BF16;
  void* mem = nullptr;              // one device allocation holding everything below
  float* blob = nullptr;            // canonical parameters
  size_t w_off[tok::L_COUNT] = {}, b_off[tok::L_COUNT] = {};  // float offsets into blob
  size_t g_off[tok::N_COUNT] = {}, be_off[tok::N_COUNT] = {};
  void* wpk[tok::L_COUNT] = {};     // packed 3x3x3 forward kernels
  void* wpkT[tok::L_COUNT] = {};    // packed adjoint kernels
  int nt[tok::L_COUNT] = {}, ntT[tok::L_COUNT] = {};
  const float* bias[tok::L_COUNT] = {};
  const float* w1x1[tok::L_COUNT] = {};   // [Cout][Cin] for the 1x1x1 layers
  float* w1x1T[tok::L_COUNT] = {};        // their transposes [Cin][Cout]
  const float* gamma[tok::N_COUNT] = {};
  const float* beta[tok::N_COUNT] = {};
  const float* zeros = nullptr;     // 128 zero floats (bias of the adjoint convs)
  float* wscale[tok::L_COUNT] = {};  // fp8 models: per-output-channel weight scales
};

namespace tok {

// Records an event pair around the launches made while it is alive (profiling only).
struct Timed {
  tok_model* m;
  hipStream_t s;
  ProfRec r;
  bool on;
  Timed(const tok_model* mc, int id, hipStream_t st) : m(const_cast<tok_model*>(mc)), s(st), on(mc->profiling) {
    if (!on) return;
    r.id = id;
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) { on = false; return; }
    hipEventRecord(r.a, s);
  }
  ~Timed() {
    if (!on) return;
    hipEventRecord(r.b, s);
    m->prof.push_back(r);
  }
};

}  // namespace tok
