// Warm-start decoder: constants and host-side launchers (kernels in kernels_dec.hip).
//
// Layouts (bf16 = bfloat16 stored as uint16_t; B = batch):
//   "TC"  time-major activations  [B][T][C]          (channels contiguous; MFMA operand rows)
//   "CT"  channel-major rows      [B][C][8 + T + 8]  (8 zero samples on each side)
//   "P"   polyphase channel rows  [B][C][s][8 + T/s + 8], element (c, r, m) = value at t = s m + r
// Weights: master FP32 [C_out][C_in][9]; forward copy bf16 [C_out][9][C_in_pad];
// data-gradient copy bf16 [C_in][9][C_out]; the output layer keeps FP32 values of its
// bf16-rounded weights [C_in][9].
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace jtfs {

constexpr int kDecC = 128;        // hidden channels
constexpr int kDecK = 9;          // taps per filter
constexpr int kDecH = 4;          // (taps - 1) / 2
constexpr int kDecPad = 8;        // zero samples at each end of a CT / P row
constexpr int kDecTile = 64;      // time rows per workgroup tile
constexpr int kDecChunk = 4096;   // longest run of time samples per weight-gradient partial
constexpr int kDecOutChunk = 2048;

// Time samples per weight-gradient partial of a hidden layer with t input samples: 4096,
// halved (down to 512) while the launch, batch * ceil(t / chunk) * (cip / 64) workgroups
// times s polyphase rows (9 taps at stride 1), would give the 256 CUs fewer than two each.
inline int dec_wgrad_chunk(int batch, int t, int cip, int s) {
  const int64_t z = int64_t(cip / 64) * (s == 1 ? kDecK : s);
  int chunk = kDecChunk;
  while (chunk > 512 && int64_t(batch) * ((t + chunk - 1) / chunk) * z < 512) chunk /= 2;
  return chunk;
}
inline int64_t dec_chunks(int batch, int t, int chunk) { return int64_t(batch) * ((t + chunk - 1) / chunk); }
inline int64_t dec_out_chunks(int batch, int t) { return int64_t(batch) * ((t + kDecOutChunk - 1) / kDecOutChunk); }

// Weight copies of one layer from the FP32 master [c_out][c_in][9].
hipError_t run_dec_cast(const float* W, int c_in, int cip, int c_out, uint16_t* wf, uint16_t* wd, float* wout,
                        hipStream_t st);
// The weight copies of every layer in one launch: layer l's master W[l] ([c_out][c_in][9]),
// its forward copy wf[l] and data-gradient copy wd[l] (either may be null) or, for the
// one-channel output layer, its rounded FP32 copy wout (non-null only there).
constexpr int kDecMaxLayers = 8;
struct DecCastSet {
  const float* W[kDecMaxLayers];
  uint16_t* wf[kDecMaxLayers];
  uint16_t* wd[kDecMaxLayers];
  int c_in[kDecMaxLayers], cip[kDecMaxLayers], c_out[kDecMaxLayers];
  int64_t end[kDecMaxLayers];   // running end of layer l's elements (wf, then wd, then wout)
  float* wout;
  int n;
};
hipError_t run_dec_cast_all(const DecCastSet& set, hipStream_t st);
// a_0 = bf16(log1p(S / eps)) in TC [B][F][cip] and CT layouts; S is [B][c_in][F] FP32.
hipError_t run_dec_input(const float* S, int batch, int c_in, int F, int cip, float eps, uint16_t* x_tc,
                         uint16_t* x_ct, hipStream_t st);
// Hidden layer forward: out = lrelu(b + W * up_s(x)), written TC and CT.
hipError_t run_dec_conv_fwd(int s, const uint16_t* x_tc, int cip, int t_in, int batch, const uint16_t* wf,
                            const float* bias, float leak, uint16_t* out_tc, uint16_t* out_ct, hipStream_t st);
// Output layer forward (stride 1, one channel): y = b + sum_{c,k} w[c][k] x[c][t + k - 4], FP32.
hipError_t run_dec_out_fwd(const uint16_t* x_ct, int T, int batch, const float* wout, const float* bias, float* y,
                           hipStream_t st);
// Output layer backward: dz of the last hidden layer (TC + P with that layer's stride s2),
// masked by its activation, and the weight/bias partials.
hipError_t run_dec_out_bwd(const float* dy, int T, int batch, const float* wout, const uint16_t* a_tc,
                           const uint16_t* a_ct, float leak, int s2, uint16_t* dz_tc, uint16_t* dzp, float* part,
                           float* grad_w, float* grad_b, hipStream_t st);
// Hidden layer data gradient: dz_prev = lrelu'(a_prev) * (W^T-adjoint of dz), written TC and P
// (P with the previous layer's stride s2).
hipError_t run_dec_dgrad(int s, int s2, const uint16_t* dz_tc, int t_out, const uint16_t* wd, int t_in, int batch,
                         const uint16_t* a_prev_tc, float leak, uint16_t* dz_prev_tc, uint16_t* dzp_prev,
                         hipStream_t st);
// Hidden layer weight and bias gradients from dz (P layout, stride s) and the layer input (CT).
hipError_t run_dec_wgrad(int s, const uint16_t* dzp, const uint16_t* x_ct, int t_in, int cip, int c_in, int batch,
                         float* part, float* grad_w, float* grad_b, hipStream_t st);
// Adam on the FP32 master parameters (bias corrections bc1 = 1 - beta1^t, bc2 = 1 - beta2^t).
hipError_t run_dec_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                        float eps, float bc1, float bc2, hipStream_t st);
// Per-signal loss: loss[i] = scale sum w (S_i - T_i)^2 / (relative ? sum w T_i^2 : 1), dS_i its
// gradient, w = w0 on the first n0 coefficients (the zeroth-order block) and 1 elsewhere.
hipError_t run_rel_loss(const float* S, const float* T, float* dS, float* loss, int64_t n, int64_t n0, float w0,
                        int relative, float scale, hipStream_t st);

}  // namespace jtfs
