// C ABI of the warm-start decoder (include/jtfs.h): configuration checks, workspace
// layout and the order of the kernel launches. Every launch goes to the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "../../include/jtfs.h"
#include "dec.hpp"

namespace jtfs {
jtfs_status report(jtfs_status s, const std::string& msg);
}

namespace {

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

struct Layer {
  int c_in, cip, c_out, stride, t_in, t_out;
  int64_t w_off, b_off;                      // floats into the parameter vector
  size_t wf = 0, wd = 0;                     // bf16 weight copies (hidden layers)
  size_t out_tc = 0, out_ct = 0;             // output activation (hidden layers)
  size_t dz_tc = 0, dzp = 0;                 // gradient of the pre-activation (hidden layers)
};

}  // namespace

struct jtfs_dec_s {
  jtfs_dec_config cfg;
  int32_t max_batch = 0;
  std::vector<Layer> layers;
  int cip0 = 0;
  size_t x_tc = 0, x_ct = 0, wout = 0, part = 0, ws_bytes = 0;
  int64_t n_params = 0, out_len = 0;
};

namespace {

jtfs_status build(jtfs_dec_s& d) {
  const jtfs_dec_config& c = d.cfg;
  const int L = c.n_layers;
  const int64_t B = d.max_batch;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  d.cip0 = (c.c_in + 63) / 64 * 64;
  int64_t T = c.n_frames, p = 0;
  int ci = c.c_in;
  size_t part_bytes = 0;
  for (int l = 0; l < L; ++l) {
    Layer ly;
    ly.c_in = ci;
    ly.cip = l == 0 ? d.cip0 : jtfs::kDecC;
    ly.c_out = l == L - 1 ? 1 : jtfs::kDecC;
    ly.stride = c.stride[l];
    ly.t_in = static_cast<int>(T);
    T *= ly.stride;
    if (T > (int64_t(1) << 26)) return jtfs::report(JTFS_ERR_UNSUPPORTED, "decoder output longer than 2^26 samples");
    ly.t_out = static_cast<int>(T);
    ly.w_off = p;
    p += int64_t(ly.c_out) * ly.c_in * jtfs::kDecK;
    ly.b_off = p;
    p += ly.c_out;
    if (l < L - 1) {
      ly.wf = take(size_t(jtfs::kDecC) * jtfs::kDecK * ly.cip * 2);
      if (l > 0) ly.wd = take(size_t(jtfs::kDecC) * jtfs::kDecK * jtfs::kDecC * 2);
      ly.out_tc = take(size_t(B) * ly.t_out * jtfs::kDecC * 2);
      ly.out_ct = take(size_t(B) * jtfs::kDecC * (ly.t_out + 2 * jtfs::kDecPad) * 2);
      ly.dz_tc = take(size_t(B) * ly.t_out * jtfs::kDecC * 2);
      ly.dzp = take(size_t(B) * jtfs::kDecC * ly.stride * (ly.t_in + 2 * jtfs::kDecPad) * 2);
      // weight partials, then the bias partials: 128 per chunk and polyphase row (strides 2 and 4)
      // or per batch item (stride 1); the chunk length depends on the batch, so take the largest
      // size over batches up to B
      for (int64_t b = 1; b <= B; ++b) {
        const int64_t n = jtfs::dec_chunks(static_cast<int>(b), ly.t_in,
                                           jtfs::dec_wgrad_chunk(static_cast<int>(b), ly.t_in, ly.cip, ly.stride));
        part_bytes = std::max(part_bytes, (size_t(n) * jtfs::kDecK * jtfs::kDecC * ly.cip +
                                           size_t(std::max<int64_t>(n * ly.stride, b)) * jtfs::kDecC) * sizeof(float));
      }
    } else {
      // weight partials, then one bias partial per 8192 samples of dy
      part_bytes = std::max(part_bytes, (size_t(jtfs::dec_out_chunks(static_cast<int>(B), ly.t_out)) * jtfs::kDecC *
                                             jtfs::kDecK + size_t((B * ly.t_out + 8191) / 8192)) * sizeof(float));
    }
    d.layers.push_back(ly);
    ci = ly.c_out;
  }
  d.x_tc = take(size_t(B) * c.n_frames * d.cip0 * 2);
  d.x_ct = take(size_t(B) * d.cip0 * (c.n_frames + 2 * jtfs::kDecPad) * 2);
  d.wout = take(size_t(jtfs::kDecC) * jtfs::kDecK * sizeof(float));
  d.part = take(part_bytes);
  d.ws_bytes = off;
  d.n_params = p;
  d.out_len = T;
  return JTFS_OK;
}

template <class T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

#define DEC_HIP(expr)                                                                        \
  do {                                                                                       \
    const hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return jtfs::report(JTFS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

jtfs_status check_call(jtfs_dec_t dec, int32_t batch, const void* ws, size_t ws_bytes) {
  if (!dec || !ws) return jtfs::report(JTFS_ERR_ARG, "NULL argument");
  if (batch < 1 || batch > dec->max_batch) return jtfs::report(JTFS_ERR_ARG, "batch outside [1, max_batch]");
  if (ws_bytes < dec->ws_bytes) return jtfs::report(JTFS_ERR_WORKSPACE, "workspace smaller than the decoder needs");
  return JTFS_OK;
}

}  // namespace

extern "C" {

jtfs_status jtfs_dec_create(const jtfs_dec_config* cfg, int32_t max_batch, jtfs_dec_t* out) {
  if (!out) return jtfs::report(JTFS_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!cfg || max_batch < 1) return jtfs::report(JTFS_ERR_ARG, "need a configuration and max_batch >= 1");
  if (cfg->channels != jtfs::kDecC || cfg->kernel != jtfs::kDecK)
    return jtfs::report(JTFS_ERR_UNSUPPORTED, "decoder needs channels = 128 and kernel = 9");
  if (cfg->c_in < 1 || cfg->c_in > 4096) return jtfs::report(JTFS_ERR_ARG, "c_in outside [1, 4096]");
  if (cfg->n_frames < 8 || cfg->n_frames % 8 != 0) return jtfs::report(JTFS_ERR_ARG, "n_frames must be a positive multiple of 8");
  if (cfg->n_layers < 2 || cfg->n_layers > JTFS_DEC_MAX_LAYERS) return jtfs::report(JTFS_ERR_ARG, "n_layers outside [2, 8]");
  for (int l = 0; l < cfg->n_layers; ++l) {
    const int s = cfg->stride[l];
    if (s != 1 && s != 2 && s != 4) return jtfs::report(JTFS_ERR_ARG, "strides must be 1, 2 or 4");
  }
  if (cfg->stride[cfg->n_layers - 1] != 1) return jtfs::report(JTFS_ERR_UNSUPPORTED, "the last layer must have stride 1");
  if (!(cfg->leak > 0.f && cfg->leak <= 1.f)) return jtfs::report(JTFS_ERR_ARG, "leak outside (0, 1]");
  if (!(cfg->eps > 0.f) || !std::isfinite(cfg->eps)) return jtfs::report(JTFS_ERR_ARG, "eps must be positive");
  jtfs_dec_s* d = new (std::nothrow) jtfs_dec_s;
  if (!d) return jtfs::report(JTFS_ERR_NOMEM, "host allocation failed");
  d->cfg = *cfg;
  d->max_batch = max_batch;
  const jtfs_status st = build(*d);
  if (st != JTFS_OK) {
    delete d;
    return st;
  }
  *out = d;
  return JTFS_OK;
}

jtfs_status jtfs_dec_query(jtfs_dec_t dec, int64_t* n_params, int64_t* out_len, size_t* ws_bytes) {
  if (!dec) return jtfs::report(JTFS_ERR_ARG, "NULL decoder");
  if (n_params) *n_params = dec->n_params;
  if (out_len) *out_len = dec->out_len;
  if (ws_bytes) *ws_bytes = dec->ws_bytes;
  return JTFS_OK;
}

jtfs_status jtfs_dec_forward(jtfs_dec_t dec, const float* params, const float* S, int32_t batch, float* y, void* ws,
                             size_t ws_bytes, jtfs_stream_t stream) {
  jtfs_status r = check_call(dec, batch, ws, ws_bytes);
  if (r != JTFS_OK) return r;
  if (!params || !S || !y) return jtfs::report(JTFS_ERR_ARG, "NULL argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const jtfs_dec_config& c = dec->cfg;
  const auto& Ls = dec->layers;
  const int L = c.n_layers;
  // every layer's bfloat16 weight copies (and the output layer's rounded FP32 copy) in one launch
  jtfs::DecCastSet cs{};
  cs.n = L;
  cs.wout = at<float>(ws, dec->wout);
  int64_t run = 0;
  for (int l = 0; l < L; ++l) {
    const Layer& ly = Ls[l];
    cs.W[l] = params + ly.w_off;
    cs.c_in[l] = ly.c_in;
    cs.c_out[l] = ly.c_out;
    if (l < L - 1) {
      cs.cip[l] = ly.cip;
      cs.wf[l] = at<uint16_t>(ws, ly.wf);
      cs.wd[l] = l > 0 ? at<uint16_t>(ws, ly.wd) : nullptr;
      run += int64_t(ly.c_out) * jtfs::kDecK * ly.cip + (l > 0 ? int64_t(ly.c_in) * jtfs::kDecK * ly.c_out : 0);
    } else {
      cs.cip[l] = ly.c_in;
      run += int64_t(ly.c_out) * ly.c_in * jtfs::kDecK;
    }
    cs.end[l] = run;
  }
  DEC_HIP(jtfs::run_dec_cast_all(cs, st));
  DEC_HIP(jtfs::run_dec_input(S, batch, c.c_in, c.n_frames, dec->cip0, c.eps, at<uint16_t>(ws, dec->x_tc),
                              at<uint16_t>(ws, dec->x_ct), st));
  for (int l = 0; l < L - 1; ++l) {
    const Layer& ly = Ls[l];
    const uint16_t* in = l == 0 ? at<uint16_t>(ws, dec->x_tc) : at<uint16_t>(ws, Ls[l - 1].out_tc);
    DEC_HIP(jtfs::run_dec_conv_fwd(ly.stride, in, ly.cip, ly.t_in, batch, at<uint16_t>(ws, ly.wf), params + ly.b_off,
                                   c.leak, at<uint16_t>(ws, ly.out_tc), at<uint16_t>(ws, ly.out_ct), st));
  }
  const Layer& lo = Ls[L - 1];
  DEC_HIP(jtfs::run_dec_out_fwd(at<uint16_t>(ws, Ls[L - 2].out_ct), lo.t_out, batch, at<float>(ws, dec->wout),
                                params + lo.b_off, y, st));
  return JTFS_OK;
}

jtfs_status jtfs_dec_backward(jtfs_dec_t dec, const float* params, int32_t batch, const float* dy, float* grad,
                              void* ws, size_t ws_bytes, jtfs_stream_t stream) {
  jtfs_status r = check_call(dec, batch, ws, ws_bytes);
  if (r != JTFS_OK) return r;
  if (!params || !dy || !grad) return jtfs::report(JTFS_ERR_ARG, "NULL argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const jtfs_dec_config& c = dec->cfg;
  const auto& Ls = dec->layers;
  const int L = c.n_layers;
  float* part = at<float>(ws, dec->part);
  const Layer& lo = Ls[L - 1];
  const Layer& lh = Ls[L - 2];
  DEC_HIP(jtfs::run_dec_out_bwd(dy, lo.t_out, batch, at<float>(ws, dec->wout), at<uint16_t>(ws, lh.out_tc),
                                at<uint16_t>(ws, lh.out_ct), c.leak, lh.stride, at<uint16_t>(ws, lh.dz_tc),
                                at<uint16_t>(ws, lh.dzp), part, grad + lo.w_off, grad + lo.b_off, st));
  for (int l = L - 2; l >= 0; --l) {
    const Layer& ly = Ls[l];
    const uint16_t* x_ct = l == 0 ? at<uint16_t>(ws, dec->x_ct) : at<uint16_t>(ws, Ls[l - 1].out_ct);
    DEC_HIP(jtfs::run_dec_wgrad(ly.stride, at<uint16_t>(ws, ly.dzp), x_ct, ly.t_in, ly.cip, ly.c_in, batch, part,
                                grad + ly.w_off, grad + ly.b_off, st));
    if (l > 0) {
      const Layer& lp = Ls[l - 1];
      DEC_HIP(jtfs::run_dec_dgrad(ly.stride, lp.stride, at<uint16_t>(ws, ly.dz_tc), ly.t_out, at<uint16_t>(ws, ly.wd),
                                  ly.t_in, batch, at<uint16_t>(ws, lp.out_tc), c.leak, at<uint16_t>(ws, lp.dz_tc),
                                  at<uint16_t>(ws, lp.dzp), st));
    }
  }
  return JTFS_OK;
}

jtfs_status jtfs_dec_adam_step(jtfs_dec_t dec, float* params, const float* grad, float* m, float* v, int64_t step,
                               float lr, float beta1, float beta2, float eps, jtfs_stream_t stream) {
  if (!dec || !params || !grad || !m || !v) return jtfs::report(JTFS_ERR_ARG, "NULL argument");
  if (step < 1) return jtfs::report(JTFS_ERR_ARG, "step counts from 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
    return jtfs::report(JTFS_ERR_ARG, "bad Adam hyperparameters");
  const float bc1 = static_cast<float>(1.0 - std::pow(double(beta1), double(step)));
  const float bc2 = static_cast<float>(1.0 - std::pow(double(beta2), double(step)));
  DEC_HIP(jtfs::run_dec_adam(params, grad, m, v, dec->n_params, lr, beta1, beta2, eps, bc1, bc2,
                             static_cast<hipStream_t>(stream)));
  return JTFS_OK;
}

jtfs_status jtfs_dec_ws_region(jtfs_dec_t dec, int32_t layer, int32_t which, size_t* offset, size_t* bytes) {
  if (!dec || !offset || !bytes) return jtfs::report(JTFS_ERR_ARG, "NULL argument");
  if (layer < 0 || layer >= dec->cfg.n_layers - 1) return jtfs::report(JTFS_ERR_ARG, "not a hidden layer");
  const Layer& ly = dec->layers[layer];
  if (which != 0 && which != 1) return jtfs::report(JTFS_ERR_ARG, "which must be 0 (activation) or 1 (its gradient)");
  *offset = which == 0 ? ly.out_tc : ly.dz_tc;
  *bytes = size_t(dec->max_batch) * ly.t_out * jtfs::kDecC * 2;
  return JTFS_OK;
}

void jtfs_dec_destroy(jtfs_dec_t dec) { delete dec; }

}  // extern "C"
