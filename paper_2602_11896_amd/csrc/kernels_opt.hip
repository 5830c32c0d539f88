// Metamer loss and updates (Sec. 2.3).
//  loss   E = sum w (S - S_target)^2 (deterministic fixed-order reduction), dS = 2 w (S - S_target),
//         w the zeroth-order weight on that block (if any) and 1 elsewhere.
//  GD     y <- y - lr grad.
//  Adam   bias-corrected moments; the step counter lives in the state scalars.
//  MOMENTUM_BOLD  y <- y + u with u <- m u - mu grad; mu grows by bold_up while E does
//         not increase; otherwise y returns to the last kept iterate, the momentum is
//         cleared, mu shrinks by bold_down and a fresh step is taken from the kept
//         iterate along its stored gradient.
// A non-finite E leaves y unchanged (momentum cleared), freezes the other scalars and
// counts the step in scalar [3].
// Scalars per signal: [0] step count (Adam) / initialised flag (momentum), [1] mu,
// [2] last kept E, [3] non-finite steps. They are updated by a one-thread kernel after
// the element update.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace jtfs {
namespace {

__global__ __launch_bounds__(1024) void k_loss(const float* S, const float* St, float* dS, float* loss, int64_t n,
                                               int64_t n0, float w0) {
  __shared__ double part[1024];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const float w = i < n0 ? w0 : 1.0f;
    const float d = S[i] - St[i];
    dS[i] = 2.0f * w * d;
    acc += static_cast<double>(w) * d * d;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = static_cast<float>(part[0]);
}

__global__ void k_update_gd(float* y, const float* g, const float* loss, float lr, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n || !isfinite(loss[0])) return;
  y[i] -= lr * g[i];
}

__global__ void k_update_adam(float* y, const float* g, const float* loss, float* m1, float* m2, const float* scal,
                              float lr, float b1, float b2, float eps, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n || !isfinite(loss[0])) return;
  const float t = scal[0] + 1.0f;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.0f - b1) * gi;
  const float b = b2 * m2[i] + (1.0f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  const float mhat = a / (1.0f - powf(b1, t));
  const float vhat = b / (1.0f - powf(b2, t));
  y[i] -= lr * mhat / (sqrtf(vhat) + eps);
}

__global__ void k_update_momentum(float* y, const float* g, const float* loss, float* u, float* yprev, float* gprev,
                                  const float* scal, float lr, float m, float up, float down, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float E = loss[0];
  if (!isfinite(E)) {
    u[i] = 0.0f;
    return;
  }
  const bool init = scal[0] != 0.0f;
  const bool accept = !init || E <= scal[2];
  const float mu = !init ? lr : (accept ? scal[1] * up : scal[1] * down);
  if (accept) {
    const float gi = g[i];
    yprev[i] = y[i];
    gprev[i] = gi;
    const float ui = m * u[i] - mu * gi;
    u[i] = ui;
    y[i] += ui;
  } else {
    const float ui = -mu * gprev[i];
    u[i] = ui;
    y[i] = yprev[i] + ui;
  }
}

__global__ void k_update_scalars(int kind, const float* loss, float* scal, float lr, float up, float down) {
  const float E = loss[0];
  if (!isfinite(E)) {
    scal[3] += 1.0f;
    return;
  }
  if (kind == JTFS_OPT_ADAM) {
    scal[0] += 1.0f;
  } else if (kind == JTFS_OPT_MOMENTUM_BOLD) {
    if (scal[0] == 0.0f) {
      scal[0] = 1.0f;
      scal[1] = lr;
      scal[2] = E;
    } else if (E <= scal[2]) {
      scal[1] *= up;
      scal[2] = E;
    } else {
      scal[1] *= down;
    }
  }
}

}  // namespace

hipError_t run_loss(const float* S, const float* S_target, float* dS, float* loss, int64_t n, int64_t n0, float w0,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(1024), 0, st, S, S_target, dS, loss, n, n0, w0);
  return hipGetLastError();
}

hipError_t run_update(const jtfs_opt& o, float* y, const float* grad, const float* loss, float* vec0, float* vec1,
                      float* vec2, float* scal, int64_t n, hipStream_t st) {
  const int blocks = static_cast<int>((n + 255) / 256);
  switch (o.kind) {
    case JTFS_OPT_GD:
      hipLaunchKernelGGL(k_update_gd, dim3(blocks), dim3(256), 0, st, y, grad, loss, o.lr, n);
      break;
    case JTFS_OPT_ADAM:
      hipLaunchKernelGGL(k_update_adam, dim3(blocks), dim3(256), 0, st, y, grad, loss, vec0, vec1, scal, o.lr, o.beta1,
                         o.beta2, o.eps, n);
      break;
    case JTFS_OPT_MOMENTUM_BOLD:
      hipLaunchKernelGGL(k_update_momentum, dim3(blocks), dim3(256), 0, st, y, grad, loss, vec0, vec1, vec2, scal,
                         o.lr, o.momentum, o.bold_up, o.bold_down, n);
      break;
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_update_scalars, dim3(1), dim3(1), 0, st, o.kind, loss, scal, o.lr, o.bold_up, o.bold_down);
  return hipGetLastError();
}

}  // namespace jtfs
