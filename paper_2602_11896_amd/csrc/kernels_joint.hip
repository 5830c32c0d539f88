// The joint time--log-frequency wavelet of a scattering path (Sec. 2.1, Fig. 1): the
// real part of psi_alpha(t) psi_beta(log2 lambda), with psi_alpha a second-order (time)
// wavelet at the signal's rate and psi_beta a frequential filter along the N_fr
// log-frequency bins, on a grid centred on both filters' origins.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace jtfs {
namespace {

// One thread per time sample t < n_t (centred time tc = t - n_t / 2):
//   a(tc) = (1 / L) sum over the band of psi_hat[m] e^{+2 pi i m tc / L}   (L = N_pad),
// summed in FP64 from the band values and the e^{-2 pi i q / L} table; then for every
// log-frequency bin r (centred rc = r - N_fr / 2) out[r][t] = Re(a(tc) g[rc mod N_fr]).
__global__ __launch_bounds__(256) void k_joint_wavelet(DevSig s, Band b, const float* taps, int n_fr_bins, int n_t,
                                                       float* out) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n_t) return;
  const uint32_t tc = static_cast<uint32_t>(t - n_t / 2);   // modular arithmetic mod 2^32
  const uint32_t mask = static_cast<uint32_t>(s.N_pad) - 1u;
  double ar = 0.0, ai = 0.0;
  for (int d = 0; d < b.len; ++d) {
    uint32_t m = static_cast<uint32_t>(b.lo + d);
    if (m >= static_cast<uint32_t>(b.L)) m -= static_cast<uint32_t>(b.L);
    const c32 w = s.tw[(m * tc) & mask];     // e^{-2 pi i m tc / L}; conjugated below
    const double h = s.bandvals[b.off + d];
    ar += h * w.x;
    ai -= h * w.y;
  }
  const double inv = 1.0 / s.N_pad;
  const float a_r = static_cast<float>(ar * inv), a_i = static_cast<float>(ai * inv);
  for (int r = 0; r < n_fr_bins; ++r) {
    int rc = r - n_fr_bins / 2;
    if (rc < 0) rc += n_fr_bins;
    const float g_r = taps[2 * rc], g_i = taps[2 * rc + 1];
    out[static_cast<int64_t>(r) * n_t + t] = a_r * g_r - a_i * g_i;
  }
}

}  // namespace

hipError_t run_joint_wavelet(const DevSig& s, const Band& b, const float* taps, int n_fr_bins, int n_t, float* out,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_joint_wavelet, dim3((n_t + 255) / 256), dim3(256), 0, st, s, b, taps, n_fr_bins, n_t, out);
  return hipGetLastError();
}

}  // namespace jtfs
