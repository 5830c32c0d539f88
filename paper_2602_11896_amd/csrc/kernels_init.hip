// The coloured-noise descent start (Sec. 2.3): Gaussian noise whose power spectral
// density matches S1 x.
//
//   m_n1 = mean over the kept frames of S1 x[n1, .]           (first layer, Eq. 3 before phi_F)
//   c_n1 = (4 / pi) m_n1^2 / E_n1,  E_n1 = (1 / N_pad) sum_k |psi1_n1^(k)|^2
//          (a circular Gaussian with E|z|^2 = P has E|z| = sqrt(pi P) / 2)
//   H_k^2 = sum_n1 c_n1 |psi1_n1^(k')|^2 / (sum_n1 |psi1_n1^(k')|^2 + 1e-12 emax),
//          k' = min(k, N_pad - k), emax the largest summed response
//   y0 = unpad(IDFT(H . DFT(pad(w))))                          (w: standard normal draws)
//
// The first layer of x and the DFT of the padded draws run through the transform's own
// stages; the inverse DFT is the one of the signal adjoint.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace jtfs {
namespace {

// Sum of one value per thread over a 256-thread block, in a fixed order (tree in LDS).
__device__ inline float block_sum(float v, float* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (static_cast<int>(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const float r = red[0];
  __syncthreads();
  return r;
}

// One block per first-order filter.
__global__ __launch_bounds__(256) void k_cn_levels(DevSig s, const int32_t* band_psi1, float* c) {
  __shared__ float red[256];
  const int n1 = blockIdx.x;
  const float* row = s.S1 + static_cast<int64_t>(n1) * s.nf_pad + s.f_lo;
  float a = 0.f;
  for (int f = threadIdx.x; f < s.nF; f += 256) a += row[f];
  const float m = block_sum(a, red) / static_cast<float>(s.nF);
  const Band b = s.bands[band_psi1[n1]];
  float e = 0.f;
  for (int d = threadIdx.x; d < b.len; d += 256) {
    const float h = s.bandvals[b.off + d];
    e += h * h;
  }
  const float E = block_sum(e, red) / static_cast<float>(s.N_pad);
  if (threadIdx.x == 0) c[n1] = E > 0.f ? (4.f / 3.14159265358979f) * m * m / E : 0.f;
}

// One thread per bin of the padded spectrum.
__global__ __launch_bounds__(256) void k_cn_shape(DevSig s, const int32_t* band_psi1, const float* c, float emax) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= s.N_pad) return;
  const int kk = min(k, s.N_pad - k);
  float num = 0.f, den = 0.f;
  for (int n1 = 0; n1 < s.N1; ++n1) {
    const Band b = s.bands[band_psi1[n1]];
    int d = kk - b.lo;
    if (d < 0) d += b.L;
    if (d < b.len) {
      const float h = s.bandvals[b.off + d];
      num += c[n1] * (h * h);
      den += h * h;
    }
  }
  // (the inverse transform that follows carries the 1 / N_pad)
  const float H = sqrtf(num / (den + 1e-12f * emax));
  const c32 X = s.Xh[k];
  s.dXh[k] = c32{X.x * H, X.y * H};
}

}  // namespace

hipError_t run_cn_levels(const DevSig& s, const SigPlan& p, const int32_t* band_psi1, float* c, hipStream_t st) {
  hipLaunchKernelGGL(k_cn_levels, dim3(p.psi1.size()), dim3(256), 0, st, s, band_psi1, c);
  return hipGetLastError();
}

hipError_t run_cn_shape(const DevSig& s, const SigPlan& p, const int32_t* band_psi1, const float* c,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_cn_shape, dim3((p.N_pad + 255) / 256), dim3(256), 0, st, s, band_psi1, c,
                     p.psi1_energy_max);
  return hipGetLastError();
}

}  // namespace jtfs
