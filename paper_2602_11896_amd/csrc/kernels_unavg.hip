// Variants of the method without local averaging (the average_local / average_local_fr
// switches of the Sec. 3.3 and 3.5 listings and the Sec. 3.6 main algorithm): the second
// order without phi_T keeps U2 = |W_g Y2| (Eq. 2) at the group's own time resolution
// 2^j2, unpadded to the signal's samples, and (with phi_F averaging) averages it along
// log-frequency only; the zeroth order is U0 = x. These outputs are as large as U2
// itself, so the variant suits short signals; its sums are direct FP32 loops (the
// averaged path runs the fused MFMA contraction instead).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.hpp"

namespace jtfs {
namespace {

// V[r, t] = sum_{n < K} W[r, n] Y2[n, t_lo + t] of group fg (four partial sums).
__device__ inline c32 unavg_v(const DevSig& s, const FreqGroup& fg, int r, int t) {
  const c32* w = s.W + static_cast<int64_t>(r) * s.NW;
  const c32* y = s.Y2 + fg.y2 + fg.t_lo + t;
  float vr[2] = {0.f, 0.f}, vi[2] = {0.f, 0.f};
  for (int n = 0; n < fg.K; ++n) {
    const c32 a = w[n], b = y[static_cast<int64_t>(n) * fg.L2];
    vr[n & 1] += a.x * b.x - a.y * b.y;
    vi[n & 1] += a.x * b.y + a.y * b.x;
  }
  return c32{vr[0] + vr[1], vi[0] + vi[1]};
}

// Frequential filter of row r of the stacked row space, or -1 for a padding row.
__device__ inline int filter_of_row(const DevSig& s, int r) {
  for (int q = 0; q < s.n_g; ++q) {
    const FrFilter c = s.frf[q];
    if (r >= c.row0 && r < c.row0 + c.M) return q;
  }
  return -1;
}

// Kept log-frequency bins of filter g's paths in a group of K rows: phi_F-averaged
// (stride 2^sF; phi_F itself at its own stride 2^sF), or at the band-pass's stride 2^k.
__device__ inline int kept_bins(const DevSig& s, const FrFilter& ff, int K) {
  const int k = (!ff.lowpass && s.no_avg_fr) ? ff.k : s.sF;
  return (K + (1 << k) - 1) >> k;
}

// u2[r, t] = |V[r, t]| over the R_pad rows and the group's kept times.
__global__ __launch_bounds__(256) void k_u2_v(DevSig s, int gi) {
  const FreqGroup fg = s.fgroups[gi];
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (e >= static_cast<int64_t>(s.R_pad) * fg.n_t) return;
  const int r = static_cast<int>(e / fg.n_t), t = static_cast<int>(e - static_cast<int64_t>(r) * fg.n_t);
  const c32 v = unavg_v(s, fg, r, t);
  s.u2[fg.u2 + e] = sqrtf(v.x * v.x + v.y * v.y);
}

// Output block (group gi, filter blockIdx.y): rows b < kept bins, times t < n_t.
__global__ __launch_bounds__(256) void k_u2_out(DevSig s, int gi) {
  const FreqGroup fg = s.fgroups[gi];
  const int g = blockIdx.y;
  const FrFilter ff = s.frf[g];
  const int nl = kept_bins(s, ff, fg.K);
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nl * fg.n_t) return;
  const int b = e / fg.n_t, t = e - b * fg.n_t;
  const float* u = s.u2 + fg.u2;
  float v;
  if (!ff.lowpass && !s.no_avg_fr) {
    const int sh = s.sF - ff.k;
    const float* ph = s.tables + ff.phiF;
    v = 0.f;
    for (int r = 0; r < ff.M; ++r) v += ph[((b << sh) - r) & (ff.M - 1)] * u[static_cast<int64_t>(ff.row0 + r) * fg.n_t + t];
  } else {
    v = u[static_cast<int64_t>(ff.row0 + b) * fg.n_t + t];
  }
  s.S[s.s_off[gi * s.n_g + g] + e] = v;
}

// dV[r, t] = dU[r, t] V / |V| (0 where V vanishes), dU the adjoint of k_u2_out.
__global__ __launch_bounds__(256) void k_u2_dv(DevSig s, int gi) {
  const FreqGroup fg = s.fgroups[gi];
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (e >= static_cast<int64_t>(s.R_pad) * fg.n_t) return;
  const int r = static_cast<int>(e / fg.n_t), t = static_cast<int>(e - static_cast<int64_t>(r) * fg.n_t);
  const int g = filter_of_row(s, r);
  c32 d{0.f, 0.f};
  if (g >= 0) {
    const FrFilter ff = s.frf[g];
    const int rr = r - ff.row0;
    const float* dout = s.dS + s.s_off[gi * s.n_g + g];
    float du = 0.f;
    if (!ff.lowpass && !s.no_avg_fr) {
      const int sh = s.sF - ff.k;
      const float* ph = s.tables + ff.phiF;
      const int nb = kept_bins(s, ff, fg.K);
      for (int b = 0; b < nb; ++b) du += ph[((b << sh) - rr) & (ff.M - 1)] * dout[b * fg.n_t + t];
    } else if (rr < kept_bins(s, ff, fg.K)) {
      du = dout[rr * fg.n_t + t];
    }
    const c32 v = unavg_v(s, fg, r, t);
    const float m2 = v.x * v.x + v.y * v.y;
    if (m2 > 0.f) {
      const float sc = du / sqrtf(m2);
      d = c32{v.x * sc, v.y * sc};
    }
  }
  s.dv[fg.u2 + e] = d;
}

// dY2[n, t] = sum_r conj(W[r, n]) dV[r, t - t_lo] at kept times, 0 elsewhere, into the
// group's first dY2 partial (the layer-2 adjoint DFT reads it).
__global__ __launch_bounds__(256) void k_u2_dy(DevSig s, int gi) {
  const FreqGroup fg = s.fgroups[gi];
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (e >= static_cast<int64_t>(fg.K) * fg.L2) return;
  const int n = static_cast<int>(e / fg.L2), t = static_cast<int>(e - static_cast<int64_t>(n) * fg.L2);
  const int tt = t - fg.t_lo;
  c32 acc{0.f, 0.f};
  if (tt >= 0 && tt < fg.n_t) {
    const c32* dvp = s.dv + fg.u2 + tt;
    for (int r = 0; r < s.R_pad; ++r) {
      const c32 w = s.W[static_cast<int64_t>(r) * s.NW + n];
      const c32 d = dvp[static_cast<int64_t>(r) * fg.n_t];
      acc.x += w.x * d.x + w.y * d.y;
      acc.y += w.x * d.y - w.y * d.x;
    }
  }
  s.dYpart[fg.dYpart + e] = acc;
}

// U0 = x into the zeroth-order block.
__global__ __launch_bounds__(256) void k_u0(DevSig s) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < s.N) s.S[s.s0_off + i] = s.x[i];
}

}  // namespace

hipError_t run_unavg_fwd(const DevSig& s, const SigPlan& p, hipStream_t st) {
  for (size_t gi = 0; gi < p.fgroups.size(); ++gi) {
    const FreqGroup& fg = p.fgroups[gi];
    const int64_t cells = static_cast<int64_t>(p.R_pad) * fg.n_t;
    hipLaunchKernelGGL(k_u2_v, dim3(static_cast<unsigned>((cells + 255) / 256)), dim3(256), 0, st, s,
                       static_cast<int>(gi));
    int most = 0;
    for (const FrFilter& ff : p.frf) {
      const int k = (!ff.lowpass && p.no_avg_fr) ? ff.k : p.sF;
      most = std::max(most, ((fg.K + (1 << k) - 1) >> k) * fg.n_t);
    }
    hipLaunchKernelGGL(k_u2_out, dim3((most + 255) / 256, p.frf.size()), dim3(256), 0, st, s, static_cast<int>(gi));
  }
  return hipGetLastError();
}

hipError_t run_unavg_bwd(const DevSig& s, const SigPlan& p, hipStream_t st) {
  for (size_t gi = 0; gi < p.fgroups.size(); ++gi) {
    const FreqGroup& fg = p.fgroups[gi];
    const int64_t cells = static_cast<int64_t>(p.R_pad) * fg.n_t;
    hipLaunchKernelGGL(k_u2_dv, dim3(static_cast<unsigned>((cells + 255) / 256)), dim3(256), 0, st, s,
                       static_cast<int>(gi));
    const int64_t ys = static_cast<int64_t>(fg.K) * fg.L2;
    hipLaunchKernelGGL(k_u2_dy, dim3(static_cast<unsigned>((ys + 255) / 256)), dim3(256), 0, st, s,
                       static_cast<int>(gi));
  }
  return hipGetLastError();
}

hipError_t run_u0(const DevSig& s, const SigPlan& p, hipStream_t st) {
  hipLaunchKernelGGL(k_u0, dim3(static_cast<unsigned>((p.N + 255) / 256)), dim3(256), 0, st, s);
  return hipGetLastError();
}

}  // namespace jtfs
