// Host-side launchers of the kernel families (one translation unit per family).
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "plan.hpp"

namespace jtfs {

// kernels_time.hip
hipError_t run_time_stage(int stage, const DevSig& s, const SigPlan& p, hipStream_t st);
hipError_t run_s1(const DevSig& s, const SigPlan& p, hipStream_t st);
hipError_t run_ds1h(const DevSig& s, const SigPlan& p, hipStream_t st);
// dx = unpad(Re((1 / N_pad) sum_k dXh[k] e^{+2 pi i k n / N_pad})): the inverse DFT of
// stage BX applied to a spectrum already in dXh (without BX's first-order gather).
hipError_t run_signal_idft(const DevSig& s, const SigPlan& p, hipStream_t st);

// kernels_init.hip (coloured-noise descent start)
// c[n1] = (4 / pi) m_n1^2 / E_n1: m_n1 the mean of S1 over the kept frames, E_n1 the
// energy per sample of filter n1 on the N_pad grid.
hipError_t run_cn_levels(const DevSig& s, const SigPlan& p, const int32_t* band_psi1, float* c, hipStream_t st);
// dXh[k] = Xh[k] H_k with H_k^2 = sum c |psi1^(k')|^2 / (sum |psi1^(k')|^2 + 1e-12 emax),
// k' = min(k, N_pad - k).
hipError_t run_cn_shape(const DevSig& s, const SigPlan& p, const int32_t* band_psi1, const float* c,
                        hipStream_t st);

// kernels_joint.hip: out[r][t] = Re(psi_alpha(t - n_t / 2) g(r - N_fr / 2)) for the band b of
// psi_alpha on the N_pad grid and the N_fr complex taps of g (Sec. 2.1, Fig. 1).
hipError_t run_joint_wavelet(const DevSig& s, const Band& b, const float* taps, int n_fr_bins, int n_t, float* out,
                             hipStream_t st);

// kernels_unavg.hip: the variants without local averaging (no phi_T on the second order:
// |W_g Y2| at the group's kept times, then phi_F or not; U0 = x as zeroth order).
hipError_t run_unavg_fwd(const DevSig& s, const SigPlan& p, hipStream_t st);
hipError_t run_unavg_bwd(const DevSig& s, const SigPlan& p, hipStream_t st);
hipError_t run_u0(const DevSig& s, const SigPlan& p, hipStream_t st);

// kernels_freq.hip
hipError_t run_order1_fwd(const DevSig& s, const SigPlan& p, hipStream_t st);
hipError_t run_freq_fwd(const DevSig& s, const SigPlan& p, hipStream_t st);
hipError_t run_freq_pool(const DevSig& s, const SigPlan& p, hipStream_t st);
hipError_t run_freq_dP(const DevSig& s, const SigPlan& p, hipStream_t st);
hipError_t run_freq_bwd(const DevSig& s, const SigPlan& p, hipStream_t st);
hipError_t run_order1_bwd(const DevSig& s, const SigPlan& p, hipStream_t st);
hipError_t run_dy_reduce(const DevSig& s, const SigPlan& p, hipStream_t st);

// kernels_opt.hip
// loss[0] = sum w (S - S_target)^2 and dS = 2 w (S - S_target) over n coefficients, with
// w = w0 on the first n0 (the zeroth-order block) and 1 elsewhere.
hipError_t run_loss(const float* S, const float* S_target, float* dS, float* loss, int64_t n, int64_t n0, float w0,
                    hipStream_t st);
// Optimiser update of n samples (see jtfs.h); `scal` = this signal's 4 state scalars.
hipError_t run_update(const jtfs_opt& opt, float* y, const float* grad, const float* loss, float* vec0, float* vec1,
                      float* vec2, float* scal, int64_t n, hipStream_t st);

}  // namespace jtfs
