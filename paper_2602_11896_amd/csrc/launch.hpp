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

// kernels_freq.hip
hipError_t run_order1_fwd(const DevSig& s, const SigPlan& p, hipStream_t st);
hipError_t run_freq_fwd(const DevSig& s, const SigPlan& p, hipStream_t st);
hipError_t run_freq_pool(const DevSig& s, const SigPlan& p, hipStream_t st);
hipError_t run_freq_dP(const DevSig& s, const SigPlan& p, hipStream_t st);
hipError_t run_freq_bwd(const DevSig& s, const SigPlan& p, hipStream_t st);
hipError_t run_order1_bwd(const DevSig& s, const SigPlan& p, hipStream_t st);
hipError_t run_dy_reduce(const DevSig& s, const SigPlan& p, hipStream_t st);

// kernels_opt.hip
// loss[0] = ||S - S_target||^2 and dS = 2 (S - S_target) over n coefficients.
hipError_t run_loss(const float* S, const float* S_target, float* dS, float* loss, int64_t n, hipStream_t st);
// Optimiser update of n samples (see jtfs.h); `scal` = this signal's 4 state scalars.
hipError_t run_update(const jtfs_opt& opt, float* y, const float* grad, const float* loss, float* vec0, float* vec1,
                      float* vec2, float* scal, int64_t n, hipStream_t st);

}  // namespace jtfs
