// Device view of one signal's plan tables and workspace, passed by value to kernels.
#pragma once
#include <cstdint>

#include "fft_core.hpp"
#include "types.hpp"

namespace jtfs {

struct DevSig {
  // ---- plan tables (device arena owned by the plan)
  const c32* tw;            // exp(-2 pi i q / N_pad), q < N_pad
  const float* bandvals;
  const Band* bands;
  const float* tables;      // time-domain phi_T / phi_F
  const c32* W;             // R_pad x NW frequential rows
  const int32_t* rt_nrange; // per 16-row tile: n_lo, n_hi
  const int32_t* live_rt;   // per group (FreqGroup::lt0, nlt): the row tiles whose band meets [0, K)
  const FrFilter* frf;
  const FreqGroup* fgroups;
  const FwdItem* fwd_items;
  const BwdItem* bwd_items;
  const RowJob* jobs;
  const RowTask* tasks;
  const int32_t* segs;      // per gather segment: first index into segterms, count
  const SegTerm* segterms;
  const SplitTask* stasks;  // two-pass transform workgroups
  const int32_t* gchunks;   // bin-parallel gather chunks: (job, first bin) pairs
  const int64_t* s_off;     // output offset of block (group gi, filter g) at gi*n_g + g;
                            // order-1 blocks at n_groups*n_g + (index in the real list)
  // ---- per-call arrays
  const float* x;           // this signal's samples (n)
  float* S;                 // this signal's coefficients
  const float* dS;          // this signal's coefficient gradient
  float* dx;                // this signal's sample gradient
  // ---- workspace regions
  c32* Xh;
  c32* Z1;
  c32* U1h;
  float* S1;
  c32* Y2;
  float* part;
  float* psum;              // per non-windowed group: partials summed over time chunks (R_pad x nF)
  c32* scr;
  float* dP;
  c32* dYpart;
  c32* dYh;
  float* dS1p;
  float* dU1;
  c32* dZh;
  c32* dXh;   // gathered spectrum of the signal gradient (before the inverse DFT)
  c32* o1;                  // order-1 modulus / gradient rows (R_pad x nF)
  // ---- sizes
  int32_t N, N_pad, pad_left, log2_Npad;
  int32_t N1, nf_pad, f_lo, nF, Lf, log2T, N_fr, sF;
  int32_t n_g, n_groups, n_real, R_pad, NW;
  int64_t y2_total, z1_total;
  int64_t s0_off;           // zeroth-order coefficients (n_frames, or N for U0), -1: none
  int32_t s0_band;          // phi_T at level 0 on the N_pad grid
  float w0;                 // loss weight of the zeroth-order block
  int32_t u0;               // the zeroth order is U0 = x
  int32_t no_avg_local;     // second order without phi_T: |V| at the group's own resolution
  int32_t no_avg_fr;        // band-pass paths without phi_F, at their own stride 2^k_fr
  float* u2;                // |V| of the unaveraged second order (R_pad x n_t per group)
  c32* dv;                  // its gradient dV (same layout, complex)
};

}  // namespace jtfs
