// Host-side JTFS plan: filterbanks, subsampling rules, path list, output layout,
// device table images, work lists and workspace layout for one signal.
// Pure C++17 (no HIP): it runs at jtfs_plan() time on the host.
#pragma once
#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/jtfs.h"
#include "types.hpp"

namespace jtfs {

struct cfloat { float x, y; };   // host image of a device float2

struct Filt {
  double xi, sigma;
  int32_t j, k, spin;
  bool lowpass;
};

struct Grp {
  int32_t n2, j2, K;
  int64_t L2;
  int32_t n_t = 0, t_lo = 0;   // output times of the group's paths and the first one (L2 grid
                               // without time averaging, the frame grid with it)
};

// Stages of the time-axis pipeline (see kernels_time.hip for what each computes).
enum Stage : int32_t {
  ST_XHAT = 0,   // DFT of the zero-padded signal
  ST_L1Z = 1,    // first-order wavelet: fold-gather of Xhat * psi1, inverse DFT -> Z1
  ST_L1UH = 2,   // DFT of |Z1| -> U1hat
  ST_L2Y = 3,    // second-order wavelet: fold-gather of U1hat * psi2^(k1), inverse DFT -> Y2
  ST_BYH = 4,    // DFT of dY2 (sum of row-split partials) -> dY2hat
  ST_BU = 5,     // adjoint gather onto U1hat, inverse DFT, real part -> dU1
  ST_BZH = 6,    // DFT of dU1 * Z1/|Z1| -> dZ1hat
  ST_BX = 7,     // adjoint gather onto Xhat, inverse DFT, real part, unpad -> dx
  ST_COUNT = 8
};

struct Launch {
  int32_t stage, n, job0, njobs;
};

// Byte offsets of workspace regions for one signal (relative to the signal's segment).
// part and dYpart are one region (never live at the same time).
struct WsLayout {
  size_t Xh, Z1, U1h, S1, Y2, part, psum, scr, S, dS, o1, u2;   // forward (+ loss scratch)
  size_t fwd_end;
  size_t dP, dYpart, dYh, dS1p, dU1, dZh, dXh, grad, dv;
  size_t bwd_end;
};

struct SigPlan {
  jtfs_params prm{};
  int64_t N = 0, N_pad = 0, pad_left = 0;
  int32_t log2T = 0, T = 0, sF = 0, N_fr = 0, nf_pad = 0, f_lo = 0, n_frames = 0, Lf = 0;
  int32_t log2_Npad = 0;
  double sigmaT = 0, sigmaF = 0;
  std::vector<Filt> psi1, psi2, fr;
  std::vector<int32_t> fr_real;          // frequential filters applied to real inputs
  std::vector<Grp> groups;
  std::vector<jtfs_path> paths;
  int64_t n_coeff = 0;

  // ---- device table images
  std::vector<cfloat> tw;                // exp(-2 pi i k / N_pad), k < N_pad
  std::vector<float> bandvals;
  std::vector<Band> bands;
  std::vector<int32_t> band_psi1;        // per n1, level 0 on the N_pad grid
  float psi1_energy_max = 0.f;           // max over bins k <= N_pad / 2 of sum_n1 |psi1_n1^(k)|^2
  std::map<std::pair<int, int>, int32_t> band_psi2;   // (n2, level) -> band
  std::vector<int32_t> band_phiT;        // per level (0..log2T), -1 if unused
  std::vector<float> tables;             // time-domain phi_T (per group) and phi_F (per g)
  std::vector<cfloat> W;                 // R_pad x NW frequential Toeplitz rows
  int32_t NW = 0, R_total = 0, R_pad = 0;
  std::vector<int32_t> rt_nrange;        // per 16-row tile: n_lo, n_hi (pairs)
  std::vector<int32_t> tap_count;        // per row: taps above 1e-7 of peak among the first n columns
  std::vector<FrFilter> frf;
  std::vector<FreqGroup> fgroups;
  std::vector<FwdItem> fwd_items;       // grouped by kernel shape, see fwd_launches
  struct FwdLaunch {
    int32_t S, RW, FT, item0, nitems;     // k-steps, row tiles per wave (0: row-tile-loop
                                          // kernel, items = (group, row split, chunk)), frame tiles
    int32_t run;                          // consecutive items sharing a time chunk
    int32_t MT;                           // row-tile-loop kernel: 16-time tiles per wave
  };
  std::vector<FwdLaunch> fwd_launches;
  std::vector<BwdItem> bwd_items;
  // Backward launches, one per k-step bucket S (4..64; the groups with 4(S/2) < K <= 4S),
  // each over bwd_items[item0, item0 + nitems).
  struct BwdLaunch {
    int32_t S, item0, nitems;
  };
  std::vector<BwdLaunch> bwd_launches;
  std::vector<RowJob> jobs;              // all stages; S1 jobs after the launches
  std::vector<GatherTerm> terms;
  // Adjoint gathers: per 512-bin segment of a gather row, the terms whose band meets it
  // (pairs: first index into segterms, count); the row's RowJob.t0 is its first segment.
  // `terms` is only the planning list the segments are cut from.
  std::vector<int32_t> segs;
  std::vector<SegTerm> segterms;
  std::vector<Launch> launches[ST_COUNT];     // two-pass (n > 4096) launches
  std::vector<RowTask> tasks;                  // single-pass workgroup tasks of every stage
  int32_t task0[ST_COUNT] = {0}, ntask[ST_COUNT] = {0};
  // Two-pass rows of a stage: every row of every length in one pass-1 launch and one
  // pass-2 launch, each row with its own scratch (tasks of stage st: [split0, split0 + nsplit)
  // for pass 1, then the same count shifted by nsplit1 for pass 2).
  std::vector<SplitTask> stasks;
  std::vector<int32_t> live_rt;                // per group: its live 16-row tiles, ascending
  // Bin-parallel adjoint gathers (stages BU and BX): chunks of up to 256 output bins of
  // one row, pairs (job, first bin); the chunks of stage st are [gch0[st], gch0[st] + gchn[st]).
  std::vector<int32_t> gchunks;
  int32_t gch0[ST_COUNT] = {0}, gchn[ST_COUNT] = {0};
  int32_t task_jobs0[ST_COUNT] = {0}, task_jobs1[ST_COUNT] = {0};   // each stage's jobs
  int32_t bx_job = -1;   // the job of the final gather onto the padded signal spectrum
  int32_t split1_0[ST_COUNT] = {0}, split1_n[ST_COUNT] = {0};
  int32_t split2_0[ST_COUNT] = {0}, split2_n[ST_COUNT] = {0};
  int32_t s1_job0 = 0;                   // N1 jobs for the S1 stage
  // zeroth order (JTFS_ZEROTH): S0 coefficients at s0_off (n_frames of them, -1: none),
  // phi_T at level 0 on the N_pad grid, and the block's loss weight
  int64_t s0_off = -1;
  int32_t s0_band = -1;
  float w0 = 0.f;
  bool u0 = false;               // the zeroth order is U0 = x (averaging not local)
  // the listings' average_local / average_local_fr switched off: second-order paths keep
  // |Y_fr| at their own time resolution (no phi_T), band-pass paths their own
  // log-frequency stride 2^j_fr (no phi_F)
  bool no_avg_local = false, no_avg_fr = false;
  int64_t u2_total = 0;          // R_pad x sum of the groups' kept times
  // forward frequential work, in complex multiply-adds (contraction) and real ones (pooling)
  double mac_dense = 0, mac_banded = 0, mac_exec = 0, mac_pool = 0;
  int32_t max_fwd_tiles = 0;

  // ---- workspace
  std::vector<int64_t> z1_off;           // complex offset of row n1 in Z1 / U1h / dZh (float offset in dU1)
  int64_t z1_total = 0, y2_total = 0, part_total = 0, psum_total = 0, dP_total = 0, dYpart_total = 0;
  int64_t scr_elems = 0;
  WsLayout ws{};
};

// Builds the plan of one signal; on failure returns a status and sets `err`.
// Fills `out` for one signal; `tune` (may be NULL) selects tile schedules (jtfs_tuning).
jtfs_status build_signal_plan(const jtfs_params& prm, SigPlan& out, std::string& err,
                              const jtfs_tuning* tune = nullptr);
// Resolves the zero fields of a tuning to their defaults; false if a field is out of range.
bool resolve_tuning(const jtfs_tuning* in, jtfs_tuning& out);

// Filterbank generator of Sec. 3.1 and the subsampling-scale rule, exposed for tests.
std::vector<std::pair<double, double>> wavelet_bank(int J, int Q);
int32_t subsampling_scale(double xi, double sigma);

}  // namespace jtfs
