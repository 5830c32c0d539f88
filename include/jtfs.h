/*
 * jtfs.h - C ABI of the MI355X joint time-frequency scattering (JTFS) library.
 *
 * The library computes the JTFS transform S of Lostanlen & Han, "Musical Metamerism
 * with Time-Frequency Scattering" (Sec. 2.1-2.2, Eqs. 2-4; implementation Sec. 3),
 * its exact gradient (Sec. 2.3, Eqs. 5-7) and one step of the metamer descent that
 * drives E(y) = ||S(y) - S(x)||^2 towards zero (Sec. 2.3).
 *
 * Conventions shared by every entry point
 *  - Every function returns jtfs_status; nothing throws or aborts across the ABI.
 *    Argument errors are reported before any device work is enqueued. On an error,
 *    jtfs_last_error() returns a thread-local description of the last failure.
 *  - Pointers named x, y, S, dS, dx, S_target, loss, ws and the optimiser state are
 *    DEVICE pointers (HIP global memory on the current device), owned by the caller.
 *    Everything else is host memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream). Work is
 *    enqueued asynchronously on it; outputs are valid once the stream has completed.
 *  - All floating point data are IEEE binary32 (FP32), packed without strides.
 *  - A plan is immutable after creation and may be shared by threads and streams as
 *    long as every concurrent call has its own workspace.
 */
#ifndef JTFS_H
#define JTFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct jtfs_plan_s* jtfs_plan_t;   /* opaque, owned by the library */
typedef void* jtfs_stream_t;               /* a hipStream_t */

typedef enum {
  JTFS_OK = 0,
  JTFS_ERR_ARG = 1,          /* invalid argument (null pointer, bad size, bad parameter) */
  JTFS_ERR_NOMEM = 2,        /* host or device allocation of plan tables failed */
  JTFS_ERR_HIP = 3,          /* a HIP runtime call or kernel launch failed */
  JTFS_ERR_WORKSPACE = 4,    /* ws_bytes smaller than the plan requires */
  JTFS_ERR_UNSUPPORTED = 5,  /* parameters outside what the kernels implement */
  JTFS_ERR_NONFINITE = 6     /* a metamer step met a non-finite loss (jtfs_opt_status) */
} jtfs_status;

/*
 * Parameters of one signal (Sec. 3.1 and Sec. 2.2). Sample rate is 1.
 *  n       number of samples N of x (Sec. 2.1).
 *  J, Q1   first-order wavelet bank: scale 2^J and Q1 wavelets per octave (Sec. 3.1).
 *  Q2      second-order temporal bank, same J (Sec. 3.1, last paragraph).
 *  J_fr, Q_fr  frequential bank along log-frequency (Sec. 3.1, last paragraph).
 *  log2_T  time averaging scale T = 2^log2_T samples (Sec. 2.2, Eqs. 3-4).
 *  F       frequential averaging scale in first-order filter bins (Sec. 2.2); the
 *          frequential subsampling is 2^floor(log2 F).
 *  periodic 0: zero-pad to 2^(ceil(log2 n)+1) samples, n split evenly on both sides
 *          (Sec. 3.2 pads both sides); 1: no padding, n must be a power of two.
 *  flags   any of (other bits: JTFS_ERR_ARG)
 *          JTFS_ZEROTH: the output starts with the zeroth-order block of the Sec. 3.6 main
 *            algorithm (one row, path order 0): S0 = (x * phi_T) at stride T over the kept
 *            frames, or U0 = x (its N samples) with JTFS_NO_AVERAGE_LOCAL;
 *          JTFS_NO_AVERAGE_LOCAL (the listings' average_local off): second-order paths
 *            without phi_T, |Y_fr| at their own time resolution 2^j2 over the kept samples
 *            t (pad_left <= t 2^j2 < pad_left + n; jtfs_path.n_frames per group); first
 *            order stays averaged. These outputs are as large as U2 itself: the plan
 *            refuses more than 2^30 of them (JTFS_ERR_UNSUPPORTED);
 *          JTFS_NO_AVERAGE_LOCAL_FR (average_local_fr off): k_fr = j_fr and no phi_F on
 *            band-pass paths, whose bins b keep b 2^k_fr < (rows of the path).
 *  zeroth_weight  weight of the zeroth-order block in the metamer loss (jtfs_metamer_step,
 *          jtfs_loss), finite and >= 0; Eqs. 5-7 hold only the first and second orders, so
 *          0 (the block is output but does not steer the descent) is the paper's loss.
 */
#define JTFS_ZEROTH 1u
#define JTFS_NO_AVERAGE_LOCAL 2u
#define JTFS_NO_AVERAGE_LOCAL_FR 4u
typedef struct {
  int64_t n;
  int32_t J, Q1, Q2, J_fr, Q_fr, log2_T;
  double F;
  int32_t periodic;
  uint32_t flags;
  float zeroth_weight;
} jtfs_params;

/*
 * One block of the output (the paths of Sec. 2.1 after averaging, Eqs. 3-4).
 * order 0 (JTFS_ZEROTH): n2 = n_fr = j2 = j_fr = -1, one row S0; order 1: n2 = j2 = -1,
 * the alpha = 0 paths; order 2: second-order filter n2 with scale j2.
 * n_fr indexes the frequential list [phi_F, psi_fr(xi > 0)..., psi_fr(xi < 0)...];
 * spin is 0 for phi_F, +1 / -1 for the two spins (Sec. 3.4). The block holds
 * n_lambda x n_frames FP32 values, row-major (log-frequency bin, then frame), starting
 * `offset` floats after the signal's first coefficient.
 */
typedef struct {
  int32_t order, n2, n_fr, spin, j2, j_fr, n_lambda, n_frames;
  int64_t offset;
} jtfs_path;

/* Sizes of a plan. Per-signal offsets come from jtfs_plan_offsets. */
typedef struct {
  int32_t batch;            /* number of signals */
  int64_t n_samples_total;  /* sum of n over signals: length of x / y / dx */
  int64_t n_coeff_total;    /* sum of coefficient counts: length of S / dS / S_target */
  size_t  ws_forward;       /* workspace bytes for jtfs_forward */
  size_t  ws_backward;      /* workspace bytes for jtfs_backward and jtfs_metamer_step */
  size_t  ws_shared_forward;   /* workspace bytes for jtfs_forward_ex with JTFS_SHARED_WORKSPACE */
  size_t  ws_shared_backward;  /* workspace bytes for jtfs_backward with JTFS_SHARED_WORKSPACE */
} jtfs_plan_info;

/* Optimiser of the metamer descent (Sec. 2.3). */
typedef enum {
  JTFS_OPT_GD = 0,             /* y <- y - lr * grad */
  JTFS_OPT_MOMENTUM_BOLD = 1,  /* y <- y + u, u <- momentum*u - mu*grad, bold-driver mu (Sec. 2.3) */
  JTFS_OPT_ADAM = 2            /* Adam with bias correction */
} jtfs_opt_kind;

typedef struct {
  int32_t kind;        /* jtfs_opt_kind */
  float lr;            /* GD/Adam learning rate; initial mu for MOMENTUM_BOLD */
  float momentum;      /* MOMENTUM_BOLD momentum m (paper: 0.9) */
  float beta1, beta2, eps;  /* ADAM */
  float bold_up, bold_down; /* MOMENTUM_BOLD learning-rate factors on accept / reject */
  float* state;        /* device buffer of jtfs_opt_state_floats() floats, zeroed by the
                          caller before the first step and left untouched in between */
} jtfs_opt;

/*
 * jtfs_plan - build a plan for `batch` signals (host work only; device tables are
 * uploaded on the first call that runs on a device). Filterbanks follow Sec. 3.1,
 * subsampling rules Sec. 3.2-3.5, path order the main algorithm of Sec. 3.6.
 * Returns JTFS_ERR_ARG for invalid parameters, JTFS_ERR_UNSUPPORTED for valid ones
 * the kernels do not cover (e.g. a second-order resolution coarser than T).
 * On success *out owns the plan; release it with jtfs_plan_destroy.
 */
jtfs_status jtfs_plan(const jtfs_params* sig, int32_t batch, jtfs_plan_t* out);

/* Fill *info. */
jtfs_status jtfs_plan_query(jtfs_plan_t plan, jtfs_plan_info* info);

/* Per-signal offsets (in elements) into x and S: arrays of batch + 1 entries, the last
 * entry being the total. Either pointer may be NULL. */
jtfs_status jtfs_plan_offsets(jtfs_plan_t plan, int64_t* x_offsets, int64_t* s_offsets);

/* Output layout of signal `signal`: at most `cap` rows written to `rows` (host), the
 * number of blocks stored in *n_rows. rows may be NULL to query the count. */
jtfs_status jtfs_plan_meta(jtfs_plan_t plan, int32_t signal, jtfs_path* rows, int64_t cap,
                           int64_t* n_rows);

/* Filterbank of signal `signal` (host arrays of at least `cap` entries, may be NULL):
 * bank 0 = first-order wavelets, 1 = second-order wavelets, 2 = frequential list
 * (phi_F first). xi, sigma in cycles per sample (or per log-frequency bin);
 * j = subsampling scale; k = subsampling applied (k1 for bank 0, k_fr for bank 2,
 * 0 for bank 1). The count is stored in *n. */
jtfs_status jtfs_plan_filters(jtfs_plan_t plan, int32_t signal, int32_t bank, double* xi,
                              double* sigma, int32_t* j, int32_t* k, int32_t cap, int32_t* n);

/* Scalar sizes of signal `signal`: N_pad, pad_left, N_fr, s_F, nf_pad, f_lo, n_frames,
 * n_coeff, in this order, into out[0..7]. */
jtfs_status jtfs_plan_sizes(jtfs_plan_t plan, int32_t signal, int64_t* out8);

/* Intermediate arrays left in the workspace by jtfs_forward, for inspection:
 * which = 0: Z1 (complex, first-order scalogram before the modulus, row n1 of length
 * N_pad / 2^k1, rows concatenated); 1: U1hat (complex, DFT of |Z1| per row, same
 * shape); 2: S1 (real, N1 x nf_pad); 3: Y2 (complex, second-order stacks for every n2
 * with pairs, K(n2) rows of N_pad / 2^j2 each, groups concatenated in n2 order).
 * *offset_bytes and *count (elements) locate it inside ws. */
jtfs_status jtfs_plan_ws_region(jtfs_plan_t plan, int32_t signal, int32_t which,
                                int64_t* offset_bytes, int64_t* count);

/* Work of the forward frequential stage of signal `signal` (Sec. 3.5, Eq. 4), for
 * rooflines: out[0] complex multiply-adds of the dense contraction W Y2 over all
 * second-order groups; out[1] the same counting only taps above 1e-7 of their filter's
 * peak (the banded contraction); out[2] complex multiply-adds the kernel executes
 * (16-row tiles, 4-column steps); out[3] real multiply-adds of the time pooling of
 * the modulus over kept frames. */
jtfs_status jtfs_plan_cost(jtfs_plan_t plan, int32_t signal, double* out4);

/* Number of floats the optimiser state of `kind` needs for this plan. */
int64_t jtfs_opt_state_floats(jtfs_plan_t plan, int32_t kind);

/*
 * jtfs_forward - S = S(x) for every signal of the plan (Eqs. 3-4 with the frequential
 * scattering of Sec. 3.5). x: n_samples_total floats; S: n_coeff_total floats.
 * ws: at least ws_forward bytes (ws_backward bytes if a jtfs_backward with
 * JTFS_REUSE_FORWARD follows). Returns JTFS_ERR_WORKSPACE if ws_bytes is too small.
 */
jtfs_status jtfs_forward(jtfs_plan_t plan, const float* x, float* S, void* ws, size_t ws_bytes,
                         jtfs_stream_t stream);

/* Flags of jtfs_forward_ex and jtfs_backward. */
#define JTFS_REUSE_FORWARD 1u   /* jtfs_backward only: ws still holds the intermediates of
                                   jtfs_forward(x) (or jtfs_forward_ex with the same flags) */
#define JTFS_SHARED_WORKSPACE 2u  /* the signals of a batch take turns in one workspace of
                                     ws_shared_* bytes (the largest signal's need) instead of
                                     each holding its own: they run one after another on
                                     `stream`. For callers that recompute the forward in the
                                     backward (the gradient of Sec. 2.3 needs only x): with a
                                     batch of more than one signal, a shared-workspace forward
                                     leaves only the last signal's intermediates, so
                                     JTFS_REUSE_FORWARD together with this flag is rejected
                                     (JTFS_ERR_ARG) unless the batch has one signal. */

/*
 * jtfs_forward_ex - jtfs_forward with flags (0 or JTFS_SHARED_WORKSPACE; anything else is
 * JTFS_ERR_ARG). With JTFS_SHARED_WORKSPACE, ws needs ws_shared_forward bytes.
 */
jtfs_status jtfs_forward_ex(jtfs_plan_t plan, const float* x, float* S, void* ws, size_t ws_bytes,
                            uint32_t flags, jtfs_stream_t stream);

/*
 * No-allocation forward, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 *
 * JTFS_NOALLOC_SCRATCH_BYTES is the size of a device array the library holds on every
 * device it runs on, until the process ends; it stands in for the forward's workspace.
 *
 * jtfs_plan_prepare - set-up on the current device (allocates; call it outside the
 * no-allocation region): uploads the plan's tables if they are not there yet and
 * resolves the device address of the scratch array. Call it once per plan and device.
 *
 * jtfs_forward_noalloc - S = S(x) exactly as jtfs_forward (the signals of a batch run one
 * after another on `stream`), with the scratch array as workspace; enqueues kernels and
 * allocates nothing. Returns JTFS_ERR_WORKSPACE if the plan's ws_shared_forward exceeds
 * JTFS_NOALLOC_SCRATCH_BYTES (e.g. N = 2^13 with J = 6, Q1 = 8 needs 14.5 MB; N = 2^16 with
 * J = 12, Q1 = 12 needs 273 MB and is refused), JTFS_ERR_ARG if jtfs_plan_prepare has not
 * run for this plan on this device. All calls on one device share its array and it keeps
 * the last call's contents: calls that overlap in time on one device race (serialise them,
 * e.g. on one stream). Stage timing (jtfs_timing_*) does not apply to this call.
 */
#define JTFS_NOALLOC_SCRATCH_BYTES (64u << 20)
jtfs_status jtfs_plan_prepare(jtfs_plan_t plan);
jtfs_status jtfs_forward_noalloc(jtfs_plan_t plan, const float* x, float* S, jtfs_stream_t stream);

/*
 * jtfs_backward - dx = J_S(x)^T dS, the exact adjoint of jtfs_forward at x
 * (Sec. 2.3, Eqs. 5-7, composed in reverse order; the modulus has subgradient 0 at 0).
 * With dS = 2 (S(y) - S(x)) this is grad E. dS: n_coeff_total floats; dx:
 * n_samples_total floats (overwritten). ws: at least ws_backward bytes (ws_shared_backward
 * with JTFS_SHARED_WORKSPACE). Without JTFS_REUSE_FORWARD the forward intermediates are
 * recomputed from x first. Unknown flags are JTFS_ERR_ARG.
 */
jtfs_status jtfs_backward(jtfs_plan_t plan, const float* x, const float* dS, float* dx, void* ws,
                          size_t ws_bytes, uint32_t flags, jtfs_stream_t stream);

/*
 * jtfs_metamer_step - one descent step of Sec. 2.3 for every signal: computes
 * S(y), loss[s] = ||S(y) - S_target||^2 (per signal, before the update, device
 * floats), grad E through jtfs_backward, and updates y in place with `opt`.
 * If a signal's loss is not finite, its y is left unchanged, its momentum is cleared,
 * the optimiser scalars are not advanced and the signal's non-finite step count (a
 * device scalar in opt->state) is incremented; this is decided on the device, so the
 * call never waits for the stream: jtfs_opt_status reports it when the host syncs.
 * Requires ws_backward bytes of workspace.
 */
jtfs_status jtfs_metamer_step(jtfs_plan_t plan, float* y, const float* S_target, const jtfs_opt* opt,
                              float* loss, void* ws, size_t ws_bytes, jtfs_stream_t stream);

/*
 * jtfs_opt_status - waits for `stream`, then reads the per-signal count of metamer steps
 * whose loss was not finite since opt->state was zeroed (counts: host array of batch
 * entries, or NULL). Returns JTFS_ERR_NONFINITE if any count is nonzero, JTFS_OK
 * otherwise (Sec. 2.3 descent; the flag of a non-finite loss, read at synchronisation).
 */
jtfs_status jtfs_opt_status(jtfs_plan_t plan, const jtfs_opt* opt, int32_t* counts, jtfs_stream_t stream);

/*
 * jtfs_colored_noise - the descent start of Sec. 2.3: Gaussian noise whose power spectral
 * density matches the first-order coefficients S1 x. The paper names the start, not its
 * construction; this reading is computed per signal:
 *   m_l   = mean of S1 x(t, l) over the kept frames (U1 x averaged by phi_T, Eq. 3)
 *   c_l   = (4 / pi) m_l^2 / E_l, E_l = (1 / N_pad) sum_k |psi1_l^(k)|^2 (a circular Gaussian
 *           with E|z|^2 = P has E|z| = sqrt(pi P) / 2)
 *   H_k^2 = sum_l c_l |psi1_l^(k')|^2 / (sum_l |psi1_l^(k')|^2 + 1e-12 max_k sum_l |psi1_l^(k)|^2),
 *           k' = min(k, N_pad - k), on the padded DFT grid
 *   y0    = unpad(IDFT(H . DFT(pad(w))))
 * x: the targets (n_samples_total device floats); w: as many independent standard normal
 * draws (the caller's generator; the library draws no random numbers); y0: output, may
 * not alias x or w. ws: at least ws_backward bytes (its contents are overwritten).
 * Enqueued on `stream`; deterministic for given x and w.
 */
jtfs_status jtfs_colored_noise(jtfs_plan_t plan, const float* x, const float* w, float* y0, void* ws,
                               size_t ws_bytes, jtfs_stream_t stream);

/*
 * jtfs_joint_wavelet - the interference pattern of a joint path (Sec. 2.1, Eq. 2 and
 * Fig. 1): out[r * n_t + t] = Re(psi_alpha(t - n_t / 2) * psi_beta(r - N_fr / 2)), r < N_fr,
 * t < n_t, where psi_alpha is the second-order wavelet n2 (Sec. 3.1 bank of Q2) at the
 * signal's rate on its N_pad-point grid (time in samples) and psi_beta the frequential
 * filter n_fr of the list [phi_F, psi_fr(xi > 0)..., psi_fr(xi < 0)...] on the N_fr
 * log-frequency bins (Sec. 3.4-3.5; index = jtfs_path.n_fr), both built from the plan's
 * tables and circularly centred. out: N_fr * n_t device floats (N_fr from
 * jtfs_plan_sizes). JTFS_ERR_ARG if n2 has no second-order paths (j2 = 0), if n_fr is out
 * of range, or if n_t is outside [1, min(N_pad, 2^20)].
 */
jtfs_status jtfs_joint_wavelet(jtfs_plan_t plan, int32_t signal, int32_t n2, int32_t n_fr, int32_t n_t, float* out,
                               jtfs_stream_t stream);

/*
 * jtfs_loss - per-signal metamer loss and its gradient with respect to S (Sec. 2.3):
 * loss[s] = scale sum_i w_i (S_s - T_s)_i^2 / N_s and dS_s = 2 scale w (S_s - T_s) / N_s,
 * where w_i is the signal's zeroth_weight on its zeroth-order block and 1 elsewhere, and
 * N_s = sum_i w_i T_s,i^2 if `relative` (the relative loss; N_s = 1 when it is 0) and 1
 * otherwise. jtfs_metamer_step uses the same weights (relative = 0, scale = 1).
 * S, S_target, dS: n_coeff_total device floats in the plan's coefficient layout (dS is
 * overwritten and may not alias S or S_target); loss: batch device floats. Enqueued
 * on `stream`; sums are taken in FP64 in a fixed order.
 */
jtfs_status jtfs_loss(jtfs_plan_t plan, const float* S, const float* S_target, float* dS, float* loss,
                      int32_t relative, float scale, jtfs_stream_t stream);

/*
 * Stage timing (for measurement). While enabled, every kernel stage enqueued by
 * jtfs_forward / jtfs_backward / jtfs_metamer_step on this plan is bracketed by two HIP
 * events on the same stream. jtfs_timing_read waits for the recorded events, writes
 * per-stage totals (milliseconds, number of bracketed launches) for stage ids
 * 0..cap-1 and clears them. Stage ids: 0 signal DFT, 1 first-order wavelets,
 * 2 DFT of |Z1|, 3 first-order averaging, 4 order-1 frequential paths, 5 second-order
 * wavelets, 6 frequential contraction + modulus + time pooling (forward), 7 phi_F pooling,
 * 8 pooled-gradient rows, 9 frequential contraction (backward), 10 order-1 adjoint,
 * 11 first-order averaging adjoint, 12 DFT of dY2, 13 second-order adjoint gather,
 * 14 DFT of dZ1, 15 first-order adjoint gather, 16 loss, 17 update, 18 sum of the
 * row-split partials of dY2. Timing state is
 * per plan and not thread-safe: use it from one thread.
 */
#define JTFS_N_STAGES 19
jtfs_status jtfs_timing_enable(jtfs_plan_t plan, int32_t on);
/* Brackets only the stages whose bit is set in `mask` (bit i: stage id i; 0 disables
 * timing; bits at or above JTFS_N_STAGES are JTFS_ERR_ARG). Each bracket records two
 * events, which cost a few microseconds of GPU time: timing one stage perturbs a step
 * far less than timing all of them. */
jtfs_status jtfs_timing_stages(jtfs_plan_t plan, uint32_t mask);
jtfs_status jtfs_timing_read(jtfs_plan_t plan, double* ms, int64_t* counts, int32_t cap);

/* Release a plan and its device tables. NULL is ignored. */
void jtfs_plan_destroy(jtfs_plan_t plan);

/*
 * Tile schedules (performance only: every choice computes the same transform, up to the
 * order of floating-point sums). Zero in a field selects the default.
 *   fwd_rows   workgroups per second-order group targeted by the forward contraction's row
 *              splits (default 256; 16 .. 8192)
 *   fwd_mt     forward time tiles per wave times the group's k-steps: 16 or 32 (default 32)
 *   bwd_rows   workgroups per group targeted by the backward's row splits (default 128)
 *   split_bias shift of the split point of transforms longer than 4096 points, n = A B with
 *              log2 A = floor(log2 n / 2) + split_bias, clamped so that A, B <= 4096 (-2 .. 2)
 *   fwd_rows_k, bwd_rows_k
 *              the same targets for the groups of one k-step bucket (a group with K stacked
 *              first-order rows needs ceil(K / 4) k-steps, rounded up to S = 4, 8, 16, 32 or
 *              64; entry log2(S) - 2); 0 takes fwd_rows / bwd_rows. The buckets' kernels
 *              differ in registers and LDS, hence in how many workgroups fit per CU.
 */
#define JTFS_N_BUCKETS 5
typedef struct {
  int32_t fwd_rows, fwd_mt, bwd_rows, split_bias;
  int32_t fwd_rows_k[JTFS_N_BUCKETS], bwd_rows_k[JTFS_N_BUCKETS];
} jtfs_tuning;

/* jtfs_plan with explicit tile schedules (NULL = defaults). JTFS_ERR_ARG on a field out of range. */
jtfs_status jtfs_plan_tuned(const jtfs_params* signals, int32_t batch, const jtfs_tuning* tuning, jtfs_plan_t* out);

/*
 * jtfs_autotune - pick tile schedules for these signals by measurement on the current
 * device: starting from the defaults, each field in turn (then each bucket's row targets)
 * takes the candidate value that makes one forward + backward fastest (median of 5 timed
 * runs on a seeded synthetic signal, HIP events on `stream`; a candidate must beat the
 * current choice by 0.5%). Allocates and frees its own device buffers; blocks until
 * done. On success *out holds the choice and, if ms is not NULL, *ms its time.
 */
jtfs_status jtfs_autotune(const jtfs_params* signals, int32_t batch, jtfs_stream_t stream, jtfs_tuning* out,
                          double* ms);

/* ------------------------------------------------------------------------------------
 * Learned warm start (an addition to the method; the paper starts descent from noise,
 * Sec. 2.3). A 1-D convolutional decoder maps the coefficients of one signal, read as
 * c_in rows of n_frames frames (every block of the coefficient layout has n_frames
 * frames per row), to a waveform y that seeds the descent:
 *   a_0 = log(1 + S / eps);  z_l[o, t] = b_l[o] + sum_{i,k} W_l[o, i, k] up(a_{l-1})[i, t + k - 4]
 *   a_l = max(z_l, leak z_l) for l < L;  y = z_L[0]
 * where up() inserts stride[l] - 1 zeros after every sample (a transposed convolution
 * with "same" alignment). Weights, activations and activation gradients are stored in
 * bfloat16, products accumulate in FP32 (MFMA), parameters and Adam state are FP32.
 *
 * Parameters are one caller-owned FP32 device vector, layer by layer: W_l as
 * [C_out][C_in][9] (row-major) followed by b_l[C_out]; C_in of layer 0 is c_in, C_out
 * of the last layer is 1, every other count is `channels`.
 * ------------------------------------------------------------------------------------ */
typedef struct jtfs_dec_s* jtfs_dec_t;
#define JTFS_DEC_MAX_LAYERS 8
typedef struct {
  int32_t c_in;        /* coefficient rows per frame (>= 1) */
  int32_t n_frames;    /* frames per row (a multiple of 8) */
  int32_t channels;    /* hidden channels: must be 128 */
  int32_t kernel;      /* taps per filter: must be 9 */
  int32_t n_layers;    /* 2 .. JTFS_DEC_MAX_LAYERS */
  int32_t stride[JTFS_DEC_MAX_LAYERS];   /* upsampling factor per layer: 1, 2 or 4; the last must be 1 */
  float leak;          /* leaky-ReLU slope, in (0, 1] */
  float eps;           /* input compression scale (> 0) */
} jtfs_dec_config;

/* Validates the configuration and sizes the workspace for up to max_batch signals. */
jtfs_status jtfs_dec_create(const jtfs_dec_config* cfg, int32_t max_batch, jtfs_dec_t* out);

/* n_params: parameter vector length; out_len: samples per output waveform
 * (n_frames times the product of the strides); ws_bytes: workspace for max_batch. */
jtfs_status jtfs_dec_query(jtfs_dec_t dec, int64_t* n_params, int64_t* out_len, size_t* ws_bytes);

/*
 * jtfs_dec_forward - y[b] = decoder(S[b]) for b < batch <= max_batch. S: batch x c_in x
 * n_frames device floats (coefficients, >= 0); y: batch x out_len device floats
 * (overwritten). ws keeps the bfloat16 weights and every activation for jtfs_dec_backward.
 */
jtfs_status jtfs_dec_forward(jtfs_dec_t dec, const float* params, const float* S, int32_t batch, float* y, void* ws,
                             size_t ws_bytes, jtfs_stream_t stream);

/*
 * jtfs_dec_backward - grad = d<dy, y>/d params summed over the batch (n_params device
 * floats, overwritten). ws must hold the state of a jtfs_dec_forward call with the same
 * params, batch and workspace, enqueued earlier on the same stream.
 */
jtfs_status jtfs_dec_backward(jtfs_dec_t dec, const float* params, int32_t batch, const float* dy, float* grad,
                              void* ws, size_t ws_bytes, jtfs_stream_t stream);

/* One bias-corrected Adam step on params (FP32); m, v: n_params device floats each,
 * zero before step 1; step counts from 1. */
jtfs_status jtfs_dec_adam_step(jtfs_dec_t dec, float* params, const float* grad, float* m, float* v, int64_t step,
                               float lr, float beta1, float beta2, float eps, jtfs_stream_t stream);

/*
 * jtfs_dec_ws_region - where a hidden layer's state lies in the workspace after
 * jtfs_dec_forward (which = 0: the activation a_l) or jtfs_dec_backward (which = 1: the
 * gradient of its pre-activation z_l), for inspection. Both are bfloat16, time-major
 * [max_batch][t_out][128] (channel fastest), t_out the layer's output length; entries of
 * signals b >= the call's batch are stale. layer < n_layers - 1 (the output layer has
 * neither); offset and bytes in bytes from the workspace's start. JTFS_ERR_ARG otherwise.
 */
jtfs_status jtfs_dec_ws_region(jtfs_dec_t dec, int32_t layer, int32_t which, size_t* offset, size_t* bytes);

/* Release a decoder description. NULL is ignored. */
void jtfs_dec_destroy(jtfs_dec_t dec);

const char* jtfs_status_str(jtfs_status s);
const char* jtfs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* JTFS_H */
