// Frequential scattering and averaging (Sec. 3.4-3.5, Eqs. 2 and 4) and their adjoints.
//
// For one second-order stack Y2 (K rows n1, L2 times t) and frequential filter g with
// subsampling 2^k_g, the frequential convolution is a dense complex contraction
//   V[r, t] = sum_n W[row0_g + r, n] Y2[n, t],  W[row0_g + r, n] = g[(r 2^k_g - n) mod N_fr]
// (a circulant Toeplitz on the zero-padded log-frequency axis, decimated by 2^k_g).
// All filters are stacked into one row space, each padded to a multiple of 16 rows.
// The modulus U2 = |V| is never stored: the forward kernel pools it over time at once,
//   P[r, f] = sum_t U2[r, t] phi_T^(j2)[(f 2^(log2T - j2) - t) mod L2],
// so the chain is MFMA (complex, FP32) -> modulus -> MFMA (pooling), as in a fused
// back-to-back GEMM. Kept frames only (the time unpadding is applied here).
// A second kernel sums the per-time-chunk partials and applies phi_F along r.
//
// MFMA v_mfma_f32_16x16x4f32 operand layout (lane l, i = l % 16, k = l / 16):
//   A[i][k] from lane l, B[k][i] from lane l, D[4k + v][i] in element v of lane l.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace jtfs {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline f4 mfma(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// Hardware square root (v_sqrt_f32, within 1 ulp) for moduli and phases.
__device__ inline float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// 1 / sqrt(x) for x >= the smallest normal float (v_rsq_f32, within 1 ulp), else 0:
// the phase scale of the modulus adjoint, with subgradient 0 where the modulus vanishes
// (below 1.1e-19 the square underflows anyway).
__device__ inline float inv_modulus(float m2) {
  return m2 >= 1.17549435e-38f ? __builtin_amdgcn_rsqf(m2) : 0.f;
}

// Read of a table the plan uploaded once and no kernel writes, through the constant
// address space: a scalar load, which does not wait behind the wave's outstanding vector
// loads (the next tile's prefetch) as a vector load of the same word would.
__device__ inline int load_table(const int* p, int i) {
  typedef const __attribute__((address_space(4))) int ConstInt;
  return ((ConstInt*)p)[i];
}

// Whether row tile rt has non-negligible taps within the first K columns (its rows then
// meet the group's K stacked rows); the plan lists exactly these tiles per group, the
// forward and backward visit only them, and the others' pooled rows are zero.
__device__ __forceinline__ bool tile_live(const DevSig& s, int rt, int K) {
  return min(load_table(s.rt_nrange, 2 * rt + 1), (K + 3) & ~3) > load_table(s.rt_nrange, 2 * rt);
}

// Keeps a value live in a register at this point: the reads that produce it are issued
// (and waited for) here, not sunk into the conditional blocks that use it.
__device__ inline void materialize(float& x) { asm volatile("" : "+v"(x)); }

// Index of the calling thread's wave, as a wave-uniform (scalar) value.
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// ------------------------------------------------------------------ forward contraction
// Work item: group, a block of 4 * RW row tiles (RW 16-row tiles per wave), a chunk of
// TC times. Per wave and 16-time tile: V^T (16 t x 16 r) = Y2^T (t x n) W^T (n x r) for
// each of its row tiles, with W^T in registers and the Y2^T fragments streamed from
// memory one tile ahead (no LDS, no barriers); then P^T (f x r) += Phi^T (f x t) |V^T|,
// the modulus taken in the D layout, which is the B layout of the pooling MFMA.
// Complex products: with a = Y2 and b = W, up to 8 k-steps use three real products
//   P1 = (a_r + a_i) b_r,  P2 = a_r (b_i - b_r),  P3 = a_i (b_r + b_i),
//   Re(ab) = P1 - P3,  Im(ab) = P1 + P2,
// longer ones four (a_r b_r, a_i b_i, a_r b_i + a_i b_r), which needs fewer registers.
constexpr int fwd_rw(int S, int FT) {
  return 2 * (2 * S + 4 * FT) <= 100 ? 2 : 1;
}

// Loads the Y2^T fragments and the Phi^T fragments of the 16-time tile starting at tt.
template <int S, int FT>
__device__ inline void fwd_load(const c32* Y, const float* phi, int L2, int K, int ulo, int nst, int lk, int li, int tt,
                                bool ok, int f_lo, int s_t, int nF, float (&ar)[S], float (&ai)[S], float (&ph)[FT][4]) {
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const int n = ulo + 4 * q + lk;
    c32 y{0.f, 0.f};
    if (ok && q < nst && n < K) y = Y[static_cast<int64_t>(n) * L2 + tt + li];
    ar[q] = y.x;
    ai[q] = y.y;
  }
#pragma unroll
  for (int ft = 0; ft < FT; ++ft) {
    const int f = ft * 16 + li;
    const int fc = (f_lo + f) << s_t;
#pragma unroll
    for (int v = 0; v < 4; ++v) ph[ft][v] = (ok && f < nF) ? phi[(fc - (tt + 4 * lk + v)) & (L2 - 1)] : 0.f;
  }
}

// Contraction, modulus and pooling of one 16-time tile for the wave's RW row tiles.
template <int S, int FT, int RW>
__device__ inline void fwd_tile(const float (&ar)[S], const float (&ai)[S], const float (&ph)[FT][4],
                                const float (&br)[RW][S], const float (&bi)[RW][S], const int (&qa)[RW],
                                const int (&qb)[RW], f4 (&pacc)[RW][FT]) {
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    if (qb[i] > qa[i]) {
      f4 p1 = {0.f, 0.f, 0.f, 0.f}, p2 = {0.f, 0.f, 0.f, 0.f}, p3 = {0.f, 0.f, 0.f, 0.f};
      float u[4];
      if constexpr (S <= 8) {
        // three products: Re = P1 - P3, Im = P1 + P2
#pragma unroll
        for (int q = 0; q < S; ++q) {
          if (q >= qa[i] && q < qb[i]) {
            p1 = mfma(ar[q] + ai[q], br[i][q], p1);
            p2 = mfma(ar[q], bi[i][q] - br[i][q], p2);
            p3 = mfma(ai[q], br[i][q] + bi[i][q], p3);
          }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float re = p1[v] - p3[v], im = p1[v] + p2[v];
          u[v] = hw_sqrt(re * re + im * im);
        }
      } else {
        // four products on the raw parts: Re = a_r b_r - a_i b_i, Im = a_r b_i + a_i b_r
#pragma unroll
        for (int q = 0; q < S; ++q) {
          if (q >= qa[i] && q < qb[i]) {
            p1 = mfma(ar[q], br[i][q], p1);
            p2 = mfma(ai[q], bi[i][q], p2);
            p3 = mfma(ar[q], bi[i][q], p3);
            p3 = mfma(ai[q], br[i][q], p3);
          }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float re = p1[v] - p2[v], im = p3[v];
          u[v] = hw_sqrt(re * re + im * im);
        }
      }
#pragma unroll
      for (int ft = 0; ft < FT; ++ft)
#pragma unroll
        for (int v = 0; v < 4; ++v) pacc[i][ft] = mfma(ph[ft][v], u[v], pacc[i][ft]);
    }
  }
}

template <int S, int FT>
__global__ __launch_bounds__(256, (S >= 32 ? 1 : 2)) void k_freq_fwd(DevSig s, int item0, int run) {
  constexpr int RW = fwd_rw(S, FT);
  // Workgroups are dealt round-robin to the 8 XCDs. A run of `run` consecutive items
  // (same group and time chunk, different row blocks: they read the same Y2 columns)
  // is given to blocks of one XCD so that its L2 serves the re-reads; consecutive runs
  // go to different XCDs to keep their loads even. gridDim.x is a multiple of 8 * run.
  const int j = blockIdx.x >> 3;
  const int item = ((j / run) * 8 + (blockIdx.x & 7)) * run + j % run;
  const FwdItem it = s.fwd_items[item0 + item];
  if (it.grp < 0) return;   // padding item (no barriers in this kernel)
  const FreqGroup fg = s.fgroups[it.grp];
  const int wave = wave_id();
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int K = fg.K;
  const int Kal = (K + 3) & ~3;
  const int rt0 = (it.rb * 4 + wave) * RW;

  int qa[RW], qb[RW];
  int ulo = Kal, uhi = 0;
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    const int lo = load_table(s.rt_nrange, 2 * (rt0 + i));
    const int hi = min(load_table(s.rt_nrange, 2 * (rt0 + i) + 1), Kal);
    qa[i] = lo;
    qb[i] = hi;
    if (hi > lo) {
      ulo = min(ulo, lo);
      uhi = max(uhi, hi);
    }
  }
  const int nst = uhi > ulo ? (uhi - ulo) >> 2 : 0;
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    const bool live = qb[i] > qa[i];
    qa[i] = live ? (qa[i] - ulo) >> 2 : 0;
    qb[i] = live ? (qb[i] - ulo) >> 2 : 0;
  }

  float br[RW][S], bi[RW][S];
#pragma unroll
  for (int i = 0; i < RW; ++i) {
#pragma unroll
    for (int q = 0; q < S; ++q) {
      br[i][q] = 0.f;
      bi[i][q] = 0.f;
      if (q >= qa[i] && q < qb[i]) {
        const c32 w = s.W[static_cast<int64_t>((rt0 + i) * 16 + li) * s.NW + ulo + 4 * q + lk];
        br[i][q] = w.x;
        bi[i][q] = w.y;
      }
    }
  }

  const c32* Y = s.Y2 + fg.y2;
  const float* phi = s.tables + fg.phiT;
  const int L2 = fg.L2;
  const int nF = s.nF;
  f4 pacc[RW][FT];
#pragma unroll
  for (int i = 0; i < RW; ++i)
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) pacc[i][ft] = f4{0.f, 0.f, 0.f, 0.f};

  if (nst > 0) {
    // Two register sets used alternately: the next tile's operands are requested
    // before the current tile is computed (TC is a power of two, at least 16).
    const int tbeg = it.tc * fg.TC, tend = tbeg + fg.TC;
    float ar0[S], ai0[S], ph0[FT][4], ar1[S], ai1[S], ph1[FT][4];
    fwd_load<S, FT>(Y, phi, L2, K, ulo, nst, lk, li, tbeg, true, s.f_lo, fg.s_t, nF, ar0, ai0, ph0);
    for (int tt = tbeg; tt < tend; tt += 32) {
      const bool second = tt + 16 < tend;
      fwd_load<S, FT>(Y, phi, L2, K, ulo, nst, lk, li, tt + 16, second, s.f_lo, fg.s_t, nF, ar1, ai1, ph1);
      fwd_tile<S, FT, RW>(ar0, ai0, ph0, br, bi, qa, qb, pacc);
      fwd_load<S, FT>(Y, phi, L2, K, ulo, nst, lk, li, tt + 32, tt + 32 < tend, s.f_lo, fg.s_t, nF, ar0, ai0, ph0);
      if (second) fwd_tile<S, FT, RW>(ar1, ai1, ph1, br, bi, qa, qb, pacc);
    }
  }
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    float* out = s.part + fg.part + (static_cast<int64_t>(it.tc) * s.R_pad + (rt0 + i) * 16 + li) * nF;
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int f = ft * 16 + 4 * lk + v;
        if (f < nF) out[f] = pacc[i][ft][v];
      }
    }
  }
}

// Integer division rounding towards minus infinity (b > 0).
__device__ inline int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Start slot (frame index on the padded time axis) of the pooling window of forward chunk
// tc of a windowed group: the first frame whose centre lies within the phi_T support.
__device__ inline int window_start(const FreqGroup& fg, int tc) {
  return -floor_div(fg.halo - tc * fg.TC, 1 << fg.s_t);   // ceil((tc TC - halo) / 2^s_t)
}

// Row-tile-loop forward (groups of at most 128 rows, at most 32 frames). Item: group, row
// split, chunk of 64 MT times. Each wave keeps the Y2 operands (as y_r, y_i - y_r,
// y_r + y_i) and the Phi_T^T fragments of its MT 16-time tiles in registers and loops over
// the row tiles of the split; W tiles are staged in LDS, double buffered as in the backward.
// Per row tile and time tile: V^T = Y2^T W^T by three real products
//   k1 = y_r (w_r + w_i),  k2 = (y_i - y_r) w_r,  k3 = (y_r + y_i) w_i,
//   Re V = k1 - k3,  Im V = k1 + k2,
// then |V| in the accumulator layout and P^T += Phi_T^T |V^T|. The four waves' partial sums
// of a row tile are added in a fixed order through LDS and written as the chunk's partial.
// Windowed groups (fg.fw > 0, plans with more than 32 frames) pool each chunk into the fw
// frames starting at window_start(tc) (slots wrap around the padded time axis; frames
// outside the kept ones get zero weight); the partial rows then hold fw window frames.
template <int MAXS, int FT, int MT>
__global__ __launch_bounds__(256, 2) void k_freq_fwd2(DevSig s, int item0) {
  constexpr int WS = 4 * MAXS;                // W tile columns
  constexpr int WSP = WS + 2;                 // LDS row pitch: a row stride of WS would put the
                                              // 16 rows read by one instruction in one bank
  constexpr int PER = (16 * WS + 255) / 256;  // W elements staged per thread
  __shared__ c32 wt[2][16 * WSP];
  __shared__ float red[2][4][FT * 256];
  const FwdItem it = s.fwd_items[item0 + blockIdx.x];
  const FreqGroup fg = s.fgroups[it.grp];
  const int wave = wave_id();
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int L2 = fg.L2;
  const int K = fg.K;
  const int Kal = (K + 3) & ~3;
  const int nF = s.nF;
  const c32* Y = s.Y2 + fg.y2;
  const float* phi = s.tables + fg.phiT;
  const int nslot = L2 >> fg.s_t;   // frame slots on the padded time axis
  const int slot0 = fg.fw > 0 ? window_start(fg, it.tc) : s.f_lo;
  const int pst = fg.fw > 0 ? fg.fw : nF;   // partial row stride
  // this item's share of the group's live row tiles
  const int32_t* live = s.live_rt + fg.lt0;
  const int i_lo = it.rb * fg.rt_fwd;
  const int i_hi = min(fg.nlt, i_lo + fg.rt_fwd);
  const int ncols = min(WS, s.NW);
  float* part = s.part + fg.part + static_cast<int64_t>(it.tc) * s.R_pad * pst;

  // nsub passes over consecutive 64 MT-time sub-chunks of the chunk; every pass adds its
  // pooled sums to the chunk's partial rows (the first pass stores them)
  // (only windowed plans, launched with two frame tiles, take more than one pass)
  const int nsub = FT == 2 ? fg.nsub : 1;
  for (int sub = 0; sub < nsub; ++sub) {
  const int tbase = it.tc * fg.TC + sub * 64 * MT;

  float yre[MT][MAXS], ydf[MT][MAXS], ysm[MT][MAXS], ph[MT][FT][4];
  bool act[MT];
#pragma unroll
  for (int j = 0; j < MT; ++j) {
    const int t0 = tbase + (4 * j + wave) * 16;
    act[j] = t0 < L2;
#pragma unroll
    for (int q = 0; q < MAXS; ++q) {
      const int n = 4 * q + lk;
      c32 y{0.f, 0.f};
      if (act[j] && n < K) y = Y[static_cast<int64_t>(n) * L2 + t0 + li];
      yre[j][q] = y.x;
      ydf[j][q] = y.y - y.x;
      ysm[j][q] = y.x + y.y;
    }
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) {
      const int sl = ((slot0 + ft * 16 + li) % nslot + nslot) % nslot;
      const int f = sl - s.f_lo;   // kept frame index
      const int fc = sl << fg.s_t;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        ph[j][ft][v] = (act[j] && f >= 0 && f < nF) ? phi[(fc - (t0 + 4 * lk + v)) & (L2 - 1)] : 0.f;
    }
  }

  c32 wreg[PER];
  int rt = i_lo < i_hi ? load_table(live, i_lo) : 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i;
    if (e < 16 * WS) {
      const int rr = e / WS, n = e - rr * WS;
      wt[0][rr * WSP + n] = n < ncols ? s.W[static_cast<int64_t>(rt * 16 + rr) * s.NW + n] : c32{0.f, 0.f};
    }
  }
  __syncthreads();
  int buf = 0;
  for (int il = i_lo; il < i_hi; ++il) {
    const bool next = il + 1 < i_hi;
    const int rt_next = next ? load_table(live, il + 1) : 0;
    if (next) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = threadIdx.x + 256 * i;
        if (e < 16 * WS) {
          const int rr = e / WS, n = e - rr * WS;
          wreg[i] = n < ncols ? s.W[static_cast<int64_t>(rt_next * 16 + rr) * s.NW + n] : c32{0.f, 0.f};
        }
      }
    }
    const int nlo = load_table(s.rt_nrange, 2 * rt);
    const int nhi = min(load_table(s.rt_nrange, 2 * rt + 1), Kal);
    const c32* w = wt[buf];
    f4 pacc[FT];
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) pacc[ft] = f4{0.f, 0.f, 0.f, 0.f};
    if (nhi > nlo) {
      // with few k-steps, the row tile's W operands are read once (one LDS wait) for all
      // MT time tiles
      constexpr bool PRE = MAXS <= 8;
      c32 av[PRE ? MAXS : 1];
      if constexpr (PRE) {
#pragma unroll
        for (int q = 0; q < MAXS; ++q) av[q] = w[li * WSP + 4 * q + lk];
#pragma unroll
        for (int q = 0; q < MAXS; ++q) {
          materialize(av[q].x);
          materialize(av[q].y);
        }
      }
#pragma unroll
      for (int j = 0; j < MT; ++j) {
        if (act[j]) {
          // otherwise each k-step's operand is read one step ahead, its wait placed after
          // the products of the step before
          c32 an = PRE ? c32{0.f, 0.f} : w[li * WSP + lk];
          f4 k1 = {0.f, 0.f, 0.f, 0.f}, k2 = {0.f, 0.f, 0.f, 0.f}, k3 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int q = 0; q < MAXS; ++q) {
            const c32 a = PRE ? av[PRE ? q : 0] : an;
            if (!PRE && q + 1 < MAXS) an = w[li * WSP + 4 * (q + 1) + lk];
            if (4 * q >= nlo && 4 * q < nhi) {
              k1 = mfma(yre[j][q], a.x + a.y, k1);
              k2 = mfma(ydf[j][q], a.x, k2);
              k3 = mfma(ysm[j][q], a.y, k3);
            }
            if (!PRE && q + 1 < MAXS) {
              materialize(an.x);
              materialize(an.y);
            }
          }
          float u[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float re = k1[v] - k3[v], im = k1[v] + k2[v];
            u[v] = hw_sqrt(re * re + im * im);
          }
#pragma unroll
          for (int ft = 0; ft < FT; ++ft)
#pragma unroll
            for (int v = 0; v < 4; ++v) pacc[ft] = mfma(ph[j][ft][v], u[v], pacc[ft]);
        }
      }
    }
#pragma unroll
    for (int ft = 0; ft < FT; ++ft)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[buf][wave][ft * 256 + lane * 4 + v] = pacc[ft][v];
    if (next) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = threadIdx.x + 256 * i;
        if (e < 16 * WS) {
          const int rr = e / WS, n = e - rr * WS;
          wt[buf ^ 1][rr * WSP + n] = wreg[i];
        }
      }
    }
    __syncthreads();
    // P^T[f][r] of this row tile: element e = ft 256 + lane 4 + v holds frame
    // ft 16 + 4 (lane / 16) + v of row lane mod 16
#pragma unroll
    for (int i = 0; i < FT; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int ln = (e & 255) >> 2, v = e & 3;
      const int f = (e >> 8) * 16 + 4 * (ln >> 4) + v;   // kept frame, or window frame
      if (f < pst) {
        const float sum = (red[buf][0][e] + red[buf][1][e]) + (red[buf][2][e] + red[buf][3][e]);
        float* dst = part + static_cast<int64_t>(rt * 16 + (ln & 15)) * pst + f;
        *dst = sub == 0 ? sum : *dst + sum;
      }
    }
    buf ^= 1;
    rt = rt_next;
  }
  __syncthreads();   // the next pass restages wt[0] and rewrites red
  }
}

// Sum over the time chunks of a non-windowed group's pooled partials, one thread per
// (row, kept frame) cell: eight independent partial sums (eight loads in flight),
// combined in a fixed order.
__global__ __launch_bounds__(256) void k_freq_psum(DevSig s) {
  const FreqGroup fg = s.fgroups[blockIdx.y];
  if (fg.psum < 0) return;
  const int64_t cells = static_cast<int64_t>(s.R_pad) * s.nF;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (e >= cells) return;
  if (!tile_live(s, static_cast<int>(e / s.nF) >> 4, fg.K)) {   // not written by the forward
    s.psum[fg.psum + e] = 0.f;
    return;
  }
  const float* src = s.part + fg.part + e;
  float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int tc = 0;
  for (; tc + 8 <= fg.n_tc; tc += 8) {
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] += src[(tc + j) * cells];
  }
  for (int j = 0; tc < fg.n_tc; ++tc, ++j) a[j] += src[tc * cells];
  s.psum[fg.psum + e] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// Sum of the time-chunk partials (read from k_freq_psum, or summed here for windowed
// groups), phi_F averaging along log-frequency (band-pass g) or nothing more (g = phi_F),
// log-frequency unpadding, store into S.
constexpr int kPoolFrames = 8;   // frames per pooling workgroup

__global__ __launch_bounds__(256) void k_freq_pool(DevSig s) {
  __shared__ float P[8192];
  const int gi = blockIdx.x / s.n_g, g = blockIdx.x % s.n_g;
  const FreqGroup fg = s.fgroups[gi];
  const FrFilter ff = s.frf[g];
  const int nF = s.nF;
  // kept bins: phi_F-averaged (stride 2^sF) or, without frequential averaging, the
  // band-pass's own stride 2^k (its rows are output as they are)
  const bool pooled = !ff.lowpass && !s.no_avg_fr;
  const int kb = pooled || ff.lowpass ? s.sF : ff.k;
  const int nb = (fg.K + (1 << kb) - 1) >> kb;
  float* out = s.S + s.s_off[gi * s.n_g + g];
  const int Mrows = pooled ? ff.M : nb;
  // blockIdx.y takes frames [8 y, 8 y + 8) (Mrows <= 1024, so the tile fits P)
  const int fw = max(1, min(nF, 8192 / Mrows));
  const int fb = min(fw, kPoolFrames);
  const int sh = s.sF - ff.k;
  const float* ph = s.tables + ff.phiF;
  for (int f0 = blockIdx.y * fb; f0 < min(nF, (blockIdx.y + 1) * fb); f0 += fb) {
    const int fc = min(fb, nF - f0);
    __syncthreads();
    for (int e = threadIdx.x; e < Mrows * fc; e += 256) {
      const int r = e / fc, fl = e - r * fc;
      float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (fg.fw > 0 && !tile_live(s, (ff.row0 + r) >> 4, fg.K)) {
        // a row the forward did not visit: zero
      } else if (fg.fw > 0) {
        // windowed partials: chunk tc holds frame slot f_lo + f at window offset o < fw. The
        // window of chunk t starts at ceil((t TC - halo) / 2^s_t), so only the chunks t with
        // (slot - fw) 2^s_t + halo < t TC <= slot 2^s_t + halo hold the slot (t taken
        // modulo the chunk count: the windows of t and t + n_tc differ by one turn).
        const int nslot = fg.L2 >> fg.s_t;
        const int w = 1 << fg.s_t;
        const int slot = s.f_lo + f0 + fl;
        const float* src = s.part + fg.part + static_cast<int64_t>(ff.row0 + r) * fg.fw;
        const int64_t stride = static_cast<int64_t>(s.R_pad) * fg.fw;
        int t_lo = floor_div((slot - fg.fw) * w + fg.halo, fg.TC);
        const int t_hi = floor_div(slot * w + fg.halo, fg.TC);
        if (t_hi - t_lo + 1 > fg.n_tc) t_lo = t_hi - fg.n_tc + 1;
        for (int t = t_lo; t <= t_hi; ++t) {
          const int tc = ((t % fg.n_tc) + fg.n_tc) % fg.n_tc;
          const int o = ((slot - window_start(fg, tc)) % nslot + nslot) % nslot;
          if (o < fg.fw) a[(t - t_lo) & 7] += src[tc * stride + o];
        }
      } else {
        // summed over the time chunks by k_freq_psum
        a[0] = s.psum[fg.psum + static_cast<int64_t>(ff.row0 + r) * nF + f0 + fl];
      }
      P[r * fc + fl] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nb * fc; e += 256) {
      const int b = e / fc, fl = e - b * fc;
      float v;
      if (!pooled) {
        v = P[b * fc + fl];
      } else {
        float acc = 0.f;
        for (int r = 0; r < ff.M; ++r) acc += ph[((b << sh) - r) & (ff.M - 1)] * P[r * fc + fl];
        v = acc;
      }
      out[b * nF + f0 + fl] = v;
    }
  }
}

// ------------------------------------------------------------------ order 1 (alpha = 0)
// Frequential filters of the real list on S1 (kept frames only): V = W_g S1; the
// band-pass paths keep |V| for phi_F averaging, phi_F itself keeps V (Eq. 3 has no
// modulus). One thread per (row of the real list, frame); rows of other filters and
// padding rows are written as zero.
__device__ inline int real_filter_of_row(const DevSig& s, int row) {
  for (int q = 0; q < s.n_real; ++q) {
    const FrFilter c = s.frf[q];
    if (row >= c.row0 && row < c.row0 + c.M) return q;
  }
  return -1;
}

__device__ inline c32 order1_v(const DevSig& s, int row, int f) {
  const c32* w = s.W + static_cast<int64_t>(row) * s.NW;
  const float* x = s.S1 + s.f_lo + f;
  // four independent partial sums (loads in flight), combined in a fixed order
  float vr[4] = {0.f, 0.f, 0.f, 0.f}, vi[4] = {0.f, 0.f, 0.f, 0.f};
  int n = 0;
  for (; n + 4 <= s.N1; n += 4) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float a = x[static_cast<int64_t>(n + j) * s.nf_pad];
      vr[j] += w[n + j].x * a;
      vi[j] += w[n + j].y * a;
    }
  }
  for (int j = 0; n < s.N1; ++n, ++j) {
    const float a = x[static_cast<int64_t>(n) * s.nf_pad];
    vr[j] += w[n].x * a;
    vi[j] += w[n].y * a;
  }
  return c32{(vr[0] + vr[1]) + (vr[2] + vr[3]), (vi[0] + vi[1]) + (vi[2] + vi[3])};
}

__global__ __launch_bounds__(64) void k_o1_v(DevSig s) {
  const int e = blockIdx.x * 64 + threadIdx.x;
  if (e >= s.R_pad * s.nF) return;
  const int row = e / s.nF, f = e - row * s.nF;
  const int g = real_filter_of_row(s, row);
  float u = 0.f;
  if (g >= 0) {
    const c32 v = order1_v(s, row, f);
    u = s.frf[g].lowpass ? v.x : sqrtf(v.x * v.x + v.y * v.y);
  }
  s.o1[e] = c32{u, 0.f};
}

// phi_F averaging along log-frequency and unpadding of the order-1 paths. One wave per
// output: the lanes split the sum over rows, then a fixed butterfly combines them.
__global__ __launch_bounds__(256) void k_o1_pool(DevSig s) {
  const int g = blockIdx.y;
  const FrFilter ff = s.frf[g];
  const int nF = s.nF;
  const bool pooled = !ff.lowpass && !s.no_avg_fr;
  const int kb = pooled || ff.lowpass ? s.sF : ff.k;
  const int nb = (s.N1 + (1 << kb) - 1) >> kb;
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (e >= nb * nF) return;   // whole waves leave together (no barriers below)
  const int b = e / nF, f = e - b * nF;
  float v = 0.f;
  if (!pooled) {
    v = lane == 0 ? s.o1[(ff.row0 + b) * nF + f].x : 0.f;
  } else {
    const int sh = s.sF - ff.k;
    const float* ph = s.tables + ff.phiF;
    for (int r = lane; r < ff.M; r += 64) v += ph[((b << sh) - r) & (ff.M - 1)] * s.o1[(ff.row0 + r) * nF + f].x;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane == 0) s.S[s.s_off[s.n_groups * s.n_g + g] + e] = v;
}

// Adjoint of the order-1 paths, step 1: per (row, frame) the gradient of V.
__global__ __launch_bounds__(64) void k_o1_dv(DevSig s) {
  const int e = blockIdx.x * 64 + threadIdx.x;
  if (e >= s.R_pad * s.nF) return;
  const int nF = s.nF;
  const int row = e / nF, f = e - row * nF;
  const int g = real_filter_of_row(s, row);
  c32 d{0.f, 0.f};
  if (g >= 0) {
    const FrFilter ff = s.frf[g];
    const int r = row - ff.row0;
    const bool pooled = !ff.lowpass && !s.no_avg_fr;
    const int kb = pooled || ff.lowpass ? s.sF : ff.k;
    const int nb = (s.N1 + (1 << kb) - 1) >> kb;
    const float* dout = s.dS + s.s_off[s.n_groups * s.n_g + g];
    if (ff.lowpass) {
      d.x = r < nb ? dout[r * nF + f] : 0.f;
    } else {
      const int sh = s.sF - ff.k;
      const float* ph = s.tables + ff.phiF;
      float du = 0.f;
      if (pooled) {
        for (int b = 0; b < nb; ++b) du += ph[((b << sh) - r) & (ff.M - 1)] * dout[b * nF + f];
      } else if (r < nb) {
        du = dout[r * nF + f];
      }
      const c32 v = order1_v(s, row, f);
      const float m = sqrtf(v.x * v.x + v.y * v.y);
      if (m > 0.f) d = c32{du * (v.x / m), du * (v.y / m)};
    }
  }
  s.o1[e] = d;
}

// Step 2: dS1 contribution of filter g, Re(W_g^H dV), on every padded frame (zero
// outside the kept ones); summed over g in a fixed order later.
__global__ __launch_bounds__(256) void k_o1_ds1(DevSig s) {
  // 64 cells per block; the four waves take interleaved quarters of the rows and their
  // sums are combined through LDS in a fixed order
  __shared__ float red[4][64];
  const int g = blockIdx.y;
  const FrFilter ff = s.frf[g];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  if (e < s.N1 * s.nf_pad) {
    const int n = e / s.nf_pad, f = e - n * s.nf_pad;
    const int fl = f - s.f_lo;
    if (fl >= 0 && fl < s.nF) {
      const int nb = (s.N1 + (1 << s.sF) - 1) >> s.sF;
      const int rows = ff.lowpass ? nb : ff.M;
      // rows wave, wave + 4, ...: four independent partial sums per thread
      int r = wave, j = 0;
      for (; r < rows; r += 4, j = (j + 1) & 3) {
        const c32 w = s.W[static_cast<int64_t>(ff.row0 + r) * s.NW + n];
        const c32 d = s.o1[(ff.row0 + r) * s.nF + fl];
        acc[j] += w.x * d.x + w.y * d.y;
      }
    }
  }
  red[wave][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (wave == 0 && e < s.N1 * s.nf_pad)
    s.dS1p[static_cast<int64_t>(g) * s.N1 * s.nf_pad + e] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// Sum of the row-split partials of dY2 into split 0 (fixed order), groups with RS > 1.
__global__ __launch_bounds__(256) void k_dy_reduce(DevSig s) {
  const FreqGroup fg = s.fgroups[blockIdx.y];
  if (fg.RS <= 1) return;
  const int64_t n = static_cast<int64_t>(fg.K) * fg.L2;
  c32* base = s.dYpart + fg.dYpart;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * 256) {
    c32 acc = base[e];
    for (int r = 1; r < fg.RS; ++r) {
      const c32 v = base[r * n + e];
      acc.x += v.x;
      acc.y += v.y;
    }
    base[e] = acc;
  }
}

// ------------------------------------------------------------------ backward
// Pooled-gradient rows: dP[row, f] = sum_b phi_F^(k_g)[(b 2^(sF - k_g) - r) mod M] dS[b, f]
// (band-pass g) or dS[r, f] (g = phi_F); zero on padding rows.
__global__ __launch_bounds__(256) void k_freq_dP(DevSig s) {
  const int gi = blockIdx.y;
  const FreqGroup fg = s.fgroups[gi];
  const int nF = s.nF;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= s.R_pad * nF) return;
  const int row = e / nF, f = e - (e / nF) * nF;
  if (!tile_live(s, row >> 4, fg.K)) return;   // (the backward reads live row tiles only)
  int g = -1;
  for (int q = 0; q < s.n_g; ++q) {
    const FrFilter c = s.frf[q];
    if (row >= c.row0 && row < c.row0 + ((c.M + 15) & ~15)) g = q;
  }
  float v = 0.f;
  if (g >= 0) {
    const FrFilter ff = s.frf[g];
    const int r = row - ff.row0;
    const bool pooled = !ff.lowpass && !s.no_avg_fr;
    const int kb = pooled || ff.lowpass ? s.sF : ff.k;
    const int nb = (fg.K + (1 << kb) - 1) >> kb;
    const float* in = s.dS + s.s_off[gi * s.n_g + g];
    if (r < ff.M) {
      if (!pooled) {
        v = r < nb ? in[r * nF + f] : 0.f;
      } else {
        const int sh = s.sF - ff.k;
        const float* ph = s.tables + ff.phiF;
        for (int b = 0; b < nb; ++b) v += ph[((b << sh) - r) & (ff.M - 1)] * in[b * nF + f];
      }
    }
  }
  s.dP[fg.dP + e] = v;
}

// Work item: group, 64 times (one 16-time tile per wave), a split of the row tiles.
// Per wave and row tile: recompute V (16 r x 16 t) = W Y2, dU = dP Phi (time-pooling
// adjoint), dV = dU V / |V|, then dY2 (n x t) += W^H dV; Y2 operands and dY2
// accumulators stay in registers over the row loop. W tiles are staged in LDS, double
// buffered: the next live tile's global loads are in flight while the current one is
// used, and one barrier per tile separates the buffers. Only the group's live row tiles
// (the plan's list) are visited.

// HF > 0: the pooled-gradient rows of each row tile travel with its W tile through LDS and
// the Phi_T fragments are loaded once (at most HF = 16 or 32 frames, MAXS <= 32); a
// separate instantiation, so that the other paths' global loads do not make the compiler
// wait for the W prefetch before the pooling products. HF = 0: the pooled gradients are
// read from global memory inside the row loop (more frames, windowed groups).
// WIN (with HF = 32, more than 32 frames): the staged frames are the slots within the
// phi_T support of the workgroup's 64 times (at most 32, checked by the launcher), and
// each wave pools only its own slots among them.
template <int MAXS, int MAXNT, int HF, bool WIN = false>
__global__ __launch_bounds__(256, 2) void k_freq_bwd(DevSig s, int item0) {
  constexpr int WS = 4 * MAXS;               // W tile columns
  // LDS row pitch (see the forward); the widest variant stays unpadded within 64 KiB
  constexpr int WSP = MAXS >= 64 ? WS : WS + 2;
  constexpr int PER = (16 * WS + 255) / 256;  // W elements staged per thread
  static_assert(HF == 0 || (MAXS <= 32 && (HF == 16 || HF == 32)), "hoisting needs MAXS <= 32, HF 16 or 32");
  static_assert(!WIN || HF == 32, "windowed hoisting stages 32 slots");
  // per buffer: the W tile, then (HF > 0) 16 HF floats of pooled-gradient rows
  __shared__ c32 wt[2][16 * WSP + 8 * HF];
  const BwdItem it = s.bwd_items[item0 + blockIdx.x];
  const FreqGroup fg = s.fgroups[it.grp];
  const int wave = wave_id();
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int t0 = it.tb * 64 + wave * 16;
  const int L2 = fg.L2;
  const bool active = t0 < L2;
  const int K = fg.K;
  const int Kal = (K + 3) & ~3;
  const int NT = (K + 15) >> 4;
  const int ncols = NT * 16;
  const c32* Y = s.Y2 + fg.y2;

  // Y2 operands kept as y_r, y_i - y_r and y_r + y_i: V = W Y2 by three real products
  //   k1 = (w_r + w_i) y_r,  k2 = w_r (y_i - y_r),  k3 = w_i (y_r + y_i),
  //   Re V = k1 - k3,  Im V = k1 + k2.
  // (the widest variant keeps four real products, y_r and y_i, for want of registers)
  constexpr bool G3 = MAXS <= 32;
  float yre[MAXS], ydf[MAXS], ysm[G3 ? MAXS : 1];
#pragma unroll
  for (int q = 0; q < MAXS; ++q) {
    yre[q] = 0.f;
    ydf[q] = 0.f;
    if constexpr (G3) ysm[q] = 0.f;
    const int n = 4 * q + lk;
    if (active && n < K) {
      const c32 y = Y[static_cast<int64_t>(n) * L2 + t0 + li];
      yre[q] = y.x;
      if constexpr (G3) {
        ydf[q] = y.y - y.x;
        ysm[q] = y.x + y.y;
      } else {
        ydf[q] = y.y;
      }
    }
  }
  // dY2 = W^H dV accumulated the same way: with w = a + ib,
  //   k1 = (a - b) dv_r,  k2 = a (dv_i - dv_r),  k3 = b (dv_r + dv_i),
  //   Re dY2 = k1 + k3,  Im dY2 = k1 + k2.
  // (four products, widest variant: dk1 = Re, dk2 = Im)
  f4 dk1[MAXNT], dk2[MAXNT], dk3[G3 ? MAXNT : 1];
#pragma unroll
  for (int q = 0; q < MAXNT; ++q) {
    dk1[q] = f4{0.f, 0.f, 0.f, 0.f};
    dk2[q] = f4{0.f, 0.f, 0.f, 0.f};
    if constexpr (G3) dk3[q] = f4{0.f, 0.f, 0.f, 0.f};
  }
  // this item's share of the group's live row tiles
  const int32_t* live = s.live_rt + fg.lt0;
  const int i_lo = it.rs * fg.rt_per_split;
  const int i_hi = min(fg.nlt, i_lo + fg.rt_per_split);
  const float* phi = s.tables + fg.phiT;
  const int nF = s.nF;
  const int nFq = (nF + 3) >> 2;
  // With at most 16 frames (and registers to spare), the Phi_T fragments of this wave's
  // times are loaded once, and each row tile's pooled gradients travel with its W tile
  // through LDS instead of being loaded inside the loop.
  auto dpt = [&](int b) { return reinterpret_cast<float*>(wt[b] + 16 * WSP); };
  constexpr bool hoist = HF > 0;
  constexpr int NQ = HF > 0 ? HF / 4 : 1;   // 4-frame k-steps of the hoisted pooling adjoint
  const float* dPg = s.dP + fg.dP;
  // frame slots within the phi_T support of this wave's 16 times
  const int sl0 = -floor_div(fg.halo - t0, 1 << fg.s_t);
  const int nsl = floor_div(t0 + 15 + fg.halo, 1 << fg.s_t) - sl0 + 1;
  const int nslot = L2 >> fg.s_t;
  // staged window: W frames per row (all kept frames, or the workgroup's WIN slots from sw0);
  // this wave's slots start at offset ow in it
  int W = nF, sw0 = s.f_lo, ow = 0;
  if constexpr (WIN) {
    const int tw0 = it.tb * 64;
    sw0 = -floor_div(fg.halo - tw0, 1 << fg.s_t);
    W = floor_div(tw0 + 63 + fg.halo, 1 << fg.s_t) - sw0 + 1;
    ow = sl0 - sw0;
  }
  float bph[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int f = 4 * q + lk;
    if constexpr (WIN) {
      const int sl = ((sl0 + f) % nslot + nslot) % nslot;
      const int fk = sl - s.f_lo;
      bph[q] = (active && f < nsl && fk >= 0 && fk < nF) ? phi[((sl << fg.s_t) - (t0 + li)) & (L2 - 1)] : 0.f;
    } else {
      bph[q] = (hoist && active && f < nF) ? phi[(((s.f_lo + f) << fg.s_t) - (t0 + li)) & (L2 - 1)] : 0.f;
    }
  }
  // complete these loads here: left pending into the loop, they make every pooling
  // product wait for all outstanding loads, the next W tile's prefetch included
#pragma unroll
  for (int q = 0; q < NQ; ++q) materialize(bph[q]);
  // staged pooled-gradient floats (16 rows of W frames): element threadIdx.x and, with 32
  // frames, threadIdx.x + 256; doff = its offset in a row tile's dP rows (-1: a slot
  // outside the kept frames, staged as zero)
  const bool dp_thread = hoist && static_cast<int>(threadIdx.x) < 16 * W;
  const bool dp_thread2 = HF > 16 && static_cast<int>(threadIdx.x) + 256 < 16 * W;
  int doff = threadIdx.x, doff2 = threadIdx.x + 256;
  if constexpr (WIN) {
    auto off = [&](int e) {
      const int rr = e / W, k = e - rr * W;
      const int fk = ((sw0 + k) % nslot + nslot) % nslot - s.f_lo;
      return (fk >= 0 && fk < nF) ? rr * nF + fk : -1;
    };
    doff = dp_thread ? off(threadIdx.x) : -1;
    doff2 = dp_thread2 ? off(threadIdx.x + 256) : -1;
  }
  auto dp_at = [&](int t, int o) { return o >= 0 ? dPg[static_cast<int64_t>(t) * 16 * nF + o] : 0.f; };
  float dreg = 0.f, dreg2 = 0.f;

  // stage the first live tile
  int il = i_lo;
  int rt = il < i_hi ? load_table(live, il) : 0;
  c32 wreg[PER];
  if (il < i_hi) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int rr = e / WS, n = e - rr * WS;
      wt[0][rr * WSP + n] = n < ncols ? s.W[static_cast<int64_t>(rt * 16 + rr) * s.NW + n] : c32{0.f, 0.f};
    }
    if (dp_thread) dpt(0)[threadIdx.x] = dp_at(rt, doff);
    if (dp_thread2) dpt(0)[threadIdx.x + 256] = dp_at(rt, doff2);
  }
  __syncthreads();
  int buf = 0;
  while (il < i_hi) {
    const bool more = il + 1 < i_hi;
    const int nxt = more ? load_table(live, il + 1) : 0;
    if (more) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = threadIdx.x + 256 * i;
        const int rr = e / WS, n = e - rr * WS;
        wreg[i] = n < ncols ? s.W[static_cast<int64_t>(nxt * 16 + rr) * s.NW + n] : c32{0.f, 0.f};
      }
      if (dp_thread) dreg = dp_at(nxt, doff);
      if (dp_thread2) dreg2 = dp_at(nxt, doff2);
    }
    const int nlo = load_table(s.rt_nrange, 2 * rt);
    const int nhi = min(load_table(s.rt_nrange, 2 * rt + 1), Kal);
    const int r0 = rt * 16;
    const c32* w = wt[buf];
    if (active) {
      // With few k-steps, all of the tile's W operands are read at once (one LDS wait)
      // before the in-band products.
      constexpr bool PRE = MAXS <= 8;
      c32 av[PRE ? MAXS : 1];
      if constexpr (PRE) {
#pragma unroll
        for (int q = 0; q < MAXS; ++q) av[q] = w[li * WSP + 4 * q + lk];
#pragma unroll
        for (int q = 0; q < MAXS; ++q) {
          materialize(av[q].x);
          materialize(av[q].y);
        }
      }
      // otherwise each k-step's operand is read one step ahead, its wait placed after
      // the products of the step before
      c32 an = PRE ? c32{0.f, 0.f} : w[li * WSP + lk];
      f4 k1 = {0.f, 0.f, 0.f, 0.f}, k2 = {0.f, 0.f, 0.f, 0.f}, k3 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < MAXS; ++q) {
        const c32 a = PRE ? av[PRE ? q : 0] : an;
        if (!PRE && q + 1 < MAXS) an = w[li * WSP + 4 * (q + 1) + lk];
        if (4 * q >= nlo && 4 * q < nhi) {
          if constexpr (G3) {
            k1 = mfma(a.x + a.y, yre[q], k1);
            k2 = mfma(a.x, ydf[q], k2);
            k3 = mfma(a.y, ysm[q], k3);
          } else {   // k1 = Re V, k2 = Im V (ydf holds y_i)
            k1 = mfma(a.x, yre[q], k1);
            k1 = mfma(-a.y, ydf[q], k1);
            k2 = mfma(a.x, ydf[q], k2);
            k2 = mfma(a.y, yre[q], k2);
          }
        }
        if (!PRE && q + 1 < MAXS) {
          materialize(an.x);
          materialize(an.y);
        }
      }
      f4 vr, vi;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        vr[v] = G3 ? k1[v] - k3[v] : k1[v];
        vi[v] = G3 ? k1[v] + k2[v] : k2[v];
      }
      f4 du = {0.f, 0.f, 0.f, 0.f};
      if constexpr (WIN) {
        // this wave's nsl slots start at ow in the staged window: read all NQ operands at
        // once (indices clamped into the row), then drop the slots beyond nsl
        const float* dp = dpt(buf) + li * W;
        float dv[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) dv[q] = dp[min(ow + 4 * q + lk, W - 1)];
#pragma unroll
        for (int q = 0; q < NQ; ++q) materialize(dv[q]);
        const int nq = (nsl + 3) >> 2;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          if (q < nq) du = mfma(4 * q + lk < nsl ? dv[q] : 0.f, bph[q], du);
        }
      } else if constexpr (hoist) {
        // li nF + f <= 15 HF + HF - 1 stays inside the staged rows: read all NQ operands
        // at once, then drop the frames beyond nF
        const float* dp = dpt(buf) + li * nF;
        float dv[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) dv[q] = dp[4 * q + lk];
#pragma unroll
        for (int q = 0; q < NQ; ++q) materialize(dv[q]);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          if (q < nFq) du = mfma(4 * q + lk < nF ? dv[q] : 0.f, bph[q], du);
        }
      } else if (nsl < nF) {   // (HF = 0)
        // only the frames whose centres lie within the phi_T support of the wave's times
        const float* dPr = dPg + static_cast<int64_t>(r0 + li) * nF;
        for (int q = 0; q < (nsl + 3) >> 2; ++q) {
          const int k = 4 * q + lk;
          const int sl = ((sl0 + k) % nslot + nslot) % nslot;
          const int f = sl - s.f_lo;
          float a = 0.f, b = 0.f;
          if (k < nsl && f >= 0 && f < nF) {
            a = dPr[f];
            b = phi[((sl << fg.s_t) - (t0 + li)) & (L2 - 1)];
          }
          du = mfma(a, b, du);
        }
      } else {
        const float* dPr = dPg + static_cast<int64_t>(r0 + li) * nF;
        for (int q = 0; q < nFq; ++q) {
          const int f = 4 * q + lk;
          float a = 0.f, b = 0.f;
          if (f < nF) {
            a = dPr[f];
            b = phi[(((s.f_lo + f) << fg.s_t) - (t0 + li)) & (L2 - 1)];
          }
          du = mfma(a, b, du);
        }
      }
      float dvr[4], ddf[4], dsm[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float sc = du[v] * inv_modulus(vr[v] * vr[v] + vi[v] * vi[v]);
        const float r = vr[v] * sc, i = vi[v] * sc;
        dvr[v] = r;
        ddf[v] = i - r;
        dsm[v] = r + i;
      }
      c32 bv[PRE ? 4 * MAXNT : 1];
      if constexpr (PRE) {
#pragma unroll
        for (int nt = 0; nt < MAXNT; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) bv[4 * nt + v] = w[(4 * lk + v) * WSP + nt * 16 + li];
#pragma unroll
        for (int e = 0; e < 4 * MAXNT; ++e) {
          materialize(bv[e].x);
          materialize(bv[e].y);
        }
      }
#pragma unroll
      for (int nt = 0; nt < MAXNT; ++nt) {
        if (nt < NT && nt * 16 < nhi && nt * 16 + 16 > nlo) {
          // (without the preload: the column tile's four operands are read together)
          c32 bq[4];
          if constexpr (!PRE) {
#pragma unroll
            for (int v = 0; v < 4; ++v) bq[v] = w[(4 * lk + v) * WSP + nt * 16 + li];
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const c32 a = PRE ? bv[PRE ? 4 * nt + v : 0] : bq[v];
            if constexpr (G3) {
              dk1[nt] = mfma(a.x - a.y, dvr[v], dk1[nt]);
              dk2[nt] = mfma(a.x, ddf[v], dk2[nt]);
              dk3[nt] = mfma(a.y, dsm[v], dk3[nt]);
            } else {   // dv_i = ddf + dv_r
              const float di = ddf[v] + dvr[v];
              dk1[nt] = mfma(a.x, dvr[v], dk1[nt]);
              dk1[nt] = mfma(a.y, di, dk1[nt]);
              dk2[nt] = mfma(a.x, di, dk2[nt]);
              dk2[nt] = mfma(-a.y, dvr[v], dk2[nt]);
            }
          }
        }
      }
    }
    if (more) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = threadIdx.x + 256 * i;
        const int rr = e / WS, n = e - rr * WS;
        wt[buf ^ 1][rr * WSP + n] = wreg[i];
      }
      if (dp_thread) dpt(buf ^ 1)[threadIdx.x] = dreg;
      if (dp_thread2) dpt(buf ^ 1)[threadIdx.x + 256] = dreg2;
    }
    __syncthreads();
    buf ^= 1;
    rt = nxt;
    ++il;
  }
  if (!active) return;
  c32* dst = s.dYpart + fg.dYpart + static_cast<int64_t>(it.rs) * K * L2;
#pragma unroll
  for (int nt = 0; nt < MAXNT; ++nt) {
    if (nt < NT) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int n = nt * 16 + 4 * lk + v;
        if (n < K) {
          c32 d{dk1[nt][v], dk2[nt][v]};
          if constexpr (G3) d = c32{dk1[nt][v] + dk3[nt][v], dk1[nt][v] + dk2[nt][v]};
          dst[static_cast<int64_t>(n) * L2 + t0 + li] = d;
        }
      }
    }
  }
}

}  // namespace

hipError_t run_order1_fwd(const DevSig& s, const SigPlan& p, hipStream_t st) {
  const int rows = (p.R_pad * p.n_frames + 63) / 64;
  hipLaunchKernelGGL(k_o1_v, dim3(rows), dim3(64), 0, st, s);
  int nb = 0;   // the most kept bins of any real-list filter
  for (int32_t g : p.fr_real) {
    const FrFilter& ff = p.frf[static_cast<size_t>(g)];
    const int kb = (!ff.lowpass && p.no_avg_fr) ? ff.k : p.sF;
    nb = std::max(nb, (static_cast<int>(p.psi1.size()) + (1 << kb) - 1) >> kb);
  }
  hipLaunchKernelGGL(k_o1_pool, dim3((nb * p.n_frames + 3) / 4, p.fr_real.size()), dim3(256), 0, st, s);
  return hipGetLastError();
}

hipError_t run_order1_bwd(const DevSig& s, const SigPlan& p, hipStream_t st) {
  const int rows = (p.R_pad * p.n_frames + 63) / 64;
  hipLaunchKernelGGL(k_o1_dv, dim3(rows), dim3(64), 0, st, s);
  const int cells = (static_cast<int>(p.psi1.size()) * p.nf_pad + 63) / 64;
  hipLaunchKernelGGL(k_o1_ds1, dim3(cells, p.fr_real.size()), dim3(256), 0, st, s);
  return hipGetLastError();
}

hipError_t run_dy_reduce(const DevSig& s, const SigPlan& p, hipStream_t st) {
  if (p.groups.empty()) return hipSuccess;
  int64_t most = 0;
  for (const FreqGroup& fg : p.fgroups)
    if (fg.RS > 1) most = std::max<int64_t>(most, static_cast<int64_t>(fg.K) * fg.L2);
  if (most == 0) return hipSuccess;
  const int blocks = static_cast<int>(std::min<int64_t>((most + 255) / 256, 1024));
  hipLaunchKernelGGL(k_dy_reduce, dim3(blocks, p.groups.size()), dim3(256), 0, st, s);
  return hipGetLastError();
}

template <int S>
hipError_t launch_fwd_s(const DevSig& s, const SigPlan::FwdLaunch& l, hipStream_t st) {
  switch (l.FT) {
    case 1: hipLaunchKernelGGL((k_freq_fwd<S, 1>), dim3(l.nitems), dim3(256), 0, st, s, l.item0, l.run); break;
    case 2: hipLaunchKernelGGL((k_freq_fwd<S, 2>), dim3(l.nitems), dim3(256), 0, st, s, l.item0, l.run); break;
    case 4: hipLaunchKernelGGL((k_freq_fwd<S, 4>), dim3(l.nitems), dim3(256), 0, st, s, l.item0, l.run); break;
    default: hipLaunchKernelGGL((k_freq_fwd<S, 8>), dim3(l.nitems), dim3(256), 0, st, s, l.item0, l.run); break;
  }
  return hipGetLastError();
}

// Time tiles per wave: 16 / S or 32 / S (at least 1); with two frame tiles 16 / S only.
template <int S>
hipError_t launch_fwd2_s(const DevSig& s, const SigPlan::FwdLaunch& l, hipStream_t st) {
  constexpr int LO = 16 / S > 1 ? 16 / S : 1, HI = 32 / S > 1 ? 32 / S : 1;
  const dim3 g(l.nitems), b(256);
  if (l.FT == 1 && l.MT == HI) {
    hipLaunchKernelGGL((k_freq_fwd2<S, 1, HI>), g, b, 0, st, s, l.item0);
  } else if (l.FT == 1 && l.MT == LO) {
    hipLaunchKernelGGL((k_freq_fwd2<S, 1, LO>), g, b, 0, st, s, l.item0);
  } else if (l.FT == 2 && l.MT == LO) {
    hipLaunchKernelGGL((k_freq_fwd2<S, 2, LO>), g, b, 0, st, s, l.item0);
  } else {
    return hipErrorInvalidValue;   // plan and kernel disagree
  }
  return hipGetLastError();
}

hipError_t run_freq_fwd(const DevSig& s, const SigPlan& p, hipStream_t st) {
  for (const SigPlan::FwdLaunch& l : p.fwd_launches) {
    if (l.RW == 0) {   // row-tile-loop kernel
      hipError_t e;
      switch (l.S) {
        case 4: e = launch_fwd2_s<4>(s, l, st); break;
        case 8: e = launch_fwd2_s<8>(s, l, st); break;
        case 16: e = launch_fwd2_s<16>(s, l, st); break;
        case 32: e = launch_fwd2_s<32>(s, l, st); break;
        default: return hipErrorInvalidValue;
      }
      if (e != hipSuccess) return e;
      continue;
    }
    if (l.RW != fwd_rw(l.S, l.FT)) return hipErrorInvalidValue;   // plan and kernel disagree
    hipError_t e;
    switch (l.S) {
      case 4: e = launch_fwd_s<4>(s, l, st); break;
      case 8: e = launch_fwd_s<8>(s, l, st); break;
      case 16: e = launch_fwd_s<16>(s, l, st); break;
      case 32: e = launch_fwd_s<32>(s, l, st); break;
      case 64: e = launch_fwd_s<64>(s, l, st); break;
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t run_freq_pool(const DevSig& s, const SigPlan& p, hipStream_t st) {
  if (p.groups.empty()) return hipSuccess;
  if (p.psum_total > 0) {
    const int blocks = static_cast<int>((static_cast<int64_t>(p.R_pad) * p.n_frames + 255) / 256);
    hipLaunchKernelGGL(k_freq_psum, dim3(blocks, p.groups.size()), dim3(256), 0, st, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_freq_pool, dim3(p.groups.size() * p.fr.size(), (p.n_frames + kPoolFrames - 1) / kPoolFrames),
                     dim3(256), 0, st, s);
  return hipGetLastError();
}

hipError_t run_freq_dP(const DevSig& s, const SigPlan& p, hipStream_t st) {
  if (p.groups.empty()) return hipSuccess;
  const int blocks = (p.R_pad * p.n_frames + 255) / 256;
  hipLaunchKernelGGL(k_freq_dP, dim3(blocks, p.groups.size()), dim3(256), 0, st, s);
  return hipGetLastError();
}

hipError_t run_freq_bwd(const DevSig& s, const SigPlan& p, hipStream_t st) {
  // pooled gradients hoisted through LDS for up to 16 or 32 frames; beyond, the slots of
  // each workgroup's phi_T window when every group of the launch keeps that within 32
  // (k-step buckets up to 16), else read in the loop
  const int hf0 = p.n_frames <= 16 ? 16 : p.n_frames <= 32 ? 32 : 0;
  for (const SigPlan::BwdLaunch& l : p.bwd_launches) {
    const dim3 grid(l.nitems);
    int hf = hf0;
    if (hf == 0 && l.S <= 16) {
      bool fits = true;
      for (const FreqGroup& fg : p.fgroups) {
        const int need = (fg.K + 3) / 4;
        const int bucket = need <= 4 ? 4 : need <= 8 ? 8 : need <= 16 ? 16 : need <= 32 ? 32 : 64;
        // widest window of a 64-time block: floor((63 + 2 halo) / 2^s_t) + 2 slots
        if (bucket == l.S && (63 + 2 * fg.halo) / (1 << fg.s_t) + 2 > 32) fits = false;
      }
      if (fits) hf = -1;
    }
#define JTFS_BWD(S_, NT_)                                                                            \
  do {                                                                                             \
    if (hf == 16) hipLaunchKernelGGL((k_freq_bwd<S_, NT_, 16>), grid, dim3(256), 0, st, s, l.item0); \
    else if (hf == 32) hipLaunchKernelGGL((k_freq_bwd<S_, NT_, 32>), grid, dim3(256), 0, st, s, l.item0); \
    else if (hf == -1) hipLaunchKernelGGL((k_freq_bwd<S_, NT_, 32, true>), grid, dim3(256), 0, st, s, l.item0); \
    else hipLaunchKernelGGL((k_freq_bwd<S_, NT_, 0>), grid, dim3(256), 0, st, s, l.item0);          \
  } while (0)
    switch (l.S) {
      case 4: JTFS_BWD(4, 1); break;
      case 8: JTFS_BWD(8, 2); break;
      case 16: JTFS_BWD(16, 4); break;
      case 32:   // (32 hoisted frames would spill at this width)
        if (hf == 16) hipLaunchKernelGGL((k_freq_bwd<32, 8, 16>), grid, dim3(256), 0, st, s, l.item0);
        else hipLaunchKernelGGL((k_freq_bwd<32, 8, 0>), grid, dim3(256), 0, st, s, l.item0);
        break;
      default: hipLaunchKernelGGL((k_freq_bwd<64, 16, 0>), grid, dim3(256), 0, st, s, l.item0); break;
    }
#undef JTFS_BWD
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace jtfs
