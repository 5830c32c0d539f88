// Warm-start decoder kernels: transposed-convolution layers as implicit GEMMs on
// v_mfma_f32_16x16x32_bf16 (bfloat16 operands, FP32 accumulation), their data and
// weight gradients, the one-channel output layer in FP32 vector arithmetic, Adam.
//
// Layer l:  z[o, t] = b[o] + sum_{i,k} W[o, i, k] up_s(a)[i, t + k - 4],  a' = lrelu(z).
// Polyphase form used by every kernel: for output t = s m + r only the taps with
// (r + k - 4) divisible by s meet a non-zero sample, at input u = m + (r + k - 4) / s.
//
// MFMA 16x16x32 operand layout (one wave): lane l holds row (l mod 16) of A and column
// (l mod 16) of B, each as 8 consecutive K values starting at 8 (l / 16); the result
// holds D[4 (l / 16) + v][l mod 16] in accumulator v. Both operands are loaded with the
// same K order, so the product does not depend on how the unit orders K internally.
#include <hip/hip_runtime.h>

#include "dec.hpp"

namespace jtfs {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kRowB = kDecC + 8;   // LDS row pitch of a bf16 tile (272 bytes)
constexpr int kRowF = kDecC + 4;   // LDS row pitch of an FP32 tile
constexpr int fwd_pitch(int s) { return s == 4 ? kDecC : kRowB; }
// input rows per workgroup of the LDS-staged forward (stride 2 or 4)
constexpr int fwd_lds_rows(int s) { return s == 2 ? 96 : 64; }
// its LDS bytes: the staged inputs and one tap's weights, or the output tile
constexpr size_t fwd_lds_bytes(int s) {
  return ((fwd_lds_rows(s) + 2 * (kDecH / s) + kDecC) * kRowB > s * fwd_lds_rows(s) * fwd_pitch(s)
              ? size_t(fwd_lds_rows(s) + 2 * (kDecH / s) + kDecC) * kRowB
              : size_t(s) * fwd_lds_rows(s) * fwd_pitch(s)) * sizeof(uint16_t);
}
static_assert(fwd_lds_bytes(2) <= 65536 && fwd_lds_bytes(4) <= 65536, "LDS-staged forward exceeds 64 KiB");

__device__ inline f32x4 mma(uint4 a, uint4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                  0, 0);
}

// Round to nearest even (finite inputs).
__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ inline float bf2f(uint32_t h) { return __uint_as_float(h << 16); }
__device__ inline float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

__device__ inline int wave_index() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

__device__ inline uint4 ld16(const uint16_t* p) { return *reinterpret_cast<const uint4*>(p); }
__device__ inline void st16(uint16_t* p, uint4 v) { *reinterpret_cast<uint4*>(p) = v; }

// Eight bf16 starting E elements into the 16 held by (lo, hi).
template <int E>
__device__ inline uint4 realign(uint4 lo, uint4 hi) {
  const uint32_t d[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
  uint32_t o[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if constexpr (E % 2 == 0) {
      o[i] = d[E / 2 + i];
    } else {
      o[i] = (d[E / 2 + i] >> 16) | (d[E / 2 + i + 1] << 16);
    }
  }
  return uint4{o[0], o[1], o[2], o[3]};
}

// ---------------------------------------------------------------------------------------
// Weight copies and input map

__global__ void k_cast_wf(const float* __restrict__ W, int c_in, int cip, int c_out, uint16_t* __restrict__ wf) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(c_out) * kDecK * cip) return;
  const int ci = static_cast<int>(i % cip);
  const int k = static_cast<int>((i / cip) % kDecK);
  const int co = static_cast<int>(i / (int64_t(cip) * kDecK));
  wf[i] = ci < c_in ? f2bf(W[(int64_t(co) * c_in + ci) * kDecK + k]) : uint16_t(0);
}

__global__ void k_cast_wd(const float* __restrict__ W, int c_in, int c_out, uint16_t* __restrict__ wd) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(c_in) * kDecK * c_out) return;
  const int co = static_cast<int>(i % c_out);
  const int k = static_cast<int>((i / c_out) % kDecK);
  const int ci = static_cast<int>(i / (int64_t(c_out) * kDecK));
  wd[i] = f2bf(W[(int64_t(co) * c_in + ci) * kDecK + k]);
}

// Every layer's copies in one launch: element i belongs to the layer whose running end
// passes it; inside the layer, first the forward copy, then the data-gradient copy (or the
// output layer's rounded FP32 copy). Same element maps as the kernels above.
__global__ void k_cast_all(DecCastSet set) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  int l = 0;
  while (l < set.n && i >= set.end[l]) ++l;
  if (l >= set.n) return;
  int64_t e = i - (l > 0 ? set.end[l - 1] : 0);
  const float* W = set.W[l];
  const int c_in = set.c_in[l], cip = set.cip[l], c_out = set.c_out[l];
  if (set.wf[l]) {
    const int64_t n = int64_t(c_out) * kDecK * cip;
    if (e < n) {
      const int ci = static_cast<int>(e % cip);
      const int k = static_cast<int>((e / cip) % kDecK);
      const int co = static_cast<int>(e / (int64_t(cip) * kDecK));
      set.wf[l][e] = ci < c_in ? f2bf(W[(int64_t(co) * c_in + ci) * kDecK + k]) : uint16_t(0);
      return;
    }
    e -= n;
  }
  if (set.wd[l]) {
    const int co = static_cast<int>(e % c_out);
    const int k = static_cast<int>((e / c_out) % kDecK);
    const int ci = static_cast<int>(e / (int64_t(c_out) * kDecK));
    set.wd[l][e] = f2bf(W[(int64_t(co) * c_in + ci) * kDecK + k]);
    return;
  }
  set.wout[e] = bf2f(f2bf(W[e]));
}

__global__ void k_cast_out(const float* __restrict__ W, int n, float* __restrict__ wo) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wo[i] = bf2f(f2bf(W[i]));
}

__global__ void k_dec_input(const float* __restrict__ S, int c_in, int F, int cip, float eps,
                            uint16_t* __restrict__ x_tc, uint16_t* __restrict__ x_ct) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= F * cip) return;
  const int c = i % cip, f = i / cip;
  const uint16_t v = c < c_in ? f2bf(log1pf(S[(int64_t(b) * c_in + c) * F + f] / eps)) : uint16_t(0);
  x_tc[(int64_t(b) * F + f) * cip + c] = v;
  uint16_t* row = x_ct + (int64_t(b) * cip + c) * (F + 2 * kDecPad);
  row[kDecPad + f] = v;
  if (f < kDecPad) {
    row[f] = 0;
    row[kDecPad + F + f] = 0;
  }
}

// ---------------------------------------------------------------------------------------
// Hidden layer forward. Workgroup: batch item blockIdx.y, input rows m in [64 bx, 64 bx + 64),
// all s phases, all 128 output channels. Wave w: 32 rows (w & 1) x 64 channels (w >> 1).

template <int S>
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t* __restrict__ x, int cip, int t_in,
                                                  const uint16_t* __restrict__ wf, const float* __restrict__ bias,
                                                  float leak, uint16_t* __restrict__ out_tc,
                                                  uint16_t* __restrict__ out_ct) {
  extern __shared__ uint16_t tile[];   // [64 S][P]; unpadded at S = 4 to stay within 64 KiB
  constexpr int P = fwd_pitch(S);
  const int b = blockIdx.y, m0 = blockIdx.x * kDecTile;
  const int w = wave_index();
  const int lane = threadIdx.x & 63, g = lane >> 4, li = lane & 15;
  const int mw = m0 + 32 * (w & 1), cw = 64 * (w >> 1);
  const int t_out = S * t_in;
  const uint16_t* xb = x + int64_t(b) * t_in * cip;
  const uint4 zero{0u, 0u, 0u, 0u};

#pragma unroll
  for (int r = 0; r < S; ++r) {
    f32x4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < kDecK; ++k) {
      if ((r + k - kDecH + 4 * S) % S != 0) continue;
      const int d = (r + k - kDecH) / S;   // exact division
      const uint16_t* arow[2];
      bool aok[2];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
        const int u = mw + 16 * mb + li + d;
        aok[mb] = u >= 0 && u < t_in;
        arow[mb] = xb + int64_t(aok[mb] ? u : 0) * cip + 8 * g;
      }
      const uint16_t* brow[4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) brow[cb] = wf + (int64_t(cw + 16 * cb + li) * kDecK + k) * cip + 8 * g;
      for (int c0 = 0; c0 < cip; c0 += 32) {
        uint4 A[2], Bv[4];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) A[mb] = aok[mb] ? ld16(arow[mb] + c0) : zero;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) Bv[cb] = ld16(brow[cb] + c0);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) acc[mb][cb] = mma(A[mb], Bv[cb], acc[mb][cb]);
      }
    }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int co = cw + 16 * cb + li;
        const float bo = bias[co];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ml = 32 * (w & 1) + 16 * mb + 4 * g + v;
          const float z = acc[mb][cb][v] + bo;
          tile[(ml * S + r) * P + co] = f2bf(z > 0.f ? z : leak * z);
        }
      }
  }
  __syncthreads();
  const int t0 = m0 * S;
  // TC rows
  for (int i = threadIdx.x; i < kDecTile * S * 16; i += 256) {
    const int row = i >> 4, c8 = (i & 15) * 8;
    if (t0 + row < t_out) st16(out_tc + (int64_t(b) * t_out + t0 + row) * kDecC + c8, ld16(tile + row * P + c8));
  }
  // CT rows: 8 consecutive samples of one channel per thread (neighbouring threads take
  // neighbouring channels, so the LDS reads are conflict-free)
  const int n8 = kDecTile * S / 8;
  const int64_t ct_len = t_out + 2 * kDecPad;
  for (int i = threadIdx.x; i < kDecC * n8; i += 256) {
    const int co = i % kDecC, ch = i / kDecC;
    const int t = t0 + 8 * ch;
    if (t >= t_out) continue;
    uint32_t o[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      o[e] = uint32_t(tile[(8 * ch + 2 * e) * P + co]) | (uint32_t(tile[(8 * ch + 2 * e + 1) * P + co]) << 16);
    st16(out_ct + (int64_t(b) * kDecC + co) * ct_len + kDecPad + t, uint4{o[0], o[1], o[2], o[3]});
  }
  if (blockIdx.x == 0)
    for (int co = threadIdx.x; co < kDecC; co += 256) st16(out_ct + (int64_t(b) * kDecC + co) * ct_len, uint4{0, 0, 0, 0});
  if (blockIdx.x == gridDim.x - 1)
    for (int co = threadIdx.x; co < kDecC; co += 256)
      st16(out_ct + (int64_t(b) * kDecC + co) * ct_len + kDecPad + t_out, uint4{0, 0, 0, 0});
}

// ---------------------------------------------------------------------------------------
// Hidden layer forward, LDS-staged (strides 2 and 4, 128 input channels). Workgroup: batch
// item blockIdx.y, input rows m in [MR bx, MR bx + MR) (MR = 96 at stride 2, 64 at stride 4,
// so that every staged tile fits in 64 KiB of LDS), all 128 output channels. The input rows (with the taps' halo of 4 / S rows on each side)
// are staged in LDS once; the weights of one tap at a time ([128 co][128 ci], 32 KiB) are
// staged in LDS and read by all four waves, so each weight is fetched from L2 once per
// workgroup and tap instead of once per wave and row block. Wave w: rows (w & 1) MR / 2 ..
// + MR / 2, channels 64 (w >> 1) .. + 64, all S phases (32 accumulator tiles).
template <int S>
__global__ __launch_bounds__(256, 2) void k_conv_fwd_lds(const uint16_t* __restrict__ x, int t_in,
                                                         const uint16_t* __restrict__ wf, const float* __restrict__ bias,
                                                         float leak, uint16_t* __restrict__ out_tc,
                                                         uint16_t* __restrict__ out_ct) {
  static_assert(S == 2 || S == 4, "LDS-staged forward: strides 2 and 4");
  constexpr int MR = fwd_lds_rows(S);  // input rows per workgroup
  constexpr int H = kDecH / S;         // halo rows: d = (r + k - 4) / S lies in [-H, H]
  constexpr int NRI = MR + 2 * H;      // staged input rows
  constexpr int RT = MR / 32;          // 16-row tiles per wave
  constexpr int P = kRowB;             // LDS pitch (bf16) of the input and weight tiles
  constexpr int PO = fwd_pitch(S);     // LDS pitch of the output tile
  extern __shared__ uint16_t lds[];
  uint16_t* xin = lds;                 // [NRI][P]
  uint16_t* wk = lds + NRI * P;        // [128][P]
  uint16_t* tile = lds;                // epilogue: [S MR][PO] (after the last product)
  const int b = blockIdx.y, m0 = blockIdx.x * MR;
  const int w = wave_index();
  const int lane = threadIdx.x & 63, g = lane >> 4, li = lane & 15;
  const int rw = (w & 1) * (MR / 2), cw = 64 * (w >> 1);
  const int t_out = S * t_in;
  const uint16_t* xb = x + int64_t(b) * t_in * kDecC;
  const uint4 zero{0u, 0u, 0u, 0u};

  // a tap's weights: eight 16-byte pieces per thread, loaded one tap ahead (in flight during
  // the previous tap's products)
  uint4 wpre[8];
  auto load_tap = [&](int k) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int co = e >> 4, c8 = (e & 15) * 8;
      wpre[q] = ld16(wf + (int64_t(co) * kDecK + k) * kDecC + c8);
    }
  };
  load_tap(0);
  {
    // input rows: every load issued before the first store (addresses clamped to row 0,
    // values outside [0, t_in) replaced by zeros)
    constexpr int NX = (NRI * 16 + 255) / 256;
    uint4 xv[NX];
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      const int e = min(int(threadIdx.x) + 256 * q, NRI * 16 - 1);
      const int u = m0 - H + (e >> 4);
      const bool ok = u >= 0 && u < t_in;
      const uint4 v = ld16(xb + int64_t(ok ? u : 0) * kDecC + (e & 15) * 8);
      xv[q] = ok ? v : zero;
    }
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (e < NRI * 16) st16(xin + (e >> 4) * P + (e & 15) * 8, xv[q]);
    }
  }
  f32x4 acc[S][RT][4];
#pragma unroll
  for (int r = 0; r < S; ++r)
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[r][i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
  for (int k = 0; k < kDecK; ++k) {
    __syncthreads();   // the previous tap's weights are consumed (and, first, the input staged)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = threadIdx.x + 256 * q;
      st16(wk + (e >> 4) * P + (e & 15) * 8, wpre[q]);
    }
    if (k + 1 < kDecK) load_tap(k + 1);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < S; ++r) {
      if ((r + k - kDecH + 4 * S) % S != 0) continue;
      const int d = (r + k - kDecH) / S;   // exact division
#pragma unroll
      for (int c0 = 0; c0 < kDecC; c0 += 32) {
        uint4 A[RT], Bv[4];
#pragma unroll
        for (int i = 0; i < RT; ++i) A[i] = ld16(xin + (rw + 16 * i + li + d + H) * P + c0 + 8 * g);
#pragma unroll
        for (int j = 0; j < 4; ++j) Bv[j] = ld16(wk + (cw + 16 * j + li) * P + c0 + 8 * g);
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[r][i][j] = mma(A[i], Bv[j], acc[r][i][j]);
      }
    }
  }
  __syncthreads();   // every wave is done with the staged inputs and weights
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int co = cw + 16 * j + li;
    const float bo = bias[co];
#pragma unroll
    for (int r = 0; r < S; ++r)
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ml = rw + 16 * i + 4 * g + v;
          const float z = acc[r][i][j][v] + bo;
          tile[(ml * S + r) * PO + co] = f2bf(z > 0.f ? z : leak * z);
        }
  }
  __syncthreads();
  const int t0 = m0 * S;
  // TC rows
  for (int i = threadIdx.x; i < S * MR * 16; i += 256) {
    const int row = i >> 4, c8 = (i & 15) * 8;
    if (t0 + row < t_out) st16(out_tc + (int64_t(b) * t_out + t0 + row) * kDecC + c8, ld16(tile + row * PO + c8));
  }
  // CT rows: 8 consecutive samples of one channel per thread (neighbouring threads take
  // neighbouring channels)
  const int64_t ct_len = t_out + 2 * kDecPad;
  for (int i = threadIdx.x; i < kDecC * (S * MR / 8); i += 256) {
    const int co = i % kDecC, ch = i / kDecC;
    const int t = t0 + 8 * ch;
    if (t >= t_out) continue;
    uint32_t o[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      o[e] = uint32_t(tile[(8 * ch + 2 * e) * PO + co]) | (uint32_t(tile[(8 * ch + 2 * e + 1) * PO + co]) << 16);
    st16(out_ct + (int64_t(b) * kDecC + co) * ct_len + kDecPad + t, uint4{o[0], o[1], o[2], o[3]});
  }
  if (blockIdx.x == 0)
    for (int co = threadIdx.x; co < kDecC; co += 256) st16(out_ct + (int64_t(b) * kDecC + co) * ct_len, uint4{0, 0, 0, 0});
  if (blockIdx.x == gridDim.x - 1)
    for (int co = threadIdx.x; co < kDecC; co += 256)
      st16(out_ct + (int64_t(b) * kDecC + co) * ct_len + kDecPad + t_out, uint4{0, 0, 0, 0});
}

// ---------------------------------------------------------------------------------------
// Shared epilogue of the data-gradient kernels: a bf16 tile of dz rows u in [u0, u0 + ROWS)
// (LDS, pitch kRowB) goes to the polyphase layout of stride S2.
template <int S2, int ROWS = kDecTile>
__device__ void store_polyphase(const uint16_t* tile, int b, int u0, int t_rows, uint16_t* __restrict__ dzp) {
  const int M2 = t_rows / S2;
  const int64_t row_len = M2 + 2 * kDecPad;
  constexpr int n8 = ROWS / S2 / 8;
  const int m20 = u0 / S2;
  for (int i = threadIdx.x; i < kDecC * S2 * n8; i += 256) {
    const int ci = i / (S2 * n8), rem = i % (S2 * n8), r2 = rem / n8, ch = rem % n8;
    const int m2 = m20 + 8 * ch;
    if (m2 >= M2) continue;
    uint32_t o[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int ua = S2 * (8 * ch + 2 * e) + r2, ub = S2 * (8 * ch + 2 * e + 1) + r2;
      o[e] = uint32_t(tile[ua * kRowB + ci]) | (uint32_t(tile[ub * kRowB + ci]) << 16);
    }
    st16(dzp + ((int64_t(b) * kDecC + ci) * S2 + r2) * row_len + kDecPad + m2, uint4{o[0], o[1], o[2], o[3]});
  }
  if (u0 == 0)
    for (int i = threadIdx.x; i < kDecC * S2; i += 256) st16(dzp + (int64_t(b) * kDecC * S2 + i) * row_len, uint4{0, 0, 0, 0});
  if (u0 + ROWS >= t_rows)
    for (int i = threadIdx.x; i < kDecC * S2; i += 256)
      st16(dzp + (int64_t(b) * kDecC * S2 + i) * row_len + kDecPad + M2, uint4{0, 0, 0, 0});
}

// Masks an FP32 tile of da (LDS, pitch kRowF) with lrelu'(a_prev), writes dz TC rows and
// the bf16 tile for the polyphase store.
__device__ void mask_store_tc(const float* ftile, uint16_t* btile, int b, int u0, int t_rows,
                              const uint16_t* __restrict__ a_tc, float leak, uint16_t* __restrict__ dz_tc) {
  for (int i = threadIdx.x; i < kDecTile * 16; i += 256) {
    const int row = i >> 4, c8 = (i & 15) * 8;
    const int u = u0 + row;
    if (u >= t_rows) continue;
    const int64_t off = (int64_t(b) * t_rows + u) * kDecC + c8;
    const uint4 a = ld16(a_tc + off);
    const uint32_t aw[4] = {a.x, a.y, a.z, a.w};
    uint32_t o[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float d0 = ftile[row * kRowF + c8 + 2 * e], d1 = ftile[row * kRowF + c8 + 2 * e + 1];
      const float m0 = bf_lo(aw[e]) > 0.f ? d0 : leak * d0;
      const float m1 = bf_hi(aw[e]) > 0.f ? d1 : leak * d1;
      o[e] = uint32_t(f2bf(m0)) | (uint32_t(f2bf(m1)) << 16);
    }
    const uint4 v{o[0], o[1], o[2], o[3]};
    st16(dz_tc + off, v);
    st16(btile + row * kRowB + c8, v);
  }
}

// Hidden layer data gradient. Rows u of the layer input, channels ci:
//   da[u, ci] = sum_k sum_co W[co, ci, k] dz[s u - k + 4, co]
// Workgroup: batch item blockIdx.y, rows [128 bx, 128 bx + 128), wave w: 64 rows (w & 1) x
// 64 channels (w >> 1). The taps with 4 - k = s q + p read only the dz rows t = s v + p
// (v = u + q), so the workgroup stages those rows of one parity p in LDS once, for half of
// the output channels at a time, and runs the parity's taps on them; each tap's weights
// for that half ([128 ci][64 co]) are staged too, loaded a tap ahead. The epilogue runs in
// two 64-row halves through the shared helpers.
constexpr int kDgradRows = 128;
constexpr int kDgradPitch = 64 + 8;   // 144 bytes: rows 16 bytes apart modulo the 128-byte bank cycle
constexpr size_t kDgradLdsBig = size_t(kDecTile) * kRowF * sizeof(float) + size_t(kDecTile) * kRowB * sizeof(uint16_t);
static_assert(size_t(kDgradRows + 2 * kDecH + kDecC) * kDgradPitch * sizeof(uint16_t) <= kDgradLdsBig,
              "staged rows and weights larger than the epilogue tiles");

// The order of a workgroup's products: parity p, then channel half h, then the taps of p.
template <int S>
struct DgradSeq {
  int p[2 * kDecK], h[2 * kDecK], k[2 * kDecK];
  constexpr DgradSeq() : p(), h(), k() {
    int n = 0;
    for (int pp = 0; pp < S; ++pp)
      for (int hh = 0; hh < 2; ++hh)
        for (int kk = 0; kk < kDecK; ++kk)
          if (((kDecH - kk - pp) % S + S) % S == 0) {
            p[n] = pp;
            h[n] = hh;
            k[n] = kk;
            ++n;
          }
  }
};

template <int S, int S2>
__global__ __launch_bounds__(256, 2) void k_conv_dgrad_lds(const uint16_t* __restrict__ dz, int t_out,
                                                           const uint16_t* __restrict__ wd, int t_in,
                                                           const uint16_t* __restrict__ a_prev, float leak,
                                                           uint16_t* __restrict__ dz_prev,
                                                           uint16_t* __restrict__ dzp_prev) {
  constexpr int H = kDecH / S;                 // |q| <= H
  constexpr int NR = kDgradRows + 2 * H;       // staged rows v = u0 - H ..
  constexpr int PA = kDgradPitch;
  constexpr int NA = (NR * 8 + 255) / 256;     // staged 16-byte pieces per thread
  constexpr DgradSeq<S> seq{};
  extern __shared__ float smem[];
  uint16_t* at = reinterpret_cast<uint16_t*>(smem);                        // [NR][PA]
  uint16_t* wk = at + NR * PA;                                             // [128][PA]
  float* ftile = smem;                                                     // epilogue: [64][kRowF]
  uint16_t* btile = reinterpret_cast<uint16_t*>(smem + kDecTile * kRowF);  // epilogue: [64][kRowB]
  const int b = blockIdx.y, u0 = blockIdx.x * kDgradRows;
  const int w = wave_index();
  const int lane = threadIdx.x & 63, g = lane >> 4, li = lane & 15;
  const int rw = 64 * (w & 1), cw = 64 * (w >> 1);
  const uint16_t* db = dz + int64_t(b) * t_out * kDecC;
  const uint4 zero{0u, 0u, 0u, 0u};
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // weights of tap k, channel half h: 4 pieces per thread (ci = e >> 3, co = 64 h + 8 (e & 7))
  uint4 wpre[4];
  auto load_w = [&](int k, int h) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q;
      wpre[q] = ld16(wd + (int64_t(e >> 3) * kDecK + k) * kDecC + 64 * h + (e & 7) * 8);
    }
  };
  // dz rows t = S v + p of channel half h (zero outside [0, t_out)); loads unconditional
  uint4 apre[NA];
  auto load_a = [&](int p, int h) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = min(int(threadIdx.x) + 256 * q, NR * 8 - 1);
      const int t = S * (u0 - H + (e >> 3)) + p;
      const bool ok = t >= 0 && t < t_out;
      const uint4 v = ld16(db + int64_t(ok ? t : 0) * kDecC + 64 * h + (e & 7) * 8);
      apre[q] = ok ? v : zero;
    }
  };
  load_w(seq.k[0], seq.h[0]);
  load_a(seq.p[0], seq.h[0]);
#pragma unroll
  for (int n = 0; n < 2 * kDecK; ++n) {
    const int p = seq.p[n], h = seq.h[n], k = seq.k[n];
    const bool restage = n == 0 || p != seq.p[n - 1] || h != seq.h[n - 1];
    const bool next_restage = n + 1 < 2 * kDecK && (p != seq.p[n + 1] || h != seq.h[n + 1]);
    __syncthreads();   // the previous products are done with the staged rows and weights
    if (restage) {
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int e = threadIdx.x + 256 * q;
        if (e < NR * 8) st16(at + (e >> 3) * PA + (e & 7) * 8, apre[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q;
      st16(wk + (e >> 3) * PA + (e & 7) * 8, wpre[q]);
    }
    if (n + 1 < 2 * kDecK) load_w(seq.k[n + 1], seq.h[n + 1]);
    if (next_restage) load_a(seq.p[n + 1], seq.h[n + 1]);
    __syncthreads();
    const int qs = (kDecH - k - p) / S + H;   // staged row of u = u0 is qs (exact division)
#pragma unroll
    for (int c0 = 0; c0 < 64; c0 += 32) {
      uint4 A[4], Bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) A[i] = ld16(at + (rw + 16 * i + li + qs) * PA + c0 + 8 * g);
#pragma unroll
      for (int j = 0; j < 4; ++j) Bv[j] = ld16(wk + (cw + 16 * j + li) * PA + c0 + 8 * g);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mma(A[i], Bv[j], acc[i][j]);
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    __syncthreads();   // the weights (h = 0) or the previous half's tiles (h = 1) are consumed
    if ((w & 1) == h) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) ftile[(16 * i + 4 * g + v) * kRowF + cw + 16 * j + li] = acc[i][j][v];
    }
    __syncthreads();
    mask_store_tc(ftile, btile, b, u0 + kDecTile * h, t_in, a_prev, leak, dz_prev);
    __syncthreads();
    store_polyphase<S2>(btile, b, u0 + kDecTile * h, t_in, dzp_prev);
  }
}

// ---------------------------------------------------------------------------------------
// Hidden layer weight gradient for one tap KT:
//   dW[co, ci, KT] = sum_b sum_m dz_P[b, co, r, m] x[b, ci, m - q],  4 - KT = s q + r, 0 <= r < s.
// Workgroup: one chunk of (b, m) (blockIdx.x), 64 input channels (blockIdx.y); all 128 output
// channels, wave w owning rows [32 w, 32 w + 32). Partials [chunk][9][128][cip], summed later.
// Launched at stride 1 (the first layer, whose 266 input channels are padded to 320); strides
// 2 and 4 use the row-wise kernel below, which shares the dz rows between taps.
template <int S, int KT>
__device__ void wgrad_tap(const uint16_t* __restrict__ dzp, const uint16_t* __restrict__ xct, int M, int cip, int b,
                          int m_begin, int m_end, int ci0, float* __restrict__ part) {
  constexpr int r = ((kDecH - KT) % S + S) % S;
  constexpr int q = (kDecH - KT - r) / S;
  constexpr int sh = -q;                       // x is read at m + sh
  constexpr int e = ((sh % 8) + 8) % 8;
  constexpr int lo_off = sh < 0 ? -8 : 0;
  const int w = wave_index();
  const int lane = threadIdx.x & 63, g = lane >> 4, li = lane & 15;
  const int64_t row_len = M + 2 * kDecPad;
  const uint4 zero{0u, 0u, 0u, 0u};
  const uint16_t* arow[2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
    arow[mb] = dzp + ((int64_t(b) * kDecC + 32 * w + 16 * mb + li) * S + r) * row_len + kDecPad;
  const uint16_t* brow[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) brow[nb] = xct + (int64_t(b) * cip + ci0 + 16 * nb + li) * row_len + kDecPad + lo_off;
  f32x4 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int m = m_begin; m < m_end; m += 32) {
    const int mm = m + 8 * g;
    const bool ok = mm < m_end;
    uint4 A[2], Bv[4];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) A[mb] = ok ? ld16(arow[mb] + mm) : zero;
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      if (ok) {
        const uint4 lo = ld16(brow[nb] + mm);
        if constexpr (e == 0) {
          Bv[nb] = lo;
        } else {
          Bv[nb] = realign<e>(lo, ld16(brow[nb] + mm + 8));
        }
      } else {
        Bv[nb] = zero;
      }
    }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = mma(A[mb], Bv[nb], acc[mb][nb]);
  }
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        part[(int64_t(KT) * kDecC + 32 * w + 16 * mb + 4 * g + v) * cip + ci0 + 16 * nb + li] = acc[mb][nb][v];
}

template <int S>
__global__ __launch_bounds__(256) void k_conv_wgrad(const uint16_t* __restrict__ dzp, const uint16_t* __restrict__ xct,
                                                    int M, int cip, int chunk, int chunks_per_b,
                                                    float* __restrict__ part) {
  const int b = blockIdx.x / chunks_per_b, mc = blockIdx.x % chunks_per_b;
  const int m_begin = mc * chunk;
  const int m_end = min(M, m_begin + chunk);
  const int ci0 = 64 * blockIdx.y;
  float* p = part + int64_t(blockIdx.x) * kDecK * kDecC * cip;
  switch (blockIdx.z) {
    case 0: wgrad_tap<S, 0>(dzp, xct, M, cip, b, m_begin, m_end, ci0, p); break;
    case 1: wgrad_tap<S, 1>(dzp, xct, M, cip, b, m_begin, m_end, ci0, p); break;
    case 2: wgrad_tap<S, 2>(dzp, xct, M, cip, b, m_begin, m_end, ci0, p); break;
    case 3: wgrad_tap<S, 3>(dzp, xct, M, cip, b, m_begin, m_end, ci0, p); break;
    case 4: wgrad_tap<S, 4>(dzp, xct, M, cip, b, m_begin, m_end, ci0, p); break;
    case 5: wgrad_tap<S, 5>(dzp, xct, M, cip, b, m_begin, m_end, ci0, p); break;
    case 6: wgrad_tap<S, 6>(dzp, xct, M, cip, b, m_begin, m_end, ci0, p); break;
    case 7: wgrad_tap<S, 7>(dzp, xct, M, cip, b, m_begin, m_end, ci0, p); break;
    default: wgrad_tap<S, 8>(dzp, xct, M, cip, b, m_begin, m_end, ci0, p); break;
  }
}

// Weight gradient of every tap of one polyphase row R at once (strides 2 and 4): the taps
// with 4 - KT = S q + R all read dz_P row R and the layer input at a shift of -q samples
// (|q| <= 2). Workgroup: chunk (blockIdx.x), 64 input channels (blockIdx.y), row R
// (blockIdx.z). The dz rows of all 128 output channels, shared by the four waves, go
// through LDS 64 samples at a time (the next 64 are loaded into registers while the
// current ones are used); wave w owns input channels ci0 + [16 w, 16 w + 16) and reads
// three aligned 16-byte pieces of each input row per 32 samples, from which every tap's
// operand is formed by realigning in registers. Partials as for one tap:
// part[chunk][KT][128][cip]. The workgroups of the first channel block also sum the dz
// rows for the bias gradient: bpart[chunk][R][128].
constexpr int kWgTile = 64;                 // samples per LDS stage
constexpr int kWgPitch = kWgTile + 8;       // 144 bytes: rows 16 bytes apart modulo the 128-byte bank cycle
constexpr int kWgPieces = kDecC * kWgTile / 8 / 256;   // 16-byte pieces per thread per stage

template <int S, int R>
__device__ void wgrad_row(const uint16_t* __restrict__ dzp, const uint16_t* __restrict__ xct, int M, int cip, int b,
                          int m_begin, int m_end, int ci0, float* __restrict__ part, float* __restrict__ bpart,
                          uint16_t* __restrict__ atile) {
  const int w = wave_index();
  const int lane = threadIdx.x & 63, g = lane >> 4, li = lane & 15;
  const int64_t row_len = M + 2 * kDecPad;
  const uint4 zero{0u, 0u, 0u, 0u};
  // staging: thread t moves piece (t & 7) of rows (t >> 3) + 32 j
  const int sp = threadIdx.x & 7, sr = threadIdx.x >> 3;
  const uint16_t* srow = dzp + ((int64_t(b) * kDecC + sr) * S + R) * row_len + kDecPad + 8 * sp;
  const int64_t srow_step = int64_t(32) * S * row_len;
  const uint16_t* xrow = xct + (int64_t(b) * cip + ci0 + 16 * w + li) * row_len + kDecPad;
  f32x4 acc[kDecK][8];
#pragma unroll
  for (int kt = 0; kt < kDecK; ++kt)
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[kt][i] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bool with_bias = bpart != nullptr;
  float bsum[kWgPieces];
#pragma unroll
  for (int j = 0; j < kWgPieces; ++j) bsum[j] = 0.f;
  // Loads are unconditional (addresses clamped into the chunk) so that they issue ahead of
  // their use; staged pieces past the chunk's end are then replaced by zeros, which also
  // cancels the clamped input pieces that meet them.
  uint4 P[kWgPieces];
  auto fetch = [&](int m0) {
    const bool in = m0 + 8 * sp < m_end;
    const int off = in ? m0 + 8 * sp : m_begin;
#pragma unroll
    for (int j = 0; j < kWgPieces; ++j) {
      const uint4 v = ld16(srow + j * srow_step + off - 8 * sp);
      P[j] = in ? v : zero;
    }
  };
  uint4 nm, n0, n8;   // input pieces of the next 32 samples
  auto fetch_x = [&](int m) {
    const int mm = min(m + 8 * g, m_end - 8);   // (mm <= M - 8: the pieces at mm - 8 and mm + 8 lie in the padded row)
    nm = ld16(xrow + mm - 8);
    n0 = ld16(xrow + mm);
    n8 = ld16(xrow + mm + 8);
  };
  fetch(m_begin);
  fetch_x(m_begin);
  for (int m0 = m_begin; m0 < m_end; m0 += kWgTile) {
    __syncthreads();   // every wave is done with the previous stage
#pragma unroll
    for (int j = 0; j < kWgPieces; ++j) {
      st16(atile + (sr + 32 * j) * kWgPitch + 8 * sp, P[j]);
      if (with_bias) {
        const uint32_t u[4] = {P[j].x, P[j].y, P[j].z, P[j].w};
#pragma unroll
        for (int i = 0; i < 4; ++i) bsum[j] += __uint_as_float(u[i] << 16) + __uint_as_float(u[i] & 0xffff0000u);
      }
    }
    __syncthreads();
    if (m0 + kWgTile < m_end) fetch(m0 + kWgTile);
#pragma unroll
    for (int step = 0; step < kWgTile / 32; ++step) {
      const uint4 cm = nm, c0 = n0, c8 = n8;
      if (m0 + 32 * step + 32 < m_end) fetch_x(m0 + 32 * step + 32);
      uint4 Bt[kDecK];
#pragma unroll
      for (int kt = 0; kt < kDecK; ++kt) {
        if (((kDecH - kt) % S + S) % S != R) continue;
        switch (-((kDecH - kt - R) / S)) {   // the input is read at m + shift (a compile-time constant)
          case -2: Bt[kt] = realign<6>(cm, c0); break;
          case -1: Bt[kt] = realign<7>(cm, c0); break;
          case 0: Bt[kt] = c0; break;
          case 1: Bt[kt] = realign<1>(c0, c8); break;
          default: Bt[kt] = realign<2>(c0, c8); break;
        }
      }
#pragma unroll
      for (int mb = 0; mb < 8; ++mb) {
        const uint4 A = ld16(atile + (16 * mb + li) * kWgPitch + 32 * step + 8 * g);
#pragma unroll
        for (int kt = 0; kt < kDecK; ++kt) {
          if (((kDecH - kt) % S + S) % S != R) continue;
          acc[kt][mb] = mma(A, Bt[kt], acc[kt][mb]);
        }
      }
    }
  }
#pragma unroll
  for (int kt = 0; kt < kDecK; ++kt) {
    if (((kDecH - kt) % S + S) % S != R) continue;
#pragma unroll
    for (int mb = 0; mb < 8; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        part[(int64_t(kt) * kDecC + 16 * mb + 4 * g + v) * cip + ci0 + 16 * w + li] = acc[kt][mb][v];
  }
  if (with_bias) {
#pragma unroll
    for (int j = 0; j < kWgPieces; ++j) {
      float t = bsum[j];
      t += __shfl_xor(t, 1);   // the eight threads of a row hold its eight pieces
      t += __shfl_xor(t, 2);
      t += __shfl_xor(t, 4);
      if (sp == 0) bpart[(int64_t(blockIdx.x) * S + R) * kDecC + sr + 32 * j] = t;
    }
  }
}

template <int S>
__global__ __launch_bounds__(256, 2) void k_conv_wgrad_rows(const uint16_t* __restrict__ dzp,
                                                            const uint16_t* __restrict__ xct, int M, int cip,
                                                            int chunk, int chunks_per_b, float* __restrict__ part,
                                                            float* __restrict__ bpart) {
  static_assert(S == 2 || S == 4, "shifts of at most two samples");
  static_assert(kWgPieces * 256 * 8 == kDecC * kWgTile, "staging covers the tile");
  const int b = blockIdx.x / chunks_per_b, mc = blockIdx.x % chunks_per_b;
  const int m_begin = mc * chunk;
  const int m_end = min(M, m_begin + chunk);
  const int ci0 = 64 * blockIdx.y;
  float* p = part + int64_t(blockIdx.x) * kDecK * kDecC * cip;
  float* bp = blockIdx.y == 0 ? bpart : nullptr;
  __shared__ uint16_t atile[kDecC * kWgPitch];
  switch (blockIdx.z) {
    case 0: wgrad_row<S, 0>(dzp, xct, M, cip, b, m_begin, m_end, ci0, p, bp, atile); break;
    case 1: wgrad_row<S, 1>(dzp, xct, M, cip, b, m_begin, m_end, ci0, p, bp, atile); break;
    case 2: if constexpr (S > 2) wgrad_row<S, 2>(dzp, xct, M, cip, b, m_begin, m_end, ci0, p, bp, atile); break;
    default: if constexpr (S > 2) wgrad_row<S, 3>(dzp, xct, M, cip, b, m_begin, m_end, ci0, p, bp, atile); break;
  }
}

// grad[(co c_in + ci) 9 + k] = sum over chunks of part[chunk][k][co][ci], fixed order.
__global__ void k_wgrad_reduce(const float* __restrict__ part, int n_chunks, int cip, int c_in,
                               float* __restrict__ grad) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;   // over (k, co, ci < cip)
  const int64_t per = int64_t(kDecK) * kDecC * cip;
  if (i >= per) return;
  const int ci = static_cast<int>(i % cip);
  if (ci >= c_in) return;
  const int co = static_cast<int>((i / cip) % kDecC);
  const int k = static_cast<int>(i / (int64_t(cip) * kDecC));
  float acc = 0.f;
#pragma unroll 8
  for (int c = 0; c < n_chunks; ++c) acc += part[c * per + i];   // (loads issue ahead of the in-order adds)
  grad[(int64_t(co) * c_in + ci) * kDecK + k] = acc;
}

// Sum of each contiguous bf16 row (one block per row, FP64 accumulation in a fixed order).
// A polyphase gradient [B][128][s][8 + M + 8] read as B * 128 rows of s (M + 16) samples
// gives the per-(batch item, channel) bias-gradient partials (the pads are zero).
__global__ __launch_bounds__(256) void k_rowsum_bf16(const uint16_t* __restrict__ x, int64_t row_len,
                                                     float* __restrict__ out) {
  __shared__ double red[256];
  const uint16_t* row = x + int64_t(blockIdx.x) * row_len;
  double acc = 0.0;
  for (int64_t m = threadIdx.x; m < row_len; m += 256) acc += bf2f(row[m]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = static_cast<float>(red[0]);
}

// out[c] = sum_{r < rows} x[r * cols + c] in a fixed order: block (64, 16) owns 64 columns;
// thread (c, j) sums rows j, j + 16, ..., and the 16 slices are added in order.
__global__ __launch_bounds__(1024) void k_colsum(const float* __restrict__ x, int rows, int cols,
                                                 float* __restrict__ out) {
  __shared__ float red[16][64];
  const int c = blockIdx.x * 64 + threadIdx.x;
  float acc = 0.f;
  if (c < cols)
    for (int r = threadIdx.y; r < rows; r += 16) acc += x[int64_t(r) * cols + c];
  red[threadIdx.y][threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.y == 0 && c < cols) {
    float t = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) t += red[j][threadIdx.x];
    out[c] = t;
  }
}

// Sum of each contiguous FP32 row of row_len values (the last row may be shorter).
__global__ __launch_bounds__(256) void k_rowsum_f32(const float* __restrict__ x, int64_t n, int64_t row_len,
                                                    float* __restrict__ out) {
  __shared__ double red[256];
  const int64_t a = int64_t(blockIdx.x) * row_len, b = min(n, a + row_len);
  double acc = 0.0;
  for (int64_t i = a + threadIdx.x; i < b; i += 256) acc += x[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = static_cast<float>(red[0]);
}

// ---------------------------------------------------------------------------------------
// Output layer (one channel, stride 1), FP32 arithmetic on bf16 activations.

// 32 samples x[t0 - 8 .. t0 + 24) of a CT row (padded index t0 .. t0 + 32); the last piece is
// read only when `more` (t0 + 8 < T: the 16 outputs reach past the first 8).
__device__ inline void load32(const uint16_t* row, int t0, bool more, float v[32]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint4 u = (q < 3 || more) ? ld16(row + t0 + 8 * q) : uint4{0u, 0u, 0u, 0u};
    const uint32_t wv[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      v[8 * q + 2 * e] = bf_lo(wv[e]);
      v[8 * q + 2 * e + 1] = bf_hi(wv[e]);
    }
  }
}

__global__ __launch_bounds__(512) void k_out_fwd(const uint16_t* __restrict__ xct, int T, const float* __restrict__ wo,
                                                 const float* __restrict__ bias, float* __restrict__ y) {
  // 64 threads x 16 samples per block; the eight waves take 16 channels each and their sums
  // are combined through LDS in a fixed order
  __shared__ float red[8][64 * 16];
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t0 = 16 * (blockIdx.x * 64 + lane);
  const bool more = t0 + 8 < T;   // (T is a multiple of 8)
  const int64_t row_len = T + 2 * kDecPad;
  float acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  if (t0 < T) {
#pragma unroll 2
    for (int ci = wave * (kDecC / 8); ci < (wave + 1) * (kDecC / 8); ++ci) {
      float v[32];
      load32(xct + (int64_t(b) * kDecC + ci) * row_len, t0, more, v);
#pragma unroll
      for (int k = 0; k < kDecK; ++k) {
        const float wk = wo[ci * kDecK + k];
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] += wk * v[i + k + 4];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) red[wave][i * 64 + lane] = acc[i];
  __syncthreads();
  if (wave == 0 && t0 < T) {
    float* yo = y + int64_t(b) * T + t0;
    const int n = more ? 16 : 8;
    for (int i = 0; i < n; ++i) {
      float t = 0.f;
#pragma unroll
      for (int w = 0; w < 8; ++w) t += red[w][i * 64 + lane];
      yo[i] = bias[0] + t;
    }
  }
}

// dz of the last hidden layer: da[u, ci] = sum_k w[ci][k] dy[u - k + 4], masked.
// Output layer data gradient: dz[u, c] = lrelu'(a[u, c]) * sum_k w[c][k] dy[u - k + 4], written
// TC and in the polyphase layout of the last hidden layer's stride S2. Workgroup: 128 rows
// u of one signal; thread: channels 8 (tid & 15) .. + 8 (their 72 weights in registers) of
// rows (tid >> 4) + 16 j, each row's 8 values packed to bf16 in one 16-byte store.
constexpr int kOutRows = 128;
template <int S2>
__global__ __launch_bounds__(256) void k_out_dgrad(const float* __restrict__ dy, int T, const float* __restrict__ wo,
                                                   const uint16_t* __restrict__ a_tc, float leak,
                                                   uint16_t* __restrict__ dz_tc, uint16_t* __restrict__ dzp) {
  __shared__ uint16_t btile[kOutRows * kRowB];
  __shared__ float dys[kOutRows + 2 * kDecH];
  const int b = blockIdx.y, u0 = blockIdx.x * kOutRows;
  for (int i = threadIdx.x; i < kOutRows + 2 * kDecH; i += 256) {
    const int t = u0 - kDecH + i;
    dys[i] = (t >= 0 && t < T) ? dy[int64_t(b) * T + t] : 0.f;
  }
  const int c8 = (threadIdx.x & 15) * 8;
  float wk[8][kDecK];
#pragma unroll
  for (int e = 0; e < 8; ++e)
#pragma unroll
    for (int k = 0; k < kDecK; ++k) wk[e][k] = wo[(c8 + e) * kDecK + k];
  __syncthreads();
#pragma unroll 2
  for (int row = threadIdx.x >> 4; row < kOutRows; row += 16) {
    const int u = u0 + row;
    if (u >= T) break;
    float d[kDecK];
#pragma unroll
    for (int k = 0; k < kDecK; ++k) d[k] = dys[row - k + 2 * kDecH];
    const int64_t off = (int64_t(b) * T + u) * kDecC + c8;
    const uint4 a = ld16(a_tc + off);
    const uint32_t aw[4] = {a.x, a.y, a.z, a.w};
    uint32_t o[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float d0 = 0.f, d1 = 0.f;
#pragma unroll
      for (int k = 0; k < kDecK; ++k) {
        d0 += wk[2 * e][k] * d[k];
        d1 += wk[2 * e + 1][k] * d[k];
      }
      const float m0 = bf_lo(aw[e]) > 0.f ? d0 : leak * d0;
      const float m1 = bf_hi(aw[e]) > 0.f ? d1 : leak * d1;
      o[e] = uint32_t(f2bf(m0)) | (uint32_t(f2bf(m1)) << 16);
    }
    const uint4 v{o[0], o[1], o[2], o[3]};
    st16(dz_tc + off, v);
    st16(btile + row * kRowB + c8, v);
  }
  __syncthreads();
  store_polyphase<S2, kOutRows>(btile, b, u0, T, dzp);
}

// Partials of dW_out[ci][k] = sum_t dy[t] x[ci][t + k - 4] over 2048-sample chunks.
// Block: chunk blockIdx.x, channels 16 blockIdx.y + (tid >> 4); 16 lanes split the chunk.
__global__ __launch_bounds__(256) void k_out_wgrad(const float* __restrict__ dy, int T, const uint16_t* __restrict__ xct,
                                                   int chunks_per_b, float* __restrict__ part) {
  const int chunk = blockIdx.x;
  const int b = chunk / chunks_per_b, tc = chunk % chunks_per_b;
  const int t_begin = tc * kDecOutChunk, t_end = min(T, t_begin + kDecOutChunk);
  const int ci = 16 * blockIdx.y + (threadIdx.x >> 4), sub = threadIdx.x & 15;
  const int64_t row_len = T + 2 * kDecPad;
  const uint16_t* row = xct + (int64_t(b) * kDecC + ci) * row_len;
  float acc[kDecK];
#pragma unroll
  for (int k = 0; k < kDecK; ++k) acc[k] = 0.f;
  for (int t0 = t_begin + 16 * sub; t0 < t_end; t0 += 256) {
    const bool more = t0 + 8 < t_end;   // (chunk ends are multiples of 8)
    float v[32];
    load32(row, t0, more, v);
    const float* dyp = dy + int64_t(b) * T + t0;
    const float4 d0 = *reinterpret_cast<const float4*>(dyp);
    const float4 d1 = *reinterpret_cast<const float4*>(dyp + 4);
    const float4 d2 = more ? *reinterpret_cast<const float4*>(dyp + 8) : float4{0.f, 0.f, 0.f, 0.f};
    const float4 d3 = more ? *reinterpret_cast<const float4*>(dyp + 12) : float4{0.f, 0.f, 0.f, 0.f};
    const float d[16] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w,
                         d2.x, d2.y, d2.z, d2.w, d3.x, d3.y, d3.z, d3.w};
#pragma unroll
    for (int k = 0; k < kDecK; ++k)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[k] += d[i] * v[i + k + 4];
  }
#pragma unroll
  for (int k = 0; k < kDecK; ++k) {
    float a = acc[k];
    a += __shfl_xor(a, 8, 16);
    a += __shfl_xor(a, 4, 16);
    a += __shfl_xor(a, 2, 16);
    a += __shfl_xor(a, 1, 16);
    acc[k] = a;
  }
  if (sub == 0)
#pragma unroll
    for (int k = 0; k < kDecK; ++k) part[(int64_t(chunk) * kDecC + ci) * kDecK + k] = acc[k];
}

// One block per output weight: the chunk partials are summed by 256 threads (fixed
// strides) and a fixed-order tree.
__global__ __launch_bounds__(256) void k_out_wgrad_reduce(const float* __restrict__ part, int n_chunks,
                                                          float* __restrict__ grad) {
  __shared__ float red[256];
  const int i = blockIdx.x;
  float acc = 0.f;
  for (int c = threadIdx.x; c < n_chunks; c += 256) acc += part[int64_t(c) * kDecC * kDecK + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (static_cast<int>(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad[i] = red[0];
}

// ---------------------------------------------------------------------------------------

__global__ void k_dec_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                           float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float bc1,
                           float bc2) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m[i] + (1.0f - b1) * gi;
  const float c = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = a;
  v[i] = c;
  p[i] -= lr * (a / bc1) / (sqrtf(c / bc2) + eps);
}

__global__ __launch_bounds__(1024) void k_rel_loss(const float* __restrict__ S, const float* __restrict__ T,
                                                   float* __restrict__ dS, float* __restrict__ loss, int64_t n,
                                                   int64_t n0, float w0, int relative, float scale) {
  __shared__ double red[2][1024];
  double e = 0.0, t2 = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const double w = i < n0 ? double(w0) : 1.0;
    const double d = double(S[i]) - double(T[i]);
    e += w * d * d;
    t2 += w * double(T[i]) * double(T[i]);
  }
  red[0][threadIdx.x] = e;
  red[1][threadIdx.x] = t2;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  const double norm = relative ? (red[1][0] > 0.0 ? red[1][0] : 1.0) : 1.0;
  const float f = static_cast<float>(2.0 * scale / norm);
  for (int64_t i = threadIdx.x; i < n; i += 1024) dS[i] = (i < n0 ? w0 : 1.0f) * f * (S[i] - T[i]);
  if (threadIdx.x == 0) loss[0] = static_cast<float>(scale * red[0][0] / norm);
}

inline int blocks_for(int64_t n, int per) { return static_cast<int>((n + per - 1) / per); }

template <int S>
hipError_t launch_fwd(const uint16_t* x_tc, int cip, int t_in, int batch, const uint16_t* wf, const float* bias,
                      float leak, uint16_t* out_tc, uint16_t* out_ct, hipStream_t st) {
  if constexpr (S == 2 || S == 4) {
    if (cip == kDecC) {
      hipLaunchKernelGGL(k_conv_fwd_lds<S>, dim3(blocks_for(t_in, fwd_lds_rows(S)), batch), dim3(256),
                         fwd_lds_bytes(S), st, x_tc, t_in, wf, bias, leak, out_tc, out_ct);
      return hipGetLastError();
    }
  }
  const size_t lds = size_t(kDecTile) * S * fwd_pitch(S) * sizeof(uint16_t);
  hipLaunchKernelGGL(k_conv_fwd<S>, dim3(blocks_for(t_in, kDecTile), batch), dim3(256), lds, st, x_tc, cip, t_in, wf,
                     bias, leak, out_tc, out_ct);
  return hipGetLastError();
}


template <int S, int S2>
hipError_t launch_dgrad(const uint16_t* dz, int t_out, const uint16_t* wd, int t_in, int batch, const uint16_t* a_prev,
                        float leak, uint16_t* dz_prev, uint16_t* dzp_prev, hipStream_t st) {
  hipLaunchKernelGGL((k_conv_dgrad_lds<S, S2>), dim3(blocks_for(t_in, kDgradRows), batch), dim3(256), kDgradLdsBig,
                     st, dz, t_out, wd, t_in, a_prev, leak, dz_prev, dzp_prev);
  return hipGetLastError();
}

template <int S>
hipError_t launch_dgrad_s(int s2, const uint16_t* dz, int t_out, const uint16_t* wd, int t_in, int batch,
                          const uint16_t* a_prev, float leak, uint16_t* dz_prev, uint16_t* dzp_prev, hipStream_t st) {
  switch (s2) {
    case 1: return launch_dgrad<S, 1>(dz, t_out, wd, t_in, batch, a_prev, leak, dz_prev, dzp_prev, st);
    case 2: return launch_dgrad<S, 2>(dz, t_out, wd, t_in, batch, a_prev, leak, dz_prev, dzp_prev, st);
    case 4: return launch_dgrad<S, 4>(dz, t_out, wd, t_in, batch, a_prev, leak, dz_prev, dzp_prev, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t run_dec_cast(const float* W, int c_in, int cip, int c_out, uint16_t* wf, uint16_t* wd, float* wout,
                        hipStream_t st) {
  if (wout) {
    const int n = c_out * c_in * kDecK;
    hipLaunchKernelGGL(k_cast_out, dim3(blocks_for(n, 256)), dim3(256), 0, st, W, n, wout);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_cast_wf, dim3(blocks_for(int64_t(c_out) * kDecK * cip, 256)), dim3(256), 0, st, W, c_in, cip,
                     c_out, wf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !wd) return e;
  hipLaunchKernelGGL(k_cast_wd, dim3(blocks_for(int64_t(c_in) * kDecK * c_out, 256)), dim3(256), 0, st, W, c_in, c_out,
                     wd);
  return hipGetLastError();
}

hipError_t run_dec_cast_all(const DecCastSet& set, hipStream_t st) {
  if (set.n < 1 || set.n > kDecMaxLayers) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cast_all, dim3(blocks_for(set.end[set.n - 1], 256)), dim3(256), 0, st, set);
  return hipGetLastError();
}

hipError_t run_dec_input(const float* S, int batch, int c_in, int F, int cip, float eps, uint16_t* x_tc,
                         uint16_t* x_ct, hipStream_t st) {
  hipLaunchKernelGGL(k_dec_input, dim3(blocks_for(int64_t(F) * cip, 256), batch), dim3(256), 0, st, S, c_in, F, cip,
                     eps, x_tc, x_ct);
  return hipGetLastError();
}

hipError_t run_dec_conv_fwd(int s, const uint16_t* x_tc, int cip, int t_in, int batch, const uint16_t* wf,
                            const float* bias, float leak, uint16_t* out_tc, uint16_t* out_ct, hipStream_t st) {
  switch (s) {
    case 1: return launch_fwd<1>(x_tc, cip, t_in, batch, wf, bias, leak, out_tc, out_ct, st);
    case 2: return launch_fwd<2>(x_tc, cip, t_in, batch, wf, bias, leak, out_tc, out_ct, st);
    case 4: return launch_fwd<4>(x_tc, cip, t_in, batch, wf, bias, leak, out_tc, out_ct, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t run_dec_out_fwd(const uint16_t* x_ct, int T, int batch, const float* wout, const float* bias, float* y,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_out_fwd, dim3(blocks_for(T, 1024), batch), dim3(512), 0, st, x_ct, T, wout, bias, y);
  return hipGetLastError();
}

hipError_t run_dec_out_bwd(const float* dy, int T, int batch, const float* wout, const uint16_t* a_tc,
                           const uint16_t* a_ct, float leak, int s2, uint16_t* dz_tc, uint16_t* dzp, float* part,
                           float* grad_w, float* grad_b, hipStream_t st) {
  const dim3 grid(blocks_for(T, kOutRows), batch);
  switch (s2) {
    case 1: hipLaunchKernelGGL(k_out_dgrad<1>, grid, dim3(256), 0, st, dy, T, wout, a_tc, leak, dz_tc, dzp); break;
    case 2: hipLaunchKernelGGL(k_out_dgrad<2>, grid, dim3(256), 0, st, dy, T, wout, a_tc, leak, dz_tc, dzp); break;
    case 4: hipLaunchKernelGGL(k_out_dgrad<4>, grid, dim3(256), 0, st, dy, T, wout, a_tc, leak, dz_tc, dzp); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int cpb = blocks_for(T, kDecOutChunk);
  const int n_chunks = cpb * batch;
  hipLaunchKernelGGL(k_out_wgrad, dim3(n_chunks, kDecC / 16), dim3(256), 0, st, dy, T, a_ct, cpb, part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_out_wgrad_reduce, dim3(kDecC * kDecK), dim3(256), 0, st, part, n_chunks, grad_w);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // output bias: partial sums over 8192-sample rows of dy, then their sum (partials after the
  // weight partials in `part`)
  const int64_t n = int64_t(batch) * T;
  const int nrow = static_cast<int>((n + 8191) / 8192);
  float* bpart = part + int64_t(n_chunks) * kDecC * kDecK;
  hipLaunchKernelGGL(k_rowsum_f32, dim3(nrow), dim3(256), 0, st, dy, n, int64_t(8192), bpart);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(64, 16), 0, st, bpart, nrow, 1, grad_b);
  return hipGetLastError();
}

hipError_t run_dec_dgrad(int s, int s2, const uint16_t* dz_tc, int t_out, const uint16_t* wd, int t_in, int batch,
                         const uint16_t* a_prev_tc, float leak, uint16_t* dz_prev_tc, uint16_t* dzp_prev,
                         hipStream_t st) {
  switch (s) {
    case 1: return launch_dgrad_s<1>(s2, dz_tc, t_out, wd, t_in, batch, a_prev_tc, leak, dz_prev_tc, dzp_prev, st);
    case 2: return launch_dgrad_s<2>(s2, dz_tc, t_out, wd, t_in, batch, a_prev_tc, leak, dz_prev_tc, dzp_prev, st);
    case 4: return launch_dgrad_s<4>(s2, dz_tc, t_out, wd, t_in, batch, a_prev_tc, leak, dz_prev_tc, dzp_prev, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t run_dec_wgrad(int s, const uint16_t* dzp, const uint16_t* x_ct, int t_in, int cip, int c_in, int batch,
                         float* part, float* grad_w, float* grad_b, hipStream_t st) {
  const int chunk = dec_wgrad_chunk(batch, t_in, cip, s);
  const int cpb = blocks_for(t_in, chunk);
  const int n_chunks = cpb * batch;
  // bias partials follow the weight partials in `part`: [chunk][row][128] from the stride-2/4
  // kernels, [batch item][128] row sums at stride 1
  float* bpart = part + int64_t(n_chunks) * kDecK * kDecC * cip;
  switch (s) {
    case 1:
      hipLaunchKernelGGL(k_conv_wgrad<1>, dim3(n_chunks, cip / 64, kDecK), dim3(256), 0, st, dzp, x_ct, t_in, cip,
                         chunk, cpb, part);
      break;
    case 2:
      hipLaunchKernelGGL(k_conv_wgrad_rows<2>, dim3(n_chunks, cip / 64, 2), dim3(256), 0, st, dzp, x_ct, t_in, cip,
                         chunk, cpb, part, bpart);
      break;
    case 4:
      hipLaunchKernelGGL(k_conv_wgrad_rows<4>, dim3(n_chunks, cip / 64, 4), dim3(256), 0, st, dzp, x_ct, t_in, cip,
                         chunk, cpb, part, bpart);
      break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(blocks_for(int64_t(kDecK) * kDecC * cip, 256)), dim3(256), 0, st, part,
                     n_chunks, cip, c_in, grad_w);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int brows = n_chunks * s;
  if (s == 1) {
    hipLaunchKernelGGL(k_rowsum_bf16, dim3(batch * kDecC), dim3(256), 0, st, dzp, int64_t(t_in + 2 * kDecPad), bpart);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    brows = batch;
  }
  hipLaunchKernelGGL(k_colsum, dim3(kDecC / 64), dim3(64, 16), 0, st, bpart, brows, kDecC, grad_b);
  return hipGetLastError();
}

hipError_t run_dec_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                        float eps, float bc1, float bc2, hipStream_t st) {
  hipLaunchKernelGGL(k_dec_adam, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, g, m, v, n, lr, beta1, beta2, eps, bc1,
                     bc2);
  return hipGetLastError();
}

hipError_t run_rel_loss(const float* S, const float* T, float* dS, float* loss, int64_t n, int64_t n0, float w0,
                        int relative, float scale, hipStream_t st) {
  hipLaunchKernelGGL(k_rel_loss, dim3(1), dim3(1024), 0, st, S, T, dS, loss, n, n0, w0, relative, scale);
  return hipGetLastError();
}

}  // namespace jtfs
