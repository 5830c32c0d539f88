// Time-axis stages of JTFS and their adjoints: batched FFTs with fused Fourier-domain
// filtering, Fourier subsampling, modulus and phase (Sec. 3.2-3.3, Eqs. 5-7).
//
// Every stage is a batch of independent rows (RowJob); a row's transform has length n.
// Rows with n <= 4096 run in one kernel (the whole row in a 4096-element LDS tile);
// longer rows run as two kernels (fft_core.hpp's split) through a scratch buffer.
// A stage supplies load(idx) producing transform input idx, and store(idx, v)
// consuming transform output idx (already scaled by 1/n for inverse transforms).
//
// Stage meanings (RowJob fields in brackets):
//  XHAT  X = DFT(x zero-padded to N_pad)                               [dst: Xh]
//  L1Z   Z1 = IDFT_L1(fold_k1(X . psi1))        (Sec. 3.2)           [band psi1, shift k1, dst: Z1 row]
//  L1UH  U1hat = DFT(|Z1|)                       (Sec. 3.2)           [src/dst: row offset]
//  L2Y   Y2 = IDFT_L2(fold_k2(U1hat . psi2^(k1)))  (Sec. 3.3)         [src: U1hat row, band, shift k2]
//  BYH   dY2hat = DFT(dY2) (row-split partials already summed in split 0)  [src: dY2 row]
//  BU    dU1 = Re IDFT_L1(sum_terms band . tile(term source))        [segments from t0]
//  BZH   dZ1hat = DFT(dU1 . Z1 / |Z1|)  (0 where Z1 = 0)              [src: dU1, aux: Z1]
//  BX    dx = unpad Re IDFT_Npad(sum_n1 psi1 . tile(dZ1hat))          [segments from t0]
// fold_k averages the 2^k aliased blocks of a spectrum; tile is its transpose up to
// 2^-k; with both, a filter-and-subsample step and its adjoint are exact.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace jtfs {
namespace {

__device__ __forceinline__ float cabs(c32 z) { return sqrtf(z.x * z.x + z.y * z.y); }

// Fourier subsampling by 2^shift of (src . band) onto an n-point grid, output bin q.
// The plan guarantees that a band is not empty and spans at most two aliased blocks
// (1 <= len <= 2 n). A band of at most n bins meets bin q in one block only, and a row's
// band is the same for all its bins (a uniform branch); otherwise both blocks are read at
// indices clamped into the band, an absent second term masked by value, so the loads of
// several bins can be in flight together.
__device__ __forceinline__ c32 fold_gather(const c32* src, const Band& b, const float* vals, int n, int shift, int q) {
  const int nmask = n - 1;
  const int d0 = (q - (b.lo & nmask)) & nmask;
  c32 acc{0.f, 0.f};
  const int nk = b.len > n ? 2 : 1;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (k < nk) {
      const int d = d0 + k * n;
      const bool in = d < b.len;
      const int dc = in ? d : 0;
      int m = b.lo + dc;
      if (m >= b.L) m -= b.L;
      const float h = vals[b.off + dc];
      const c32 v = src[m];
      const float hm = in ? h : 0.f;
      acc.x += v.x * hm;
      acc.y += v.y * hm;
    }
  }
  const float sc = ldexpf(1.0f, -shift);
  return c32{acc.x * sc, acc.y * sc};
}

template <int ST>
struct Ops;

// Each stage's Ops: transform direction DIR, the element load and store, and LB, how
// many element loads a thread keeps in flight before storing them to LDS (16: all of
// them; fewer where one element is itself a gather of several loads, to bound registers).
template <>
struct Ops<ST_XHAT> {
  static constexpr int DIR = -1, LB = 16;
  __device__ __forceinline__ static c32 load(const DevSig& s, const RowJob&, const Band&, int idx) {
    const int j = idx - s.pad_left;
    return c32{(j >= 0 && j < s.N) ? s.x[j] : 0.f, 0.f};
  }
  __device__ __forceinline__ static void store(const DevSig& s, const RowJob&, int idx, c32 v) { s.Xh[idx] = v; }
};

template <>
struct Ops<ST_L1Z> {
  static constexpr int DIR = +1, LB = 8;
  __device__ __forceinline__ static c32 load(const DevSig& s, const RowJob& j, const Band& b, int idx) {
    return fold_gather(s.Xh, b, s.bandvals, j.n, j.shift, idx);
  }
  __device__ __forceinline__ static void store(const DevSig& s, const RowJob& j, int idx, c32 v) { s.Z1[j.dst + idx] = v; }
};

template <>
struct Ops<ST_L1UH> {
  static constexpr int DIR = -1, LB = 16;
  __device__ __forceinline__ static c32 load(const DevSig& s, const RowJob& j, const Band&, int idx) {
    return c32{cabs(s.Z1[j.src + idx]), 0.f};
  }
  __device__ __forceinline__ static void store(const DevSig& s, const RowJob& j, int idx, c32 v) { s.U1h[j.dst + idx] = v; }
};

template <>
struct Ops<ST_L2Y> {
  static constexpr int DIR = +1, LB = 8;
  __device__ __forceinline__ static c32 load(const DevSig& s, const RowJob& j, const Band& b, int idx) {
    return fold_gather(s.U1h + j.src, b, s.bandvals, j.n, j.shift, idx);
  }
  __device__ __forceinline__ static void store(const DevSig& s, const RowJob& j, int idx, c32 v) { s.Y2[j.dst + idx] = v; }
};

template <>
struct Ops<ST_BYH> {
  static constexpr int DIR = -1, LB = 16;
  __device__ __forceinline__ static c32 load(const DevSig& s, const RowJob& j, const Band&, int idx) { return s.dYpart[j.src + idx]; }
  __device__ __forceinline__ static void store(const DevSig& s, const RowJob& j, int idx, c32 v) { s.dYh[j.dst + idx] = v; }
};

template <>
struct Ops<ST_BU> {
  static constexpr int DIR = +1, LB = 16;
  // the gather itself runs beforehand in k_seg_gather, into the row's slot of dZh
  __device__ __forceinline__ static c32 load(const DevSig& s, const RowJob& j, const Band&, int idx) {
    return s.dZh[j.dst + idx];
  }
  __device__ __forceinline__ static void store(const DevSig& s, const RowJob& j, int idx, c32 v) { s.dU1[j.dst + idx] = v.x; }
};

template <>
struct Ops<ST_BZH> {
  static constexpr int DIR = -1, LB = 16;
  __device__ __forceinline__ static c32 load(const DevSig& s, const RowJob& j, const Band&, int idx) {
    // u times the phase z / |z| (rsq, within 1 ulp; subgradient 0 where |z| vanishes,
    // below 1.1e-19 the square underflows anyway)
    const float u = s.dU1[j.src + idx];
    const c32 z = s.Z1[j.aux + idx];
    const float m2 = z.x * z.x + z.y * z.y;
    const float r = m2 >= 1.17549435e-38f ? u * __builtin_amdgcn_rsqf(m2) : 0.f;
    return c32{z.x * r, z.y * r};
  }
  __device__ __forceinline__ static void store(const DevSig& s, const RowJob& j, int idx, c32 v) { s.dZh[j.dst + idx] = v; }
};

template <>
struct Ops<ST_BX> {
  static constexpr int DIR = +1, LB = 16;
  // the gather itself runs beforehand in k_seg_gather, over the whole spectrum at once
  __device__ __forceinline__ static c32 load(const DevSig& s, const RowJob&, const Band&, int idx) { return s.dXh[idx]; }
  // (U0 = x as zeroth order adds its gradient directly)
  __device__ __forceinline__ static void store(const DevSig& s, const RowJob&, int idx, c32 v) {
    const int k = idx - s.pad_left;
    if (k >= 0 && k < s.N) s.dx[k] = v.x + ((s.u0 && s.dS != nullptr) ? s.dS[s.s0_off + k] : 0.f);
  }
};

// Bin-parallel adjoint gathers, run before the stage's inverse transforms:
//  BU: dU1hat_n1[m] = sum_n2 psi2_n2^(k1)[m] dY2hat_(n1,n2)[m mod L2] (+ the phi_T term),
//      into the row's slot in dZh (free until stage BZH writes it);
//  BX: dXhat[m] = sum_n1 psi1_n1[m] dZ1hat_n1[m mod L1_n1].
// One thread per output bin, one chunk of up to 256 bins of one row per workgroup (the
// plan's chunk list). A wave's 64 bins lie in one 512-bin segment, so its term records
// come by scalar loads. Terms go in batches of eight: the batch's records, then its
// sixteen element loads, then the sums (a band that misses the bin is read at a clamped
// index and masked by value: no branch).
template <int ST>
__global__ __launch_bounds__(256) void k_seg_gather(DevSig s, int ch0) {
  const int c = ch0 + blockIdx.x;
  const int job = s.gchunks[2 * c];
  const int m = s.gchunks[2 * c + 1] + threadIdx.x;
  const RowJob j = s.jobs[job];
  if (m >= j.n) return;
  const c32* base = ST == ST_BU ? s.dYh : s.dZh;
  c32 acc{0.f, 0.f};
  const int sg = __builtin_amdgcn_readfirstlane(j.t0 + (m >> 9));
  const int first = s.segs[2 * sg], count = s.segs[2 * sg + 1];
  for (int i0 = 0; i0 < count; i0 += 8) {
    SegTerm g[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) g[k] = s.segterms[first + min(i0 + k, count - 1)];
    float h[8];
    c32 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      int d = m - g[k].lo;
      if (d < 0) d += g[k].L;
      const bool in = d < g[k].len && i0 + k < count;
      const float hv = s.bandvals[g[k].off + (in ? d : 0)];
      h[k] = in ? hv : 0.f;
      v[k] = base[g[k].src + (m & (g[k].src_len - 1))];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      acc.x += v[k].x * h[k];
      acc.y += v[k].y * h[k];
    }
  }
  if constexpr (ST == ST_BU)
    s.dZh[j.dst + m] = acc;
  else
    s.dXh[m] = acc;
}

// Twiddle powers of every pass of a 2^LOG2N-point tile transform for this thread (pass
// PI has span 2^(4 PI) and radix min(16, 2^(LOG2N - 4 PI)); pass 0 needs none), read
// before the data so that their latency overlaps the element loads.
template <int LOG2N>
struct TileTw {
  static constexpr int NP = (LOG2N + 3) / 4;
  c32 w[NP][8];
};

template <int DIR, int LOG2N, int PI>
__device__ __forceinline__ void tile_twiddles_rec(TileTw<LOG2N>& f, int t, const c32* tw, int log2tw) {
  if constexpr (PI < TileTw<LOG2N>::NP) {
    constexpr int LOG2P = 4 * PI;
    constexpr int LR = (LOG2N - LOG2P) >= 4 ? 4 : (LOG2N - LOG2P);
    if constexpr (PI > 0) stockham_twiddles<DIR, LR>(LOG2N, LOG2P, t, (1 << LOG2N) >> 4, tw, log2tw, f.w[PI]);
    tile_twiddles_rec<DIR, LOG2N, PI + 1>(f, t, tw, log2tw);
  }
}

template <int DIR, int LOG2N>
__device__ __forceinline__ TileTw<LOG2N> tile_twiddles(const c32* tw, int log2tw) {
  TileTw<LOG2N> f;
  tile_twiddles_rec<DIR, LOG2N, 0>(f, threadIdx.x & ((1 << (LOG2N - 4)) - 1), tw, log2tw);
  return f;
}

// Pass PI over the tile (two barriers: all reads before any write). The length and span
// are compile-time constants, so every index folds to a constant offset from the
// thread's base slot.
template <int DIR, int LOG2N, int PI>
__device__ __forceinline__ void tile_passes_ct(c32* tile, int cbase, int t, const TileTw<LOG2N>& f) {
  if constexpr (PI < TileTw<LOG2N>::NP) {
    constexpr int LOG2P = 4 * PI;
    constexpr int LR = (LOG2N - LOG2P) >= 4 ? 4 : (LOG2N - LOG2P);
    constexpr int TPF = (1 << LOG2N) >> 4;
    c32 v[16];
    stockham_compute_tw<DIR, LR>(tile, cbase, LOG2N, LOG2P, t, TPF, f.w[PI], v);
    __syncthreads();
    stockham_store<LR>(tile, cbase, LOG2P, t, TPF, v);
    __syncthreads();
    tile_passes_ct<DIR, LOG2N, PI + 1>(tile, cbase, t, f);
  }
}

// In-place FFT of the 4096 / 2^LOG2N columns of the tile (natural order in and out;
// element e at LDS slot tile_slot(e)); the caller has synchronised after its writes.
template <int DIR, int LOG2N>
__device__ __forceinline__ void fft_tile_ct(c32* lds, const TileTw<LOG2N>& f) {
  const int t = threadIdx.x & ((1 << (LOG2N - 4)) - 1);
  const int cbase = (threadIdx.x >> (LOG2N - 4)) << LOG2N;
  tile_passes_ct<DIR, LOG2N, 0>(lds, cbase, t, f);
}

// Row of tile element e for rows of 2^LOG2N points. From 64 points on, the 64 lanes of
// a wave lie in one row (e = threadIdx.x + 256 i), so the row is wave-uniform and its job
// and band records come through scalar loads.
template <int LOG2N>
__device__ __forceinline__ int tile_row(int e) {
  const int row = e >> LOG2N;
  if constexpr (LOG2N >= 6) return __builtin_amdgcn_readfirstlane(row);
  return row;
}

// The job's band travels inside the job record (zeros for a row without one).
template <int ST>
__device__ __forceinline__ Band job_band(const DevSig&, const RowJob& j) {
  return j.b;
}

// Single-pass task: `count` rows of 2^LOG2N points in one tile. All sixteen element loads
// of a thread are issued before any is stored to LDS, and all sixteen results are read
// from LDS before the first store to global memory.
template <int ST, int LOG2N>
__device__ __forceinline__ void rows_body_ct(const DevSig& s, c32* lds, const RowTask& tk) {
  using O = Ops<ST>;
  constexpr int N = 1 << LOG2N;
  const int count = tk.count;
  const TileTw<LOG2N> twp = tile_twiddles<O::DIR, LOG2N>(s.tw, s.log2_Npad);
  // rows under 64 points: each lane reads its own job record, so fewer loads in flight
  constexpr int LB = LOG2N >= 6 ? O::LB : (O::LB < 4 ? O::LB : 4);
#pragma unroll
  for (int i0 = 0; i0 < 16; i0 += LB) {
    c32 vb[LB];
#pragma unroll
    for (int b = 0; b < LB; ++b) {
      // (elements past the last row load from it and are zeroed by value)
      const int e = threadIdx.x + 256 * (i0 + b);
      const int row = tile_row<LOG2N>(e);
      const int rc = min(row, count - 1);
      const RowJob j = s.jobs[tk.job0 + rc];
      const c32 x = O::load(s, j, job_band<ST>(s, j), e & (N - 1));
      vb[b] = row < count ? x : c32{0.f, 0.f};
    }
#pragma unroll
    for (int b = 0; b < LB; ++b) lds[tile_slot(threadIdx.x + 256 * (i0 + b))] = vb[b];
  }
  __syncthreads();
  c32 v[16];
  fft_tile_ct<O::DIR, LOG2N>(lds, twp);
  const float sc = O::DIR > 0 ? 1.0f / N : 1.0f;
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = lds[tile_slot(threadIdx.x + 256 * i)];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int e = threadIdx.x + 256 * i;
    const int row = tile_row<LOG2N>(e);
    if (row < count) O::store(s, s.jobs[tk.job0 + row], e & (N - 1), cscale(v[i], sc));
  }
}

template <int ST>
__device__ __forceinline__ void rows_body(const DevSig& s, c32* lds, int task) {
  const RowTask tk = s.tasks[task];
  switch (tk.log2n) {
    case 4: rows_body_ct<ST, 4>(s, lds, tk); break;
    case 5: rows_body_ct<ST, 5>(s, lds, tk); break;
    case 6: rows_body_ct<ST, 6>(s, lds, tk); break;
    case 7: rows_body_ct<ST, 7>(s, lds, tk); break;
    case 8: rows_body_ct<ST, 8>(s, lds, tk); break;
    case 9: rows_body_ct<ST, 9>(s, lds, tk); break;
    case 10: rows_body_ct<ST, 10>(s, lds, tk); break;
    case 11: rows_body_ct<ST, 11>(s, lds, tk); break;
    default: rows_body_ct<ST, 12>(s, lds, tk); break;
  }
}

// Pass 1 of a two-pass row (n = A B, B = 2^LOG2B): C1 = 4096 / B consecutive columns n1,
// each a B-point transform over n2, twiddled by w_n^(n1 k2) and written to scratch.
template <int ST, int LOG2B>
__device__ __forceinline__ void split1_ct(const DevSig& s, c32* lds, const SplitTask& tk) {
  using O = Ops<ST>;
  const SplitGeom g = split_geom(LOG2B + tk.log2A, tk.log2A);
  const RowJob& job = tk.j;
  const Band band = job_band<ST>(s, job);
  const int n1_0 = tk.blk << g.log2C1;
  const TileTw<LOG2B> twp = tile_twiddles<O::DIR, LOG2B>(s.tw, s.log2_Npad);
  c32 b5[5];
  split_p1_twiddle_bases<O::DIR>(g, n1_0, threadIdx.x, s.tw, s.log2_Npad - g.log2n, b5);
  constexpr int LB = O::LB;
#pragma unroll
  for (int i0 = 0; i0 < 16; i0 += LB) {
    c32 vb[LB];
#pragma unroll
    for (int b = 0; b < LB; ++b) {
      int idx, slot;
      split_p1_load(g, n1_0, threadIdx.x + 256 * (i0 + b), idx, slot);
      vb[b] = O::load(s, job, band, idx);
    }
#pragma unroll
    for (int b = 0; b < LB; ++b) {
      int idx, slot;
      split_p1_load(g, n1_0, threadIdx.x + 256 * (i0 + b), idx, slot);
      lds[tile_slot(slot)] = vb[b];
    }
  }
  __syncthreads();
  c32 v[16];
  fft_tile_ct<O::DIR, LOG2B>(lds, twp);
  c32* scr = s.scr + tk.scr;
  c32 w16[16];
  split_p1_twiddle_expand(b5, w16);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    int slot, sidx, te;
    split_p1_store(g, n1_0, threadIdx.x + 256 * i, slot, sidx, te);
    v[i] = cmul(lds[tile_slot(slot)], w16[i]);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    int slot, sidx, te;
    split_p1_store(g, n1_0, threadIdx.x + 256 * i, slot, sidx, te);
    scr[sidx] = v[i];
  }
}

template <int ST>
__device__ __forceinline__ void split1_body(const DevSig& s, c32* lds, int task) {
  const SplitTask tk = s.stasks[task];
  switch (tk.log2n - tk.log2A) {
    case 4: split1_ct<ST, 4>(s, lds, tk); break;
    case 5: split1_ct<ST, 5>(s, lds, tk); break;
    case 6: split1_ct<ST, 6>(s, lds, tk); break;
    case 7: split1_ct<ST, 7>(s, lds, tk); break;
    case 8: split1_ct<ST, 8>(s, lds, tk); break;
    case 9: split1_ct<ST, 9>(s, lds, tk); break;
    case 10: split1_ct<ST, 10>(s, lds, tk); break;
    case 11: split1_ct<ST, 11>(s, lds, tk); break;
    default: split1_ct<ST, 12>(s, lds, tk); break;
  }
}

// First launch of a stage: the short-row tasks (whole rows in one tile), then pass 1 of
// every long row; the two sets are independent, so they share one launch. Three waves per
// SIMD, except for stage BZH, whose two loads per element would spill registers under
// that bound (a kernel with scratch also pays for its set-up at every launch).
template <int ST>
__global__ __launch_bounds__(256, ST == ST_BZH ? 2 : 3) void k_fft_stage1(DevSig s, int task0, int ntask, int split0) {
  __shared__ c32 lds[4096];
  if (static_cast<int>(blockIdx.x) < ntask)
    rows_body<ST>(s, lds, task0 + blockIdx.x);
  else
    split1_body<ST>(s, lds, split0 + blockIdx.x - ntask);
}

// Pass 2 of a two-pass row (A = 2^LOG2A): C2 = 4096 / A consecutive scratch rows k2, each
// an A-point transform over n1, giving X[k2 + B k1].
template <int ST, int LOG2A>
__device__ __forceinline__ void split2_ct(const DevSig& s, c32* lds, const SplitTask& tk) {
  using O = Ops<ST>;
  const SplitGeom g = split_geom(tk.log2n, LOG2A);
  const RowJob& job = tk.j;
  const int k2_0 = tk.blk << g.log2C2;
  const c32* scr = s.scr + tk.scr;
  const TileTw<LOG2A> twp = tile_twiddles<O::DIR, LOG2A>(s.tw, s.log2_Npad);
  c32 v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = scr[split_p2_load(g, k2_0, threadIdx.x + 256 * i)];
#pragma unroll
  for (int i = 0; i < 16; ++i) lds[tile_slot(threadIdx.x + 256 * i)] = v[i];
  __syncthreads();
  fft_tile_ct<O::DIR, LOG2A>(lds, twp);
  const float sc = O::DIR > 0 ? 1.0f / static_cast<float>(1 << g.log2n) : 1.0f;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    int slot, oidx;
    split_p2_store(g, k2_0, threadIdx.x + 256 * i, slot, oidx);
    v[i] = lds[tile_slot(slot)];
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    int slot, oidx;
    split_p2_store(g, k2_0, threadIdx.x + 256 * i, slot, oidx);
    O::store(s, job, oidx, cscale(v[i], sc));
  }
}

template <int ST>
__global__ __launch_bounds__(256) void k_fft_split2(DevSig s, int task0) {
  __shared__ c32 lds[4096];
  const SplitTask tk = s.stasks[task0 + blockIdx.x];
  switch (tk.log2A) {
    case 4: split2_ct<ST, 4>(s, lds, tk); break;
    case 5: split2_ct<ST, 5>(s, lds, tk); break;
    case 6: split2_ct<ST, 6>(s, lds, tk); break;
    case 7: split2_ct<ST, 7>(s, lds, tk); break;
    case 8: split2_ct<ST, 8>(s, lds, tk); break;
    case 9: split2_ct<ST, 9>(s, lds, tk); break;
    case 10: split2_ct<ST, 10>(s, lds, tk); break;
    case 11: split2_ct<ST, 11>(s, lds, tk); break;
    default: split2_ct<ST, 12>(s, lds, tk); break;
  }
}

// The Lf twiddles exp(-2 pi i q / Lf), q < Lf <= 1024, into LDS (the direct DFTs below
// read each of them Lf times).
__device__ __forceinline__ void stage_twiddles(const DevSig& s, c32* Tw, int Lf, int log2Lf) {
  const int tshift = s.log2_Npad - log2Lf;
  for (int q = threadIdx.x; q < Lf; q += 256) Tw[q] = s.tw[q << tshift];
}

// First-order averaging (Eq. 3 before phi_F): S1 = Re IDFT_Lf(fold(U1hat . phi_T^(k1))),
// one workgroup per first-order row; the Lf-point inverse DFT is computed directly.
__global__ __launch_bounds__(256) void k_s1(DevSig s, int job0) {
  __shared__ c32 F[1024];
  __shared__ c32 Tw[1024];
  const RowJob j = s.jobs[job0 + blockIdx.x];
  const int Lf = j.n;
  const int log2Lf = 31 - __clz(Lf);
  const Band b = j.b;
  for (int q = threadIdx.x; q < Lf; q += 256) F[q] = fold_gather(s.U1h + j.src, b, s.bandvals, Lf, j.shift, q);
  stage_twiddles(s, Tw, Lf, log2Lf);
  __syncthreads();
  for (int f = threadIdx.x; f < Lf; f += 256) {
    float acc = 0.f;
    for (int q = 0; q < Lf; ++q) {
      const c32 w = Tw[(q * f) & (Lf - 1)];   // exp(-2 pi i q f / Lf)
      acc += F[q].x * w.x + F[q].y * w.y;     // Re(F exp(+2 pi i q f / Lf))
    }
    s.S1[j.dst + f] = acc / Lf;
  }
}

// Zeroth order (Sec. 3.6 main algorithm): S0 = Re IDFT_Lf(fold(Xhat . phi_T)) at the kept
// frames, one workgroup; the Lf-point inverse DFT is computed directly.
__global__ __launch_bounds__(256) void k_s0(DevSig s) {
  __shared__ c32 F[1024];
  __shared__ c32 Tw[1024];
  const int Lf = s.Lf;
  const int log2Lf = 31 - __clz(Lf);
  const Band b = s.bands[s.s0_band];
  for (int q = threadIdx.x; q < Lf; q += 256) F[q] = fold_gather(s.Xh, b, s.bandvals, Lf, s.log2T, q);
  stage_twiddles(s, Tw, Lf, log2Lf);
  __syncthreads();
  for (int i = threadIdx.x; i < s.nF; i += 256) {
    const int f = s.f_lo + i;
    float acc = 0.f;
    for (int q = 0; q < Lf; ++q) {
      const c32 w = Tw[(q * f) & (Lf - 1)];   // exp(-2 pi i q f / Lf)
      acc += F[q].x * w.x + F[q].y * w.y;     // Re(F exp(+2 pi i q f / Lf))
    }
    s.S[s.s0_off + i] = acc / Lf;
  }
}

// Adjoint of the first-order averaging onto the spectrum: for each first-order row,
// dS1hat = DFT_Lf(sum over the real frequential filters of their dS1 contributions).
// Block N1 (zeroth order present): the DFT of the padded dS0 row, after the dZ1hat rows
// (the signal-spectrum gather of stage BX reads it with phi_T).
__global__ __launch_bounds__(256) void k_ds1h(DevSig s) {
  __shared__ float d[1024];
  __shared__ c32 Tw[1024];
  const int n1 = blockIdx.x;
  const int Lf = s.nf_pad;
  const int log2Lf = 31 - __clz(Lf);
  const bool zeroth = n1 == s.N1;
  for (int f = threadIdx.x; f < Lf; f += 256) {
    float acc = 0.f;
    if (zeroth) {
      const int i = f - s.f_lo;
      acc = (i >= 0 && i < s.nF) ? s.dS[s.s0_off + i] : 0.f;
    } else {
      for (int g = 0; g < s.n_real; ++g) acc += s.dS1p[(static_cast<int64_t>(g) * s.N1 + n1) * Lf + f];
    }
    d[f] = acc;
  }
  stage_twiddles(s, Tw, Lf, log2Lf);
  __syncthreads();
  for (int m = threadIdx.x; m < Lf; m += 256) {
    c32 acc{0.f, 0.f};
    for (int f = 0; f < Lf; ++f) {
      const c32 w = Tw[(m * f) & (Lf - 1)];
      acc.x += d[f] * w.x;
      acc.y += d[f] * w.y;
    }
    if (zeroth)
      s.dZh[s.z1_total + m] = acc;
    else
      s.dYh[s.y2_total + static_cast<int64_t>(n1) * Lf + m] = acc;
  }
}

template <int ST, bool GATHER = true>
hipError_t run_stage_t(const DevSig& s, const SigPlan& p, hipStream_t st) {
  if constexpr (ST == ST_BU || (ST == ST_BX && GATHER)) {
    if (p.gchn[ST] > 0) {
      hipLaunchKernelGGL(k_seg_gather<ST>, dim3(p.gchn[ST]), dim3(256), 0, st, s, p.gch0[ST]);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  if (p.ntask[ST] + p.split1_n[ST] > 0) {
    hipLaunchKernelGGL(k_fft_stage1<ST>, dim3(p.ntask[ST] + p.split1_n[ST]), dim3(256), 0, st, s, p.task0[ST],
                       p.ntask[ST], p.split1_0[ST]);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (p.split2_n[ST] > 0) {
    hipLaunchKernelGGL(k_fft_split2<ST>, dim3(p.split2_n[ST]), dim3(256), 0, st, s, p.split2_0[ST]);
    return hipGetLastError();
  }
  return hipSuccess;
}

}  // namespace

hipError_t run_time_stage(int stage, const DevSig& s, const SigPlan& p, hipStream_t st) {
  switch (stage) {
    case ST_XHAT: return run_stage_t<ST_XHAT>(s, p, st);
    case ST_L1Z: return run_stage_t<ST_L1Z>(s, p, st);
    case ST_L1UH: return run_stage_t<ST_L1UH>(s, p, st);
    case ST_L2Y: return run_stage_t<ST_L2Y>(s, p, st);
    case ST_BYH: return run_stage_t<ST_BYH>(s, p, st);
    case ST_BU: return run_stage_t<ST_BU>(s, p, st);
    case ST_BZH: return run_stage_t<ST_BZH>(s, p, st);
    case ST_BX: return run_stage_t<ST_BX>(s, p, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t run_signal_idft(const DevSig& s, const SigPlan& p, hipStream_t st) {
  return run_stage_t<ST_BX, false>(s, p, st);
}

hipError_t run_s1(const DevSig& s, const SigPlan& p, hipStream_t st) {
  hipLaunchKernelGGL(k_s1, dim3(p.psi1.size()), dim3(256), 0, st, s, p.s1_job0);
  // (the zeroth order is an output of the forward only: a backward recomputing the
  // first layer passes no coefficient array)
  if (p.s0_off >= 0 && s.S != nullptr) {
    if (p.u0) return run_u0(s, p, st);
    hipLaunchKernelGGL(k_s0, dim3(1), dim3(256), 0, st, s);
  }
  return hipGetLastError();
}

hipError_t run_ds1h(const DevSig& s, const SigPlan& p, hipStream_t st) {
  hipLaunchKernelGGL(k_ds1h, dim3(p.psi1.size() + (p.s0_off >= 0 && !p.u0 ? 1 : 0)), dim3(256), 0, st, s);
  return hipGetLastError();
}

}  // namespace jtfs
