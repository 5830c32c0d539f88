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

__device__ inline float cabs(c32 z) { return sqrtf(z.x * z.x + z.y * z.y); }

// Fourier subsampling by 2^shift of (src . band) onto an n-point grid, output bin q.
// The plan guarantees that a band is not empty and spans at most two aliased blocks
// (1 <= len <= 2 n), so both are read without a loop, at indices clamped into the band and with an absent second
// term masked by value: the loads of several bins can be in flight together.
__device__ inline c32 fold_gather(const c32* src, const Band& b, const float* vals, int n, int shift, int q) {
  const int nmask = n - 1;
  const int d0 = (q - (b.lo & nmask)) & nmask;
  c32 acc{0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
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
  const float sc = ldexpf(1.0f, -shift);
  return c32{acc.x * sc, acc.y * sc};
}

// Adjoint gather: sum over terms of band[m] * src_t[m mod len_t], output bin m; only the
// terms whose band meets m's 512-bin segment are visited. Every band is non-empty, so a
// term whose band misses m reads the band at a clamped index and is masked by value: no
// branch, so the loads of several terms can be in flight together.
__device__ inline void term_add(const DevSig& s, const c32* base, const SegTerm& g, int m, c32& acc) {
  int d = m - g.lo;
  if (d < 0) d += g.L;
  const bool in = d < g.len;
  const float h = s.bandvals[g.off + (in ? d : 0)];
  const c32 v = base[g.src + (m & (g.src_len - 1))];
  const float hm = in ? h : 0.f;
  acc.x += v.x * hm;
  acc.y += v.y * hm;
}

// seg0 = the row's first segment. When the whole wave's bins lie in one segment (single-
// tile rows of 64 bins or more, the bin-parallel gather), its terms come by scalar loads.
__device__ inline c32 term_gather(const DevSig& s, const c32* base, int seg0, int m) {
  c32 acc{0.f, 0.f};
  const int sg = seg0 + (m >> 9);
  const int sgu = __builtin_amdgcn_readfirstlane(sg);
  if (__all(sg == sgu)) {
    const int first = s.segs[2 * sgu], count = s.segs[2 * sgu + 1];
#pragma unroll 4
    for (int i = 0; i < count; ++i) term_add(s, base, s.segterms[first + i], m, acc);
  } else {
    const int first = s.segs[2 * sg], count = s.segs[2 * sg + 1];
#pragma unroll 4
    for (int i = 0; i < count; ++i) term_add(s, base, s.segterms[first + i], m, acc);
  }
  return acc;
}

template <int ST>
struct Ops;

template <>
struct Ops<ST_XHAT> {
  static constexpr int DIR = -1;
  __device__ static c32 load(const DevSig& s, const RowJob&, const Band&, int idx) {
    const int j = idx - s.pad_left;
    return c32{(j >= 0 && j < s.N) ? s.x[j] : 0.f, 0.f};
  }
  __device__ static void store(const DevSig& s, const RowJob&, int idx, c32 v) { s.Xh[idx] = v; }
};

template <>
struct Ops<ST_L1Z> {
  static constexpr int DIR = +1;
  __device__ static c32 load(const DevSig& s, const RowJob& j, const Band& b, int idx) {
    return fold_gather(s.Xh, b, s.bandvals, j.n, j.shift, idx);
  }
  __device__ static void store(const DevSig& s, const RowJob& j, int idx, c32 v) { s.Z1[j.dst + idx] = v; }
};

template <>
struct Ops<ST_L1UH> {
  static constexpr int DIR = -1;
  __device__ static c32 load(const DevSig& s, const RowJob& j, const Band&, int idx) {
    return c32{cabs(s.Z1[j.src + idx]), 0.f};
  }
  __device__ static void store(const DevSig& s, const RowJob& j, int idx, c32 v) { s.U1h[j.dst + idx] = v; }
};

template <>
struct Ops<ST_L2Y> {
  static constexpr int DIR = +1;
  __device__ static c32 load(const DevSig& s, const RowJob& j, const Band& b, int idx) {
    return fold_gather(s.U1h + j.src, b, s.bandvals, j.n, j.shift, idx);
  }
  __device__ static void store(const DevSig& s, const RowJob& j, int idx, c32 v) { s.Y2[j.dst + idx] = v; }
};

template <>
struct Ops<ST_BYH> {
  static constexpr int DIR = -1;
  __device__ static c32 load(const DevSig& s, const RowJob& j, const Band&, int idx) { return s.dYpart[j.src + idx]; }
  __device__ static void store(const DevSig& s, const RowJob& j, int idx, c32 v) { s.dYh[j.dst + idx] = v; }
};

template <>
struct Ops<ST_BU> {
  static constexpr int DIR = +1;
  __device__ static c32 load(const DevSig& s, const RowJob& j, const Band&, int idx) {
    return term_gather(s, s.dYh, j.t0, idx);
  }
  __device__ static void store(const DevSig& s, const RowJob& j, int idx, c32 v) { s.dU1[j.dst + idx] = v.x; }
};

template <>
struct Ops<ST_BZH> {
  static constexpr int DIR = -1;
  __device__ static c32 load(const DevSig& s, const RowJob& j, const Band&, int idx) {
    // u times the phase z / |z| (rsq, within 1 ulp; subgradient 0 where |z| vanishes,
    // below 1.1e-19 the square underflows anyway)
    const float u = s.dU1[j.src + idx];
    const c32 z = s.Z1[j.aux + idx];
    const float m2 = z.x * z.x + z.y * z.y;
    const float r = m2 >= 1.17549435e-38f ? u * __builtin_amdgcn_rsqf(m2) : 0.f;
    return c32{z.x * r, z.y * r};
  }
  __device__ static void store(const DevSig& s, const RowJob& j, int idx, c32 v) { s.dZh[j.dst + idx] = v; }
};

template <>
struct Ops<ST_BX> {
  static constexpr int DIR = +1;
  // the gather itself runs beforehand in k_bx_gather, over the whole spectrum at once
  __device__ static c32 load(const DevSig& s, const RowJob&, const Band&, int idx) { return s.dXh[idx]; }
  __device__ static void store(const DevSig& s, const RowJob&, int idx, c32 v) {
    const int k = idx - s.pad_left;
    if (k >= 0 && k < s.N) s.dx[k] = v.x;
  }
};

// Gather of the first-order adjoint onto the padded signal spectrum,
//   dXhat[m] = sum_n1 psi1_n1[m] dZ1hat_n1[m mod L1_n1],
// one thread per bin (the inverse DFT of stage BX reads the result).
__global__ __launch_bounds__(256) void k_bx_gather(DevSig s, int job) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= s.N_pad) return;
  s.dXh[m] = term_gather(s, s.dZh, s.jobs[job].t0, m);
}

// One radix-2^LR pass over the tile (two barriers: all reads before any write).
template <int DIR, int LR>
__device__ inline void tile_pass(c32* tile, int cbase, int log2n, int log2p, int t, int tpf, const c32* tw,
                                 int log2tw) {
  c32 v[16];
  stockham_compute<DIR, LR>(tile, cbase, log2n, log2p, t, tpf, tw, log2tw, v);
  __syncthreads();
  stockham_store<LR>(tile, cbase, log2p, t, tpf, v);
  __syncthreads();
}

// In-place FFT of the 4096 / n columns of the tile (natural order in and out; element
// e at LDS slot tile_slot(e)).
template <int DIR>
__device__ void fft_tile(c32* lds, int log2n, const c32* tw, int log2tw) {
  const int tpf = 1 << (log2n - 4);
  const int t = threadIdx.x & (tpf - 1);
  const int cbase = (threadIdx.x >> (log2n - 4)) << log2n;
  int lr[8];
  const int np = fft_radices(log2n, lr);
  int log2p = 0;
  for (int p = 0; p < np; ++p) {
    switch (lr[p]) {
      case 1: tile_pass<DIR, 1>(lds, cbase, log2n, log2p, t, tpf, tw, log2tw); break;
      case 2: tile_pass<DIR, 2>(lds, cbase, log2n, log2p, t, tpf, tw, log2tw); break;
      case 3: tile_pass<DIR, 3>(lds, cbase, log2n, log2p, t, tpf, tw, log2tw); break;
      default: tile_pass<DIR, 4>(lds, cbase, log2n, log2p, t, tpf, tw, log2tw); break;
    }
    log2p += lr[p];
  }
}

// One workgroup per task: `count` rows of one length, all in one 4096-element tile. The
// rows' jobs and bands are staged in LDS first (count <= 4096 / 16), so that each element
// reads only its data from global memory.
constexpr int kMaxTileRows = 256;

template <int ST>
__device__ void rows_body(const DevSig& s, c32* lds, RowJob* tj, Band* tb, int task) {
  using O = Ops<ST>;
  const RowTask tk = s.tasks[task];
  const int log2n = tk.log2n;
  const int n = 1 << log2n;
  const int count = min(tk.count, kMaxTileRows);
  for (int r = threadIdx.x; r < count; r += 256) {
    const RowJob j = s.jobs[tk.job0 + r];
    tj[r] = j;
    tb[r] = j.band >= 0 ? s.bands[j.band] : Band{0, 0, 0, 0, 0};
  }
  __syncthreads();
#pragma unroll 4
  for (int i = 0; i < 16; ++i) {
    // (elements past the last row load from it and are zeroed by value: no branch, so
    // the loads of consecutive elements can be in flight together)
    const int e = threadIdx.x + 256 * i;
    const int row = e >> log2n;
    const int rc = min(row, count - 1);
    const c32 v = O::load(s, tj[rc], tb[rc], e & (n - 1));
    lds[tile_slot(e)] = row < count ? v : c32{0.f, 0.f};
  }
  __syncthreads();
  fft_tile<O::DIR>(lds, log2n, s.tw, s.log2_Npad);
  const float sc = O::DIR > 0 ? 1.0f / n : 1.0f;
#pragma unroll 4
  for (int i = 0; i < 16; ++i) {
    const int e = threadIdx.x + 256 * i;
    const int row = e >> log2n;
    if (row < count) O::store(s, tj[row], e & (n - 1), cscale(lds[tile_slot(e)], sc));
  }
}

// Two-pass transforms: every row of a stage, of any length above 4096, in one launch per
// pass; each workgroup reads its row, length, block and scratch offset from the task list.
template <int ST>
__device__ void split1_body(const DevSig& s, c32* lds, int task) {
  using O = Ops<ST>;
  const SplitTask tk = s.stasks[task];
  const int log2n = tk.log2n;
  const SplitGeom g = split_geom(log2n, tk.log2A);
  const RowJob job = s.jobs[tk.job];
  const Band band = job.band >= 0 ? s.bands[job.band] : Band{0, 0, 0, 0, 0};
  const int n1_0 = tk.blk << g.log2C1;
#pragma unroll 4
  for (int i = 0; i < 16; ++i) {
    int idx, slot;
    split_p1_load(g, n1_0, threadIdx.x + 256 * i, idx, slot);
    lds[tile_slot(slot)] = O::load(s, job, band, idx);
  }
  __syncthreads();
  fft_tile<O::DIR>(lds, g.log2B, s.tw, s.log2_Npad);
  c32* scr = s.scr + tk.scr;
  const int tshift = s.log2_Npad - log2n;
  c32 w16[16];
  split_p1_twiddles<O::DIR>(g, n1_0, threadIdx.x, s.tw, tshift, w16);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    int slot, sidx, te;
    split_p1_store(g, n1_0, threadIdx.x + 256 * i, slot, sidx, te);
    scr[sidx] = cmul(lds[tile_slot(slot)], w16[i]);
  }
}

// First launch of a stage: the short-row tasks (whole rows in one tile), then pass 1 of
// every long row; the two sets are independent, so they share one launch.
template <int ST>
__global__ __launch_bounds__(256) void k_fft_stage1(DevSig s, int task0, int ntask, int split0) {
  __shared__ c32 lds[4096];
  __shared__ RowJob tj[kMaxTileRows];
  __shared__ Band tb[kMaxTileRows];
  if (static_cast<int>(blockIdx.x) < ntask)
    rows_body<ST>(s, lds, tj, tb, task0 + blockIdx.x);
  else
    split1_body<ST>(s, lds, split0 + blockIdx.x - ntask);
}

template <int ST>
__global__ __launch_bounds__(256) void k_fft_split2(DevSig s, int task0) {
  __shared__ c32 lds[4096];
  using O = Ops<ST>;
  const SplitTask tk = s.stasks[task0 + blockIdx.x];
  const int log2n = tk.log2n;
  const SplitGeom g = split_geom(log2n, tk.log2A);
  const RowJob job = s.jobs[tk.job];
  const int k2_0 = tk.blk << g.log2C2;
  const c32* scr = s.scr + tk.scr;
  for (int i = 0; i < 16; ++i) {
    const int e = threadIdx.x + 256 * i;
    lds[tile_slot(e)] = scr[split_p2_load(g, k2_0, e)];
  }
  __syncthreads();
  fft_tile<O::DIR>(lds, g.log2A, s.tw, s.log2_Npad);
  const float sc = O::DIR > 0 ? 1.0f / static_cast<float>(1 << log2n) : 1.0f;
  for (int i = 0; i < 16; ++i) {
    int slot, oidx;
    split_p2_store(g, k2_0, threadIdx.x + 256 * i, slot, oidx);
    O::store(s, job, oidx, cscale(lds[tile_slot(slot)], sc));
  }
}

// First-order averaging (Eq. 3 before phi_F): S1 = Re IDFT_Lf(fold(U1hat . phi_T^(k1))),
// one workgroup per first-order row; the Lf-point inverse DFT is computed directly.
__global__ __launch_bounds__(256) void k_s1(DevSig s, int job0) {
  __shared__ c32 F[1024];
  const RowJob j = s.jobs[job0 + blockIdx.x];
  const int Lf = j.n;
  const int log2Lf = 31 - __clz(Lf);
  const Band b = s.bands[j.band];
  for (int q = threadIdx.x; q < Lf; q += 256) F[q] = fold_gather(s.U1h + j.src, b, s.bandvals, Lf, j.shift, q);
  __syncthreads();
  const int tshift = s.log2_Npad - log2Lf;
  for (int f = threadIdx.x; f < Lf; f += 256) {
    float acc = 0.f;
    for (int q = 0; q < Lf; ++q) {
      const c32 w = s.tw[((q * f) & (Lf - 1)) << tshift];   // exp(-2 pi i q f / Lf)
      acc += F[q].x * w.x + F[q].y * w.y;                    // Re(F exp(+2 pi i q f / Lf))
    }
    s.S1[j.dst + f] = acc / Lf;
  }
}

// Adjoint of the first-order averaging onto the spectrum: for each first-order row,
// dS1hat = DFT_Lf(sum over the real frequential filters of their dS1 contributions).
__global__ __launch_bounds__(256) void k_ds1h(DevSig s) {
  __shared__ float d[1024];
  const int n1 = blockIdx.x;
  const int Lf = s.nf_pad;
  const int log2Lf = 31 - __clz(Lf);
  for (int f = threadIdx.x; f < Lf; f += 256) {
    float acc = 0.f;
    for (int g = 0; g < s.n_real; ++g) acc += s.dS1p[(static_cast<int64_t>(g) * s.N1 + n1) * Lf + f];
    d[f] = acc;
  }
  __syncthreads();
  const int tshift = s.log2_Npad - log2Lf;
  for (int m = threadIdx.x; m < Lf; m += 256) {
    c32 acc{0.f, 0.f};
    for (int f = 0; f < Lf; ++f) {
      const c32 w = s.tw[((m * f) & (Lf - 1)) << tshift];
      acc.x += d[f] * w.x;
      acc.y += d[f] * w.y;
    }
    s.dYh[s.y2_total + static_cast<int64_t>(n1) * Lf + m] = acc;
  }
}

template <int ST, bool GATHER = true>
hipError_t run_stage_t(const DevSig& s, const SigPlan& p, hipStream_t st) {
  if (ST == ST_BX && GATHER) {
    hipLaunchKernelGGL(k_bx_gather, dim3((p.N_pad + 255) / 256), dim3(256), 0, st, s, p.bx_job);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
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
  return hipGetLastError();
}

hipError_t run_ds1h(const DevSig& s, const SigPlan& p, hipStream_t st) {
  hipLaunchKernelGGL(k_ds1h, dim3(p.psi1.size()), dim3(256), 0, st, s);
  return hipGetLastError();
}

}  // namespace jtfs
