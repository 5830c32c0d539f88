// Radix-2/4/8/16 Stockham FFT passes over a 4096-element LDS tile.
//
// The tile holds C = 4096 / n transforms of length n (16 <= n <= 4096, a power of two),
// column c at [c*n, c*n + n). 256 threads cooperate; thread t of a column owns 16
// elements in every pass (16 / R butterflies of radix R). A pass of radix R with span p
// (product of the earlier radices) reads butterfly i's inputs at i + r*(n/R), multiplies
// input r by w^(r*k) (w = exp(s*2*pi*i/(p*R)), k = i mod p, s = -1 forward, +1 inverse),
// takes the R-point DFT and writes output r to ((i - k)*R + k) + r*p. After the last
// pass the column holds its DFT in natural order (self-sorting, no bit reversal).
//
// Tile element e lives at LDS slot tile_slot(e) (below), a bank swizzle; every access
// to the tile goes through it. The per-thread steps are __host__ __device__ so that the
// same code can be driven by a sequential host emulation of the barrier-separated phases.
#pragma once
#include <cstdint>

#ifdef __HIPCC__
#define JTFS_HD __host__ __device__
#else
#define JTFS_HD
#endif

namespace jtfs {

struct __attribute__((aligned(8))) c32 {
  float x, y;
};

JTFS_HD inline c32 cadd(c32 a, c32 b) { return c32{a.x + b.x, a.y + b.y}; }
JTFS_HD inline c32 csub(c32 a, c32 b) { return c32{a.x - b.x, a.y - b.y}; }
JTFS_HD inline c32 cmul(c32 a, c32 b) { return c32{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
JTFS_HD inline c32 cscale(c32 a, float s) { return c32{a.x * s, a.y * s}; }
JTFS_HD inline c32 cconj(c32 a) { return c32{a.x, -a.y}; }

// cos / sin of 2 pi j / 16, j = 0..15
constexpr float kCos16[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                              0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                              -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
                              0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
constexpr float kSin16[16] = {0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
                              1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                              0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                              -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f};

// LDS slot of tile element e (0 <= e < 4096): bits 0-3 of e are XORed with bits 4-7 and
// 8-11, bit 4 with bit 8. The accesses of a wave move along strides that are powers of
// two (1 in the loads and the reads of long columns, 16 in the first pass's writes, the
// row length across the columns of short transforms, the column length in the
// transposes of the two-pass split); in the natural layout most of those strides put
// many lanes on one bank, and the swizzle spreads each of them over all the banks. It is
// a bijection (each changed bit takes only higher bits) and linear over GF(2):
// tile_slot(a + b) = tile_slot(a) ^ tile_slot(b) when a and b have no set bit in common,
// which lets a thread swizzle its base once and add offsets shared by the workgroup
// with a single XOR.
JTFS_HD constexpr int tile_slot(int e) { return e ^ ((e >> 4) & 31) ^ ((e >> 8) & 15); }

constexpr int bitrev(int v, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((v >> b) & 1) << (bits - 1 - b);
  return r;
}

// In-register R-point DFT (R = 2^LR), sign DIR (-1 forward, +1 inverse): iterative
// decimation in time on bit-reversed input with constant twiddles.
template <int LR, int DIR>
JTFS_HD inline void dft_reg(c32* v) {
  constexpr int R = 1 << LR;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int j = bitrev(i, LR);
    if (i < j) {
      c32 t = v[i];
      v[i] = v[j];
      v[j] = t;
    }
  }
#pragma unroll
  for (int len = 2; len <= R; len <<= 1) {
    const int half = len >> 1;
#pragma unroll
    for (int s = 0; s < R; s += len) {
#pragma unroll
      for (int k = 0; k < half; ++k) {
        const int e = k * (16 / len);           // twiddle exp(DIR 2 pi i k / len) = entry e of 16
        c32 w{kCos16[e], DIR * kSin16[e]};
        c32 t = (k == 0) ? v[s + k + half] : cmul(v[s + k + half], w);
        v[s + k + half] = csub(v[s + k], t);
        v[s + k] = cadd(v[s + k], t);
      }
    }
  }
}

// Radix sequence of an n-point transform: as many radix-16 passes as fit, then one of 2, 4 or 8.
JTFS_HD inline int fft_radices(int log2n, int* lr) {
  int np = 0, rem = log2n;
  while (rem >= 4) {
    lr[np++] = 4;
    rem -= 4;
  }
  if (rem) lr[np++] = rem;
  return np;
}

// Twiddle table reads of one radix-2^LR pass for thread t: for each of its 16 / R
// butterflies i, the powers w^(2^q), q < LR, of w = exp(-+2 pi i k / (R p)), k = i mod p
// (wp[b * LR + q]). They depend only on the thread, so a kernel can issue them before
// it waits for its data. `tw` holds exp(-2 pi i q / 2^log2tw); DIR > 0 conjugates.
template <int DIR, int LR>
JTFS_HD inline void stockham_twiddles(int log2n, int log2p, int t, int tpf, const c32* tw, int log2tw, c32* wp) {
  constexpr int NB = 16 >> LR;
  const int pmask = (1 << log2p) - 1;
  const int tshift = log2tw - (log2p + LR);
  (void)log2n;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int k = (t + tpf * b) & pmask;
#pragma unroll
    for (int q = 0; q < LR; ++q) {
      c32 x = tw[(k << q) << tshift];
      if (DIR > 0) x.y = -x.y;
      wp[b * LR + q] = x;
    }
  }
}

// Read phase of one radix-2^LR pass for thread t (of tpf threads on the column whose
// first element is tile element cbase), with the twiddle powers of stockham_twiddles:
// loads, twiddles and transforms the thread's 16 / R butterflies into v[0..16). A pass
// of span p > 1 multiplies input r by w^r, the powers not read from the table being
// products of those that are, in binary order (at most LR - 1 complex multiplications
// each). cbase (a multiple of n), i < n / R and r * (n / R) share no bits, so the slot
// of cbase + i + r * (n / R) is the XOR of their slots.
template <int DIR, int LR>
JTFS_HD inline void stockham_compute_tw(const c32* tile, int cbase, int log2n, int log2p, int t, int tpf,
                                        const c32* wp, c32* v) {
  constexpr int R = 1 << LR;
  constexpr int NB = 16 >> LR;
  const int stride = (1 << log2n) >> LR;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int i = t + tpf * b;
    const int sb = tile_slot(cbase + i);
#pragma unroll
    for (int r = 0; r < R; ++r) v[b * R + r] = tile[sb ^ tile_slot(r * stride)];
    if (log2p > 0) {
      c32 w[R];
#pragma unroll
      for (int q = 0; q < LR; ++q) w[1 << q] = wp[b * LR + q];
#pragma unroll
      for (int r = 3; r < R; ++r)
        if (r & (r - 1)) w[r] = cmul(w[r & (r - 1)], w[r & -r]);
#pragma unroll
      for (int r = 1; r < R; ++r) v[b * R + r] = cmul(v[b * R + r], w[r]);
    }
    dft_reg<LR, DIR>(v + b * R);
  }
}

// Both of the above in one call (twiddles read at the point of use).
template <int DIR, int LR>
JTFS_HD inline void stockham_compute(const c32* tile, int cbase, int log2n, int log2p, int t, int tpf,
                                     const c32* tw, int log2tw, c32* v) {
  c32 wp[16];
  if (log2p > 0) stockham_twiddles<DIR, LR>(log2n, log2p, t, tpf, tw, log2tw, wp);
  stockham_compute_tw<DIR, LR>(tile, cbase, log2n, log2p, t, tpf, wp, v);
}

// Write phase of the same pass: stores the 16 results of thread t. The output index
// j + r * p has j = (i - k) * R + k with k < p and (i - k) * R a multiple of p * R, so
// j, r * p and cbase share no bits either.
template <int LR>
JTFS_HD inline void stockham_store(c32* tile, int cbase, int log2p, int t, int tpf, const c32* v) {
  constexpr int R = 1 << LR;
  constexpr int NB = 16 >> LR;
  const int p = 1 << log2p;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int i = t + tpf * b;
    const int k = i & (p - 1);
    const int sb = tile_slot(cbase + ((i - k) << LR) + k);
#pragma unroll
    for (int r = 0; r < R; ++r) tile[sb ^ tile_slot(r * p)] = v[b * R + r];
  }
}

// Two-pass split of an n-point transform, n = A * B > 4096 (A = 2^floor(log2n / 2),
// B = n / A): with input index n1 + A*n2 and output index k2 + B*k1,
//   pass 1: for each column n1, a B-point transform over n2, times w_n^(n1*k2), written
//           to scratch at k2*A + n1;
//   pass 2: for each k2, an A-point transform over n1 of scratch row k2, giving X[k2 + B*k1].
// A pass-1 workgroup takes C1 = 4096 / B consecutive columns, a pass-2 workgroup
// C2 = 4096 / A consecutive rows; element e of the 4096 a workgroup moves maps as below
// (consecutive e touch consecutive global addresses).
struct SplitGeom {
  int log2n, log2A, log2B, log2C1, log2C2;
};

// log2A: the split point (A, B <= 4096 is required; default floor(log2n / 2)).
JTFS_HD inline SplitGeom split_geom(int log2n, int log2A) {
  SplitGeom g;
  g.log2n = log2n;
  g.log2A = log2A;
  g.log2B = log2n - g.log2A;
  g.log2C1 = 12 - g.log2B;
  g.log2C2 = 12 - g.log2A;
  return g;
}
JTFS_HD inline SplitGeom split_geom(int log2n) { return split_geom(log2n, log2n / 2); }

// pass 1 load: input index and tile element ("slot", stored at tile_slot(slot)) of
// element e (column base n1_0)
JTFS_HD inline void split_p1_load(const SplitGeom& g, int n1_0, int e, int& idx, int& slot) {
  const int c = e & ((1 << g.log2C1) - 1), n2 = e >> g.log2C1;
  idx = (n1_0 + c) + (n2 << g.log2A);
  slot = (c << g.log2B) + n2;
}

// pass 1 store: tile element, scratch index and twiddle exponent n1*k2 of element e
JTFS_HD inline void split_p1_store(const SplitGeom& g, int n1_0, int e, int& slot, int& sidx, int& twexp) {
  const int c = e & ((1 << g.log2C1) - 1), k2 = e >> g.log2C1;
  slot = (c << g.log2B) + k2;
  sidx = (k2 << g.log2A) + n1_0 + c;
  twexp = (n1_0 + c) * k2;
}

// Pass-1 twiddles of thread t, w_n^(n1 k2) for its 16 elements e = t + 256 i: since
// C1 <= 256 (B >= 16), they share the column n1 = n1_0 + (t mod C1) and take
// k2 = k2_0 + i s with s = 256 / C1. Five table reads, w^(n1 k2_0) and w^(n1 s 2^q),
// q < 4, and the rest as products in binary order (at most four complex
// multiplications each) instead of sixteen scattered reads. tw: exp(-2 pi i q / 2^log2tw);
// DIR > 0 conjugates.
template <int DIR>
JTFS_HD inline void split_p1_twiddle_bases(const SplitGeom& g, int n1_0, int t, const c32* tw, int tshift, c32* b5) {
  const int c = t & ((1 << g.log2C1) - 1), k2_0 = t >> g.log2C1;
  const int n1 = n1_0 + c;
  const int step = 256 >> g.log2C1;
  for (int q = 0; q < 4; ++q) {
    b5[q] = tw[((n1 * step) << q) << tshift];
    if (DIR > 0) b5[q].y = -b5[q].y;
  }
  b5[4] = tw[(n1 * k2_0) << tshift];
  if (DIR > 0) b5[4].y = -b5[4].y;
}

// The sixteen twiddles from the five table reads above (b5[4] = w^(n1 k2_0),
// b5[q] = w^(n1 s 2^q)).
JTFS_HD inline void split_p1_twiddle_expand(const c32* b5, c32* w16) {
  w16[0] = b5[4];
  for (int i = 1; i < 16; ++i) {
    const int low = i & -i;
    const int q = low == 1 ? 0 : low == 2 ? 1 : low == 4 ? 2 : 3;
    w16[i] = cmul(w16[i - low], b5[q]);
  }
}

template <int DIR>
JTFS_HD inline void split_p1_twiddles(const SplitGeom& g, int n1_0, int t, const c32* tw, int tshift, c32* w16) {
  c32 b5[5];
  split_p1_twiddle_bases<DIR>(g, n1_0, t, tw, tshift, b5);
  split_p1_twiddle_expand(b5, w16);
}

// pass 2 load: scratch index of element e (row base k2_0); the tile element is e itself
JTFS_HD inline int split_p2_load(const SplitGeom& g, int k2_0, int e) {
  const int c = e >> g.log2A, n1 = e & ((1 << g.log2A) - 1);
  return ((k2_0 + c) << g.log2A) + n1;
}

// pass 2 store: tile element and output index of element e
JTFS_HD inline void split_p2_store(const SplitGeom& g, int k2_0, int e, int& slot, int& oidx) {
  const int c = e & ((1 << g.log2C2) - 1), k1 = e >> g.log2C2;
  slot = (c << g.log2A) + k1;
  oidx = (k2_0 + c) + (k1 << g.log2B);
}

}  // namespace jtfs
