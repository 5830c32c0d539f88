// Host emulation of the LDS Stockham FFT tile (fft_core.hpp): the 256 threads of a
// workgroup run sequentially, phase by phase, exactly as the barriers separate them on
// the GPU. Checks every length 16..4096 in both directions against a direct DFT in FP64,
// and the two-pass split used for longer transforms.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2602_11896_amd/csrc/fft_core.hpp"

using namespace jtfs;

static std::vector<c32> twiddles(int log2N) {
  int N = 1 << log2N;
  std::vector<c32> tw(N);
  for (int k = 0; k < N; ++k) {
    double a = -2.0 * M_PI * k / N;
    tw[k] = c32{(float)std::cos(a), (float)std::sin(a)};
  }
  return tw;
}

template <int DIR, int LR>
static void one_pass(std::vector<c32>& lds, int log2n, int log2p, const std::vector<c32>& tw, int log2tw) {
  const int n = 1 << log2n, tpf = n / 16;
  std::vector<c32> regs(256 * 16);
  for (int tid = 0; tid < 256; ++tid)
    stockham_compute<DIR, LR>(lds.data(), (tid / tpf) * n, log2n, log2p, tid % tpf, tpf, tw.data(), log2tw,
                              &regs[tid * 16]);
  for (int tid = 0; tid < 256; ++tid)
    stockham_store<LR>(lds.data(), (tid / tpf) * n, log2p, tid % tpf, tpf, &regs[tid * 16]);
}

template <int DIR>
static void tile_fft(std::vector<c32>& lds, int log2n, const std::vector<c32>& tw, int log2tw) {
  int lr[8];
  int np = fft_radices(log2n, lr);
  int log2p = 0;
  for (int s = 0; s < np; ++s) {
    switch (lr[s]) {
      case 1: one_pass<DIR, 1>(lds, log2n, log2p, tw, log2tw); break;
      case 2: one_pass<DIR, 2>(lds, log2n, log2p, tw, log2tw); break;
      case 3: one_pass<DIR, 3>(lds, log2n, log2p, tw, log2tw); break;
      default: one_pass<DIR, 4>(lds, log2n, log2p, tw, log2tw); break;
    }
    log2p += lr[s];
  }
}

static double check(int log2n, int dir, const std::vector<c32>& tw, int log2tw) {
  const int n = 1 << log2n, C = 4096 / n;
  std::vector<c32> lds(4096);
  std::vector<double> xr(4096), xi(4096);
  unsigned s = 12345u + log2n * 7 + dir;
  for (int e = 0; e < 4096; ++e) {
    s = s * 1664525u + 1013904223u;
    xr[e] = ((s >> 8) & 0xffff) / 65536.0 - 0.5;
    s = s * 1664525u + 1013904223u;
    xi[e] = ((s >> 8) & 0xffff) / 65536.0 - 0.5;
    lds[tile_slot(e)] = c32{(float)xr[e], (float)xi[e]};
  }
  if (dir < 0) tile_fft<-1>(lds, log2n, tw, log2tw);
  else tile_fft<+1>(lds, log2n, tw, log2tw);
  double err = 0, ref = 0;
  for (int c = 0; c < C; ++c)
    for (int k = 0; k < n; ++k) {
      double sr = 0, si = 0;
      for (int j = 0; j < n; ++j) {
        double a = dir * 2.0 * M_PI * (double)((long long)j * k % n) / n;
        sr += xr[c * n + j] * std::cos(a) - xi[c * n + j] * std::sin(a);
        si += xr[c * n + j] * std::sin(a) + xi[c * n + j] * std::cos(a);
      }
      const c32 o = lds[tile_slot(c * n + k)];
      double dr = o.x - sr, di = o.y - si;
      err += dr * dr + di * di;
      ref += sr * sr + si * si;
    }
  return std::sqrt(err / ref);
}

// Reference FFT in FP64 (recursive radix 2).
static void ref_fft(std::vector<double>& re, std::vector<double>& im, int dir) {
  const size_t n = re.size();
  if (n == 1) return;
  std::vector<double> er(n / 2), ei(n / 2), odr(n / 2), odi(n / 2);
  for (size_t i = 0; i < n / 2; ++i) {
    er[i] = re[2 * i]; ei[i] = im[2 * i]; odr[i] = re[2 * i + 1]; odi[i] = im[2 * i + 1];
  }
  ref_fft(er, ei, dir);
  ref_fft(odr, odi, dir);
  for (size_t k = 0; k < n / 2; ++k) {
    double a = dir * 2.0 * M_PI * k / n, c = std::cos(a), s = std::sin(a);
    double tr = odr[k] * c - odi[k] * s, ti = odr[k] * s + odi[k] * c;
    re[k] = er[k] + tr; im[k] = ei[k] + ti;
    re[k + n / 2] = er[k] - tr; im[k + n / 2] = ei[k] - ti;
  }
}

// Emulates pass 1 and pass 2 workgroups of the two-pass split for one n-point row.
static double check_split(int log2n, int log2A, int dir, const std::vector<c32>& tw, int log2tw) {
  const int n = 1 << log2n;
  SplitGeom g = split_geom(log2n, log2A);
  std::vector<double> xr(n), xi(n);
  std::vector<c32> x(n), scr(n), out(n);
  unsigned s = 777u + log2n;
  for (int i = 0; i < n; ++i) {
    s = s * 1664525u + 1013904223u; xr[i] = ((s >> 8) & 0xffff) / 65536.0 - 0.5;
    s = s * 1664525u + 1013904223u; xi[i] = ((s >> 8) & 0xffff) / 65536.0 - 0.5;
    x[i] = c32{(float)xr[i], (float)xi[i]};
  }
  std::vector<c32> lds(4096);
  const int A = 1 << g.log2A, B = 1 << g.log2B;
  for (int n1_0 = 0; n1_0 < A; n1_0 += 1 << g.log2C1) {
    for (int e = 0; e < 4096; ++e) { int idx, slot; split_p1_load(g, n1_0, e, idx, slot); lds[tile_slot(slot)] = x[idx]; }
    if (dir < 0) tile_fft<-1>(lds, g.log2B, tw, log2tw); else tile_fft<+1>(lds, g.log2B, tw, log2tw);
    // per thread t: its 16 elements e = t + 256 i take the composed twiddles of
    // split_p1_twiddles, whose exponents must be the n1 k2 of split_p1_store
    for (int t = 0; t < 256; ++t) {
      c32 w16[16];
      if (dir < 0) split_p1_twiddles<-1>(g, n1_0, t, tw.data(), log2tw - log2n, w16);
      else split_p1_twiddles<+1>(g, n1_0, t, tw.data(), log2tw - log2n, w16);
      for (int i = 0; i < 16; ++i) {
        int slot, sidx, te; split_p1_store(g, n1_0, t + 256 * i, slot, sidx, te);
        c32 wr = tw[(size_t)te << (log2tw - log2n)];
        if (dir > 0) wr.y = -wr.y;
        if (std::fabs(wr.x - w16[i].x) > 1e-6f || std::fabs(wr.y - w16[i].y) > 1e-6f) {
          std::printf("twiddle mismatch log2n=%d log2A=%d t=%d i=%d\n", log2n, log2A, t, i);
          std::exit(1);
        }
        scr[sidx] = cmul(lds[tile_slot(slot)], w16[i]);
      }
    }
  }
  for (int k2_0 = 0; k2_0 < B; k2_0 += 1 << g.log2C2) {
    for (int e = 0; e < 4096; ++e) lds[tile_slot(e)] = scr[split_p2_load(g, k2_0, e)];
    if (dir < 0) tile_fft<-1>(lds, g.log2A, tw, log2tw); else tile_fft<+1>(lds, g.log2A, tw, log2tw);
    for (int e = 0; e < 4096; ++e) { int slot, oidx; split_p2_store(g, k2_0, e, slot, oidx); out[oidx] = lds[tile_slot(slot)]; }
  }
  ref_fft(xr, xi, dir);
  double err = 0, ref = 0;
  for (int k = 0; k < n; ++k) {
    double dr = out[k].x - xr[k], di = out[k].y - xi[k];
    err += dr * dr + di * di; ref += xr[k] * xr[k] + xi[k] * xi[k];
  }
  return std::sqrt(err / ref);
}

// Bank spread of the swizzled tile: in every LDS write of a Stockham pass and in the
// transposes of the two-pass split, each 16 consecutive lanes of a wave must reach 16
// different slots modulo 16 (16 eight-byte elements fill one row of 32 four-byte banks).
// The writes are recorded by running the pass's store phase with values that name the
// writing lane and register.
static int bank_spread_failures() {
  int bad = 0;
  auto distinct16 = [](const int* slot16) {
    unsigned seen = 0;
    for (int l = 0; l < 16; ++l) seen |= 1u << (slot16[l] & 15);
    return seen == 0xffffu;
  };
  for (int log2n = 4; log2n <= 12; ++log2n) {
    const int n = 1 << log2n, tpf = n / 16;
    int lr[8];
    const int np = fft_radices(log2n, lr);
    int log2p = 0;
    for (int ps = 0; ps < np; ++ps) {
      std::vector<c32> tile(4096);
      for (int tid = 0; tid < 256; ++tid) {
        c32 v[16];
        for (int q = 0; q < 16; ++q) v[q] = c32{(float)tid, (float)q};
        switch (lr[ps]) {
          case 1: stockham_store<1>(tile.data(), (tid / tpf) * n, log2p, tid % tpf, tpf, v); break;
          case 2: stockham_store<2>(tile.data(), (tid / tpf) * n, log2p, tid % tpf, tpf, v); break;
          case 3: stockham_store<3>(tile.data(), (tid / tpf) * n, log2p, tid % tpf, tpf, v); break;
          default: stockham_store<4>(tile.data(), (tid / tpf) * n, log2p, tid % tpf, tpf, v); break;
        }
      }
      std::vector<int> where(256 * 16, -1);
      for (int q = 0; q < 4096; ++q) where[(int)tile[q].x * 16 + (int)tile[q].y] = q;
      for (int reg = 0; reg < 16; ++reg)
        for (int g = 0; g < 256; g += 16) {
          int s16[16];
          for (int l = 0; l < 16; ++l) s16[l] = where[(g + l) * 16 + reg];
          if (!distinct16(s16)) {
            std::printf("bank conflict: store n=%d pass=%d reg=%d lanes %d..%d\n", n, ps, reg, g, g + 15);
            bad = 1;
          }
        }
      log2p += lr[ps];
    }
  }
  for (int log2n = 13; log2n <= 17; ++log2n)
    for (int log2A = (log2n - 12 > 4 ? log2n - 12 : 4); log2A <= (log2n - 4 < 12 ? log2n - 4 : 12); ++log2A) {
      SplitGeom g = split_geom(log2n, log2A);
      for (int base = 0; base < 4096; base += 16) {
        int s1[16], s2[16];
        for (int l = 0; l < 16; ++l) {
          int idx, slot, sidx, te, oidx;
          split_p1_load(g, 0, base + l, idx, slot);
          s1[l] = tile_slot(slot);
          split_p2_store(g, 0, base + l, slot, oidx);
          s2[l] = tile_slot(slot);
          split_p1_store(g, 0, base + l, slot, sidx, te);
          if (tile_slot(slot) != s1[l]) bad = 1;   // pass 1 reads its tile as it loaded it
        }
        if (!distinct16(s1) || !distinct16(s2)) {
          std::printf("bank conflict: split n=%d A=%d elements %d..%d\n", 1 << log2n, 1 << log2A, base, base + 15);
          bad = 1;
        }
      }
    }
  return bad;
}

int main() {
  const int log2tw = 17;
  auto tw = twiddles(log2tw);
  int bad = 0;
  // the LDS swizzle must be a permutation of the tile
  {
    std::vector<int> seen(4096, 0);
    for (int e = 0; e < 4096; ++e) {
      const int q = tile_slot(e);
      if (q < 0 || q >= 4096 || seen[q]++) bad = 1;
    }
    std::printf("tile_slot permutation %s\n", bad ? "BROKEN" : "ok");
  }
  if (bank_spread_failures()) bad = 1;
  else std::printf("tile bank spread ok\n");
  for (int log2n = 4; log2n <= 12; ++log2n)
    for (int dir : {-1, 1}) {
      double e = check(log2n, dir, tw, log2tw);
      std::printf("n=%6d dir=%+d rel_l2=%.3e\n", 1 << log2n, dir, e);
      if (!(e < 2e-6)) bad = 1;
    }
  // every split point a plan may choose: both factors between 16 and 4096
  for (int log2n = 13; log2n <= 17; ++log2n)
    for (int log2A = (log2n - 12 > 4 ? log2n - 12 : 4); log2A <= (log2n - 4 < 12 ? log2n - 4 : 12); ++log2A)
      for (int dir : {-1, 1}) {
        double e = check_split(log2n, log2A, dir, tw, log2tw);
        std::printf("split n=%6d A=%5d dir=%+d rel_l2=%.3e\n", 1 << log2n, 1 << log2A, dir, e);
        if (!(e < 3e-6)) bad = 1;
      }
  std::printf(bad ? "FAIL\n" : "OK\n");
  return bad;
}
