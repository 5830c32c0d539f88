// Host-side JTFS plan (see plan.hpp). All tables are computed in FP64 and rounded
// once to FP32 when stored.
#include "plan.hpp"

#include "fft_core.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <system_error>
#include <thread>

namespace jtfs {
namespace {

constexpr double kSigma0 = 0.1;      // sigma0 of the Sec. 3.1 generator
constexpr double kBandThresh = 1e-10; // Fourier bins below this fraction of the peak are dropped
constexpr double kTapThresh = 1e-9;   // frequential taps below this fraction of the peak are skipped
constexpr int kPeriods = 4;           // period-1 images of a Fourier Gaussian on each side
constexpr double kPi = 3.14159265358979323846;
constexpr int64_t kPlanThreads = 16;  // host threads evaluating one long filter band

int ceil_log2(int64_t n) {
  int p = 0;
  while ((int64_t(1) << p) < n) ++p;
  return p;
}

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

double gauss(double u, double s) { return std::exp(-(u * u) / (2.0 * s * s)); }

// Fourier closed form of a Morlet at a given level: periodised Gaussian bump minus kappa
// times the periodised Gaussian envelope, kappa making the value at w = 0 vanish.
struct Morlet {
  double xs, ss, kappa;
  Morlet(double xi, double sigma, int level) {
    xs = std::ldexp(xi, level);
    ss = std::ldexp(sigma, level);
    double num = 0.0, den = 0.0;
    for (int p = -kPeriods; p <= kPeriods; ++p) {
      num += gauss(p - xs, ss);
      den += gauss(static_cast<double>(p), ss);
    }
    kappa = num / den;
  }
  double operator()(double w) const {
    double bump = 0.0, env = 0.0;
    for (int p = -kPeriods; p <= kPeriods; ++p) {
      bump += gauss(w + p - xs, ss);
      env += gauss(w + p, ss);
    }
    return bump - kappa * env;
  }
};

// Fourier closed form of a Gaussian low-pass at a given level, unit gain at w = 0.
struct Lowpass {
  double ss, norm;
  Lowpass(double sigma, int level) {
    ss = std::ldexp(sigma, level);
    norm = 0.0;
    for (int p = -kPeriods; p <= kPeriods; ++p) norm += gauss(static_cast<double>(p), ss);
  }
  double operator()(double w) const {
    double env = 0.0;
    for (int p = -kPeriods; p <= kPeriods; ++p) env += gauss(w + p, ss);
    return env / norm;
  }
};

// Appends the band-limited image of a real Fourier filter on an L-point grid.
// [wlo, whi] is a frequency window (cycles per sample, may leave [0, 1)) outside
// which the filter is known to be negligible.
template <class Fn>
int32_t add_band(SigPlan& p, int64_t L, const Fn& value, double wlo, double whi) {
  int64_t mlo = static_cast<int64_t>(std::floor(wlo * L));
  int64_t mhi = static_cast<int64_t>(std::ceil(whi * L));
  if (mhi - mlo + 1 >= L) {
    mlo = 0;
    mhi = L - 1;
  }
  const int64_t nv = mhi - mlo + 1;
  std::vector<double> v(static_cast<size_t>(nv));
  // Every bin is evaluated on its own, so long windows (up to a few million bins for the
  // first-order bank of a 2^20-sample signal) are split across host threads; the values,
  // and hence the tables, are the same as in one thread.
  auto fill = [&](int64_t a, int64_t b) {
    for (int64_t i = a; i < b; ++i) v[static_cast<size_t>(i)] = value(static_cast<double>(mlo + i) / static_cast<double>(L));
  };
  const unsigned hw = std::thread::hardware_concurrency();
  const int64_t nt = nv >= (int64_t{1} << 16) ? std::max<int64_t>(1, std::min<int64_t>(kPlanThreads, hw)) : 1;
  if (nt > 1) {
    std::vector<std::thread> th;
    th.reserve(static_cast<size_t>(nt - 1));
    for (int64_t t = 1; t < nt; ++t) {
      try {
        th.emplace_back(fill, nv * t / nt, nv * (t + 1) / nt);
      } catch (const std::system_error&) {   // no thread to be had: the rest runs here
        fill(nv * t / nt, nv);
        break;
      }
    }
    fill(0, nv / nt);
    for (std::thread& x : th) x.join();
  } else {
    fill(0, nv);
  }
  double peak = 0.0;
  for (double x : v) peak = std::max(peak, std::fabs(x));
  int64_t first = 0, last = static_cast<int64_t>(v.size()) - 1;
  const double thr = kBandThresh * peak;
  while (first < last && std::fabs(v[first]) <= thr) ++first;
  while (last > first && std::fabs(v[last]) <= thr) --last;
  Band b{};
  b.L = static_cast<int32_t>(L);
  b.lo = static_cast<int32_t>(((mlo + first) % L + L) % L);
  b.len = static_cast<int32_t>(last - first + 1);
  b.off = static_cast<int64_t>(p.bandvals.size());
  for (int64_t i = first; i <= last; ++i) p.bandvals.push_back(static_cast<float>(v[i]));
  p.bands.push_back(b);
  return static_cast<int32_t>(p.bands.size() - 1);
}

int32_t add_morlet_band(SigPlan& p, int64_t L, double xi, double sigma, int level) {
  Morlet h(xi, sigma, level);
  double lo = std::min(h.xs, 0.0) - 8.0 * h.ss, hi = std::max(h.xs, 0.0) + 8.0 * h.ss;
  return add_band(p, L, h, lo, hi);
}

int32_t add_lowpass_band(SigPlan& p, int64_t L, double sigma, int level) {
  Lowpass h(sigma, level);
  return add_band(p, L, h, -8.0 * h.ss, 8.0 * h.ss);
}

// Time-domain Gaussian low-pass at a level on an L-point grid: the continuous Gaussian
// sampled at integers and periodised, normalised to unit sum (the inverse DFT of the
// Fourier closed form, by Poisson summation).
int64_t add_lowpass_time(SigPlan& p, int64_t L, double sigma, int level) {
  const double ss = std::ldexp(sigma, level);
  const double a = 2.0 * kPi * kPi * ss * ss;
  const double width = 40.0 / (2.0 * kPi * ss);
  const int64_t q = static_cast<int64_t>(std::ceil(width / static_cast<double>(L))) + 1;
  std::vector<double> h(static_cast<size_t>(L), 0.0);
  double total = 0.0;
  for (int64_t d = 0; d < L; ++d) {
    double s = 0.0;
    for (int64_t img = -q; img <= q; ++img) {
      double t = static_cast<double>(d + img * L);
      s += std::exp(-a * t * t);
    }
    h[d] = s;
    total += s;
  }
  int64_t off = static_cast<int64_t>(p.tables.size());
  for (int64_t d = 0; d < L; ++d) p.tables.push_back(static_cast<float>(h[d] / total));
  return off;
}

}  // namespace

// Number of constant-Q members of a Sec. 3.1 bank: widths sigma_top 2^(-k/Q) strictly
// above the floor sigma_min, i.e. every k < R = Q log2(sigma_top / sigma_min); R within
// 1e-9 of an integer counts as that integer (the member of width exactly sigma_min is
// not constant-Q). No room (sigma_top <= sigma_min) gives 0.
static int constant_q_members(double sigma_top, double sigma_min, int Q) {
  if (sigma_top <= sigma_min) return 0;
  const double R = Q * std::log2(sigma_top / sigma_min);
  const double m = std::round(R);
  if (std::fabs(R - m) <= 1e-9 * std::max(1.0, R)) return std::max(1, static_cast<int>(m));
  return std::max(1, static_cast<int>(std::ceil(R)));
}

// Sec. 3.1 bank in closed form: the top filter (xi_top, sigma_top), whose neighbours a
// factor 2^(1/Q) away cross it at sqrt(1/2) of the peak; the constant-Q members scaled
// by 2^(-k/Q); then Q - 1 members of width sigma_min with centres e (Q - q) / Q, e the
// last constant-Q centre (sigma_top when there is none).
std::vector<std::pair<double, double>> wavelet_bank(int J, int Q) {
  std::vector<std::pair<double, double>> bank;
  const double xi_top = std::max(1.0 / (1.0 + std::pow(2.0, 3.0 / Q)), 0.35);
  const double f = std::pow(2.0, -1.0 / Q);
  const double sigma_top = (1.0 - f) / (1.0 + f) * xi_top / std::sqrt(2.0 * std::log(1.0 / std::sqrt(0.5)));
  const double sigma_min = kSigma0 / std::pow(2.0, J);
  const int n_cq = constant_q_members(sigma_top, sigma_min, Q);
  for (int k = 0; k < n_cq; ++k) {
    const double g = std::pow(2.0, -static_cast<double>(k) / Q);
    bank.emplace_back(xi_top * g, sigma_top * g);
  }
  const double elbow = n_cq ? bank.back().first : sigma_top;
  for (int q = 1; q < Q; ++q) bank.emplace_back(elbow * (Q - q) / Q, sigma_min);
  return bank;
}

int32_t subsampling_scale(double xi, double sigma) {
  const double edge = std::fabs(xi) + 5.0 * sigma;
  int32_t j = 0;
  while (edge <= std::ldexp(1.0, -(j + 2))) ++j;
  return j;
}

bool resolve_tuning(const jtfs_tuning* in, jtfs_tuning& t) {
  t = jtfs_tuning{256, 32, 128, 0, {0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};
  if (in) {
    if (in->fwd_rows) t.fwd_rows = in->fwd_rows;
    if (in->fwd_mt) t.fwd_mt = in->fwd_mt;
    if (in->bwd_rows) t.bwd_rows = in->bwd_rows;
    t.split_bias = in->split_bias;
  }
  bool ok = t.fwd_rows >= 16 && t.fwd_rows <= 8192 && (t.fwd_mt == 16 || t.fwd_mt == 32) && t.bwd_rows >= 16 &&
            t.bwd_rows <= 8192 && t.split_bias >= -2 && t.split_bias <= 2;
  for (int b = 0; b < JTFS_N_BUCKETS; ++b) {
    const int32_t f = in ? in->fwd_rows_k[b] : 0, w = in ? in->bwd_rows_k[b] : 0;
    ok = ok && (f == 0 || (f >= 16 && f <= 8192)) && (w == 0 || (w >= 16 && w <= 8192));
    t.fwd_rows_k[b] = f ? f : t.fwd_rows;
    t.bwd_rows_k[b] = w ? w : t.bwd_rows;
  }
  return ok;
}

jtfs_status build_signal_plan(const jtfs_params& prm, SigPlan& p, std::string& err, const jtfs_tuning* tune) {
  jtfs_tuning tu;
  if (!resolve_tuning(tune, tu)) {
    err = "tuning field out of range";
    return JTFS_ERR_ARG;
  }
  p = SigPlan{};
  p.prm = prm;
  p.no_avg_local = (prm.flags & JTFS_NO_AVERAGE_LOCAL) != 0;
  p.no_avg_fr = (prm.flags & JTFS_NO_AVERAGE_LOCAL_FR) != 0;
  if (prm.n < 2 || prm.J < 0 || prm.Q1 < 1 || prm.Q2 < 1 || prm.J_fr < 0 || prm.Q_fr < 1 || prm.log2_T < 0 ||
      !(prm.F >= 1.0) || prm.J > 24 || prm.J_fr > 24 || prm.Q1 > 64 || prm.Q2 > 64 || prm.Q_fr > 64) {
    err = "invalid JTFS parameters";
    return JTFS_ERR_ARG;
  }
  if ((prm.flags & ~(JTFS_ZEROTH | JTFS_NO_AVERAGE_LOCAL | JTFS_NO_AVERAGE_LOCAL_FR)) ||
      !(prm.zeroth_weight >= 0.f) || !std::isfinite(prm.zeroth_weight)) {
    err = "unknown flags or a zeroth-order weight that is not finite and non-negative";
    return JTFS_ERR_ARG;
  }
  p.N = prm.n;
  if (prm.periodic) {
    if (prm.n & (prm.n - 1)) {
      err = "periodic mode needs n a power of two";
      return JTFS_ERR_ARG;
    }
    p.N_pad = prm.n;
    p.pad_left = 0;
  } else {
    p.N_pad = int64_t(1) << (ceil_log2(prm.n) + 1);
    p.pad_left = (p.N_pad - p.N) / 2;
  }
  p.log2_Npad = ceil_log2(p.N_pad);
  if (p.N_pad > (int64_t(1) << 24)) {
    err = "padded length above 2^24 is not supported";
    return JTFS_ERR_UNSUPPORTED;
  }
  p.log2T = prm.log2_T;
  if (prm.log2_T > p.log2_Npad) {
    err = "T exceeds the padded length";
    return JTFS_ERR_ARG;
  }
  p.T = 1 << prm.log2_T;
  p.sF = 0;
  while (std::ldexp(1.0, p.sF + 1) <= prm.F) ++p.sF;
  p.sigmaT = kSigma0 / p.T;
  p.sigmaF = kSigma0 / prm.F;

  for (auto& xs : wavelet_bank(prm.J, prm.Q1)) {
    Filt f{xs.first, xs.second, subsampling_scale(xs.first, xs.second), 0, 0, false};
    f.k = std::min(f.j, p.log2T);
    p.psi1.push_back(f);
  }
  for (auto& xs : wavelet_bank(prm.J, prm.Q2)) {
    p.psi2.push_back(Filt{xs.first, xs.second, subsampling_scale(xs.first, xs.second), 0, 0, false});
  }
  const int32_t N1 = static_cast<int32_t>(p.psi1.size());
  if (N1 == 0) {
    err = "empty first-order filterbank";
    return JTFS_ERR_ARG;
  }
  p.N_fr = 2 * (1 << ceil_log2(N1));
  if ((1 << p.sF) > p.N_fr) {
    err = "F exceeds the padded frequential axis";
    return JTFS_ERR_ARG;
  }
  p.fr.push_back(Filt{0.0, p.sigmaF, p.sF, p.sF, 0, true});
  auto bank_fr = wavelet_bank(prm.J_fr, prm.Q_fr);
  for (int sign : {+1, -1}) {
    for (auto& xs : bank_fr) {
      Filt f{sign * xs.first, xs.second, subsampling_scale(xs.first, xs.second), 0, sign, false};
      // without frequential averaging a band-pass keeps its own stride 2^j_fr
      f.k = p.no_avg_fr ? f.j : std::min(f.j, p.sF);
      p.fr.push_back(f);
    }
  }
  for (int32_t g = 0; g < static_cast<int32_t>(p.fr.size()); ++g)
    if (p.fr[g].spin >= 0) p.fr_real.push_back(g);

  // Second-order groups: rows n1 with j1 < j2 are a prefix (j1 never decreases).
  for (int32_t n2 = 0; n2 < static_cast<int32_t>(p.psi2.size()); ++n2) {
    const Filt& b2 = p.psi2[n2];
    int32_t K = 0;
    while (K < N1 && p.psi1[K].j < b2.j) ++K;
    for (int32_t i = K; i < N1; ++i) {
      if (p.psi1[i].j < b2.j) {
        err = "first-order scales are not monotone";
        return JTFS_ERR_UNSUPPORTED;
      }
    }
    if (K == 0) continue;
    for (int32_t n1 = 0; n1 < K; ++n1) {
      int32_t k1 = p.psi1[n1].k;
      int32_t k2 = std::min(b2.j - k1, p.log2T);
      if (k1 + k2 > p.log2T || k1 + k2 != b2.j) {
        err = "second-order resolution coarser than T is not supported";
        return JTFS_ERR_UNSUPPORTED;
      }
    }
    p.groups.push_back(Grp{n2, b2.j, K, p.N_pad >> b2.j});
  }

  p.nf_pad = static_cast<int32_t>(p.N_pad >> p.log2T);
  p.Lf = p.nf_pad;
  int64_t f_hi;
  if (prm.periodic) {
    p.f_lo = 0;
    f_hi = p.nf_pad;
  } else {
    p.f_lo = static_cast<int32_t>((p.pad_left + p.T - 1) / p.T);
    f_hi = (p.pad_left + p.N + p.T - 1) / p.T;
  }
  p.n_frames = static_cast<int32_t>(f_hi - p.f_lo);
  // Kernel limits: transforms of at least 16 points, at most 128 kept frames.
  for (const Grp& g : p.groups) {
    if (g.L2 < 16) {
      err = "second-order signals shorter than 16 samples are not supported";
      return JTFS_ERR_UNSUPPORTED;
    }
  }
  for (const Filt& f : p.psi1) {
    if ((p.N_pad >> f.k) < 16) {
      err = "first-order signals shorter than 16 samples are not supported";
      return JTFS_ERR_UNSUPPORTED;
    }
  }
  if (p.nf_pad > 1024) {
    err = "more than 1024 padded frames (N_pad / T) are not supported";
    return JTFS_ERR_UNSUPPORTED;
  }
  if (p.n_frames > 128 || p.n_frames < 1) {
    err = "between 1 and 128 output frames are supported";
    return JTFS_ERR_UNSUPPORTED;
  }
  if (N1 > 256) {
    err = "at most 256 first-order filters are supported";
    return JTFS_ERR_UNSUPPORTED;
  }

  // ---- output layout: (order 0,) order 1, then order 2 by ascending n2
  // Kept log-frequency bins of a path: phi_F-averaged (stride 2^sF), or a band-pass
  // without frequential averaging at its own stride 2^k_fr.
  auto lam = [&](int32_t K, const Filt& f) {
    const int32_t k = (!f.lowpass && p.no_avg_fr) ? f.k : p.sF;
    return (K + (1 << k) - 1) >> k;
  };
  // kept samples on a grid of stride 2^j (unpadded part of the signal)
  auto kept = [&](int32_t j, int32_t& lo) {
    if (prm.periodic) {
      lo = 0;
      return static_cast<int32_t>(p.N_pad >> j);
    }
    const int64_t st = int64_t(1) << j;
    lo = static_cast<int32_t>((p.pad_left + st - 1) / st);
    return static_cast<int32_t>((p.pad_left + p.N + st - 1) / st - lo);
  };
  int64_t off = 0;
  if (prm.flags & JTFS_ZEROTH) {
    p.u0 = p.no_avg_local;
    jtfs_path r{0, -1, -1, 0, -1, -1, 1, p.u0 ? static_cast<int32_t>(p.N) : p.n_frames, off};
    p.paths.push_back(r);
    p.s0_off = off;
    p.w0 = prm.zeroth_weight;
    off += r.n_frames;
  }
  for (int32_t g : p.fr_real) {
    jtfs_path r{1, -1, g, p.fr[g].spin, -1, p.fr[g].j, lam(N1, p.fr[g]), p.n_frames, off};
    p.paths.push_back(r);
    off += int64_t(r.n_lambda) * r.n_frames;
  }
  for (Grp& grp : p.groups) {
    int32_t t_lo = p.f_lo;
    const int32_t n_t = p.no_avg_local ? kept(grp.j2, t_lo) : p.n_frames;
    grp.n_t = n_t;
    grp.t_lo = t_lo;
    for (int32_t g = 0; g < static_cast<int32_t>(p.fr.size()); ++g) {
      jtfs_path r{2, grp.n2, g, p.fr[g].spin, grp.j2, p.fr[g].j, lam(grp.K, p.fr[g]), n_t, off};
      p.paths.push_back(r);
      off += int64_t(r.n_lambda) * r.n_frames;
    }
  }
  p.n_coeff = off;

  // ---- twiddles exp(-2 pi i k / N_pad)
  p.tw.resize(static_cast<size_t>(p.N_pad));
  for (int64_t k = 0; k < p.N_pad; ++k) {
    double a = -2.0 * kPi * static_cast<double>(k) / static_cast<double>(p.N_pad);
    p.tw[k] = cfloat{static_cast<float>(std::cos(a)), static_cast<float>(std::sin(a))};
  }

  // ---- band tables
  for (const Filt& f : p.psi1) p.band_psi1.push_back(add_morlet_band(p, p.N_pad, f.xi, f.sigma, 0));
  {
    // summed squared response of the first-order bank on the non-negative frequencies
    // (the coloured-noise start normalises by it)
    std::vector<double> e(static_cast<size_t>(p.N_pad / 2 + 1), 0.0);
    for (int32_t bi : p.band_psi1) {
      const Band& b = p.bands[bi];
      for (int32_t d = 0; d < b.len; ++d) {
        const int64_t k = (static_cast<int64_t>(b.lo) + d) % b.L;
        if (k <= p.N_pad / 2) {
          const double h = p.bandvals[static_cast<size_t>(b.off + d)];
          e[static_cast<size_t>(k)] += h * h;
        }
      }
    }
    p.psi1_energy_max = static_cast<float>(*std::max_element(e.begin(), e.end()));
  }
  p.band_phiT.assign(static_cast<size_t>(p.log2T + 1), -1);
  for (const Filt& f : p.psi1) {
    if (p.band_phiT[f.k] < 0) p.band_phiT[f.k] = add_lowpass_band(p, p.N_pad >> f.k, p.sigmaT, f.k);
  }
  if (p.s0_off >= 0 && !p.u0) {
    if (p.band_phiT[0] < 0) p.band_phiT[0] = add_lowpass_band(p, p.N_pad, p.sigmaT, 0);
    p.s0_band = p.band_phiT[0];
    if (p.bands[static_cast<size_t>(p.s0_band)].len > 2 * p.Lf) {
      err = "phi_T spans more than two aliased blocks of the frame grid";
      return JTFS_ERR_UNSUPPORTED;
    }
  }
  for (const Grp& grp : p.groups) {
    const Filt& b2 = p.psi2[grp.n2];
    for (int32_t n1 = 0; n1 < grp.K; ++n1) {
      int32_t k1 = p.psi1[n1].k;
      auto key = std::make_pair(grp.n2, k1);
      if (!p.band_psi2.count(key)) p.band_psi2[key] = add_morlet_band(p, p.N_pad >> k1, b2.xi, b2.sigma, k1);
    }
  }

  // ---- frequential rows W: row r of filter g holds g[(r 2^k_g - n) mod N_fr], n < N1
  p.NW = static_cast<int32_t>(round_up(N1, 16));
  int32_t rows = 0;
  for (const Filt& f : p.fr) {
    FrFilter ff{};
    ff.row0 = rows;
    ff.M = p.N_fr >> f.k;
    ff.k = f.k;
    ff.lowpass = f.lowpass ? 1 : 0;
    ff.spin = f.spin;
    p.frf.push_back(ff);
    rows += static_cast<int32_t>(round_up(ff.M, 16));
  }
  p.R_total = rows;
  p.R_pad = static_cast<int32_t>(round_up(rows, 512));   // whole workgroup row blocks
  p.W.assign(static_cast<size_t>(p.R_pad) * p.NW, cfloat{0.f, 0.f});
  {
    const int32_t L = p.N_fr;
    std::vector<double> cs(L), sn(L);
    for (int32_t j = 0; j < L; ++j) {
      cs[j] = std::cos(2.0 * kPi * j / L);
      sn[j] = std::sin(2.0 * kPi * j / L);
    }
    std::vector<double> tap_mag(static_cast<size_t>(p.R_pad) * p.NW, 0.0);
    for (size_t g = 0; g < p.fr.size(); ++g) {
      const Filt& f = p.fr[g];
      std::vector<double> hat(L);
      if (f.lowpass) {
        Lowpass h(f.sigma, 0);
        for (int32_t m = 0; m < L; ++m) hat[m] = h(static_cast<double>(m) / L);
      } else {
        Morlet h(f.xi, f.sigma, 0);
        for (int32_t m = 0; m < L; ++m) hat[m] = h(static_cast<double>(m) / L);
      }
      // time (log-frequency) taps by a direct inverse DFT of the closed form
      std::vector<double> re(L), im(L);
      double peak = 0.0;
      for (int32_t d = 0; d < L; ++d) {
        double sr = 0.0, si = 0.0;
        for (int32_t m = 0; m < L; ++m) {
          int32_t e = static_cast<int32_t>((static_cast<int64_t>(m) * d) % L);
          sr += hat[m] * cs[e];
          si += hat[m] * sn[e];
        }
        re[d] = sr / L;
        im[d] = si / L;
        peak = std::max(peak, std::hypot(re[d], im[d]));
      }
      FrFilter& ff = p.frf[g];
      ff.taps = static_cast<int64_t>(p.tables.size());
      for (int32_t d = 0; d < L; ++d) {
        p.tables.push_back(static_cast<float>(re[d]));
        p.tables.push_back(static_cast<float>(im[d]));
      }
      for (int32_t r = 0; r < ff.M; ++r) {
        for (int32_t n = 0; n < N1; ++n) {
          int32_t d = static_cast<int32_t>(((static_cast<int64_t>(r) << f.k) - n) % L);
          if (d < 0) d += L;
          size_t idx = static_cast<size_t>(ff.row0 + r) * p.NW + n;
          p.W[idx] = cfloat{static_cast<float>(re[d]), static_cast<float>(im[d])};
          tap_mag[idx] = std::hypot(re[d], im[d]) / peak;
        }
      }
    }
    // algorithmic work: taps above 1e-7 of the filter's peak (the "banded" contraction)
    p.tap_count.assign(static_cast<size_t>(p.R_pad) * (N1 + 1), 0);
    for (int32_t r = 0; r < p.R_pad; ++r) {
      int32_t c = 0;
      for (int32_t n = 0; n < N1; ++n) {
        if (tap_mag[static_cast<size_t>(r) * p.NW + n] > 1e-7) ++c;
        p.tap_count[static_cast<size_t>(r) * (N1 + 1) + n + 1] = c;
      }
    }
    // per 16-row tile, the convex hull of columns with non-negligible taps, in steps of 4
    const int32_t n_tiles = p.R_pad / 16;
    p.rt_nrange.assign(static_cast<size_t>(2 * n_tiles), 0);
    for (int32_t t = 0; t < n_tiles; ++t) {
      int32_t lo = p.NW, hi = 0;
      for (int32_t r = t * 16; r < t * 16 + 16; ++r) {
        for (int32_t n = 0; n < N1; ++n) {
          if (tap_mag[static_cast<size_t>(r) * p.NW + n] > kTapThresh) {
            lo = std::min(lo, n);
            hi = std::max(hi, n + 1);
          }
        }
      }
      if (hi <= lo) {
        lo = hi = 0;
      } else {
        lo = lo / 4 * 4;
        hi = static_cast<int32_t>(round_up(hi, 4));
      }
      p.rt_nrange[2 * t] = lo;
      p.rt_nrange[2 * t + 1] = hi;
    }
  }
  for (size_t g = 0; g < p.fr.size(); ++g)
    p.frf[g].phiF = add_lowpass_time(p, p.frf[g].M, p.sigmaF, p.frf[g].k);

  // ---- workspace arrays (element counts) and row offsets
  p.z1_off.resize(N1);
  for (int32_t n1 = 0; n1 < N1; ++n1) {
    p.z1_off[n1] = p.z1_total;
    p.z1_total += p.N_pad >> p.psi1[n1].k;
  }
  const int32_t nF = p.n_frames;
  const int32_t n_rt = p.R_pad / 16;
  const int32_t FT = nF <= 16 ? 1 : nF <= 32 ? 2 : nF <= 64 ? 4 : 8;
  auto bucket_of = [](int32_t K) {
    const int32_t need = (K + 3) / 4;
    return need <= 4 ? 4 : need <= 8 ? 8 : need <= 16 ? 16 : need <= 32 ? 32 : 64;
  };
  auto bucket_index = [](int32_t S) { return S <= 4 ? 0 : S == 8 ? 1 : S == 16 ? 2 : S == 32 ? 3 : 4; };
  // Forward kernel per group: the row-tile-loop kernel (W tiles in LDS, each wave keeping
  // MT 16-time tiles of Y2 in registers) where its registers allow (S <= 32, FT <= 2),
  // otherwise the register-W kernel.
  auto fwd_loop = [&](int32_t S) { return S <= 32 && FT <= 2; };
  auto fwd_mt = [&](int32_t S) { return std::max(1, (FT == 1 ? tu.fwd_mt : 16) / S); };
  // With more than 32 frames, a group whose phi_T is short next to its row can still use the
  // row-tile-loop kernel: a chunk of TC times only reaches the frames whose centres lie
  // within the phi_T support of it, at most (TC - 1 + 2 halo) / 2^s_t + 2 of them; if that is
  // at most 32, the chunk pools into a 32-frame window starting at ceil((t0 - halo) / 2^s_t).
  // A workgroup covers 64 MT times per pass (registers); long rows take nsub passes per
  // chunk (at most 64 chunks), all pooled into the chunk's window.
  constexpr int32_t kWindow = 32;
  auto window_nsub = [&](int32_t S, const FreqGroup& fg) {
    if (FT <= 2 || S > 32) return 0;
    const int64_t sub = 64 * std::max(1, 16 / S);
    if (sub >= fg.L2) return 0;
    const int64_t nsub = std::max<int64_t>(1, fg.L2 / sub / 64);
    const int64_t TC = sub * nsub;
    if (TC >= fg.L2) return 0;
    return (TC - 1 + 2 * int64_t(fg.halo)) / (int64_t(1) << fg.s_t) + 2 <= kWindow ? static_cast<int32_t>(nsub) : 0;
  };
  for (const Grp& grp : p.groups) {
    FreqGroup fg{};
    fg.y2 = p.y2_total;
    fg.n_t = grp.n_t;
    fg.t_lo = grp.t_lo;
    fg.u2 = p.u2_total;
    if (p.no_avg_local) p.u2_total += static_cast<int64_t>(p.R_pad) * grp.n_t;
    fg.K = grp.K;
    fg.L2 = static_cast<int32_t>(grp.L2);
    fg.j2 = grp.j2;
    fg.s_t = p.log2T - grp.j2;
    fg.phiT = add_lowpass_time(p, grp.L2, p.sigmaT, grp.j2);
    {
      float peak = 0.f;
      for (int64_t d = 0; d < grp.L2; ++d) peak = std::max(peak, std::fabs(p.tables[fg.phiT + d]));
      int64_t h = 0;
      for (int64_t d = 0; d <= grp.L2 / 2; ++d)
        if (std::fabs(p.tables[fg.phiT + d]) > 1e-9f * peak ||
            std::fabs(p.tables[fg.phiT + (grp.L2 - d) % grp.L2]) > 1e-9f * peak)
          h = d;
      fg.halo = static_cast<int32_t>(h);
    }
    // Time chunks of the forward contraction: at least 256 samples (or the whole row), at
    // most 128 chunks per group (64 when there are more than 16 frames, whose partial rows
    // are longer). Smaller chunks give more workgroups to hide load latency; every chunk
    // adds a partial row to sum (measured on MI355X at N = 2^16 with 8 and 128 frames).
    const int64_t max_chunks = nF <= 16 ? 128 : 64;
    const int32_t S = bucket_of(grp.K);
    // Live row tiles: those whose band of non-negligible taps meets the group's K rows
    // (the others contribute nothing to V; their pooled rows are zero). Work is split
    // over these only.
    fg.lt0 = static_cast<int32_t>(p.live_rt.size());
    for (int32_t t = 0; t < n_rt; ++t)
      if (std::min<int32_t>(p.rt_nrange[2 * t + 1], (grp.K + 3) & ~3) > p.rt_nrange[2 * t]) p.live_rt.push_back(t);
    if (static_cast<int32_t>(p.live_rt.size()) == fg.lt0) p.live_rt.push_back(0);   // (a dead tile: zeros)
    fg.nlt = static_cast<int32_t>(p.live_rt.size()) - fg.lt0;
    const int32_t wnsub = window_nsub(S, fg);
    fg.fw = wnsub > 0 ? kWindow : 0;
    fg.nsub = std::max(1, wnsub);
    if (fwd_loop(S) || fg.fw > 0) {
      // a workgroup's four waves cover 64 MT consecutive times per pass, nsub passes per
      // chunk (the last chunk may be short)
      fg.TC = 64 * (fg.fw > 0 ? std::max(1, 16 / S) : fwd_mt(S)) * fg.nsub;
      fg.n_tc = static_cast<int32_t>(std::max<int64_t>(1, grp.L2 / fg.TC));
      // about 256 workgroups per group: more row splits re-load the same Y2 operands
      // (measured on MI355X, config 2: targets 16..4096 swept, 256 fastest)
      const int32_t want = (tu.fwd_rows_k[bucket_index(S)] + fg.n_tc - 1) / fg.n_tc;
      const int32_t rs = std::max(1, std::min(want, fg.nlt / 4));
      fg.rt_fwd = (fg.nlt + rs - 1) / rs;
    } else {
      fg.TC = static_cast<int32_t>(std::max<int64_t>(std::min<int64_t>(grp.L2, 256), grp.L2 / max_chunks));
      fg.n_tc = static_cast<int32_t>(grp.L2 / fg.TC);
      fg.rt_fwd = 0;
    }
    fg.part = p.part_total;
    p.part_total += static_cast<int64_t>(fg.n_tc) * p.R_pad * (fg.fw > 0 ? fg.fw : nF);
    fg.psum = fg.fw > 0 ? -1 : p.psum_total;
    if (fg.fw == 0) p.psum_total += static_cast<int64_t>(p.R_pad) * nF;
    fg.dP = p.dP_total;
    p.dP_total += static_cast<int64_t>(p.R_pad) * nF;
    fg.n_tb = static_cast<int32_t>((grp.L2 + 63) / 64);
    int32_t want = (tu.bwd_rows_k[bucket_index(S)] + fg.n_tb - 1) / fg.n_tb;
    fg.RS = std::max(1, std::min(want, fg.nlt / 4));
    fg.rt_per_split = (fg.nlt + fg.RS - 1) / fg.RS;
    fg.RS = (fg.nlt + fg.rt_per_split - 1) / fg.rt_per_split;
    fg.dYpart = p.dYpart_total;
    p.dYpart_total += static_cast<int64_t>(fg.RS) * grp.K * grp.L2;
    p.y2_total += static_cast<int64_t>(grp.K) * grp.L2;
    p.fgroups.push_back(fg);
  }
  if (p.u2_total > (int64_t(1) << 30)) {
    err = "the second-order output without time averaging exceeds 2^30 values";
    return JTFS_ERR_UNSUPPORTED;
  }
  for (const FreqGroup& fg : p.fgroups) {
    for (size_t g = 0; g < p.frf.size(); ++g) {
      const FrFilter& ff = p.frf[g];
      p.mac_dense += double(ff.M) * fg.K * fg.L2;
      p.mac_pool += double(ff.M) * fg.L2 * nF;
      for (int32_t r = 0; r < ff.M; ++r)
        p.mac_banded += double(p.tap_count[static_cast<size_t>(ff.row0 + r) * (N1 + 1) + fg.K]) * fg.L2;
    }
    for (int32_t t = 0; t < p.R_pad / 16; ++t) {
      const int32_t lo = p.rt_nrange[2 * t];
      const int32_t hi = std::min<int32_t>(p.rt_nrange[2 * t + 1], (fg.K + 3) & ~3);
      if (hi > lo) p.mac_exec += 16.0 * (hi - lo) * fg.L2;
    }
  }
  // Forward items, one launch per kernel shape: S = k-steps covering the group's rows
  // (a power of two), FT = 16-frame tiles, RW = 16-row tiles per wave chosen so that the
  // register-resident operands of a wave stay near 100 VGPRs.
  {
    for (int32_t S = 4; S <= 64; S *= 2) {
      // windowed groups: the row-tile-loop kernel with two frame tiles
      if (S <= 32 && FT > 2) {
        SigPlan::FwdLaunch fl{S, 0, 2, static_cast<int32_t>(p.fwd_items.size()), 0, 0, std::max(1, 16 / S)};
        for (int32_t gi = 0; gi < static_cast<int32_t>(p.fgroups.size()); ++gi) {
          const FreqGroup& fg = p.fgroups[gi];
          if (bucket_of(fg.K) != S || fg.fw == 0) continue;
          const int32_t nrs = (fg.nlt + fg.rt_fwd - 1) / fg.rt_fwd;
          for (int32_t tc = 0; tc < fg.n_tc; ++tc)
            for (int32_t rs = 0; rs < nrs; ++rs) p.fwd_items.push_back(FwdItem{gi, rs, tc, 0});
        }
        fl.nitems = static_cast<int32_t>(p.fwd_items.size()) - fl.item0;
        if (fl.nitems > 0) p.fwd_launches.push_back(fl);
      }
      if (fwd_loop(S)) {
        // items (group, row split, time chunk)
        SigPlan::FwdLaunch fl{S, 0, FT, static_cast<int32_t>(p.fwd_items.size()), 0, 0, fwd_mt(S)};
        for (int32_t gi = 0; gi < static_cast<int32_t>(p.fgroups.size()); ++gi) {
          const FreqGroup& fg = p.fgroups[gi];
          if (bucket_of(fg.K) != S) continue;
          const int32_t nrs = (fg.nlt + fg.rt_fwd - 1) / fg.rt_fwd;
          for (int32_t tc = 0; tc < fg.n_tc; ++tc)
            for (int32_t rs = 0; rs < nrs; ++rs) p.fwd_items.push_back(FwdItem{gi, rs, tc, 0});
        }
        fl.nitems = static_cast<int32_t>(p.fwd_items.size()) - fl.item0;
        if (fl.nitems > 0) p.fwd_launches.push_back(fl);
        continue;
      }
      int32_t RW = 2;   // at most two row tiles per wave (measured: four cost occupancy)
      while (RW > 1 && RW * (2 * S + 4 * FT) > 100) RW /= 2;
      SigPlan::FwdLaunch fl{S, RW, FT, static_cast<int32_t>(p.fwd_items.size()), 0, 0, 0};
      for (int32_t gi = 0; gi < static_cast<int32_t>(p.fgroups.size()); ++gi) {
        const FreqGroup& fg = p.fgroups[gi];
        if (bucket_of(fg.K) != S || fg.fw > 0) continue;
        for (int32_t tc = 0; tc < fg.n_tc; ++tc)
          for (int32_t rb = 0; rb < p.R_pad / (64 * RW); ++rb) p.fwd_items.push_back(FwdItem{gi, rb, tc, 0});
      }
      fl.nitems = static_cast<int32_t>(p.fwd_items.size()) - fl.item0;
      // Items come in runs of R_pad / (64 RW) row blocks sharing one time chunk; the
      // kernel gives each run to one XCD and consecutive runs to different XCDs, so the
      // count is padded to a multiple of 8 runs.
      // (measured: neutral in time, about 10x less HBM traffic for S <= 16; for S >= 32
      // the few long runs unbalance the XCDs, so those launches keep plain round-robin)
      fl.run = S >= 32 ? 1 : p.R_pad / (64 * RW);
      while (fl.nitems % (8 * fl.run)) {
        p.fwd_items.push_back(FwdItem{-1, 0, 0, 0});
        ++fl.nitems;
      }
      if (fl.nitems > 0) p.fwd_launches.push_back(fl);
    }
  }
  // Backward items bucketed like the forward, so that a group's launch sizes its
  // registers and its staged W tiles (4 S columns) to its own row count.
  for (int32_t S = 4; S <= 64; S *= 2) {
    SigPlan::BwdLaunch bl{S, static_cast<int32_t>(p.bwd_items.size()), 0};
    for (int32_t gi = 0; gi < static_cast<int32_t>(p.fgroups.size()); ++gi) {
      const FreqGroup& fg = p.fgroups[gi];
      const int32_t need = (fg.K + 3) / 4;
      const int32_t bucket = need <= 4 ? 4 : need <= 8 ? 8 : need <= 16 ? 16 : need <= 32 ? 32 : 64;
      if (bucket != S) continue;
      for (int32_t tb = 0; tb < fg.n_tb; ++tb)
        for (int32_t rs = 0; rs < fg.RS; ++rs) p.bwd_items.push_back(BwdItem{gi, tb, rs, 0});
    }
    bl.nitems = static_cast<int32_t>(p.bwd_items.size()) - bl.item0;
    if (bl.nitems > 0) p.bwd_launches.push_back(bl);
  }

  // ---- row jobs of the time-axis stages, grouped by transform length
  // Rows of a stage are sorted by length; lengths above 4096 become two-pass launches,
  // the others workgroup tasks of one launch per stage (4096 / n rows per workgroup).
  auto emit = [&](int stage, std::vector<RowJob> js) {
    std::stable_sort(js.begin(), js.end(), [](const RowJob& a, const RowJob& b) { return a.n > b.n; });
    p.task_jobs0[stage] = static_cast<int32_t>(p.jobs.size());
    p.task_jobs1[stage] = static_cast<int32_t>(p.jobs.size() + js.size());
    p.task0[stage] = static_cast<int32_t>(p.tasks.size());
    int64_t stage_scr = 0;
    size_t i = 0;
    while (i < js.size()) {
      size_t j = i;
      while (j < js.size() && js[j].n == js[i].n) ++j;
      Launch l{stage, js[i].n, static_cast<int32_t>(p.jobs.size()), static_cast<int32_t>(j - i)};
      for (size_t q = i; q < j; ++q) p.jobs.push_back(js[q]);
      if (l.n > 4096) {
        stage_scr += int64_t(l.n) * l.njobs;
        p.launches[stage].push_back(l);
      } else {
        const int32_t per = 4096 / l.n;
        int32_t log2n = 0;
        while ((1 << log2n) < l.n) ++log2n;
        for (int32_t r = 0; r < l.njobs; r += per)
          p.tasks.push_back(RowTask{l.job0 + r, std::min(per, l.njobs - r), log2n, 0});
      }
      i = j;
    }
    p.ntask[stage] = static_cast<int32_t>(p.tasks.size()) - p.task0[stage];
    // two-pass rows: one scratch row each, all lengths in one launch per pass
    p.scr_elems = std::max(p.scr_elems, stage_scr);
    for (int pass = 1; pass <= 2; ++pass) {
      (pass == 1 ? p.split1_0 : p.split2_0)[stage] = static_cast<int32_t>(p.stasks.size());
      int64_t scr = 0;
      for (const Launch& l : p.launches[stage]) {
        int32_t log2n = 0;
        while ((1 << log2n) < l.n) ++log2n;
        // both factors between 16 (one radix-16 pass per thread) and 4096 (one LDS tile)
        const int32_t log2A = std::min(std::min(12, log2n - 4), std::max(std::max(4, log2n - 12), log2n / 2 + tu.split_bias));
        const SplitGeom g = split_geom(log2n, log2A);
        const int32_t nblk = pass == 1 ? (1 << g.log2A) >> g.log2C1 : (1 << g.log2B) >> g.log2C2;
        for (int32_t r = 0; r < l.njobs; ++r, scr += l.n)
          for (int32_t b = 0; b < nblk; ++b) p.stasks.push_back(SplitTask{l.job0 + r, log2n, b, log2A, scr, RowJob{}});
      }
      (pass == 1 ? p.split1_n : p.split2_n)[stage] =
          static_cast<int32_t>(p.stasks.size()) - (pass == 1 ? p.split1_0 : p.split2_0)[stage];
    }
  };
  auto job = [](int64_t src, int64_t dst, int64_t aux, int32_t band, int32_t src_len, int32_t n, int32_t shift) {
    RowJob r{};
    r.src = src;
    r.dst = dst;
    r.aux = aux;
    r.band = band;
    r.src_len = src_len;
    r.n = n;
    r.shift = shift;
    r.t0 = r.t1 = 0;
    return r;
  };
  const int32_t Np = static_cast<int32_t>(p.N_pad);
  emit(ST_XHAT, {job(0, 0, 0, -1, Np, Np, 0)});
  {
    std::vector<RowJob> a, b;
    for (int32_t n1 = 0; n1 < N1; ++n1) {
      int32_t L1 = Np >> p.psi1[n1].k;
      a.push_back(job(0, p.z1_off[n1], 0, p.band_psi1[n1], Np, L1, p.psi1[n1].k));
      b.push_back(job(p.z1_off[n1], p.z1_off[n1], 0, -1, L1, L1, 0));
    }
    emit(ST_L1Z, a);
    emit(ST_L1UH, b);
  }
  {
    std::vector<RowJob> a, b;
    for (size_t gi = 0; gi < p.groups.size(); ++gi) {
      const Grp& grp = p.groups[gi];
      const FreqGroup& fg = p.fgroups[gi];
      for (int32_t n1 = 0; n1 < grp.K; ++n1) {
        int32_t k1 = p.psi1[n1].k;
        int32_t L1 = Np >> k1;
        a.push_back(job(p.z1_off[n1], fg.y2 + int64_t(n1) * fg.L2, 0, p.band_psi2.at({grp.n2, k1}), L1, fg.L2,
                        grp.j2 - k1));
        // the row-split partials are summed into split 0 before this stage
        b.push_back(job(fg.dYpart + int64_t(n1) * fg.L2, fg.y2 + int64_t(n1) * fg.L2, 0, -1, fg.L2, fg.L2, 0));
      }
    }
    emit(ST_L2Y, a);
    emit(ST_BYH, b);
  }
  {
    // adjoint gather per n1: second-order terms (dY2hat rows), then the phi_T term (dS1hat)
    std::vector<RowJob> a, b;
    const int64_t dS1h_base = p.y2_total;   // dS1hat rows follow the dY2hat stacks
    for (int32_t n1 = 0; n1 < N1; ++n1) {
      int32_t k1 = p.psi1[n1].k;
      int32_t L1 = Np >> k1;
      RowJob r = job(0, p.z1_off[n1], 0, -1, L1, L1, 0);
      r.t0 = static_cast<int32_t>(p.terms.size());
      for (size_t gi = 0; gi < p.groups.size(); ++gi) {
        const Grp& grp = p.groups[gi];
        if (n1 >= grp.K) continue;
        GatherTerm t{p.fgroups[gi].y2 + int64_t(n1) * p.fgroups[gi].L2, p.band_psi2.at({grp.n2, k1}),
                     p.fgroups[gi].L2};
        p.terms.push_back(t);
      }
      p.terms.push_back(GatherTerm{dS1h_base + int64_t(n1) * p.Lf, p.band_phiT[k1], p.Lf});
      r.t1 = static_cast<int32_t>(p.terms.size());
      a.push_back(r);
      b.push_back(job(p.z1_off[n1], p.z1_off[n1], p.z1_off[n1], -1, L1, L1, 0));
    }
    emit(ST_BU, a);
    emit(ST_BZH, b);
  }
  {
    RowJob r = job(0, 0, 0, -1, Np, Np, 0);
    r.t0 = static_cast<int32_t>(p.terms.size());
    for (int32_t n1 = 0; n1 < N1; ++n1)
      p.terms.push_back(GatherTerm{p.z1_off[n1], p.band_psi1[n1], Np >> p.psi1[n1].k});
    // zeroth order: phi_T times the DFT of the padded dS0 row, kept after the dZ1hat rows
    if (p.s0_off >= 0 && !p.u0) p.terms.push_back(GatherTerm{p.z1_total, p.s0_band, p.Lf});
    r.t1 = static_cast<int32_t>(p.terms.size());
    p.bx_job = static_cast<int32_t>(p.jobs.size());   // emit() appends this single row next
    emit(ST_BX, {r});
  }
  // Segment lists of the adjoint gathers (rows with a term range).
  for (RowJob& j : p.jobs) {
    if (j.t1 <= j.t0) continue;
    const int32_t nseg = (j.n + 511) / 512;
    const int32_t seg0 = static_cast<int32_t>(p.segs.size() / 2);
    for (int32_t sg = 0; sg < nseg; ++sg) {
      const int64_t a = int64_t(sg) * 512, b = std::min<int64_t>(j.n, a + 512);
      const int32_t first = static_cast<int32_t>(p.segterms.size());
      for (int32_t t = j.t0; t < j.t1; ++t) {
        const Band& bd = p.bands[p.terms[t].band];
        const int64_t L = bd.L;
        const bool meets = L != j.n || bd.len >= L || ((a - bd.lo) % L + L) % L < bd.len || ((bd.lo - a) % L + L) % L < b - a;
        if (meets) p.segterms.push_back(SegTerm{p.terms[t].src, bd.off, bd.lo, bd.len, bd.L, p.terms[t].src_len});
      }
      p.segs.push_back(first);
      p.segs.push_back(static_cast<int32_t>(p.segterms.size()) - first);
    }
    j.t0 = seg0;
    j.t1 = seg0 + nseg;
  }
  // Chunks of the bin-parallel gathers: every row of the stage, 256 bins at a time.
  for (int st : {ST_BU, ST_BX}) {
    p.gch0[st] = static_cast<int32_t>(p.gchunks.size() / 2);
    const int32_t j0 = st == ST_BX ? p.bx_job : p.task_jobs0[st];
    const int32_t j1 = st == ST_BX ? p.bx_job + 1 : p.task_jobs1[st];
    for (int32_t j = j0; j < j1; ++j)
      for (int32_t m0 = 0; m0 < p.jobs[j].n; m0 += 256) {
        p.gchunks.push_back(j);
        p.gchunks.push_back(m0);
      }
    p.gchn[st] = static_cast<int32_t>(p.gchunks.size() / 2) - p.gch0[st];
  }
  p.s1_job0 = static_cast<int32_t>(p.jobs.size());
  for (int32_t n1 = 0; n1 < N1; ++n1) {
    int32_t k1 = p.psi1[n1].k;
    p.jobs.push_back(job(p.z1_off[n1], int64_t(n1) * p.nf_pad, 0, p.band_phiT[k1], Np >> k1, p.Lf, p.log2T - k1));
  }

  // Inline copies: each job carries its band, each two-pass task its job.
  for (RowJob& j : p.jobs) j.b = j.band >= 0 ? p.bands[static_cast<size_t>(j.band)] : Band{0, 0, 0, 0, 0};
  for (SplitTask& t : p.stasks) t.j = p.jobs[static_cast<size_t>(t.job)];

  // The Fourier-subsampling gathers read, per output bin, one or two aliased blocks of a
  // non-empty band (the subsampling rule keeps a filter's band within two periods of the
  // coarser grid).
  for (const RowJob& j : p.jobs) {
    if (j.band < 0 || j.n <= 0) continue;
    const int32_t len = p.bands[static_cast<size_t>(j.band)].len;
    if (len < 1 || len > 2 * j.n) {
      err = "a filter band is empty or spans more than two periods of its subsampled grid";
      return JTFS_ERR_UNSUPPORTED;
    }
  }
  // The adjoint gathers read a term's band at an index clamped into it: no term band may
  // be empty.
  for (const SegTerm& t : p.segterms)
    if (t.len < 1 || t.len > t.L) {
      err = "an adjoint-gather term has an empty filter band";
      return JTFS_ERR_UNSUPPORTED;
    }

  // ---- workspace layout (bytes, 256-aligned regions)
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += (bytes + 255) / 256 * 256;
    return at;
  };
  WsLayout& w = p.ws;
  w.Xh = take(sizeof(cfloat) * p.N_pad);
  w.Z1 = take(sizeof(cfloat) * p.z1_total);
  w.U1h = take(sizeof(cfloat) * p.z1_total);
  w.S1 = take(sizeof(float) * N1 * p.nf_pad);
  w.Y2 = take(sizeof(cfloat) * std::max<int64_t>(p.y2_total, 1));
  // The frequential forward's pooled partials are dead once φ_F pooling has read them;
  // the backward's dY2 row-split partials live from the frequential backward to the
  // layer-2 adjoint DFT. No stage uses both, so they share one region.
  w.part = take(std::max(sizeof(float) * std::max<int64_t>(p.part_total, 1),
                         sizeof(cfloat) * std::max<int64_t>(p.dYpart_total, 1)));
  w.psum = take(sizeof(float) * std::max<int64_t>(p.psum_total, 1));
  w.scr = take(sizeof(cfloat) * std::max<int64_t>(p.scr_elems, 1));
  w.S = take(sizeof(float) * p.n_coeff);
  w.dS = take(sizeof(float) * p.n_coeff);
  w.o1 = take(sizeof(cfloat) * p.R_pad * p.n_frames);
  w.u2 = take(sizeof(float) * std::max<int64_t>(p.u2_total, 1));
  w.fwd_end = o;
  w.dP = take(sizeof(float) * std::max<int64_t>(p.dP_total, 1));
  w.dYpart = w.part;
  w.dYh = take(sizeof(cfloat) * (p.y2_total + int64_t(N1) * p.Lf));
  w.dS1p = take(sizeof(float) * p.fr_real.size() * N1 * p.nf_pad);
  w.dU1 = take(sizeof(float) * p.z1_total);
  w.dZh = take(sizeof(cfloat) * (p.z1_total + (p.s0_off >= 0 ? p.Lf : 0)));
  w.dXh = take(sizeof(cfloat) * p.N_pad);
  w.grad = take(sizeof(float) * p.N);
  w.dv = take(sizeof(cfloat) * std::max<int64_t>(p.u2_total, 1));
  w.bwd_end = o;
  return JTFS_OK;
}

}  // namespace jtfs
