// Tile-schedule autotuner (jtfs_autotune, include/jtfs.h): a coordinate search over the
// fields of jtfs_tuning, each candidate timed as one forward + backward of a seeded
// synthetic signal on the current device. It is a client of the public C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/jtfs.h"

namespace jtfs {
jtfs_status report(jtfs_status s, const std::string& msg);
}

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t ensure(size_t bytes) {
    if (bytes <= n) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    const hipError_t e = hipMalloc(&p, bytes);
    if (e == hipSuccess) n = bytes;
    return e;
  }
};

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Three tones with slow amplitude modulation plus a little noise from a 64-bit LCG.
std::vector<float> synth(int64_t n) {
  std::vector<float> x(static_cast<size_t>(n));
  uint64_t st = 0x9E3779B97F4A7C15ull;
  for (int64_t i = 0; i < n; ++i) {
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    const double noise = (static_cast<double>(st >> 11) / 9007199254740992.0 - 0.5) * 0.06;
    const double t = static_cast<double>(i);
    const double env = 0.5 * (1.0 + std::sin(2.0 * M_PI * t / 9000.0));
    x[static_cast<size_t>(i)] = static_cast<float>(
        env * (std::sin(0.031 * t) + 0.5 * std::sin(0.0713 * t + 1.0) + 0.33 * std::sin(0.1937 * t + 2.0)) + noise);
  }
  return x;
}

struct Bench {
  const jtfs_params* sig;
  int32_t batch;
  hipStream_t st;
  DevBuf x, S, dx, ws;
  Events ev;
  std::vector<float> host;

  // Median of five timed forward + backward runs (after one untimed run) of a plan.
  jtfs_status time(const jtfs_tuning& t, double& ms) {
    jtfs_plan_t plan = nullptr;
    jtfs_status r = jtfs_plan_tuned(sig, batch, &t, &plan);
    if (r != JTFS_OK) return r;
    jtfs_plan_info info;
    r = jtfs_plan_query(plan, &info);
    if (r == JTFS_OK) r = run(plan, info, ms);
    jtfs_plan_destroy(plan);
    return r;
  }

  jtfs_status run(jtfs_plan_t plan, const jtfs_plan_info& info, double& ms) {
    const size_t nx = sizeof(float) * static_cast<size_t>(info.n_samples_total);
    const size_t ns = sizeof(float) * static_cast<size_t>(info.n_coeff_total);
    if (x.ensure(nx) != hipSuccess || S.ensure(ns) != hipSuccess || dx.ensure(nx) != hipSuccess ||
        ws.ensure(std::max<size_t>(info.ws_backward, 1)) != hipSuccess)
      return jtfs::report(JTFS_ERR_NOMEM, "autotune: device allocation failed");
    if (host.size() != static_cast<size_t>(info.n_samples_total)) {
      host = synth(info.n_samples_total);
      if (hipMemcpyAsync(x.p, host.data(), nx, hipMemcpyHostToDevice, st) != hipSuccess)
        return jtfs::report(JTFS_ERR_HIP, "autotune: upload failed");
    }
    auto once = [&]() {
      jtfs_status r = jtfs_forward(plan, static_cast<float*>(x.p), static_cast<float*>(S.p), ws.p, ws.n, st);
      if (r == JTFS_OK)
        r = jtfs_backward(plan, static_cast<float*>(x.p), static_cast<float*>(S.p), static_cast<float*>(dx.p), ws.p,
                          ws.n, JTFS_REUSE_FORWARD, st);
      return r;
    };
    jtfs_status r = once();
    if (r != JTFS_OK) return r;
    std::vector<double> t;
    for (int rep = 0; rep < 5; ++rep) {
      if (hipEventRecord(ev.a, st) != hipSuccess) return jtfs::report(JTFS_ERR_HIP, "autotune: event failed");
      if ((r = once()) != JTFS_OK) return r;
      float e = 0.f;
      if (hipEventRecord(ev.b, st) != hipSuccess || hipEventSynchronize(ev.b) != hipSuccess ||
          hipEventElapsedTime(&e, ev.a, ev.b) != hipSuccess)
        return jtfs::report(JTFS_ERR_HIP, "autotune: timing failed");
      t.push_back(e);
    }
    std::sort(t.begin(), t.end());
    ms = t[2];
    return JTFS_OK;
  }
};

}  // namespace

extern "C" jtfs_status jtfs_autotune(const jtfs_params* signals, int32_t batch, jtfs_stream_t stream, jtfs_tuning* out,
                                     double* ms) {
  if (!signals || batch < 1 || !out) return jtfs::report(JTFS_ERR_ARG, "NULL argument or empty batch");
  Bench b{signals, batch, static_cast<hipStream_t>(stream), {}, {}, {}, {}, {}, {}};
  if (hipEventCreate(&b.ev.a) != hipSuccess || hipEventCreate(&b.ev.b) != hipSuccess)
    return jtfs::report(JTFS_ERR_HIP, "autotune: event creation failed");
  jtfs_tuning cur{256, 32, 128, 0, {0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};
  double best = 0.0;
  jtfs_status r = b.time(cur, best);
  if (r != JTFS_OK) return r;
  // a candidate replaces the current choice only if clearly faster (run-to-run spread of
  // the median is a few tenths of a percent)
  auto consider = [&](const jtfs_tuning& cand) -> jtfs_status {
    double t = 0.0;
    const jtfs_status rr = b.time(cand, t);
    if (rr != JTFS_OK) return rr;
    if (t < 0.995 * best) {
      best = t;
      cur = cand;
    }
    return JTFS_OK;
  };
  struct Knob {
    int32_t jtfs_tuning::*field;
    std::vector<int32_t> values;
  };
  const Knob knobs[] = {{&jtfs_tuning::fwd_rows, {128, 512, 1024}},
                        {&jtfs_tuning::fwd_mt, {16}},
                        {&jtfs_tuning::bwd_rows, {128, 512, 1024}},
                        {&jtfs_tuning::split_bias, {-1, 1}}};
  for (const Knob& k : knobs) {
    const jtfs_tuning base = cur;
    for (int32_t v : k.values) {
      jtfs_tuning cand = base;
      cand.*(k.field) = v;
      if ((r = consider(cand)) != JTFS_OK) return r;
    }
  }
  // then each k-step bucket's own row targets (its kernels fit a different number of
  // workgroups per CU); a bucket without groups leaves the time unchanged and keeps 0
  const int32_t per_bucket[] = {64, 128, 256, 512, 1024};
  for (int bk = 0; bk < JTFS_N_BUCKETS; ++bk) {
    for (int which = 0; which < 2; ++which) {
      const jtfs_tuning base = cur;
      const int32_t global = which == 0 ? base.fwd_rows : base.bwd_rows;
      for (int32_t v : per_bucket) {
        if (v == global) continue;
        jtfs_tuning cand = base;
        (which == 0 ? cand.fwd_rows_k : cand.bwd_rows_k)[bk] = v;
        if ((r = consider(cand)) != JTFS_OK) return r;
      }
    }
  }
  *out = cur;
  if (ms) *ms = best;
  return JTFS_OK;
}
