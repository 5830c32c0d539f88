// C ABI of the JTFS library (include/jtfs.h): plan objects, lazy per-device upload of
// the plan tables, argument checks and the order of the kernel stages.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/jtfs.h"
#include "dec.hpp"
#include "device.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace {

thread_local std::string g_last_error;

jtfs_status fail(jtfs_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

// Device copy of one signal's tables inside the plan's arena.
struct SigTables {
  const jtfs::c32* tw;
  const float* bandvals;
  const jtfs::Band* bands;
  const float* tables;
  const jtfs::c32* W;
  const int32_t* rt_nrange;
  const jtfs::FrFilter* frf;
  const jtfs::FreqGroup* fgroups;
  const jtfs::FwdItem* fwd_items;
  const jtfs::BwdItem* bwd_items;
  const jtfs::RowJob* jobs;
  const jtfs::RowTask* tasks;
  const int32_t* segs;
  const jtfs::SegTerm* segterms;
  const jtfs::SplitTask* stasks;
  const int64_t* s_off;
  const int32_t* band_psi1;   // per first-order filter: its band (level 0, N_pad grid)
  const int32_t* gchunks;
  const int32_t* live_rt;
};

struct DeviceArena {
  void* base = nullptr;
  std::vector<SigTables> sig;
  // streams over which the signals of a batch are spread, and the fork / join events
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> joins;
  hipEvent_t fork = nullptr;
};

constexpr int kMaxStreams = 8;

}  // namespace

struct jtfs_plan_s {
  std::vector<jtfs::SigPlan> sig;
  std::vector<std::vector<int64_t>> block_off;   // per signal: the s_off table
  std::vector<int64_t> x_off, s_off;             // batch + 1
  std::vector<size_t> ws_off;                    // per signal segment start (bytes)
  size_t ws_fwd = 0, ws_bwd = 0;
  size_t ws_fwd_shared = 0, ws_bwd_shared = 0;   // the largest signal's forward / backward segment
  int64_t n_total = 0, c_total = 0;
  std::mutex mu;
  std::map<int, DeviceArena> dev;
  // stage timing: (stage, start, stop) event triples recorded since the last read
  uint32_t timing = 0;   // bit i: bracket stage i
  struct Mark {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  ~jtfs_plan_s() {
    for (auto& m : marks) {
      (void)hipEventDestroy(m.a);
      (void)hipEventDestroy(m.b);
    }
    for (auto& kv : dev) {
      int cur = 0;
      if (hipGetDevice(&cur) == hipSuccess && hipSetDevice(kv.first) == hipSuccess) {
        for (hipStream_t s : kv.second.streams) (void)hipStreamDestroy(s);
        for (hipEvent_t e : kv.second.joins) (void)hipEventDestroy(e);
        if (kv.second.fork) (void)hipEventDestroy(kv.second.fork);
        (void)hipFree(kv.second.base);
        (void)hipSetDevice(cur);
      }
    }
  }
};

namespace {

template <class T>
void append_bytes(std::vector<char>& buf, std::vector<size_t>& offs, const std::vector<T>& v) {
  size_t at = (buf.size() + 255) / 256 * 256;
  buf.resize(at + sizeof(T) * v.size());
  if (!v.empty()) std::memcpy(buf.data() + at, v.data(), sizeof(T) * v.size());
  offs.push_back(at);
}

// Uploads the plan tables to the current device once; returns the arena.
jtfs_status device_tables(jtfs_plan_t p, const DeviceArena** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(JTFS_ERR_HIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lock(p->mu);
  auto it = p->dev.find(dev);
  if (it != p->dev.end()) {
    *out = &it->second;
    return JTFS_OK;
  }
  std::vector<char> buf;
  std::vector<std::vector<size_t>> offs(p->sig.size());
  for (size_t s = 0; s < p->sig.size(); ++s) {
    const jtfs::SigPlan& sp = p->sig[s];
    auto& o = offs[s];
    append_bytes(buf, o, sp.tw);
    append_bytes(buf, o, sp.bandvals);
    append_bytes(buf, o, sp.bands);
    append_bytes(buf, o, sp.tables);
    append_bytes(buf, o, sp.W);
    append_bytes(buf, o, sp.rt_nrange);
    append_bytes(buf, o, sp.frf);
    append_bytes(buf, o, sp.fgroups);
    append_bytes(buf, o, sp.fwd_items);
    append_bytes(buf, o, sp.bwd_items);
    append_bytes(buf, o, sp.jobs);
    append_bytes(buf, o, p->block_off[s]);
    append_bytes(buf, o, sp.tasks);
    append_bytes(buf, o, sp.segs);
    append_bytes(buf, o, sp.segterms);
    append_bytes(buf, o, sp.stasks);
    append_bytes(buf, o, sp.band_psi1);
    append_bytes(buf, o, sp.gchunks);
    append_bytes(buf, o, sp.live_rt);
  }
  DeviceArena a;
  if (hipMalloc(&a.base, buf.size() + 256) != hipSuccess) return fail(JTFS_ERR_NOMEM, "hipMalloc of plan tables failed");
  if (hipMemcpy(a.base, buf.data(), buf.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(a.base);
    return fail(JTFS_ERR_HIP, "upload of plan tables failed");
  }
  char* b = static_cast<char*>(a.base);
  for (size_t s = 0; s < p->sig.size(); ++s) {
    const auto& o = offs[s];
    SigTables t;
    t.tw = reinterpret_cast<const jtfs::c32*>(b + o[0]);
    t.bandvals = reinterpret_cast<const float*>(b + o[1]);
    t.bands = reinterpret_cast<const jtfs::Band*>(b + o[2]);
    t.tables = reinterpret_cast<const float*>(b + o[3]);
    t.W = reinterpret_cast<const jtfs::c32*>(b + o[4]);
    t.rt_nrange = reinterpret_cast<const int32_t*>(b + o[5]);
    t.frf = reinterpret_cast<const jtfs::FrFilter*>(b + o[6]);
    t.fgroups = reinterpret_cast<const jtfs::FreqGroup*>(b + o[7]);
    t.fwd_items = reinterpret_cast<const jtfs::FwdItem*>(b + o[8]);
    t.bwd_items = reinterpret_cast<const jtfs::BwdItem*>(b + o[9]);
    t.jobs = reinterpret_cast<const jtfs::RowJob*>(b + o[10]);
    t.s_off = reinterpret_cast<const int64_t*>(b + o[11]);
    t.tasks = reinterpret_cast<const jtfs::RowTask*>(b + o[12]);
    t.segs = reinterpret_cast<const int32_t*>(b + o[13]);
    t.segterms = reinterpret_cast<const jtfs::SegTerm*>(b + o[14]);
    t.stasks = reinterpret_cast<const jtfs::SplitTask*>(b + o[15]);
    t.band_psi1 = reinterpret_cast<const int32_t*>(b + o[16]);
    t.gchunks = reinterpret_cast<const int32_t*>(b + o[17]);
    t.live_rt = reinterpret_cast<const int32_t*>(b + o[18]);
    a.sig.push_back(t);
  }
  if (p->sig.size() > 1) {
    const size_t ns = std::min<size_t>(p->sig.size(), kMaxStreams);
    bool ok = hipEventCreateWithFlags(&a.fork, hipEventDisableTiming) == hipSuccess;
    for (size_t i = 0; ok && i < ns; ++i) {
      hipStream_t st = nullptr;
      hipEvent_t ev = nullptr;
      ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
      if (st) a.streams.push_back(st);
      if (ev) a.joins.push_back(ev);
    }
    if (!ok) {
      for (hipStream_t st : a.streams) (void)hipStreamDestroy(st);
      for (hipEvent_t ev : a.joins) (void)hipEventDestroy(ev);
      if (a.fork) (void)hipEventDestroy(a.fork);
      (void)hipFree(a.base);
      return fail(JTFS_ERR_HIP, "creating the batch streams failed");
    }
  }
  auto ins = p->dev.emplace(dev, std::move(a));
  *out = &ins.first->second;
  return JTFS_OK;
}

// The arena of the current device if the plan's tables are already there (no upload).
jtfs_status find_tables(jtfs_plan_t p, const DeviceArena** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(JTFS_ERR_HIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lock(p->mu);
  auto it = p->dev.find(dev);
  if (it == p->dev.end())
    return fail(JTFS_ERR_ARG, "the plan's tables are not on this device: call jtfs_plan_prepare first");
  *out = &it->second;
  return JTFS_OK;
}

// Runs body(signal, stream) for every signal. A single signal, or every signal when
// `serial` is set, runs on the caller's stream; otherwise a batch is spread over the arena's streams, which first wait for the work
// already enqueued on the caller's stream and are waited for by it at the end (event
// fork / join, so the pattern is also valid under stream capture).
template <class Body>
jtfs_status for_each_signal(jtfs_plan_t plan, const DeviceArena* a, hipStream_t caller, Body body,
                            bool serial = false) {
  if (serial || plan->sig.size() == 1 || a->streams.empty()) {
    for (size_t s = 0; s < plan->sig.size(); ++s) {
      jtfs_status r = body(s, caller);
      if (r != JTFS_OK) return r;
    }
    return JTFS_OK;
  }
  std::lock_guard<std::mutex> lock(plan->mu);
  if (hipEventRecord(a->fork, caller) != hipSuccess) return fail(JTFS_ERR_HIP, "fork event record failed");
  for (hipStream_t st : a->streams)
    if (hipStreamWaitEvent(st, a->fork, 0) != hipSuccess) return fail(JTFS_ERR_HIP, "fork wait failed");
  jtfs_status r = JTFS_OK;
  for (size_t s = 0; s < plan->sig.size() && r == JTFS_OK; ++s) r = body(s, a->streams[s % a->streams.size()]);
  for (size_t i = 0; i < a->streams.size(); ++i) {
    if (hipEventRecord(a->joins[i], a->streams[i]) != hipSuccess ||
        hipStreamWaitEvent(caller, a->joins[i], 0) != hipSuccess)
      return fail(JTFS_ERR_HIP, "join failed");
  }
  return r;
}

// `shared`: every signal's segment starts at ws (JTFS_SHARED_WORKSPACE).
jtfs::DevSig make_devsig(const jtfs_plan_t p, size_t s, const SigTables& t, void* ws, bool shared = false) {
  const jtfs::SigPlan& sp = p->sig[s];
  char* base = static_cast<char*>(ws) + (shared ? 0 : p->ws_off[s]);
  const jtfs::WsLayout& w = sp.ws;
  jtfs::DevSig d{};
  d.tw = t.tw;
  d.bandvals = t.bandvals;
  d.bands = t.bands;
  d.tables = t.tables;
  d.W = t.W;
  d.rt_nrange = t.rt_nrange;
  d.live_rt = t.live_rt;
  d.frf = t.frf;
  d.fgroups = t.fgroups;
  d.fwd_items = t.fwd_items;
  d.bwd_items = t.bwd_items;
  d.jobs = t.jobs;
  d.tasks = t.tasks;
  d.segs = t.segs;
  d.segterms = t.segterms;
  d.stasks = t.stasks;
  d.gchunks = t.gchunks;
  d.s_off = t.s_off;
  d.Xh = reinterpret_cast<jtfs::c32*>(base + w.Xh);
  d.Z1 = reinterpret_cast<jtfs::c32*>(base + w.Z1);
  d.U1h = reinterpret_cast<jtfs::c32*>(base + w.U1h);
  d.S1 = reinterpret_cast<float*>(base + w.S1);
  d.Y2 = reinterpret_cast<jtfs::c32*>(base + w.Y2);
  d.part = reinterpret_cast<float*>(base + w.part);
  d.psum = reinterpret_cast<float*>(base + w.psum);
  d.scr = reinterpret_cast<jtfs::c32*>(base + w.scr);
  d.dP = reinterpret_cast<float*>(base + w.dP);
  d.dYpart = reinterpret_cast<jtfs::c32*>(base + w.dYpart);
  d.dYh = reinterpret_cast<jtfs::c32*>(base + w.dYh);
  d.dS1p = reinterpret_cast<float*>(base + w.dS1p);
  d.dU1 = reinterpret_cast<float*>(base + w.dU1);
  d.dZh = reinterpret_cast<jtfs::c32*>(base + w.dZh);
  d.dXh = reinterpret_cast<jtfs::c32*>(base + w.dXh);
  d.o1 = reinterpret_cast<jtfs::c32*>(base + w.o1);
  d.N = static_cast<int32_t>(sp.N);
  d.N_pad = static_cast<int32_t>(sp.N_pad);
  d.pad_left = static_cast<int32_t>(sp.pad_left);
  d.log2_Npad = sp.log2_Npad;
  d.N1 = static_cast<int32_t>(sp.psi1.size());
  d.nf_pad = sp.nf_pad;
  d.f_lo = sp.f_lo;
  d.nF = sp.n_frames;
  d.Lf = sp.Lf;
  d.log2T = sp.log2T;
  d.N_fr = sp.N_fr;
  d.sF = sp.sF;
  d.n_g = static_cast<int32_t>(sp.fr.size());
  d.n_groups = static_cast<int32_t>(sp.groups.size());
  d.n_real = static_cast<int32_t>(sp.fr_real.size());
  d.R_pad = sp.R_pad;
  d.NW = sp.NW;
  d.y2_total = sp.y2_total;
  d.z1_total = sp.z1_total;
  d.s0_off = sp.s0_off;
  d.s0_band = sp.s0_band;
  d.w0 = sp.w0;
  d.u0 = sp.u0 ? 1 : 0;
  d.no_avg_local = sp.no_avg_local ? 1 : 0;
  d.no_avg_fr = sp.no_avg_fr ? 1 : 0;
  d.u2 = reinterpret_cast<float*>(base + w.u2);
  d.dv = reinterpret_cast<jtfs::c32*>(base + w.dv);
  return d;
}

// Runs `launch` (a callable returning hipError_t) and, when timing is on, brackets it
// with two events on `st`. A null plan never times (the no-allocation path: creating
// events is not allowed there).
template <class F>
hipError_t timed(jtfs_plan_t p, int stage, hipStream_t st, F launch) {
  if (!p || !((p->timing >> stage) & 1u)) return launch();
  jtfs_plan_s::Mark m{stage, nullptr, nullptr};
  hipError_t e = hipEventCreate(&m.a);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&m.b);
  if (e != hipSuccess) return e;
  e = hipEventRecord(m.a, st);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(m.b, st);
  p->marks.push_back(m);
  return e;
}

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(JTFS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define STAGE(id, call) HIPCHK(timed(p, id, st, [&]() { return (call); }))

jtfs_status forward_time(jtfs_plan_t p, const jtfs::DevSig& d, const jtfs::SigPlan& sp, hipStream_t st) {
  STAGE(0, jtfs::run_time_stage(jtfs::ST_XHAT, d, sp, st));
  STAGE(1, jtfs::run_time_stage(jtfs::ST_L1Z, d, sp, st));
  STAGE(2, jtfs::run_time_stage(jtfs::ST_L1UH, d, sp, st));
  STAGE(3, jtfs::run_s1(d, sp, st));
  STAGE(5, jtfs::run_time_stage(jtfs::ST_L2Y, d, sp, st));
  return JTFS_OK;
}

jtfs_status forward_signal(jtfs_plan_t p, const jtfs::DevSig& d, const jtfs::SigPlan& sp, hipStream_t st) {
  jtfs_status r = forward_time(p, d, sp, st);
  if (r != JTFS_OK) return r;
  STAGE(4, jtfs::run_order1_fwd(d, sp, st));
  if (sp.no_avg_local) {
    STAGE(6, jtfs::run_unavg_fwd(d, sp, st));
  } else {
    STAGE(6, jtfs::run_freq_fwd(d, sp, st));
    STAGE(7, jtfs::run_freq_pool(d, sp, st));
  }
  return JTFS_OK;
}

jtfs_status backward_signal(jtfs_plan_t p, const jtfs::DevSig& d, const jtfs::SigPlan& sp, bool reuse,
                            hipStream_t st) {
  if (!reuse) {
    jtfs_status r = forward_time(p, d, sp, st);
    if (r != JTFS_OK) return r;
  }
  if (sp.no_avg_local) {
    STAGE(9, jtfs::run_unavg_bwd(d, sp, st));
  } else {
    STAGE(8, jtfs::run_freq_dP(d, sp, st));
    STAGE(9, jtfs::run_freq_bwd(d, sp, st));
    STAGE(18, jtfs::run_dy_reduce(d, sp, st));
  }
  STAGE(10, jtfs::run_order1_bwd(d, sp, st));
  STAGE(11, jtfs::run_ds1h(d, sp, st));
  STAGE(12, jtfs::run_time_stage(jtfs::ST_BYH, d, sp, st));
  STAGE(13, jtfs::run_time_stage(jtfs::ST_BU, d, sp, st));
  STAGE(14, jtfs::run_time_stage(jtfs::ST_BZH, d, sp, st));
  STAGE(15, jtfs::run_time_stage(jtfs::ST_BX, d, sp, st));
  return JTFS_OK;
}

int64_t state_vectors(int32_t kind) {
  switch (kind) {
    case JTFS_OPT_GD: return 0;
    case JTFS_OPT_ADAM: return 2;
    case JTFS_OPT_MOMENTUM_BOLD: return 3;
    default: return -1;
  }
}

}  // namespace

extern "C" {

jtfs_status jtfs_plan(const jtfs_params* sig, int32_t batch, jtfs_plan_t* out) {
  return jtfs_plan_tuned(sig, batch, nullptr, out);
}

jtfs_status jtfs_plan_tuned(const jtfs_params* sig, int32_t batch, const jtfs_tuning* tuning, jtfs_plan_t* out) {
  if (!out) return fail(JTFS_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!sig || batch < 1) return fail(JTFS_ERR_ARG, "need at least one signal");
  jtfs_tuning tu;
  if (!jtfs::resolve_tuning(tuning, tu)) return fail(JTFS_ERR_ARG, "tuning field out of range");
  std::unique_ptr<jtfs_plan_s> p(new (std::nothrow) jtfs_plan_s());
  if (!p) return fail(JTFS_ERR_NOMEM, "host allocation failed");
  try {
    p->sig.resize(batch);
    p->x_off.push_back(0);
    p->s_off.push_back(0);
    size_t ws = 0;
    for (int32_t s = 0; s < batch; ++s) {
      std::string err;
      jtfs_status st = jtfs::build_signal_plan(sig[s], p->sig[s], err, &tu);
      if (st != JTFS_OK) return fail(st, "signal " + std::to_string(s) + ": " + err);
      const jtfs::SigPlan& sp = p->sig[s];
      p->x_off.push_back(p->x_off.back() + sp.N);
      p->s_off.push_back(p->s_off.back() + sp.n_coeff);
      p->ws_off.push_back(ws);
      p->ws_fwd = ws + sp.ws.fwd_end;
      ws += sp.ws.bwd_end;
      p->ws_fwd_shared = std::max(p->ws_fwd_shared, sp.ws.fwd_end);
      p->ws_bwd_shared = std::max(p->ws_bwd_shared, sp.ws.bwd_end);
      std::vector<int64_t> bo(sp.groups.size() * sp.fr.size() + sp.fr_real.size(), -1);
      size_t gi = 0, ri = 0;
      for (const jtfs_path& r : sp.paths) {
        if (r.order == 0) continue;   // the zeroth-order block is written by its own kernel
        if (r.order == 1) {
          bo[sp.groups.size() * sp.fr.size() + ri++] = r.offset;
        } else {
          while (sp.groups[gi].n2 != r.n2) ++gi;
          bo[gi * sp.fr.size() + r.n_fr] = r.offset;
        }
      }
      p->block_off.push_back(std::move(bo));
    }
    p->ws_bwd = ws;
    p->n_total = p->x_off.back();
    p->c_total = p->s_off.back();
  } catch (const std::bad_alloc&) {
    return fail(JTFS_ERR_NOMEM, "host allocation failed while planning");
  }
  *out = p.release();
  return JTFS_OK;
}

jtfs_status jtfs_plan_query(jtfs_plan_t plan, jtfs_plan_info* info) {
  if (!plan || !info) return fail(JTFS_ERR_ARG, "NULL argument");
  info->batch = static_cast<int32_t>(plan->sig.size());
  info->n_samples_total = plan->n_total;
  info->n_coeff_total = plan->c_total;
  info->ws_forward = plan->ws_fwd;
  info->ws_backward = plan->ws_bwd;
  info->ws_shared_forward = plan->ws_fwd_shared;
  info->ws_shared_backward = plan->ws_bwd_shared;
  return JTFS_OK;
}

jtfs_status jtfs_plan_offsets(jtfs_plan_t plan, int64_t* x_offsets, int64_t* s_offsets) {
  if (!plan) return fail(JTFS_ERR_ARG, "NULL plan");
  if (x_offsets) std::memcpy(x_offsets, plan->x_off.data(), sizeof(int64_t) * plan->x_off.size());
  if (s_offsets) std::memcpy(s_offsets, plan->s_off.data(), sizeof(int64_t) * plan->s_off.size());
  return JTFS_OK;
}

jtfs_status jtfs_plan_meta(jtfs_plan_t plan, int32_t signal, jtfs_path* rows, int64_t cap, int64_t* n_rows) {
  if (!plan || !n_rows || signal < 0 || signal >= static_cast<int32_t>(plan->sig.size()))
    return fail(JTFS_ERR_ARG, "bad plan, signal or n_rows");
  const auto& paths = plan->sig[signal].paths;
  *n_rows = static_cast<int64_t>(paths.size());
  if (rows) {
    int64_t m = std::min<int64_t>(cap, static_cast<int64_t>(paths.size()));
    for (int64_t i = 0; i < m; ++i) rows[i] = paths[i];
  }
  return JTFS_OK;
}

jtfs_status jtfs_plan_filters(jtfs_plan_t plan, int32_t signal, int32_t bank, double* xi, double* sigma, int32_t* j,
                              int32_t* k, int32_t cap, int32_t* n) {
  if (!plan || !n || signal < 0 || signal >= static_cast<int32_t>(plan->sig.size()) || bank < 0 || bank > 2)
    return fail(JTFS_ERR_ARG, "bad plan, signal, bank or n");
  const jtfs::SigPlan& sp = plan->sig[signal];
  const std::vector<jtfs::Filt>& f = bank == 0 ? sp.psi1 : (bank == 1 ? sp.psi2 : sp.fr);
  *n = static_cast<int32_t>(f.size());
  for (int32_t i = 0; i < std::min<int32_t>(cap, *n); ++i) {
    if (xi) xi[i] = f[i].xi;
    if (sigma) sigma[i] = f[i].sigma;
    if (j) j[i] = f[i].j;
    if (k) k[i] = f[i].k;
  }
  return JTFS_OK;
}

jtfs_status jtfs_plan_sizes(jtfs_plan_t plan, int32_t signal, int64_t* out8) {
  if (!plan || !out8 || signal < 0 || signal >= static_cast<int32_t>(plan->sig.size()))
    return fail(JTFS_ERR_ARG, "bad plan, signal or output");
  const jtfs::SigPlan& sp = plan->sig[signal];
  const int64_t v[8] = {sp.N_pad, sp.pad_left, sp.N_fr, sp.sF, sp.nf_pad, sp.f_lo, sp.n_frames, sp.n_coeff};
  std::memcpy(out8, v, sizeof(v));
  return JTFS_OK;
}

jtfs_status jtfs_plan_ws_region(jtfs_plan_t plan, int32_t signal, int32_t which, int64_t* offset_bytes,
                                int64_t* count) {
  if (!plan || !offset_bytes || !count || signal < 0 || signal >= static_cast<int32_t>(plan->sig.size()))
    return fail(JTFS_ERR_ARG, "bad plan, signal or outputs");
  const jtfs::SigPlan& sp = plan->sig[signal];
  const size_t base = plan->ws_off[signal];
  switch (which) {
    case 0: *offset_bytes = base + sp.ws.Z1; *count = sp.z1_total; break;
    case 1: *offset_bytes = base + sp.ws.U1h; *count = sp.z1_total; break;
    case 2: *offset_bytes = base + sp.ws.S1; *count = static_cast<int64_t>(sp.psi1.size()) * sp.nf_pad; break;
    case 3: *offset_bytes = base + sp.ws.Y2; *count = sp.y2_total; break;
    default: return fail(JTFS_ERR_ARG, "unknown region");
  }
  return JTFS_OK;
}

jtfs_status jtfs_plan_cost(jtfs_plan_t plan, int32_t signal, double* out4) {
  if (!plan || !out4 || signal < 0 || signal >= static_cast<int32_t>(plan->sig.size()))
    return fail(JTFS_ERR_ARG, "bad plan, signal or output");
  const jtfs::SigPlan& sp = plan->sig[signal];
  out4[0] = sp.mac_dense;
  out4[1] = sp.mac_banded;
  out4[2] = sp.mac_exec;
  out4[3] = sp.mac_pool;
  return JTFS_OK;
}

int64_t jtfs_opt_state_floats(jtfs_plan_t plan, int32_t kind) {
  if (!plan) return -1;
  int64_t v = state_vectors(kind);
  if (v < 0) return -1;
  return v * plan->n_total + 4 * static_cast<int64_t>(plan->sig.size());
}

jtfs_status jtfs_forward(jtfs_plan_t plan, const float* x, float* S, void* ws, size_t ws_bytes, jtfs_stream_t stream) {
  return jtfs_forward_ex(plan, x, S, ws, ws_bytes, 0u, stream);
}

jtfs_status jtfs_forward_ex(jtfs_plan_t plan, const float* x, float* S, void* ws, size_t ws_bytes, uint32_t flags,
                            jtfs_stream_t stream) {
  if (!plan || !x || !S || !ws) return fail(JTFS_ERR_ARG, "NULL argument");
  if (flags & ~JTFS_SHARED_WORKSPACE) return fail(JTFS_ERR_ARG, "unknown flags");
  const bool shared = (flags & JTFS_SHARED_WORKSPACE) != 0;
  if (ws_bytes < (shared ? plan->ws_fwd_shared : plan->ws_fwd))
    return fail(JTFS_ERR_WORKSPACE, shared ? "workspace smaller than ws_shared_forward"
                                           : "workspace smaller than ws_forward");
  const DeviceArena* a = nullptr;
  jtfs_status r = device_tables(plan, &a);
  if (r != JTFS_OK) return r;
  return for_each_signal(
      plan, a, static_cast<hipStream_t>(stream),
      [&](size_t s, hipStream_t st) {
        jtfs::DevSig d = make_devsig(plan, s, a->sig[s], ws, shared);
        d.x = x + plan->x_off[s];
        d.S = S + plan->s_off[s];
        return forward_signal(plan, d, plan->sig[s], st);
      },
      shared);
}

jtfs_status jtfs_backward(jtfs_plan_t plan, const float* x, const float* dS, float* dx, void* ws, size_t ws_bytes,
                          uint32_t flags, jtfs_stream_t stream) {
  if (!plan || !x || !dS || !dx || !ws) return fail(JTFS_ERR_ARG, "NULL argument");
  if (flags & ~(JTFS_REUSE_FORWARD | JTFS_SHARED_WORKSPACE)) return fail(JTFS_ERR_ARG, "unknown flags");
  const bool reuse = (flags & JTFS_REUSE_FORWARD) != 0;
  const bool shared = (flags & JTFS_SHARED_WORKSPACE) != 0;
  if (reuse && shared && plan->sig.size() > 1)
    return fail(JTFS_ERR_ARG, "a shared workspace holds one signal's forward: JTFS_REUSE_FORWARD needs a batch of one");
  if (ws_bytes < (shared ? plan->ws_bwd_shared : plan->ws_bwd))
    return fail(JTFS_ERR_WORKSPACE, shared ? "workspace smaller than ws_shared_backward"
                                           : "workspace smaller than ws_backward");
  const DeviceArena* a = nullptr;
  jtfs_status r = device_tables(plan, &a);
  if (r != JTFS_OK) return r;
  return for_each_signal(
      plan, a, static_cast<hipStream_t>(stream),
      [&](size_t s, hipStream_t st) {
        jtfs::DevSig d = make_devsig(plan, s, a->sig[s], ws, shared);
        d.x = x + plan->x_off[s];
        d.dS = dS + plan->s_off[s];
        d.dx = dx + plan->x_off[s];
        return backward_signal(plan, d, plan->sig[s], reuse, st);
      },
      shared);
}

jtfs_status jtfs_metamer_step(jtfs_plan_t plan, float* y, const float* S_target, const jtfs_opt* opt, float* loss,
                              void* ws, size_t ws_bytes, jtfs_stream_t stream) {
  if (!plan || !y || !S_target || !opt || !loss || !ws) return fail(JTFS_ERR_ARG, "NULL argument");
  if (state_vectors(opt->kind) < 0) return fail(JTFS_ERR_ARG, "unknown optimiser kind");
  if (!opt->state) return fail(JTFS_ERR_ARG, "optimiser state is NULL");
  if (ws_bytes < plan->ws_bwd) return fail(JTFS_ERR_WORKSPACE, "workspace smaller than ws_backward");
  const DeviceArena* a = nullptr;
  jtfs_status r = device_tables(plan, &a);
  if (r != JTFS_OK) return r;
  const int64_t nv = state_vectors(opt->kind);
  const int64_t Nt = plan->n_total;
  float* scal_base = opt->state + nv * Nt;
  return for_each_signal(plan, a, static_cast<hipStream_t>(stream), [&](size_t s, hipStream_t st) -> jtfs_status {
    const jtfs::SigPlan& sp = plan->sig[s];
    char* seg = static_cast<char*>(ws) + plan->ws_off[s];
    float* S_y = reinterpret_cast<float*>(seg + sp.ws.S);
    float* dS = reinterpret_cast<float*>(seg + sp.ws.dS);
    float* grad = reinterpret_cast<float*>(seg + sp.ws.grad);
    jtfs::DevSig d = make_devsig(plan, s, a->sig[s], ws);
    float* ys = y + plan->x_off[s];
    d.x = ys;
    d.S = S_y;
    jtfs_status r = forward_signal(plan, d, sp, st);
    if (r != JTFS_OK) return r;
    jtfs_plan_t p = plan;
    STAGE(16, jtfs::run_loss(S_y, S_target + plan->s_off[s], dS, loss + s, sp.n_coeff, sp.s0_off >= 0 ? sp.n_frames : 0,
                             sp.w0, st));
    d.dS = dS;
    d.dx = grad;
    r = backward_signal(plan, d, sp, true, st);
    if (r != JTFS_OK) return r;
    float* v0 = nv > 0 ? opt->state + plan->x_off[s] : nullptr;
    float* v1 = nv > 1 ? opt->state + Nt + plan->x_off[s] : nullptr;
    float* v2 = nv > 2 ? opt->state + 2 * Nt + plan->x_off[s] : nullptr;
    STAGE(17, jtfs::run_update(*opt, ys, grad, loss + s, v0, v1, v2, scal_base + 4 * s, sp.N, st));
    return JTFS_OK;
  });
}

jtfs_status jtfs_opt_status(jtfs_plan_t plan, const jtfs_opt* opt, int32_t* counts, jtfs_stream_t stream) {
  if (!plan || !opt || !opt->state) return fail(JTFS_ERR_ARG, "NULL argument");
  const int64_t nv = state_vectors(opt->kind);
  if (nv < 0) return fail(JTFS_ERR_ARG, "unknown optimiser kind");
  const size_t batch = plan->sig.size();
  std::vector<float> scal(4 * batch);
  HIPCHK(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  HIPCHK(hipMemcpy(scal.data(), opt->state + nv * plan->n_total, sizeof(float) * scal.size(), hipMemcpyDeviceToHost));
  bool any = false;
  for (size_t s = 0; s < batch; ++s) {
    const int32_t c = static_cast<int32_t>(scal[4 * s + 3]);
    if (counts) counts[s] = c;
    any = any || c != 0;
  }
  if (any) return fail(JTFS_ERR_NONFINITE, "a metamer step met a non-finite loss; y was left unchanged");
  return JTFS_OK;
}

jtfs_status jtfs_colored_noise(jtfs_plan_t plan, const float* x, const float* w, float* y0, void* ws, size_t ws_bytes,
                               jtfs_stream_t stream) {
  if (!plan || !x || !w || !y0 || !ws) return fail(JTFS_ERR_ARG, "NULL argument");
  if (y0 == x || y0 == w) return fail(JTFS_ERR_ARG, "y0 may not alias x or w");
  if (ws_bytes < plan->ws_bwd) return fail(JTFS_ERR_WORKSPACE, "workspace smaller than ws_backward");
  const DeviceArena* a = nullptr;
  jtfs_status r = device_tables(plan, &a);
  if (r != JTFS_OK) return r;
  return for_each_signal(plan, a, static_cast<hipStream_t>(stream), [&](size_t s, hipStream_t st) -> jtfs_status {
    const jtfs::SigPlan& sp = plan->sig[s];
    jtfs::DevSig d = make_devsig(plan, s, a->sig[s], ws);
    // first layer of x up to S1 (the levels go to the dU1 region: z1_total >= N1 floats)
    d.x = x + plan->x_off[s];
    HIPCHK(jtfs::run_time_stage(jtfs::ST_XHAT, d, sp, st));
    HIPCHK(jtfs::run_time_stage(jtfs::ST_L1Z, d, sp, st));
    HIPCHK(jtfs::run_time_stage(jtfs::ST_L1UH, d, sp, st));
    HIPCHK(jtfs::run_s1(d, sp, st));
    HIPCHK(jtfs::run_cn_levels(d, sp, a->sig[s].band_psi1, d.dU1, st));
    // DFT of the padded draws, shaped into dXh, inverse DFT and unpad into y0
    d.x = w + plan->x_off[s];
    HIPCHK(jtfs::run_time_stage(jtfs::ST_XHAT, d, sp, st));
    HIPCHK(jtfs::run_cn_shape(d, sp, a->sig[s].band_psi1, d.dU1, st));
    d.dx = y0 + plan->x_off[s];
    HIPCHK(jtfs::run_signal_idft(d, sp, st));
    return JTFS_OK;
  });
}

jtfs_status jtfs_joint_wavelet(jtfs_plan_t plan, int32_t signal, int32_t n2, int32_t n_fr, int32_t n_t, float* out,
                               jtfs_stream_t stream) {
  if (!plan || !out || signal < 0 || signal >= static_cast<int32_t>(plan->sig.size()))
    return fail(JTFS_ERR_ARG, "bad plan, signal or out");
  const jtfs::SigPlan& sp = plan->sig[signal];
  if (n_fr < 0 || n_fr >= static_cast<int32_t>(sp.fr.size())) return fail(JTFS_ERR_ARG, "n_fr out of range");
  auto it = sp.band_psi2.find({n2, 0});
  if (it == sp.band_psi2.end()) return fail(JTFS_ERR_ARG, "n2 has no second-order paths in this plan");
  if (n_t < 1 || n_t > sp.N_pad || n_t > (1 << 20)) return fail(JTFS_ERR_ARG, "n_t outside [1, min(N_pad, 2^20)]");
  const DeviceArena* a = nullptr;
  jtfs_status r = device_tables(plan, &a);
  if (r != JTFS_OK) return r;
  // only the plan tables are read: no workspace
  jtfs::DevSig d = make_devsig(plan, static_cast<size_t>(signal), a->sig[signal], nullptr, true);
  const jtfs::Band band = sp.bands[static_cast<size_t>(it->second)];
  const float* taps = a->sig[signal].tables + sp.frf[static_cast<size_t>(n_fr)].taps;
  HIPCHK(jtfs::run_joint_wavelet(d, band, taps, sp.N_fr, n_t, out, static_cast<hipStream_t>(stream)));
  return JTFS_OK;
}

jtfs_status jtfs_loss(jtfs_plan_t plan, const float* S, const float* S_target, float* dS, float* loss,
                      int32_t relative, float scale, jtfs_stream_t stream) {
  if (!plan || !S || !S_target || !dS || !loss) return fail(JTFS_ERR_ARG, "NULL argument");
  if (dS == S || dS == S_target) return fail(JTFS_ERR_ARG, "dS may not alias S or S_target");
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (size_t s = 0; s + 1 < plan->s_off.size(); ++s) {
    const int64_t o = plan->s_off[s], n = plan->s_off[s + 1] - o;
    const jtfs::SigPlan& sp = plan->sig[s];
    const hipError_t e = jtfs::run_rel_loss(S + o, S_target + o, dS + o, loss + s, n, sp.s0_off >= 0 ? sp.n_frames : 0,
                                            sp.w0, relative, scale, st);
    if (e != hipSuccess) return fail(JTFS_ERR_HIP, std::string("loss kernel: ") + hipGetErrorString(e));
  }
  return JTFS_OK;
}

jtfs_status jtfs_timing_enable(jtfs_plan_t plan, int32_t on) {
  if (!plan) return fail(JTFS_ERR_ARG, "NULL plan");
  plan->timing = on != 0 ? (1u << JTFS_N_STAGES) - 1u : 0u;
  return JTFS_OK;
}

jtfs_status jtfs_timing_stages(jtfs_plan_t plan, uint32_t mask) {
  if (!plan) return fail(JTFS_ERR_ARG, "NULL plan");
  if (mask >> JTFS_N_STAGES) return fail(JTFS_ERR_ARG, "stage mask has bits beyond JTFS_N_STAGES");
  plan->timing = mask;
  return JTFS_OK;
}

jtfs_status jtfs_timing_read(jtfs_plan_t plan, double* ms, int64_t* counts, int32_t cap) {
  if (!plan || cap < 0) return fail(JTFS_ERR_ARG, "bad plan or cap");
  for (int32_t i = 0; i < cap; ++i) {
    if (ms) ms[i] = 0.0;
    if (counts) counts[i] = 0;
  }
  jtfs_status st = JTFS_OK;
  for (auto& m : plan->marks) {
    float t = 0.f;
    if (hipEventSynchronize(m.b) != hipSuccess || hipEventElapsedTime(&t, m.a, m.b) != hipSuccess)
      st = fail(JTFS_ERR_HIP, "timing event failed");
    if (m.stage < cap) {
      if (ms) ms[m.stage] += t;
      if (counts) counts[m.stage] += 1;
    }
    (void)hipEventDestroy(m.a);
    (void)hipEventDestroy(m.b);
  }
  plan->marks.clear();
  return st;
}

void jtfs_plan_destroy(jtfs_plan_t plan) { delete plan; }

const char* jtfs_status_str(jtfs_status s) {
  switch (s) {
    case JTFS_OK: return "ok";
    case JTFS_ERR_ARG: return "invalid argument";
    case JTFS_ERR_NOMEM: return "out of memory";
    case JTFS_ERR_HIP: return "HIP error";
    case JTFS_ERR_WORKSPACE: return "workspace too small";
    case JTFS_ERR_UNSUPPORTED: return "unsupported parameters";
    case JTFS_ERR_NONFINITE: return "non-finite loss";
  }
  return "unknown status";
}

const char* jtfs_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace jtfs {
// Records the detail string of a failure for jtfs_last_error (used by the decoder ABI).
jtfs_status report(jtfs_status s, const std::string& msg) { return fail(s, msg); }

jtfs_status prepare_tables(jtfs_plan_t plan) {
  if (!plan) return fail(JTFS_ERR_ARG, "NULL plan");
  const DeviceArena* a = nullptr;
  return device_tables(plan, &a);
}

size_t shared_forward_bytes(jtfs_plan_t plan) { return plan->ws_fwd_shared; }

// Forward of every signal in turn on `stream`, each in the one segment at ws, with the
// plan's tables already on the device and no stage timing: enqueues kernels only.
jtfs_status forward_prepared(jtfs_plan_t plan, const float* x, float* S, void* ws, hipStream_t stream) {
  const DeviceArena* a = nullptr;
  jtfs_status r = find_tables(plan, &a);
  if (r != JTFS_OK) return r;
  for (size_t s = 0; s < plan->sig.size(); ++s) {
    jtfs::DevSig d = make_devsig(plan, s, a->sig[s], ws, true);
    d.x = x + plan->x_off[s];
    d.S = S + plan->s_off[s];
    r = forward_signal(nullptr, d, plan->sig[s], stream);
    if (r != JTFS_OK) return r;
  }
  return JTFS_OK;
}
}  // namespace jtfs
