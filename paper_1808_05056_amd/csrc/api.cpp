// C ABI entry points and the HIP backend that runs an operation list.
//
// The paper's MMOOC (Section V, Fig. 2) issues, per C block, asynchronous
// copies and a DGEMM on two streams, tied together with events, and
// synchronises both streams before returning.  Here the operation list from
// the scheduler is issued in order: each op first makes its stream wait for
// the events of the ops listed in its wait set, then enqueues a pitched copy
// (hipMemcpy2DAsync between page-locked host memory and the device arena) or
// a tile kernel, and records an event if a later op on another stream waits
// for it.  The call returns after every stream has drained.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <future>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

namespace ooc {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

ooc_status fail(ooc_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

namespace {

constexpr int kMaxDevices = 64;

struct DevCtx {
  std::mutex mu;       // guards everything below; held for the whole of a call on the device
  bool arch_ok = false;  // the device was checked to be a gfx950
  bool init = false;     // streams created
  hipStream_t st[3] = {nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> ev;   // dependency events (no timing)
  std::vector<hipEvent_t> tev;  // timing events (profile mode)
  std::vector<hipEvent_t> kev;  // timing events around slice-product kernels alone (profile mode)
  void* arena = nullptr;
  size_t arena_bytes = 0;
};

DevCtx g_dev[kMaxDevices];

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

ooc_status hip_fail(hipError_t e, const char* what) {
  return fail(OOC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr, what)                       \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// Select the device (checked once to be a gfx950).
ooc_status ensure_device(int dev) {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    return fail(OOC_ERR_NO_DEVICE, "no HIP device available");
  }
  if (dev < 0 || dev >= count || dev >= kMaxDevices) return fail(OOC_ERR_NO_DEVICE, "device ordinal out of range");
  HIPCHK(hipSetDevice(dev), "hipSetDevice");
  DevCtx& c = g_dev[dev];
  std::lock_guard<std::mutex> lock(c.mu);
  if (!c.arch_ok) {
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      return fail(OOC_ERR_NO_DEVICE, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
    c.arch_ok = true;
  }
  return OOC_OK;
}

// Create the device's three streams (default priority) if they do not exist;
// the caller holds c.mu, so ooc_release cannot destroy them during the call.
ooc_status ensure_streams(DevCtx& c) {
  if (!c.init) {
    for (int s = 0; s < 3; ++s) HIPCHK(hipStreamCreateWithFlags(&c.st[s], hipStreamNonBlocking), "hipStreamCreate");
    c.init = true;
  }
  return OOC_OK;
}

ooc_status ensure_events(std::vector<hipEvent_t>& pool, size_t n, unsigned flags) {
  while (pool.size() < n) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, flags), "hipEventCreate");
    pool.push_back(e);
  }
  return OOC_OK;
}

bool is_pinned(const void* p) {
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeHost;
}

bool range_pinned(const double* base, int64_t rows, int64_t cols, int64_t ld) {
  if (rows == 0 || cols == 0) return true;
  return is_pinned(base) && is_pinned(base + (rows - 1) * ld + (cols - 1));
}

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

// A host matrix an operation list copies from or to (op.mat indexes them).
struct HostMat {
  double* p;
  int64_t ld;
};
typedef std::vector<HostMat> HostMats;

// What an operation list needs from its plan: stream count and the split
// precision of its SPLIT_GEMM ops.
struct RunCfg {
  int nstreams;
  int precision;
  int slices;
};

// Length of the union of intervals [a, b).
double union_length(std::vector<std::pair<double, double>> iv) {
  std::sort(iv.begin(), iv.end());
  double total = 0.0, lo = 0.0, hi = -1.0;
  for (const auto& x : iv) {
    if (x.first > hi) {
      if (hi > lo) total += hi - lo;
      lo = x.first;
      hi = x.second;
    } else {
      hi = std::max(hi, x.second);
    }
  }
  if (hi > lo) total += hi - lo;
  return total;
}

// Fraction of the copy-busy time (union of copy intervals) during which a
// kernel also ran: |U_copy ∩ U_kernel| / |U_copy| = (|U_c| + |U_k| - |U_c ∪ U_k|) / |U_c|.
double overlap_fraction(const std::vector<std::pair<double, double>>& copies,
                        const std::vector<std::pair<double, double>>& kernels) {
  const double uc = union_length(copies);
  if (uc <= 0.0) return 0.0;
  std::vector<std::pair<double, double>> all(copies);
  all.insert(all.end(), kernels.begin(), kernels.end());
  const double both = uc + union_length(kernels) - union_length(all);
  return std::max(0.0, std::min(1.0, both / uc));
}

ooc_status run_ops(DevCtx& c, hipStream_t* streams, const RunCfg& plan, const std::vector<ooc_op>& ops,
                   double* arena, int64_t arena_elems, const HostMats& hm, bool profile, double* timeline,
                   int64_t timeline_cap, ooc_stats* st) {
  const size_t n = ops.size();
  std::vector<int> evidx(n, -1);
  size_t nev = 0;
  for (const ooc_op& o : ops)
    for (int k = 0; k < o.nwait; ++k)
      if (evidx[o.wait[k]] < 0) evidx[o.wait[k]] = (int)nev++;
  ooc_status s0 = ensure_events(c.ev, nev, hipEventDisableTiming);
  if (s0 != OOC_OK) return s0;
  // slice-product launches of each split op, for their kernel-only timing events
  std::vector<int64_t> kfirst(n + 1, 0);
  for (size_t x = 0; x < n; ++x)
    kfirst[x + 1] = kfirst[x] + (ops[x].kind == OOC_OP_SPLIT_GEMM ? split_launches(ops[x].k) : 0);
  if (profile) {
    s0 = ensure_events(c.tev, 2 * n, hipEventDefault);
    if (s0 == OOC_OK) s0 = ensure_events(c.kev, (size_t)(2 * kfirst[n]), hipEventDefault);
    if (s0 != OOC_OK) return s0;
  }
  const int fail_at = env_int("OOC_FAIL_AT", -1);
  // Race testing (OOC_STRESS_SEED >= 0): the arena starts as NaN, and before
  // a third of the operations (chosen by the seed) a wait of up to
  // OOC_STRESS_US microseconds is enqueued on the operation's stream, after
  // its waits.  A correct operation list gives bit-identical results.
  const int stress_seed = env_int("OOC_STRESS_SEED", -1);
  const int stress_us = std::max(0, std::min(env_int("OOC_STRESS_US", 300), 5000));
  uint64_t rng = 0x9E3779B97F4A7C15ull * (uint64_t)(stress_seed + 2);
  auto next_rand = [&]() {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return rng;
  };
  if (stress_seed >= 0) {
    hipError_t e = launch_fill_nan(arena, arena_elems, streams[0]);
    if (e == hipSuccess) e = hipStreamSynchronize(streams[0]);
    if (e != hipSuccess) return hip_fail(e, "poisoning the arena");
  }
  ooc_status status = OOC_OK;
  std::string msg;
  int64_t d2h_issued = 0;
  size_t issued = 0;
  const double t0 = now_s();
  for (size_t x = 0; x < n; ++x) {
    const ooc_op& o = ops[x];
    if ((int)x == fail_at) {
      status = OOC_ERR_INJECTED;
      msg = "failure injected at op " + std::to_string(x);
      break;
    }
    hipStream_t s = streams[o.stream];
    hipError_t e = hipSuccess;
    for (int k = 0; k < o.nwait && e == hipSuccess; ++k) e = hipStreamWaitEvent(s, c.ev[evidx[o.wait[k]]], 0);
    if (e == hipSuccess && stress_seed >= 0 && next_rand() % 3 == 0)
      e = launch_spin((uint32_t)(next_rand() % (uint64_t)(stress_us + 1)), s);
    if (e == hipSuccess && profile) e = hipEventRecord(c.tev[2 * x], s);
    if (e == hipSuccess) {
      switch (o.kind) {
        case OOC_OP_H2D:
        case OOC_OP_D2H: {
          const int64_t hld = hm[o.mat].ld;
          double* host = hm[o.mat].p + o.row0 * hld + o.col0;
          double* dev = arena + o.off_c;
          // Always a 2-D (row-pitched) copy, also for contiguous blocks: on
          // MI355X a plain 1-D host-to-device copy running beside a 1-D
          // device-to-host copy was seen to share one copy engine with it
          // (each at half rate), while 2-D copies in the two directions ran
          // at full duplex (56.7 and 48.7 GB/s).
          if (o.kind == OOC_OP_H2D) {
            e = hipMemcpy2DAsync(dev, (size_t)o.ld_c * 8, host, (size_t)hld * 8, (size_t)o.cols * 8, (size_t)o.rows,
                                 hipMemcpyHostToDevice, s);
          } else {
            e = hipMemcpy2DAsync(host, (size_t)hld * 8, dev, (size_t)o.ld_c * 8, (size_t)o.cols * 8, (size_t)o.rows,
                                 hipMemcpyDeviceToHost, s);
            ++d2h_issued;
          }
          break;
        }
        case OOC_OP_GEMM:
          e = launch_dgemm_f64(o.rows, o.cols, o.k, o.alpha, arena + o.off_a, o.ld_a, arena + o.off_b, o.ld_b,
                               o.beta, arena + o.off_c, o.ld_c, o.gamma, arena + o.off_d, o.ld_d, s,
                               (o.flags & OOC_OPF_TRANSB) != 0,
                               (o.flags & OOC_OPF_LOWER) ? o.col0 - o.row0 : kNoTri);
          break;
        case OOC_OP_SPLIT_GEMM: {
          KernelTimer kt;
          if (profile) {
            kt.events = c.kev.data() + 2 * kfirst[x];
            kt.count = (int)(kfirst[x + 1] - kfirst[x]);
          }
          e = launch_split_gemm(slice_format(plan.precision), o.rows, o.cols, o.k, plan.slices, o.alpha,
                                arena + o.off_a, o.ld_a, arena + o.off_b, o.ld_b, o.beta, arena + o.off_c, o.ld_c,
                                o.gamma, arena + o.off_d, o.ld_d, arena + o.off_w, (size_t)o.len_w * 8, s,
                                profile ? &kt : nullptr, (o.flags & OOC_OPF_TRANSB) != 0,
                                (o.flags & OOC_OPF_REUSE_A) != 0, (o.flags & OOC_OPF_REUSE_B) != 0);
          break;
        }
        case OOC_OP_POTRF:
          e = launch_potrf_lower(o.rows, arena + o.off_c, o.ld_c, arena + o.off_w, o.k0, s);
          break;
        case OOC_OP_TRSM:
          e = (o.flags & OOC_OPF_BACK)
                  ? launch_trsm_rln(o.rows, o.cols, arena + o.off_c, o.ld_c, arena + o.off_a, o.ld_a, s)
                  : launch_trsm_rlt(o.rows, o.cols, arena + o.off_c, o.ld_c, arena + o.off_a, o.ld_a, s);
          break;
        default:
          status = OOC_ERR_ARG;
          msg = "unknown operation kind";
          break;
      }
    }
    if (status != OOC_OK) break;
    if (e == hipSuccess && profile) e = hipEventRecord(c.tev[2 * x + 1], s);
    if (e == hipSuccess && evidx[x] >= 0) e = hipEventRecord(c.ev[evidx[x]], s);
    if (e != hipSuccess) {
      status = OOC_ERR_HIP;
      msg = std::string("issuing op ") + std::to_string(x) + ": " + hipGetErrorString(e);
      break;
    }
    ++issued;
  }
  // drain every stream, also after a failure, so no work outlives the call
  for (int k = 0; k < plan.nstreams; ++k) {
    hipError_t e = hipStreamSynchronize(streams[k]);
    if (e != hipSuccess && status == OOC_OK) {
      status = OOC_ERR_HIP;
      msg = std::string("stream synchronise: ") + hipGetErrorString(e);
    }
  }
  const double t1 = now_s();
  if (st) {
    st->t_pipeline_s = t1 - t0;
    st->blocks_done = (status == OOC_OK || status == OOC_ERR_INJECTED) ? d2h_issued : 0;
    if (profile && status == OOC_OK) {
      double th = 0, td = 0, tk = 0;
      std::vector<std::pair<double, double>> copies, kernels;
      for (size_t x = 0; x < issued; ++x) {
        float ms = 0.f, a = 0.f, b = 0.f;
        if (hipEventElapsedTime(&ms, c.tev[2 * x], c.tev[2 * x + 1]) != hipSuccess) continue;
        const bool copy = ops[x].kind == OOC_OP_H2D || ops[x].kind == OOC_OP_D2H;
        if (ops[x].kind == OOC_OP_H2D) th += ms * 1e-3;
        else if (ops[x].kind == OOC_OP_D2H) td += ms * 1e-3;
        else tk += ms * 1e-3;
        if (hipEventElapsedTime(&a, c.tev[0], c.tev[2 * x]) == hipSuccess &&
            hipEventElapsedTime(&b, c.tev[0], c.tev[2 * x + 1]) == hipSuccess)
          (copy ? copies : kernels).emplace_back(a * 1e-3, b * 1e-3);
      }
      st->t_h2d_busy_s = th;
      st->t_d2h_busy_s = td;
      st->t_kernel_busy_s = tk;
      st->overlap = overlap_fraction(copies, kernels);
      // matrix-core kernels alone: FP64 tile kernels are whole ops; split ops
      // count their slice-product launches without the slicing kernels
      double tm = 0.0;
      int64_t nm = 0;
      for (size_t x = 0; x < issued; ++x) {
        if (ops[x].kind == OOC_OP_GEMM) {
          float ms = 0.f;
          if (ops[x].k > 0 && hipEventElapsedTime(&ms, c.tev[2 * x], c.tev[2 * x + 1]) == hipSuccess) {
            tm += ms * 1e-3;
            ++nm;
          }
        } else if (ops[x].kind == OOC_OP_SPLIT_GEMM) {
          for (int64_t y = kfirst[x]; y < kfirst[x + 1]; ++y) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, c.kev[2 * y], c.kev[2 * y + 1]) == hipSuccess) {
              tm += ms * 1e-3;
              ++nm;
            }
          }
        }
      }
      st->t_mma_busy_s = tm;
      st->mma_launches = nm;
      if (timeline) {
        for (size_t x = 0; x < issued && (int64_t)x < timeline_cap; ++x) {
          float a = 0.f, b = 0.f;
          if (hipEventElapsedTime(&a, c.tev[0], c.tev[2 * x]) != hipSuccess) a = -1.f;
          if (hipEventElapsedTime(&b, c.tev[0], c.tev[2 * x + 1]) != hipSuccess) b = -1.f;
          timeline[2 * x] = a * 1e-3;
          timeline[2 * x + 1] = b * 1e-3;
        }
      }
    }
  }
  if (status != OOC_OK) return fail(status, msg);
  return OOC_OK;
}

// Run an operation list on device `dev` (selected, page-lock checks done by
// the caller): the device arena of arena_bytes is opts->arena when given,
// else the device's cached arena (reallocated when too small or larger than
// budget_bytes, freed afterwards with opts->release_arena); pipeline stream x
// is opts->streams[x] when given, else the device's own.
ooc_status exec_list(int dev, const std::vector<ooc_op>& ops, const HostMats& hm, uint64_t arena_bytes,
                     uint64_t budget_bytes, const RunCfg& cfg, const ooc_opts* opts, ooc_stats* stats) {
  DevCtx& c = g_dev[dev];
  std::lock_guard<std::mutex> lock(c.mu);
  ooc_status st = ensure_streams(c);
  if (st != OOC_OK) return st;
  double* arena = nullptr;
  if (opts && opts->arena) {
    if (opts->arena_bytes < arena_bytes) return fail(OOC_ERR_ARG, "opts->arena is smaller than the plan's footprint");
    arena = static_cast<double*>(opts->arena);
  } else {
    if (c.arena && (c.arena_bytes < arena_bytes || c.arena_bytes > budget_bytes)) {
      HIPCHK(hipFree(c.arena), "hipFree");
      c.arena = nullptr;
      c.arena_bytes = 0;
    }
    if (!c.arena && arena_bytes > 0) {
      size_t fr = 0, tot = 0;
      HIPCHK(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
      if (arena_bytes > fr)
        return fail(OOC_ERR_DEVICE_MEM, "plan needs " + std::to_string(arena_bytes) + " bytes, device has " +
                                            std::to_string(fr) + " free");
      hipError_t e = hipMalloc(&c.arena, arena_bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        c.arena = nullptr;
        return fail(OOC_ERR_DEVICE_MEM, std::string("hipMalloc of the arena failed: ") + hipGetErrorString(e));
      }
      c.arena_bytes = arena_bytes;
    }
    arena = static_cast<double*>(c.arena);
  }
  // pipeline streams: the caller's where given (borrowed), else the device's own
  hipStream_t streams[3];
  for (int x = 0; x < 3; ++x)
    streams[x] = (opts && opts->streams[x]) ? static_cast<hipStream_t>(opts->streams[x]) : c.st[x];
  st = run_ops(c, streams, cfg, ops, arena, (int64_t)(arena_bytes / 8), hm, opts && opts->profile,
               opts ? opts->timeline : nullptr, opts ? opts->timeline_cap : 0, stats);
  if (opts && opts->release_arena && !opts->arena && c.arena) {
    // run_ops drained every stream it used, so nothing reads the arena any more
    const hipError_t e = hipFree(c.arena);
    c.arena = nullptr;
    c.arena_bytes = 0;
    if (e != hipSuccess && st == OOC_OK) st = hip_fail(e, "hipFree of the arena");
  }
  return st;
}

ooc_status check_args(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda, const double* B,
                      int64_t ldb, double beta, double* C, int64_t ldc, bool transb = false) {
  (void)beta;
  if (M < 0 || N < 0 || K < 0) return fail(OOC_ERR_ARG, "negative matrix size");
  const bool need_ab = M > 0 && N > 0 && K > 0 && alpha != 0.0;
  if (M > 0 && N > 0) {
    if (!C) return fail(OOC_ERR_ARG, "C is NULL");
    if (ldc < N) return fail(OOC_ERR_ARG, "ldc < N");
  }
  if (need_ab) {
    if (!A || !B) return fail(OOC_ERR_ARG, "A or B is NULL");
    if (lda < K) return fail(OOC_ERR_ARG, "lda < K");
    if (transb ? ldb < K : ldb < N) return fail(OOC_ERR_ARG, transb ? "ldb < K (B transposed)" : "ldb < N");
  }
  return OOC_OK;
}

ooc_status gemm_impl(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda, const double* B,
                     int64_t ldb, double beta, double* C, int64_t ldc, size_t budget_bytes, const ooc_plan_t* given,
                     const ooc_opts* opts, ooc_stats* stats, bool transb = false, bool lower = false,
                     bool allow_sweep = true);

namespace {
// Plans chosen by the measured sweep, keyed by what the choice depends on.
struct SweepKey {
  int64_t M, N, K;
  bool beta_nonzero;
  uint64_t budget;
  int precision, slices, nstreams;
  bool transb, lower;
  bool operator<(const SweepKey& o) const {
    return std::tie(M, N, K, beta_nonzero, budget, precision, slices, nstreams, transb, lower) <
           std::tie(o.M, o.N, o.K, o.beta_nonzero, o.budget, o.precision, o.slices, o.nstreams, o.transb, o.lower);
  }
};
std::mutex g_sweep_mu;
std::map<SweepKey, ooc_plan_t> g_sweep;
}  // namespace

// The measured sweep: the cost model's n best candidates, each timed by one
// product on the caller's A and B into a page-locked scratch C of C's shape
// (zeroed, so that beta * C stays finite), after one warm-up product that
// also allocates the device arena; the fastest is returned and remembered.
// Without a scratch C the model's choice is returned and not remembered.
ooc_status sweep_plan(const Problem& pb, const double* A, int64_t lda, const double* B, int64_t ldb,
                      size_t budget_bytes, const ooc_opts* opts, ooc_plan_t* out) {
  const SweepKey key{pb.M, pb.N, pb.keff(), pb.beta != 0.0, budget_bytes, opts ? opts->precision : 0,
                     opts ? opts->slices : 0, opts ? opts->nstreams : 0, pb.transb, pb.lower};
  {
    std::lock_guard<std::mutex> lock(g_sweep_mu);
    auto it = g_sweep.find(key);
    if (it != g_sweep.end()) {
      *out = it->second;
      return OOC_OK;
    }
  }
  ooc_opts mo{};
  if (opts) mo = *opts;
  mo.planner = OOC_PLAN_MODEL;
  mo.profile = 0;
  mo.timeline = nullptr;
  mo.timeline_cap = 0;
  std::vector<ooc_plan_t> plans;
  std::vector<double> times;
  ooc_status st = plan_candidates(pb, budget_bytes, &mo, &plans, &times);
  if (st != OOC_OK) return st;
  const size_t n = std::min<size_t>(plans.size(), (size_t)std::max(1, env_int("OOC_SWEEP_TOP", 8)));
  *out = plans[0];
  if (n == 1) return OOC_OK;
  double* scratch = nullptr;
  const size_t cbytes = (size_t)pb.M * (size_t)pb.N * sizeof(double);
  if (hipHostMalloc(reinterpret_cast<void**>(&scratch), cbytes) != hipSuccess) {
    (void)hipGetLastError();
    return OOC_OK;
  }
  std::memset(scratch, 0, cbytes);
  size_t best = 0;
  double best_t = 0.0;
  for (size_t c = 0; c <= n && st == OOC_OK; ++c) {
    const size_t x = c == 0 ? 0 : c - 1;  // trial 0 warms up with the model's choice
    ooc_stats ts{};
    const double t0 = now_s();
    st = gemm_impl(pb.M, pb.N, pb.K, pb.alpha, A, lda, B, ldb, pb.beta, scratch, pb.N, budget_bytes, &plans[x], &mo,
                   &ts, pb.transb, pb.lower, false);
    const double dt = now_s() - t0;
    if (st == OOC_OK && c > 0 && (c == 1 || dt < best_t)) {
      best = x;
      best_t = dt;
    }
  }
  (void)hipHostFree(scratch);
  if (st != OOC_OK) return st;
  *out = plans[best];
  std::lock_guard<std::mutex> lock(g_sweep_mu);
  if (g_sweep.size() > 4096) g_sweep.clear();
  g_sweep[key] = plans[best];
  return OOC_OK;
}

ooc_status gemm_impl(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda, const double* B,
                     int64_t ldb, double beta, double* C, int64_t ldc, size_t budget_bytes, const ooc_plan_t* given,
                     const ooc_opts* opts, ooc_stats* stats, bool transb, bool lower, bool allow_sweep) {
  const double t_enter = now_s();
  if (stats) std::memset(stats, 0, sizeof(*stats));
  ooc_status st = check_args(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, transb);
  if (st != OOC_OK) return st;
  if (M == 0 || N == 0) return OOC_OK;
  if (lower && opts && opts->precision != OOC_FP64)
    return fail(OOC_ERR_ARG, "lower-triangle products run in FP64 precision only");
  Problem pb;
  pb.M = M; pb.N = N; pb.K = K; pb.alpha = alpha; pb.beta = beta;
  pb.transb = transb;
  pb.lower = lower;
  ooc_plan_t plan;
  double predicted = 0.0;
  bool measured = false;  // chosen by the measured sweep: its prediction is simulated below
  if (given) {
    plan = *given;
  } else {
    bool declined = false;
    st = choose_plan(pb, budget_bytes, opts, &plan, &predicted, &declined);
    if (st != OOC_OK) return st;
    const int planner = opts ? opts->planner : OOC_PLAN_AUTO;
    if (allow_sweep && (planner == OOC_PLAN_SWEEP || (planner == OOC_PLAN_MLP && declined))) {
      // the operands are page-locked (checked again below); the sweep's
      // trial products need them to be
      if (pb.keff() > 0 && (!range_pinned(A, M, K, lda) || !(transb ? range_pinned(B, N, K, ldb)
                                                                      : range_pinned(B, K, N, ldb))))
        return fail(OOC_ERR_NOT_PINNED, "A or B is not page-locked host memory (use ooc_host_alloc)");
      st = ensure_device(opts ? opts->device : 0);
      if (st != OOC_OK) return st;
      st = sweep_plan(pb, A, lda, B, ldb, budget_bytes, opts, &plan);
      if (st != OOC_OK) return st;
      measured = true;
    }
  }
  Layout lay;
  st = plan_layout(pb, plan, &lay);
  if (st != OOC_OK) return st;
  if (lay.bytes > budget_bytes)
    return fail(OOC_ERR_BUDGET, "plan footprint " + std::to_string(lay.bytes) + " bytes exceeds the budget of " +
                                    std::to_string(budget_bytes));
  std::vector<ooc_op> ops;
  st = build_schedule(pb, plan, lay, &ops);
  if (st != OOC_OK) return st;
  if (given || measured) predicted = simulate(pb, plan, ops);
  const double t_plan = now_s() - t_enter;

  const int dev = opts ? opts->device : 0;
  st = ensure_device(dev);
  if (st != OOC_OK) return st;
  const int64_t keff = pb.keff();
  if (keff > 0 && (!range_pinned(A, M, K, lda) || !(transb ? range_pinned(B, N, K, ldb) : range_pinned(B, K, N, ldb))))
    return fail(OOC_ERR_NOT_PINNED, "A or B is not page-locked host memory (use ooc_host_alloc)");
  if (!range_pinned(C, M, N, ldc)) return fail(OOC_ERR_NOT_PINNED, "C is not page-locked host memory (use ooc_host_alloc)");

  HostMats hm{{const_cast<double*>(A), lda}, {const_cast<double*>(B), ldb}, {C, ldc}};
  st = exec_list(dev, ops, hm, lay.bytes, budget_bytes, RunCfg{plan.nstreams, plan.precision, plan.slices}, opts,
                 stats);
  if (stats) {
    stats->t_plan_s = t_plan;
    stats->plan = plan;
    stats->t_total_s = now_s() - t_enter;
    stats->t_predicted_s = predicted;
    // useful flops: every element of C, or with lower those with i >= j
    const double elems = !lower ? (double)M * (double)N
                                : (M >= N ? (double)N * (N + 1) / 2.0 + (double)(M - N) * N : (double)M * (M + 1) / 2.0);
    stats->flops = 2.0 * elems * (double)K;
    stats->arena_bytes = lay.bytes;
    stats->ops = (int64_t)ops.size();
    int64_t tasks = 0, kern = 0;
    uint64_t bh = 0, bd = 0;
    for (const ooc_op& o : ops) {
      if (o.kind == OOC_OP_H2D) bh += (uint64_t)(o.rows * o.cols) * 8;
      else if (o.kind == OOC_OP_D2H) bd += (uint64_t)(o.rows * o.cols) * 8;
      else ++kern;
      if (o.kind == OOC_OP_GEMM || o.kind == OOC_OP_SPLIT_GEMM) ++tasks;
    }
    stats->tasks = tasks;
    stats->kernels = kern;
    stats->bytes_h2d = bh;
    stats->bytes_d2h = bd;
  }
  if (env_int("OOC_LOG", 0) > 0) {
    // one line per call on stderr: problem, plan, times and outcome
    std::fprintf(stderr,
                 "[ooc] M=%lld N=%lld K=%lld budget=%llu plan mb=%lld nb=%lld kb=%lld order=%d bufs=%d/%d/%d/%d "
                 "streams=%d group=%d %s%s ops=%zu arena=%llu t=%.6fs predicted=%.6fs status=%d\n",
                 (long long)M, (long long)N, (long long)K, (unsigned long long)budget_bytes, (long long)plan.mb,
                 (long long)plan.nb, (long long)plan.kb, plan.order, plan.nbuf_a, plan.nbuf_b, plan.nbuf_c,
                 plan.nbuf_d, plan.nstreams, plan.group,
                 plan.precision == OOC_SPLIT_BF16 ? "split-bf16 s=" : (plan.precision == OOC_SPLIT_INT8 ? "split-int8 s=" : "fp64"),
                 plan.precision != OOC_FP64 ? std::to_string(plan.slices).c_str() : "", ops.size(),
                 (unsigned long long)lay.bytes, now_s() - t_enter, predicted, (int)st);
  }
  return st;
}

// Totals of one more call's stats into `t` (ooc_potrf adds its products and panels).
void add_stats(ooc_stats* t, const ooc_stats& s) {
  t->t_pipeline_s += s.t_pipeline_s;
  t->t_h2d_busy_s += s.t_h2d_busy_s;
  t->t_d2h_busy_s += s.t_d2h_busy_s;
  t->t_kernel_busy_s += s.t_kernel_busy_s;
  t->t_plan_s += s.t_plan_s;
  t->t_mma_busy_s += s.t_mma_busy_s;
  t->mma_launches += s.mma_launches;
  t->bytes_h2d += s.bytes_h2d;
  t->bytes_d2h += s.bytes_d2h;
  t->arena_bytes = std::max(t->arena_bytes, s.arena_bytes);
  t->ops += s.ops;
  t->tasks += s.tasks;
  t->kernels += s.kernels;
}

// Copy and kernel counts and bytes of an operation list (stats of ooc_run_ops and the panels of ooc_potrf).
void list_stats(const std::vector<ooc_op>& ops, ooc_stats* st) {
  for (const ooc_op& o : ops) {
    if (o.kind == OOC_OP_H2D) st->bytes_h2d += (uint64_t)(o.rows * o.cols) * 8;
    else if (o.kind == OOC_OP_D2H) st->bytes_d2h += (uint64_t)(o.rows * o.cols) * 8;
    else ++st->kernels;
  }
  st->ops = (int64_t)ops.size();
}

// Panel width of the out-of-core Cholesky factorisation: the largest multiple
// of 64 up to 8192 (and N rounded up to 64) whose b x b diagonal block takes
// at most a quarter of the budget, leaving the rest to the two chunk buffers
// of the solve (tall chunks keep the device solve's products wide), with at
// least 256 rows per chunk.
int64_t potrf_panel(int64_t N, uint64_t budget_elems) {
  int64_t b = std::min<int64_t>(8192, (N + 63) / 64 * 64);
  auto fits = [&](int64_t x) {
    return (uint64_t)(x * x) <= budget_elems / 4 && (uint64_t)(x * x + 2 * 256 * x + 8) <= budget_elems;
  };
  while (b > 64 && !fits(b)) b -= 64;
  return fits(b) ? b : 0;
}

// Plan, on a host thread, the out-of-core product of a level-3 routine's
// next block column while the device works on the current one: the plan lands
// in the plan cache, where the product's own call finds it (planning a new
// shape takes tens of milliseconds on the host).
std::future<void> plan_ahead(int64_t M, int64_t N, int64_t K, bool transb, bool lower, size_t budget_bytes,
                             const ooc_opts& opts) {
  Problem pb;
  pb.M = M; pb.N = N; pb.K = K; pb.alpha = -1.0; pb.beta = 1.0;
  pb.transb = transb;
  pb.lower = lower;
  return std::async(std::launch::async, [pb, budget_bytes, opts]() {
    (void)hipSetDevice(opts.device);  // the learned planner's inference runs on the caller's device
    ooc_plan_t p;
    (void)choose_plan(pb, budget_bytes, &opts, &p, nullptr);
  });
}

// Append op `o` with the wait set `waits` (negative entries skipped); returns its index.
int push_op(std::vector<ooc_op>& ops, ooc_op o, std::initializer_list<int> waits) {
  o.nwait = 0;
  for (int w : waits)
    if (w >= 0) o.wait[o.nwait++] = w;
  ops.push_back(o);
  return (int)ops.size() - 1;
}

// Ops that solve rows [i0, i0 + rows) x columns [j0, j0 + jb) of host matrix
// `mat` against the lower-triangular jb x jb block at arena offset 0 (X <- X
// L^{-T}, or X <- X L^{-1} with `back`), in chunks of r rows through two arena buffers after `base`
// elements: H2D on stream 0, TRSM on stream 1 (also after op `after` when it
// is >= 0), D2H on stream 2; a buffer is refilled only after its last chunk
// went home.
void append_chunked_solve(std::vector<ooc_op>& ops, int mat, int64_t i0, int64_t rows, int64_t j0, int64_t jb,
                          int64_t base, int64_t r, int after, bool back = false) {
  int home[2] = {-1, -1};
  for (int64_t q = 0; q * r < rows; ++q) {
    const int64_t r0 = i0 + q * r, rr = std::min(r, rows - q * r);
    const int buf = (int)(q & 1);
    ooc_op o{};
    o.kind = OOC_OP_H2D; o.stream = 0; o.mat = mat;
    o.row0 = r0; o.col0 = j0; o.rows = rr; o.cols = jb; o.off_c = base + buf * r * jb; o.ld_c = jb;
    const int h = push_op(ops, o, {home[buf]});
    o = ooc_op{};
    o.kind = OOC_OP_TRSM; o.stream = 1; o.rows = rr; o.cols = jb;
    o.off_c = base + buf * r * jb; o.ld_c = jb; o.off_a = 0; o.ld_a = jb;
    o.flags = back ? OOC_OPF_BACK : 0;
    const int k = push_op(ops, o, {h, after});
    o = ooc_op{};
    o.kind = OOC_OP_D2H; o.stream = 2; o.mat = mat;
    o.row0 = r0; o.col0 = j0; o.rows = rr; o.cols = jb; o.off_c = base + buf * r * jb; o.ld_c = jb;
    home[buf] = push_op(ops, o, {k});
  }
}

ooc_status potrf_impl(int64_t N, double* A, int64_t lda, size_t budget_bytes, const ooc_opts* opts, int64_t* info,
                      ooc_stats* stats) {
  const double t_enter = now_s();
  ooc_stats total{};
  if (info) *info = 0;
  if (N < 0) return fail(OOC_ERR_ARG, "negative matrix size");
  if (N == 0) {
    if (stats) *stats = total;
    return OOC_OK;
  }
  if (!A || lda < N) return fail(OOC_ERR_ARG, "bad A or lda");
  const int64_t b = potrf_panel(N, budget_bytes / 8);
  if (b == 0) return fail(OOC_ERR_BUDGET, "the budget holds no 64-column panel of the factorisation");
  const int dev = opts ? opts->device : 0;
  ooc_status st = ensure_device(dev);
  if (st != OOC_OK) return st;
  if (!range_pinned(A, N, N, lda)) return fail(OOC_ERR_NOT_PINNED, "A is not page-locked host memory");
  ooc_opts gopts{};
  if (opts) gopts = *opts;
  gopts.precision = OOC_FP64;
  gopts.timeline = nullptr;
  gopts.timeline_cap = 0;
  double* hstat = nullptr;  // the panel's status word comes home here
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hstat), 8), "hipHostMalloc");
  for (int64_t j0 = 0; j0 < N && st == OOC_OK; j0 += b) {
    const int64_t jb = std::min(b, N - j0);
    double* panel = A + j0 * lda + j0;
    // the block column's update by the columns to its left: C = C - L_left L_top^T (lower triangle)
    if (j0 > 0) {
      ooc_stats gs{};
      st = gemm_impl(N - j0, jb, j0, -1.0, A + j0 * lda, lda, A + j0 * lda, lda, 1.0, panel, lda, budget_bytes,
                     nullptr, &gopts, &gs, true, true, false);
      add_stats(&total, gs);
      if (st != OOC_OK) break;
    }
    // the panel: factor the diagonal block, then solve the rows below against it in chunks
    const int64_t below = N - j0 - jb;
    const int64_t base = jb * jb + 8;  // chunk buffers after the block and the status word
    const int64_t r = below > 0 ? std::max<int64_t>(1, std::min<int64_t>(below, ((int64_t)(budget_bytes / 8) - base) / (2 * jb))) : 0;
    std::vector<ooc_op> ops;
    ooc_op o{};
    o.kind = OOC_OP_H2D; o.stream = 0; o.mat = 0;
    o.row0 = j0; o.col0 = j0; o.rows = jb; o.cols = jb; o.off_c = 0; o.ld_c = jb;
    const int h_diag = push_op(ops, o, {});
    o = ooc_op{};
    o.kind = OOC_OP_H2D; o.stream = 0; o.mat = 1; o.rows = 1; o.cols = 1; o.off_c = jb * jb; o.ld_c = 1;
    const int h_stat = push_op(ops, o, {});
    o = ooc_op{};
    o.kind = OOC_OP_POTRF; o.stream = 1; o.rows = jb; o.cols = jb; o.off_c = 0; o.ld_c = jb;
    o.off_w = jb * jb; o.len_w = 1; o.k0 = j0;
    const int k_potrf = push_op(ops, o, {h_diag, h_stat});
    o = ooc_op{};
    o.kind = OOC_OP_D2H; o.stream = 2; o.mat = 0;
    o.row0 = j0; o.col0 = j0; o.rows = jb; o.cols = jb; o.off_c = 0; o.ld_c = jb;
    push_op(ops, o, {k_potrf});
    o = ooc_op{};
    o.kind = OOC_OP_D2H; o.stream = 2; o.mat = 1; o.rows = 1; o.cols = 1; o.off_c = jb * jb; o.ld_c = 1;
    push_op(ops, o, {k_potrf});
    // the solves run on stream 1 after the factorisation
    append_chunked_solve(ops, 0, j0 + jb, below, j0, jb, base, r, -1);
    *hstat = 0.0;
    ooc_stats ps{};
    HostMats hm{{A, lda}, {hstat, 1}};
    const uint64_t arena_bytes = (uint64_t)(base + 2 * r * jb) * 8;
    std::future<void> next;  // the next block column's update, planned meanwhile
    if (j0 + jb < N) next = plan_ahead(N - j0 - jb, std::min(b, N - j0 - jb), j0 + jb, true, true, budget_bytes, gopts);
    st = exec_list(dev, ops, hm, arena_bytes, budget_bytes, RunCfg{3, OOC_FP64, 0}, &gopts, &ps);
    if (next.valid()) next.wait();
    list_stats(ops, &ps);
    ps.arena_bytes = arena_bytes;
    add_stats(&total, ps);
    if (st == OOC_OK && *hstat != 0.0) {
      if (info) *info = (int64_t)*hstat;
      st = fail(OOC_ERR_NOT_SPD, "the matrix is not positive definite: pivot " + std::to_string((int64_t)*hstat - 1) +
                                     " is not positive");
      break;
    }
    if (st == OOC_OK) ++total.blocks_done;
  }
  (void)hipHostFree(hstat);
  const double n = (double)N;
  total.flops = n * n * n / 3.0 + n * n / 2.0 + n / 6.0;
  total.t_total_s = now_s() - t_enter;
  if (stats) *stats = total;
  return st;
}

// Out-of-core triangular solve Y L^T = X (X <- X L^{-T}, the right-hand,
// lower, transposed form; Y^T = L^{-1} X^T is forward substitution for the
// columns of X^T), left-looking by block columns of b columns (the panel rule
// of the factorisation): block column j of X is first updated by the columns
// to its left, X_j = X_j - Y_left L_j,left^T (one out-of-core product with a
// transposed B), then solved against the diagonal block L_jj on the device,
// chunk by chunk.  With `back` it solves Y L = X (X <- X L^{-1}, back
// substitution for the columns of X^T: L^T Y^T = X^T) instead, walking the
// same block columns from the last: X_j = X_j - Y_right L_right,j (an
// out-of-core product without transposition), then X_j <- X_j L_jj^{-1}.
ooc_status trsm_impl(int64_t M, int64_t N, const double* L, int64_t ldl, double* X, int64_t ldx, size_t budget_bytes,
                     const ooc_opts* opts, ooc_stats* stats, bool back = false) {
  const double t_enter = now_s();
  ooc_stats total{};
  if (M < 0 || N < 0) return fail(OOC_ERR_ARG, "negative matrix size");
  if (M == 0 || N == 0) {
    if (stats) *stats = total;
    return OOC_OK;
  }
  if (!L || ldl < N || !X || ldx < N) return fail(OOC_ERR_ARG, "bad L, X or leading dimension");
  const int64_t b = potrf_panel(N, budget_bytes / 8);
  if (b == 0) return fail(OOC_ERR_BUDGET, "the budget holds no 64-column panel of the solve");
  const int dev = opts ? opts->device : 0;
  ooc_status st = ensure_device(dev);
  if (st != OOC_OK) return st;
  if (!range_pinned(L, N, N, ldl)) return fail(OOC_ERR_NOT_PINNED, "L is not page-locked host memory");
  if (!range_pinned(X, M, N, ldx)) return fail(OOC_ERR_NOT_PINNED, "X is not page-locked host memory");
  ooc_opts gopts{};
  if (opts) gopts = *opts;
  gopts.precision = OOC_FP64;
  gopts.timeline = nullptr;
  gopts.timeline_cap = 0;
  const int64_t nblk = (N + b - 1) / b;
  for (int64_t step = 0; step < nblk && st == OOC_OK; ++step) {
    const int64_t j0 = (back ? nblk - 1 - step : step) * b;
    const int64_t jb = std::min(b, N - j0);
    // the columns already solved that update this block column
    const int64_t kdone = back ? N - j0 - jb : j0;
    if (kdone > 0) {
      ooc_stats gs{};
      if (back)  // X_j = X_j - Y_right L_right,j
        st = gemm_impl(M, jb, kdone, -1.0, X + j0 + jb, ldx, L + (j0 + jb) * ldl + j0, ldl, 1.0, X + j0, ldx,
                       budget_bytes, nullptr, &gopts, &gs, false, false, false);
      else  // X_j = X_j - Y_left L_j,left^T
        st = gemm_impl(M, jb, j0, -1.0, X, ldx, L + j0 * ldl, ldl, 1.0, X + j0, ldx, budget_bytes, nullptr, &gopts,
                       &gs, true, false, false);
      add_stats(&total, gs);
      if (st != OOC_OK) break;
    }
    // L_jj in, then the rows of X_j through two chunk buffers
    const int64_t base = jb * jb;
    const int64_t r = std::max<int64_t>(1, std::min<int64_t>(M, ((int64_t)(budget_bytes / 8) - base) / (2 * jb)));
    std::vector<ooc_op> ops;
    ooc_op o{};
    o.kind = OOC_OP_H2D; o.stream = 0; o.mat = 1;
    o.row0 = j0; o.col0 = j0; o.rows = jb; o.cols = jb; o.off_c = 0; o.ld_c = jb;
    const int h_diag = push_op(ops, o, {});
    append_chunked_solve(ops, 0, 0, M, j0, jb, base, r, h_diag, back);
    ooc_stats ps{};
    HostMats hm{{X, ldx}, {const_cast<double*>(L), ldl}};
    const uint64_t arena_bytes = (uint64_t)(base + 2 * r * jb) * 8;
    std::future<void> next;  // the next block column's update, planned meanwhile
    if (step + 1 < nblk) {  // forward: the next block may be the ragged last one; back: blocks are whole
      const int64_t nb = back ? b : std::min(b, N - j0 - jb);
      next = plan_ahead(M, nb, kdone + jb, !back, false, budget_bytes, gopts);
    }
    st = exec_list(dev, ops, hm, arena_bytes, budget_bytes, RunCfg{3, OOC_FP64, 0}, &gopts, &ps);
    if (next.valid()) next.wait();
    list_stats(ops, &ps);
    ps.arena_bytes = arena_bytes;
    add_stats(&total, ps);
    if (st == OOC_OK) ++total.blocks_done;
  }
  total.flops = (double)M * (double)N * (double)N;
  total.t_total_s = now_s() - t_enter;
  if (stats) *stats = total;
  return st;
}

// ---- accumulation sessions: C += alpha_s * A_s * B_s over several calls ---------------
//
// The paper's MMOOC can be called once per step of an outer algorithm (SUMMA
// or HSUMMA, Section V, the step/nsteps logic of Fig. 2): C is read at the
// first step only, and the C blocks still on the device at the end of a step
// are written back only after the last one.  A session generalises this: the
// first R rows of C (as many as fit in half the budget) stay on the device for
// the whole session, are loaded once (when beta != 0) and written back once at
// the end; the remaining rows are streamed through the other half by the
// ordinary pipeline at every step (read and written back each time).

// Rows of C a session keeps on the device: all of C when it takes at most
// half the budget, else as many rows as fit in half the budget, a multiple of
// 128 (the tile height) when there are at least 128.
int64_t accum_resident_rows(int64_t M, int64_t N, uint64_t budget) {
  if (M <= 0 || N <= 0) return 0;
  const uint64_t half = budget / 2;
  if ((uint64_t)M * (uint64_t)N * 8u <= half) return M;
  int64_t r = (int64_t)(half / (8u * (uint64_t)N));
  if (r >= 128) r = r / 128 * 128;
  return std::min(r, M);
}

// One part of a session step: rows [0, R) with C resident (part 0) or rows
// [R, M) streamed through buffers placed after the resident rows (part 1).
// Host rows of part 1 count from row R.
ooc_status accum_part(int part, int64_t M, int64_t N, int64_t K, double alpha, double beta_eff, int64_t R,
                      uint64_t budget, const ooc_opts* opts, Problem* pb_out, ooc_plan_t* plan, Layout* lay,
                      std::vector<ooc_op>* ops, double* predicted) {
  Problem pb;
  pb.N = N; pb.K = K; pb.alpha = alpha; pb.beta = beta_eff;
  pb.base = R > 0 ? ceil_div(R * N, 32) * 32 : 0;
  if (part == 0) {
    pb.M = R;
    pb.c_resident = true;
    pb.c_ld = N;
  } else {
    pb.M = M - R;
  }
  *pb_out = pb;
  ops->clear();
  if (pb.M <= 0 || N <= 0) return OOC_OK;
  ooc_status st = choose_plan(pb, budget, opts, plan, predicted);
  if (st != OOC_OK) return st;
  st = plan_layout(pb, *plan, lay);
  if (st != OOC_OK) return st;
  if (lay->bytes > budget) return fail(OOC_ERR_BUDGET, "session step plan exceeds the budget");
  return build_schedule(pb, *plan, *lay, ops);
}

}  // namespace

ooc_status use_device(int dev) { return ensure_device(dev); }

}  // namespace ooc

struct ooc_accum_s {
  int dev = 0;
  int64_t M = 0, N = 0;
  double beta = 0.0;
  double* C = nullptr;
  int64_t ldc = 0;
  uint64_t budget = 0;
  ooc_opts opts{};
  int64_t R = 0;         // resident rows
  void* mem = nullptr;   // session arena: resident C rows, then the step plans' buffers
  int64_t steps = 0;
};

namespace ooc {
namespace {

// Step of a session (the device lease is held by the caller).
ooc_status accum_step_locked(DevCtx& c, ooc_accum_s* a, int64_t K, double alpha, const double* A, int64_t lda,
                             const double* B, int64_t ldb, ooc_stats* stats) {
  const double t_enter = now_s();
  const double beta_eff = a->steps == 0 ? a->beta : 1.0;
  hipStream_t streams[3];
  for (int x = 0; x < 3; ++x)
    streams[x] = a->opts.streams[x] ? static_cast<hipStream_t>(a->opts.streams[x]) : c.st[x];
  ooc_stats total{};
  for (int part = 0; part < 2; ++part) {
    Problem pb;
    ooc_plan_t plan{};
    Layout lay;
    std::vector<ooc_op> ops;
    double pred = 0.0;
    ooc_status st = accum_part(part, a->M, a->N, K, alpha, beta_eff, a->R, a->budget, &a->opts, &pb, &plan, &lay,
                               &ops, &pred);
    if (st != OOC_OK) return st;
    if (ops.empty()) continue;
    const int64_t r0 = part == 0 ? 0 : a->R;
    HostMats hm{{const_cast<double*>(A ? A + r0 * lda : nullptr), lda}, {const_cast<double*>(B), ldb},
                {a->C + r0 * a->ldc, a->ldc}};
    ooc_stats ps{};
    const double t_plan = now_s() - t_enter;
    st = run_ops(c, streams, RunCfg{plan.nstreams, plan.precision, plan.slices}, ops, static_cast<double*>(a->mem),
                 (int64_t)(lay.bytes / 8), hm,
                 a->opts.profile != 0, nullptr, 0, &ps);
    total.plan = plan;
    total.t_plan_s = t_plan;
    total.t_pipeline_s += ps.t_pipeline_s;
    total.t_h2d_busy_s += ps.t_h2d_busy_s;
    total.t_d2h_busy_s += ps.t_d2h_busy_s;
    total.t_kernel_busy_s += ps.t_kernel_busy_s;
    total.t_mma_busy_s += ps.t_mma_busy_s;
    total.mma_launches += ps.mma_launches;
    total.t_predicted_s += pred;
    total.arena_bytes = std::max<uint64_t>(total.arena_bytes, lay.bytes);
    total.ops += (int64_t)ops.size();
    total.blocks_done += ps.blocks_done;
    for (const ooc_op& o : ops) {
      if (o.kind == OOC_OP_H2D) total.bytes_h2d += (uint64_t)(o.rows * o.cols) * 8;
      else if (o.kind == OOC_OP_D2H) total.bytes_d2h += (uint64_t)(o.rows * o.cols) * 8;
      else ++total.kernels;
      if (o.kind == OOC_OP_GEMM || o.kind == OOC_OP_SPLIT_GEMM) ++total.tasks;
    }
    if (st != OOC_OK) {
      if (stats) *stats = total;
      return st;
    }
  }
  ++a->steps;
  total.flops = 2.0 * (double)a->M * (double)a->N * (double)K;
  total.t_total_s = now_s() - t_enter;
  if (stats) *stats = total;
  return OOC_OK;
}

}  // namespace
}  // namespace ooc

using namespace ooc;

extern "C" {

ooc_status ooc_gemm(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda, const double* B,
                    int64_t ldb, double beta, double* C, int64_t ldc, size_t budget_bytes, const ooc_opts* opts,
                    ooc_stats* stats) {
  return gemm_impl(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, budget_bytes, nullptr, opts, stats);
}

ooc_status ooc_gemm_ex(int32_t transb, int32_t lower, int64_t M, int64_t N, int64_t K, double alpha,
                       const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                       int64_t ldc, size_t budget_bytes, const ooc_opts* opts, ooc_stats* stats) {
  if ((transb != 0 && transb != 1) || (lower != 0 && lower != 1))
    return fail(OOC_ERR_ARG, "transb and lower must be 0 or 1");
  return gemm_impl(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, budget_bytes, nullptr, opts, stats, transb != 0,
                   lower != 0);
}

ooc_status ooc_syrk(int64_t N, int64_t K, double alpha, const double* A, int64_t lda, double beta, double* C,
                    int64_t ldc, size_t budget_bytes, const ooc_opts* opts, ooc_stats* stats) {
  return ooc_gemm_ex(1, 1, N, N, K, alpha, A, lda, A, lda, beta, C, ldc, budget_bytes, opts, stats);
}

ooc_status ooc_potrf(int64_t N, double* A, int64_t lda, size_t budget_bytes, const ooc_opts* opts, int64_t* info,
                     ooc_stats* stats) {
  if (stats) std::memset(stats, 0, sizeof(*stats));
  return potrf_impl(N, A, lda, budget_bytes, opts, info, stats);
}

ooc_status ooc_trsm(int64_t M, int64_t N, const double* L, int64_t ldl, double* X, int64_t ldx, size_t budget_bytes,
                    const ooc_opts* opts, ooc_stats* stats) {
  if (stats) std::memset(stats, 0, sizeof(*stats));
  return trsm_impl(M, N, L, ldl, X, ldx, budget_bytes, opts, stats);
}

ooc_status ooc_trsm_ex(int32_t trans, int64_t M, int64_t N, const double* L, int64_t ldl, double* X, int64_t ldx,
                       size_t budget_bytes, const ooc_opts* opts, ooc_stats* stats) {
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (trans != 0 && trans != 1) return fail(OOC_ERR_ARG, "trans must be 0 or 1");
  return trsm_impl(M, N, L, ldl, X, ldx, budget_bytes, opts, stats, trans == 0);
}

ooc_status ooc_potrs(int64_t M, int64_t N, const double* L, int64_t ldl, double* B, int64_t ldb, size_t budget_bytes,
                     const ooc_opts* opts, ooc_stats* stats) {
  if (stats) std::memset(stats, 0, sizeof(*stats));
  ooc_stats fwd{}, bwd{};
  ooc_status st = trsm_impl(M, N, L, ldl, B, ldb, budget_bytes, opts, &fwd, false);
  if (st == OOC_OK) st = trsm_impl(M, N, L, ldl, B, ldb, budget_bytes, opts, &bwd, true);
  if (stats) {
    add_stats(stats, fwd);
    add_stats(stats, bwd);
    stats->flops = 2.0 * (double)M * (double)N * (double)N;
    stats->t_total_s = fwd.t_total_s + bwd.t_total_s;
    stats->blocks_done = fwd.blocks_done + bwd.blocks_done;
  }
  return st;
}

ooc_status ooc_run_ops(const ooc_op* ops, int64_t nops, const ooc_host_matrix* mats, int32_t nmats,
                       uint64_t arena_bytes, const ooc_opts* opts, ooc_stats* stats) {
  const double t_enter = now_s();
  if (stats) std::memset(stats, 0, sizeof(*stats));
  const int prec = opts ? opts->precision : OOC_FP64;
  const int slices = (opts && opts->slices > 0) ? opts->slices : 6;
  int ns = 1;
  ooc_status st = validate_ops(ops, nops, mats, nmats, (int64_t)(arena_bytes / 8), prec, slices, &ns);
  if (st != OOC_OK) return st;
  if (nops == 0) return OOC_OK;
  const int dev = opts ? opts->device : 0;
  st = ensure_device(dev);
  if (st != OOC_OK) return st;
  std::vector<char> used(nmats, 0);
  for (int64_t x = 0; x < nops; ++x)
    if (ops[x].kind == OOC_OP_H2D || ops[x].kind == OOC_OP_D2H) used[ops[x].mat] = 1;
  HostMats hm;
  for (int m = 0; m < nmats; ++m) {
    if (used[m] && !range_pinned(mats[m].ptr, mats[m].rows, mats[m].cols, mats[m].ld))
      return fail(OOC_ERR_NOT_PINNED, "host matrix " + std::to_string(m) + " is not page-locked");
    hm.push_back({mats[m].ptr, mats[m].ld});
  }
  std::vector<ooc_op> v(ops, ops + nops);
  st = exec_list(dev, v, hm, arena_bytes, arena_bytes, RunCfg{ns, prec, slices}, opts, stats);
  if (stats) {
    list_stats(v, stats);
    stats->arena_bytes = arena_bytes;
    stats->t_total_s = now_s() - t_enter;
  }
  return st;
}

ooc_status ooc_check_ops(const ooc_op* ops, int64_t nops, int64_t* x, int64_t* y) {
  if (nops < 0 || (nops > 0 && !ops) || !x || !y) return fail(OOC_ERR_ARG, "NULL argument");
  if (nops > 32768) return fail(OOC_ERR_CAPACITY, "ooc_check_ops handles at most 32768 ops");
  for (int64_t k = 0; k < nops; ++k)
    for (int w = 0; w < ops[k].nwait; ++w)
      if (ops[k].nwait > OOC_MAX_WAITS || ops[k].wait[w] < 0 || ops[k].wait[w] >= k)
        return fail(OOC_ERR_ARG, "op " + std::to_string(k) + " waits on an op that is not earlier in the list");
  *x = *y = -1;
  if (find_hazard(ops, nops, x, y))
    return fail(OOC_ERR_ARG, "ops " + std::to_string(*y) + " and " + std::to_string(*x) +
                                 " touch a common arena element, one writing it, and are not ordered");
  return OOC_OK;
}

ooc_status ooc_gemm_planned(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                            const double* B, int64_t ldb, double beta, double* C, int64_t ldc, size_t budget_bytes,
                            const ooc_plan_t* plan, const ooc_opts* opts, ooc_stats* stats) {
  if (!plan) return fail(OOC_ERR_ARG, "plan is NULL");
  return gemm_impl(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, budget_bytes, plan, opts, stats);
}

ooc_status ooc_plan(int64_t M, int64_t N, int64_t K, double beta, size_t budget_bytes, const ooc_opts* opts,
                    ooc_plan_t* out) {
  if (!out) return fail(OOC_ERR_ARG, "out is NULL");
  if (M <= 0 || N <= 0 || K < 0) return fail(OOC_ERR_ARG, "M and N must be positive, K non-negative");
  Problem pb;
  pb.M = M; pb.N = N; pb.K = K; pb.alpha = 1.0; pb.beta = beta;
  return choose_plan(pb, budget_bytes, opts, out, nullptr);
}

ooc_status ooc_plan_footprint(int64_t M, int64_t N, int64_t K, double beta, const ooc_plan_t* plan, uint64_t* bytes) {
  if (!plan || !bytes) return fail(OOC_ERR_ARG, "NULL argument");
  if (M <= 0 || N <= 0 || K < 0) return fail(OOC_ERR_ARG, "M and N must be positive, K non-negative");
  Problem pb;
  pb.M = M; pb.N = N; pb.K = K; pb.beta = beta;
  Layout lay;
  ooc_status st = plan_layout(pb, *plan, &lay);
  if (st != OOC_OK) return st;
  *bytes = lay.bytes;
  return OOC_OK;
}

ooc_status ooc_partition(int64_t M, int64_t N, int64_t K, size_t budget_bytes, int64_t* h, int64_t* w) {
  if (!h || !w) return fail(OOC_ERR_ARG, "NULL argument");
  if (M <= 0 || N <= 0 || K < 0) return fail(OOC_ERR_ARG, "M and N must be positive, K non-negative");
  if (!paper_partition(M, N, K, budget_bytes / 8, h, w)) return fail(OOC_ERR_BUDGET, "no split fits the budget");
  return OOC_OK;
}

ooc_status ooc_plan_candidates(int64_t M, int64_t N, int64_t K, double beta, size_t budget_bytes,
                               const ooc_opts* opts, ooc_plan_t* plans, double* model_s, int64_t cap, int64_t* n) {
  if (!n) return fail(OOC_ERR_ARG, "n is NULL");
  if (M <= 0 || N <= 0 || K < 0) return fail(OOC_ERR_ARG, "M and N must be positive, K non-negative");
  Problem pb;
  pb.M = M; pb.N = N; pb.K = K; pb.beta = beta;
  std::vector<ooc_plan_t> ps;
  std::vector<double> ts;
  ooc_status st = plan_candidates(pb, budget_bytes, opts, &ps, &ts);
  if (st != OOC_OK) return st;
  *n = (int64_t)ps.size();
  for (int64_t x = 0; x < (int64_t)ps.size() && x < cap; ++x) {
    if (plans) plans[x] = ps[x];
    if (model_s) model_s[x] = ts[x];
  }
  if ((int64_t)ps.size() > cap) return fail(OOC_ERR_CAPACITY, "more candidates than cap");
  return OOC_OK;
}

ooc_status ooc_plan_predict(int64_t M, int64_t N, int64_t K, double beta, const ooc_plan_t* plan, double* seconds) {
  if (!plan || !seconds) return fail(OOC_ERR_ARG, "NULL argument");
  if (M <= 0 || N <= 0 || K < 0) return fail(OOC_ERR_ARG, "M and N must be positive, K non-negative");
  Problem pb;
  pb.M = M; pb.N = N; pb.K = K; pb.beta = beta;
  Layout lay;
  ooc_status st = plan_layout(pb, *plan, &lay);
  if (st != OOC_OK) return st;
  std::vector<ooc_op> ops;
  st = build_schedule(pb, *plan, lay, &ops);
  if (st != OOC_OK) return st;
  *seconds = simulate(pb, *plan, ops);
  return OOC_OK;
}

ooc_status ooc_plan_simulate(int64_t M, int64_t N, int64_t K, double beta, const ooc_plan_t* plan, double* times,
                             int64_t cap, int64_t* nops) {
  if (!plan || !nops) return fail(OOC_ERR_ARG, "NULL argument");
  if (M <= 0 || N <= 0 || K < 0) return fail(OOC_ERR_ARG, "M and N must be positive, K non-negative");
  Problem pb;
  pb.M = M; pb.N = N; pb.K = K; pb.beta = beta;
  Layout lay;
  ooc_status st = plan_layout(pb, *plan, &lay);
  if (st != OOC_OK) return st;
  std::vector<ooc_op> ops;
  st = build_schedule(pb, *plan, lay, &ops);
  if (st != OOC_OK) return st;
  std::vector<double> tv;
  simulate(pb, *plan, ops, &tv);
  *nops = (int64_t)ops.size();
  if (times)
    for (int64_t x = 0; x < 2 * (int64_t)ops.size() && x < 2 * cap; ++x) times[x] = tv[x];
  if ((int64_t)ops.size() > cap) return fail(OOC_ERR_CAPACITY, "more ops than cap");
  return OOC_OK;
}

ooc_status ooc_schedule(int64_t M, int64_t N, int64_t K, double alpha, double beta, const ooc_plan_t* plan,
                        ooc_op* ops, int64_t cap, int64_t* nops, uint64_t* arena_bytes) {
  return ooc_schedule_ex(0, 0, M, N, K, alpha, beta, plan, ops, cap, nops, arena_bytes);
}

ooc_status ooc_schedule_ex(int32_t transb, int32_t lower, int64_t M, int64_t N, int64_t K, double alpha,
                           double beta, const ooc_plan_t* plan, ooc_op* ops, int64_t cap, int64_t* nops,
                           uint64_t* arena_bytes) {
  if (!plan || !nops) return fail(OOC_ERR_ARG, "NULL argument");
  if (M < 0 || N < 0 || K < 0) return fail(OOC_ERR_ARG, "negative size");
  Problem pb;
  pb.M = M; pb.N = N; pb.K = K; pb.alpha = alpha; pb.beta = beta;
  pb.transb = transb != 0;
  pb.lower = lower != 0;
  Layout lay;
  ooc_status st = OOC_OK;
  if (M > 0 && N > 0) {
    st = plan_layout(pb, *plan, &lay);
    if (st != OOC_OK) return st;
  }
  std::vector<ooc_op> v;
  st = build_schedule(pb, *plan, lay, &v);
  if (st != OOC_OK) return st;
  *nops = (int64_t)v.size();
  if (arena_bytes) *arena_bytes = lay.bytes;
  for (int64_t x = 0; x < (int64_t)v.size() && x < cap; ++x)
    if (ops) ops[x] = v[x];
  if ((int64_t)v.size() > cap) return fail(OOC_ERR_CAPACITY, "more ops than cap");
  return OOC_OK;
}

ooc_status ooc_host_alloc(void** ptr, size_t bytes) {
  if (!ptr) return fail(OOC_ERR_ARG, "ptr is NULL");
  *ptr = nullptr;
  if (bytes == 0) return OOC_OK;
  hipError_t e = hipHostMalloc(ptr, bytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return hip_fail(e, "hipHostMalloc");
  }
  return OOC_OK;
}

ooc_status ooc_host_free(void* ptr) {
  if (!ptr) return OOC_OK;
  HIPCHK(hipHostFree(ptr), "hipHostFree");
  return OOC_OK;
}

ooc_status ooc_device_alloc(int32_t device, void** ptr, size_t bytes) {
  if (!ptr) return fail(OOC_ERR_ARG, "ptr is NULL");
  ooc_status st = ensure_device(device);
  if (st != OOC_OK) return st;
  *ptr = nullptr;
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return fail(OOC_ERR_DEVICE_MEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  return OOC_OK;
}

ooc_status ooc_device_free(int32_t device, void* ptr) {
  if (!ptr) return OOC_OK;
  ooc_status st = ensure_device(device);
  if (st != OOC_OK) return st;
  HIPCHK(hipFree(ptr), "hipFree");
  return OOC_OK;
}

ooc_status ooc_copy_to_device(int32_t device, void* dst, const void* src, size_t bytes) {
  ooc_status st = ensure_device(device);
  if (st != OOC_OK) return st;
  HIPCHK(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice), "hipMemcpy H2D");
  return OOC_OK;
}

ooc_status ooc_copy_to_host(int32_t device, void* dst, const void* src, size_t bytes) {
  ooc_status st = ensure_device(device);
  if (st != OOC_OK) return st;
  HIPCHK(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost), "hipMemcpy D2H");
  return OOC_OK;
}

ooc_status ooc_accum_resident_rows(int64_t M, int64_t N, size_t budget_bytes, int64_t* rows) {
  if (!rows) return fail(OOC_ERR_ARG, "rows is NULL");
  if (M < 0 || N < 0) return fail(OOC_ERR_ARG, "negative matrix size");
  *rows = accum_resident_rows(M, N, budget_bytes);
  return OOC_OK;
}

ooc_status ooc_accum_schedule(int64_t M, int64_t N, int64_t K, double alpha, double beta_eff, size_t budget_bytes,
                              const ooc_opts* opts, int32_t part, ooc_op* ops, int64_t cap, int64_t* nops,
                              uint64_t* arena_bytes) {
  if (!nops) return fail(OOC_ERR_ARG, "nops is NULL");
  if (M < 0 || N < 0 || K < 0) return fail(OOC_ERR_ARG, "negative size");
  if (part != 0 && part != 1) return fail(OOC_ERR_ARG, "part must be 0 or 1");
  Problem pb;
  ooc_plan_t plan{};
  Layout lay;
  std::vector<ooc_op> v;
  ooc_status st = accum_part(part, M, N, K, alpha, beta_eff, accum_resident_rows(M, N, budget_bytes), budget_bytes,
                             opts, &pb, &plan, &lay, &v, nullptr);
  if (st != OOC_OK) return st;
  *nops = (int64_t)v.size();
  if (arena_bytes) *arena_bytes = v.empty() ? 0 : lay.bytes;
  for (int64_t x = 0; x < (int64_t)v.size() && x < cap; ++x)
    if (ops) ops[x] = v[x];
  if ((int64_t)v.size() > cap) return fail(OOC_ERR_CAPACITY, "more ops than cap");
  return OOC_OK;
}

ooc_status ooc_accum_begin(int64_t M, int64_t N, double beta, double* C, int64_t ldc, size_t budget_bytes,
                           const ooc_opts* opts, ooc_accum* out) {
  if (!out) return fail(OOC_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (M < 0 || N < 0) return fail(OOC_ERR_ARG, "negative matrix size");
  if (M > 0 && N > 0 && (!C || ldc < N)) return fail(OOC_ERR_ARG, "bad C or ldc");
  const int dev = opts ? opts->device : 0;
  ooc_status st = ensure_device(dev);
  if (st != OOC_OK) return st;
  if (!range_pinned(C, M, N, ldc)) return fail(OOC_ERR_NOT_PINNED, "C is not page-locked host memory (use ooc_host_alloc)");
  ooc_accum_s* a = new ooc_accum_s();
  a->dev = dev;
  a->M = M; a->N = N; a->beta = beta; a->C = C; a->ldc = ldc; a->budget = budget_bytes;
  if (opts) a->opts = *opts;
  a->opts.timeline = nullptr;
  a->opts.timeline_cap = 0;
  a->opts.arena = nullptr;
  a->opts.arena_bytes = 0;
  a->R = accum_resident_rows(M, N, budget_bytes);
  DevCtx& c = g_dev[dev];
  std::lock_guard<std::mutex> lock(c.mu);
  st = ensure_streams(c);
  if (st == OOC_OK && M > 0 && N > 0) {
    size_t fr = 0, tot = 0;
    hipError_t e = hipMemGetInfo(&fr, &tot);
    if (e != hipSuccess) st = hip_fail(e, "hipMemGetInfo");
    else if (budget_bytes > fr)
      st = fail(OOC_ERR_DEVICE_MEM, "session budget " + std::to_string(budget_bytes) + " bytes, device has " +
                                        std::to_string(fr) + " free");
    else if ((e = hipMalloc(&a->mem, budget_bytes)) != hipSuccess) {
      (void)hipGetLastError();
      a->mem = nullptr;
      st = fail(OOC_ERR_DEVICE_MEM, std::string("hipMalloc of the session arena: ") + hipGetErrorString(e));
    }
  }
  // the resident rows start as C_in (only read when beta != 0)
  if (st == OOC_OK && a->R > 0 && beta != 0.0) {
    hipError_t e = hipMemcpy2DAsync(a->mem, (size_t)N * 8, C, (size_t)ldc * 8, (size_t)N * 8, (size_t)a->R,
                                    hipMemcpyHostToDevice, c.st[0]);
    const hipError_t es = hipStreamSynchronize(c.st[0]);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) st = hip_fail(e, "loading the resident rows of C");
  }
  if (st != OOC_OK) {
    if (a->mem) (void)hipFree(a->mem);
    delete a;
    return st;
  }
  *out = a;
  return OOC_OK;
}

ooc_status ooc_accum_step(ooc_accum acc, int64_t K, double alpha, const double* A, int64_t lda, const double* B,
                          int64_t ldb, ooc_stats* stats) {
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (!acc) return fail(OOC_ERR_ARG, "session is NULL");
  if (K < 0) return fail(OOC_ERR_ARG, "negative K");
  ooc_status st = check_args(acc->M, acc->N, K, alpha, A, lda, B, ldb, 1.0, acc->C, acc->ldc);
  if (st != OOC_OK) return st;
  if (acc->M == 0 || acc->N == 0) {
    ++acc->steps;
    return OOC_OK;
  }
  if (K > 0 && alpha != 0.0 && (!range_pinned(A, acc->M, K, lda) || !range_pinned(B, K, acc->N, ldb)))
    return fail(OOC_ERR_NOT_PINNED, "A or B is not page-locked host memory (use ooc_host_alloc)");
  st = ensure_device(acc->dev);
  if (st != OOC_OK) return st;
  DevCtx& c = g_dev[acc->dev];
  std::lock_guard<std::mutex> lock(c.mu);
  return accum_step_locked(c, acc, K, alpha, A, lda, B, ldb, stats);
}

ooc_status ooc_accum_end(ooc_accum acc, ooc_stats* stats) {
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (!acc) return fail(OOC_ERR_ARG, "session is NULL");
  ooc_status st = OOC_OK;
  if (acc->M > 0 && acc->N > 0) {
    st = ensure_device(acc->dev);
    if (st == OOC_OK) {
      DevCtx& c = g_dev[acc->dev];
      std::lock_guard<std::mutex> lock(c.mu);
      // no step: the result is beta*C (a step with K = 0 reads neither A nor B)
      if (acc->steps == 0) st = accum_step_locked(c, acc, 0, 0.0, nullptr, 1, nullptr, 1, stats);
      if (st == OOC_OK && acc->R > 0) {
        hipError_t e = hipMemcpy2DAsync(acc->C, (size_t)acc->ldc * 8, acc->mem, (size_t)acc->N * 8,
                                        (size_t)acc->N * 8, (size_t)acc->R, hipMemcpyDeviceToHost, c.st[2]);
        const hipError_t es = hipStreamSynchronize(c.st[2]);
        if (e == hipSuccess) e = es;
        if (e != hipSuccess) st = hip_fail(e, "writing the resident rows of C back");
        else if (stats) stats->bytes_d2h += (uint64_t)acc->R * acc->N * 8;
      }
      if (acc->mem) {
        const hipError_t e = hipFree(acc->mem);
        if (e != hipSuccess && st == OOC_OK) st = hip_fail(e, "hipFree of the session arena");
      }
    }
  }
  delete acc;
  return st;
}

ooc_status ooc_release(int32_t device) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) {
    (void)hipGetLastError();
    return OOC_OK;
  }
  for (int d = 0; d < count && d < kMaxDevices; ++d) {
    if (device >= 0 && d != device) continue;
    DevCtx& c = g_dev[d];
    std::lock_guard<std::mutex> lock(c.mu);
    if (!c.init) continue;
    HIPCHK(hipSetDevice(d), "hipSetDevice");
    for (int s = 0; s < 3; ++s) HIPCHK(hipStreamSynchronize(c.st[s]), "hipStreamSynchronize");
    if (c.arena) HIPCHK(hipFree(c.arena), "hipFree");
    c.arena = nullptr;
    c.arena_bytes = 0;
    for (hipEvent_t e : c.ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : c.tev) (void)hipEventDestroy(e);
    for (hipEvent_t e : c.kev) (void)hipEventDestroy(e);
    c.ev.clear();
    c.tev.clear();
    c.kev.clear();
    for (int s = 0; s < 3; ++s) (void)hipStreamDestroy(c.st[s]);
    c.init = false;
  }
  return OOC_OK;
}

ooc_status ooc_dgemm_device(int32_t device, int64_t m, int64_t n, int64_t k, double alpha, const double* A,
                            int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                            int32_t reps, double* ms_out) {
  if (m < 0 || n < 0 || k < 0) return fail(OOC_ERR_ARG, "negative size");
  if (m == 0 || n == 0) return OOC_OK;
  if (!C || ldc < n) return fail(OOC_ERR_ARG, "bad C or ldc");
  if (k > 0 && (!A || !B || lda < k || ldb < n)) return fail(OOC_ERR_ARG, "bad A, B, lda or ldb");
  ooc_status st = ensure_device(device);
  if (st != OOC_OK) return st;
  DevCtx& c = g_dev[device];
  std::lock_guard<std::mutex> lock(c.mu);
  st = ensure_streams(c);
  if (st != OOC_OK) return st;
  hipStream_t s = c.st[1];
  const int r = reps > 0 ? reps : 1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipSuccess;
  if (ms_out) {
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
  }
  for (int x = 0; x < r && e == hipSuccess; ++x)
    e = launch_dgemm_f64(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, 0.0, nullptr, 0, s);
  if (e == hipSuccess && ms_out) e = hipEventRecord(e1, s);
  const hipError_t es = hipStreamSynchronize(s);  // also after a failed launch: nothing outlives the call
  if (e == hipSuccess) e = es;
  if (e == hipSuccess && ms_out) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, e0, e1);
    *ms_out = ms / r;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "dgemm");
  return OOC_OK;
}

static ooc_status split_gemm_device(SliceFormat f, int32_t device, int64_t m, int64_t n, int64_t k, int32_t s,
                                    double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                                    double beta, double* C, int64_t ldc, int32_t reps, double* ms_out) {
  if (m < 0 || n < 0 || k < 0) return fail(OOC_ERR_ARG, "negative size");
  if (s < 1 || s > 8) return fail(OOC_ERR_ARG, "slices must be 1..8");
  if (m == 0 || n == 0) return OOC_OK;
  if (!C || ldc < n) return fail(OOC_ERR_ARG, "bad C or ldc");
  if (k > 0 && (!A || !B || lda < k || ldb < n)) return fail(OOC_ERR_ARG, "bad A, B, lda or ldb");
  ooc_status st = ensure_device(device);
  if (st != OOC_OK) return st;
  DevCtx& c = g_dev[device];
  std::lock_guard<std::mutex> lock(c.mu);
  st = ensure_streams(c);
  if (st != OOC_OK) return st;
  hipStream_t strm = c.st[1];
  const size_t wsb = split_workspace_bytes(m, n, k, s, f);
  void* ws = nullptr;
  HIPCHK(hipMalloc(&ws, wsb), "hipMalloc workspace");
  const int r = reps > 0 ? reps : 1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipSuccess;
  if (ms_out) {
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, strm);
  }
  for (int x = 0; x < r && e == hipSuccess; ++x)
    e = launch_split_gemm(f, m, n, k, s, alpha, A, lda, B, ldb, beta, C, ldc, 0.0, nullptr, 0, ws, wsb, strm);
  if (e == hipSuccess && ms_out) e = hipEventRecord(e1, strm);
  const hipError_t es = hipStreamSynchronize(strm);  // also after a failed launch, before the workspace is freed
  if (e == hipSuccess) e = es;
  if (e == hipSuccess && ms_out) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, e0, e1);
    *ms_out = ms / r;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(ws);
  if (e != hipSuccess) return hip_fail(e, "split gemm");
  return OOC_OK;
}

ooc_status ooc_split_gemm_device(int32_t device, int64_t m, int64_t n, int64_t k, int32_t s, double alpha,
                                 const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                                 int64_t ldc, int32_t reps, double* ms_out) {
  return split_gemm_device(kSliceBF16, device, m, n, k, s, alpha, A, lda, B, ldb, beta, C, ldc, reps, ms_out);
}

ooc_status ooc_split_int8_gemm_device(int32_t device, int64_t m, int64_t n, int64_t k, int32_t s, double alpha,
                                      const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                                      double* C, int64_t ldc, int32_t reps, double* ms_out) {
  return split_gemm_device(kSliceInt8, device, m, n, k, s, alpha, A, lda, B, ldb, beta, C, ldc, reps, ms_out);
}

int32_t ooc_split_int8_wide_tiles(int64_t m, int64_t n, int32_t cus) {
  if (m < 1 || n < 1 || cus < 1) return -1;
  return split_i8_wide(m, n, cus) ? 1 : 0;
}

ooc_status ooc_device_copy(int32_t device, void* dst, const void* src, size_t bytes) {
  if (!dst || !src || bytes % 16 || (reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16)
    return fail(OOC_ERR_ARG, "copy needs 16-byte aligned pointers and a multiple of 16 bytes");
  ooc_status st = ensure_device(device);
  if (st != OOC_OK) return st;
  DevCtx& c = g_dev[device];
  std::lock_guard<std::mutex> lock(c.mu);
  st = ensure_streams(c);
  if (st != OOC_OK) return st;
  const hipError_t e = launch_copy(dst, src, bytes, c.st[1]);
  const hipError_t es = hipStreamSynchronize(c.st[1]);
  if (e != hipSuccess) return hip_fail(e, "copy launch");
  HIPCHK(es, "hipStreamSynchronize");
  return OOC_OK;
}

const char* ooc_last_error(void) { return g_err.c_str(); }

const char* ooc_version(void) { return "ooc-mi355x 0.1 (gfx950)"; }

}  // extern "C"
