// The learned planner: features of a candidate plan, training on measured
// timings with the library's own GPU kernels, prediction for plan choice.
//
// A candidate's features are the problem size and budget, the plan's shape
// (block and panel sizes, order, buffer and stream counts, precision) and the
// analytic cost model's prediction, all on log scales where they span
// decades.  The network predicts the log of the measured run time; features
// and targets are standardised with the training set's mean and deviation,
// which are stored with the weights.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

extern "C" ooc_status ooc_mlp_load(const char* path);

namespace ooc {
namespace {

struct Net {
  bool loaded = false;
  int d = 0, H = 0;
  std::vector<float> params, fmean, fstd;
  float ymean = 0.f, ystd = 1.f;
};

std::mutex g_net_mu;
Net g_net;

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes > 0 ? bytes : 4); }
  float* f() { return static_cast<float*>(p); }
};

#define MLPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return fail(OOC_ERR_HIP, std::string("mlp: ") + hipGetErrorString(e_)); \
  } while (0)

ooc_status select_device(int device) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    return fail(OOC_ERR_NO_DEVICE, "no HIP device available");
  }
  if (device < 0 || device >= count) return fail(OOC_ERR_NO_DEVICE, "device ordinal out of range");
  MLPCHK(hipSetDevice(device));
  return OOC_OK;
}

// Full-batch Adam on the GPU; params are updated in place (host array).
ooc_status train_impl(int device, int d, int H, float* params, const float* X, const float* t, int64_t n, int epochs,
                      float lr, float wd, float* loss_hist) {
  ooc_status st = select_device(device);
  if (st != OOC_OK) return st;
  const int64_t np = mlp_param_count(d, H);
  DevBuf dP, dG, dM, dV, dX, dT, dS, dL;
  MLPCHK(dP.alloc(np * 4));
  MLPCHK(dG.alloc(np * 4));
  MLPCHK(dM.alloc(np * 4));
  MLPCHK(dV.alloc(np * 4));
  MLPCHK(dX.alloc((size_t)n * d * 4));
  MLPCHK(dT.alloc((size_t)n * 4));
  MLPCHK(dS.alloc((size_t)mlp_scratch_floats(n, d, H) * 4));
  MLPCHK(dL.alloc((size_t)(epochs > 0 ? epochs : 1) * 4));
  MLPCHK(hipMemcpy(dP.p, params, np * 4, hipMemcpyHostToDevice));
  MLPCHK(hipMemcpy(dX.p, X, (size_t)n * d * 4, hipMemcpyHostToDevice));
  MLPCHK(hipMemcpy(dT.p, t, (size_t)n * 4, hipMemcpyHostToDevice));
  std::vector<float> zeros(np, 0.f);
  MLPCHK(hipMemcpy(dM.p, zeros.data(), np * 4, hipMemcpyHostToDevice));
  MLPCHK(hipMemcpy(dV.p, zeros.data(), np * 4, hipMemcpyHostToDevice));
  for (int ep = 0; ep < epochs; ++ep) {
    MLPCHK(launch_mlp_grad(n, d, H, dP.f(), dX.f(), dT.f(), wd, dS.f(), dG.f(), dL.f() + ep, nullptr));
    MLPCHK(launch_adam(np, dP.f(), dG.f(), dM.f(), dV.f(), lr, 0.9f, 0.999f, 1e-8f, ep + 1, nullptr));
  }
  MLPCHK(hipDeviceSynchronize());
  MLPCHK(hipMemcpy(params, dP.p, np * 4, hipMemcpyDeviceToHost));
  if (loss_hist && epochs > 0) MLPCHK(hipMemcpy(loss_hist, dL.p, (size_t)epochs * 4, hipMemcpyDeviceToHost));
  return OOC_OK;
}

ooc_status forward_impl(int device, int d, int H, const float* params, const float* X, int64_t n, float* y) {
  ooc_status st = select_device(device);
  if (st != OOC_OK) return st;
  const int64_t np = mlp_param_count(d, H);
  DevBuf dP, dX, dS, dY;
  MLPCHK(dP.alloc(np * 4));
  MLPCHK(dX.alloc((size_t)n * d * 4));
  MLPCHK(dS.alloc((size_t)mlp_scratch_floats(n, d, H) * 4));
  MLPCHK(dY.alloc((size_t)n * 4));
  MLPCHK(hipMemcpy(dP.p, params, np * 4, hipMemcpyHostToDevice));
  MLPCHK(hipMemcpy(dX.p, X, (size_t)n * d * 4, hipMemcpyHostToDevice));
  MLPCHK(launch_mlp_forward(n, d, H, dP.f(), dX.f(), dS.f(), dY.f(), nullptr));
  MLPCHK(hipDeviceSynchronize());
  MLPCHK(hipMemcpy(y, dY.p, (size_t)n * 4, hipMemcpyDeviceToHost));
  return OOC_OK;
}

double log2p(double x) { return std::log2(x > 1e-300 ? x : 1e-300); }

}  // namespace

// Features of one candidate plan (OOC_MLP_FEATURES values).
void plan_features(const Problem& pb, uint64_t budget, const ooc_plan_t& p, double model_s, double h2d_bytes,
                   float* f) {
  int x = 0;
  f[x++] = (float)log2p((double)pb.M);
  f[x++] = (float)log2p((double)pb.N);
  f[x++] = (float)log2p((double)pb.K + 1);
  f[x++] = (float)log2p((double)budget);
  f[x++] = (float)log2p((double)std::min<int64_t>(p.mb, pb.M));
  f[x++] = (float)log2p((double)std::min<int64_t>(p.nb, pb.N));
  f[x++] = (float)log2p((double)std::min<int64_t>(p.kb, pb.K) + 1);
  // the backwards-alternating orders share their base order's indicator (the
  // cost model's prediction, also a feature, tells them apart)
  const int base = p.order == OOC_ORDER_COLS_PS ? OOC_ORDER_COLS_P : (p.order == OOC_ORDER_ROWS_PS ? OOC_ORDER_ROWS_P : p.order);
  for (int o = 0; o < 4; ++o) f[x++] = base == o ? 1.f : 0.f;
  f[x++] = (float)p.nbuf_a;
  f[x++] = (float)p.nbuf_b;
  f[x++] = (float)log2p((double)p.nbuf_c);
  f[x++] = (float)p.nbuf_d;
  f[x++] = (float)p.nstreams;
  f[x++] = (float)log2p(model_s);
  f[x++] = (float)log2p(h2d_bytes + 1);
  f[x++] = (float)(p.precision != OOC_FP64 ? p.slices : 0);
}

ooc_status features_for(const Problem& pb, uint64_t budget, const ooc_plan_t* plans, int64_t n, float* X) {
  for (int64_t c = 0; c < n; ++c) {
    Layout lay;
    ooc_status st = plan_layout(pb, plans[c], &lay);
    if (st != OOC_OK) return st;
    std::vector<ooc_op> ops;
    st = build_schedule(pb, plans[c], lay, &ops);
    if (st != OOC_OK) return st;
    double h2d = 0;
    for (const ooc_op& o : ops)
      if (o.kind == OOC_OP_H2D) h2d += (double)o.rows * o.cols * 8.0;
    plan_features(pb, budget, plans[c], simulate(pb, plans[c], ops), h2d, X + c * OOC_MLP_FEATURES);
  }
  return OOC_OK;
}

// The planner network shipped next to the library (planner_mlp.txt in the
// directory holding libooc.so), loaded on first use when no other is loaded.
static void load_default_network() {
  static bool tried = false;
  {
    std::lock_guard<std::mutex> lock(g_net_mu);
    if (g_net.loaded || tried) return;
    tried = true;
  }
  Dl_info info;
  if (!dladdr(reinterpret_cast<void*>(&load_default_network), &info) || !info.dli_fname) return;
  std::string path(info.dli_fname);
  const size_t slash = path.rfind('/');
  path = (slash == std::string::npos ? std::string(".") : path.substr(0, slash)) + "/planner_mlp.txt";
  if (FILE* f = std::fopen(path.c_str(), "r")) {
    std::fclose(f);
    (void)ooc_mlp_load(path.c_str());
  }
}

bool mlp_predict(const Problem& pb, uint64_t budget_bytes, const std::vector<ooc_plan_t>& plans,
                 std::vector<double>* seconds) {
  load_default_network();
  Net net;
  {
    std::lock_guard<std::mutex> lock(g_net_mu);
    if (!g_net.loaded) return false;
    net = g_net;
  }
  // A network whose training set held FP64 plans only saw a constant slice
  // count (stored as mean 0, deviation 1): it does not rank split plans.
  constexpr int kSliceFeature = OOC_MLP_FEATURES - 1;
  const bool knows_split = net.fmean[kSliceFeature] != 0.f || net.fstd[kSliceFeature] != 1.f;
  // Nor was it trained on INT8 slice timings, which run at twice the BF16 rate
  // per product: it declines those plans too.
  for (const ooc_plan_t& p : plans)
    if ((p.precision == OOC_SPLIT_BF16 && !knows_split) || p.precision == OOC_SPLIT_INT8) return false;
  const int64_t n = (int64_t)plans.size();
  std::vector<float> X((size_t)n * OOC_MLP_FEATURES), y(n);
  if (features_for(pb, budget_bytes, plans.data(), n, X.data()) != OOC_OK) return false;
  for (int64_t c = 0; c < n; ++c)
    for (int j = 0; j < net.d; ++j) X[c * net.d + j] = (X[c * net.d + j] - net.fmean[j]) / net.fstd[j];
  // M, N, K and the budget (the first four features, the same for every
  // candidate) more than kMaxZ deviations from the training problems' mean:
  // the prediction would be an extrapolation, so the network declines
  constexpr float kMaxZ = 4.f;
  if (n > 0)
    for (int j = 0; j < 4; ++j)
      if (std::fabs(X[j]) > kMaxZ) return false;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  if (forward_impl(dev, net.d, net.H, net.params.data(), X.data(), n, y.data()) != OOC_OK) return false;
  seconds->resize(n);
  for (int64_t c = 0; c < n; ++c) (*seconds)[c] = std::exp((double)(y[c] * net.ystd + net.ymean));
  return true;
}

}  // namespace ooc

using namespace ooc;

extern "C" {

ooc_status ooc_mlp_features(int64_t M, int64_t N, int64_t K, double beta, size_t budget_bytes,
                            const ooc_plan_t* plans, int64_t n, float* X_out) {
  if (!plans || !X_out || n < 0) return fail(OOC_ERR_ARG, "NULL argument");
  if (M <= 0 || N <= 0 || K < 0) return fail(OOC_ERR_ARG, "M and N must be positive, K non-negative");
  Problem pb;
  pb.M = M; pb.N = N; pb.K = K; pb.beta = beta;
  return features_for(pb, budget_bytes, plans, n, X_out);
}

ooc_status ooc_mlp_forward(int32_t device, int32_t d, int32_t hidden, const float* params, const float* X, int64_t n,
                           float* y_out) {
  if (!params || !X || !y_out || d <= 0 || hidden <= 0 || n <= 0) return fail(OOC_ERR_ARG, "bad argument");
  return forward_impl(device, d, hidden, params, X, n, y_out);
}

ooc_status ooc_mlp_grad(int32_t device, int32_t d, int32_t hidden, const float* params, const float* X,
                        const float* t, int64_t n, float weight_decay, float* grad_out, float* loss_out) {
  if (!params || !X || !t || !grad_out || d <= 0 || hidden <= 0 || n <= 0 || !(weight_decay >= 0.f))
    return fail(OOC_ERR_ARG, "bad argument");
  ooc_status st = select_device(device);
  if (st != OOC_OK) return st;
  const int64_t np = mlp_param_count(d, hidden);
  DevBuf dP, dG, dX, dT, dS, dL;
  MLPCHK(dP.alloc(np * 4));
  MLPCHK(dG.alloc(np * 4));
  MLPCHK(dX.alloc((size_t)n * d * 4));
  MLPCHK(dT.alloc((size_t)n * 4));
  MLPCHK(dS.alloc((size_t)mlp_scratch_floats(n, d, hidden) * 4));
  MLPCHK(dL.alloc(4));
  MLPCHK(hipMemcpy(dP.p, params, np * 4, hipMemcpyHostToDevice));
  MLPCHK(hipMemcpy(dX.p, X, (size_t)n * d * 4, hipMemcpyHostToDevice));
  MLPCHK(hipMemcpy(dT.p, t, (size_t)n * 4, hipMemcpyHostToDevice));
  MLPCHK(launch_mlp_grad(n, d, hidden, dP.f(), dX.f(), dT.f(), weight_decay, dS.f(), dG.f(), dL.f(), nullptr));
  MLPCHK(hipDeviceSynchronize());
  MLPCHK(hipMemcpy(grad_out, dG.p, np * 4, hipMemcpyDeviceToHost));
  if (loss_out) MLPCHK(hipMemcpy(loss_out, dL.p, 4, hipMemcpyDeviceToHost));
  return OOC_OK;
}

ooc_status ooc_mlp_adam(int32_t device, int64_t count, float* params, const float* grad, float* m, float* v,
                        int32_t step, float lr, float beta1, float beta2, float eps) {
  if (!params || !grad || !m || !v || count <= 0 || step < 1) return fail(OOC_ERR_ARG, "bad argument");
  ooc_status st = select_device(device);
  if (st != OOC_OK) return st;
  DevBuf dP, dG, dM, dV;
  MLPCHK(dP.alloc(count * 4));
  MLPCHK(dG.alloc(count * 4));
  MLPCHK(dM.alloc(count * 4));
  MLPCHK(dV.alloc(count * 4));
  MLPCHK(hipMemcpy(dP.p, params, count * 4, hipMemcpyHostToDevice));
  MLPCHK(hipMemcpy(dG.p, grad, count * 4, hipMemcpyHostToDevice));
  MLPCHK(hipMemcpy(dM.p, m, count * 4, hipMemcpyHostToDevice));
  MLPCHK(hipMemcpy(dV.p, v, count * 4, hipMemcpyHostToDevice));
  MLPCHK(launch_adam(count, dP.f(), dG.f(), dM.f(), dV.f(), lr, beta1, beta2, eps, step, nullptr));
  MLPCHK(hipDeviceSynchronize());
  MLPCHK(hipMemcpy(params, dP.p, count * 4, hipMemcpyDeviceToHost));
  MLPCHK(hipMemcpy(m, dM.p, count * 4, hipMemcpyDeviceToHost));
  MLPCHK(hipMemcpy(v, dV.p, count * 4, hipMemcpyDeviceToHost));
  return OOC_OK;
}

ooc_status ooc_mlp_train(int32_t device, int32_t d, int32_t hidden, float* params, const float* X, const float* t,
                         int64_t n, int32_t epochs, float lr, float weight_decay, float* loss_hist) {
  if (!params || !X || !t || d <= 0 || hidden <= 0 || n <= 0 || epochs < 0 || !(weight_decay >= 0.f))
    return fail(OOC_ERR_ARG, "bad argument");
  return train_impl(device, d, hidden, params, X, t, n, epochs, lr, weight_decay, loss_hist);
}

ooc_status ooc_mlp_fit(int32_t device, const float* X, const float* y_seconds, int64_t n, int32_t hidden,
                       int32_t epochs, float lr, float weight_decay, uint64_t seed, float* loss_hist) {
  const int d = OOC_MLP_FEATURES;
  if (!X || !y_seconds || n <= 1 || hidden <= 0 || epochs < 0 || !(weight_decay >= 0.f))
    return fail(OOC_ERR_ARG, "bad argument");
  Net net;
  net.d = d;
  net.H = hidden;
  net.fmean.assign(d, 0.f);
  net.fstd.assign(d, 1.f);
  for (int j = 0; j < d; ++j) {
    double s = 0, s2 = 0;
    for (int64_t r = 0; r < n; ++r) {
      const double v = X[r * d + j];
      s += v;
      s2 += v * v;
    }
    const double mean = s / n, var = s2 / n - mean * mean;
    net.fmean[j] = (float)mean;
    net.fstd[j] = var > 1e-12 ? (float)std::sqrt(var) : 1.f;  // constant features pass through centred
  }
  std::vector<float> Xs((size_t)n * d), t(n);
  double s = 0, s2 = 0;
  for (int64_t r = 0; r < n; ++r) {
    if (!(y_seconds[r] > 0)) return fail(OOC_ERR_ARG, "timings must be positive");
    const double ly = std::log((double)y_seconds[r]);
    s += ly;
    s2 += ly * ly;
  }
  const double ym = s / n, yv = s2 / n - ym * ym;
  net.ymean = (float)ym;
  net.ystd = yv > 1e-12 ? (float)std::sqrt(yv) : 1.f;
  for (int64_t r = 0; r < n; ++r) {
    for (int j = 0; j < d; ++j) Xs[r * d + j] = (X[r * d + j] - net.fmean[j]) / net.fstd[j];
    t[r] = (float)((std::log((double)y_seconds[r]) - ym) / net.ystd);
  }
  // weights ~ normal(0, 1/fan_in), biases zero
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  net.params.assign(mlp_param_count(d, hidden), 0.f);
  float* W1 = net.params.data();
  float* W2 = W1 + (size_t)d * hidden + hidden;
  float* W3 = W2 + (size_t)hidden * hidden + hidden;
  for (int64_t i = 0; i < (int64_t)d * hidden; ++i) W1[i] = (float)(nd(rng) / std::sqrt((double)d));
  for (int64_t i = 0; i < (int64_t)hidden * hidden; ++i) W2[i] = (float)(nd(rng) / std::sqrt((double)hidden));
  for (int64_t i = 0; i < hidden; ++i) W3[i] = (float)(nd(rng) / std::sqrt((double)hidden));
  ooc_status st =
      train_impl(device, d, hidden, net.params.data(), Xs.data(), t.data(), n, epochs, lr, weight_decay, loss_hist);
  if (st != OOC_OK) return st;
  net.loaded = true;
  {
    std::lock_guard<std::mutex> lock(g_net_mu);
    g_net = net;
  }
  clear_plan_cache();
  return OOC_OK;
}

ooc_status ooc_mlp_save(const char* path) {
  if (!path) return fail(OOC_ERR_ARG, "path is NULL");
  Net net;
  {
    std::lock_guard<std::mutex> lock(g_net_mu);
    if (!g_net.loaded) return fail(OOC_ERR_ARG, "no planner network loaded");
    net = g_net;
  }
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(OOC_ERR_ARG, std::string("cannot write ") + path);
  std::fprintf(f, "ooc-mlp-planner 1\n%d %d\n%.9g %.9g\n", net.d, net.H, net.ymean, net.ystd);
  for (int j = 0; j < net.d; ++j) std::fprintf(f, "%.9g %.9g\n", net.fmean[j], net.fstd[j]);
  for (float p : net.params) std::fprintf(f, "%.9g\n", p);
  std::fclose(f);
  return OOC_OK;
}

ooc_status ooc_mlp_load(const char* path) {
  if (!path) return fail(OOC_ERR_ARG, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(OOC_ERR_ARG, std::string("cannot read ") + path);
  Net net;
  int version = 0;
  bool ok = std::fscanf(f, "ooc-mlp-planner %d %d %d %f %f", &version, &net.d, &net.H, &net.ymean, &net.ystd) == 5;
  ok = ok && version == 1 && net.d == OOC_MLP_FEATURES && net.H > 0 && net.H <= 4096;
  if (ok) {
    net.fmean.resize(net.d);
    net.fstd.resize(net.d);
    for (int j = 0; j < net.d && ok; ++j) ok = std::fscanf(f, "%f %f", &net.fmean[j], &net.fstd[j]) == 2;
    net.params.resize(mlp_param_count(net.d, net.H));
    for (size_t i = 0; i < net.params.size() && ok; ++i) ok = std::fscanf(f, "%f", &net.params[i]) == 1;
  }
  std::fclose(f);
  if (!ok) return fail(OOC_ERR_ARG, std::string("malformed planner network file ") + path);
  net.loaded = true;
  {
    std::lock_guard<std::mutex> lock(g_net_mu);
    g_net = net;
  }
  clear_plan_cache();
  return OOC_OK;
}

int32_t ooc_mlp_loaded(void) {
  std::lock_guard<std::mutex> lock(g_net_mu);
  return g_net.loaded ? 1 : 0;
}

ooc_status ooc_mlp_predict(int64_t M, int64_t N, int64_t K, double beta, size_t budget_bytes, const ooc_plan_t* plans,
                           int64_t n, double* seconds_out) {
  if (!plans || !seconds_out || n <= 0) return fail(OOC_ERR_ARG, "bad argument");
  if (M <= 0 || N <= 0 || K < 0) return fail(OOC_ERR_ARG, "M and N must be positive, K non-negative");
  Problem pb;
  pb.M = M; pb.N = N; pb.K = K; pb.beta = beta;
  std::vector<ooc_plan_t> v(plans, plans + n);
  std::vector<double> s;
  if (!mlp_predict(pb, budget_bytes, v, &s)) return fail(OOC_ERR_ARG, "no planner network loaded (or inference failed)");
  for (int64_t c = 0; c < n; ++c) seconds_out[c] = s[c];
  return OOC_OK;
}

}  // extern "C"
