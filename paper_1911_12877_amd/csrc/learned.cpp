// Learned schedule choice (host side): schedule features on a given graph,
// the installed cost model, BF16 ranking on the device, and the C-ABI of the
// MLP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "gz_internal.h"

namespace gz {

bool read_pattern_checked(const uint8_t* adj, int32_t k, Pattern* p);
gz_status build_schedule_for(const Pattern& p, int32_t induced, uint32_t flags, const int8_t* order,
                             gz_schedule** out);
gz_status mlp_forward(const float* P, const float* X, int n, int D, int H, bool bf16, float* hpre,
                      float* y, hipStream_t st);
gz_status mlp_loss_grad(const float* P, const float* X, const float* t, int n, int D, int H,
                        float* G, float* hpre, float* y, float* dy, float* loss, hipStream_t st);
gz_status mlp_adam(float* P, const float* G, float* m, float* v, int D, int H, float lr, float b1,
                   float b2, float eps, int step, hipStream_t st);
long long mlp_param_count(int D, int H);

namespace {

std::mutex g_model_mu;
std::vector<float> g_model;
int g_model_h = 0;
float g_model_margin = 0.0f;
int32_t g_model_kmax = 0;
// range of the graph statistics (the last GZ_GRAPH_STATS features) over the
// model's training corpus; graphs outside it keep the analytic pick
bool g_model_ranged = false;
float g_model_gmin[GZ_GRAPH_STATS], g_model_gmax[GZ_GRAPH_STATS];
constexpr float kRangeSlack = 0.05f;  // in the features' scaled-log units

double lg(double x) { return std::log10(std::max(x, 1e-30)); }
float clampf(double x, double lo, double hi) { return (float)std::min(hi, std::max(lo, x)); }

// Features of one schedule (see gz.h for the list).
void schedule_features(const gz_graph* g, const Pattern& p, const std::vector<Perm>& aut,
                       bool induced, const int8_t* order, float* f) {
  std::fill(f, f + GZ_FEATURES, 0.0f);
  int8_t bound[kMaxK];
  reduced_bounds(p, aut, order, bound);
  const Plan plan = lower_plan(p, order, bound, induced);
  const double n = std::max(g->stats[0], 2.0);
  const double pr = std::min(0.5, g->stats[2] / (n - 1.0));
  double prod = n;
  double total = n;
  for (int i = 1; i < p.k && i < 8; ++i) {
    const Level& L = plan.lv[i];
    const int c = __builtin_popcount(L.isect);
    const int d = __builtin_popcount(L.sub);
    const double size = n * std::pow(pr, c) * std::pow(1.0 - pr, d);
    prod *= size;
    int z[kMaxK];
    for (int j = 0; j <= i; ++j) z[j] = 1;
    for (int j = i; j >= 1; --j)
      if (bound[j] >= 0) z[bound[j]] += z[j];
    double rate = 1.0;
    for (int j = 0; j <= i; ++j) rate /= z[j];
    // owners of the loop's lists that are themselves bounded from above:
    // with degree-descending ids they tend to be high-degree vertices
    int own_isect = 0, own_sub = 0;
    for (int j = 0; j < i; ++j) {
      const bool bounded_owner = bound[j] >= 0;
      if (((L.isect >> j) & 1) && bounded_owner) ++own_isect;
      if (((L.sub >> j) & 1) && bounded_owner) ++own_sub;
    }
    int depth = 0;
    for (int x = L.bound; x >= 0; x = bound[x]) ++depth;
    float* q = f + (i - 1) * 14;
    q[0] = 1.0f;
    q[1] = c / 7.0f;
    q[2] = d / 7.0f;
    q[3] = L.bound >= 0 ? 1.0f : 0.0f;
    q[4] = L.bound == i - 1 ? 1.0f : 0.0f;
    q[5] = (L.bound < 0 && L.src < 0) ? 1.0f : 0.0f;
    q[6] = clampf(lg(size) / 10.0, -3.0, 3.0);
    q[7] = clampf(lg(rate) / 3.0, -3.0, 0.0);
    q[8] = i == p.k - 1 ? 1.0f : 0.0f;
    q[9] = L.src >= 0 ? 1.0f : 0.0f;
    q[10] = clampf(lg(prod * rate) / 10.0, -3.0, 3.0);
    q[11] = own_isect / 7.0f;
    q[12] = own_sub / 7.0f;
    q[13] = depth / 7.0f;
    total += prod * rate;
  }
  // whole-schedule costs: this graph's G(n, p) and the paper's G(1000, 5/999)
  f[98] = clampf(lg(total) / 10.0, -3.0, 3.0);
  f[99] = clampf(lg(analytic_cost(p, order, bound, induced)) / 10.0, -3.0, 3.0);
  float* s = f + 100;
  s[0] = (float)(lg(n) / 7.0);
  s[1] = (float)(lg(g->stats[1] + 1) / 9.0);
  s[2] = (float)(lg(g->stats[2] + 1e-3) / 3.0);
  s[3] = (float)(lg(g->stats[3] + 1e-3) / 5.0);
  s[4] = (float)(lg(g->stats[4] + 1) / 6.0);
  s[5] = (float)(lg(g->stats[5] + 1e-3) / 3.0);
  s[6] = (float)(lg(g->stats[6] + 1e-3) / 4.0);
  s[7] = (float)(lg(g->stats[7] + 1) / 4.0);
}

#define GZ_L_HIP(call)                                                    \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess) {                                               \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));     \
      rc = GZ_EDEVICE;                                                    \
      goto done;                                                          \
    }                                                                     \
  } while (0)

// Predicted costs (BF16 inference) of n feature rows with the model P.
gz_status predict(const std::vector<float>& P, int H, const std::vector<float>& X, int n,
                  std::vector<float>* y) {
  gz_status rc = GZ_OK;
  float *dP = nullptr, *dX = nullptr, *dh = nullptr, *dy = nullptr;
  const int D = GZ_FEATURES;
  y->assign(n, 0.0f);
  GZ_L_HIP(hipMalloc(&dP, P.size() * sizeof(float)));
  GZ_L_HIP(hipMalloc(&dX, X.size() * sizeof(float)));
  GZ_L_HIP(hipMalloc(&dh, (size_t)n * H * sizeof(float)));
  GZ_L_HIP(hipMalloc(&dy, (size_t)n * sizeof(float)));
  GZ_L_HIP(hipMemcpy(dP, P.data(), P.size() * sizeof(float), hipMemcpyHostToDevice));
  GZ_L_HIP(hipMemcpy(dX, X.data(), X.size() * sizeof(float), hipMemcpyHostToDevice));
  rc = mlp_forward(dP, dX, n, D, H, true, dh, dy, nullptr);
  if (rc) goto done;
  GZ_L_HIP(hipMemcpy(y->data(), dy, (size_t)n * sizeof(float), hipMemcpyDeviceToHost));
done:
  for (float* q : {dP, dX, dh, dy})
    if (q) (void)hipFree(q);
  return rc;
}

}  // namespace
}  // namespace gz

using namespace gz;

extern "C" {

gz_status gz_schedule_features(const gz_graph* g, const uint8_t* adj, int32_t k, int32_t induced,
                               const int8_t* order, float* out) {
  if (!g || !out || !order) {
    set_error("NULL argument");
    return GZ_EINVAL;
  }
  Pattern p;
  if (!read_pattern_checked(adj, k, &p)) return GZ_EINVAL;
  if (!schedule_valid(p, order)) {
    set_error("order is not a valid schedule");
    return GZ_EINVAL;
  }
  schedule_features(g, p, automorphisms(p), induced != 0, order, out);
  return GZ_OK;
}

gz_status gz_set_cost_model(const float* params, int32_t D, int32_t H, float margin,
                            int32_t k_max, const float* graph_range) {
  std::lock_guard<std::mutex> lock(g_model_mu);
  if (!params) {
    g_model.clear();
    g_model_h = 0;
    g_model_margin = 0.0f;
    g_model_kmax = 0;
    g_model_ranged = false;
    return GZ_OK;
  }
  if (D != GZ_FEATURES || H < 1 || H > 1024 || !(margin >= 0.0f && margin < 100.0f) ||
      k_max < 2 || k_max > kMaxK) {
    set_error("cost model must have D == GZ_FEATURES, 1 <= H <= 1024, 0 <= margin < 100 "
              "and 2 <= k_max <= 8");
    return GZ_EINVAL;
  }
  g_model.assign(params, params + mlp_param_count(D, H));
  g_model_h = H;
  g_model_margin = margin;
  g_model_kmax = k_max;
  g_model_ranged = graph_range != nullptr;
  for (int i = 0; i < GZ_GRAPH_STATS && graph_range; ++i) {
    g_model_gmin[i] = graph_range[i];
    g_model_gmax[i] = graph_range[GZ_GRAPH_STATS + i];
  }
  return GZ_OK;
}

gz_status gz_compile_pattern_graph(const gz_graph* g, const uint8_t* adj, int32_t k, int32_t induced,
                                   uint32_t flags, gz_schedule** out) {
  if (!g || !out) {
    set_error("NULL argument");
    return GZ_EINVAL;
  }
  Pattern p;
  if (!read_pattern_checked(adj, k, &p)) return GZ_EINVAL;
  std::vector<float> model;
  int H = 0;
  float margin = 0.0f;
  int32_t kmax = 0;
  bool ranged = false;
  float gmin[GZ_GRAPH_STATS], gmax[GZ_GRAPH_STATS];
  {
    std::lock_guard<std::mutex> lock(g_model_mu);
    model = g_model;
    H = g_model_h;
    margin = g_model_margin;
    kmax = g_model_kmax;
    ranged = g_model_ranged;
    std::copy(g_model_gmin, g_model_gmin + GZ_GRAPH_STATS, gmin);
    std::copy(g_model_gmax, g_model_gmax + GZ_GRAPH_STATS, gmax);
  }
  const uint32_t rest = flags & ~(uint32_t)GZ_SCHED_LEARNED;
  // no model, or a pattern larger than any in its corpus (features of loops
  // the network never saw): the analytic model's pick
  if (!(flags & GZ_SCHED_LEARNED) || model.empty() || p.k > kmax)
    return build_schedule_for(p, induced, rest, nullptr, out);
  std::vector<Perm> aut = automorphisms(p);
  std::vector<Perm> ds = explore_schedules(p, aut);
  const int n = (int)ds.size();
  std::vector<float> X((size_t)n * GZ_FEATURES);
  for (int i = 0; i < n; ++i)
    schedule_features(g, p, aut, induced != 0, ds[i].data(), X.data() + (size_t)i * GZ_FEATURES);
  // a graph whose statistics lie outside the corpus's range: the network
  // would extrapolate, so the analytic model decides
  if (ranged && n > 0) {
    const float* st = X.data() + GZ_FEATURES - GZ_GRAPH_STATS;
    for (int i = 0; i < GZ_GRAPH_STATS; ++i)
      if (st[i] < gmin[i] - kRangeSlack || st[i] > gmax[i] + kRangeSlack)
        return build_schedule_for(p, induced, rest, nullptr, out);
  }
  std::vector<float> y;
  gz_status rc = predict(model, H, X, n, &y);
  if (rc) return rc;
  int best = 0;
  for (int i = 1; i < n; ++i)
    if (y[i] < y[best] - 1e-6f * std::max(1.0f, std::fabs(y[best]))) best = i;
  // the analytic model's pick stays unless the network predicts the best
  // schedule faster by more than its validation error (log10 time)
  gz_schedule* analytic = nullptr;
  rc = build_schedule_for(p, induced, rest, nullptr, &analytic);
  if (rc) return rc;
  int an = -1;
  for (int i = 0; i < n && an < 0; ++i)
    if (std::equal(ds[i].begin(), ds[i].end(), analytic->order)) an = i;
  if (an >= 0 && y[an] - y[best] <= margin) {
    *out = analytic;
    return GZ_OK;
  }
  gz_free_schedule(analytic);
  return build_schedule_for(p, induced, rest, ds[best].data(), out);
}

gz_status gz_mlp_forward(const float* params, const float* X, int32_t n, int32_t D, int32_t H,
                         int32_t bf16, float* y, void* hip_stream) {
  if (n < 0 || D < 1 || H < 1 || (n > 0 && (!params || !X || !y))) {
    set_error("bad MLP arguments");
    return GZ_EINVAL;
  }
  if (n == 0) return GZ_OK;
  float* dh = nullptr;
  if (hipMalloc(&dh, (size_t)n * H * sizeof(float)) != hipSuccess) {
    set_error("device allocation failed");
    return GZ_ENOMEM;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  gz_status rc = mlp_forward(params, X, n, D, H, bf16 != 0, dh, y, st);
  if (!rc && hipStreamSynchronize(st) != hipSuccess) {
    set_error("MLP forward failed");
    rc = GZ_EDEVICE;
  }
  (void)hipFree(dh);
  return rc;
}

gz_status gz_mlp_loss_grad(const float* params, const float* X, const float* t, int32_t n,
                           int32_t D, int32_t H, float* grad, float* loss_host, void* hip_stream) {
  if (n < 1 || D < 1 || H < 1 || !params || !X || !t || !grad || !loss_host) {
    set_error("bad MLP arguments");
    return GZ_EINVAL;
  }
  float* scratch = nullptr;
  const size_t need = (size_t)n * H + 2 * (size_t)n + 1;
  if (hipMalloc(&scratch, need * sizeof(float)) != hipSuccess) {
    set_error("device allocation failed");
    return GZ_ENOMEM;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  float* hpre = scratch;
  float* y = hpre + (size_t)n * H;
  float* dy = y + n;
  float* loss = dy + n;
  gz_status rc = mlp_loss_grad(params, X, t, n, D, H, grad, hpre, y, dy, loss, st);
  if (!rc && (hipMemcpyAsync(loss_host, loss, sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess ||
              hipStreamSynchronize(st) != hipSuccess)) {
    set_error("MLP gradient failed");
    rc = GZ_EDEVICE;
  }
  (void)hipFree(scratch);
  return rc;
}

gz_status gz_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t D, int32_t H,
                      float lr, float beta1, float beta2, float eps, int32_t step, void* hip_stream) {
  if (D < 1 || H < 1 || step < 1 || !params || !grad || !m || !v) {
    set_error("bad Adam arguments");
    return GZ_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  gz_status rc = mlp_adam(params, grad, m, v, D, H, lr, beta1, beta2, eps, step, st);
  if (!rc && hipStreamSynchronize(st) != hipSuccess) {
    set_error("Adam step failed");
    rc = GZ_EDEVICE;
  }
  return rc;
}

}  // extern "C"
