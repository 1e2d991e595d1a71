// Host runtime around the kernels: the cadence graph (re-plan + fused pass
// captured once in a HIP graph and replayed per cadence) and the tile-size
// autotuner.
#include <cstdio>
#include <map>
#include <new>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.h"

struct rts_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  rts_plan_t plan = nullptr;
};

using namespace rts;

namespace {

#define RTS_HIP_R(expr)                                                         \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      set_error("%s failed: %s", #expr, hipGetErrorString(e_));                 \
      return e_ == hipErrorOutOfMemory ? RTS_E_NOMEM : RTS_E_HIP;               \
    }                                                                           \
  } while (0)

using TuneKey = std::tuple<int, int, int, int, int, int, int, long long>;
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune_cache;

// Live cadence graphs per plan: a graph holds the plan's buffer addresses.
std::mutex g_graph_mu;
std::map<const Plan *, int> g_graph_count;

}  // namespace

namespace rts {
int live_graphs(const Plan *p) {
  std::lock_guard<std::mutex> lock(g_graph_mu);
  const auto it = g_graph_count.find(p);
  return it == g_graph_count.end() ? 0 : it->second;
}
}  // namespace rts

extern "C" {

rts_status rts_cadence_graph_create(rts_graph_t *out, rts_plan_t plan, const double *uvw_m, const float *vis,
                                    const float *weights, const float *grid_in, float *model_out,
                                    float *grid_out, double *chi2_out, void *stream) {
  if (!out || !plan) {
    set_error("out and plan must be non-NULL");
    return RTS_E_INVALID;
  }
  *out = nullptr;
  if (plan->ncopy != 1) {
    set_error("cadence graphs need a plan without conjugate copies");
    return RTS_E_UNSUPPORTED;
  }
  const bool mfma_plan = plan->precision == RTS_PREC_BF16X3 || plan->precision == RTS_PREC_FP32_MFMA;
  if (!mfma_plan && (plan->W > kMaxW || plan->d_pb_thl)) {
    set_error("cadence graphs of FP32 plans need support <= %d and the shared kernel", kMaxW);
    return RTS_E_UNSUPPORTED;
  }
  if (mfma_plan && !model_out) {
    set_error("cadence graphs of matrix-core plans need model_out");
    return RTS_E_INVALID;
  }
  hipStream_t cs = nullptr;
  RTS_HIP_R(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  // the captured work must follow whatever the caller already queued
  hipEvent_t ev = nullptr;
  hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(ev, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(cs, ev, 0);
  if (e == hipSuccess) e = hipStreamSynchronize(cs);
  rts_status st = RTS_OK;
  hipGraph_t graph = nullptr;
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = rts_plan_update(plan, uvw_m, weights, cs);
    if (st == RTS_OK) st = rts_grid_degrid(plan, vis, weights, grid_in, model_out, grid_out, chi2_out, cs);
    const hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (st == RTS_OK && e2 != hipSuccess) e = e2;
  }
  hipGraphExec_t exec = nullptr;
  if (e == hipSuccess && st == RTS_OK) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ev) hipEventDestroy(ev);
  hipStreamDestroy(cs);
  if (st != RTS_OK || e != hipSuccess) {
    if (graph) hipGraphDestroy(graph);
    if (st != RTS_OK) return st;
    set_error("cadence graph capture failed: %s", hipGetErrorString(e));
    return RTS_E_HIP;
  }
  rts_graph_s *g = new (std::nothrow) rts_graph_s();
  if (!g) {
    hipGraphExecDestroy(exec);
    hipGraphDestroy(graph);
    set_error("host allocation failed");
    return RTS_E_NOMEM;
  }
  g->graph = graph;
  g->exec = exec;
  g->plan = plan;
  {
    std::lock_guard<std::mutex> lock(g_graph_mu);
    ++g_graph_count[plan];
  }
  *out = g;
  return RTS_OK;
}

rts_status rts_cadence_graph_launch(rts_graph_t graph, void *stream) {
  if (!graph) {
    set_error("graph is NULL");
    return RTS_E_INVALID;
  }
  RTS_HIP_R(hipGraphLaunch(graph->exec, (hipStream_t)stream));
  graph->plan->stats_pending = true;
  return RTS_OK;
}

rts_status rts_cadence_graph_destroy(rts_graph_t graph) {
  if (!graph) return RTS_OK;
  {
    std::lock_guard<std::mutex> lock(g_graph_mu);
    const auto it = g_graph_count.find(graph->plan);
    if (it != g_graph_count.end() && --it->second <= 0) g_graph_count.erase(it);
  }
  hipGraphExecDestroy(graph->exec);
  hipGraphDestroy(graph->graph);
  delete graph;
  return RTS_OK;
}

rts_status rts_autotune_tile(const rts_params *params, const double *uvw_m, const double *freq_hz,
                             const float *weights, const float *vis, const float *grid_in, void *stream,
                             int32_t *best_tile, float *ms_out, int32_t *tiles_out, int32_t capacity,
                             int32_t *n_tried) {
  if (!params || !uvw_m || !freq_hz || !weights || !vis || !grid_in || !best_tile) {
    set_error("null pointer argument");
    return RTS_E_INVALID;
  }
  const int N = params->n_grid, W = params->support;
  const TuneKey key{N, W, params->oversample, params->n_chan, params->n_base, params->n_time,
                    params->conjugate, (long long)(params->cell_lambda * 1e9)};
  if (n_tried) *n_tried = 0;
  if (!ms_out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      *best_tile = it->second;
      return RTS_OK;
    }
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t nvis = (size_t)params->n_chan * params->n_base * params->n_time;
  const size_t ngrid = (size_t)params->n_chan * N * N;
  float *model = nullptr, *gout = nullptr;
  double *chi2 = nullptr;
  RTS_HIP_R(hipMalloc((void **)&model, nvis * 8));
  hipError_t e = hipMalloc((void **)&gout, ngrid * 8);
  if (e == hipSuccess) e = hipMalloc((void **)&chi2, 8);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  rts_status st = RTS_OK;
  float best_ms = 1e30f;
  int best = 0, tried = 0;
  const int cands[] = {16, 32, 64};
  for (int t : cands) {
    if (e != hipSuccess || st != RTS_OK) break;
    if (t < W + 1 || N % t != 0) continue;
    rts_params p = *params;
    p.tile = t;
    rts_plan_t plan = nullptr;
    st = rts_grid_plan(&plan, &p, uvw_m, freq_hz, weights, stream);
    if (st != RTS_OK) break;
    // one untimed pass, then three timed cadence steps
    st = rts_grid_degrid(plan, vis, weights, grid_in, model, gout, chi2, stream);
    if (st == RTS_OK) e = hipEventRecord(e0, s);
    for (int r = 0; r < 3 && st == RTS_OK && e == hipSuccess; ++r) {
      st = rts_plan_update(plan, uvw_m, weights, stream);
      if (st == RTS_OK) st = rts_grid_degrid(plan, vis, weights, grid_in, model, gout, chi2, stream);
    }
    float ms = 0.0f;
    if (st == RTS_OK && e == hipSuccess) e = hipEventRecord(e1, s);
    if (st == RTS_OK && e == hipSuccess) e = hipEventSynchronize(e1);
    if (st == RTS_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    rts_plan_destroy(plan);
    if (st != RTS_OK || e != hipSuccess) break;
    ms /= 3.0f;
    if (ms_out && tried < capacity) {
      ms_out[tried] = ms;
      if (tiles_out) tiles_out[tried] = t;
    }
    ++tried;
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipFree(model);
  hipFree(gout);
  hipFree(chi2);
  if (st != RTS_OK) return st;
  if (e != hipSuccess) {
    set_error("autotune: %s", hipGetErrorString(e));
    return RTS_E_HIP;
  }
  if (best == 0) {
    set_error("no legal tile size for n_grid=%d support=%d", N, W);
    return RTS_E_UNSUPPORTED;
  }
  *best_tile = best;
  if (n_tried) *n_tried = tried;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = best;
  return RTS_OK;
}

}  // extern "C"
