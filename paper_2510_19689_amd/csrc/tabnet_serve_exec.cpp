// Executors of the serving runtime and the serving part of the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/tabnet_internal.h"
#include "tabnet_handle.hpp"
#include "tabnet_serve.hpp"
#include "tabnet_stats.hpp"

namespace tabnet {
namespace {

// ---------------------------------------------------------------- HIP executor
struct HipSlot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  float *d_x = nullptr, *d_lo = nullptr, *d_ag = nullptr, *d_ms = nullptr;
  float *h_x = nullptr, *h_lo = nullptr, *h_ag = nullptr, *h_ms = nullptr;
  int64_t* d_rows = nullptr;     // live row count read by the kernel
  int64_t* h_rows = nullptr;     // pinned source of d_rows
  void* d_sws = nullptr;         // mask-statistics workspace (max_rows_per_launch rows)
  double *d_st = nullptr, *h_st = nullptr;   // mean[D], M2[D], n of the last launch
  std::vector<hipGraphExec_t> graphs;   // per model
  int model = 0;
  int64_t rows = 0;
};

class HipExecutor : public Executor {
 public:
  std::vector<ModelInfo> models;
  tabnet_serve_opts o;
  Dims dm;
  int device = 0;
  std::vector<HipSlot> slots;

  hipError_t init() {
    device = models[0].handle->device;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return e;
    dm = max_dims(models);
    const size_t R = (size_t)o.max_rows_per_launch;
    slots.resize(o.slots);
    for (HipSlot& s : slots) {
      if ((e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking)) != hipSuccess) return e;
      if ((e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming)) != hipSuccess) return e;
      if ((e = hipMalloc(&s.d_x, R * dm.D * 4)) != hipSuccess) return e;
      if ((e = hipMalloc(&s.d_lo, R * dm.n_out * 4)) != hipSuccess) return e;
      if ((e = hipMalloc(&s.d_ag, R * dm.D * 4)) != hipSuccess) return e;
      if ((e = hipMalloc(&s.d_rows, sizeof(int64_t))) != hipSuccess) return e;
      if ((e = hipHostMalloc(&s.h_x, R * dm.D * 4, hipHostMallocDefault)) != hipSuccess) return e;
      if ((e = hipHostMalloc(&s.h_lo, R * dm.n_out * 4, hipHostMallocDefault)) != hipSuccess) return e;
      if ((e = hipHostMalloc(&s.h_ag, R * dm.D * 4, hipHostMallocDefault)) != hipSuccess) return e;
      if ((e = hipHostMalloc(&s.h_rows, sizeof(int64_t), hipHostMallocDefault)) != hipSuccess) return e;
      if (o.with_step_masks) {
        if ((e = hipMalloc(&s.d_ms, R * dm.S * dm.D * 4)) != hipSuccess) return e;
        if ((e = hipHostMalloc(&s.h_ms, R * dm.S * dm.D * 4, hipHostMallocDefault)) != hipSuccess) return e;
      }
      if (o.mask_stats_window > 0) {
        if ((e = hipMalloc(&s.d_sws, mask_stats_workspace_bytes((int64_t)R, dm.D))) != hipSuccess) return e;
        if ((e = hipMalloc(&s.d_st, (2 * (size_t)dm.D + 1) * sizeof(double))) != hipSuccess) return e;
        if ((e = hipHostMalloc(&s.h_st, (2 * (size_t)dm.D + 1) * sizeof(double), hipHostMallocDefault)) !=
            hipSuccess)
          return e;
      }
      if (o.use_graph) {
        // One graph per model: the live row count (pinned -> device) and the forward,
        // whose grid covers max_rows_per_launch and which reads the count on the device.
        for (const ModelInfo& m : models) {
          hipGraph_t g = nullptr;
          hipGraphExec_t ge = nullptr;
          if ((e = hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
          hipError_t e1 = hipMemcpyAsync(s.d_rows, s.h_rows, sizeof(int64_t), hipMemcpyHostToDevice, s.stream);
          hipError_t e2 = enqueue_forward(m.handle, s.d_x, (int64_t)R, s.d_rows, s.d_lo, s.d_ag, s.d_ms, s.stream);
          hipError_t e3 = hipSuccess;
          if (e2 == hipSuccess && o.mask_stats_window > 0) e3 = enqueue_stats(s, m.cfg.D, (int64_t)R, s.d_rows);
          if ((e = hipStreamEndCapture(s.stream, &g)) != hipSuccess) return e;
          if (e1 != hipSuccess) return e1;
          if (e2 != hipSuccess) return e2;
          if (e3 != hipSuccess) return e3;
          e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
          (void)hipGraphDestroy(g);
          if (e != hipSuccess) return e;
          s.graphs.push_back(ge);
        }
      }
    }
    return hipSuccess;
  }

  // Statistics of the slot's masks_agg (rows, or the live count in rows_dev): mean, M2, n.
  hipError_t enqueue_stats(HipSlot& s, int D, int64_t rows, const int64_t* rows_dev) {
    return enqueue_mask_stats(s.d_ag, rows, rows_dev, D, s.d_st, nullptr, s.d_st + D, s.d_st + 2 * (size_t)D,
                              s.d_sws, s.stream);
  }

  ~HipExecutor() override {
    (void)hipSetDevice(device);
    for (HipSlot& s : slots) {
      if (s.stream) (void)hipStreamSynchronize(s.stream);
      for (hipGraphExec_t ge : s.graphs) (void)hipGraphExecDestroy(ge);
      if (s.done) (void)hipEventDestroy(s.done);
      if (s.stream) (void)hipStreamDestroy(s.stream);
      for (float* p : {s.d_x, s.d_lo, s.d_ag, s.d_ms})
        if (p) (void)hipFree(p);
      if (s.d_rows) (void)hipFree(s.d_rows);
      if (s.d_sws) (void)hipFree(s.d_sws);
      if (s.d_st) (void)hipFree(s.d_st);
      if (s.h_st) (void)hipHostFree(s.h_st);
      for (float* p : {s.h_x, s.h_lo, s.h_ag, s.h_ms})
        if (p) (void)hipHostFree(p);
      if (s.h_rows) (void)hipHostFree(s.h_rows);
    }
  }

  float* input(int slot) override { return slots[slot].h_x; }

  bool launch(int slot, int model, int64_t rows) override {
    HipSlot& s = slots[slot];
    const ModelInfo& m = models[model];
    const int D = m.cfg.D, n_out = m.cfg.n_out, S = m.cfg.n_steps;
    s.model = model;
    s.rows = rows;
    if (hipSetDevice(device) != hipSuccess) return false;
    if (hipMemcpyAsync(s.d_x, s.h_x, (size_t)rows * D * 4, hipMemcpyHostToDevice, s.stream) != hipSuccess)
      return false;
    if (o.use_graph) {
      *s.h_rows = rows;
      if (hipGraphLaunch(s.graphs[model], s.stream) != hipSuccess) return false;
    } else {
      if (enqueue_forward(m.handle, s.d_x, rows, nullptr, s.d_lo, s.d_ag, s.d_ms, s.stream) != hipSuccess)
        return false;
      if (o.mask_stats_window > 0 && enqueue_stats(s, D, rows, nullptr) != hipSuccess) return false;
    }
    if (o.mask_stats_window > 0 &&
        hipMemcpyAsync(s.h_st, s.d_st, (2 * (size_t)D + 1) * sizeof(double), hipMemcpyDeviceToHost, s.stream) !=
            hipSuccess)
      return false;
    if (hipMemcpyAsync(s.h_lo, s.d_lo, (size_t)rows * n_out * 4, hipMemcpyDeviceToHost, s.stream) != hipSuccess)
      return false;
    if (hipMemcpyAsync(s.h_ag, s.d_ag, (size_t)rows * D * 4, hipMemcpyDeviceToHost, s.stream) != hipSuccess)
      return false;
    if (s.d_ms && hipMemcpyAsync(s.h_ms, s.d_ms, (size_t)S * rows * D * 4, hipMemcpyDeviceToHost, s.stream) !=
                      hipSuccess)
      return false;
    return hipEventRecord(s.done, s.stream) == hipSuccess;
  }

  bool wait(int slot) override {
    HipSlot& s = slots[slot];
    // Poll briefly (low latency), then block.
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
      const hipError_t q = hipEventQuery(s.done);
      if (q == hipSuccess) return true;
      if (q != hipErrorNotReady) return false;
      if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) break;
      std::this_thread::yield();
    }
    return hipEventSynchronize(s.done) == hipSuccess;
  }

  const float* out_logits(int slot) override { return slots[slot].h_lo; }
  const float* out_agg(int slot) override { return slots[slot].h_ag; }
  const float* out_steps(int slot) override { return slots[slot].h_ms; }
  const double* out_mask_stats(int slot) override { return slots[slot].h_st; }
};

}  // namespace

Executor* make_hip_executor(const std::vector<ModelInfo>& models, const tabnet_serve_opts& o, tabnet_status* st) {
  HipExecutor* x = new HipExecutor();
  x->models = models;
  x->o = o;
  hipError_t e = x->init();
  if (e != hipSuccess) {
    set_error(std::string("tabnet_serve_start: ") + hipGetErrorString(e));
    *st = e == hipErrorOutOfMemory ? TABNET_E_OOM : TABNET_E_HIP;
    delete x;
    return nullptr;
  }
  *st = TABNET_OK;
  return x;
}

}  // namespace tabnet

using namespace tabnet;

struct tabnet_server {
  ServerImpl* impl;
};

namespace tabnet {

tabnet_status fill_opts(const tabnet_serve_opts* in, tabnet_serve_opts* o) {
  std::memset(o, 0, sizeof *o);
  if (in) *o = *in;
  if (o->mem_budget_bytes == 0) o->mem_budget_bytes = 8ull << 30;
  if (o->max_rows_per_launch == 0) o->max_rows_per_launch = 65536;
  if (o->slots == 0) o->slots = 3;
  if (in == nullptr) o->use_graph = 1;
  if (o->max_rows_per_launch < 1 || o->slots < 1 || o->slots > 8 || o->mask_stats_window < 0) {
    set_error("tabnet_serve_start: max_rows_per_launch must be >= 1, slots in [1, 8], mask_stats_window >= 0");
    return TABNET_E_INVALID;
  }
  return TABNET_OK;
}

ModelInfo info_of(const tabnet_config& c, bool steps, tabnet_handle* h) {
  ModelInfo m;
  m.cfg = c;
  m.bytes_per_row = 4ull * ((uint64_t)c.D + c.n_out + c.D + (steps ? (uint64_t)c.n_steps * c.D : 0));
  m.handle = h;
  return m;
}

tabnet_status start_with(std::vector<ModelInfo> models, Executor* ex, const tabnet_serve_opts& o,
                         tabnet_server** out) {
  ServerImpl* impl = nullptr;
  tabnet_status st = server_create(std::move(models), ex, o, &impl);
  if (st != TABNET_OK) return st;
  *out = new tabnet_server{impl};
  return TABNET_OK;
}

}  // namespace tabnet

extern "C" {

tabnet_status tabnet_serve_start(tabnet_handle* const* hs, int n, const tabnet_serve_opts* opts,
                                 tabnet_server** out) {
  if (!hs || n < 1 || !out) {
    set_error("tabnet_serve_start: NULL models or out, or n_models < 1");
    return TABNET_E_INVALID;
  }
  *out = nullptr;
  tabnet_serve_opts o;
  tabnet_status st = fill_opts(opts, &o);
  if (st != TABNET_OK) return st;
  std::vector<ModelInfo> models;
  for (int i = 0; i < n; ++i) {
    if (!hs[i] || hs[i]->failed || hs[i]->device != hs[0]->device) {
      set_error("tabnet_serve_start: a model handle is NULL, failed, or on another device");
      return TABNET_E_INVALID;
    }
    models.push_back(info_of(hs[i]->cfg, o.with_step_masks != 0, hs[i]));
  }
  Executor* ex = make_hip_executor(models, o, &st);
  if (!ex) return st;
  return start_with(std::move(models), ex, o, out);
}

tabnet_status tabnet_serve_submit(tabnet_server* s, int model, const float* X_host, int64_t rows,
                                  float* logits_host, float* masks_agg_host, float* masks_step_host,
                                  int64_t arrival_ns, uint64_t* req_id) {
  if (!s) {
    set_error("tabnet_serve_submit: NULL server");
    return TABNET_E_INVALID;
  }
  return server_submit(s->impl, model, X_host, rows, logits_host, masks_agg_host, masks_step_host,
                       arrival_ns, req_id);
}

tabnet_status tabnet_serve_wait(tabnet_server* s, uint64_t req_id, int64_t timeout_us) {
  if (!s) return TABNET_E_INVALID;
  return server_wait(s->impl, req_id, timeout_us);
}

tabnet_status tabnet_serve_poll(tabnet_server* s, uint64_t req_id, int* done) {
  if (!s || !done) return TABNET_E_INVALID;
  return server_poll(s->impl, req_id, done);
}

tabnet_status tabnet_serve_get_stats(tabnet_server* s, tabnet_serve_stats* out) {
  if (!s || !out) return TABNET_E_INVALID;
  return server_stats(s->impl, out);
}

tabnet_status tabnet_serve_get_model_stats(tabnet_server* s, int model, tabnet_serve_stats* out) {
  if (!s || !out) return TABNET_E_INVALID;
  return server_model_stats(s->impl, model, out);
}

tabnet_status tabnet_serve_reset_stats(tabnet_server* s) {
  if (!s) return TABNET_E_INVALID;
  return server_reset_stats(s->impl);
}

tabnet_status tabnet_serve_mask_stats(tabnet_server* s, int model, double* mean_host, double* var_host,
                                      int64_t* rows) {
  if (!s) return TABNET_E_INVALID;
  return server_mask_stats(s->impl, model, mean_host, var_host, rows);
}

int64_t tabnet_serve_now_ns(void) { return now_ns(); }

tabnet_status tabnet_serve_stop(tabnet_server* s) {
  if (!s) return TABNET_E_INVALID;
  tabnet_status st = server_stop(s->impl);
  delete s;
  return st;
}

}  // extern "C"
