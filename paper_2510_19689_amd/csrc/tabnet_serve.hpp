// Serving runtime internals: executor interface and scheduler entry points.
#pragma once
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/tabnet.h"

struct tabnet_handle;
struct tabnet_server;

namespace tabnet {

struct ModelInfo {
  tabnet_config cfg;
  uint64_t bytes_per_row;        // admission cost: X in + all requested outputs (FP32)
  tabnet_handle* handle;         // null for the fake executor
};

// Device side of the server.  A slot is one launch buffer: pinned input rows, the
// outputs of its last launch, and (for the HIP executor) a stream, an event, device
// buffers and one captured graph per model.
struct Executor {
  virtual ~Executor() {}
  virtual float* input(int slot) = 0;                 // [max_rows, D] host, pinned
  virtual bool launch(int slot, int model, int64_t rows) = 0;   // asynchronous
  virtual bool wait(int slot) = 0;                    // false: the launch failed
  virtual const float* out_logits(int slot) = 0;      // [rows, n_out]
  virtual const float* out_agg(int slot) = 0;         // [rows, D]
  virtual const float* out_steps(int slot) = 0;       // [n_steps, rows, D] or null
  // Statistics of the last launch's masks_agg when the server keeps them:
  // mean[D], M2[D] (sums of squared deviations), n -- 2 D + 1 doubles of that model's D.
  virtual const double* out_mask_stats(int slot) = 0;
};

// Largest D, n_out and n_steps over the served models (sizes of the slot buffers).
struct Dims {
  int D = 0, n_out = 0, S = 0;
};
inline Dims max_dims(const std::vector<ModelInfo>& models) {
  Dims d;
  for (const ModelInfo& m : models) {
    d.D = m.cfg.D > d.D ? m.cfg.D : d.D;
    d.n_out = m.cfg.n_out > d.n_out ? m.cfg.n_out : d.n_out;
    d.S = m.cfg.n_steps > d.S ? m.cfg.n_steps : d.S;
  }
  return d;
}

struct ServerImpl;
int64_t now_ns();
tabnet_status server_create(std::vector<ModelInfo> models, Executor* exec, const tabnet_serve_opts& o,
                            ServerImpl** out);
tabnet_status server_submit(ServerImpl* s, int model, const float* X, int64_t rows, float* logits,
                            float* magg, float* msteps, int64_t arrival_ns, uint64_t* id);
tabnet_status server_wait(ServerImpl* s, uint64_t id, int64_t timeout_us);
tabnet_status server_poll(ServerImpl* s, uint64_t id, int* done);
tabnet_status server_stats(ServerImpl* s, tabnet_serve_stats* o);
tabnet_status server_model_stats(ServerImpl* s, int model, tabnet_serve_stats* o);
tabnet_status server_reset_stats(ServerImpl* s);
tabnet_status server_mask_stats(ServerImpl* s, int model, double* mean, double* var, int64_t* rows);
tabnet_status server_stop(ServerImpl* s);   // joins the threads, deletes the executor and s

Executor* make_hip_executor(const std::vector<ModelInfo>& models, const tabnet_serve_opts& o, tabnet_status* st);
// CPU stand-in (test library only); launch number fail_launch fails to launch and launch
// number fail_wait fails when waited on (-1: never).
Executor* make_fake_executor(const std::vector<ModelInfo>& models, const tabnet_serve_opts& o, int delay_us,
                             int fail_launch = -1, int fail_wait = -1);
// Option defaults and validation, the per-model admission cost, and server start-up with
// a given executor (shared by tabnet_serve_start and the test library's CPU server).
tabnet_status fill_opts(const tabnet_serve_opts* in, tabnet_serve_opts* o);
ModelInfo info_of(const tabnet_config& c, bool steps, tabnet_handle* h);
tabnet_status start_with(std::vector<ModelInfo> models, Executor* ex, const tabnet_serve_opts& o,
                         tabnet_server** out);
void set_error(const std::string& msg);

// The serving path's host copy of n bytes: streaming stores from 4 KiB up where the CPU
// has AVX2, memcpy otherwise.
void serve_copy(void* dst, const void* src, size_t n);

}  // namespace tabnet
