// CPU stand-in executor of the serving runtime (no HIP): the scheduler's admission,
// ordering, splitting, scattering and failure handling can be tested, and sanitised,
// without a GPU.  Test code only: it is linked into the test library, not libtabnet.so.
#include <algorithm>
#include <chrono>
#include <thread>
#include <vector>

#include "tabnet_serve.hpp"

namespace tabnet {
namespace {

// ---------------------------------------------------------------- fake executor
// Runs on the CPU: logits[r][o] = X[r][o % D] + o, masks_agg[r][j] = 2 X[r][j],
// masks_step[s][r][j] = X[r][j] + s.  It exercises batching, splitting and scattering.
class FakeExecutor : public Executor {
 public:
  std::vector<ModelInfo> models;
  tabnet_serve_opts o;
  Dims dm;
  int delay_us = 0;
  int fail_launch = -1, fail_wait = -1;   // index of the launch that fails (-1: none)
  int n_launch = 0;
  std::vector<int> slot_launch;           // launch index held by each slot
  struct Slot {
    std::vector<float> x, lo, ag, ms;
    std::vector<double> st;      // mean[D], M2[D], n of the last launch's masks_agg
  };
  std::vector<Slot> slots;

  void init() {
    dm = max_dims(models);
    const size_t R = (size_t)o.max_rows_per_launch;
    slots.resize(o.slots);
    slot_launch.assign(o.slots, -1);
    for (Slot& s : slots) {
      s.x.resize(R * dm.D);
      s.lo.resize(R * dm.n_out);
      s.ag.resize(R * dm.D);
      if (o.with_step_masks) s.ms.resize(R * dm.S * dm.D);
    }
  }
  float* input(int slot) override { return slots[slot].x.data(); }
  bool launch(int slot, int model, int64_t rows) override {
    const int k = n_launch++;
    slot_launch[slot] = k;
    if (k == fail_launch) return false;
    Slot& s = slots[slot];
    const int D = models[model].cfg.D, n_out = models[model].cfg.n_out, S = models[model].cfg.n_steps;
    for (int64_t r = 0; r < rows; ++r) {
      for (int oo = 0; oo < n_out; ++oo) s.lo[r * n_out + oo] = s.x[r * D + oo % D] + (float)oo;
      for (int j = 0; j < D; ++j) s.ag[r * D + j] = 2.f * s.x[r * D + j];
      if (!s.ms.empty())
        for (int st = 0; st < S; ++st)
          for (int j = 0; j < D; ++j) s.ms[((int64_t)st * rows + r) * D + j] = s.x[r * D + j] + (float)st;
    }
    if (o.mask_stats_window > 0) {
      // two-pass column statistics of this launch's masks_agg (the GPU computes the same
      // three quantities in its statistics kernels)
      s.st.assign(2 * (size_t)D + 1, 0.0);
      for (int j = 0; j < D; ++j) {
        double sum = 0.0;
        for (int64_t r = 0; r < rows; ++r) sum += s.ag[r * D + j];
        const double mean = sum / (double)rows;
        double q = 0.0;
        for (int64_t r = 0; r < rows; ++r) q += ((double)s.ag[r * D + j] - mean) * ((double)s.ag[r * D + j] - mean);
        s.st[j] = mean;
        s.st[D + j] = q;
      }
      s.st[2 * (size_t)D] = (double)rows;
    }
    if (delay_us > 0) std::this_thread::sleep_for(std::chrono::microseconds(delay_us));
    return true;
  }
  bool wait(int slot) override { return slot_launch[slot] != fail_wait; }
  const float* out_logits(int slot) override { return slots[slot].lo.data(); }
  const float* out_agg(int slot) override { return slots[slot].ag.data(); }
  const float* out_steps(int slot) override { return slots[slot].ms.empty() ? nullptr : slots[slot].ms.data(); }
  const double* out_mask_stats(int slot) override { return slots[slot].st.empty() ? nullptr : slots[slot].st.data(); }
};

}  // namespace

Executor* make_fake_executor(const std::vector<ModelInfo>& models, const tabnet_serve_opts& o, int delay_us,
                             int fail_launch, int fail_wait) {
  FakeExecutor* x = new FakeExecutor();
  x->models = models;
  x->o = o;
  x->delay_us = delay_us;
  x->fail_launch = fail_launch;
  x->fail_wait = fail_wait;
  x->init();
  return x;
}

}  // namespace tabnet
