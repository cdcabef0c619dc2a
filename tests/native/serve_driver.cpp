// Host-only driver for the serving scheduler with the CPU stand-in executor; built by
// tests/test_sanitizers.py under ThreadSanitizer and under AddressSanitizer+UBSan.
// Several submitter threads, requests split across launches, concurrent waits, stop; then
// megabyte requests that take the split path of the server's host copies; then a split
// request whose second launch fails.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "../../paper_2510_19689_amd/csrc/tabnet_serve.hpp"

namespace tabnet {
void set_error(const std::string&) {}
}  // namespace tabnet

using namespace tabnet;

int main() {
  tabnet_config c{};
  c.D = 9;
  c.n_d = 4;
  c.n_a = 4;
  c.n_steps = 2;
  c.n_shared = 1;
  c.n_indep = 1;
  c.n_out = 3;
  c.gamma = 1.3;
  c.bn_eps = 1e-5;
  std::vector<ModelInfo> models{ModelInfo{c, 4ull * (9 + 3 + 9 + 18), nullptr}};
  tabnet_serve_opts o{};
  o.mem_budget_bytes = 4ull * (9 + 3 + 9 + 18) * 300;
  o.max_rows_per_launch = 64;
  o.slots = 3;
  o.with_step_masks = 1;
  Executor* ex = make_fake_executor(models, o, 50);
  ServerImpl* s = nullptr;
  if (server_create(models, ex, o, &s) != TABNET_OK) return 2;
  std::atomic<int> bad{0};
  std::vector<std::thread> ts;
  for (int t = 0; t < 4; ++t)
    ts.emplace_back([&, t] {
      std::mt19937 rng(t);
      for (int k = 0; k < 40; ++k) {
        const int rows = 1 + (int)(rng() % 150);
        std::vector<float> X(rows * 9), lo(rows * 3), ag(rows * 9), ms(2 * rows * 9);
        for (auto& v : X) v = (float)(rng() % 1000) / 100.f;
        uint64_t id = 0;
        if (server_submit(s, 0, X.data(), rows, lo.data(), ag.data(), ms.data(), 0, &id) != TABNET_OK) {
          ++bad;
          continue;
        }
        if (server_wait(s, id, -1) != TABNET_OK) ++bad;
        for (int r = 0; r < rows; ++r) {
          for (int o2 = 0; o2 < 3; ++o2)
            if (lo[r * 3 + o2] != X[r * 9 + o2 % 9] + (float)o2) ++bad;
          for (int j = 0; j < 9; ++j) {
            if (ag[r * 9 + j] != 2.f * X[r * 9 + j]) ++bad;
            for (int st = 0; st < 2; ++st)
              if (ms[(st * rows + r) * 9 + j] != X[r * 9 + j] + (float)st) ++bad;
          }
        }
      }
    });
  for (auto& th : ts) th.join();
  tabnet_serve_stats st{};
  server_stats(s, &st);
  // requests left queued at stop are cancelled, not leaked
  std::vector<float> X(50 * 9, 1.f), lo(50 * 3), ag(50 * 9);
  uint64_t id = 0;
  for (int k = 0; k < 5; ++k) server_submit(s, 0, X.data(), 50, lo.data(), ag.data(), nullptr, 0, &id);
  server_stop(s);
  std::printf("completed=%llu bad=%d\n", (unsigned long long)st.completed, bad.load());
  if (bad.load() != 0 || st.completed != 160) return 1;

  // Wide rows: requests of megabytes, so that the server's host copies (input at submit,
  // gather into the launch buffer, scatter of the outputs) take their split path.
  const int D = 2048;
  tabnet_config w = c;
  w.D = D;
  w.n_out = 2;
  w.n_steps = 1;
  std::vector<ModelInfo> wide{ModelInfo{w, 4ull * (D + 2 + D + D), nullptr}};
  tabnet_serve_opts ow = o;
  ow.mem_budget_bytes = 1ull << 30;
  ow.max_rows_per_launch = 512;
  ow.slots = 2;
  Executor* ew = make_fake_executor(wide, ow, 50);
  ServerImpl* sw = nullptr;
  if (server_create(wide, ew, ow, &sw) != TABNET_OK) return 2;
  std::atomic<int> bad2{0};
  std::vector<std::thread> tw;
  for (int t = 0; t < 2; ++t)
    tw.emplace_back([&, t] {
      std::mt19937 rng(100 + t);
      for (int k = 0; k < 4; ++k) {
        const int rows = 300 + (int)(rng() % 400);
        std::vector<float> X((size_t)rows * D), lo(rows * 2), ag((size_t)rows * D), ms((size_t)rows * D);
        for (size_t i = 0; i < X.size(); ++i) X[i] = (float)((i * 7 + k + 3 * t) % 1000) / 100.f;
        uint64_t id = 0;
        if (server_submit(sw, 0, X.data(), rows, lo.data(), ag.data(), ms.data(), 0, &id) != TABNET_OK ||
            server_wait(sw, id, -1) != TABNET_OK) {
          ++bad2;
          continue;
        }
        for (int r = 0; r < rows; ++r) {
          for (int o2 = 0; o2 < 2; ++o2)
            if (lo[r * 2 + o2] != X[(size_t)r * D + o2] + (float)o2) ++bad2;
          for (int j = 0; j < D; ++j) {
            if (ag[(size_t)r * D + j] != 2.f * X[(size_t)r * D + j]) ++bad2;
            if (ms[(size_t)r * D + j] != X[(size_t)r * D + j]) ++bad2;
          }
        }
      }
    });
  for (auto& th : tw) th.join();
  tabnet_serve_stats sw_st{};
  server_stats(sw, &sw_st);
  server_stop(sw);
  std::printf("wide completed=%llu bad=%d\n", (unsigned long long)sw_st.completed, bad2.load());
  if (bad2.load() != 0 || sw_st.completed != 8) return 1;

  // A request split over four launches whose second launch fails when waited on: once
  // wait reports the failure the caller frees its buffers at once (AddressSanitizer sees
  // any later write), and the next requests are served.
  tabnet_serve_opts of = o;
  of.max_rows_per_launch = 100;
  of.slots = 2;
  of.with_step_masks = 0;
  of.mem_budget_bytes = 1ull << 30;
  Executor* ef = make_fake_executor(models, of, 2000, -1, 1);
  ServerImpl* sf = nullptr;
  if (server_create(models, ef, of, &sf) != TABNET_OK) return 2;
  int bad3 = 0;
  {
    const int rows = 350;
    float* Xf = new float[rows * 9];
    float* lof = new float[rows * 3];
    float* agf = new float[rows * 9];
    for (int k = 0; k < rows * 9; ++k) Xf[k] = (float)(k % 17);
    uint64_t fid = 0;
    if (server_submit(sf, 0, Xf, rows, lof, agf, nullptr, 0, &fid) != TABNET_OK) ++bad3;
    if (server_wait(sf, fid, -1) != TABNET_E_HIP) ++bad3;
    delete[] Xf;
    delete[] lof;
    delete[] agf;
  }
  for (int k = 0; k < 4; ++k) {
    std::vector<float> Xg(60 * 9, 1.5f), log(60 * 3), agg(60 * 9);
    uint64_t gid = 0;
    if (server_submit(sf, 0, Xg.data(), 60, log.data(), agg.data(), nullptr, 0, &gid) != TABNET_OK ||
        server_wait(sf, gid, -1) != TABNET_OK)
      ++bad3;
    for (float v : agg)
      if (v != 3.f) ++bad3;
  }
  tabnet_serve_stats sf_st{};
  server_stats(sf, &sf_st);
  if (sf_st.inflight_bytes != 0) ++bad3;
  server_stop(sf);
  std::printf("failed split request: bad=%d\n", bad3);
  return bad3 == 0 ? 0 : 1;
}
