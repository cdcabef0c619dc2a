// Host-only driver for the serving scheduler with the CPU stand-in executor; built by
// tests/test_sanitizers.py under ThreadSanitizer and under AddressSanitizer+UBSan.
// Several submitter threads, requests split across launches, concurrent waits, stop.
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
  return (bad.load() == 0 && st.completed == 160) ? 0 : 1;
}
